"""ctypes front end of the plain FP64 CPU oracle (``mgfr_oracle.c``).

Test infrastructure only: the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it to check the HIP library; the library never calls it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mgfr_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")          # plain build, one thread
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")  # the same source with -fopenmp

C_OVER_H0 = 2997.92458
C_KMS = 299792.458


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math): the plain single-thread
    build and the OpenMP build of the same source (bitwise the same results)."""
    for out, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
            tmp = out + ".tmp"
            subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", *extra, "-o", tmp, SRC, "-lm"],
                                  stderr=subprocess.DEVNULL)
            os.replace(tmp, out)
    return LIB


class Params(C.Structure):
    _fields_ = [("box", C.c_double), ("a", C.c_double), ("omega_m", C.c_double),
                ("omega_l", C.c_double), ("fr0_abs", C.c_double), ("n", C.c_int),
                ("mesh", C.c_int), ("tol", C.c_double), ("pre_smooth", C.c_int),
                ("post_smooth", C.c_int), ("coarse_sweeps", C.c_int),
                ("max_vcycles", C.c_int), ("prolong", C.c_int), ("max_du", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("vcycles", C.c_int), ("status", C.c_int), ("res0", C.c_double),
                ("res", C.c_double), ("scale", C.c_double), ("res_hist", C.c_double * 512)]


_libs = {}


def lib(serial: bool | None = None):
    """The oracle library: the OpenMP build unless serial (or MGFR_ORACLE_SERIAL=1)."""
    if serial is None:
        serial = os.environ.get("MGFR_ORACLE_SERIAL", "0") == "1"
    path = LIB if serial else LIB_OMP
    if path not in _libs:
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
            build(force=False)
        L = C.CDLL(path)
        L.or_threads.argtypes = [C.c_int]
        L.or_threads.restype = C.c_int
        dp = C.POINTER(C.c_double)
        fp = C.POINTER(C.c_float)
        L.or_background.argtypes = [C.POINTER(Params), dp, dp, dp]
        L.or_cic_assign.argtypes = [C.c_int, C.c_double, C.c_int64, fp, dp, dp]
        L.or_delta.argtypes = [C.c_int, dp, dp]
        L.or_source.argtypes = [C.POINTER(Params), dp, dp]
        L.or_screened_guess.argtypes = [C.POINTER(Params), dp, dp]
        L.or_effective_density.argtypes = [C.POINTER(Params), dp, dp, dp]
        L.or_apply_L.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, dp, dp]
        L.or_apply_J.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, dp, dp]
        L.or_residual_max.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, dp, dp]
        L.or_residual_max.restype = C.c_double
        L.or_ngs_sweep.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, C.c_double, dp, dp]
        L.or_restrict.argtypes = [C.c_int, dp, dp]
        L.or_prolong_add.argtypes = [C.c_int, C.c_int, dp, dp, dp]
        L.or_num_levels.argtypes = [C.c_int]
        L.or_num_levels.restype = C.c_int
        L.or_solve.argtypes = [C.POINTER(Params), dp, dp, dp, C.POINTER(Stats)]
        L.or_solve.restype = C.c_int
        L.or_vcycle_once.argtypes = [C.POINTER(Params), dp, dp]
        L.or_fifth_force.argtypes = [C.POINTER(Params), dp, C.c_int64, fp, dp]
        ip = C.POINTER(C.c_int64)
        L.or_residual_at.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, dp, dp, C.c_int64, ip, dp]
        L.or_cic_cells.argtypes = [C.c_int, C.c_double, C.c_int64, fp, dp, C.c_int64, ip, C.c_void_p, dp]
        L.or_fifth_force_at.argtypes = [C.POINTER(Params), dp, C.c_int64, fp, dp]
        L.or_amr_solve.argtypes = [C.POINTER(Params), C.c_int, C.c_int64, fp, C.POINTER(dp),
                                   C.POINTER(C.c_void_p), C.POINTER(Stats)]
        L.or_amr_solve.restype = C.c_int
        L.or_amr_flags.argtypes = [C.POINTER(Params), C.c_int, C.c_int64, fp, C.POINTER(C.c_void_p)]
        L.or_amr_cic.argtypes = [C.POINTER(Params), C.c_int, C.POINTER(C.c_void_p), C.c_int64, fp, dp,
                                 C.POINTER(dp)]
        L.or_amr_solve_fields.argtypes = [C.POINTER(Params), C.c_int, C.POINTER(C.c_void_p), C.POINTER(dp),
                                          C.POINTER(dp), C.POINTER(C.c_void_p), C.POINTER(Stats)]
        L.or_amr_solve_fields.restype = C.c_int
        L.or_amr_cic_cells.argtypes = [C.POINTER(Params), C.c_int, C.POINTER(C.c_void_p), C.c_int64, fp, dp,
                                       C.c_int64, C.c_void_p, C.c_void_p, dp]
        L.or_op_stencil.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int64, dp, dp, dp]
        L.or_gather_gradient.argtypes = [C.c_int, C.c_double, dp, C.c_int64, fp, C.c_double, dp]
        L.or_kick_drift.argtypes = [C.c_int64, fp, fp, fp, C.c_double, C.c_double, C.c_double]
        _libs[path] = L
    return _libs[path]


def threads(n: int = 0, serial: bool | None = None) -> int:
    """Set (n > 0) and return the oracle's thread count."""
    return int(lib(serial).or_threads(int(n)))


def _d(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f(a):
    assert a.dtype == np.float32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_float))


def params(mesh=32, box=100.0, a=1.0, omega_m=0.3, omega_l=0.7, fr0_abs=1e-5, n=1,
           tol=1e-8, pre_smooth=2, post_smooth=2, coarse_sweeps=30, max_vcycles=100,
           prolong=0, max_du=2.0) -> Params:
    return Params(box, a, omega_m, omega_l, fr0_abs, n, mesh, tol, pre_smooth, post_smooth,
                  coarse_sweeps, max_vcycles, prolong, max_du)


def background(p: Params):
    fb, beta, Cc = C.c_double(), C.c_double(), C.c_double()
    lib().or_background(C.byref(p), C.byref(fb), C.byref(beta), C.byref(Cc))
    return fb.value, beta.value, Cc.value


def cic_assign(N, box, pos, mass=None, serial=None):
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    m = np.zeros((N, N, N), np.float64)
    mp = None if mass is None else _d(np.ascontiguousarray(mass, np.float64))
    lib(serial).or_cic_assign(N, box, pos.shape[0], _f(pos), mp, _d(m))
    return m


def density_contrast(m, serial=None):
    m = np.ascontiguousarray(m, np.float64)
    d = np.empty_like(m)
    lib(serial).or_delta(m.shape[0], _d(m), _d(d))
    return d


def source(p, delta):
    delta = np.ascontiguousarray(delta, np.float64)
    f = np.empty_like(delta)
    lib().or_source(C.byref(p), _d(delta), _d(f))
    return f


def screened_guess(p, delta):
    """Initial guess from the screened limit of the field equation (local balance)."""
    delta = np.ascontiguousarray(delta, np.float64)
    u = np.empty_like(delta)
    lib().or_screened_guess(C.byref(p), _d(delta), _d(u))
    return u


def effective_density(p, delta, u):
    """delta rho_eff / rho_bar of the effective-mass formulation (Sec. 3.4)."""
    delta = np.ascontiguousarray(delta, np.float64)
    u = np.ascontiguousarray(u, np.float64)
    out = np.empty_like(delta)
    lib().or_effective_density(C.byref(p), _d(delta), _d(u), _d(out))
    return out


def power_ratio(box, delta, delta_eff, nbins):
    """Shell power spectra by the definition (numpy's real FFT as the transform):
    returns k_i, P_{delta+delta_eff}/P_delta, P_delta and the mode count per shell,
    shell i = integer wave vectors n with round(|n|) = i, i = 1..nbins."""
    delta = np.asarray(delta, np.float64)
    N = delta.shape[0]
    F1 = np.fft.rfftn(delta)
    F2 = np.fft.rfftn(delta + np.asarray(delta_eff, np.float64))
    n1 = np.fft.fftfreq(N, 1.0 / N)
    nz = np.arange(N // 2 + 1)
    n2 = n1[:, None, None] ** 2 + n1[None, :, None] ** 2 + nz[None, None, :] ** 2
    shell = np.floor(np.sqrt(n2) + 0.5).astype(np.int64)
    w = np.where((nz == 0) | (nz == N // 2), 1.0, 2.0)[None, None, :] * np.ones_like(n2)
    s1 = np.bincount(shell.ravel(), (w * np.abs(F1) ** 2).ravel(), minlength=nbins + 1)[1:nbins + 1]
    s2 = np.bincount(shell.ravel(), (w * np.abs(F2) ** 2).ravel(), minlength=nbins + 1)[1:nbins + 1]
    cnt = np.bincount(shell.ravel(), w.ravel(), minlength=nbins + 1)[1:nbins + 1]
    k = 2 * np.pi * np.arange(1, nbins + 1) / box
    ratio = np.where(s1 > 0, s2 / np.where(s1 > 0, s1, 1), 0.0)
    p = np.where(cnt > 0, box ** 3 / N ** 6 * s1 / np.where(cnt > 0, cnt, 1), 0.0)
    return k, ratio, p, cnt


def apply_L(u, h, bC, n=1):
    u = np.ascontiguousarray(u, np.float64)
    out = np.empty_like(u)
    lib().or_apply_L(u.shape[0], h, bC, n, _d(u), _d(out))
    return out


def apply_J(u, h, bC, n=1):
    u = np.ascontiguousarray(u, np.float64)
    out = np.empty_like(u)
    lib().or_apply_J(u.shape[0], h, bC, n, _d(u), _d(out))
    return out


def residual_max(u, f, h, bC, n=1):
    u = np.ascontiguousarray(u, np.float64)
    f = np.ascontiguousarray(f, np.float64)
    return lib().or_residual_max(u.shape[0], h, bC, n, _d(u), _d(f))


def ngs_sweep(u, f, h, bC, n=1, max_du=2.0):
    """One red+black sweep; returns a new array."""
    u = np.array(u, dtype=np.float64, order="C", copy=True)
    f = np.ascontiguousarray(f, np.float64)
    lib().or_ngs_sweep(u.shape[0], h, bC, n, max_du, _d(u), _d(f))
    return u


def restrict(fine):
    fine = np.ascontiguousarray(fine, np.float64)
    N = fine.shape[0] // 2
    c = np.empty((N, N, N), np.float64)
    lib().or_restrict(fine.shape[0], _d(fine), _d(c))
    return c


def prolong_add(u, uc, ubar, mode=0):
    u = np.array(u, dtype=np.float64, order="C", copy=True)
    lib().or_prolong_add(u.shape[0], mode, _d(np.ascontiguousarray(uc, np.float64)),
                         _d(np.ascontiguousarray(ubar, np.float64)), _d(u))
    return u


def num_levels(N):
    return lib().or_num_levels(N)


def solve(p, delta, u0=None, want_dfr=True, serial=None):
    """Returns (status, u, dfr, stats)."""
    delta = np.ascontiguousarray(delta, np.float64)
    N = p.mesh
    u = np.zeros((N, N, N), np.float64) if u0 is None else np.array(u0, np.float64, order="C", copy=True)
    dfr = np.empty_like(u) if want_dfr else None
    st = Stats()
    s = lib(serial).or_solve(C.byref(p), _d(delta), _d(u), _d(dfr) if want_dfr else None, C.byref(st))
    return s, u, dfr, st


def vcycle_once(p, f, u):
    u = np.array(u, dtype=np.float64, order="C", copy=True)
    lib().or_vcycle_once(C.byref(p), _d(np.ascontiguousarray(f, np.float64)), _d(u))
    return u


def fifth_force(p, u, pos, serial=None):
    pos = np.ascontiguousarray(pos, np.float32)
    u = np.ascontiguousarray(u, np.float64)
    acc = np.empty((pos.shape[0], 3), np.float64)
    lib(serial).or_fifth_force(C.byref(p), _d(u), pos.shape[0], _f(pos), _d(acc))
    return acc


def _i64(a):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def residual_at(u, f, h, bC, cells, n=1):
    """f - L(u) at the flat cell indices ``cells`` (arrays may be any C-contiguous N^3 float64)."""
    u = np.ascontiguousarray(u, np.float64)
    f = np.ascontiguousarray(f, np.float64)
    cells = np.ascontiguousarray(cells, np.int64)
    out = np.empty(cells.size, np.float64)
    lib().or_residual_at(u.shape[0], h, bC, n, _d(u), _d(f), cells.size, _i64(cells), _d(out))
    return out


def cic_cells(N, box, pos, cells, mass=None):
    pos = np.ascontiguousarray(pos, np.float32)
    cells = np.ascontiguousarray(cells, np.int64)
    mark = np.empty(N ** 3, np.uint8)
    out = np.empty(cells.size, np.float64)
    mp = None if mass is None else _d(np.ascontiguousarray(mass, np.float64))
    lib().or_cic_cells(N, box, pos.shape[0], _f(pos), mp, cells.size, _i64(cells),
                       mark.ctypes.data_as(C.c_void_p), _d(out))
    return out


def fifth_force_at(p, u, pos):
    pos = np.ascontiguousarray(pos, np.float32)
    u = np.ascontiguousarray(u, np.float64)
    acc = np.empty((pos.shape[0], 3), np.float64)
    lib().or_fifth_force_at(C.byref(p), _d(u), pos.shape[0], _f(pos), _d(acc))
    return acc


def amr_solve(p, nref, pos):
    """Base solve plus ``nref`` refined levels; returns (status, [u_l], [mask_l], [stats_l])."""
    pos = np.ascontiguousarray(pos, np.float32)
    N0 = p.mesh
    us = [np.zeros((N0 << l,) * 3, np.float64) for l in range(nref + 1)]
    ms = [np.zeros((N0 << l,) * 3, np.uint8) for l in range(nref + 1)]
    up = (C.POINTER(C.c_double) * (nref + 1))(*[_d(a) for a in us])
    mp = (C.c_void_p * (nref + 1))(*[a.ctypes.data_as(C.c_void_p) for a in ms])
    st = (Stats * (nref + 1))()
    s = lib().or_amr_solve(C.byref(p), nref, pos.shape[0], _f(pos), up, mp, st)
    return s, us, ms, list(st)


def _blk_ptrs(blk):
    """blk: list indexed by level (entry 0 unused) of uint8 block maps."""
    arrs = [None] + [np.ascontiguousarray(b, np.uint8) for b in blk[1:]]
    ptrs = (C.c_void_p * len(arrs))(None, *[a.ctypes.data_as(C.c_void_p) for a in arrs[1:]])
    return arrs, ptrs


def amr_flags(p, nref, pos):
    """Block maps [None, blk1, blk2] ((N_l/8)^3 uint8) from nearest-grid-point counts and nesting."""
    pos = np.ascontiguousarray(pos, np.float32)
    N0 = p.mesh
    blk = [None] + [np.zeros(((N0 << l) // 8,) * 3, np.uint8) for l in range(1, nref + 1)]
    _, ptrs = _blk_ptrs(blk)
    lib().or_amr_flags(C.byref(p), nref, pos.shape[0], _f(pos), ptrs)
    return blk


def amr_cic(p, nref, blk, pos, mass=None):
    """Composite cloud-in-cell masses [m_0 .. m_nref] (Sec. 3.1) on the levels of ``blk``."""
    pos = np.ascontiguousarray(pos, np.float32)
    N0 = p.mesh
    ms = [np.zeros((N0 << l,) * 3, np.float64) for l in range(nref + 1)]
    arrs, ptrs = _blk_ptrs(blk)
    mp = (C.POINTER(C.c_double) * (nref + 1))(*[_d(a) for a in ms])
    mass_p = None if mass is None else _d(np.ascontiguousarray(mass, np.float64))
    lib().or_amr_cic(C.byref(p), nref, ptrs, pos.shape[0], _f(pos), mass_p, mp)
    return ms


def amr_solve_fields(p, nref, blk, deltas):
    """Adaptive solve for given per-level density contrasts; returns (status, [u_l], [mask_l], [stats_l])."""
    N0 = p.mesh
    ds = [np.ascontiguousarray(d, np.float64) for d in deltas]
    us = [np.zeros((N0 << l,) * 3, np.float64) for l in range(nref + 1)]
    ms = [np.zeros((N0 << l,) * 3, np.uint8) for l in range(nref + 1)]
    arrs, ptrs = _blk_ptrs(blk)
    dp_ = (C.POINTER(C.c_double) * (nref + 1))(*[_d(a) for a in ds])
    up = (C.POINTER(C.c_double) * (nref + 1))(*[_d(a) for a in us])
    mp = (C.c_void_p * (nref + 1))(*[a.ctypes.data_as(C.c_void_p) for a in ms])
    st = (Stats * (nref + 1))()
    s = lib().or_amr_solve_fields(C.byref(p), nref, ptrs, dp_, up, mp, st)
    return s, us, ms, list(st)


def amr_cic_cells(p, nref, blk, pos, levels, ijk, mass=None):
    """Composite CIC masses of listed cells (level, i, j, k) from the given particles."""
    pos = np.ascontiguousarray(pos, np.float32)
    lev = np.ascontiguousarray(levels, np.int32)
    ijk = np.ascontiguousarray(ijk, np.int32).reshape(-1, 3)
    out = np.zeros(lev.size, np.float64)
    arrs, ptrs = _blk_ptrs(blk)
    mass_p = None if mass is None else _d(np.ascontiguousarray(mass, np.float64))
    lib().or_amr_cic_cells(C.byref(p), nref, ptrs, pos.shape[0], _f(pos), mass_p, lev.size,
                           lev.ctypes.data_as(C.c_void_p), ijk.ctypes.data_as(C.c_void_p), _d(out))
    return out


def op_stencil(h, bC, uc, nb, n=1):
    """The operator L at cells given their value uc [count] and neighbours nb [count, 6] (+x,-x,+y,-y,+z,-z)."""
    uc = np.ascontiguousarray(uc, np.float64)
    nb = np.ascontiguousarray(nb, np.float64).reshape(-1, 6)
    out = np.empty(uc.size, np.float64)
    lib().or_op_stencil(h, bC, n, uc.size, _d(uc), _d(nb), _d(out))
    return out


# ------------------------------------------------------ chained particle-mesh steps

H0 = 100.0  # km/s per Mpc/h


def hubble(a, omega_m, omega_l):
    """H(a) of flat LCDM in km/s per Mpc/h."""
    return H0 * np.sqrt(omega_m / a ** 3 + omega_l)


def pm_potential(box, a, omega_m, delta):
    """phi with lap phi = (3/2) Omega_m H0^2 delta / a for the periodic 7-point
    Laplacian, by the definition: divide each Fourier mode by the stencil's
    eigenvalue -(4/h^2) sum_d sin^2(pi n_d / N) (numpy's FFT as the transform);
    the k = 0 mode of phi is zero."""
    delta = np.asarray(delta, np.float64)
    N = delta.shape[0]
    h = box / N
    F = np.fft.rfftn(delta)
    n = np.fft.fftfreq(N) * N
    nz = np.arange(N // 2 + 1)
    s2 = (np.sin(np.pi * n / N) ** 2)[:, None, None] + (np.sin(np.pi * n / N) ** 2)[None, :, None] \
        + (np.sin(np.pi * nz / N) ** 2)[None, None, :]
    lam = -4.0 / h ** 2 * s2
    lam[0, 0, 0] = 1.0
    G = 1.5 * omega_m * H0 ** 2 / a / lam
    G[0, 0, 0] = 0.0
    return np.fft.irfftn(F * G, s=delta.shape, axes=(0, 1, 2))


def gather_gradient(box, field, pos, pref):
    field = np.ascontiguousarray(field, np.float64)
    pos = np.ascontiguousarray(pos, np.float32)
    acc = np.empty((pos.shape[0], 3), np.float64)
    lib().or_gather_gradient(field.shape[0], box, _d(field), pos.shape[0], _f(pos), pref, _d(acc))
    return acc


def pm_accel(p, delta, u, pos):
    """-(1/a) grad (phi + (c^2/2) |fbar| e^u) at the particles (u None: phi alone)."""
    fb, _, _ = background(p)
    psi = pm_potential(p.box, p.a, p.omega_m, delta)
    if u is not None:
        psi = psi + 0.5 * C_KMS ** 2 * fb * np.exp(np.asarray(u, np.float64))
    return gather_gradient(p.box, psi, pos, -1.0 / p.a)


def kick_drift(pos, mom, acc, kick, drift, box):
    """In place on float32 arrays [np, 3]."""
    assert pos.dtype == np.float32 and mom.dtype == np.float32 and pos.flags.c_contiguous and mom.flags.c_contiguous
    ap = None if acc is None else _f(np.ascontiguousarray(acc, np.float32))
    lib().or_kick_drift(pos.shape[0], _f(pos), _f(mom), ap, kick, drift, box)


def pm_step(p, pos, mom, acc, a1, u):
    """One kick-drift-kick step from a = p.a to a1 (midpoint-rule kick and
    drift integrals of dp/da = g/H, dx/da = p/(a^3 H)); the solve at a1 starts
    from u (the previous step's solution).  pos, mom (float32) are updated in
    place; returns (delta, u, acc32, stats) at a1 and sets p.a = a1."""
    a0 = p.a
    am = 0.5 * (a0 + a1)
    H = lambda a: hubble(a, p.omega_m, p.omega_l)
    K1 = (am - a0) / H(0.5 * (a0 + am))
    D = (a1 - a0) / (am ** 3 * H(am))
    K2 = (a1 - am) / H(0.5 * (am + a1))
    kick_drift(pos, mom, acc, K1, D, p.box)
    p.a = a1
    delta = density_contrast(cic_assign(p.mesh, p.box, pos))
    s, u1, _, st = solve(p, delta, u0=u, want_dfr=False)
    acc1 = pm_accel(p, delta, u1, pos).astype(np.float32)
    kick_drift(pos, mom, acc1, K2, 0.0, p.box)
    return delta, u1, acc1, st


def amr_levels(p, nref, pos):
    """The adaptive solve step by step (flags, composite masses, delta_l =
    m_l / (total / N_l^3) - 1, field-driven solve): returns
    (status, blk, [delta_l], [u_l], [mask_l], [stats_l])."""
    blk = amr_flags(p, nref, pos)
    ms = amr_cic(p, nref, blk, pos)
    total = ms[0].sum()
    deltas = [m / (total / m.size) - 1.0 for m in ms]
    s, us, masks, st = amr_solve_fields(p, nref, blk, deltas)
    return s, blk, deltas, us, masks, st


def amr_composite(p, deltas, us, masks):
    """delta and the effective density (Sec. 3.4) of the finest level covering
    each cell, on the finest level's uniform mesh (a coarser leaf's value fills
    its sub-cells)."""
    fb, beta, C = background(p)
    om = p.omega_m / p.a ** 3
    q = 1.0 / (p.n + 1)
    L = len(deltas) - 1
    Nf = deltas[L].shape[0]
    d = np.empty((Nf,) * 3)
    u = np.empty((Nf,) * 3)
    have = np.zeros((Nf,) * 3, bool)
    for l in range(L, -1, -1):
        r = 1 << (L - l)
        up = lambda a: np.repeat(np.repeat(np.repeat(a, r, 0), r, 1), r, 2)
        m = up(masks[l].astype(bool)) & ~have
        d[m] = up(deltas[l])[m]
        u[m] = up(us[l])[m]
        have |= m
    assert have.all()
    return d, d / 3.0 - C * np.expm1(-q * u) / (3.0 * om)
