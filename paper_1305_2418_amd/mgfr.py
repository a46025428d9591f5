"""Thin ctypes binding of the HIP library ``libmgfr.so`` (C ABI in include/mgfr.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Arrays are torch tensors on the HIP device; the binding checks
dtype, shape, contiguity and device, passes raw pointers and the current
torch stream, and turns negative return codes into exceptions.  There is no
CPU fallback: a missing library raises at import of the first call.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmgfr.so")

MGFR_OK, MGFR_NOT_CONVERGED = 0, 1
MGFR_ERR_ARG, MGFR_ERR_HIP, MGFR_ERR_NONFINITE, MGFR_ERR_OOM = -1, -2, -3, -4
PROLONG_LINEAR, PROLONG_INJECT = 0, 1
FP64, MIXED = 0, 1
NN_NONE, NN_COARSE = 0, 1
MAX_HIST = 256


class MgfrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mgfr error {code}: {msg}")
        self.code = code


class _Params(C.Structure):
    _fields_ = [("box", C.c_double), ("a", C.c_double), ("omega_m", C.c_double),
                ("omega_l", C.c_double), ("fr0_abs", C.c_double), ("n", C.c_int),
                ("mesh", C.c_int), ("refine_levels", C.c_int), ("tol", C.c_double),
                ("pre_smooth", C.c_int), ("post_smooth", C.c_int), ("coarse_sweeps", C.c_int),
                ("max_vcycles", C.c_int), ("prolong", C.c_int), ("precision", C.c_int),
                ("nn_mode", C.c_int), ("max_du", C.c_double), ("coarse_cycles", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("status", C.c_int), ("vcycles", C.c_int), ("outer_iters", C.c_int),
                ("fell_back", C.c_int), ("res0", C.c_double), ("res", C.c_double),
                ("scale", C.c_double), ("l2res", C.c_double), ("res_hist", C.c_double * MAX_HIST),
                ("t_solve_ms", C.c_double), ("t_sweep_ms", C.c_double),
                ("n_sweep_launches", C.c_int), ("t_nn_ms", C.c_double), ("smooth_used", C.c_int)]


@dataclass
class Params:
    """Mirror of ``mgfr_params`` (defaults: the paper's model, V(2,2), tol 1e-8)."""
    mesh: int = 32
    box: float = 100.0
    a: float = 1.0
    omega_m: float = 0.3
    omega_l: float = 0.7
    fr0_abs: float = 1e-5
    n: int = 1
    refine_levels: int = 0
    tol: float = 1e-8
    pre_smooth: int = 2
    post_smooth: int = 2
    coarse_sweeps: int = 30
    max_vcycles: int = 100
    prolong: int = PROLONG_LINEAR
    precision: int = FP64
    nn_mode: int = NN_NONE
    max_du: float = 2.0
    coarse_cycles: int = 0

    def to_c(self) -> _Params:
        return _Params(self.box, self.a, self.omega_m, self.omega_l, self.fr0_abs, self.n,
                       self.mesh, self.refine_levels, self.tol, self.pre_smooth, self.post_smooth,
                       self.coarse_sweeps, self.max_vcycles, self.prolong, self.precision,
                       self.nn_mode, self.max_du, self.coarse_cycles)


@dataclass
class Stats:
    status: int = 0
    vcycles: int = 0
    outer_iters: int = 0
    fell_back: int = 0
    res0: float = 0.0
    res: float = 0.0
    scale: float = 0.0
    l2res: float = 0.0
    res_hist: list = field(default_factory=list)
    t_solve_ms: float = 0.0
    t_sweep_ms: float = 0.0
    n_sweep_launches: int = 0
    t_nn_ms: float = 0.0
    smooth_used: int = 0

    @classmethod
    def from_c(cls, s: _Stats) -> "Stats":
        n = min(s.outer_iters, MAX_HIST)  # one entry per residual check
        return cls(s.status, s.vcycles, s.outer_iters, s.fell_back, s.res0, s.res, s.scale,
                   s.l2res, list(s.res_hist[:n]), s.t_solve_ms, s.t_sweep_ms,
                   s.n_sweep_launches, s.t_nn_ms, s.smooth_used)


_lib = None
_VP = C.c_void_p


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                              "or python paper_1305_2418_amd/build.py")
        L = C.CDLL(LIB_PATH)
        L.mgfr_last_error.restype = C.c_char_p
        L.mgfr_background.argtypes = [C.POINTER(_Params), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.mgfr_create.argtypes = [C.POINTER(_Params), _VP, C.POINTER(_VP)]
        L.mgfr_destroy.argtypes = [_VP]
        L.mgfr_destroy.restype = None
        L.mgfr_set_stream.argtypes = [_VP, _VP]
        L.mgfr_set_timing.argtypes = [_VP, C.c_int]
        L.mgfr_set_fused_min_mesh.argtypes = [_VP, C.c_int]
        L.mgfr_set_colour_min_mesh.argtypes = [_VP, C.c_int]
        L.mgfr_set_fused_sweep32.argtypes = [_VP, C.c_int]
        L.mgfr_set_relaxation32.argtypes = [_VP, C.c_double]
        L.mgfr_set_inner_cycles.argtypes = [_VP, C.c_int]
        L.mgfr_set_adaptive_smoothing.argtypes = [_VP, C.c_int]
        L.mgfr_screened_guess.argtypes = [_VP, _VP, _VP]
        L.mgfr_effective_density.argtypes = [_VP, _VP, _VP, _VP]
        L.mgfr_power_ratio.argtypes = [_VP, _VP, _VP, C.c_int, _VP, _VP, _VP, _VP]
        L.mgfr_assign_density.argtypes = [_VP, _VP, _VP, C.c_int64, _VP]
        L.mgfr_assign_density_noalloc.argtypes = [C.c_int, C.c_double, _VP, _VP, _VP, C.c_int64, _VP]
        L.mgfr_reserve_particles.argtypes = [_VP, C.c_int64]
        L.mgfr_set_binning.argtypes = [_VP, C.c_int]
        L.mgfr_solve.argtypes = [_VP, _VP, _VP, _VP, C.POINTER(_Stats)]
        L.mgfr_fifth_force.argtypes = [_VP, _VP, _VP, C.c_int64, _VP]
        L.mgfr_set_scale_factor.argtypes = [_VP, C.c_double]
        L.mgfr_pm_accel.argtypes = [_VP, _VP, _VP, _VP, C.c_int64, _VP]
        L.mgfr_kick_drift.argtypes = [_VP, _VP, _VP, _VP, C.c_int64, C.c_double, C.c_double]
        L.mgfr_pm_step.argtypes = [_VP, _VP, _VP, _VP, C.c_int64, C.c_double, _VP, _VP, C.POINTER(_Stats)]
        L.mgfr_ngs_sweep.argtypes = [_VP, _VP, _VP, C.c_int]
        L.mgfr_vcycle.argtypes = [_VP, _VP, _VP]
        L.mgfr_residual.argtypes = [_VP, _VP, _VP, _VP]
        L.mgfr_net_create.argtypes = [C.c_int, C.c_int64, _VP, C.POINTER(_VP)]
        L.mgfr_net_destroy.argtypes = [_VP]
        L.mgfr_net_destroy.restype = None
        L.mgfr_net_set_stream.argtypes = [_VP, _VP]
        L.mgfr_net_num_params.argtypes = [_VP]
        L.mgfr_net_num_params.restype = C.c_int64
        L.mgfr_net_get_params.argtypes = [_VP, _VP]
        L.mgfr_net_set_params.argtypes = [_VP, _VP]
        L.mgfr_net_save.argtypes = [_VP, C.c_char_p]
        L.mgfr_net_load.argtypes = [_VP, C.c_char_p]
        L.mgfr_net_predict.argtypes = [_VP, _VP, C.c_int, C.c_int, _VP, _VP]
        L.mgfr_net_activation.argtypes = [_VP, C.c_int, _VP, C.c_int64]
        L.mgfr_net_train_step.argtypes = [_VP, _VP, _VP, C.c_int, C.c_int, _VP, C.c_float,
                                          C.POINTER(C.c_float)]
        L.mgfr_net_grads.argtypes = [_VP, _VP, _VP, C.c_int, C.c_int, _VP, C.POINTER(C.c_float), _VP]
        L.mgfr_set_net.argtypes = [_VP, _VP]
        L.mgfr_nn_init.argtypes = [_VP, C.c_int]
        L.mgfr_nn_train_step.argtypes = [_VP, _VP, _VP, C.c_int, C.c_int, _VP, C.c_float, C.POINTER(C.c_float)]
        L.mgfr_nn_predict.argtypes = [_VP, _VP, _VP]
        L.mgfr_nn_save.argtypes = [_VP, C.c_char_p]
        L.mgfr_nn_load.argtypes = [_VP, C.c_char_p]
        L.mgfr_conv3d_fwd.argtypes = [_VP, C.c_int, C.c_int, C.c_int, _VP, _VP, C.c_int, C.c_int, _VP, _VP, _VP]
        L.mgfr_conv3d_bwd_data.argtypes = [_VP, C.c_int, C.c_int, C.c_int, _VP, C.c_int, _VP, _VP, _VP]
        L.mgfr_conv3d_bwd_weight.argtypes = [_VP, _VP, C.c_int, C.c_int, C.c_int, C.c_int, _VP, _VP, _VP]
        L.mgfr_amr_create.argtypes = [C.POINTER(_Params), C.c_int64, _VP, C.POINTER(_VP)]
        L.mgfr_amr_destroy.argtypes = [_VP]
        L.mgfr_amr_destroy.restype = None
        L.mgfr_amr_set_relaxation32.argtypes = [_VP, C.c_double]
        L.mgfr_amr_solve.argtypes = [_VP, _VP, C.c_int64, _VP, _VP]
        L.mgfr_amr_reserve_particles.argtypes = [_VP, C.c_int64]
        L.mgfr_amr_num_blocks.argtypes = [_VP, C.c_int]
        L.mgfr_amr_num_blocks.restype = C.c_int64
        L.mgfr_amr_get_level.argtypes = [_VP, C.c_int, _VP, _VP]
        L.mgfr_amr_composite.argtypes = [_VP, _VP, _VP]
        _lib = L
    return _lib


def exported_symbols():
    """Names declared by include/mgfr.h (checked against the built library by the tests)."""
    import re
    hdr = open(os.path.join(os.path.dirname(_PKG), "include", "mgfr.h")).read()
    return sorted(set(re.findall(r"\b(mgfr_[a-z0-9_]+)\s*\(", hdr)))


def _check(rc: int, allow_not_converged: bool = False) -> int:
    if rc < 0 or (rc == MGFR_NOT_CONVERGED and not allow_not_converged):
        msg = lib().mgfr_last_error().decode(errors="replace")
        raise MgfrError(rc, msg)
    return rc


def _stream_ptr():
    return torch.cuda.current_stream().cuda_stream


def _dev(t: torch.Tensor, dtype, shape, name, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a torch tensor on the HIP device")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def background(p: Params):
    fb, beta, Cc = C.c_double(), C.c_double(), C.c_double()
    pc = p.to_c()
    _check(lib().mgfr_background(C.byref(pc), C.byref(fb), C.byref(beta), C.byref(Cc)))
    return fb.value, beta.value, Cc.value


def assign_density_noalloc(pos: torch.Tensor, mesh: int, box: float, mass: torch.Tensor | None = None,
                           out: torch.Tensor | None = None) -> torch.Tensor:
    """Context-free CIC assignment whose library side allocates nothing (its
    workspace is a fixed device array); ``out`` may be passed pre-allocated."""
    if pos.dim() != 2 or pos.shape[1] != 3:
        raise ValueError("pos must be [np, 3]")
    npart = pos.shape[0]
    shape = (mesh, mesh, mesh)
    pp = _dev(pos, torch.float32, None, "pos")
    mp = _dev(mass, torch.float64, (npart,), "mass", allow_none=True)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=pos.device)
    op = _dev(out, torch.float64, shape, "delta")
    _check(lib().mgfr_assign_density_noalloc(int(mesh), float(box), _stream_ptr(), pp, mp, npart, op))
    return out


class Solver:
    """One mgfr context: the level hierarchy for an N^3 mesh on the current device."""

    def __init__(self, params: Params, stream=None, binning: bool = True):
        self.params = params
        self._p = params.to_c()
        h = _VP()
        s = _stream_ptr() if stream is None else stream
        _check(lib().mgfr_create(C.byref(self._p), s, C.byref(h)))
        self._h = h
        self.N = params.mesh
        self._binning = bool(binning)
        self._bin_cap = 0
        _check(lib().mgfr_set_binning(h, 1 if binning else 0))

    def close(self):
        if getattr(self, "_h", None):
            lib().mgfr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        _check(lib().mgfr_set_stream(self._h, _stream_ptr()))

    @property
    def shape(self):
        return (self.N, self.N, self.N)

    def set_timing(self, on: bool):
        _check(lib().mgfr_set_timing(self._h, 1 if on else 0))

    def set_fused_min_mesh(self, n: int):
        _check(lib().mgfr_set_fused_min_mesh(self._h, int(n)))

    def set_colour_min_mesh(self, n: int):
        _check(lib().mgfr_set_colour_min_mesh(self._h, int(n)))

    def set_relaxation32(self, omega: float):
        """Over-relaxation factor of the float32 correction sweeps (mixed solve)."""
        _check(lib().mgfr_set_relaxation32(self._h, float(omega)))

    def set_adaptive_smoothing(self, max_sweeps: int):
        """Double the smoothing sweeps (up to max_sweeps) when the residual stalls; 0: off."""
        _check(lib().mgfr_set_adaptive_smoothing(self._h, int(max_sweeps)))

    def set_inner_cycles(self, max_inner: int):
        """Float32 correction V-cycles per float64 residual check of the mixed solve (at most)."""
        _check(lib().mgfr_set_inner_cycles(self._h, int(max_inner)))

    def set_fused_sweep32(self, on: bool):
        """Float32 correction sweeps as one fused red-black kernel per sweep."""
        _check(lib().mgfr_set_fused_sweep32(self._h, int(bool(on))))

    def reserve_particles(self, max_np: int):
        """Allocate the particle-binning workspace for up to max_np particles."""
        self._sync_stream()
        _check(lib().mgfr_reserve_particles(self._h, int(max_np)))
        self._bin_cap = max(self._bin_cap, int(max_np))

    def set_binning(self, on: bool):
        self._binning = bool(on)
        _check(lib().mgfr_set_binning(self._h, 1 if on else 0))

    def assign_density(self, pos: torch.Tensor, mass: torch.Tensor | None = None,
                       out: torch.Tensor | None = None) -> torch.Tensor:
        self._sync_stream()
        if pos.dim() != 2 or pos.shape[1] != 3:
            raise ValueError("pos must be [np, 3]")
        npart = pos.shape[0]
        if self._binning and self._bin_cap < npart < 2 ** 31:
            self.reserve_particles(npart)
        pp = _dev(pos, torch.float32, None, "pos")
        mp = _dev(mass, torch.float64, (npart,), "mass", allow_none=True)
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=pos.device)
        op = _dev(out, torch.float64, self.shape, "delta")
        _check(lib().mgfr_assign_density(self._h, pp, mp, npart, op))
        return out

    def screened_guess(self, delta: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Initial guess from the screened limit (local balance) of the field equation."""
        self._sync_stream()
        dp = _dev(delta, torch.float64, self.shape, "delta")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=delta.device)
        up = _dev(out, torch.float64, self.shape, "u")
        _check(lib().mgfr_screened_guess(self._h, dp, up))
        return out

    def effective_density(self, delta: torch.Tensor, u: torch.Tensor, out: torch.Tensor | None = None):
        """delta rho_eff / rho_bar (Sec. 3.4) from delta and the solved u."""
        self._sync_stream()
        dp = _dev(delta, torch.float64, self.shape, "delta")
        up = _dev(u, torch.float64, self.shape, "u")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=delta.device)
        op = _dev(out, torch.float64, self.shape, "out")
        _check(lib().mgfr_effective_density(self._h, dp, up, op))
        return out

    def power_ratio(self, delta: torch.Tensor, delta_eff: torch.Tensor, nbins: int | None = None):
        """(k, P_{delta+delta_eff}/P_delta, P_delta, modes) per |k| shell (numpy arrays)."""
        import numpy as np
        self._sync_stream()
        nb = self.shape[0] // 2 if nbins is None else int(nbins)
        dp = _dev(delta, torch.float64, self.shape, "delta")
        ep = _dev(delta_eff, torch.float64, self.shape, "delta_eff")
        out = [np.zeros(nb) for _ in range(4)]
        _check(lib().mgfr_power_ratio(self._h, dp, ep, nb, *[o.ctypes.data_as(C.c_void_p) for o in out]))
        return tuple(out)

    def solve(self, delta: torch.Tensor, u: torch.Tensor | None = None, want_dfr: bool = True,
              allow_not_converged: bool = False):
        """Returns (u, dfr or None, Stats); u is updated in place if given."""
        self._sync_stream()
        dp = _dev(delta, torch.float64, self.shape, "delta")
        if u is None:
            u = torch.zeros(self.shape, dtype=torch.float64, device=delta.device)
        up = _dev(u, torch.float64, self.shape, "u")
        dfr = torch.empty_like(u) if want_dfr else None
        st = _Stats()
        rc = lib().mgfr_solve(self._h, dp, up, dfr.data_ptr() if want_dfr else None, C.byref(st))
        _check(rc, allow_not_converged=allow_not_converged)
        return u, dfr, Stats.from_c(st)

    def fifth_force(self, u: torch.Tensor, pos: torch.Tensor, out: torch.Tensor | None = None):
        self._sync_stream()
        npart = pos.shape[0]
        up = _dev(u, torch.float64, self.shape, "u")
        pp = _dev(pos, torch.float32, (npart, 3), "pos")
        if out is None:
            out = torch.empty((npart, 3), dtype=torch.float32, device=pos.device)
        ap = _dev(out, torch.float32, (npart, 3), "acc")
        _check(lib().mgfr_fifth_force(self._h, up, pp, npart, ap))
        return out

    def set_scale_factor(self, a: float):
        _check(lib().mgfr_set_scale_factor(self._h, float(a)))
        self.params.a = float(a)

    def pm_accel(self, delta: torch.Tensor, u: torch.Tensor | None, pos: torch.Tensor, out: torch.Tensor | None = None):
        """Peculiar acceleration -(1/a) grad (phi + (c^2/2) fbar e^u) at the particles (float32 [np, 3])."""
        self._sync_stream()
        npart = pos.shape[0]
        dp = _dev(delta, torch.float64, self.shape, "delta")
        up = _dev(u, torch.float64, self.shape, "u", allow_none=True)
        pp = _dev(pos, torch.float32, (npart, 3), "pos")
        if out is None:
            out = torch.empty((npart, 3), dtype=torch.float32, device=pos.device)
        ap = _dev(out, torch.float32, (npart, 3), "acc")
        _check(lib().mgfr_pm_accel(self._h, dp, up, pp, npart, ap))
        return out

    def kick_drift(self, pos: torch.Tensor, mom: torch.Tensor, acc: torch.Tensor | None, kick: float, drift: float):
        """mom += acc kick; pos += mom drift (in place, float32 [np, 3])."""
        self._sync_stream()
        npart = pos.shape[0]
        pp = _dev(pos, torch.float32, (npart, 3), "pos")
        mp = _dev(mom, torch.float32, (npart, 3), "mom")
        ap = _dev(acc, torch.float32, (npart, 3), "acc", allow_none=True)
        _check(lib().mgfr_kick_drift(self._h, pp, mp, ap, npart, float(kick), float(drift)))

    def pm_step(self, pos, mom, acc, a1: float, delta, u, allow_not_converged: bool = True):
        """One kick-drift-kick step to a1 (all arrays updated in place); returns the solve's Stats."""
        self._sync_stream()
        npart = pos.shape[0]
        args = [_dev(pos, torch.float32, (npart, 3), "pos"), _dev(mom, torch.float32, (npart, 3), "mom"),
                _dev(acc, torch.float32, (npart, 3), "acc")]
        dp = _dev(delta, torch.float64, self.shape, "delta")
        up = _dev(u, torch.float64, self.shape, "u")
        st = _Stats()
        rc = lib().mgfr_pm_step(self._h, *args, npart, float(a1), dp, up, C.byref(st))
        _check(rc, allow_not_converged=allow_not_converged)
        self.params.a = float(a1)
        return Stats.from_c(st)

    def set_net(self, net):
        _check(lib().mgfr_set_net(self._h, None if net is None else net._h))
        self._net = net

    # the context's own network (mgfr_nn_*)
    def nn_init(self, seed: int = 0):
        _check(lib().mgfr_nn_init(self._h, int(seed)))
        self._net = None

    def nn_train_step(self, delta: torch.Tensor, u_target: torch.Tensor, cond, lr: float) -> float:
        self._sync_stream()
        B, S = delta.shape[0], delta.shape[1]
        _dev(delta, torch.float64, (B, S, S, S), "delta")
        _dev(u_target, torch.float64, (B, S, S, S), "u_target")
        arr, cp = _cond_array(cond)
        loss = C.c_float()
        _check(lib().mgfr_nn_train_step(self._h, delta.data_ptr(), u_target.data_ptr(), B, S, cp, float(lr),
                                        C.byref(loss)))
        return loss.value

    def nn_predict(self, delta: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """The network's initial guess at N (prediction on N/4, prolonged twice)."""
        self._sync_stream()
        dp = _dev(delta, torch.float64, self.shape, "delta")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=delta.device)
        up = _dev(out, torch.float64, self.shape, "u0")
        _check(lib().mgfr_nn_predict(self._h, dp, up))
        return out

    def nn_save(self, path: str):
        _check(lib().mgfr_nn_save(self._h, os.fsencode(path)))

    def nn_load(self, path: str):
        _check(lib().mgfr_nn_load(self._h, os.fsencode(path)))

    def ngs_sweep(self, u: torch.Tensor, f: torch.Tensor, sweeps: int = 1):
        self._sync_stream()
        _check(lib().mgfr_ngs_sweep(self._h, _dev(u, torch.float64, self.shape, "u"),
                                    _dev(f, torch.float64, self.shape, "f"), sweeps))
        return u

    def vcycle(self, u: torch.Tensor, f: torch.Tensor):
        self._sync_stream()
        _check(lib().mgfr_vcycle(self._h, _dev(u, torch.float64, self.shape, "u"),
                                 _dev(f, torch.float64, self.shape, "f")))
        return u

    def residual(self, u: torch.Tensor, f: torch.Tensor):
        self._sync_stream()
        r = torch.empty_like(u)
        _check(lib().mgfr_residual(self._h, _dev(u, torch.float64, self.shape, "u"),
                                   _dev(f, torch.float64, self.shape, "f"),
                                   _dev(r, torch.float64, self.shape, "r")))
        return r


def _cond_array(cond):
    import numpy as np
    arr = np.ascontiguousarray(np.asarray(cond, dtype=np.float64).reshape(-1, 2))
    return arr, arr.ctypes.data_as(C.c_void_p)


class Net:
    """The learned warm-start network (weights, Adam state, workspace on the device)."""

    def __init__(self, seed: int = 0, max_voxels: int = 128 ** 3, stream=None):
        h = _VP()
        s = _stream_ptr() if stream is None else stream
        _check(lib().mgfr_net_create(int(seed), int(max_voxels), s, C.byref(h)))
        self._h = h
        self.max_voxels = max_voxels
        self._last = None  # (B, S, device) of the last predict()

    def close(self):
        if getattr(self, "_h", None):
            lib().mgfr_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync(self):
        _check(lib().mgfr_net_set_stream(self._h, _stream_ptr()))

    @property
    def num_params(self) -> int:
        return int(lib().mgfr_net_num_params(self._h))

    def get_params(self):
        import numpy as np
        out = np.empty(self.num_params, dtype=np.float32)
        _check(lib().mgfr_net_get_params(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.num_params:
            raise ValueError("wrong parameter count")
        _check(lib().mgfr_net_set_params(self._h, p.ctypes.data_as(C.c_void_p)))

    def save(self, path: str):
        """Checkpoint parameters and Adam state to a file."""
        _check(lib().mgfr_net_save(self._h, os.fsencode(path)))

    def load(self, path: str):
        """Restore parameters and Adam state written by save()."""
        _check(lib().mgfr_net_load(self._h, os.fsencode(path)))

    def predict(self, delta: torch.Tensor, cond) -> torch.Tensor:
        self._sync()
        B, S = delta.shape[0], delta.shape[1]
        _dev(delta, torch.float64, (B, S, S, S), "delta")
        u = torch.empty_like(delta)
        arr, cp = _cond_array(cond)
        if arr.shape[0] != B:
            raise ValueError("cond must have one (a, |f_R0|) row per volume")
        _check(lib().mgfr_net_predict(self._h, delta.data_ptr(), B, S, cp, u.data_ptr()))
        self._last = (B, S, delta.device)
        return u

    # (channels, pooling depth) of the tensors mgfr_net_activation exports, in forward order
    ACTIVATIONS = ((16, 0), (16, 0), (16, 0), (16, 1), (32, 1), (32, 1), (32, 2), (64, 2), (64, 2),
                   (96, 1), (32, 1), (32, 1), (48, 0), (16, 0), (16, 0), (1, 0))

    def activation(self, index: int) -> torch.Tensor:
        """Tensor `index` of the last predict(): bf16 [B, s, s, s, C] for 0-14, the head's
        float32 output [B, S, S, S] for 15."""
        if self._last is None:
            raise MgfrError(MGFR_ERR_ARG, "no predict() has run on this network yet")
        B, S, dev = self._last
        ch, depth = self.ACTIVATIONS[index]
        s = S >> depth
        if index == 15:
            out = torch.empty((B, S, S, S), dtype=torch.float32, device=dev)
        else:
            out = torch.empty((B, s, s, s, ch), dtype=torch.bfloat16, device=dev)
        _check(lib().mgfr_net_activation(self._h, int(index), out.data_ptr(), out.numel()))
        return out

    def train_step(self, delta: torch.Tensor, u_target: torch.Tensor, cond, lr: float) -> float:
        self._sync()
        B, S = delta.shape[0], delta.shape[1]
        _dev(delta, torch.float64, (B, S, S, S), "delta")
        _dev(u_target, torch.float64, (B, S, S, S), "u_target")
        arr, cp = _cond_array(cond)
        loss = C.c_float()
        _check(lib().mgfr_net_train_step(self._h, delta.data_ptr(), u_target.data_ptr(), B, S, cp,
                                         float(lr), C.byref(loss)))
        return loss.value

    def grads(self, delta: torch.Tensor, u_target: torch.Tensor, cond):
        import numpy as np
        self._sync()
        B, S = delta.shape[0], delta.shape[1]
        arr, cp = _cond_array(cond)
        g = np.empty(self.num_params, dtype=np.float32)
        loss = C.c_float()
        _check(lib().mgfr_net_grads(self._h, delta.data_ptr(), u_target.data_ptr(), B, S, cp, C.byref(loss),
                                    g.ctypes.data_as(C.c_void_p)))
        return loss.value, g


def conv3d_fwd(x: torch.Tensor, w: torch.Tensor, bias=None, relu=False, out32=False):
    """x bf16 [B,S,S,S,Cin], w bf16 [27,Cout,Cin] -> bf16 (or float32) [B,S,S,S,Cout]."""
    B, S, Cin = x.shape[0], x.shape[1], x.shape[-1]
    Cout = w.shape[1]
    _dev(x, torch.bfloat16, None, "x")
    _dev(w, torch.bfloat16, (27, Cout, Cin), "w")
    if bias is not None:
        _dev(bias, torch.float32, (Cout,), "bias")
    y = torch.empty((B, S, S, S, Cout), dtype=torch.float32 if out32 else torch.bfloat16, device=x.device)
    _check(lib().mgfr_conv3d_fwd(x.data_ptr(), B, S, Cin, w.data_ptr(),
                                 None if bias is None else bias.data_ptr(), Cout, 1 if relu else 0,
                                 None if out32 else y.data_ptr(), y.data_ptr() if out32 else None,
                                 _stream_ptr()))
    return y


def conv3d_bwd_data(dz: torch.Tensor, w: torch.Tensor):
    B, S, Cout = dz.shape[0], dz.shape[1], dz.shape[-1]
    Cin = w.shape[2]
    _dev(dz, torch.bfloat16, None, "dz")
    _dev(w, torch.bfloat16, (27, Cout, Cin), "w")
    work = torch.empty_like(w)
    dx = torch.empty((B, S, S, S, Cin), dtype=torch.bfloat16, device=dz.device)
    _check(lib().mgfr_conv3d_bwd_data(dz.data_ptr(), B, S, Cout, w.data_ptr(), Cin, work.data_ptr(),
                                      dx.data_ptr(), _stream_ptr()))
    return dx


def conv3d_bwd_weight(x: torch.Tensor, dz: torch.Tensor):
    B, S, Cin, Cout = x.shape[0], x.shape[1], x.shape[-1], dz.shape[-1]
    dw = torch.zeros((27, Cout, Cin), dtype=torch.float32, device=x.device)
    db = torch.zeros((Cout,), dtype=torch.float32, device=x.device)
    _check(lib().mgfr_conv3d_bwd_weight(x.data_ptr(), dz.data_ptr(), B, S, Cin, Cout, dw.data_ptr(),
                                        db.data_ptr(), _stream_ptr()))
    return dw, db


class Amr:
    """Base mesh plus block-refined levels (one-way interface)."""

    def __init__(self, params: Params, max_blocks: int = 65536, stream=None):
        if params.refine_levels < 1:
            raise ValueError("refine_levels must be 1 or 2")
        self.params = params
        self._p = params.to_c()
        h = _VP()
        s = _stream_ptr() if stream is None else stream
        _check(lib().mgfr_amr_create(C.byref(self._p), int(max_blocks), s, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().mgfr_amr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_relaxation32(self, omega: float):
        """Over-relaxation factor of the float32 correction sweeps (base and refined levels)."""
        _check(lib().mgfr_amr_set_relaxation32(self._h, float(omega)))

    def reserve_particles(self, max_np: int):
        """Workspace for the binned composite assignment of up to max_np particles (0 frees it)."""
        _check(lib().mgfr_amr_reserve_particles(self._h, int(max_np)))

    def solve(self, pos: torch.Tensor, allow_not_converged=False):
        """Returns (u0 [N0^3] tensor, [Stats per level])."""
        N0 = self.params.mesh
        npart = pos.shape[0]
        _dev(pos, torch.float32, (npart, 3), "pos")
        u0 = torch.empty((N0, N0, N0), dtype=torch.float64, device=pos.device)
        nl = self.params.refine_levels + 1
        sts = (_Stats * nl)()
        rc = lib().mgfr_amr_solve(self._h, pos.data_ptr(), npart, u0.data_ptr(), sts)
        _check(rc, allow_not_converged=allow_not_converged)
        return u0, [Stats.from_c(sts[i]) for i in range(nl)]

    def composite(self):
        """(delta, delta_eff) of the last solve on the finest level's uniform mesh."""
        Nf = self.params.mesh << self.params.refine_levels
        d = torch.empty((Nf, Nf, Nf), dtype=torch.float64, device="cuda")
        e = torch.empty_like(d)
        _check(lib().mgfr_amr_composite(self._h, d.data_ptr(), e.data_ptr()))
        return d, e

    def level(self, l: int):
        """(origins int32 [nb, 3] numpy, u float64 [nb, 8, 8, 8] tensor) of refined level l."""
        import numpy as np
        nb = int(lib().mgfr_amr_num_blocks(self._h, l))
        if nb < 0:
            raise ValueError("invalid level")
        org = np.zeros((nb, 3), dtype=np.int32)
        u = torch.empty((nb, 8, 8, 8), dtype=torch.float64, device="cuda")
        _check(lib().mgfr_amr_get_level(self._h, l, org.ctypes.data_as(C.c_void_p) if nb else None,
                                        u.data_ptr() if nb else None))
        return org, u
