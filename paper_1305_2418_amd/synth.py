"""Seeded synthetic particle loads and simple density fields.

This module is the only code shared by the solver's tests, the benchmark and
the CPU reference checks.  It holds no part of the field solve: it only draws
particle positions (and simple analytic density fields) with the shapes and
statistics of the paper's workloads:

* a uniform lattice of equal-mass particles displaced by the Zel'dovich
  approximation of a Gaussian random field with P(k) proportional to k^-2,
  standing in for the cosmological particle snapshots of the paper's
  Sec. 5 (which are not available);
* Plummer or NFW halos, built by relocating a random subset of lattice
  particles, so that the particle count stays exactly n^3 and the mesh sees
  strongly screened, deeply non-linear clumps (density contrasts ~1e4);
* the point-mass and Gaussian-sphere density set-ups of the paper's Sec. 4.1.

Random numbers come from seeded ``torch.Generator`` objects on the CPU, so a
(config, seed) pair names one input exactly; heavy FFT work may run on any
torch device.
"""
from __future__ import annotations

import math

import numpy as np
import torch

#: critical density today in (M_sun/h) / (Mpc/h)^3
RHO_CRIT = 2.775e11


def _gen(seed: int) -> torch.Generator:
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed))
    return g


def lattice(n: int, box: float, device="cpu") -> torch.Tensor:
    """Particles at the centres (q + 1/2) L/n of an n^3 lattice, float64 [n^3, 3]."""
    q = (torch.arange(n, dtype=torch.float64, device=device) + 0.5) * (box / n)
    gx, gy, gz = torch.meshgrid(q, q, q, indexing="ij")
    return torch.stack([gx.reshape(-1), gy.reshape(-1), gz.reshape(-1)], dim=1)


def _kgrid(n: int, box: float, device):
    k1 = torch.fft.fftfreq(n, d=box / n, device=device, dtype=torch.float64) * 2 * math.pi
    kz = torch.fft.rfftfreq(n, d=box / n, device=device, dtype=torch.float64) * 2 * math.pi
    return k1.view(n, 1, 1), k1.view(1, n, 1), kz.view(1, 1, n // 2 + 1)


def gaussian_field_k(n: int, box: float, rms: float, seed: int, slope: float = -2.0,
                     device="cpu") -> torch.Tensor:
    """Fourier modes (rfft layout) of a Gaussian field with P(k) ~ k^slope.

    Modes with |k| above the Nyquist wavenumber pi n / L and the k = 0 mode are
    zero.  The amplitude is set so that the real-space rms on the n^3 grid is
    ``rms``.
    """
    noise = torch.randn((n, n, n), generator=_gen(seed), dtype=torch.float64).to(device)
    dk = torch.fft.rfftn(noise)
    kx, ky, kz = _kgrid(n, box, device)
    k2 = kx * kx + ky * ky + kz * kz
    knyq = math.pi * n / box
    amp = torch.where((k2 > 0) & (k2 <= knyq * knyq), k2.clamp_min(1e-300) ** (slope / 4.0),
                      torch.zeros_like(k2))
    dk = dk * amp
    field = torch.fft.irfftn(dk, s=(n, n, n))
    s = field.std().item()
    return dk * (rms / s if s > 0 else 0.0)


def zeldovich(n: int, box: float, rms: float, seed: int, device="cpu", displacement: bool = False):
    """n^3 lattice particles displaced by psi = -grad(Laplacian^-1 delta_L), float64 [n^3,3].

    delta_L is the P(k) ~ k^-2 Gaussian field of :func:`gaussian_field_k`;
    the displacement obeys div psi = -delta_L, i.e. psi_k = i k delta_k / k^2.
    With ``displacement`` the displacements psi [n^3, 3] are returned too.
    """
    dk = gaussian_field_k(n, box, rms, seed, device=device)
    kx, ky, kz = _kgrid(n, box, device)
    k2 = kx * kx + ky * ky + kz * kz
    inv = torch.where(k2 > 0, 1.0 / k2.clamp_min(1e-300), torch.zeros_like(k2))
    pos = lattice(n, box, device)
    disp = torch.empty_like(pos) if displacement else None
    for d, kd in enumerate((kx, ky, kz)):
        psi = torch.fft.irfftn(1j * kd * inv * dk, s=(n, n, n)).reshape(-1)
        pos[:, d] += psi
        if displacement:
            disp[:, d] = psi
        del psi
    pos = torch.remainder(pos, box)
    return (pos, disp) if displacement else pos


def _directions(m: int, g: torch.Generator) -> torch.Tensor:
    v = torch.randn((m, 3), generator=g, dtype=torch.float64)
    return v / v.norm(dim=1, keepdim=True).clamp_min(1e-300)


def plummer_radii(m: int, r200: float, g: torch.Generator) -> torch.Tensor:
    """Radii of a Plummer sphere (scale b = 0.2 r200) truncated at r200 (inverse CDF)."""
    b = 0.2 * r200
    mt = r200 ** 3 / (r200 ** 2 + b * b) ** 1.5
    y = torch.rand(m, generator=g, dtype=torch.float64) * mt
    y23 = y ** (2.0 / 3.0)
    return b * y ** (1.0 / 3.0) / torch.sqrt(1.0 - y23)


def nfw_radii(m: int, r200: float, conc: float, g: torch.Generator) -> torch.Tensor:
    """Radii of an NFW halo (r_s = r200/c) truncated at r200 (bisection on M(<r))."""
    mu = lambda x: torch.log1p(x) - x / (1.0 + x)
    target = torch.rand(m, generator=g, dtype=torch.float64) * mu(torch.tensor(conc, dtype=torch.float64))
    lo = torch.zeros(m, dtype=torch.float64)
    hi = torch.full((m,), float(conc), dtype=torch.float64)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        below = mu(mid) < target
        lo = torch.where(below, mid, lo)
        hi = torch.where(below, hi, mid)
    return 0.5 * (lo + hi) * (r200 / conc)


def add_halos(pos: torch.Tensor, box: float, n_halos: int, m_lo: float, m_hi: float,
              omega_m: float, seed: int, profile: str = "plummer",
              conc=(5.0, 10.0)) -> torch.Tensor:
    """Relocate random lattice particles into ``n_halos`` halos (on a copy, on pos's device).

    Halo masses are log-uniform in [m_lo, m_hi] (M_sun/h); the particle mass is
    Omega_m rho_crit L^3 / N_p; r200 = (3 M / (4 pi 200 rho_crit))^(1/3).
    """
    g = _gen(seed + 7919)
    npart = pos.shape[0]
    mp = omega_m * RHO_CRIT * box ** 3 / npart
    masses = torch.exp(torch.empty(n_halos, dtype=torch.float64).uniform_(
        math.log(m_lo), math.log(m_hi), generator=g))
    counts = [max(1, int(round(m / mp))) for m in masses.tolist()]
    total = sum(counts)
    if total > npart // 2:
        raise ValueError("halos would take more than half of the particles")
    order = torch.randperm(npart, generator=g)
    centres = torch.rand((n_halos, 3), generator=g, dtype=torch.float64) * box
    cs = torch.empty(n_halos, dtype=torch.float64).uniform_(conc[0], conc[1], generator=g)
    out = pos.detach().to(torch.float64).clone()
    start = 0
    for h in range(n_halos):
        c = counts[h]
        idx = order[start:start + c]
        start += c
        r200 = (3.0 * masses[h].item() / (4.0 * math.pi * 200.0 * RHO_CRIT)) ** (1.0 / 3.0)
        if profile == "plummer":
            r = plummer_radii(c, r200, g)
        elif profile == "nfw":
            r = nfw_radii(c, r200, cs[h].item(), g)
        else:
            raise ValueError(profile)
        # drawn on the CPU generator, placed on the positions' device
        out[idx.to(out.device)] = (centres[h] + r.unsqueeze(1) * _directions(c, g)).to(out.device)
    return torch.remainder(out, box)


def to_f32(pos: torch.Tensor, box: float) -> torch.Tensor:
    """Float32 positions wrapped into [0, box)."""
    p = pos.to(torch.float32)
    p = torch.where(p >= box, p - box, p)
    return p.contiguous()


# -- named workloads -------------------------------------------------------------------

def clustered_load(n: int, box: float = 100.0, rms: float = 1.0, seed: int = 1,
                   n_halos: int = 0, profile: str = "plummer", m_lo: float = 1e13,
                   m_hi: float = 1e15, omega_m: float = 0.3, device="cpu") -> torch.Tensor:
    """float32 [n^3, 3] positions: Zel'dovich lattice (+ optional halos)."""
    pos = zeldovich(n, box, rms, seed, device=device)
    if n_halos:
        pos = add_halos(pos, box, n_halos, m_lo, m_hi, omega_m, seed, profile)
    return to_f32(pos, box).cpu() if str(device) == "cpu" else to_f32(pos, box)


def initial_conditions(n: int, box: float, rms: float, seed: int, a: float, omega_m: float = 0.3,
                       omega_l: float = 0.7, n_halos: int = 0, profile: str = "plummer", device="cpu"):
    """Positions and momenta (float32 [n^3, 3] each) for a chain of time steps:
    the Zel'dovich load of :func:`clustered_load` at scale factor ``a`` with the
    linear-theory momentum p = a^2 dx/dt = a^2 H(a) f(a) psi, f = Omega_m(a)^0.55
    (H in km/s per Mpc/h, so p is in km/s); particles relocated into halos start
    at rest."""
    pos, disp = zeldovich(n, box, rms, seed, device=device, displacement=True)
    hub = 100.0 * math.sqrt(omega_m / a ** 3 + omega_l)
    om_a = omega_m / a ** 3 / (omega_m / a ** 3 + omega_l)
    mom = disp * (a * a * hub * om_a ** 0.55)
    del disp
    if n_halos:
        moved = add_halos(pos, box, n_halos, 1e13, 1e15, omega_m, seed, profile)
        mom[(moved != pos).any(dim=1)] = 0.0
        pos = moved
    pos32, mom32 = to_f32(pos, box), mom.to(torch.float32).contiguous()
    if str(device) == "cpu":
        return pos32.cpu(), mom32.cpu()
    return pos32, mom32


# -- simple density fields (delta on an N^3 mesh, C order, float64 numpy) -------------

def point_mass_delta(N: int, amp: float = 1e-4, cell=(0, 0, 0)) -> np.ndarray:
    """delta = -amp everywhere except one cell with amp (N^3 - 1) (mean exactly 0)."""
    d = np.full((N, N, N), -amp, dtype=np.float64)
    d[cell] = amp * (N ** 3 - 1)
    return d


def gaussian_sphere_delta(N: int, box: float, width: float, mass_delta_cells: float,
                          centre=None) -> np.ndarray:
    """Periodic Gaussian overdensity exp(-r^2/w^2) with the same integrated excess as a
    point mass of ``mass_delta_cells`` (in units of mean-density cells); mean removed."""
    h = box / N
    x = (np.arange(N) + 0.5) * h
    c = (box / 2,) * 3 if centre is None else centre
    dx = [np.minimum(np.abs(x - c[d]), box - np.abs(x - c[d])) for d in range(3)]
    r2 = dx[0][:, None, None] ** 2 + dx[1][None, :, None] ** 2 + dx[2][None, None, :] ** 2
    g = np.exp(-r2 / width ** 2)
    g *= mass_delta_cells / g.sum()
    return g - g.mean()


def cosine_delta(N: int, eps: float, mode=(1, 0, 0)) -> np.ndarray:
    """delta = eps cos(2 pi m.x / L) sampled at cell centres."""
    idx = (np.arange(N) + 0.5) / N
    ph = (2 * np.pi * mode[0] * idx[:, None, None] + 2 * np.pi * mode[1] * idx[None, :, None]
          + 2 * np.pi * mode[2] * idx[None, None, :])
    return eps * np.cos(ph)


def spheres_delta(N: int, box: float, n_spheres: int, seed: int, width=(1.0, 4.0), peak=(1e2, 1e4),
                  device="cpu") -> torch.Tensor:
    """Sum of periodic Gaussian overdensities peak * exp(-r^2/w^2) at seeded random centres,
    mean removed, float64 [N, N, N] on ``device`` (for meshes too large for particle loads)."""
    g = _gen(seed)
    cen = torch.rand((n_spheres, 3), generator=g, dtype=torch.float64) * box
    w = torch.empty(n_spheres, dtype=torch.float64).uniform_(width[0], width[1], generator=g)
    pk = torch.exp(torch.empty(n_spheres, dtype=torch.float64).uniform_(math.log(peak[0]), math.log(peak[1]),
                                                                          generator=g))
    x = (torch.arange(N, dtype=torch.float64, device=device) + 0.5) * (box / N)
    d = torch.zeros((N, N, N), dtype=torch.float64, device=device)
    for s in range(n_spheres):
        comp = []
        for ax in range(3):
            dx = torch.abs(x - cen[s, ax].item())
            dx = torch.minimum(dx, box - dx)
            comp.append(torch.exp(-(dx * dx) / (w[s].item() ** 2)))
        d += pk[s].item() * comp[0].view(N, 1, 1) * comp[1].view(1, N, 1) * comp[2].view(1, 1, N)
    d -= d.mean()
    return d
