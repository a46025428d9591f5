"""Independent references used to pin the oracle (no code shared with it).

* the background from the Hu-Sawicki f(R) itself (exact f_R(R), not the
  large-curvature approximation) and R_bar from 12 H^2 + 6 H dH/dln a;
* the periodic discrete linear (Yukawa) solution by FFT;
* a vectorised numpy form of the discrete operator for brute-force Newton;
* the continuum Yukawa profile of a point mass.
"""
from __future__ import annotations

import math

import numpy as np

C_OVER_H0 = 2997.92458


# ----------------------------------------------------------------------- background

def hubble2(a, om, ol):
    """H^2 / H0^2 of flat LCDM."""
    return om * a ** -3 + ol


def rbar_from_friedmann(a, om, ol, eps=1e-6):
    """R_bar / H0^2 = 12 H^2 + 6 H dH/dln a, derivative by central differences."""
    H = lambda x: math.sqrt(hubble2(x, om, ol))
    la = math.log(a)
    dH = (H(math.exp(la + eps)) - H(math.exp(la - eps))) / (2 * eps)
    return 12 * H(a) ** 2 + 6 * H(a) * dH


def hu_sawicki_fR(R, n, c1, c2, m2):
    """Exact f_R = df/dR of f(R) = -m^2 c1 (R/m^2)^n / (c2 (R/m^2)^n + 1)."""
    x = R / m2
    return -n * c1 * x ** (n - 1) / (c2 * x ** n + 1) ** 2


def hu_sawicki_constants(fr0_abs, n, om, ol):
    """c1, c2 from c1/c2 = 6 Omega_L/Omega_m and fbar_R0 = f_R(R_bar0) (units H0 = 1)."""
    m2 = om
    R0 = rbar_from_friedmann(1.0, om, ol)
    ratio = 6 * ol / om
    # f_R(R0) = -n ratio c2^-1 x^(n-1) / (x^n + 1/c2)^2 with x = R0/m2: solve for c2 by bisection
    x = R0 / m2
    f = lambda c2: -n * ratio * c2 * x ** (n - 1) / (c2 * x ** n + 1) ** 2 + fr0_abs
    lo, hi = 1.0, 1e15
    for _ in range(300):
        mid = math.sqrt(lo * hi)
        if f(mid) > 0:  # |f_R| too small -> c2 too large
            hi = mid
        else:
            lo = mid
    c2 = math.sqrt(lo * hi)
    return ratio * c2, c2, m2


def fbar_exact(a, fr0_abs, n, om, ol):
    c1, c2, m2 = hu_sawicki_constants(fr0_abs, n, om, ol)
    return abs(hu_sawicki_fR(rbar_from_friedmann(a, om, ol), n, c1, c2, m2))


def lambda2_comoving(a, fr0_abs, n, om, ol, rel=1e-5):
    """a^2 lambda^2 in (h/Mpc)^2 with lambda^2 = (1/3c^2) dR/df_R at fbar_R (Sec. 4.1),
    derivative of the exact Hu-Sawicki f_R(R) by central differences."""
    c1, c2, m2 = hu_sawicki_constants(fr0_abs, n, om, ol)
    R = rbar_from_friedmann(a, om, ol)
    dR = R * rel
    dfdR = (hu_sawicki_fR(R + dR, n, c1, c2, m2) - hu_sawicki_fR(R - dR, n, c1, c2, m2)) / (2 * dR)
    lam2_H0 = 1.0 / (3.0 * dfdR)  # in units of H0^2/c^2
    return a * a * lam2_H0 / C_OVER_H0 ** 2


# ------------------------------------------------------------- numpy discrete operator

def L_numpy(u, h, bC, n=1):
    """Flux-form operator of Sec. 3.2 in vectorised numpy (periodic)."""
    e = np.exp(u)
    out = np.zeros_like(u)
    for ax in range(3):
        for s in (1, -1):
            un = np.roll(u, -s, axis=ax)
            en = np.roll(e, -s, axis=ax)
            out += 0.5 * (en + e) * (un - u)
    return out / h ** 2 - bC * (1.0 - np.exp(-u / (n + 1)))


def jacobian_dense(u, h, bC, n=1):
    """Dense Jacobian of L_numpy (analytic, 7-point)."""
    N = u.shape[0]
    M = N ** 3
    J = np.zeros((M, M))
    e = np.exp(u)
    idx = np.arange(M).reshape(N, N, N)
    diag = -bC / (n + 1) * np.exp(-u / (n + 1))
    for ax in range(3):
        for s in (1, -1):
            un = np.roll(u, -s, axis=ax)
            en = np.roll(e, -s, axis=ax)
            nb = np.roll(idx, -s, axis=ax)
            # d/du_c of 1/2 (e_n + e_c)(u_n - u_c) and d/du_n
            diag = diag + (0.5 * e * (un - u) - 0.5 * (en + e)) / h ** 2
            off = (0.5 * en * (un - u) + 0.5 * (en + e)) / h ** 2
            np.add.at(J, (idx.ravel(), nb.ravel()), off.ravel())
    J[idx.ravel(), idx.ravel()] += diag.ravel()
    return J


def dense_newton(f, h, bC, n=1, u0=None, tol=1e-14, maxit=200):
    """Newton with Armijo backtracking on L(u) = f; returns (u, ||F||_inf)."""
    u = np.zeros_like(f) if u0 is None else u0.copy()
    F = L_numpy(u, h, bC, n) - f
    for _ in range(maxit):
        nf = np.abs(F).max()
        if nf <= tol:
            break
        J = jacobian_dense(u, h, bC, n)
        du = np.linalg.solve(J, -F.ravel()).reshape(u.shape)
        t = 1.0
        while True:
            un = u + t * du
            Fn = L_numpy(un, h, bC, n) - f
            if np.abs(Fn).max() <= (1 - 1e-4 * t) * nf or t < 1e-8:
                break
            t *= 0.5
        u, F = un, Fn
    return u, np.abs(F).max()


# ------------------------------------------------------------------ linear solutions

def discrete_k2(N, h):
    k = 2 * np.pi * np.fft.fftfreq(N)  # k h
    s = (4.0 / h ** 2) * np.sin(k / 2) ** 2
    return s[:, None, None] + s[None, :, None] + s[None, None, :]


def linear_solution(f, h, mu2):
    """Periodic solution of (discrete Laplacian - mu^2) u = f by FFT."""
    N = f.shape[0]
    fk = np.fft.fftn(f)
    uk = -fk / (discrete_k2(N, h) + mu2)
    return np.real(np.fft.ifftn(uk))


def yukawa_point(r, mass_term, lam):
    """(2 G m / 3 c^2) e^{-lambda r} / r with 2 G m / 3 c^2 given as ``mass_term``."""
    return mass_term * np.exp(-lam * r) / r
