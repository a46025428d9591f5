// Device helpers shared by the float64 and mixed-precision kernels.
#pragma once

#include "mgfr_internal.h"

namespace mgfr {

__device__ __forceinline__ size_t cidx(int i, int j, int k, int lg)
{
    return (((((size_t)i) << lg) + (size_t)j) << lg) + (size_t)k;
}

// Copy the exponential's table into LDS for a kernel's own use (before any
// early return; kc is the kernel's OpConst parameter).
#define MGFR_EXP_TABLE_TO_LDS(kc)                                                \
    __shared__ double s_exp2tab_[64];                                           \
    if (threadIdx.x < 64) s_exp2tab_[threadIdx.x] = (kc).tab[threadIdx.x];      \
    __syncthreads();                                                            \
    (kc).tab = s_exp2tab_

// e^x and e^x - 1 in float64 by table-driven reduction (Tang's method):
// x = (64 m + j) ln2/64 + r with |r| <= ln2/128, so e^x = 2^m 2^(j/64) e^r, and
// e^r - 1 is its Taylor series to r^5 (truncation below 2^-56).  ln2/64 is
// split into a head with 32 trailing zero bits and a tail (the fdlibm split
// of ln2 scaled by 1/64), so (64 m + j) times the head is exact.  tab[j] =
// 2^(j/64), j = 0..63 (kept in LDS by the kernels that use it).  The parts
// are S = 2^m tab[j] and p = e^r - 1: e^x = S + S p, and e^x - 1 = (S - 1) + S p,
// where S - 1 is exact for S in [1/2, 2] (|x| < ln2), so no cancellation.
struct Exp64 {
    double S, p;
};

__device__ __forceinline__ Exp64 exp64_parts(double x, const double *tab)
{
    const double kd = rint(x * 92.33248261689366);
    double r = fma(kd, -0.01083042469326756, x);
    r = fma(kd, -2.9815858269852933e-12, r);
    const int k = (int)kd;
    const double p = r * (1.0 + r * (0.5 + r * (1.0 / 6.0 + r * (1.0 / 24.0 + r * (1.0 / 120.0)))));
    return Exp64{ldexp(tab[k & 63], k >> 6), p};
}

__device__ __forceinline__ double exp64(double x, const double *tab)
{
    const Exp64 e = exp64_parts(x, tab);
    return fma(e.S, e.p, e.S);
}

__device__ __forceinline__ double expm1_64(double x, const double *tab)
{
    const Exp64 e = exp64_parts(x, tab);
    return fma(e.S, e.p, e.S - 1.0);
}

__device__ __forceinline__ double nanmax(double a, double b)
{
    return (a != a || a > b) ? a : b;
}

// Residuals r = f - L(u) at the 8 daughters of coarse cell (I,J,K) and their
// mean values of u and r.  The 2x2x2 block plus its 24 face neighbours are
// loaded once and each is exponentiated once.
struct BlockRes {
    double r[8];
    double umean, rmean;
};

__device__ __forceinline__ void block_residuals(const double *__restrict__ u, const double *__restrict__ f,
                                                int I, int J, int K, int lg, const OpConst &kc, BlockRes &out)
{
    const int m = (1 << lg) - 1;
    const int i0 = 2 * I, j0 = 2 * J, k0 = 2 * K;
    double B[2][2][2], EB[2][2][2];
    double Xm[2][2], Xp[2][2], Ym[2][2], Yp[2][2], Zm[2][2], Zp[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                B[a][b][c] = u[cidx(i0 + a, j0 + b, k0 + c, lg)];
                EB[a][b][c] = exp64(B[a][b][c], kc.tab);
            }
            Xm[a][b] = u[cidx((i0 - 1) & m, j0 + a, k0 + b, lg)];
            Xp[a][b] = u[cidx((i0 + 2) & m, j0 + a, k0 + b, lg)];
            Ym[a][b] = u[cidx(i0 + a, (j0 - 1) & m, k0 + b, lg)];
            Yp[a][b] = u[cidx(i0 + a, (j0 + 2) & m, k0 + b, lg)];
            Zm[a][b] = u[cidx(i0 + a, j0 + b, (k0 - 1) & m, lg)];
            Zp[a][b] = u[cidx(i0 + a, j0 + b, (k0 + 2) & m, lg)];
        }
    double su = 0.0, sr = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                double uc = B[a][b][c], ec = EB[a][b][c];
                double nx0 = a ? Xp[b][c] : B[1][b][c];       // +x
                double nx1 = a ? B[0][b][c] : Xm[b][c];       // -x
                double ny0 = b ? Yp[a][c] : B[a][1][c];
                double ny1 = b ? B[a][0][c] : Ym[a][c];
                double nz0 = c ? Zp[a][b] : B[a][b][1];
                double nz1 = c ? B[a][b][0] : Zm[a][b];
                double ex0 = a ? exp64(nx0, kc.tab) : EB[1][b][c];
                double ex1 = a ? EB[0][b][c] : exp64(nx1, kc.tab);
                double ey0 = b ? exp64(ny0, kc.tab) : EB[a][1][c];
                double ey1 = b ? EB[a][0][c] : exp64(ny1, kc.tab);
                double ez0 = c ? exp64(nz0, kc.tab) : EB[a][b][1];
                double ez1 = c ? EB[a][b][0] : exp64(nz1, kc.tab);
                double d0 = nx0 - uc, d1 = nx1 - uc, d2 = ny0 - uc, d3 = ny1 - uc, d4 = nz0 - uc, d5 = nz1 - uc;
                double S1 = ((d0 + d1) + (d2 + d3)) + (d4 + d5);
                double S3 = ((ex0 * d0 + ex1 * d1) + (ey0 * d2 + ey1 * d3)) + (ez0 * d4 + ez1 * d5);
                double L = kc.ih2 * 0.5 * (S3 + ec * S1) + kc.bC * expm1_64(-kc.q * uc, kc.tab);
                double r = f[cidx(i0 + a, j0 + b, k0 + c, lg)] - L;
                out.r[(a * 2 + b) * 2 + c] = r;
                su += uc;
                sr += r;
            }
    out.umean = su / 8.0;
    out.rmean = sr / 8.0;
}

// Linear (mode 0) or injected (mode 1) correction at fine cell (i,j,k):
// P(uc - ubar) with the central-difference gradient at the parent centre.
__device__ __forceinline__ double prolong_value(const double *__restrict__ uc, const double *__restrict__ ub,
                                                int i, int j, int k, int lgc, int mode)
{
    const int m = (1 << lgc) - 1;
    int I = i >> 1, J = j >> 1, K = k >> 1;
    size_t P = cidx(I, J, K, lgc);
    double v = uc[P] - ub[P];
    if (mode == 0) {
        size_t xp = cidx((I + 1) & m, J, K, lgc), xm = cidx((I - 1) & m, J, K, lgc);
        size_t yp = cidx(I, (J + 1) & m, K, lgc), ym = cidx(I, (J - 1) & m, K, lgc);
        size_t zp = cidx(I, J, (K + 1) & m, lgc), zm = cidx(I, J, (K - 1) & m, lgc);
        double gx = (uc[xp] - ub[xp]) - (uc[xm] - ub[xm]);
        double gy = (uc[yp] - ub[yp]) - (uc[ym] - ub[ym]);
        double gz = (uc[zp] - ub[zp]) - (uc[zm] - ub[zm]);
        double sx = (i & 1) ? 0.125 : -0.125, sy = (j & 1) ? 0.125 : -0.125, sz = (k & 1) ? 0.125 : -0.125;
        v += sx * gx;
        v += sy * gy;
        v += sz * gz;
    }
    return v;
}


// Correction u += P(uc - ub) for the 8 daughters of coarse cell (I,J,K) of a
// 2^lgc mesh: the parent value and gradient are formed once (same arithmetic
// order as prolong_value).
template <typename T>
__device__ __forceinline__ void prolong_block(T *__restrict__ u, const T *__restrict__ uc, const T *__restrict__ ub,
                                              int I, int J, int K, int lgc, int mode)
{
    const int m = (1 << lgc) - 1;
    const size_t P = cidx(I, J, K, lgc);
    const T v0 = uc[P] - ub[P];
    T gx = 0, gy = 0, gz = 0;
    if (mode == 0) {
        const size_t xp = cidx((I + 1) & m, J, K, lgc), xm = cidx((I - 1) & m, J, K, lgc);
        const size_t yp = cidx(I, (J + 1) & m, K, lgc), ym = cidx(I, (J - 1) & m, K, lgc);
        const size_t zp = cidx(I, J, (K + 1) & m, lgc), zm = cidx(I, J, (K - 1) & m, lgc);
        gx = (uc[xp] - ub[xp]) - (uc[xm] - ub[xm]);
        gy = (uc[yp] - ub[yp]) - (uc[ym] - ub[ym]);
        gz = (uc[zp] - ub[zp]) - (uc[zm] - ub[zm]);
    }
    const int lg = lgc + 1;
    const T eighth = (T)0.125;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                T v = v0;
                if (mode == 0) {
                    v += (a ? eighth : -eighth) * gx;
                    v += (b ? eighth : -eighth) * gy;
                    v += (c ? eighth : -eighth) * gz;
                }
                u[cidx(2 * I + a, 2 * J + b, 2 * K + c, lg)] += v;
            }
}

// ------------------------------------------------ float32 correction cycle
// Shared by the uniform mixed-precision solve and the refined levels.

struct MxConst {
    float ih2, bC, q, max_du;
    float omega = 1.0f;  // relaxation factor of the Newton step (1: plain Newton-Gauss-Seidel)
};

// e^x for the float32 correction cycle: the hardware base-2 exponential of
// x log2(e) (relative error a few float32 ulps times |x log2 e|, which only
// perturbs the linearisation point the float64 outer loop corrects anyway).
__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }

// e^x - 1 for the float32 correction cycle: x + x^2/2 for |x| < 2^-10
// (truncation below 2e-7 relative), fexp(x) - 1 otherwise (cancellation at
// most ~1.2e-4 relative, at |x| = 2^-10, falling as 1/|x|).  Its relative
// error is proportional to expm1 itself, so the correction operator stays
// free of the O(ulp) absolute error that would stall the outer loop; the
// float64 residual decides convergence.
__device__ __forceinline__ float fexpm1(float x)
{
    const float q = fexp(x) - 1.0f;  // evaluated unconditionally: a select, not a branch
    const float p = fmaf(0.5f * x, x, x);
    return fabsf(x) < 0x1p-10f ? p : q;
}

// Newton step on e at one cell from precomputed per-cell quantities:
//   centre: e, X = expm1(e), u, w = e^u; neighbours likewise.
__device__ __forceinline__ float mx_step(float ec, float Xc, float uc, float wc, const float en[6],
                                         const float Xn[6], const float un[6], const float wn[6], float r,
                                         const MxConst &k)
{
    float Su = 0.f, Se = 0.f, A = 0.f, B = 0.f, SW = 0.f;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        const float du = un[t] - uc, de = en[t] - ec;
        const float Wn = wn[t] + wn[t] * Xn[t];
        Su += du;
        Se += de;
        A += wn[t] * Xn[t] * du;
        B += Wn * de;
        SW += Wn;
    }
    const float wXc = wc * Xc, Wc = wc + wXc;
    const float flux = 0.5f * ((A + wXc * Su) + (B + Wc * Se));
    const float dflux = 0.5f * (Wc * (Su + Se - 6.0f) - SW);
    const float sc = fexp(-k.q * uc);
    const float cm = fexpm1(-k.q * ec);
    const float N = k.ih2 * flux + k.bC * sc * cm;
    const float J = k.ih2 * dflux - k.q * k.bC * sc * (1.0f + cm);
    float d = -(N - r) / J * k.omega;
    if (k.max_du > 0.f) d = fminf(fmaxf(d, -k.max_du), k.max_du);
    return d;
}

__device__ __forceinline__ float mx_value(float ec, float Xc, float uc, float wc, const float en[6],
                                          const float Xn[6], const float un[6], const float wn[6],
                                          const MxConst &k)
{
    float Su = 0.f, Se = 0.f, A = 0.f, B = 0.f;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        const float du = un[t] - uc, de = en[t] - ec;
        Su += du;
        Se += de;
        A += wn[t] * Xn[t] * du;
        B += (wn[t] + wn[t] * Xn[t]) * de;
    }
    const float wXc = wc * Xc, Wc = wc + wXc;
    const float flux = 0.5f * ((A + wXc * Su) + (B + Wc * Se));
    return k.ih2 * flux + k.bC * fexp(-k.q * uc) * fexpm1(-k.q * ec);
}

}  // namespace mgfr
