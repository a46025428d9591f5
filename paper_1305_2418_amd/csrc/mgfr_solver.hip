// FP64 multigrid path of the f(R) field solve on gfx950.
//
// Operator (Sec. 3.2, Eq. u_discrete_field_eq, multiplied by a^2 to the
// comoving dimensionless form):
//   L_c(u) = (1/h^2) sum_nb (e^{u_nb} + e^{u_c})/2 (u_nb - u_c) - bC (1 - e^{-q u_c})
//   f_c    = beta Omega_m a^-3 delta_c,      q = 1/(n+1)
// Smoother: red-black Newton-Gauss-Seidel (Sec. 3.3, Eq. iterative_correction).
// Cycle: FAS V-cycle with 8-daughter-mean restriction, coarse source
// f_2h = L_2h(R u) + R(f - L_h u) and correction u += P(u_2h - R u)
// (Sec. 3.3, Eq. fine_correction), down to a 4^3 grid.
//
// Memory layout: every level is a dense N^3 float64 array in C order
// (k fastest).  Index arithmetic uses N = 2^lg.
#include "mgfr_internal.h"
#include "mgfr_ops.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace mgfr {

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;

int set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what, const char *file, int line)
{
    return set_error(e == hipErrorOutOfMemory ? MGFR_ERR_OOM : MGFR_ERR_HIP, "%s failed: %s (%s:%d)", what,
                     hipGetErrorString(e), file, line);
}

// ------------------------------------------------------------ device helpers

// Newton-Gauss-Seidel step for one cell from its value, its six neighbours and
// its source: -(L_c - f_c) / (dL_c/du_c), optionally limited to |du| <= max_du.
// With S1 = sum (u_n - u_c), S2 = sum e^{u_n}, S3 = sum e^{u_n} (u_n - u_c):
//   flux sum          = (S3 + e^{u_c} S1) / 2
//   d(flux sum)/du_c  = (e^{u_c} (S1 - 6) - S2) / 2
__device__ __forceinline__ double ngs_step(double uc, double n0, double n1, double n2, double n3,
                                           double n4, double n5, double f, const OpConst &k)
{
    double ec = exp64(uc, k.tab);
    double d0 = n0 - uc, d1 = n1 - uc, d2 = n2 - uc, d3 = n3 - uc, d4 = n4 - uc, d5 = n5 - uc;
    double e0 = exp64(n0, k.tab), e1 = exp64(n1, k.tab), e2 = exp64(n2, k.tab), e3 = exp64(n3, k.tab),
           e4 = exp64(n4, k.tab), e5 = exp64(n5, k.tab);
    double S1 = ((d0 + d1) + (d2 + d3)) + (d4 + d5);
    double S2 = ((e0 + e1) + (e2 + e3)) + (e4 + e5);
    double S3 = ((e0 * d0 + e1 * d1) + (e2 * d2 + e3 * d3)) + (e4 * d4 + e5 * d5);
    double em = expm1_64(-k.q * uc, k.tab);
    double L = k.ih2 * 0.5 * (S3 + ec * S1) + k.bC * em;
    double J = k.ih2 * 0.5 * (ec * (S1 - 6.0) - S2) - k.bC * k.q * (1.0 + em);
    double du = -(L - f) / J;
    if (k.max_du > 0.0) du = fmin(fmax(du, -k.max_du), k.max_du);
    return du;
}

__device__ __forceinline__ double op_value(double uc, double n0, double n1, double n2, double n3,
                                           double n4, double n5, const OpConst &k)
{
    double ec = exp64(uc, k.tab);
    double d0 = n0 - uc, d1 = n1 - uc, d2 = n2 - uc, d3 = n3 - uc, d4 = n4 - uc, d5 = n5 - uc;
    double e0 = exp64(n0, k.tab), e1 = exp64(n1, k.tab), e2 = exp64(n2, k.tab), e3 = exp64(n3, k.tab),
           e4 = exp64(n4, k.tab), e5 = exp64(n5, k.tab);
    double S1 = ((d0 + d1) + (d2 + d3)) + (d4 + d5);
    double S3 = ((e0 * d0 + e1 * d1) + (e2 * d2 + e3 * d3)) + (e4 * d4 + e5 * d5);
    return k.ih2 * 0.5 * (S3 + ec * S1) + k.bC * expm1_64(-k.q * uc, k.tab);
}

// L_c at (i,j,k) of a periodic 2^lg mesh.
__device__ __forceinline__ double op_at(const double *__restrict__ u, int i, int j, int k, int lg,
                                        const OpConst &kc)
{
    const int m = (1 << lg) - 1;
    double uc = u[cidx(i, j, k, lg)];
    return op_value(uc, u[cidx((i + 1) & m, j, k, lg)], u[cidx((i - 1) & m, j, k, lg)],
                    u[cidx(i, (j + 1) & m, k, lg)], u[cidx(i, (j - 1) & m, k, lg)],
                    u[cidx(i, j, (k + 1) & m, lg)], u[cidx(i, j, (k - 1) & m, lg)], kc);
}

// Update one cell of colour `colour` given its flat index t over that colour's cells.
__device__ __forceinline__ void sweep_cell(double *__restrict__ u, const double *__restrict__ f, size_t t,
                                           int lg, int colour, const OpConst &kc)
{
    const int m = (1 << lg) - 1;
    int mh = (int)(t & (size_t)((1 << (lg - 1)) - 1));
    size_t row = t >> (lg - 1);
    int j = (int)(row & m);
    int i = (int)(row >> lg);
    int k = 2 * mh + ((i + j + colour) & 1);
    size_t c = cidx(i, j, k, lg);
    double uc = u[c];
    double du = ngs_step(uc, u[cidx((i + 1) & m, j, k, lg)], u[cidx((i - 1) & m, j, k, lg)],
                         u[cidx(i, (j + 1) & m, k, lg)], u[cidx(i, (j - 1) & m, k, lg)],
                         u[cidx(i, j, (k + 1) & m, lg)], u[cidx(i, j, (k - 1) & m, lg)], f[c], kc);
    u[c] = uc + du;
}

// 1/x for finite non-zero x: hardware reciprocal refined by two Newton steps.
__device__ __forceinline__ double recip(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// Newton-Gauss-Seidel step from precomputed exponentials: ec = e^{u_c},
// em = e^{-q u_c} - 1, neighbour values n* and their exponentials e*.
__device__ __forceinline__ double ngs_step_e(double uc, double ec, double em, double n0, double e0, double n1,
                                             double e1, double n2, double e2, double n3, double e3, double n4,
                                             double e4, double n5, double e5, double f, const OpConst &k)
{
    double d0 = n0 - uc, d1 = n1 - uc, d2 = n2 - uc, d3 = n3 - uc, d4 = n4 - uc, d5 = n5 - uc;
    double S1 = ((d0 + d1) + (d2 + d3)) + (d4 + d5);
    double S2 = ((e0 + e1) + (e2 + e3)) + (e4 + e5);
    double S3 = ((e0 * d0 + e1 * d1) + (e2 * d2 + e3 * d3)) + (e4 * d4 + e5 * d5);
    double L = k.ih2 * 0.5 * (S3 + ec * S1) + k.bC * em;
    double J = k.ih2 * 0.5 * (ec * (S1 - 6.0) - S2) - k.bC * k.q * (1.0 + em);
    double du = -(L - f) * recip(J);
    if (k.max_du > 0.0) du = fmin(fmax(du, -k.max_du), k.max_du);
    return du;
}

// e^{-q u} - 1 given e^{u}: for n = 1 (q = 1/2) this is rsqrt(e^u) - 1.
template <bool N1>
__device__ __forceinline__ double curv_em(double uc, double ec, double q, const double *tab)
{
    if constexpr (N1) return rsqrt(ec) - 1.0;
    else return expm1_64(-q * uc, tab);
}

// One full red-black sweep, out of place: uout = sweep(uin).
//
// A workgroup owns a (y, z) tile of (JL - 4) x FKI interior cells and marches
// along x over `chunk` planes, staging a JL x 64 tile (halo 2) of each plane in
// LDS.  Red cells are updated on the interior plus a one-cell ring (which needs
// old black values two cells out), black cells on the interior; plane p+1 is
// red-updated while plane p is black-updated.
//
// Lanes map to z columns and each thread owns one pair of consecutive y rows.
// In every column exactly one row of the pair is red on plane p+1, and that
// same row is black on plane p, so every lane does one red and one black
// update per plane with straight-line code.  Each cell's e^u is computed once
// when loaded and once more after its red update; for n = 1 the curvature term
// reuses e^u through rsqrt.  Every cell of uin and f is read and every cell of
// uout written once (24 B/cell) apart from the halo and the 4 warm-up planes of
// each chunk; the next plane is prefetched one iteration ahead.
constexpr int FKL = 64, FKI = 60;

template <int JL>
struct FusedShape {
    static constexpr int JI = JL - 4;       // interior rows
    static constexpr int THREADS = 32 * JL; // one thread per row pair and column
};

template <bool N1, int JL>
__global__ __launch_bounds__(32 * JL) void k_sweep_fused(const double *__restrict__ uin,
                                                           const double *__restrict__ f,
                                                           double *__restrict__ uout, int lg, int chunk,
                                                           OpConst kc)
{
    MGFR_EXP_TABLE_TO_LDS(kc);
    constexpr int JI = JL - 4;
    __shared__ double sV[2][JL][FKL];
    __shared__ double sE[2][JL][FKL];
    const int N = 1 << lg, m = N - 1;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int k0 = blockIdx.x * FKI, j0 = blockIdx.y * JI, i0 = blockIdx.z * chunk;
    const int kku = k0 - 2 + lane;
    const int kg = kku & m;
    const bool kin1 = lane >= 1 && lane <= FKL - 2;
    const bool kint = lane >= 2 && lane <= FKL - 3 && kku < N;
    const int ra = 2 * w, rb = ra + 1;  // the thread's two rows in the tile
    const int jga = (j0 - 2 + ra) & m, jgb = (j0 - 2 + rb) & m;
    const bool in1a = ra >= 1 && ra <= JL - 2, in1b = rb >= 1 && rb <= JL - 2;
    const bool inta = ra >= 2 && ra <= JL - 3 && j0 - 2 + ra < N;
    const bool intb = rb >= 2 && rb <= JL - 3 && j0 - 2 + rb < N;
    const bool lda = in1a && kin1, ldb = in1b && kin1;  // f needed (red ring / black interior)
    const int lm = lane > 0 ? lane - 1 : 0, lp = lane < FKL - 1 ? lane + 1 : FKL - 1;
    auto at = [&](int i, int jg) { return (((((size_t)(i & m)) << lg) + (size_t)jg) << lg) + (size_t)kg; };

    // plane p-1: red value (and e^u) in the row that is black on plane p
    double V0s = 0.0, E0s = 0.0;
    // plane p: red cells updated, black cells old
    double V1a = uin[at(i0 - 2, jga)], V1b = uin[at(i0 - 2, jgb)];
    // plane p+1: old values
    double V2a = uin[at(i0 - 1, jga)], V2b = uin[at(i0 - 1, jgb)];
    double F1s = 0.0;
    double F2a = lda ? f[at(i0 - 1, jga)] : 0.0, F2b = ldb ? f[at(i0 - 1, jgb)] : 0.0;
    double V4a = uin[at(i0, jga)], V4b = uin[at(i0, jgb)];
    double F4a = lda ? f[at(i0, jga)] : 0.0, F4b = ldb ? f[at(i0, jgb)] : 0.0;
    double E1a = exp64(V1a, kc.tab), E1b = exp64(V1b, kc.tab), E2a = exp64(V2a, kc.tab), E2b = exp64(V2b, kc.tab);
    int xb = 0;
    for (int p = i0 - 2; p < i0 + chunk; ++p) {
        // plane p+2 (prefetched last iteration); prefetch plane p+3
        const double V3a = V4a, V3b = V4b, F3a = F4a, F3b = F4b;
        if (p + 1 < i0 + chunk) {
            V4a = uin[at(p + 3, jga)];
            V4b = uin[at(p + 3, jgb)];
            F4a = lda ? f[at(p + 3, jga)] : 0.0;
            F4b = ldb ? f[at(p + 3, jgb)] : 0.0;
        }
        const double E3a = exp64(V3a, kc.tab), E3b = exp64(V3b, kc.tab);
        __syncthreads();  // the previous plane's readers of buffer xb are done
        sV[xb][ra][lane] = V2a;
        sV[xb][rb][lane] = V2b;
        sE[xb][ra][lane] = E2a;
        sE[xb][rb][lane] = E2b;
        __syncthreads();
        // red cell of plane p+1 in row r = ra + sel; the same row holds the black cell of plane p
        const int sel = ((p + 1) + jga + kg) & 1;
        const int r = ra + sel;
        const int rc = r < 1 ? 1 : (r > JL - 2 ? JL - 2 : r);
        {
            const bool act = kin1 && (sel ? in1b : in1a);
            const double uc = sel ? V2b : V2a, ec = sel ? E2b : E2a;
            const double du = ngs_step_e(uc, ec, curv_em<N1>(uc, ec, kc.q, kc.tab), sel ? V1b : V1a, sel ? E1b : E1a,
                                         sel ? V3b : V3a, sel ? E3b : E3a, sV[xb][rc - 1][lane],
                                         sE[xb][rc - 1][lane], sV[xb][rc + 1][lane], sE[xb][rc + 1][lane],
                                         sV[xb][rc][lm], sE[xb][rc][lm], sV[xb][rc][lp], sE[xb][rc][lp],
                                         sel ? F2b : F2a, kc);
            const double un = uc + du;
            const double en = exp64(un, kc.tab);
            V2a = (act && !sel) ? un : V2a;
            E2a = (act && !sel) ? en : E2a;
            V2b = (act && sel) ? un : V2b;
            E2b = (act && sel) ? en : E2b;
            // only black positions of this buffer are read by other red updates
            if (act) {
                sV[xb][r][lane] = un;
                sE[xb][r][lane] = en;
            }
        }
        // black cell of plane p (buffer xb^1 holds plane p with its red cells updated)
        if (p >= i0) {
            const int yb = xb ^ 1;
            const bool act = kint && (sel ? intb : inta);
            const double uc = sel ? V1b : V1a, ec = sel ? E1b : E1a;
            const double du = ngs_step_e(uc, ec, curv_em<N1>(uc, ec, kc.q, kc.tab), V0s, E0s, sel ? V2b : V2a,
                                         sel ? E2b : E2a, sV[yb][rc - 1][lane], sE[yb][rc - 1][lane],
                                         sV[yb][rc + 1][lane], sE[yb][rc + 1][lane], sV[yb][rc][lm],
                                         sE[yb][rc][lm], sV[yb][rc][lp], sE[yb][rc][lp], F1s, kc);
            const double un = uc + du;
            V1a = (act && !sel) ? un : V1a;
            V1b = (act && sel) ? un : V1b;
            if (kint && inta) uout[at(p, jga)] = V1a;
            if (kint && intb) uout[at(p, jgb)] = V1b;
        }
        // rotate: the red row of plane p is the black row of plane p+1
        V0s = sel ? V1a : V1b;
        E0s = sel ? E1a : E1b;
        F1s = sel ? F2a : F2b;
        V1a = V2a;
        V1b = V2b;
        E1a = E2a;
        E1b = E2b;
        V2a = V3a;
        V2b = V3b;
        E2a = E3a;
        E2b = E3b;
        F2a = F3a;
        F2b = F3b;
        xb ^= 1;
    }
}

// --------------------------------------------------------------- grid kernels

__global__ __launch_bounds__(kBlock) void k_sweep_half(double *__restrict__ u, const double *__restrict__ f,
                                                         int lg, int colour, OpConst kc)
{
    MGFR_EXP_TABLE_TO_LDS(kc);
    size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    sweep_cell(u, f, t, lg, colour, kc);
}

// rbar -> fc, R u -> ubar_c
__global__ __launch_bounds__(kBlock) void k_residual_restrict(const double *__restrict__ u,
                                                                const double *__restrict__ f, int lg,
                                                                OpConst kc, double *__restrict__ ubar_c,
                                                                double *__restrict__ f_c)
{
    MGFR_EXP_TABLE_TO_LDS(kc);
    const int lgc = lg - 1;
    size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    int K = (int)(t & ((1u << lgc) - 1));
    int J = (int)((t >> lgc) & ((1u << lgc) - 1));
    int I = (int)(t >> (2 * lgc));
    BlockRes br;
    block_residuals(u, f, I, J, K, lg, kc, br);
    ubar_c[t] = br.umean;
    f_c[t] = br.rmean;
}

// f_c += L_c(ubar), u_c = ubar
__global__ __launch_bounds__(kBlock) void k_coarse_rhs(const double *__restrict__ ubar, int lg, OpConst kc,
                                                         double *__restrict__ fc, double *__restrict__ uc)
{
    MGFR_EXP_TABLE_TO_LDS(kc);
    size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int m = (1 << lg) - 1;
    int k = (int)(t & m), j = (int)((t >> lg) & m), i = (int)(t >> (2 * lg));
    fc[t] += op_at(ubar, i, j, k, lg, kc);
    uc[t] = ubar[t];
}

// one thread per coarse cell: its 8 daughters of the 2^lg mesh
__global__ __launch_bounds__(kBlock) void k_prolong_add(double *__restrict__ u, const double *__restrict__ uc,
                                                          const double *__restrict__ ub, int lg, int mode)
{
    const int lgc = lg - 1;
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int K = (int)(t & ((1u << lgc) - 1)), J = (int)((t >> lgc) & ((1u << lgc) - 1)), I = (int)(t >> (2 * lgc));
    prolong_block(u, uc, ub, I, J, K, lgc, mode);
}

template <int BS>
__device__ __forceinline__ void block_reduce_max_sum(double &mx, double &sm, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) {
        mx = nanmax(mx, __shfl_xor(mx, o, 64));
        sm += __shfl_xor(sm, o, 64);
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        sh[w] = mx;
        sh[BS / 64 + w] = sm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < BS / 64; ++i) {
            mx = nanmax(mx, sh[i]);
            sm += sh[BS / 64 + i];
        }
    }
}

// per-block max |r| and sum r^2 over the fine level (thread per 2x2x2 block)
__global__ __launch_bounds__(kBlock) void k_residual_norm(const double *__restrict__ u,
                                                            const double *__restrict__ f, int lg, OpConst kc,
                                                            double *__restrict__ partial, int nparts)
{
    MGFR_EXP_TABLE_TO_LDS(kc);
    __shared__ double sh[2 * kBlock / 64];
    const int lgc = lg - 1;
    const size_t nblk = (size_t)1 << (3 * lgc);
    double mx = 0.0, sm = 0.0;
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < nblk; t += (size_t)gridDim.x * kBlock) {
        int K = (int)(t & ((1u << lgc) - 1));
        int J = (int)((t >> lgc) & ((1u << lgc) - 1));
        int I = (int)(t >> (2 * lgc));
        BlockRes br;
        block_residuals(u, f, I, J, K, lg, kc, br);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            mx = nanmax(mx, fabs(br.r[c]));
            sm += br.r[c] * br.r[c];
        }
    }
    block_reduce_max_sum<kBlock>(mx, sm, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = mx;
        partial[nparts + blockIdx.x] = sm;
    }
}

__global__ __launch_bounds__(kBlock) void k_residual_field(const double *__restrict__ u,
                                                             const double *__restrict__ f, int lg, OpConst kc,
                                                             double *__restrict__ r)
{
    MGFR_EXP_TABLE_TO_LDS(kc);
    size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int m = (1 << lg) - 1;
    int k = (int)(t & m), j = (int)((t >> lg) & m), i = (int)(t >> (2 * lg));
    r[t] = f[t] - op_at(u, i, j, k, lg, kc);
}

// final reduction of nparts partials -> out[0] = max, out[1] = sum
__global__ __launch_bounds__(1024) void k_final_reduce(const double *__restrict__ partial, int nparts,
                                                        double *__restrict__ out)
{
    __shared__ double sh[2 * 1024 / 64];
    double mx = 0.0, sm = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 1024) {
        mx = nanmax(mx, partial[i]);
        sm += partial[nparts + i];
    }
    block_reduce_max_sum<1024>(mx, sm, sh);
    if (threadIdx.x == 0) {
        out[0] = mx;
        out[1] = sm;
    }
}

// f = s * delta with per-block max |f| partials
__global__ __launch_bounds__(kBlock) void k_source(const double *__restrict__ delta, double s, size_t n,
                                                     double *__restrict__ f, double *__restrict__ partial,
                                                     int nparts)
{
    __shared__ double sh[2 * kBlock / 64];
    double mx = 0.0, sm = 0.0;
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (size_t)gridDim.x * kBlock) {
        double v = s * delta[t];
        f[t] = v;
        mx = nanmax(mx, fabs(v));
    }
    block_reduce_max_sum<kBlock>(mx, sm, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = mx;
        partial[nparts + blockIdx.x] = 0.0;
    }
}

// Screened-limit initial guess: u = -(n+1) log1p(s max(delta, 0)) with
// s = Omega_m a^-3 / C(a) (the local balance of the field equation where the
// Laplacian term is negligible).
__global__ __launch_bounds__(kBlock) void k_screened_guess(const double *__restrict__ delta, double s,
                                                             double np1, size_t n, double *__restrict__ u)
{
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (size_t)gridDim.x * kBlock) {
        const double d = delta[t];
        u[t] = -np1 * log1p(s * (d > 0.0 ? d : 0.0));
    }
}

// delta_eff = delta/3 - c expm1(-q u) with c = C / (3 Omega_m a^-3)
__global__ __launch_bounds__(kBlock) void k_effective_density(const double *__restrict__ delta,
                                                                const double *__restrict__ u, double c, double q,
                                                                size_t n, double *__restrict__ out)
{
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (size_t)gridDim.x * kBlock)
        out[t] = delta[t] / 3.0 - c * expm1(-q * u[t]);
}

__global__ __launch_bounds__(kBlock) void k_dfr(const double *__restrict__ u, double fbar, size_t n,
                                                  double *__restrict__ dfr)
{
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (size_t)gridDim.x * kBlock)
        dfr[t] = -fbar * expm1(u[t]);
}

// ------------------------------------------------------------- tail kernel
// All levels with N <= kTailN inside one workgroup: the V-cycle from level l0
// down to the 4^3 grid and back, with workgroup barriers between steps.

struct TailArgs {
    double *u[kMaxLevels];
    double *f[kMaxLevels];
    double *ub[kMaxLevels];
    double ih2[kMaxLevels];
    int lg[kMaxLevels];
    int l0, nlev, pre, post, coarse, mode;
    double bC, q, max_du;
    const double *tab;  // exponential's table (the kernel points it at its LDS copy)
};

__device__ void tail_sweeps(const TailArgs &A, int l, int sweeps)
{
    OpConst kc{A.ih2[l], A.bC, A.q, A.max_du, A.tab};
    const int lg = A.lg[l];
    const size_t half = (size_t)1 << (3 * lg - 1);
    for (int s = 0; s < sweeps; ++s)
        for (int colour = 0; colour < 2; ++colour) {
            for (size_t t = threadIdx.x; t < half; t += kTailThreads) sweep_cell(A.u[l], A.f[l], t, lg, colour, kc);
            __syncthreads();
        }
}

__global__ __launch_bounds__(kTailThreads) void k_tail(TailArgs A)
{
    __shared__ double s_tab[64];
    if (threadIdx.x < 64) s_tab[threadIdx.x] = A.tab[threadIdx.x];
    __syncthreads();
    A.tab = s_tab;
    for (int l = A.l0; l < A.nlev - 1; ++l) {
        tail_sweeps(A, l, A.pre);
        OpConst kc{A.ih2[l], A.bC, A.q, A.max_du, A.tab};
        const int lg = A.lg[l], lgc = lg - 1;
        const size_t nc = (size_t)1 << (3 * lgc);
        for (size_t t = threadIdx.x; t < nc; t += kTailThreads) {
            int K = (int)(t & ((1u << lgc) - 1));
            int J = (int)((t >> lgc) & ((1u << lgc) - 1));
            int I = (int)(t >> (2 * lgc));
            BlockRes br;
            block_residuals(A.u[l], A.f[l], I, J, K, lg, kc, br);
            A.ub[l + 1][t] = br.umean;
            A.f[l + 1][t] = br.rmean;
        }
        __syncthreads();
        OpConst kcc{A.ih2[l + 1], A.bC, A.q, A.max_du, A.tab};
        const int mc = (1 << lgc) - 1;
        for (size_t t = threadIdx.x; t < nc; t += kTailThreads) {
            int k = (int)(t & mc), j = (int)((t >> lgc) & mc), i = (int)(t >> (2 * lgc));
            A.f[l + 1][t] += op_at(A.ub[l + 1], i, j, k, lgc, kcc);
            A.u[l + 1][t] = A.ub[l + 1][t];
        }
        __syncthreads();
    }
    tail_sweeps(A, A.nlev - 1, A.coarse);
    for (int l = A.nlev - 2; l >= A.l0; --l) {
        const int lg = A.lg[l];
        const size_t n = (size_t)1 << (3 * lg);
        const int m = (1 << lg) - 1;
        for (size_t t = threadIdx.x; t < n; t += kTailThreads) {
            int k = (int)(t & m), j = (int)((t >> lg) & m), i = (int)(t >> (2 * lg));
            A.u[l][t] += prolong_value(A.u[l + 1], A.ub[l + 1], i, j, k, lg - 1, A.mode);
        }
        __syncthreads();
        tail_sweeps(A, l, A.post);
    }
}

// ------------------------------------------------------------ host launches

static inline unsigned nblocks(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

static int timer_slot(mgfr_ctx *c, int *slot)
{
    Timer &T = c->sweep_timer;
    if (T.used + 2 > (int)T.ev.size()) {
        for (int e = 0; e < 16; ++e) {
            hipEvent_t ev;
            MGFR_HIP(hipEventCreate(&ev));
            T.ev.push_back(ev);
        }
    }
    *slot = T.used;
    T.used += 2;
    return MGFR_OK;
}

#ifndef MGFR_FUSED_JL
#define MGFR_FUSED_JL 16
#endif

static int fused_chunk(int N)
{
    int ch = N / 8;
    return ch < 8 ? 8 : ch;
}

// `sweeps` red-black sweeps on level l.  Levels with N >= fused_min_n use the
// out-of-place fused kernel and swap L.u / L.alt after each sweep; the others
// update L.u in place with one kernel per colour.
int launch_sweep64(mgfr_ctx *c, int l, double *u_unused, const double *f, int sweeps, bool timed)
{
    (void)u_unused;
    Level &L = c->lev[l];
    OpConst kc = level_const(c, l);
    const bool fused = c->fused_min_n > 0 && L.N >= c->fused_min_n && L.alt != nullptr;
    const size_t half = (size_t)1 << (3 * L.lg - 1);
    for (int s = 0; s < sweeps; ++s) {
        int slot = -1;
        if (timed) {
            int rc = timer_slot(c, &slot);
            if (rc) return rc;
            MGFR_HIP(hipEventRecord(c->sweep_timer.ev[slot], c->stream));
        }
        if (fused) {
            const int chunk = fused_chunk(L.N);
            constexpr int JL = MGFR_FUSED_JL;
            constexpr int JI = FusedShape<JL>::JI;
            dim3 grid((unsigned)((L.N + FKI - 1) / FKI), (unsigned)((L.N + JI - 1) / JI), (unsigned)(L.N / chunk));
            if (c->p.n == 1)
                k_sweep_fused<true, JL><<<grid, FusedShape<JL>::THREADS, 0, c->stream>>>(L.u, f, L.alt, L.lg, chunk, kc);
            else
                k_sweep_fused<false, JL><<<grid, FusedShape<JL>::THREADS, 0, c->stream>>>(L.u, f, L.alt, L.lg, chunk, kc);
            std::swap(L.u, L.alt);
        } else {
            for (int colour = 0; colour < 2; ++colour)
                k_sweep_half<<<nblocks(half), kBlock, 0, c->stream>>>(L.u, f, L.lg, colour, kc);
        }
        if (timed) MGFR_HIP(hipEventRecord(c->sweep_timer.ev[slot + 1], c->stream));
    }
    MGFR_HIP(hipGetLastError());
    return MGFR_OK;
}

static int launch_tail(mgfr_ctx *c, int l0)
{
    TailArgs A;
    memset(&A, 0, sizeof A);
    for (int l = 0; l < c->nlev; ++l) {
        A.u[l] = c->lev[l].u;
        A.f[l] = c->lev[l].f;
        A.ub[l] = c->lev[l].ubar;
        A.ih2[l] = 1.0 / (c->lev[l].h * c->lev[l].h);
        A.lg[l] = c->lev[l].lg;
    }
    A.l0 = l0;
    A.nlev = c->nlev;
    A.pre = c->p.pre_smooth;
    A.post = c->p.post_smooth;
    A.coarse = c->p.coarse_sweeps;
    A.mode = c->p.prolong;
    A.bC = c->bC;
    A.q = c->q;
    A.max_du = c->p.max_du;
    A.tab = c->exp2tab;
    k_tail<<<1, kTailThreads, 0, c->stream>>>(A);
    MGFR_HIP(hipGetLastError());
    return MGFR_OK;
}

int vcycle64(mgfr_ctx *c, int l)
{
    Level &L = c->lev[l];
    if (L.N <= kTailN) return launch_tail(c, l);
    int rc;
    if ((rc = launch_sweep64(c, l, L.u, L.f, c->p.pre_smooth, l == 0 && c->timing))) return rc;
    Level &Lc = c->lev[l + 1];
    const size_t nc = (size_t)1 << (3 * Lc.lg);
    k_residual_restrict<<<nblocks(nc), kBlock, 0, c->stream>>>(L.u, L.f, L.lg, level_const(c, l), Lc.ubar, Lc.f);
    k_coarse_rhs<<<nblocks(nc), kBlock, 0, c->stream>>>(Lc.ubar, Lc.lg, level_const(c, l + 1), Lc.f, Lc.u);
    MGFR_HIP(hipGetLastError());
    if ((rc = vcycle64(c, l + 1))) return rc;
    k_prolong_add<<<nblocks(nc), kBlock, 0, c->stream>>>(L.u, Lc.u, Lc.ubar, L.lg, c->p.prolong);
    MGFR_HIP(hipGetLastError());
    return launch_sweep64(c, l, L.u, L.f, c->p.post_smooth, l == 0 && c->timing);
}

int launch_residual_norm64(mgfr_ctx *c, int l, const double *u, const double *f, double *rmax, double *rsumsq)
{
    Level &L = c->lev[l];
    const size_t nblk = (size_t)1 << (3 * (L.lg - 1));
    unsigned g = (unsigned)std::min<size_t>(nblocks(nblk), (size_t)c->nparts);
    k_residual_norm<<<g, kBlock, 0, c->stream>>>(u, f, L.lg, level_const(c, l), c->partial, (int)g);
    k_final_reduce<<<1, 1024, 0, c->stream>>>(c->partial, (int)g, c->dscal);
    MGFR_HIP(hipGetLastError());
    MGFR_HIP(hipMemcpyAsync(c->hscal, c->dscal, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    MGFR_HIP(hipStreamSynchronize(c->stream));
    *rmax = c->hscal[0];
    *rsumsq = c->hscal[1];
    return MGFR_OK;
}

int collect_timing(mgfr_ctx *c, mgfr_stats *st)
{
    Timer &T = c->sweep_timer;
    for (int e = 0; e + 1 < T.used; e += 2) {
        float ms = 0;
        MGFR_HIP(hipEventElapsedTime(&ms, T.ev[e], T.ev[e + 1]));
        if (st) {
            st->t_sweep_ms += ms;
            st->n_sweep_launches += 1;
        }
    }
    T.used = 0;
    return MGFR_OK;
}

// ---------------------------------------------------------------- validation

static int validate(const mgfr_params *p)
{
    if (!p) return set_error(MGFR_ERR_ARG, "params is NULL");
    if (!(p->box > 0) || !std::isfinite(p->box)) return set_error(MGFR_ERR_ARG, "box must be > 0");
    if (!(p->a > 0) || !std::isfinite(p->a)) return set_error(MGFR_ERR_ARG, "a must be > 0");
    if (!(p->omega_m > 0)) return set_error(MGFR_ERR_ARG, "omega_m must be > 0");
    if (!(p->omega_l >= 0)) return set_error(MGFR_ERR_ARG, "omega_l must be >= 0");
    if (!(p->fr0_abs > 0) || !std::isfinite(p->fr0_abs)) return set_error(MGFR_ERR_ARG, "fr0_abs must be > 0");
    if (p->n < 1) return set_error(MGFR_ERR_ARG, "n must be >= 1");
    if (p->mesh < 8 || p->mesh > 1024 || (p->mesh & (p->mesh - 1)))
        return set_error(MGFR_ERR_ARG, "mesh must be a power of two in [8, 1024], got %d", p->mesh);
    if (p->refine_levels != 0) return set_error(MGFR_ERR_ARG, "refine_levels must be 0 for a uniform mesh");
    if (!(p->tol > 0)) return set_error(MGFR_ERR_ARG, "tol must be > 0");
    if (p->pre_smooth < 0 || p->post_smooth < 0) return set_error(MGFR_ERR_ARG, "smoothing counts must be >= 0");
    if (p->coarse_sweeps < 1) return set_error(MGFR_ERR_ARG, "coarse_sweeps must be >= 1");
    if (p->max_vcycles < 0) return set_error(MGFR_ERR_ARG, "max_vcycles must be >= 0");
    if (p->coarse_cycles < 0) return set_error(MGFR_ERR_ARG, "coarse_cycles must be >= 0");
    if (p->prolong != MGFR_PROLONG_LINEAR && p->prolong != MGFR_PROLONG_INJECT)
        return set_error(MGFR_ERR_ARG, "prolong must be 0 (linear) or 1 (injection)");
    if (p->precision != MGFR_FP64 && p->precision != MGFR_MIXED)
        return set_error(MGFR_ERR_ARG, "precision must be MGFR_FP64 or MGFR_MIXED");
    if (p->nn_mode != MGFR_NN_NONE && p->nn_mode != MGFR_NN_COARSE)
        return set_error(MGFR_ERR_ARG, "nn_mode must be MGFR_NN_NONE or MGFR_NN_COARSE");
    return MGFR_OK;
}

static void background(const mgfr_params *p, double *fbar, double *beta, double *C)
{
    // Sec. 2: R_bar = 3 H0^2 (Omega_m a^-3 + 4 Omega_L); fbar_R(a) = fbar_R0 (R_bar0/R_bar(a))^(n+1)
    double r = 4.0 * p->omega_l / p->omega_m;
    double a3 = 1.0 / (p->a * p->a * p->a);
    *fbar = p->fr0_abs * std::pow((1.0 + r) / (a3 + r), p->n + 1);
    *C = p->omega_m * a3 + 4.0 * p->omega_l;
    *beta = p->a * p->a / (kCOverH0 * kCOverH0) / *fbar;
}

}  // namespace mgfr

using namespace mgfr;

// ================================================================== C ABI

extern "C" const char *mgfr_last_error(void) { return g_err.c_str(); }

extern "C" int mgfr_background(const mgfr_params *p, double *fbar, double *beta, double *C)
{
    int rc = validate(p);
    if (rc) return rc;
    double a, b, c;
    background(p, &a, &b, &c);
    if (fbar) *fbar = a;
    if (beta) *beta = b;
    if (C) *C = c;
    return MGFR_OK;
}

static void free_ctx(mgfr_ctx *c)
{
    if (!c) return;
    nn_free(c);
    bin_free(c);
    pm_free(c);
    for (int l = 0; l < kMaxLevels; ++l) {
        Level &L = c->lev[l];
        if (l > 0) {
            (void)hipFree(L.u);
            (void)hipFree(L.alt);
        }
        (void)hipFree(L.f);
        (void)hipFree(L.ubar);
        (void)hipFree(L.e32);
        (void)hipFree(L.r32);
        (void)hipFree(L.u32);
        (void)hipFree(L.ebar32);
        (void)hipFree(L.e32alt);
    }
    (void)hipFree(c->alt0);
    (void)hipFree(c->partial);
    (void)hipFree(c->dscal);
    (void)hipFree(c->dflag);
    (void)hipFree(c->r64);
    (void)hipFree(c->exp2tab);
    if (c->hscal) (void)hipHostFree(c->hscal);
    for (hipEvent_t e : c->sweep_timer.ev) (void)hipEventDestroy(e);
    if (c->ev_a) (void)hipEventDestroy(c->ev_a);
    if (c->ev_b) (void)hipEventDestroy(c->ev_b);
    if (c->ev_c) (void)hipEventDestroy(c->ev_c);
    delete c;
}

static int create_impl(const mgfr_params *p, void *stream, mgfr_ctx *c)
{
    c->p = *p;
    c->stream = (hipStream_t)stream;
    MGFR_HIP(hipGetDevice(&c->device));
    background(p, &c->fbar, &c->beta, &c->C);
    c->bC = c->beta * c->C;
    c->q = 1.0 / (p->n + 1);
    int N = p->mesh, lg = 0;
    while ((1 << lg) < N) ++lg;
    c->nlev = 0;
    for (int n = N, l = 0; n >= 4; n /= 2, ++l) {
        Level &L = c->lev[l];
        L.N = n;
        L.lg = lg - l;
        L.h = p->box / n;
        size_t bytes = sizeof(double) * (size_t)n * n * n;
        MGFR_HIP(hipMalloc(&L.f, bytes));
        if (l > 0) {
            MGFR_HIP(hipMalloc(&L.u, bytes));
            MGFR_HIP(hipMalloc(&L.ubar, bytes));
        }
        if (n >= 64) {  // second buffer for out-of-place fused sweeps
            MGFR_HIP(hipMalloc(&L.alt, bytes));
            if (l == 0) c->alt0 = L.alt;
        }
        c->nlev = l + 1;
    }
    c->nparts = 4096;
    MGFR_HIP(hipMalloc(&c->partial, sizeof(double) * 2 * c->nparts));
    {
        double tab[64];
        for (int j = 0; j < 64; ++j) tab[j] = (double)exp2l((long double)j / 64.0L);
        MGFR_HIP(hipMalloc(&c->exp2tab, sizeof tab));
        MGFR_HIP(hipMemcpy(c->exp2tab, tab, sizeof tab, hipMemcpyHostToDevice));
    }
    MGFR_HIP(hipMalloc(&c->dscal, sizeof(double) * 8));
    MGFR_HIP(hipMalloc(&c->dflag, sizeof(int) * 4));
    MGFR_HIP(hipHostMalloc(&c->hscal, sizeof(double) * 8, hipHostMallocDefault));
    MGFR_HIP(hipEventCreate(&c->ev_a));
    MGFR_HIP(hipEventCreate(&c->ev_b));
    MGFR_HIP(hipEventCreate(&c->ev_c));
    if (p->precision == MGFR_MIXED) {
        int rc = mixed_alloc(c);
        if (rc) return rc;
    }
    return MGFR_OK;
}

extern "C" int mgfr_create(const mgfr_params *p, void *stream, mgfr_ctx **out)
{
    if (!out) return set_error(MGFR_ERR_ARG, "out is NULL");
    *out = nullptr;
    int rc = validate(p);
    if (rc) return rc;
    mgfr_ctx *c = new (std::nothrow) mgfr_ctx();
    if (!c) return set_error(MGFR_ERR_OOM, "host allocation failed");
    rc = create_impl(p, stream, c);
    if (rc) {
        free_ctx(c);
        return rc;
    }
    *out = c;
    return MGFR_OK;
}

extern "C" void mgfr_destroy(mgfr_ctx *c) { free_ctx(c); }

extern "C" int mgfr_set_stream(mgfr_ctx *c, void *stream)
{
    if (!c) return set_error(MGFR_ERR_ARG, "ctx is NULL");
    c->stream = (hipStream_t)stream;
    return MGFR_OK;
}

extern "C" int mgfr_set_scale_factor(mgfr_ctx *c, double a)
{
    if (!c) return set_error(MGFR_ERR_ARG, "ctx is NULL");
    if (!(a > 0) || !std::isfinite(a)) return set_error(MGFR_ERR_ARG, "a must be > 0 and finite");
    mgfr_params q = c->p;
    q.a = a;
    double fb, beta, C;
    if (int rc = mgfr_background(&q, &fb, &beta, &C)) return rc;
    c->p.a = a;
    c->fbar = fb;
    c->beta = beta;
    c->C = C;
    c->bC = beta * C;
    return MGFR_OK;
}

extern "C" int mgfr_set_timing(mgfr_ctx *c, int on)
{
    if (!c) return set_error(MGFR_ERR_ARG, "ctx is NULL");
    c->timing = on != 0;
    return MGFR_OK;
}

static int check_ptr(const void *p, const char *name)
{
    if (!p) return set_error(MGFR_ERR_ARG, "%s is NULL", name);
    return MGFR_OK;
}

// Form f on level 0 and return D = max|f| (bC if f == 0) on the host.
static int prepare_source(mgfr_ctx *c, const double *delta, double *D)
{
    Level &L0 = c->lev[0];
    size_t n = (size_t)L0.N * L0.N * L0.N;
    double s = c->beta * c->p.omega_m / (c->p.a * c->p.a * c->p.a);
    unsigned g = (unsigned)std::min<size_t>(nblocks(n), (size_t)c->nparts);
    k_source<<<g, kBlock, 0, c->stream>>>(delta, s, n, L0.f, c->partial, (int)g);
    k_final_reduce<<<1, 1024, 0, c->stream>>>(c->partial, (int)g, c->dscal + 2);
    MGFR_HIP(hipGetLastError());
    MGFR_HIP(hipMemcpyAsync(c->hscal + 2, c->dscal + 2, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    MGFR_HIP(hipStreamSynchronize(c->stream));
    double d = c->hscal[2];
    if (!std::isfinite(d)) return set_error(MGFR_ERR_NONFINITE, "delta contains NaN or Inf");
    *D = d > 0 ? d : c->bC;
    return MGFR_OK;
}

// After out-of-place sweeps the current level-0 iterate may sit in the
// context's buffer: copy it back into the caller's array.
static int restore_level0(mgfr_ctx *c, double *user_u)
{
    Level &L0 = c->lev[0];
    if (L0.u != user_u) {
        size_t n = (size_t)L0.N * L0.N * L0.N;
        MGFR_HIP(hipMemcpyAsync(user_u, L0.u, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        L0.alt = L0.u;
        L0.u = user_u;
    }
    return MGFR_OK;
}

static int finish(mgfr_ctx *c, double *u, double *dfr, mgfr_stats *st, int status)
{
    if (dfr) {
        size_t n = (size_t)c->lev[0].N * c->lev[0].N * c->lev[0].N;
        unsigned g = (unsigned)std::min<size_t>(nblocks(n), 8192);
        k_dfr<<<g, kBlock, 0, c->stream>>>(u, c->fbar, n, dfr);
        MGFR_HIP(hipGetLastError());
    }
    MGFR_HIP(hipEventRecord(c->ev_b, c->stream));
    MGFR_HIP(hipEventSynchronize(c->ev_b));
    float ms = 0;
    MGFR_HIP(hipEventElapsedTime(&ms, c->ev_a, c->ev_b));
    if (st) {
        st->t_solve_ms = ms;
        st->status = status;
    }
    if (status == MGFR_ERR_NONFINITE) return set_error(status, "the iteration produced NaN or Inf");
    return status;
}

void mgfr::adapt_smoothing(mgfr_ctx *c, double res, double res2)
{
    if (c->smooth_max <= 0 || !(res2 >= 0.0) || !(res >= res2)) return;
    c->p.pre_smooth = std::min(std::max(1, 2 * c->p.pre_smooth), c->smooth_max);
    c->p.post_smooth = std::min(std::max(1, 2 * c->p.post_smooth), c->smooth_max);
}

int mgfr::solve_fp64_from(mgfr_ctx *c, double *u, mgfr_stats *st, double D)
{
    Level &L0 = c->lev[0];
    double rmax, rsq;
    const double ncell = (double)L0.N * L0.N * L0.N;
    int rc = launch_residual_norm64(c, 0, u, L0.f, &rmax, &rsq);
    if (rc) return rc;
    double res = rmax / D, res1 = res, res2 = -1.0;  // res1, res2: one and two checks back
    st->res0 = res;
    int cyc = 0, status;
    for (;;) {
        if (!std::isfinite(res)) { status = MGFR_ERR_NONFINITE; break; }
        if (res <= c->p.tol) { status = MGFR_OK; break; }
        if (cyc >= c->p.max_vcycles) { status = MGFR_NOT_CONVERGED; break; }
        if ((rc = vcycle64(c, 0))) return rc;
        if ((rc = launch_residual_norm64(c, 0, u, L0.f, &rmax, &rsq))) return rc;
        if (c->timing && (rc = collect_timing(c, st))) return rc;
        res2 = cyc >= 1 ? res1 : -1.0;
        res1 = res;
        res = rmax / D;
        adapt_smoothing(c, res, res2);
        if (cyc < MGFR_MAX_HIST) st->res_hist[cyc] = res;
        ++cyc;
    }
    st->vcycles = cyc;
    st->outer_iters = cyc;
    st->res = res;
    st->l2res = std::sqrt(rsq / ncell) / D;
    return status;
}

extern "C" int mgfr_screened_guess(mgfr_ctx *c, const double *delta, double *u)
{
    int rc;
    if ((rc = check_ptr(c, "ctx")) || (rc = check_ptr(delta, "delta")) || (rc = check_ptr(u, "u"))) return rc;
    const size_t n = (size_t)c->lev[0].N * c->lev[0].N * c->lev[0].N;
    const double s = c->p.omega_m / (c->p.a * c->p.a * c->p.a) / c->C;
    const unsigned g = (unsigned)std::min<size_t>((n + kBlock - 1) / kBlock, 16384);
    k_screened_guess<<<g, kBlock, 0, c->stream>>>(delta, s, (double)(c->p.n + 1), n, u);
    MGFR_HIP(hipGetLastError());
    return MGFR_OK;
}

extern "C" int mgfr_effective_density(mgfr_ctx *c, const double *delta, const double *u, double *out)
{
    int rc;
    if ((rc = check_ptr(c, "ctx")) || (rc = check_ptr(delta, "delta")) || (rc = check_ptr(u, "u")) ||
        (rc = check_ptr(out, "out")))
        return rc;
    const size_t n = (size_t)c->lev[0].N * c->lev[0].N * c->lev[0].N;
    const double om = c->p.omega_m / (c->p.a * c->p.a * c->p.a);
    const unsigned g = (unsigned)std::min<size_t>((n + kBlock - 1) / kBlock, 16384);
    k_effective_density<<<g, kBlock, 0, c->stream>>>(delta, u, c->C / (3.0 * om), c->q, n, out);
    MGFR_HIP(hipGetLastError());
    return MGFR_OK;
}

extern "C" int mgfr_solve(mgfr_ctx *c, const double *delta, double *u, double *dfr, mgfr_stats *st_out)
{
    int rc;
    if ((rc = check_ptr(c, "ctx")) || (rc = check_ptr(delta, "delta")) || (rc = check_ptr(u, "u"))) return rc;
    mgfr_stats local;
    mgfr_stats *st = st_out ? st_out : &local;
    memset(st, 0, sizeof *st);
    c->lev[0].u = u;
    c->lev[0].alt = c->alt0;
    c->sweep_timer.used = 0;
    MGFR_HIP(hipEventRecord(c->ev_a, c->stream));
    double D;
    if ((rc = prepare_source(c, delta, &D))) {
        st->status = rc;
        return rc;
    }
    st->scale = D;
    if (c->p.nn_mode == MGFR_NN_COARSE) {
        double tnn = 0;
        if ((rc = nn_warm_start(c, delta, u, &tnn))) return rc;
        st->t_nn_ms = tnn;
    }
    int status;
    const int pre = c->p.pre_smooth, post = c->p.post_smooth;  // adaptive smoothing changes them per solve
    if (c->p.precision == MGFR_MIXED) {
        status = solve_mixed(c, u, st, D);
    } else {
        status = solve_fp64_from(c, u, st, D);
    }
    st->smooth_used = c->p.pre_smooth;
    c->p.pre_smooth = pre;
    c->p.post_smooth = post;
    if (status < 0 && status != MGFR_ERR_NONFINITE) return status;
    if ((rc = restore_level0(c, u))) return rc;
    return finish(c, u, dfr, st, status);
}

extern "C" int mgfr_ngs_sweep(mgfr_ctx *c, double *u, const double *f, int sweeps)
{
    int rc;
    if ((rc = check_ptr(c, "ctx")) || (rc = check_ptr(u, "u")) || (rc = check_ptr(f, "f"))) return rc;
    if (sweeps < 0) return set_error(MGFR_ERR_ARG, "sweeps must be >= 0");
    Level &L0 = c->lev[0];
    L0.u = u;
    L0.alt = c->alt0;
    if ((rc = launch_sweep64(c, 0, nullptr, f, sweeps, false))) return rc;
    if ((rc = restore_level0(c, u))) return rc;
    MGFR_HIP(hipStreamSynchronize(c->stream));
    return MGFR_OK;
}

extern "C" int mgfr_set_fused_min_mesh(mgfr_ctx *c, int n)
{
    if (!c) return set_error(MGFR_ERR_ARG, "ctx is NULL");
    if (n != 0 && n < 64) return set_error(MGFR_ERR_ARG, "fused sweeps need levels of at least 64^3 (or 0 = off)");
    c->fused_min_n = n;
    return MGFR_OK;
}

extern "C" int mgfr_set_colour_min_mesh(mgfr_ctx *c, int n)
{
    if (!c) return set_error(MGFR_ERR_ARG, "ctx is NULL");
    if (n != 0 && n < 128) return set_error(MGFR_ERR_ARG, "one-colour pass kernels need levels of at least 128^3 (or 0 = off)");
    c->colour32_min_n = n;
    return MGFR_OK;
}

extern "C" int mgfr_set_relaxation32(mgfr_ctx *c, double omega)
{
    if (!c) return set_error(MGFR_ERR_ARG, "ctx is NULL");
    if (!(omega > 0.0 && omega < 2.0)) return set_error(MGFR_ERR_ARG, "omega must be in (0, 2)");
    c->omega32 = omega;
    return MGFR_OK;
}

extern "C" int mgfr_set_adaptive_smoothing(mgfr_ctx *c, int max_sweeps)
{
    if (!c) return set_error(MGFR_ERR_ARG, "ctx is NULL");
    if (max_sweeps != 0 && (max_sweeps < std::max(c->p.pre_smooth, c->p.post_smooth) || max_sweeps > 32))
        return set_error(MGFR_ERR_ARG, "max_sweeps must be 0 or in [max(pre_smooth, post_smooth), 32]");
    c->smooth_max = max_sweeps;
    return MGFR_OK;
}

extern "C" int mgfr_set_inner_cycles(mgfr_ctx *c, int max_inner)
{
    if (!c) return set_error(MGFR_ERR_ARG, "ctx is NULL");
    if (max_inner < 1 || max_inner > 4) return set_error(MGFR_ERR_ARG, "max_inner must be in [1, 4]");
    c->inner_max = max_inner;
    return MGFR_OK;
}

extern "C" int mgfr_set_fused_sweep32(mgfr_ctx *c, int on)
{
    if (!c) return set_error(MGFR_ERR_ARG, "ctx is NULL");
    if (on != 0 && on != 1) return set_error(MGFR_ERR_ARG, "on must be 0 or 1");
    if (on && c->p.precision == MGFR_MIXED && c->lev[0].N >= 128 && !c->lev[0].e32alt)
        return set_error(MGFR_ERR_ARG, "no second correction buffer (the context was not created for mixed precision)");
    c->fused32 = on;
    return MGFR_OK;
}

extern "C" int mgfr_vcycle(mgfr_ctx *c, double *u, const double *f)
{
    int rc;
    if ((rc = check_ptr(c, "ctx")) || (rc = check_ptr(u, "u")) || (rc = check_ptr(f, "f"))) return rc;
    Level &L0 = c->lev[0];
    size_t n = (size_t)L0.N * L0.N * L0.N;
    MGFR_HIP(hipMemcpyAsync(L0.f, f, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    L0.u = u;
    L0.alt = c->alt0;
    if ((rc = vcycle64(c, 0))) return rc;
    if ((rc = restore_level0(c, u))) return rc;
    MGFR_HIP(hipStreamSynchronize(c->stream));
    return MGFR_OK;
}

extern "C" int mgfr_residual(mgfr_ctx *c, const double *u, const double *f, double *r)
{
    int rc;
    if ((rc = check_ptr(c, "ctx")) || (rc = check_ptr(u, "u")) || (rc = check_ptr(f, "f")) ||
        (rc = check_ptr(r, "r")))
        return rc;
    Level &L0 = c->lev[0];
    size_t n = (size_t)L0.N * L0.N * L0.N;
    k_residual_field<<<nblocks(n), kBlock, 0, c->stream>>>(u, f, L0.lg, level_const(c, 0), r);
    MGFR_HIP(hipGetLastError());
    MGFR_HIP(hipStreamSynchronize(c->stream));
    return MGFR_OK;
}
