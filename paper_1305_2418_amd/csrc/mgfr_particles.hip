// Particle <-> mesh steps: cloud-in-cell assignment (Sec. 3.1) and the fifth
// force gathered back to the particles (Sec. 2, Eq. modgrav_accel).
#include "mgfr_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace mgfr {

namespace {

__device__ __forceinline__ double nanmax2(double a, double b) { return (a != a || a > b) ? a : b; }

// Cloud-in-cell weights along one axis: xi = x/h - 1/2, i0 = floor(xi), t = xi - i0,
// weights (1 - t, t) on cells (i0, i0 + 1) mod N.  Returns false for positions
// that are not finite or so large that floor(xi) does not fit an int64.
__device__ __forceinline__ bool cic_axis(float x, double h, int mask, int &i0, double &t)
{
    double xi = (double)x / h - 0.5;
    if (!(fabs(xi) < 4.0e18)) return false;
    double fl = floor(xi);
    t = xi - fl;
    i0 = (int)((long long)fl & (long long)mask);
    return true;
}

__global__ __launch_bounds__(kBlock) void k_cic_scatter(const float *__restrict__ pos,
                                                          const double *__restrict__ mass, int64_t np, int lg,
                                                          double h, double *__restrict__ m, int *__restrict__ flag)
{
    int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= np) return;
    const int mask = (1 << lg) - 1;
    int i0, j0, k0;
    double tx, ty, tz;
    bool ok = cic_axis(pos[3 * p + 0], h, mask, i0, tx) && cic_axis(pos[3 * p + 1], h, mask, j0, ty) &&
              cic_axis(pos[3 * p + 2], h, mask, k0, tz);
    double mp = mass ? mass[p] : 1.0;
    if (!ok || !isfinite(mp)) {
        flag[0] = 1;
        return;
    }
    const int i1 = (i0 + 1) & mask, j1 = (j0 + 1) & mask, k1 = (k0 + 1) & mask;
    const double wx[2] = {1.0 - tx, tx}, wy[2] = {1.0 - ty, ty}, wz[2] = {1.0 - tz, tz};
    const int ii[2] = {i0, i1}, jj[2] = {j0, j1}, kk[2] = {k0, k1};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                size_t cell = ((((size_t)ii[a] << lg) + jj[b]) << lg) + kk[c];
                unsafeAtomicAdd(&m[cell], wx[a] * wy[b] * wz[c] * mp);
            }
}

__global__ __launch_bounds__(kBlock) void k_sum_partial(const double *__restrict__ x, size_t n,
                                                          double *__restrict__ partial)
{
    __shared__ double sh[kBlock / 64];
    double s = 0.0;
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (size_t)gridDim.x * kBlock) s += x[t];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) s += sh[w];
        partial[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(1024) void k_sum_final(const double *__restrict__ partial, int n,
                                                     double *__restrict__ out)
{
    __shared__ double sh[16];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) s += partial[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 16; ++w) s += sh[w];
        out[0] = s;
    }
}

// delta = m / mbar - 1, mbar = total / ncell read from the device
__global__ __launch_bounds__(kBlock) void k_delta(double *__restrict__ m, size_t n, const double *__restrict__ total)
{
    const double mbar = total[0] / (double)n;
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (size_t)gridDim.x * kBlock)
        m[t] = m[t] / mbar - 1.0;
}

// f_R = fbar_R e^u at every cell
__global__ __launch_bounds__(kBlock) void k_fr(const double *__restrict__ u, double fbar, size_t n,
                                                 double *__restrict__ fr)
{
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (size_t)gridDim.x * kBlock)
        fr[t] = -fbar * exp(u[t]);
}

// a = pref * sum_cells w_cell * (f_R[+d] - f_R[-d]) / (2h)
__global__ __launch_bounds__(kBlock) void k_force_gather(const double *__restrict__ fr, const float *__restrict__ pos,
                                                           int64_t np, int lg, double h, double pref,
                                                           float *__restrict__ acc, int *__restrict__ flag)
{
    int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= np) return;
    const int mask = (1 << lg) - 1;
    int i0, j0, k0;
    double tx, ty, tz;
    bool ok = cic_axis(pos[3 * p + 0], h, mask, i0, tx) && cic_axis(pos[3 * p + 1], h, mask, j0, ty) &&
              cic_axis(pos[3 * p + 2], h, mask, k0, tz);
    if (!ok) {
        flag[0] = 1;
        const float nan = __builtin_nanf("");
        acc[3 * p + 0] = nan;
        acc[3 * p + 1] = nan;
        acc[3 * p + 2] = nan;
        return;
    }
    const double wx[2] = {1.0 - tx, tx}, wy[2] = {1.0 - ty, ty}, wz[2] = {1.0 - tz, tz};
    const int ii[2] = {i0, (i0 + 1) & mask}, jj[2] = {j0, (j0 + 1) & mask}, kk[2] = {k0, (k0 + 1) & mask};
    auto at = [&](int i, int j, int k) { return fr[((((size_t)i << lg) + j) << lg) + k]; };
    double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int i = ii[a], j = jj[b], k = kk[c];
                const double w = wx[a] * wy[b] * wz[c];
                gx += w * (at((i + 1) & mask, j, k) - at((i - 1) & mask, j, k));
                gy += w * (at(i, (j + 1) & mask, k) - at(i, (j - 1) & mask, k));
                gz += w * (at(i, j, (k + 1) & mask) - at(i, j, (k - 1) & mask));
            }
    const double s = pref / (2.0 * h);
    acc[3 * p + 0] = (float)(s * gx);
    acc[3 * p + 1] = (float)(s * gy);
    acc[3 * p + 2] = (float)(s * gz);
}

inline unsigned grid_for(size_t n, size_t cap) { return (unsigned)std::min<size_t>((n + kBlock - 1) / kBlock, cap); }

}  // namespace

}  // namespace mgfr

using namespace mgfr;

extern "C" int mgfr_assign_density(mgfr_ctx *c, const float *pos, const double *mass, int64_t np, double *delta)
{
    if (!c) return set_error(MGFR_ERR_ARG, "ctx is NULL");
    if (!pos) return set_error(MGFR_ERR_ARG, "pos is NULL");
    if (!delta) return set_error(MGFR_ERR_ARG, "delta is NULL");
    if (np < 1) return set_error(MGFR_ERR_ARG, "np must be >= 1, got %lld", (long long)np);
    const Level &L0 = c->lev[0];
    const size_t n = (size_t)L0.N * L0.N * L0.N;
    MGFR_HIP(hipMemsetAsync(delta, 0, n * sizeof(double), c->stream));
    MGFR_HIP(hipMemsetAsync(c->dflag, 0, sizeof(int), c->stream));
    const size_t pblocks = (size_t)((np + kBlock - 1) / kBlock);
    if (pblocks > 0x7fffffffULL) return set_error(MGFR_ERR_ARG, "np too large");
    k_cic_scatter<<<(unsigned)pblocks, kBlock, 0, c->stream>>>(pos, mass, np, L0.lg, L0.h, delta, c->dflag);
    unsigned g = grid_for(n, (size_t)c->nparts);
    k_sum_partial<<<g, kBlock, 0, c->stream>>>(delta, n, c->partial);
    k_sum_final<<<1, 1024, 0, c->stream>>>(c->partial, (int)g, c->dscal + 4);
    k_delta<<<grid_for(n, 8192), kBlock, 0, c->stream>>>(delta, n, c->dscal + 4);
    MGFR_HIP(hipGetLastError());
    int *hflag = (int *)(c->hscal + 6);
    MGFR_HIP(hipMemcpyAsync(hflag, c->dflag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    MGFR_HIP(hipMemcpyAsync(c->hscal + 5, c->dscal + 4, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    MGFR_HIP(hipStreamSynchronize(c->stream));
    if (*hflag) return set_error(MGFR_ERR_NONFINITE, "a particle position or mass is not finite");
    if (!(c->hscal[5] > 0) || !std::isfinite(c->hscal[5]))
        return set_error(MGFR_ERR_NONFINITE, "total assigned mass is not positive and finite");
    return MGFR_OK;
}

extern "C" int mgfr_fifth_force(mgfr_ctx *c, const double *u, const float *pos, int64_t np, float *acc)
{
    if (!c) return set_error(MGFR_ERR_ARG, "ctx is NULL");
    if (!u || !pos || !acc) return set_error(MGFR_ERR_ARG, "u, pos and acc must be non-NULL");
    if (np < 0) return set_error(MGFR_ERR_ARG, "np must be >= 0");
    if (np == 0) return MGFR_OK;
    const Level &L0 = c->lev[0];
    const size_t n = (size_t)L0.N * L0.N * L0.N;
    double *fr = L0.f;  // the level-0 source buffer is free between solves
    k_fr<<<grid_for(n, 8192), kBlock, 0, c->stream>>>(u, c->fbar, n, fr);
    MGFR_HIP(hipMemsetAsync(c->dflag, 0, sizeof(int), c->stream));
    const size_t pblocks = (size_t)((np + kBlock - 1) / kBlock);
    if (pblocks > 0x7fffffffULL) return set_error(MGFR_ERR_ARG, "np too large");
    const double pref = kCkms * kCkms / (2.0 * c->p.a);
    k_force_gather<<<(unsigned)pblocks, kBlock, 0, c->stream>>>(fr, pos, np, L0.lg, L0.h, pref, acc, c->dflag);
    MGFR_HIP(hipGetLastError());
    int *hflag = (int *)(c->hscal + 6);
    MGFR_HIP(hipMemcpyAsync(hflag, c->dflag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    MGFR_HIP(hipStreamSynchronize(c->stream));
    if (*hflag) return set_error(MGFR_ERR_NONFINITE, "a particle position is not finite");
    return MGFR_OK;
}
