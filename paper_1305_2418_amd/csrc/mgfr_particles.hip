// Particle <-> mesh steps: cloud-in-cell assignment (Sec. 3.1) and the fifth
// force gathered back to the particles (Sec. 2, Eq. modgrav_accel).
#include "mgfr_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

namespace mgfr {

namespace {

__device__ __forceinline__ double nanmax2(double a, double b) { return (a != a || a > b) ? a : b; }

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

// Cloud-in-cell assignment of binned particles.  A workgroup takes one work
// unit at a time (up to kUnit particles of one 8^3 tile, kUnitPer per
// thread), accumulates it in a 9^3 LDS window (lower corners in the tile,
// upper corners one cell beyond) and adds the window's non-zero entries to
// the mesh with float64 atomics.  (Storing the window cells 1..7 of a tile
// that is a single unit, which no other unit reaches, instead of adding them
// was slower: plain stores and atomics then share cache lines.)
__global__ __launch_bounds__(kBlock) void k_cic_units(const float *__restrict__ pos, const double *__restrict__ mass,
                                                        const uint32_t *__restrict__ perm,
                                                        const uint4 *__restrict__ units,
                                                        const uint32_t *__restrict__ total, int lg, double h,
                                                        double *__restrict__ m, int *__restrict__ flag)
{
    __shared__ double win[kWin3];
    const int tid = threadIdx.x;
    const int mask = (1 << lg) - 1, tl = lg - kBinLg, tmask = (1 << tl) - 1;
    const double r = 1.0 / h;
    const uint32_t U = *total;
    for (int e = tid; e < kWin3; e += kBlock) win[e] = 0.0;
    for (uint32_t u = blockIdx.x; u < U; u += gridDim.x) {
        const uint4 d = units[u];
        const int ti = (int)(d.x >> (2 * tl)) << kBinLg, tj = (int)((d.x >> tl) & tmask) << kBinLg,
                  tk = (int)(d.x & tmask) << kBinLg;
        float px[kUnitPer], py[kUnitPer], pz[kUnitPer];
        double pm[kUnitPer];
        bool live[kUnitPer];
#pragma unroll
        for (int q = 0; q < kUnitPer; ++q) {
            const uint32_t sl = d.y + tid + q * kBlock;
            live[q] = sl < d.z;
            px[q] = py[q] = pz[q] = 0.0f;
            pm[q] = 0.0;
            if (live[q]) {
                const size_t p = perm[sl];
                px[q] = pos[3 * p + 0];
                py[q] = pos[3 * p + 1];
                pz[q] = pos[3 * p + 2];
                pm[q] = mass ? mass[p] : 1.0;
            }
        }
        __syncthreads();  // the window is clear
#pragma unroll
        for (int q = 0; q < kUnitPer; ++q) {
            if (!live[q]) continue;
            int i0 = 0, j0 = 0, k0 = 0;
            double tx = 0.0, ty = 0.0, tz = 0.0;
            const bool ok = cic_axis_r(px[q], h, r, mask, i0, tx) & cic_axis_r(py[q], h, r, mask, j0, ty) &
                            cic_axis_r(pz[q], h, r, mask, k0, tz) & (bool)isfinite(pm[q]);
            const int a = i0 - ti, b = j0 - tj, c = k0 - tk;
            if (!ok || (unsigned)a >= (1u << kBinLg) || (unsigned)b >= (1u << kBinLg) ||
                (unsigned)c >= (1u << kBinLg)) {
                flag[0] = 1;
                continue;
            }
            const double mp = pm[q];
            const double wx0 = (1.0 - tx) * mp, wx1 = tx * mp, wy0 = 1.0 - ty, wy1 = ty, wz0 = 1.0 - tz, wz1 = tz;
            double *w0 = win + (a * kWin + b) * kWin + c;
            atomicAdd(w0, wx0 * wy0 * wz0);
            atomicAdd(w0 + 1, wx0 * wy0 * wz1);
            atomicAdd(w0 + kWin, wx0 * wy1 * wz0);
            atomicAdd(w0 + kWin + 1, wx0 * wy1 * wz1);
            atomicAdd(w0 + kWin * kWin, wx1 * wy0 * wz0);
            atomicAdd(w0 + kWin * kWin + 1, wx1 * wy0 * wz1);
            atomicAdd(w0 + kWin * kWin + kWin, wx1 * wy1 * wz0);
            atomicAdd(w0 + kWin * kWin + kWin + 1, wx1 * wy1 * wz1);
        }
        __syncthreads();
        // flush, clearing what was flushed for the next unit
        for (int e = tid; e < kWin3; e += kBlock) {
            const double v = win[e];
            if (v != 0.0) {
                const int a = e / (kWin * kWin), b = (e / kWin) % kWin, c = e % kWin;
                const size_t g = ((((size_t)((ti + a) & mask) << lg) + (size_t)((tj + b) & mask)) << lg) +
                                 (size_t)((tk + c) & mask);
                unsafeAtomicAdd(&m[g], v);
                win[e] = 0.0;
            }
        }
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

// Gradient sum g = sum_cells w_cell (f_R[+d] - f_R[-d]) at a particle with CIC
// fractions (tx, ty, tz), f_R read through get(di, dj, dk) = f_R at the lower
// CIC corner + (di, dj, dk), di in -1..2: the 32 distinct cells of the eight
// central differences (the 2x2x2 block and one layer beyond it on each side).
template <class G>
__device__ __forceinline__ void grad_sum(G get, double tx, double ty, double tz, double &gx, double &gy, double &gz)
{
    const double wx[2] = {1.0 - tx, tx}, wy[2] = {1.0 - ty, ty}, wz[2] = {1.0 - tz, tz};
    double B[2][2][2], X[2][2][2], Y[2][2][2], Z[2][2][2];  // X[s][b][c]: x layer s (0: -1, 1: +2)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
            for (int c = 0; c < 2; ++c) B[a][b][c] = get(a, b, c);
            X[0][a][b] = get(-1, a, b);
            X[1][a][b] = get(2, a, b);
            Y[0][a][b] = get(a, -1, b);
            Y[1][a][b] = get(a, 2, b);
            Z[0][a][b] = get(a, b, -1);
            Z[1][a][b] = get(a, b, 2);
        }
    gx = gy = gz = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const double w = wx[a] * wy[b] * wz[c];
                // f at +d and -d of block cell (a,b,c)
                const double xp = a ? X[1][b][c] : B[1][b][c], xm = a ? B[0][b][c] : X[0][b][c];
                const double yp = b ? Y[1][a][c] : B[a][1][c], ym = b ? B[a][0][c] : Y[0][a][c];
                const double zp = c ? Z[1][a][b] : B[a][b][1], zm = c ? B[a][b][0] : Z[0][a][b];
                gx += w * (xp - xm);
                gy += w * (yp - ym);
                gz += w * (zp - zm);
            }
}

__device__ __forceinline__ void store_nan3(float *__restrict__ acc, int64_t p)
{
    const float nan = __builtin_nanf("");
    acc[3 * p + 0] = nan;
    acc[3 * p + 1] = nan;
    acc[3 * p + 2] = nan;
}

// a = pref * sum_cells w_cell * (f_R[+d] - f_R[-d]) / (2h), f_R from global memory.
// Particles are visited in the order perm (the binning's tile order) when it
// is given, else in index order; each particle's result is the same either way.
__global__ __launch_bounds__(kBlock) void k_force_gather(const double *__restrict__ fr, const float *__restrict__ pos,
                                                           const uint32_t *__restrict__ perm, int64_t np, int lg,
                                                           double h, double pref, float *__restrict__ acc,
                                                           int *__restrict__ flag)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= np) return;
    const int64_t p = perm ? (int64_t)perm[i] : i;
    const int mask = (1 << lg) - 1;
    int i0, j0, k0;
    double tx, ty, tz;
    if (!(cic_axis(pos[3 * p + 0], h, mask, i0, tx) && cic_axis(pos[3 * p + 1], h, mask, j0, ty) &&
          cic_axis(pos[3 * p + 2], h, mask, k0, tz))) {
        flag[0] = 1;
        store_nan3(acc, p);
        return;
    }
    double gx, gy, gz;
    grad_sum([&](int di, int dj, int dk) {
        return fr[(((((size_t)((i0 + di) & mask)) << lg) + (size_t)((j0 + dj) & mask)) << lg) +
                  (size_t)((k0 + dk) & mask)];
    }, tx, ty, tz, gx, gy, gz);
    const double s = pref / (2.0 * h);
    acc[3 * p + 0] = (float)(s * gx);
    acc[3 * p + 1] = (float)(s * gy);
    acc[3 * p + 2] = (float)(s * gz);
}

constexpr int kFW = (1 << kBinLg) + 3;  // f_R window edge: a tile plus one cell below and two above
constexpr int kFW3 = kFW * kFW * kFW;
constexpr int kFWinMin = 48;             // smaller units read f_R from global memory

// The gradient sum of one particle read from global memory: the rare particle
// whose current position has left the tile it was binned in (positions changed
// since the binning).  Out of line and one block cell at a time, so that it
// adds neither registers nor code to the window path; the terms are those of
// grad_sum, in its order.
__device__ __noinline__ double3 grad_sum_global(const double *__restrict__ fr, int lg, int i0, int j0, int k0,
                                                double tx, double ty, double tz)
{
    const int mask = (1 << lg) - 1;
    auto at = [&](int di, int dj, int dk) {
        return fr[(((((size_t)((i0 + di) & mask)) << lg) + (size_t)((j0 + dj) & mask)) << lg) +
                  (size_t)((k0 + dk) & mask)];
    };
    double3 g = make_double3(0.0, 0.0, 0.0);
#pragma unroll 1
    for (int e = 0; e < 8; ++e) {
        const int a = e >> 2, b = (e >> 1) & 1, c = e & 1;
        const double w = (a ? tx : 1.0 - tx) * (b ? ty : 1.0 - ty) * (c ? tz : 1.0 - tz);
        g.x += w * (at(a + 1, b, c) - at(a - 1, b, c));
        g.y += w * (at(a, b + 1, c) - at(a, b - 1, c));
        g.z += w * (at(a, b, c + 1) - at(a, b, c - 1));
    }
    return g;
}

// The fifth force for binned particles: a workgroup takes one work unit at a
// time (up to kUnit particles of one tile), stages the tile's f_R window
// (11^3 values: one cell below the tile, two above) in LDS, loaded together
// with the unit's particles, and gathers from there (units of fewer than
// kFWinMin particles gather from global memory).  Any positions give the same
// result as k_force_gather.
__global__ __launch_bounds__(kBlock) void k_force_units(const double *__restrict__ fr, const float *__restrict__ pos,
                                                          const uint32_t *__restrict__ perm,
                                                          const uint4 *__restrict__ units,
                                                          const uint32_t *__restrict__ total, int lg, double h,
                                                          double pref, float *__restrict__ acc,
                                                          int *__restrict__ flag)
{
    __shared__ double win[kFW3];
    const int tid = threadIdx.x;
    const int mask = (1 << lg) - 1, tl = lg - kBinLg, tmask = (1 << tl) - 1;
    const double s = pref / (2.0 * h), r = 1.0 / h;
    const uint32_t U = *total;
    constexpr int kFWPer = (kFW3 + kBlock - 1) / kBlock;  // window values staged per thread
    for (uint32_t u = blockIdx.x; u < U; u += gridDim.x) {
        const uint4 d = units[u];
        const int ti = (int)(d.x >> (2 * tl)) << kBinLg, tj = (int)((d.x >> tl) & tmask) << kBinLg,
                  tk = (int)(d.x & tmask) << kBinLg;
        const bool use_win = d.z - d.y >= (uint32_t)kFWinMin;  // uniform over the workgroup
        // the window through registers, loaded together with the particles
        double wv[kFWPer];
#pragma unroll
        for (int q = 0; q < kFWPer; ++q) {
            const int e = tid + q * kBlock;
            wv[q] = 0.0;
            if (use_win && e < kFW3) {
                const int a = e / (kFW * kFW), b = (e / kFW) % kFW, c = e % kFW;
                wv[q] = fr[(((((size_t)((ti - 1 + a) & mask)) << lg) + (size_t)((tj - 1 + b) & mask)) << lg) +
                           (size_t)((tk - 1 + c) & mask)];
            }
        }
        uint32_t pid[kUnitPer];
        float px[kUnitPer], py[kUnitPer], pz[kUnitPer];
#pragma unroll
        for (int q = 0; q < kUnitPer; ++q) {
            const uint32_t sl = d.y + tid + q * kBlock;
            pid[q] = 0xffffffffu;
            px[q] = py[q] = pz[q] = 0.0f;
            if (sl < d.z) {
                pid[q] = perm[sl];
                px[q] = pos[3 * (size_t)pid[q] + 0];
                py[q] = pos[3 * (size_t)pid[q] + 1];
                pz[q] = pos[3 * (size_t)pid[q] + 2];
            }
        }
        __syncthreads();  // the previous unit's gathers are done
        if (use_win) {
#pragma unroll
            for (int q = 0; q < kFWPer; ++q)
                if (tid + q * kBlock < kFW3) win[tid + q * kBlock] = wv[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kUnitPer; ++q) {
            if (pid[q] == 0xffffffffu) continue;
            const size_t p = pid[q];
            int i0 = 0, j0 = 0, k0 = 0;
            double tx = 0.0, ty = 0.0, tz = 0.0;
            if (!(cic_axis_r(px[q], h, r, mask, i0, tx) & cic_axis_r(py[q], h, r, mask, j0, ty) &
                  cic_axis_r(pz[q], h, r, mask, k0, tz))) {
                flag[0] = 1;
                store_nan3(acc, (int64_t)p);
                continue;
            }
            const int a0 = i0 - ti, b0 = j0 - tj, c0 = k0 - tk;
            double gx, gy, gz;
            if (use_win && (unsigned)a0 < (1u << kBinLg) && (unsigned)b0 < (1u << kBinLg) &&
                (unsigned)c0 < (1u << kBinLg))
                grad_sum([&](int di, int dj, int dk) {
                    return win[((a0 + di + 1) * kFW + (b0 + dj + 1)) * kFW + (c0 + dk + 1)];
                }, tx, ty, tz, gx, gy, gz);
            else {
                const double3 g = grad_sum_global(fr, lg, i0, j0, k0, tx, ty, tz);
                gx = g.x;
                gy = g.y;
                gz = g.z;
            }
            acc[3 * p + 0] = (float)(s * gx);
            acc[3 * p + 1] = (float)(s * gy);
            acc[3 * p + 2] = (float)(s * gz);
        }
    }
}

// Psi = phi + (c^2/2) fbar e^u in place (the total potential of a
// particle-mesh step: g = -(1/a) grad Psi; u == NULL: phi alone)
__global__ __launch_bounds__(kBlock) void k_psi(double *__restrict__ phi, const double *__restrict__ u, double s,
                                                size_t n)
{
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (size_t)gridDim.x * kBlock)
        phi[t] = fma(s, exp(u[t]), phi[t]);
}

// mom += acc kick, then pos += mom drift, per component in float64 with
// explicit fused multiply-adds (the rounding is part of the definition), both
// stored as float32; positions are wrapped into [0, box).
__global__ __launch_bounds__(kBlock) void k_kick_drift(float *__restrict__ pos, float *__restrict__ mom,
                                                       const float *__restrict__ acc, size_t n3, double kick,
                                                       double drift, double box)
{
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < n3; t += (size_t)gridDim.x * kBlock) {
        double m = (double)mom[t];
        if (acc) m = fma((double)acc[t], kick, m);
        const float mf = (float)m;
        mom[t] = mf;
        double x = fma((double)mf, drift, (double)pos[t]);
        x -= box * floor(x / box);
        pos[t] = (float)x;
    }
}

// Zero an array of n doubles and one int flag: the clearing step of the
// allocation-free assignment (a kernel, not a memset, so that a captured
// graph replays it faithfully).
__global__ __launch_bounds__(kBlock) void k_zero_mesh(double *__restrict__ x, size_t n, int *__restrict__ flag)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) flag[0] = 0;
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (size_t)gridDim.x * kBlock) x[t] = 0.0;
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
    c->perm_np = 0;
    if (c->binning && np <= c->bin_cap) {
        if (int e = bin_particles(c, pos, np)) return e;
        k_cic_units<<<c->unit_grid, kBlock, 0, c->stream>>>(pos, mass, c->perm, c->units, c->unit_total, L0.lg,
                                                             L0.h, delta, c->dflag);
    } else {
        k_cic_scatter<<<(unsigned)pblocks, kBlock, 0, c->stream>>>(pos, mass, np, L0.lg, L0.h, delta, c->dflag);
    }
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
    if (c->perm_np == np && c->perm) {
        k_force_units<<<c->unit_grid, kBlock, 0, c->stream>>>(fr, pos, c->perm, c->units, c->unit_total, L0.lg,
                                                               L0.h, pref, acc, c->dflag);
    } else {
        k_force_gather<<<(unsigned)pblocks, kBlock, 0, c->stream>>>(fr, pos, nullptr, np, L0.lg, L0.h, pref, acc,
                                                                     c->dflag);
    }
    MGFR_HIP(hipGetLastError());
    int *hflag = (int *)(c->hscal + 6);
    MGFR_HIP(hipMemcpyAsync(hflag, c->dflag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    MGFR_HIP(hipStreamSynchronize(c->stream));
    if (*hflag) return set_error(MGFR_ERR_NONFINITE, "a particle position is not finite");
    return MGFR_OK;
}

extern "C" int mgfr_pm_accel(mgfr_ctx *c, const double *delta, const double *u, const float *pos, int64_t np,
                             float *acc)
{
    if (!c) return set_error(MGFR_ERR_ARG, "ctx is NULL");
    if (!delta || !pos || !acc) return set_error(MGFR_ERR_ARG, "delta, pos and acc must be non-NULL");
    if (np < 0) return set_error(MGFR_ERR_ARG, "np must be >= 0");
    if (np == 0) return MGFR_OK;
    const Level &L0 = c->lev[0];
    const size_t n = (size_t)L0.N * L0.N * L0.N;
    double *psi = L0.f;  // the level-0 source buffer is free between solves
    if (int rc = pm_potential(c, delta, psi)) return rc;
    if (u) k_psi<<<grid_for(n, 8192), kBlock, 0, c->stream>>>(psi, u, 0.5 * kCkms * kCkms * c->fbar, n);
    MGFR_HIP(hipMemsetAsync(c->dflag, 0, sizeof(int), c->stream));
    const size_t pblocks = (size_t)((np + kBlock - 1) / kBlock);
    if (pblocks > 0x7fffffffULL) return set_error(MGFR_ERR_ARG, "np too large");
    const double pref = -1.0 / c->p.a;
    if (c->perm_np == np && c->perm) {
        k_force_units<<<c->unit_grid, kBlock, 0, c->stream>>>(psi, pos, c->perm, c->units, c->unit_total, L0.lg,
                                                               L0.h, pref, acc, c->dflag);
    } else {
        k_force_gather<<<(unsigned)pblocks, kBlock, 0, c->stream>>>(psi, pos, nullptr, np, L0.lg, L0.h, pref, acc,
                                                                     c->dflag);
    }
    MGFR_HIP(hipGetLastError());
    int *hflag = (int *)(c->hscal + 6);
    MGFR_HIP(hipMemcpyAsync(hflag, c->dflag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    MGFR_HIP(hipStreamSynchronize(c->stream));
    if (*hflag) return set_error(MGFR_ERR_NONFINITE, "a particle position is not finite");
    return MGFR_OK;
}

extern "C" int mgfr_kick_drift(mgfr_ctx *c, float *pos, float *mom, const float *acc, int64_t np, double kick,
                               double drift)
{
    if (!c) return set_error(MGFR_ERR_ARG, "ctx is NULL");
    if (!pos || !mom) return set_error(MGFR_ERR_ARG, "pos and mom must be non-NULL");
    if (np < 0) return set_error(MGFR_ERR_ARG, "np must be >= 0");
    if (!std::isfinite(kick) || !std::isfinite(drift)) return set_error(MGFR_ERR_ARG, "kick and drift must be finite");
    if (np == 0) return MGFR_OK;
    const size_t n3 = 3 * (size_t)np;
    k_kick_drift<<<grid_for(n3, 65536), kBlock, 0, c->stream>>>(pos, mom, acc, n3, kick, drift, c->p.box);
    MGFR_HIP(hipGetLastError());
    return MGFR_OK;
}

extern "C" int mgfr_pm_step(mgfr_ctx *c, float *pos, float *mom, float *acc, int64_t np, double a1, double *delta,
                            double *u, mgfr_stats *st)
{
    if (!c) return set_error(MGFR_ERR_ARG, "ctx is NULL");
    if (!pos || !mom || !acc || !delta || !u) return set_error(MGFR_ERR_ARG, "null argument");
    if (np < 1) return set_error(MGFR_ERR_ARG, "np must be >= 1");
    const double a0 = c->p.a;
    if (!(a1 > a0) || !std::isfinite(a1)) return set_error(MGFR_ERR_ARG, "a1 must exceed the current a = %g", a0);
    const double om = c->p.omega_m, ol = c->p.omega_l;
    auto H = [&](double a) { return 100.0 * std::sqrt(om / (a * a * a) + ol); };  // km/s per Mpc/h
    const double am = 0.5 * (a0 + a1);
    const double K1 = (am - a0) / H(0.5 * (a0 + am)), K2 = (a1 - am) / H(0.5 * (am + a1));
    const double D = (a1 - a0) / (am * am * am * H(am));
    int rc;
    if ((rc = mgfr_kick_drift(c, pos, mom, acc, np, K1, D))) return rc;
    if ((rc = mgfr_set_scale_factor(c, a1))) return rc;
    if ((rc = mgfr_assign_density(c, pos, nullptr, np, delta))) return rc;
    const int status = mgfr_solve(c, delta, u, nullptr, st);
    if (status < 0) return status;
    if ((rc = mgfr_pm_accel(c, delta, u, pos, np, acc))) return rc;
    if ((rc = mgfr_kick_drift(c, pos, mom, acc, np, K2, 0.0))) return rc;
    return status;
}

extern "C" int mgfr_reserve_particles(mgfr_ctx *c, int64_t max_np)
{
    if (!c) return set_error(MGFR_ERR_ARG, "ctx is NULL");
    if (max_np < 0) return set_error(MGFR_ERR_ARG, "max_np must be >= 0");
    return bin_reserve(c, max_np);
}

extern "C" int mgfr_set_binning(mgfr_ctx *c, int on)
{
    if (!c) return set_error(MGFR_ERR_ARG, "ctx is NULL");
    c->binning = on ? 1 : 0;
    c->perm_np = 0;
    return MGFR_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free assignment.  The context-free variant of
// mgfr_assign_density keeps its reduction workspace in a file-scope device
// array instead of a context: kStaticParts partial sums of the total mass,
// the total, and the non-finite flag.  Each device the library runs on holds
// one copy until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns for that device.
namespace {

constexpr int kStaticParts = 2048;
constexpr int kStaticMaxMesh = 1024;
constexpr int kStaticMaxDevices = 64;
static __device__ __align__(256) double scratch[kStaticParts + 4];

std::mutex g_scratch_mu;
double *g_scratch_ptr[kStaticMaxDevices] = {};

int static_scratch(double **out)
{
    int dev = 0;
    MGFR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kStaticMaxDevices)
        return set_error(MGFR_ERR_ARG, "device %d is beyond the %d devices the allocation-free assignment supports",
                         dev, kStaticMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        double *ptr = nullptr;
        MGFR_HIP(hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return set_error(MGFR_ERR_HIP, "hipGetSymbolAddress returned NULL for the assignment scratch");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MGFR_OK;
}

}  // namespace

extern "C" int mgfr_assign_density_noalloc(int mesh, double box, void *stream, const float *pos, const double *mass,
                                           int64_t np, double *delta)
{
    if (!pos) return set_error(MGFR_ERR_ARG, "pos is NULL");
    if (!delta) return set_error(MGFR_ERR_ARG, "delta is NULL");
    if (np < 1) return set_error(MGFR_ERR_ARG, "np must be >= 1, got %lld", (long long)np);
    if (mesh < 8 || (mesh & (mesh - 1)))
        return set_error(MGFR_ERR_ARG, "mesh must be a power of two >= 8, got %d", mesh);
    if (mesh > kStaticMaxMesh)
        return set_error(MGFR_ERR_ARG, "mesh %d exceeds the maximum %d of the allocation-free assignment", mesh,
                         kStaticMaxMesh);
    if (!(box > 0) || !std::isfinite(box)) return set_error(MGFR_ERR_ARG, "box must be > 0 and finite");
    const size_t pblocks = (size_t)((np + kBlock - 1) / kBlock);
    if (pblocks > 0x7fffffffULL) return set_error(MGFR_ERR_ARG, "np too large");
    double *sc = nullptr;
    if (int e = static_scratch(&sc)) return e;
    double *partial = sc, *total = sc + kStaticParts;
    int *flag = (int *)(sc + kStaticParts + 1);
    int lg = 0;
    while ((1 << lg) < mesh) ++lg;
    const double h = box / mesh;
    const size_t n = (size_t)mesh * mesh * mesh;
    hipStream_t st = (hipStream_t)stream;
    k_zero_mesh<<<grid_for(n, 8192), kBlock, 0, st>>>(delta, n, flag);
    k_cic_scatter<<<(unsigned)pblocks, kBlock, 0, st>>>(pos, mass, np, lg, h, delta, flag);
    const unsigned g = grid_for(n, (size_t)kStaticParts);
    k_sum_partial<<<g, kBlock, 0, st>>>(delta, n, partial);
    k_sum_final<<<1, 1024, 0, st>>>(partial, (int)g, total);
    k_delta<<<grid_for(n, 8192), kBlock, 0, st>>>(delta, n, total);
    MGFR_HIP(hipGetLastError());
    double back[2] = {0.0, 0.0};  // total, flag word
    MGFR_HIP(hipMemcpyAsync(back, total, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    MGFR_HIP(hipStreamSynchronize(st));
    int hflag = 0;
    memcpy(&hflag, &back[1], sizeof(int));
    if (hflag) return set_error(MGFR_ERR_NONFINITE, "a particle position or mass is not finite");
    if (!(back[0] > 0) || !std::isfinite(back[0]))
        return set_error(MGFR_ERR_NONFINITE, "total assigned mass is not positive and finite");
    return MGFR_OK;
}
