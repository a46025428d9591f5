// Block-structured refined levels with the one-way interface of Sec. 3.3
// (steps 9-12).  The base mesh (N0^3) is solved by the uniform solver; level
// l = 1, 2 has N_l = N0 2^l cells per side and consists of 8^3-cell blocks:
// a cell of level l-1 holding more than 8 particles (nearest-grid-point
// count) refines the aligned 4^3 group of level-(l-1) cells around it into
// one level-l block.  Level-2 blocks also refine every level-1 block within
// two level-1 cells of them (proper nesting: the ghost cells of level 2 and
// the parents they are prolonged from lie on level 1).
//
// Masses (Sec. 3.1): one pass over the particles assigns each one's cube --
// side of the finest cell containing it -- to the leaf cells of the composite
// mesh it overlaps; coarser cells covered by a finer level then receive the
// sums of their daughters, and the base mesh is solved from the result.
//
// A level is solved after its parent.  Its initial guess and the ghost layer
// around the union of its blocks are the linear prolongation (Sec. 3.3) of the
// parent solution; ghosts stay fixed.  The level's FAS V-cycles use the union
// of blocks at 1/2, 1/4 and 1/8 resolution as coarse grids (block-aligned, so
// every coarse cell is fully covered and the paper's mask is 1 on all of
// them); coarse cells outside the union hold the solution of the level at
// that resolution (restricted from the base below the base resolution) and
// are never updated, and the correction is zero there.
//
// Storage: each block keeps, per sublevel m (side b = 8 >> m), a padded
// (b+2)^3 array; ghost faces towards a neighbouring block are refreshed by a
// halo exchange after every update, the others hold the frozen values.
#include "mgfr_internal.h"
#include "mgfr_ops.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

namespace mgfr {
namespace {

constexpr int kSub = 4;  // sublevels 8^3, 4^3, 2^3, 1^3 per block
constexpr int kMaxRef = 2;

__host__ __device__ inline int sub_b(int m) { return 8 >> m; }
__host__ __device__ inline int sub_p(int m) { return (8 >> m) + 2; }
__host__ __device__ inline int sub_vol(int m) { return sub_p(m) * sub_p(m) * sub_p(m); }

struct LevelDev {
    int lg;                  // N_l = 2^lg
    int nb;                  // blocks
    int mlg;                 // block-map side 2^mlg (= N_l / 8)
    const int *map;          // block id or -1 for every 8^3 block position
    const int *org;          // [nb][3] block origin in level cells
    const int *nbr;          // [nb][6] face neighbours (-x,+x,-y,+y,-z,+z) or -1
    double *u[kSub], *f[kSub], *ub[kSub], *E[kSub];
    // float32 correction cycle (mixed precision): e, u in float32, r, restricted e
    float *e32[kSub], *u32[kSub], *r32[kSub], *eb32[kSub];
    const double *exp2tab;   // 2^(j/64) for the table-driven exponential (copied to LDS by the kernels)
};

struct Composite {  // solutions available for frozen / ghost values
    const double *u0;
    int lg0;
    LevelDev lev[kMaxRef + 1];  // lev[1], lev[2] valid when solved
    int nsolved;                // levels 1..nsolved hold solutions
};

__device__ __forceinline__ int wrapn(int i, int n) { return i & (n - 1); }

__device__ __forceinline__ size_t pidx(int m, int x, int y, int z)
{
    const int p = sub_p(m);
    return ((size_t)(x + 1) * p + (y + 1)) * p + (z + 1);
}

// solution of level lr at one of its cells (lr <= nsolved; lr < 0: base means)
__device__ double comp_at(const Composite &C, int lr, int i, int j, int k)
{
    if (lr >= 1) {
        const LevelDev &L = C.lev[lr];
        const int N = 1 << L.lg;
        i = wrapn(i, N);
        j = wrapn(j, N);
        k = wrapn(k, N);
        const int M = 1 << L.mlg;
        const int b = L.map[((size_t)(i >> 3) * M + (j >> 3)) * M + (k >> 3)];
        if (b >= 0) return L.u[0][(size_t)b * sub_vol(0) + pidx(0, i & 7, j & 7, k & 7)];
        // outside the level: excluded by proper nesting; make a violation loud
        return __builtin_nan("");
    }
    const int N0 = 1 << C.lg0;
    if (lr == 0) return C.u0[cidx(wrapn(i, N0), wrapn(j, N0), wrapn(k, N0), C.lg0)];
    const int f = 1 << (-lr), Nr = N0 >> (-lr);
    i = wrapn(i, Nr);
    j = wrapn(j, Nr);
    k = wrapn(k, Nr);
    double s = 0.0;
    for (int a = 0; a < f; ++a)
        for (int b = 0; b < f; ++b)
            for (int c = 0; c < f; ++c) s += C.u0[cidx(i * f + a, j * f + b, k * f + c, C.lg0)];
    return s / (double)(f * f * f);
}

// linear prolongation of the level-(l-1) solution to cell (i,j,k) of level l
__device__ double prolong_parent(const Composite &C, int l, int i, int j, int k)
{
    const int lp = l - 1;
    const int I = i >> 1, J = j >> 1, K = k >> 1;  // arithmetic shift: floor for negatives
    double v = comp_at(C, lp, I, J, K);
    v += ((i & 1) ? 0.125 : -0.125) * (comp_at(C, lp, I + 1, J, K) - comp_at(C, lp, I - 1, J, K));
    v += ((j & 1) ? 0.125 : -0.125) * (comp_at(C, lp, I, J + 1, K) - comp_at(C, lp, I, J - 1, K));
    v += ((k & 1) ? 0.125 : -0.125) * (comp_at(C, lp, I, J, K + 1) - comp_at(C, lp, I, J, K - 1));
    return v;
}

// ------------------------------------------------------------------ kernels

// (The particle loops below run in the caller's particle order: in the base
// binning's tile order, same-cell atomics of dense halos collide within a wave
// and these loops ran slower.)
__global__ void k_ngp_count(const float *__restrict__ pos, int64_t np, int lg, double h, int *__restrict__ cnt)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int N = 1 << lg;
    int c[3];
    for (int d = 0; d < 3; ++d) {
        const double x = (double)pos[3 * p + d] / h;
        if (!(fabs(x) < 4.0e18)) return;
        c[d] = (int)((long long)floor(x) & (N - 1));
    }
    atomicAdd(&cnt[cidx(c[0], c[1], c[2], lg)], 1);
}

// nearest-grid-point counts at level-l resolution, into the level's blocks
__global__ void k_ngp_count_blocks(const float *__restrict__ pos, int64_t np, LevelDev L, double h,
                                   int *__restrict__ cnt)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int N = 1 << L.lg, M = 1 << L.mlg;
    int c[3];
    for (int d = 0; d < 3; ++d) {
        const double x = (double)pos[3 * p + d] / h;
        if (!(fabs(x) < 4.0e18)) return;
        c[d] = (int)((long long)floor(x) & (N - 1));
    }
    const int b = L.map[((size_t)(c[0] >> 3) * M + (c[1] >> 3)) * M + (c[2] >> 3)];
    if (b >= 0) atomicAdd(&cnt[(size_t)b * 512 + ((c[0] & 7) * 8 + (c[1] & 7)) * 8 + (c[2] & 7)], 1);
}

// Refinement flags (device byte maps of block positions, one per refined level).
// Level 1: the aligned 4^3 group of base cells around every base cell holding
// more than 8 particles.
__global__ void k_flag_base(const int *__restrict__ cnt, int lg0, unsigned char *__restrict__ blk1)
{
    const int N = 1 << lg0, M = N / 4;
    const size_t n = (size_t)N * N * N;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        if (cnt[t] > 8) {
            const int k = (int)(t & (N - 1)), j = (int)((t >> lg0) & (N - 1)), i = (int)(t >> (2 * lg0));
            blk1[((size_t)(i >> 2) * M + (j >> 2)) * M + (k >> 2)] = 1;
        }
}

// Level 2: the same around every cell of a level-1 block holding more than 8 particles.
__global__ void k_flag_l1(const int *__restrict__ cntb, int nb1, const int *__restrict__ org1, int N1,
                          unsigned char *__restrict__ blk2)
{
    const int M = N1 / 4;
    const size_t n = (size_t)nb1 * 512;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        if (cntb[t] > 8) {
            const int b = (int)(t >> 9), c = (int)(t & 511);
            const int i = org1[3 * b] + (c >> 6), j = org1[3 * b + 1] + ((c >> 3) & 7), k = org1[3 * b + 2] + (c & 7);
            blk2[((size_t)(i >> 2) * M + (j >> 2)) * M + (k >> 2)] = 1;
        }
}

// Proper nesting: every level-1 block holding a level-1 cell within two cells of
// a flagged level-2 block is flagged too.  The 8-cell range [4b - 2, 4b + 5]
// along an axis touches at most two level-1 blocks: those of its two ends.
__global__ void k_nest(const unsigned char *__restrict__ blk2, int N1, unsigned char *__restrict__ blk1)
{
    const int M2 = N1 / 4, M1 = N1 / 8;
    const size_t n = (size_t)M2 * M2 * M2;
    auto blk_of = [&](int c) { return (((c % N1) + N1) % N1) / 8; };
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        if (!blk2[t]) continue;
        const int bk = (int)(t % M2), bj = (int)((t / M2) % M2), bi = (int)(t / ((size_t)M2 * M2));
        const int xi[2] = {blk_of(4 * bi - 2), blk_of(4 * bi + 5)}, xj[2] = {blk_of(4 * bj - 2), blk_of(4 * bj + 5)},
                  xk[2] = {blk_of(4 * bk - 2), blk_of(4 * bk + 5)};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c) blk1[((size_t)xi[a] * M1 + xj[b]) * M1 + xk[c]] = 1;
    }
}

// Composite-mesh view for the mass assignment: block maps of the refined
// levels and the mass accumulators of every level (base mesh; interior cells
// of sublevel 0 of each level's blocks).
struct CicMaps {
    int nref, lg0;
    double box;
    const int *map[kMaxRef + 1];  // map[l], l >= 1: block id or -1 per block position (side N_l / 8)
    double *m0;                   // [N0^3]
    double *f0[kMaxRef + 1];      // f0[l], l >= 1: sublevel-0 padded arrays of level l's blocks
};

// block id of cell (i,j,k) of level l, any integer indices (wrapped periodically)
__device__ __forceinline__ int cic_blk(const CicMaps &Q, int l, long long i, long long j, long long k)
{
    const int lg = Q.lg0 + l, M = 1 << (lg - 3);
    const long long m = (1LL << lg) - 1;
    const int a = (int)(i & m), b = (int)(j & m), c = (int)(k & m);
    return Q.map[l][((size_t)(a >> 3) * M + (b >> 3)) * M + (c >> 3)];
}

// cell (i,j,k) (wrapped) of level l is a leaf of the composite mesh: inside a
// level-l block (every base cell) and not covered by a level-(l+1) block
__device__ __forceinline__ bool cic_leaf(const CicMaps &Q, int l, long long i, long long j, long long k)
{
    if (l >= 1 && cic_blk(Q, l, i, j, k) < 0) return false;
    if (l < Q.nref && cic_blk(Q, l + 1, 2 * i, 2 * j, 2 * k) >= 0) return false;
    return true;
}

// add v to the mass of leaf cell (i,j,k) of level l (cic_leaf must hold)
__device__ __forceinline__ void cic_add(const CicMaps &Q, int l, long long ii, long long jj, long long kk, double v)
{
    const long long m = (1LL << (Q.lg0 + l)) - 1;
    const int i = (int)(ii & m), j = (int)(jj & m), k = (int)(kk & m);
    if (l == 0) {
        unsafeAtomicAdd(&Q.m0[cidx(i, j, k, Q.lg0)], v);
    } else {
        const int b = cic_blk(Q, l, i, j, k);
        unsafeAtomicAdd(&Q.f0[l][(size_t)b * sub_vol(0) + pidx(0, i & 7, j & 7, k & 7)], v);
    }
}

// Cloud-in-cell masses on the composite mesh (Sec. 3.1): each particle is a
// cube whose side is that of the finest cell containing it; every leaf cell
// it overlaps, of any level, gets the overlapping fraction of the unit mass.
// When the cube's eight cells at that level are all leaves (the common case)
// these are the usual weights (1 - t, t) per axis; otherwise the overlaps are
// computed cell by cell over every level.
// finest level whose blocks contain position x (0: the base mesh)
__device__ __forceinline__ int cic_level(const CicMaps &Q, const double x[3])
{
    for (int l = Q.nref; l >= 1; --l) {
        const double h = Q.box / (double)(1 << (Q.lg0 + l));
        if (cic_blk(Q, l, (long long)floor(x[0] / h), (long long)floor(x[1] / h), (long long)floor(x[2] / h)) >= 0)
            return l;
    }
    return 0;
}

// the eight CIC cells (i0..i0+1, ...) of level lp are all leaves
__device__ __forceinline__ bool cic_all_leaf(const CicMaps &Q, int lp, int i0, int j0, int k0)
{
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c)
                if (!cic_leaf(Q, lp, i0 + a, j0 + b, k0 + c)) return false;
    return true;
}

// position of particle p; false (and the flag set) if it is not finite or
// absurdly distant (cell indices must fit 64 bits)
__device__ __forceinline__ bool cic_position(const float *__restrict__ pos, int64_t p, double x[3],
                                             int *__restrict__ flag)
{
    for (int d = 0; d < 3; ++d) x[d] = (double)pos[3 * p + d];
    if (!(fabs(x[0]) < 1e15 && fabs(x[1]) < 1e15 && fabs(x[2]) < 1e15)) {
        flag[0] = 1;
        return false;
    }
    return true;
}

// The whole assignment of particle p with global atomics: the usual weights
// when its eight cells at level lp are leaves, else the overlaps cell by cell
// over every level.
__device__ void cic_composite_one(const float *__restrict__ pos, int64_t p, const CicMaps &Q, int *__restrict__ flag)
{
    double x[3];
    if (!cic_position(pos, p, x, flag)) return;
    const int lp = cic_level(Q, x);
    const int lgp = Q.lg0 + lp, mask = (1 << lgp) - 1;
    const double s = Q.box / (double)(1 << lgp);
    int i0, j0, k0;
    double tx, ty, tz;
    if (!(cic_axis((float)x[0], s, mask, i0, tx) && cic_axis((float)x[1], s, mask, j0, ty) &&
          cic_axis((float)x[2], s, mask, k0, tz))) {
        flag[0] = 1;
        return;
    }
    if (cic_all_leaf(Q, lp, i0, j0, k0)) {
        const double wx[2] = {1.0 - tx, tx}, wy[2] = {1.0 - ty, ty}, wz[2] = {1.0 - tz, tz};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c) cic_add(Q, lp, i0 + a, j0 + b, k0 + c, wx[a] * wy[b] * wz[c]);
        return;
    }
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = x[d] - 0.5 * s;
        hi[d] = x[d] + 0.5 * s;
    }
    for (int l = 0; l <= Q.nref; ++l) {
        const double h = Q.box / (double)(1 << (Q.lg0 + l));
        long long c0[3], c1[3];
        for (int d = 0; d < 3; ++d) {
            c0[d] = (long long)floor(lo[d] / h);
            c1[d] = (long long)floor(hi[d] / h);
        }
        for (long long i = c0[0]; i <= c1[0]; ++i)
            for (long long j = c0[1]; j <= c1[1]; ++j)
                for (long long k = c0[2]; k <= c1[2]; ++k) {
                    const long long c[3] = {i, j, k};
                    double v = 1.0;
                    for (int d = 0; d < 3; ++d) {
                        const double a = fmax(lo[d], (double)c[d] * h), b = fmin(hi[d], (double)(c[d] + 1) * h);
                        v *= b > a ? (b - a) / s : 0.0;
                    }
                    if (v > 0.0 && cic_leaf(Q, l, i, j, k)) cic_add(Q, l, i, j, k, v);
                }
    }
}

__global__ void k_amr_cic_composite(const float *__restrict__ pos, int64_t np, CicMaps Q, int *__restrict__ flag)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < np) cic_composite_one(pos, p, Q, flag);
}

// Binned composite assignment.  Sort keys: a particle whose eight CIC cells
// at its level lp are all leaves gets koff[lp] + the position of the aligned
// 8^3 group of level-lp cells holding its lower corner (row-major over the
// N_lp / 8 groups per axis); every other particle (a cube overlapping leaves
// of several levels, a bad position) gets the largest key koff[nref + 1] and
// takes the general path.
struct CicKeys {
    uint32_t koff[kMaxRef + 2];
};

__global__ __launch_bounds__(kBlock) void k_amr_cic_keys(const float *__restrict__ pos, int64_t np, CicMaps Q,
                                                           CicKeys K, uint32_t *__restrict__ key,
                                                           uint32_t *__restrict__ idx)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= np) return;
    idx[p] = (uint32_t)p;
    uint32_t k = K.koff[Q.nref + 1];
    double x[3];
    int dummy = 0;
    if (cic_position(pos, p, x, &dummy)) {
        const int lp = cic_level(Q, x);
        const int lgp = Q.lg0 + lp, mask = (1 << lgp) - 1;
        const double s = Q.box / (double)(1 << lgp);
        int i0, j0, k0;
        double t;
        if (cic_axis(pos[3 * p + 0], s, mask, i0, t) && cic_axis(pos[3 * p + 1], s, mask, j0, t) &&
            cic_axis(pos[3 * p + 2], s, mask, k0, t) && cic_all_leaf(Q, lp, i0, j0, k0)) {
            const uint32_t gl = (uint32_t)(lgp - kBinLg);
            k = K.koff[lp] + (((((uint32_t)i0 >> kBinLg) << gl) | ((uint32_t)j0 >> kBinLg)) << gl) +
                ((uint32_t)k0 >> kBinLg);
        }
    }
    key[p] = k;
}

// Workgroup b takes the sorted slots [b kCicChunk, (b + 1) kCicChunk) and
// walks their runs of equal key as the uniform binned assignment does: each
// run of a group of level-l cells is accumulated in a 9^3 LDS window (lower
// corners in the group, upper corners one cell beyond, all leaves), whose
// non-zero entries then go to the level's cells with float64 atomics (the
// cells one beyond may belong to a neighbouring block).  The general-path
// runs, last in the order, are left to k_amr_cic_general.
__global__ __launch_bounds__(kBlock) void k_amr_cic_binned(const float *__restrict__ pos,
                                                             const uint32_t *__restrict__ key_s,
                                                             const uint32_t *__restrict__ perm, int64_t np,
                                                             CicMaps Q, CicKeys K, int *__restrict__ flag)
{
    __shared__ double win[kWin3];
    __shared__ int red[kBlock / 64];
    const int tid = threadIdx.x;
    const int64_t start = (int64_t)blockIdx.x * kCicChunk;
    const int64_t end = start + kCicChunk < np ? start + kCicChunk : np;
    const uint32_t ksent = K.koff[Q.nref + 1];
    uint32_t key[kCicPer];
    float px[kCicPer], py[kCicPer], pz[kCicPer];
#pragma unroll
    for (int s = 0; s < kCicPer; ++s) {
        const int64_t i = start + tid + (int64_t)s * kBlock;
        key[s] = 0xffffffffu;  // above every key
        px[s] = py[s] = pz[s] = 0.0f;
        if (i < end) {
            key[s] = key_s[i];
            const size_t p = perm[i];
            px[s] = pos[3 * p + 0];
            py[s] = pos[3 * p + 1];
            pz[s] = pos[3 * p + 2];
        }
    }
    for (int e = tid; e < kWin3; e += kBlock) win[e] = 0.0;
    int64_t cur = start;
    while (cur < end) {
        const uint32_t t = key_s[cur];  // the same in every thread
        if (t >= ksent) break;          // the rest of the chunk takes the general path
        int cnt = 0;
#pragma unroll
        for (int s = 0; s < kCicPer; ++s) cnt += key[s] <= t ? 1 : 0;
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        if ((tid & 63) == 0) red[tid >> 6] = cnt;
        __syncthreads();
        int total = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) total += red[w];
        const int64_t rend = start + total > cur ? start + total : cur + 1;
        int l = 0;
        while (l < Q.nref && t >= K.koff[l + 1]) ++l;
        const int lg = Q.lg0 + l, gl = lg - kBinLg, gmask = (1 << gl) - 1, mask = (1 << lg) - 1;
        const uint32_t q = t - K.koff[l];
        const int ti = (int)(q >> (2 * gl)) << kBinLg, tj = (int)((q >> gl) & gmask) << kBinLg,
                  tk = (int)(q & gmask) << kBinLg;
        const double h = Q.box / (double)(1 << lg);
#pragma unroll
        for (int s = 0; s < kCicPer; ++s) {
            if (key[s] != t) continue;
            int i0, j0, k0;
            double tx, ty, tz;
            const bool ok = cic_axis(px[s], h, mask, i0, tx) && cic_axis(py[s], h, mask, j0, ty) &&
                            cic_axis(pz[s], h, mask, k0, tz);
            const int a = i0 - ti, b = j0 - tj, c = k0 - tk;
            if (!ok || (unsigned)a >= (1u << kBinLg) || (unsigned)b >= (1u << kBinLg) ||
                (unsigned)c >= (1u << kBinLg)) {
                flag[0] = 1;
                continue;
            }
            const double wx0 = 1.0 - tx, wx1 = tx, wy0 = 1.0 - ty, wy1 = ty, wz0 = 1.0 - tz, wz1 = tz;
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
        for (int e = tid; e < kWin3; e += kBlock) {
            const double v = win[e];
            if (v != 0.0) {
                const int a = e / (kWin * kWin), b = (e / kWin) % kWin, c = e % kWin;
                cic_add(Q, l, ti + a, tj + b, tk + c, v);
                win[e] = 0.0;
            }
        }
        __syncthreads();
        cur = rend;
    }
}

// the particles of the general path (largest key, sorted last)
__global__ void k_amr_cic_general(const float *__restrict__ pos, const uint32_t *__restrict__ key_s,
                                  const uint32_t *__restrict__ perm, int64_t np, CicMaps Q, uint32_t ksent,
                                  int *__restrict__ flag)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x)
        if (key_s[i] == ksent) cic_composite_one(pos, (int64_t)perm[i], Q, flag);
}

// Masses of the level-l cells covered by level-(l+1) blocks: the sum of their
// eight daughters (Sec. 3.1).  One thread per coarse cell: each level-(l+1)
// block covers an aligned 4^3 group of level-l cells.
__global__ void k_amr_mass_up(CicMaps Q, int l, int nbf, const int *__restrict__ orgf)
{
    const size_t n = (size_t)nbf * 64;
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
        const int b = (int)(id >> 6), c = (int)(id & 63);
        const int a0 = c >> 4, b0 = (c >> 2) & 3, c0 = c & 3;
        const double *F = Q.f0[l + 1] + (size_t)b * sub_vol(0);
        double sum = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int bb = 0; bb < 2; ++bb)
                for (int cc = 0; cc < 2; ++cc) sum += F[pidx(0, 2 * a0 + a, 2 * b0 + bb, 2 * c0 + cc)];
        const int i = (orgf[3 * b] >> 1) + a0, j = (orgf[3 * b + 1] >> 1) + b0, k = (orgf[3 * b + 2] >> 1) + c0;
        if (l == 0) {
            Q.m0[cidx(i, j, k, Q.lg0)] = sum;
        } else {
            const int pb = cic_blk(Q, l, i, j, k);  // exists: level-(l+1) blocks nest in level l
            if (pb >= 0) Q.f0[l][(size_t)pb * sub_vol(0) + pidx(0, i & 7, j & 7, k & 7)] = sum;
        }
    }
}

__global__ __launch_bounds__(256) void k_amr_sum_partial(const double *__restrict__ x, size_t n,
                                                          double *__restrict__ partial)
{
    __shared__ double sh[4];
    double s = 0.0;
    for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (size_t)gridDim.x * 256) s += x[t];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ __launch_bounds__(1024) void k_amr_sum_final(const double *__restrict__ partial, int n,
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

// delta = m / mbar - 1 in place on the base mesh
__global__ void k_amr_delta0(double *__restrict__ m, size_t n, double mbar)
{
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        m[t] = m[t] / mbar - 1.0;
}

// f = s (m / mbar - 1) on interior cells, per-block max |f| partials
__global__ __launch_bounds__(512) void k_amr_source(LevelDev L, double s, double mbar, double *__restrict__ partial)
{
    __shared__ double sh[8];
    const int blk = blockIdx.x, t = threadIdx.x;
    const int x = t >> 6, y = (t >> 3) & 7, z = t & 7;
    double *f = L.f[0] + (size_t)blk * sub_vol(0);
    const size_t q = pidx(0, x, y, z);
    const double v = s * (f[q] / mbar - 1.0);
    f[q] = v;
    double mx = fabs(v);
    for (int o = 32; o > 0; o >>= 1) {
        const double other = __shfl_xor(mx, o, 64);
        mx = (other != other || other > mx) ? other : mx;
    }
    if ((t & 63) == 0) sh[t >> 6] = mx;
    __syncthreads();
    if (t == 0) {
        for (int w = 1; w < 8; ++w) mx = (sh[w] != sh[w] || sh[w] > mx) ? sh[w] : mx;
        partial[blk] = mx;
    }
}

// frozen values on ghost faces without a neighbour (u[m]), zero corrections there (E[m]);
// for m == 0 also the initial guess on interior cells
__global__ void k_amr_frozen(LevelDev L, Composite C, int l, int m)
{
    const int b = sub_b(m), p = sub_p(m);
    const int vol = p * p * p;
    const size_t n = (size_t)L.nb * vol;
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
        const int blk = (int)(id / vol), q = (int)(id % vol);
        const int x = q / (p * p) - 1, y = (q / p) % p - 1, z = q % p - 1;
        const int outside = (x < 0 || x >= b) + (y < 0 || y >= b) + (z < 0 || z >= b);
        const int gx = (L.org[3 * blk + 0] >> m) + x, gy = (L.org[3 * blk + 1] >> m) + y,
                  gz = (L.org[3 * blk + 2] >> m) + z;
        if (outside == 0) {
            if (m == 0) L.u[0][id] = prolong_parent(C, l, gx, gy, gz);
            continue;
        }
        if (outside != 1) continue;  // edges and corners are never read by the 7-point stencil
        const int face = x < 0 ? 0 : x >= b ? 1 : y < 0 ? 2 : y >= b ? 3 : z < 0 ? 4 : 5;
        if (L.nbr[6 * blk + face] >= 0) continue;
        L.u[m][id] = (m == 0) ? prolong_parent(C, l, gx, gy, gz) : comp_at(C, l - m, gx, gy, gz);
        L.E[m][id] = 0.0;
    }
}

// copy neighbours' boundary layers into the ghost faces of X (sublevel m)
__global__ void k_amr_exchange(LevelDev L, double *__restrict__ X, int m)
{
    const int b = sub_b(m);
    const size_t per = (size_t)6 * b * b;
    const size_t n = (size_t)L.nb * per;
    const size_t vol = sub_vol(m);
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
        const int blk = (int)(id / per);
        const int r = (int)(id % per);
        const int face = r / (b * b), s = (r / b) % b, t = r % b;
        const int nb = L.nbr[6 * blk + face];
        if (nb < 0) continue;
        int dst[3], src[3];
        const int ax = face >> 1, hi = face & 1;
        const int o1 = ax == 0 ? 1 : 0, o2 = ax == 2 ? 1 : 2;  // the two in-face axes
        dst[ax] = hi ? b : -1;
        src[ax] = hi ? 0 : b - 1;
        dst[o1] = src[o1] = s;
        dst[o2] = src[o2] = t;
        X[(size_t)blk * vol + pidx(m, dst[0], dst[1], dst[2])] = X[(size_t)nb * vol + pidx(m, src[0], src[1], src[2])];
    }
}

__device__ __forceinline__ void amr_op_vals(double uc, const double nb[6], double ih2, double bC, double q,
                                            double &L, double &J, const double *tab)
{
    const double ec = exp64(uc, tab);
    double S1 = 0.0, S2 = 0.0, S3 = 0.0;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const double d = nb[s] - uc, en = exp64(nb[s], tab);
        S1 += d;
        S2 += en;
        S3 += en * d;
    }
    const double em = expm1_64(-q * uc, tab);
    L = ih2 * 0.5 * (S3 + ec * S1) + bC * em;
    J = ih2 * 0.5 * (ec * (S1 - 6.0) - S2) - bC * q * (1.0 + em);
}

// L and J at an interior cell of sublevel m, neighbours from the padded block
__device__ __forceinline__ void amr_op(const double *__restrict__ U, int m, int x, int y, int z, double ih2,
                                       double bC, double q, double &L, double &J, const double *tab)
{
    const double nb[6] = {U[pidx(m, x + 1, y, z)], U[pidx(m, x - 1, y, z)], U[pidx(m, x, y + 1, z)],
                          U[pidx(m, x, y - 1, z)], U[pidx(m, x, y, z + 1)], U[pidx(m, x, y, z - 1)]};
    amr_op_vals(U[pidx(m, x, y, z)], nb, ih2, bC, q, L, J, tab);
}

// u of sublevel m at (x, y, z) of block blk, where one coordinate may lie one
// cell outside the block: the neighbouring block's cell if that block exists
// (read directly, so sweeps need no ghost exchange between colours), else the
// block's own frozen ghost value.
template <typename T>
__device__ __forceinline__ T amr_nbval(const LevelDev &L, const T *__restrict__ U, int blk, int m, int b, int vol,
                                       int x, int y, int z)
{
    int f = -1, xx = x, yy = y, zz = z;
    if (x < 0) { f = 0; xx = b - 1; }
    else if (x >= b) { f = 1; xx = 0; }
    else if (y < 0) { f = 2; yy = b - 1; }
    else if (y >= b) { f = 3; yy = 0; }
    else if (z < 0) { f = 4; zz = b - 1; }
    else if (z >= b) { f = 5; zz = 0; }
    if (f >= 0) {
        const int nb = L.nbr[6 * blk + f];
        if (nb >= 0) return U[(size_t)nb * vol + pidx(m, xx, yy, zz)];
    }
    return U[(size_t)blk * vol + pidx(m, x, y, z)];
}

__global__ void k_amr_sweep(LevelDev L, int m, int colour, double ih2, double bC, double q, double max_du)
{
    __shared__ double tab[64];
    if (threadIdx.x < 64) tab[threadIdx.x] = L.exp2tab[threadIdx.x];
    __syncthreads();
    const int b = sub_b(m), vol = sub_vol(m);
    // threads cover the cells of this colour only (b even); 1^3 blocks: one thread per block
    const int per = b > 1 ? b * b * b / 2 : 1;
    const size_t n = (size_t)L.nb * per;
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
        const int blk = (int)(id / per), c = (int)(id % per);
        const int ox = L.org[3 * blk] >> m, oy = L.org[3 * blk + 1] >> m, oz = L.org[3 * blk + 2] >> m;
        int x = 0, y = 0, z = 0;
        if (b > 1) {
            const int hb = b >> 1;
            x = c / (b * hb);
            y = (c / hb) % b;
            z = 2 * (c % hb) + ((colour + ox + oy + oz + x + y) & 1);
        } else if (((ox + oy + oz) & 1) != colour) {
            continue;
        }
        double *U = L.u[m] + (size_t)blk * vol;
        const double uc = U[pidx(m, x, y, z)];
        const double nbv[6] = {amr_nbval(L, L.u[m], blk, m, b, vol, x + 1, y, z),
                               amr_nbval(L, L.u[m], blk, m, b, vol, x - 1, y, z),
                               amr_nbval(L, L.u[m], blk, m, b, vol, x, y + 1, z),
                               amr_nbval(L, L.u[m], blk, m, b, vol, x, y - 1, z),
                               amr_nbval(L, L.u[m], blk, m, b, vol, x, y, z + 1),
                               amr_nbval(L, L.u[m], blk, m, b, vol, x, y, z - 1)};
        double Lv, J;
        amr_op_vals(uc, nbv, ih2, bC, q, Lv, J, tab);
        double du = -(Lv - L.f[m][(size_t)blk * vol + pidx(m, x, y, z)]) / J;
        if (max_du > 0.0) du = fmin(fmax(du, -max_du), max_du);
        U[pidx(m, x, y, z)] = uc + du;
    }
}

// coarse interior cell: ubar = mean of children's u, f_c = mean of children's residuals,
// u_c = ubar
__global__ void k_amr_restrict(LevelDev L, int m, double ih2, double bC, double q)
{
    __shared__ double tab[64];
    if (threadIdx.x < 64) tab[threadIdx.x] = L.exp2tab[threadIdx.x];
    __syncthreads();
    const int bc = sub_b(m + 1), volf = sub_vol(m), volc = sub_vol(m + 1);
    const int cells = bc * bc * bc;
    const size_t n = (size_t)L.nb * cells;
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
        const int blk = (int)(id / cells), c = (int)(id % cells);
        const int X = c / (bc * bc), Y = (c / bc) % bc, Z = c % bc;
        const double *U = L.u[m] + (size_t)blk * volf;
        const double *F = L.f[m] + (size_t)blk * volf;
        double su = 0.0, sr = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b2 = 0; b2 < 2; ++b2)
                for (int d = 0; d < 2; ++d) {
                    const int x = 2 * X + a, y = 2 * Y + b2, z = 2 * Z + d;
                    double Lv, J;
                    amr_op(U, m, x, y, z, ih2, bC, q, Lv, J, tab);
                    su += U[pidx(m, x, y, z)];
                    sr += F[pidx(m, x, y, z)] - Lv;
                }
        const size_t qc = (size_t)blk * volc + pidx(m + 1, X, Y, Z);
        L.ub[m + 1][qc] = su / 8.0;
        L.f[m + 1][qc] = sr / 8.0;
        L.u[m + 1][qc] = su / 8.0;
    }
}

// f += L(u) on interior cells of sublevel m (the FAS coarse source)
__global__ void k_amr_coarse_rhs(LevelDev L, int m, double ih2, double bC, double q)
{
    __shared__ double tab[64];
    if (threadIdx.x < 64) tab[threadIdx.x] = L.exp2tab[threadIdx.x];
    __syncthreads();
    const int b = sub_b(m), vol = sub_vol(m);
    const int cells = b * b * b;
    const size_t n = (size_t)L.nb * cells;
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
        const int blk = (int)(id / cells), c = (int)(id % cells);
        const int x = c / (b * b), y = (c / b) % b, z = c % b;
        double Lv, J;
        amr_op(L.u[m] + (size_t)blk * vol, m, x, y, z, ih2, bC, q, Lv, J, tab);
        L.f[m][(size_t)blk * vol + pidx(m, x, y, z)] += Lv;
    }
}

__global__ void k_amr_make_e(LevelDev L, int m)
{
    const int b = sub_b(m), vol = sub_vol(m);
    const int cells = b * b * b;
    const size_t n = (size_t)L.nb * cells;
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
        const int blk = (int)(id / cells), c = (int)(id % cells);
        const size_t q = (size_t)blk * vol + pidx(m, c / (b * b), (c / b) % b, c % b);
        L.E[m][q] = L.u[m][q] - L.ub[m][q];
    }
}

// u[m] += P(E[m+1]) with the linear (mode 0) or injected (mode 1) reconstruction
__global__ void k_amr_prolong(LevelDev L, int m, int mode)
{
    const int b = sub_b(m), vol = sub_vol(m), volc = sub_vol(m + 1);
    const int cells = b * b * b;
    const size_t n = (size_t)L.nb * cells;
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
        const int blk = (int)(id / cells), c = (int)(id % cells);
        const int x = c / (b * b), y = (c / b) % b, z = c % b;
        const double *E = L.E[m + 1] + (size_t)blk * volc;
        const int X = x >> 1, Y = y >> 1, Z = z >> 1;
        double v = E[pidx(m + 1, X, Y, Z)];
        if (mode == 0) {
            v += ((x & 1) ? 0.125 : -0.125) * (E[pidx(m + 1, X + 1, Y, Z)] - E[pidx(m + 1, X - 1, Y, Z)]);
            v += ((y & 1) ? 0.125 : -0.125) * (E[pidx(m + 1, X, Y + 1, Z)] - E[pidx(m + 1, X, Y - 1, Z)]);
            v += ((z & 1) ? 0.125 : -0.125) * (E[pidx(m + 1, X, Y, Z + 1)] - E[pidx(m + 1, X, Y, Z - 1)]);
        }
        L.u[m][(size_t)blk * vol + pidx(m, x, y, z)] += v;
    }
}

__global__ __launch_bounds__(512) void k_amr_resnorm(LevelDev L, double ih2, double bC, double q,
                                                      double *__restrict__ partial)
{
    __shared__ double tab[64];
    if (threadIdx.x < 64) tab[threadIdx.x] = L.exp2tab[threadIdx.x];
    __syncthreads();
    __shared__ double sh[8];
    const int blk = blockIdx.x, t = threadIdx.x;
    const int x = t >> 6, y = (t >> 3) & 7, z = t & 7;
    double Lv, J;
    amr_op(L.u[0] + (size_t)blk * sub_vol(0), 0, x, y, z, ih2, bC, q, Lv, J, tab);
    double mx = fabs(L.f[0][(size_t)blk * sub_vol(0) + pidx(0, x, y, z)] - Lv);
    for (int o = 32; o > 0; o >>= 1) {
        const double other = __shfl_xor(mx, o, 64);
        mx = (other != other || other > mx) ? other : mx;
    }
    if ((t & 63) == 0) sh[t >> 6] = mx;
    __syncthreads();
    if (t == 0) {
        for (int w = 1; w < 8; ++w) mx = (sh[w] != sh[w] || sh[w] > mx) ? sh[w] : mx;
        partial[blk] = mx;
    }
}

__global__ void k_max_final(const double *__restrict__ partial, int n, double *__restrict__ out)
{
    __shared__ double sh[16];
    double mx = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) mx = (partial[i] != partial[i] || partial[i] > mx) ? partial[i] : mx;
    for (int o = 32; o > 0; o >>= 1) {
        const double other = __shfl_xor(mx, o, 64);
        mx = (other != other || other > mx) ? other : mx;
    }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x / 64); ++w) mx = (sh[w] != sh[w] || sh[w] > mx) ? sh[w] : mx;
        out[0] = mx;
    }
}

// ------------------------------------------ mixed precision on the refined levels
//
// The float32 correction cycle of the uniform mixed solve on the block arrays:
// e solves N_u(e) = r (N_u(e) = L(u + e) - L(u) without cancellation) with u the
// level's float64 iterate held in float32; e is zero on frozen ghosts (their
// values never change) and neighbouring blocks are read directly.

// u32 = float(u) and e32 = eb32 = 0 on every padded cell of sublevel m
__global__ void k_amrx_init(LevelDev L, int m)
{
    const size_t n = (size_t)L.nb * sub_vol(m);
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
        L.u32[m][id] = (float)L.u[m][id];
        L.e32[m][id] = 0.f;
        L.eb32[m][id] = 0.f;
    }
}

// float64 residual r = f - L(u) on sublevel 0 (ghosts exchanged): r32 = r,
// u32 = u, e32 = 0 on interior cells, per-block max|r|
__global__ __launch_bounds__(512) void k_amrx_outer(LevelDev L, double ih2, double bC, double q,
                                                     double *__restrict__ partial)
{
    __shared__ double tab[64];
    if (threadIdx.x < 64) tab[threadIdx.x] = L.exp2tab[threadIdx.x];
    __syncthreads();
    __shared__ double sh[8];
    const int blk = blockIdx.x, t = threadIdx.x;
    const int x = t >> 6, y = (t >> 3) & 7, z = t & 7;
    const size_t o = (size_t)blk * sub_vol(0) + pidx(0, x, y, z);
    double Lv, J;
    amr_op(L.u[0] + (size_t)blk * sub_vol(0), 0, x, y, z, ih2, bC, q, Lv, J, tab);
    const double r = L.f[0][o] - Lv;
    L.r32[0][o] = (float)r;
    L.u32[0][o] = (float)L.u[0][o];
    L.e32[0][o] = 0.f;
    double mx = fabs(r);
    for (int s = 32; s > 0; s >>= 1) {
        const double other = __shfl_xor(mx, s, 64);
        mx = (other != other || other > mx) ? other : mx;
    }
    if ((t & 63) == 0) sh[t >> 6] = mx;
    __syncthreads();
    if (t == 0) {
        for (int w = 1; w < 8; ++w) mx = (sh[w] != sh[w] || sh[w] > mx) ? sh[w] : mx;
        partial[blk] = mx;
    }
}

// the cell (x,y,z) of sublevel m and its six neighbours: e, X = expm1(e), u, w = e^u
struct AmrxCell {
    float ec, Xc, uc, wc, en[6], Xn[6], un[6], wn[6];
};

__device__ __forceinline__ void amrx_gather(const LevelDev &L, const float *__restrict__ E, int blk, int m, int b,
                                            int vol, int x, int y, int z, AmrxCell &c)
{
    const size_t o = (size_t)blk * vol + pidx(m, x, y, z);
    c.ec = E[o];
    c.uc = L.u32[m][o];
    c.Xc = fexpm1(c.ec);
    c.wc = fexp(c.uc);
    const int dx[6] = {1, -1, 0, 0, 0, 0}, dy[6] = {0, 0, 1, -1, 0, 0}, dz[6] = {0, 0, 0, 0, 1, -1};
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        c.en[s] = amr_nbval(L, E, blk, m, b, vol, x + dx[s], y + dy[s], z + dz[s]);
        c.un[s] = amr_nbval(L, (const float *)L.u32[m], blk, m, b, vol, x + dx[s], y + dy[s], z + dz[s]);
        c.Xn[s] = fexpm1(c.en[s]);
        c.wn[s] = fexp(c.un[s]);
    }
}

// one colour of a float32 correction sweep on sublevel m (threads on that colour only)
__global__ void k_amrx_sweep(LevelDev L, int m, int colour, MxConst kc)
{
    const int b = sub_b(m), vol = sub_vol(m);
    const int per = b > 1 ? b * b * b / 2 : 1;
    const size_t n = (size_t)L.nb * per;
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
        const int blk = (int)(id / per), c = (int)(id % per);
        const int ox = L.org[3 * blk] >> m, oy = L.org[3 * blk + 1] >> m, oz = L.org[3 * blk + 2] >> m;
        int x = 0, y = 0, z = 0;
        if (b > 1) {
            const int hb = b >> 1;
            x = c / (b * hb);
            y = (c / hb) % b;
            z = 2 * (c % hb) + ((colour + ox + oy + oz + x + y) & 1);
        } else if (((ox + oy + oz) & 1) != colour) {
            continue;
        }
        AmrxCell cell;
        amrx_gather(L, L.e32[m], blk, m, b, vol, x, y, z, cell);
        const size_t o = (size_t)blk * vol + pidx(m, x, y, z);
        L.e32[m][o] = cell.ec + mx_step(cell.ec, cell.Xc, cell.uc, cell.wc, cell.en, cell.Xn, cell.un, cell.wn,
                                        L.r32[m][o], kc);
    }
}

// coarse interior cell of sublevel m + 1: eb = mean of the daughters' e, u32 =
// mean of their u32, r = mean of their r - N(e)
__global__ void k_amrx_restrict(LevelDev L, int m, MxConst kc)
{
    const int b = sub_b(m), vol = sub_vol(m), bc = sub_b(m + 1), volc = sub_vol(m + 1);
    const int cells = bc * bc * bc;
    const size_t n = (size_t)L.nb * cells;
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
        const int blk = (int)(id / cells), c = (int)(id % cells);
        const int X = c / (bc * bc), Y = (c / bc) % bc, Z = c % bc;
        float se = 0.f, su = 0.f, sr = 0.f;
        for (int a = 0; a < 2; ++a)
            for (int b2 = 0; b2 < 2; ++b2)
                for (int d = 0; d < 2; ++d) {
                    const int x = 2 * X + a, y = 2 * Y + b2, z = 2 * Z + d;
                    AmrxCell cell;
                    amrx_gather(L, L.e32[m], blk, m, b, vol, x, y, z, cell);
                    const float N = mx_value(cell.ec, cell.Xc, cell.uc, cell.wc, cell.en, cell.Xn, cell.un, cell.wn, kc);
                    se += cell.ec;
                    su += cell.uc;
                    sr += L.r32[m][(size_t)blk * vol + pidx(m, x, y, z)] - N;
                }
        const size_t q = (size_t)blk * volc + pidx(m + 1, X, Y, Z);
        L.eb32[m + 1][q] = 0.125f * se;
        L.u32[m + 1][q] = 0.125f * su;
        L.r32[m + 1][q] = 0.125f * sr;
    }
}

// r += N_c(eb), e = eb on the interior cells of sublevel m (the FAS source)
__global__ void k_amrx_coarse_rhs(LevelDev L, int m, MxConst kc)
{
    const int b = sub_b(m), vol = sub_vol(m);
    const int cells = b * b * b;
    const size_t n = (size_t)L.nb * cells;
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
        const int blk = (int)(id / cells), c = (int)(id % cells);
        const int x = c / (b * b), y = (c / b) % b, z = c % b;
        AmrxCell cell;
        amrx_gather(L, L.eb32[m], blk, m, b, vol, x, y, z, cell);
        const size_t o = (size_t)blk * vol + pidx(m, x, y, z);
        L.r32[m][o] += mx_value(cell.ec, cell.Xc, cell.uc, cell.wc, cell.en, cell.Xn, cell.un, cell.wn, kc);
        L.e32[m][o] = cell.ec;
    }
}

// e[m] += P(e[m+1] - eb[m+1]) on interior cells (linear: mode 0, injection: mode 1)
__global__ void k_amrx_prolong(LevelDev L, int m, int mode)
{
    const int b = sub_b(m), vol = sub_vol(m), bc = sub_b(m + 1), volc = sub_vol(m + 1);
    const int cells = b * b * b;
    const size_t n = (size_t)L.nb * cells;
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
        const int blk = (int)(id / cells), c = (int)(id % cells);
        const int x = c / (b * b), y = (c / b) % b, z = c % b;
        const int X = x >> 1, Y = y >> 1, Z = z >> 1;
        auto d = [&](int i, int j, int k) {
            return amr_nbval(L, (const float *)L.e32[m + 1], blk, m + 1, bc, volc, i, j, k) -
                   amr_nbval(L, (const float *)L.eb32[m + 1], blk, m + 1, bc, volc, i, j, k);
        };
        float v = d(X, Y, Z);
        if (mode == 0) {
            v += ((x & 1) ? 0.125f : -0.125f) * (d(X + 1, Y, Z) - d(X - 1, Y, Z));
            v += ((y & 1) ? 0.125f : -0.125f) * (d(X, Y + 1, Z) - d(X, Y - 1, Z));
            v += ((z & 1) ? 0.125f : -0.125f) * (d(X, Y, Z + 1) - d(X, Y, Z - 1));
        }
        L.e32[m][(size_t)blk * vol + pidx(m, x, y, z)] += v;
    }
}

// u += e on the interior cells of sublevel 0
__global__ void k_amrx_update(LevelDev L)
{
    const size_t n = (size_t)L.nb * 512;
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
        const int blk = (int)(id / 512), c = (int)(id % 512);
        const size_t o = (size_t)blk * sub_vol(0) + pidx(0, c >> 6, (c >> 3) & 7, c & 7);
        L.u[0][o] += (double)L.e32[0][o];
    }
}

__global__ void k_amr_copy_out(LevelDev L, double *__restrict__ out)
{
    const size_t n = (size_t)L.nb * 512;
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
        const int blk = (int)(id / 512), c = (int)(id % 512);
        out[id] = L.u[0][(size_t)blk * sub_vol(0) + pidx(0, c >> 6, (c >> 3) & 7, c & 7)];
    }
}

// Composite fields on the uniform mesh of the finest level (side 2^lgf): every
// cell takes delta and the effective density of the finest level covering it
// (a coarse leaf's value fills all its sub-cells: its mass spread over its
// volume).  delta_l = f_l / s on the refined levels (f_l = s delta_l is the
// level's source), delta_0 on the base;
// delta_eff = delta / 3 - C expm1(-q u) / (3 Omega_m a^-3)  (Sec. 3.4).
struct CompArgs {
    int nref, lgf;
    const double *d0, *u0;
    int lg0;
    const int *map[kMaxRef + 1];
    const double *u[kMaxRef + 1], *f[kMaxRef + 1];
    double inv_s, third_C_om, q;
    double *dout, *eout;
};

__global__ void k_amr_composite(CompArgs A)
{
    const size_t n = (size_t)1 << (3 * A.lgf);
    const int mf = (1 << A.lgf) - 1;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(t & mf), j = (int)((t >> A.lgf) & mf), i = (int)(t >> (2 * A.lgf));
        double d = 0.0, u = 0.0;
        bool found = false;
        for (int l = A.nref; l >= 1 && !found; --l) {
            const int sh = A.nref - l, lg = A.lg0 + l, M = 1 << (lg - 3);
            const int a = i >> sh, b = j >> sh, c = k >> sh;
            const int blk = A.map[l][((size_t)(a >> 3) * M + (b >> 3)) * M + (c >> 3)];
            if (blk >= 0) {
                const size_t o = (size_t)blk * sub_vol(0) + pidx(0, a & 7, b & 7, c & 7);
                d = A.f[l][o] * A.inv_s;
                u = A.u[l][o];
                found = true;
            }
        }
        if (!found) {
            const int sh = A.nref;
            const size_t o = cidx(i >> sh, j >> sh, k >> sh, A.lg0);
            d = A.d0[o];
            u = A.u0[o];
        }
        A.dout[t] = d;
        A.eout[t] = d / 3.0 - A.third_C_om * expm1(-A.q * u);
    }
}

inline unsigned grid_of(size_t n, unsigned cap = 65535) { return (unsigned)std::max<size_t>(1, std::min<size_t>((n + 255) / 256, cap)); }

}  // namespace
}  // namespace mgfr

using namespace mgfr;

// ====================================================================== host

struct mgfr_amr {
    mgfr_params p{};
    hipStream_t stream = nullptr;
    int nref = 0, N0 = 0, lg0 = 0;
    int64_t max_blocks = 0;
    mgfr_ctx *base = nullptr;
    double *delta0 = nullptr, *u0 = nullptr;
    int *cnt0 = nullptr;      // [N0^3] counts
    int *cntb = nullptr;      // [max_blocks * 512] counts
    unsigned char *flag[kMaxRef + 1] = {nullptr};  // refinement flags per level-l block position
    double *partial = nullptr, *dscal = nullptr, *hscal = nullptr;
    int *dflag = nullptr;       // non-finite particle position seen by the assignment
    double total_mass = 0.0;    // of the last assignment (sum over the base mesh)
    // per refined level
    int nb[kMaxRef + 1] = {0, 0, 0};
    int *map[kMaxRef + 1] = {nullptr}, *org[kMaxRef + 1] = {nullptr}, *nbr[kMaxRef + 1] = {nullptr};
    double *arr[kMaxRef + 1][4][kSub] = {};  // u, f, ub, E per sublevel
    float *arr32[kMaxRef + 1][4][kSub] = {};  // e, u, r, eb per sublevel (mixed precision only)
    std::vector<int> horg[kMaxRef + 1];
    mgfr_stats st[kMaxRef + 1];
    double beta = 0, C = 0, fbar = 0;
    double omega32 = 1.0;  // relaxation factor of the refined levels' float32 correction sweeps
    // binned composite assignment (mgfr_amr_reserve_particles): sort keys, indices, workspace
    uint32_t *bkey = nullptr, *bkey_s = nullptr, *bidx = nullptr, *perm = nullptr;
    void *sort_tmp = nullptr;
    size_t sort_tmp_bytes = 0;
    int64_t bin_cap = 0;
};

namespace {

LevelDev level_dev(const mgfr_amr *A, int l)
{
    LevelDev L{};
    L.lg = A->lg0 + l;
    L.nb = A->nb[l];
    L.mlg = L.lg - 3;
    L.map = A->map[l];
    L.org = A->org[l];
    L.nbr = A->nbr[l];
    L.exp2tab = A->base->exp2tab;
    for (int m = 0; m < kSub; ++m) {
        L.u[m] = A->arr[l][0][m];
        L.f[m] = A->arr[l][1][m];
        L.ub[m] = A->arr[l][2][m];
        L.E[m] = A->arr[l][3][m];
        L.e32[m] = A->arr32[l][0][m];
        L.u32[m] = A->arr32[l][1][m];
        L.r32[m] = A->arr32[l][2][m];
        L.eb32[m] = A->arr32[l][3][m];
    }
    return L;
}

Composite composite(const mgfr_amr *A, int nsolved)
{
    Composite C{};
    C.u0 = A->u0;
    C.lg0 = A->lg0;
    for (int l = 1; l <= A->nref; ++l) C.lev[l] = level_dev(A, l);
    C.nsolved = nsolved;
    return C;
}

void amr_bin_free(mgfr_amr *A)
{
    (void)hipFree(A->bkey);
    (void)hipFree(A->bkey_s);
    (void)hipFree(A->bidx);
    (void)hipFree(A->perm);
    (void)hipFree(A->sort_tmp);
    A->bkey = A->bkey_s = A->bidx = A->perm = nullptr;
    A->sort_tmp = nullptr;
    A->sort_tmp_bytes = 0;
    A->bin_cap = 0;
}

// key offsets of the binned assignment: level l's groups of 8^3 cells follow
// those of the coarser levels; the last entry is the general path's key
CicKeys cic_keys(const mgfr_amr *A)
{
    CicKeys K{};
    uint32_t off = 0;
    for (int l = 0; l <= A->nref; ++l) {
        K.koff[l] = off;
        const uint32_t g = (uint32_t)1 << (A->lg0 + l - kBinLg);
        off += g * g * g;
    }
    K.koff[A->nref + 1] = off;
    return K;
}

unsigned cic_key_bits(const mgfr_amr *A)
{
    const uint32_t top = cic_keys(A).koff[A->nref + 1];
    unsigned b = 1;
    while (b < 32 && (top >> b) != 0) ++b;
    return b;
}

void amr_free(mgfr_amr *A)
{
    if (!A) return;
    if (A->base) mgfr_destroy(A->base);
    (void)hipFree(A->delta0);
    (void)hipFree(A->u0);
    (void)hipFree(A->cnt0);
    (void)hipFree(A->cntb);
    for (int l = 1; l <= kMaxRef; ++l) (void)hipFree(A->flag[l]);
    (void)hipFree(A->partial);
    (void)hipFree(A->dscal);
    (void)hipFree(A->dflag);
    amr_bin_free(A);
    if (A->hscal) (void)hipHostFree(A->hscal);
    for (int l = 1; l <= kMaxRef; ++l) {
        (void)hipFree(A->map[l]);
        (void)hipFree(A->org[l]);
        (void)hipFree(A->nbr[l]);
        for (int a = 0; a < 4; ++a)
            for (int m = 0; m < kSub; ++m) {
                (void)hipFree(A->arr[l][a][m]);
                (void)hipFree(A->arr32[l][a][m]);
            }
    }
    delete A;
}

// Upload block list `blocks` (sorted linear block indices) of level l: origins,
// block map and face neighbours.
int upload_level(mgfr_amr *A, int l, const std::vector<int64_t> &blocks)
{
    const int N = A->N0 << l, M = N / 8;
    if ((int64_t)blocks.size() > A->max_blocks)
        return set_error(MGFR_ERR_ARG, "level %d needs %zu blocks, more than max_blocks = %lld", l, blocks.size(),
                         (long long)A->max_blocks);
    std::vector<int> map((size_t)M * M * M, -1), org(3 * blocks.size()), nbr(6 * blocks.size());
    for (size_t b = 0; b < blocks.size(); ++b) map[blocks[b]] = (int)b;
    for (size_t b = 0; b < blocks.size(); ++b) {
        const int64_t li = blocks[b];
        const int bx = (int)(li / ((int64_t)M * M)), by = (int)((li / M) % M), bz = (int)(li % M);
        org[3 * b] = 8 * bx;
        org[3 * b + 1] = 8 * by;
        org[3 * b + 2] = 8 * bz;
        const int d[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
        for (int f = 0; f < 6; ++f) {
            const int x = (bx + d[f][0] + M) % M, y = (by + d[f][1] + M) % M, z = (bz + d[f][2] + M) % M;
            nbr[6 * b + f] = map[((size_t)x * M + y) * M + z];
        }
    }
    A->nb[l] = (int)blocks.size();
    A->horg[l] = org;
    MGFR_HIP(hipMemcpyAsync(A->map[l], map.data(), map.size() * sizeof(int), hipMemcpyHostToDevice, A->stream));
    if (!blocks.empty()) {
        MGFR_HIP(hipMemcpyAsync(A->org[l], org.data(), org.size() * sizeof(int), hipMemcpyHostToDevice, A->stream));
        MGFR_HIP(hipMemcpyAsync(A->nbr[l], nbr.data(), nbr.size() * sizeof(int), hipMemcpyHostToDevice, A->stream));
    }
    MGFR_HIP(hipStreamSynchronize(A->stream));  // host vectors go out of scope
    return MGFR_OK;
}

int read_max(mgfr_amr *A, int n, double *out)
{
    k_max_final<<<1, 1024, 0, A->stream>>>(A->partial, n, A->dscal);
    MGFR_HIP(hipGetLastError());
    MGFR_HIP(hipMemcpyAsync(A->hscal, A->dscal, sizeof(double), hipMemcpyDeviceToHost, A->stream));
    MGFR_HIP(hipStreamSynchronize(A->stream));
    *out = A->hscal[0];
    return MGFR_OK;
}

struct SubConst {
    double ih2[kSub];
};

int amr_sweeps(mgfr_amr *A, const LevelDev &L, int m, int sweeps, const SubConst &K)
{
    const int b = sub_b(m);
    const size_t cells = (size_t)L.nb * b * b * b, faces = (size_t)L.nb * 6 * b * b;
    for (int s = 0; s < sweeps; ++s)
        for (int colour = 0; colour < 2; ++colour)
            k_amr_sweep<<<grid_of(b > 1 ? cells / 2 : cells), 256, 0, A->stream>>>(L, m, colour, K.ih2[m], A->beta * A->C,
                                                                1.0 / (A->p.n + 1), A->p.max_du);
    // ghost faces between blocks for the kernels that read them (restriction, residual)
    if (sweeps > 0) k_amr_exchange<<<grid_of(faces), 256, 0, A->stream>>>(L, L.u[m], m);
    MGFR_HIP(hipGetLastError());
    return MGFR_OK;
}

int amr_vcycle(mgfr_amr *A, const LevelDev &L, int m, const SubConst &K)
{
    const double bC = A->beta * A->C, q = 1.0 / (A->p.n + 1);
    if (m == kSub - 1) return amr_sweeps(A, L, m, A->p.coarse_sweeps, K);
    int rc;
    if ((rc = amr_sweeps(A, L, m, A->p.pre_smooth, K))) return rc;
    const int bc = sub_b(m + 1);
    const size_t cc = (size_t)L.nb * bc * bc * bc, fc = (size_t)L.nb * 6 * bc * bc;
    const int b = sub_b(m);
    const size_t cf = (size_t)L.nb * b * b * b, ff = (size_t)L.nb * 6 * b * b;
    k_amr_restrict<<<grid_of(cc), 256, 0, A->stream>>>(L, m, K.ih2[m], bC, q);
    k_amr_exchange<<<grid_of(fc), 256, 0, A->stream>>>(L, L.u[m + 1], m + 1);
    k_amr_coarse_rhs<<<grid_of(cc), 256, 0, A->stream>>>(L, m + 1, K.ih2[m + 1], bC, q);
    MGFR_HIP(hipGetLastError());
    if ((rc = amr_vcycle(A, L, m + 1, K))) return rc;
    k_amr_make_e<<<grid_of(cc), 256, 0, A->stream>>>(L, m + 1);
    k_amr_exchange<<<grid_of(fc), 256, 0, A->stream>>>(L, L.E[m + 1], m + 1);
    k_amr_prolong<<<grid_of(cf), 256, 0, A->stream>>>(L, m, A->p.prolong);
    if (A->p.post_smooth == 0) k_amr_exchange<<<grid_of(ff), 256, 0, A->stream>>>(L, L.u[m], m);
    MGFR_HIP(hipGetLastError());
    return amr_sweeps(A, L, m, A->p.post_smooth, K);
}

// float32 correction V-cycle on sublevels m.. of a refined level (mixed precision)
int amrx_vcycle(mgfr_amr *A, const LevelDev &L, int m, const MxConst *K)
{
    auto sweeps = [&](int mm, int count) {
        const int b = sub_b(mm);
        const size_t cells = (size_t)L.nb * b * b * b;
        for (int s = 0; s < count; ++s)
            for (int colour = 0; colour < 2; ++colour)
                k_amrx_sweep<<<grid_of(b > 1 ? cells / 2 : cells), 256, 0, A->stream>>>(L, mm, colour, K[mm]);
    };
    if (m == kSub - 1) {
        sweeps(m, A->p.coarse_sweeps);
        MGFR_HIP(hipGetLastError());
        return MGFR_OK;
    }
    sweeps(m, A->p.pre_smooth);
    const int bc = sub_b(m + 1), b = sub_b(m);
    const size_t cc = (size_t)L.nb * bc * bc * bc, cf = (size_t)L.nb * b * b * b;
    k_amrx_restrict<<<grid_of(cc), 256, 0, A->stream>>>(L, m, K[m]);
    k_amrx_coarse_rhs<<<grid_of(cc), 256, 0, A->stream>>>(L, m + 1, K[m + 1]);
    MGFR_HIP(hipGetLastError());
    int rc;
    if ((rc = amrx_vcycle(A, L, m + 1, K))) return rc;
    k_amrx_prolong<<<grid_of(cf), 256, 0, A->stream>>>(L, m, A->p.prolong);
    sweeps(m, A->p.post_smooth);
    MGFR_HIP(hipGetLastError());
    return MGFR_OK;
}

int solve_level(mgfr_amr *A, int l)
{
    mgfr_stats &st = A->st[l];
    memset(&st, 0, sizeof st);
    LevelDev L = level_dev(A, l);
    if (L.nb == 0) {
        st.status = MGFR_OK;
        return MGFR_OK;
    }
    const int N = 1 << L.lg;
    const double h = A->p.box / N;
    SubConst K;
    for (int m = 0; m < kSub; ++m) {
        const double hm = h * (1 << m);
        K.ih2[m] = 1.0 / (hm * hm);
    }
    // clear every array (ghost faces included) of this level but the masses
    // the assignment left in f[0]
    for (int a = 0; a < 4; ++a)
        for (int m = 0; m < kSub; ++m)
            if (a != 1 || m != 0)
                MGFR_HIP(hipMemsetAsync(A->arr[l][a][m], 0, (size_t)L.nb * sub_vol(m) * sizeof(double), A->stream));
    // source from the composite masses: delta = m / mbar_l - 1, mbar_l = total / N_l^3
    const double mbar = A->total_mass / ((double)N * N * N);
    const double s = A->beta * A->p.omega_m / (A->p.a * A->p.a * A->p.a);
    k_amr_source<<<L.nb, 512, 0, A->stream>>>(L, s, mbar, A->partial);
    double D;
    int rc;
    if ((rc = read_max(A, L.nb, &D))) return rc;
    if (!std::isfinite(D)) return set_error(MGFR_ERR_NONFINITE, "level %d source is not finite", l);
    if (D == 0.0) D = A->beta * A->C;
    st.scale = D;
    // initial guess, frozen ghosts and zero-correction ghosts for every sublevel
    const Composite Cp = composite(A, l - 1);
    for (int m = 0; m < kSub; ++m)
        k_amr_frozen<<<grid_of((size_t)L.nb * sub_vol(m)), 256, 0, A->stream>>>(L, Cp, l, m);
    const size_t ff = (size_t)L.nb * 6 * 64;
    k_amr_exchange<<<grid_of(ff), 256, 0, A->stream>>>(L, L.u[0], 0);
    MGFR_HIP(hipGetLastError());
    const double bC = A->beta * A->C, q = 1.0 / (A->p.n + 1);
    int cyc = 0, status = MGFR_OK;
    double res = 0.0, rmax = 0.0;
    bool done = false;
    if (A->p.precision == MGFR_MIXED) {
        // float64 defect correction around float32 correction V-cycles; falls back
        // to the float64 cycles from the prolonged guess after 3 consecutive
        // residual increases or a non-finite residual
        MxConst KM[kSub];
        for (int m = 0; m < kSub; ++m)
            KM[m] = MxConst{(float)K.ih2[m], (float)bC, (float)q, (float)A->p.max_du, (float)A->omega32};
        for (int m = 0; m < kSub; ++m)
            k_amrx_init<<<grid_of((size_t)L.nb * sub_vol(m)), 256, 0, A->stream>>>(L, m);
        int grow = 0;
        double prev = 0.0;
        for (;;) {
            k_amrx_outer<<<L.nb, 512, 0, A->stream>>>(L, K.ih2[0], bC, q, A->partial);
            if ((rc = read_max(A, L.nb, &rmax))) return rc;
            res = rmax / D;
            if (cyc == 0) st.res0 = res;
            else {
                grow = (res > prev) ? grow + 1 : 0;
                if (grow)  // over-relaxation off for the rest of this level's solve
                    for (int m = 0; m < kSub; ++m) KM[m].omega = 1.0f;
                if (cyc - 1 < MGFR_MAX_HIST) st.res_hist[cyc - 1] = res;
            }
            prev = res;
            if (!std::isfinite(res) || grow >= 3) break;  // fall back below
            if (res <= A->p.tol) { status = MGFR_OK; done = true; break; }
            if (cyc >= A->p.max_vcycles) { status = MGFR_NOT_CONVERGED; done = true; break; }
            if ((rc = amrx_vcycle(A, L, 0, KM))) return rc;
            k_amrx_update<<<grid_of((size_t)L.nb * 512), 256, 0, A->stream>>>(L);
            k_amr_exchange<<<grid_of(ff), 256, 0, A->stream>>>(L, L.u[0], 0);
            MGFR_HIP(hipGetLastError());
            ++cyc;
        }
        if (!done) {
            st.fell_back = 1;
            k_amr_frozen<<<grid_of((size_t)L.nb * sub_vol(0)), 256, 0, A->stream>>>(L, Cp, l, 0);
            k_amr_exchange<<<grid_of(ff), 256, 0, A->stream>>>(L, L.u[0], 0);
            MGFR_HIP(hipGetLastError());
        }
    }
    if (!done) {
        const int outer = cyc;
        cyc = 0;
        k_amr_resnorm<<<L.nb, 512, 0, A->stream>>>(L, K.ih2[0], bC, q, A->partial);
        if ((rc = read_max(A, L.nb, &rmax))) return rc;
        res = rmax / D;
        if (!st.fell_back) st.res0 = res;
        for (;;) {
            if (!std::isfinite(res)) { status = MGFR_ERR_NONFINITE; break; }
            if (res <= A->p.tol) { status = MGFR_OK; break; }
            if (cyc >= A->p.max_vcycles) { status = MGFR_NOT_CONVERGED; break; }
            if ((rc = amr_vcycle(A, L, 0, K))) return rc;
            k_amr_resnorm<<<L.nb, 512, 0, A->stream>>>(L, K.ih2[0], bC, q, A->partial);
            if ((rc = read_max(A, L.nb, &rmax))) return rc;
            res = rmax / D;
            if (cyc < MGFR_MAX_HIST) st.res_hist[cyc] = res;
            ++cyc;
        }
        cyc += outer;
    }
    st.vcycles = st.outer_iters = cyc;
    st.res = res;
    st.status = status;
    return MGFR_OK;
}

}  // namespace

extern "C" int mgfr_amr_create(const mgfr_params *p, int64_t max_blocks, void *stream, mgfr_amr **out)
{
    if (!out) return set_error(MGFR_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!p) return set_error(MGFR_ERR_ARG, "params is NULL");
    if (p->refine_levels < 1 || p->refine_levels > kMaxRef)
        return set_error(MGFR_ERR_ARG, "refine_levels must be 1 or 2 for the adaptive solver");
    if (p->mesh < 32 || p->mesh > 512) return set_error(MGFR_ERR_ARG, "the base mesh must be 32..512");
    if (max_blocks < 1 || max_blocks > (1 << 22)) return set_error(MGFR_ERR_ARG, "max_blocks must be in [1, 2^22]");
    mgfr_params bp = *p;
    bp.refine_levels = 0;
    bp.nn_mode = MGFR_NN_NONE;
    mgfr_amr *A = new (std::nothrow) mgfr_amr();
    if (!A) return set_error(MGFR_ERR_OOM, "host allocation failed");
    A->p = *p;
    A->stream = (hipStream_t)stream;
    A->nref = p->refine_levels;
    A->N0 = p->mesh;
    while ((1 << A->lg0) < A->N0) ++A->lg0;
    A->max_blocks = max_blocks;
    int rc = mgfr_create(&bp, stream, &A->base);
    auto fail = [&](int code) {
        amr_free(A);
        return code;
    };
    if (rc) return fail(rc);
    mgfr_background(&bp, &A->fbar, &A->beta, &A->C);
    const size_t n0 = (size_t)A->N0 * A->N0 * A->N0;
    hipError_t e = hipSuccess;
    auto M = [&](void **ptr, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(ptr, bytes);
    };
    M((void **)&A->delta0, n0 * sizeof(double));
    M((void **)&A->u0, n0 * sizeof(double));
    M((void **)&A->cnt0, n0 * sizeof(int));
    M((void **)&A->cntb, (size_t)max_blocks * 512 * sizeof(int));
    M((void **)&A->partial, (size_t)std::max<int64_t>(max_blocks, 1024) * sizeof(double));
    M((void **)&A->dscal, 8 * sizeof(double));
    M((void **)&A->dflag, sizeof(int));
    for (int l = 1; l <= A->nref; ++l) {
        const size_t Mside = (size_t)(A->N0 << l) / 8;
        M((void **)&A->map[l], Mside * Mside * Mside * sizeof(int));
        M((void **)&A->flag[l], Mside * Mside * Mside);  // one byte per level-l block position
        M((void **)&A->org[l], (size_t)max_blocks * 3 * sizeof(int));
        M((void **)&A->nbr[l], (size_t)max_blocks * 6 * sizeof(int));
        for (int a = 0; a < 4; ++a)
            for (int m = 0; m < kSub; ++m) {
                M((void **)&A->arr[l][a][m], (size_t)max_blocks * sub_vol(m) * sizeof(double));
                if (p->precision == MGFR_MIXED)
                    M((void **)&A->arr32[l][a][m], (size_t)max_blocks * sub_vol(m) * sizeof(float));
            }
    }
    if (e == hipSuccess) e = hipHostMalloc(&A->hscal, 8 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) return fail(hip_fail(e, "adaptive-mesh allocation", __FILE__, __LINE__));
    *out = A;
    return MGFR_OK;
}

extern "C" void mgfr_amr_destroy(mgfr_amr *A) { amr_free(A); }

extern "C" int mgfr_amr_set_relaxation32(mgfr_amr *A, double omega)
{
    if (!A) return set_error(MGFR_ERR_ARG, "amr is NULL");
    int rc = mgfr_set_relaxation32(A->base, omega);  // validates omega
    if (rc) return rc;
    A->omega32 = omega;
    return MGFR_OK;
}

extern "C" int mgfr_amr_solve(mgfr_amr *A, const float *pos, int64_t np, double *u0_out, mgfr_stats *st_levels)
{
    if (!A || !pos) return set_error(MGFR_ERR_ARG, "amr and pos must be non-NULL");
    if (np < 1) return set_error(MGFR_ERR_ARG, "np must be >= 1");
    int rc;
    const int N0 = A->N0;
    const size_t n0 = (size_t)N0 * N0 * N0;
    if ((rc = mgfr_set_stream(A->base, A->stream))) return rc;
    const unsigned pg = (unsigned)((np + 255) / 256);
    auto listof = [](const std::vector<unsigned char> &v) {
        std::vector<int64_t> L;
        for (size_t i = 0; i < v.size(); ++i)
            if (v[i]) L.push_back((int64_t)i);
        return L;
    };
    auto fetch = [&](int l, std::vector<unsigned char> &v) {
        const size_t Ml = (size_t)(N0 << l) / 8;
        v.resize(Ml * Ml * Ml);
        return hipMemcpyAsync(v.data(), A->flag[l], v.size(), hipMemcpyDeviceToHost, A->stream);
    };
    // 1. refinement: level-1 blocks from base counts (flags built on the device)
    const int M1 = N0 / 4;
    MGFR_HIP(hipMemsetAsync(A->cnt0, 0, n0 * sizeof(int), A->stream));
    MGFR_HIP(hipMemsetAsync(A->flag[1], 0, (size_t)M1 * M1 * M1, A->stream));
    k_ngp_count<<<pg, 256, 0, A->stream>>>(pos, np, A->lg0, A->p.box / N0, A->cnt0);
    k_flag_base<<<(unsigned)std::min<size_t>((n0 + 255) / 256, 16384), 256, 0, A->stream>>>(A->cnt0, A->lg0,
                                                                                           A->flag[1]);
    MGFR_HIP(hipGetLastError());
    std::vector<unsigned char> blk1, blk2;
    MGFR_HIP(fetch(1, blk1));
    MGFR_HIP(hipStreamSynchronize(A->stream));
    if ((rc = upload_level(A, 1, listof(blk1)))) return rc;
    if (A->nref >= 2) {
        // level-2 blocks from level-1 counts inside level-1 blocks, then proper nesting
        const int N1 = 2 * N0, M2 = N1 / 4;
        LevelDev L1 = level_dev(A, 1);
        const size_t nc = (size_t)A->nb[1] * 512;
        MGFR_HIP(hipMemsetAsync(A->flag[2], 0, (size_t)M2 * M2 * M2, A->stream));
        if (nc) {
            MGFR_HIP(hipMemsetAsync(A->cntb, 0, nc * sizeof(int), A->stream));
            k_ngp_count_blocks<<<pg, 256, 0, A->stream>>>(pos, np, L1, A->p.box / N1, A->cntb);
            k_flag_l1<<<(unsigned)std::min<size_t>((nc + 255) / 256, 16384), 256, 0, A->stream>>>(
                A->cntb, A->nb[1], A->org[1], N1, A->flag[2]);
            const size_t n2 = (size_t)M2 * M2 * M2;
            k_nest<<<(unsigned)std::min<size_t>((n2 + 255) / 256, 16384), 256, 0, A->stream>>>(A->flag[2], N1,
                                                                                              A->flag[1]);
            MGFR_HIP(hipGetLastError());
        }
        MGFR_HIP(fetch(1, blk1));
        MGFR_HIP(fetch(2, blk2));
        MGFR_HIP(hipStreamSynchronize(A->stream));
        if ((rc = upload_level(A, 1, listof(blk1)))) return rc;
        if ((rc = upload_level(A, 2, listof(blk2)))) return rc;
    }
    // 2. composite cloud-in-cell masses (Sec. 3.1) on the base mesh and the blocks,
    //    then the covered coarser cells as sums of their daughters
    CicMaps Q{};
    Q.nref = A->nref;
    Q.lg0 = A->lg0;
    Q.box = A->p.box;
    Q.m0 = A->delta0;
    MGFR_HIP(hipMemsetAsync(A->delta0, 0, n0 * sizeof(double), A->stream));
    for (int l = 1; l <= A->nref; ++l) {
        Q.map[l] = A->map[l];
        Q.f0[l] = A->arr[l][1][0];
        if (A->nb[l])
            MGFR_HIP(hipMemsetAsync(A->arr[l][1][0], 0, (size_t)A->nb[l] * sub_vol(0) * sizeof(double), A->stream));
    }
    MGFR_HIP(hipMemsetAsync(A->dflag, 0, sizeof(int), A->stream));
    if (np <= A->bin_cap) {
        // binned: particles sorted by the group of cells they deposit into, one
        // LDS window per run; the few cubes across levels take the general path
        const CicKeys K = cic_keys(A);
        k_amr_cic_keys<<<(unsigned)((np + kBlock - 1) / kBlock), kBlock, 0, A->stream>>>(pos, np, Q, K, A->bkey,
                                                                                       A->bidx);
        MGFR_HIP(hipGetLastError());
        size_t tmp = A->sort_tmp_bytes;
        MGFR_HIP(sort_pairs_u32(A->sort_tmp, &tmp, A->bkey, A->bkey_s, A->bidx, A->perm, (size_t)np, cic_key_bits(A),
                                A->stream));
        k_amr_cic_binned<<<(unsigned)((np + kCicChunk - 1) / kCicChunk), kBlock, 0, A->stream>>>(
            pos, A->bkey_s, A->perm, np, Q, K, A->dflag);
        k_amr_cic_general<<<(unsigned)std::min<int64_t>((np + 255) / 256, 8192), 256, 0, A->stream>>>(
            pos, A->bkey_s, A->perm, np, Q, K.koff[A->nref + 1], A->dflag);
    } else {
        k_amr_cic_composite<<<pg, 256, 0, A->stream>>>(pos, np, Q, A->dflag);
    }
    for (int l = A->nref - 1; l >= 0; --l)
        if (A->nb[l + 1])
            k_amr_mass_up<<<grid_of((size_t)A->nb[l + 1] * 64), 256, 0, A->stream>>>(Q, l, A->nb[l + 1],
                                                                                    A->org[l + 1]);
    const unsigned sg = (unsigned)std::min<size_t>((n0 + 255) / 256, 1024);
    k_amr_sum_partial<<<sg, 256, 0, A->stream>>>(A->delta0, n0, A->partial);
    k_amr_sum_final<<<1, 1024, 0, A->stream>>>(A->partial, (int)sg, A->dscal);
    MGFR_HIP(hipGetLastError());
    MGFR_HIP(hipMemcpyAsync(A->hscal, A->dscal, sizeof(double), hipMemcpyDeviceToHost, A->stream));
    MGFR_HIP(hipMemcpyAsync(A->hscal + 1, A->dflag, sizeof(int), hipMemcpyDeviceToHost, A->stream));
    MGFR_HIP(hipStreamSynchronize(A->stream));
    int hflag = 0;
    memcpy(&hflag, A->hscal + 1, sizeof(int));
    if (hflag) return set_error(MGFR_ERR_NONFINITE, "a particle position is not finite");
    A->total_mass = A->hscal[0];
    if (!(A->total_mass > 0) || !std::isfinite(A->total_mass))
        return set_error(MGFR_ERR_NONFINITE, "total assigned mass is not positive and finite");
    // 3. base level: delta = m / mbar - 1, solved by the uniform solver
    k_amr_delta0<<<grid_of(n0, 8192), 256, 0, A->stream>>>(A->delta0, n0, A->total_mass / (double)n0);
    MGFR_HIP(hipGetLastError());
    MGFR_HIP(hipMemsetAsync(A->u0, 0, n0 * sizeof(double), A->stream));
    rc = mgfr_solve(A->base, A->delta0, A->u0, nullptr, &A->st[0]);
    if (rc < 0) return rc;
    // 4. refined levels, coarse to fine
    int worst = A->st[0].status;
    for (int l = 1; l <= A->nref; ++l) {
        if ((rc = solve_level(A, l))) return rc;
        const int s = A->st[l].status;
        if (s != MGFR_OK && (worst == MGFR_OK || s < 0)) worst = s;
    }
    if (u0_out) MGFR_HIP(hipMemcpyAsync(u0_out, A->u0, n0 * sizeof(double), hipMemcpyDeviceToDevice, A->stream));
    MGFR_HIP(hipStreamSynchronize(A->stream));
    if (st_levels)
        for (int l = 0; l <= A->nref; ++l) st_levels[l] = A->st[l];
    return worst;
}

extern "C" int mgfr_amr_reserve_particles(mgfr_amr *A, int64_t max_np)
{
    if (!A) return set_error(MGFR_ERR_ARG, "amr is NULL");
    if (max_np < 0) return set_error(MGFR_ERR_ARG, "max_np must be >= 0");
    if (max_np > (int64_t)0x7fffffff) return set_error(MGFR_ERR_ARG, "binning holds at most 2^31 - 1 particles");
    MGFR_HIP(hipStreamSynchronize(A->stream));
    amr_bin_free(A);
    if (max_np == 0) return MGFR_OK;
    size_t tmp = 0;
    MGFR_HIP(sort_pairs_u32(nullptr, &tmp, nullptr, nullptr, nullptr, nullptr, (size_t)max_np, cic_key_bits(A),
                            A->stream));
    const size_t b = (size_t)max_np * sizeof(uint32_t);
    if (hipMalloc(&A->bkey, b) != hipSuccess || hipMalloc(&A->bkey_s, b) != hipSuccess ||
        hipMalloc(&A->bidx, b) != hipSuccess || hipMalloc(&A->perm, b) != hipSuccess ||
        hipMalloc(&A->sort_tmp, std::max<size_t>(tmp, 256)) != hipSuccess) {
        (void)hipGetLastError();
        amr_bin_free(A);
        return set_error(MGFR_ERR_OOM, "binning workspace for %lld particles", (long long)max_np);
    }
    A->sort_tmp_bytes = std::max<size_t>(tmp, 256);
    A->bin_cap = max_np;
    return MGFR_OK;
}

extern "C" int mgfr_amr_composite(mgfr_amr *A, double *delta, double *delta_eff)
{
    if (!A || !delta || !delta_eff) return set_error(MGFR_ERR_ARG, "amr, delta and delta_eff must be non-NULL");
    CompArgs C{};
    C.nref = A->nref;
    C.lg0 = A->lg0;
    C.lgf = A->lg0 + A->nref;
    C.d0 = A->delta0;
    C.u0 = A->u0;
    for (int l = 1; l <= A->nref; ++l) {
        C.map[l] = A->map[l];
        C.u[l] = A->arr[l][0][0];
        C.f[l] = A->arr[l][1][0];
    }
    const double a3 = 1.0 / (A->p.a * A->p.a * A->p.a);
    C.inv_s = 1.0 / (A->beta * A->p.omega_m * a3);
    C.third_C_om = A->C / (3.0 * A->p.omega_m * a3);
    C.q = 1.0 / (A->p.n + 1);
    C.dout = delta;
    C.eout = delta_eff;
    const size_t n = (size_t)1 << (3 * C.lgf);
    k_amr_composite<<<grid_of(n, 16384), 256, 0, A->stream>>>(C);
    MGFR_HIP(hipGetLastError());
    MGFR_HIP(hipStreamSynchronize(A->stream));
    return MGFR_OK;
}

extern "C" int64_t mgfr_amr_num_blocks(const mgfr_amr *A, int level)
{
    if (!A || level < 1 || level > A->nref) return -1;
    return A->nb[level];
}

extern "C" int mgfr_amr_get_level(mgfr_amr *A, int level, int32_t *origins_host, double *u)
{
    if (!A || level < 1 || level > A->nref) return set_error(MGFR_ERR_ARG, "invalid level");
    const LevelDev L = level_dev(A, level);
    if (origins_host && L.nb) memcpy(origins_host, A->horg[level].data(), 3 * sizeof(int) * (size_t)L.nb);
    if (u && L.nb) {
        k_amr_copy_out<<<grid_of((size_t)L.nb * 512), 256, 0, A->stream>>>(L, u);
        MGFR_HIP(hipGetLastError());
        MGFR_HIP(hipStreamSynchronize(A->stream));
    }
    return MGFR_OK;
}
