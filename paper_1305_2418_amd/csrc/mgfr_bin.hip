// Particle binning for the particle <-> mesh steps (Sec. 3.1, Sec. 2).
//
// The cloud-in-cell assignment adds eight weights per particle to the mesh.
// Done in the caller's particle order, each weight is a float64 atomic add
// to a line that is usually not in any cache.  Binning orders the particle
// indices by the 8^3-cell tile that holds their lower CIC corner, so that one
// workgroup can accumulate a run of particles of one tile in LDS and write
// the 9^3 window once, and the force gather reads the mesh in tile order.
//
// The order is a counting sort over the T = 2^(3 (lg - 3)) tiles.  One pass
// computes each particle's tile and its rank within the tile; a scan of the
// counts gives each tile's first slot; a second pass writes the particle index
// to slot start + rank.  The count of a tile is split over S replicas (S = 64
// up to 2^18 tiles, fewer above): the particles 64 g .. 64 g + 63 (one wave)
// count into replica g mod S, so that a dense halo whose particles sit at
// scattered indices does not serialise hundreds of thousands of atomics on one
// address.  Replica s of tile t lives at s T + t (the replicas of a tile in
// different cache lines); the scan reads the counts tile-major, so slots are
// ascending in tile and the replicas of a tile follow one another.  Within a
// wave the lanes that share a tile are counted by one atomic and take
// consecutive ranks.  The order within a tile depends on the order of the
// atomics, which may differ between runs; no consumer depends on it (the
// assignment sums in LDS with atomics anyway, and the force is per particle).
//
// The consumers do not look for runs of equal tiles: the binning ends by
// cutting each tile's slots into work units of at most kUnit particles, and a
// workgroup takes one unit at a time, so that the dense tiles of a halo are
// spread over many workgroups.
#include "mgfr_internal.h"

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/iterator/counting_iterator.hpp>
#include <rocprim/iterator/transform_iterator.hpp>

namespace mgfr {

namespace {

// Tile of the lower CIC corner of a particle.  A particle with a non-finite
// position gets tile 0; the assignment kernel skips it and reports it.
__device__ __forceinline__ uint32_t tile_key(const float *__restrict__ pos, int64_t p, int lg, double h, double r)
{
    const int mask = (1 << lg) - 1, tl = lg - kBinLg;
    int i0 = 0, j0 = 0, k0 = 0;
    double t;
    uint32_t k = 0;
    if (cic_axis_r(pos[3 * p + 0], h, r, mask, i0, t) & cic_axis_r(pos[3 * p + 1], h, r, mask, j0, t) &
        cic_axis_r(pos[3 * p + 2], h, r, mask, k0, t))
        k = ((((uint32_t)(i0 >> kBinLg) << tl) | (uint32_t)(j0 >> kBinLg)) << tl) | (uint32_t)(k0 >> kBinLg);
    return k;
}

// key[p] = tile of particle p, rank[p] = its rank in replica (p / 64) mod S
// of that tile's count.  The lanes of a wave (64 consecutive particles) are
// grouped by tile (a ballot per distinct tile); the lowest lane of each group
// adds the group's size to the replica, all groups in one atomic instruction,
// and the group's lanes take consecutive ranks from the value it returns.
__global__ __launch_bounds__(kBlock) void k_bin_count(const float *__restrict__ pos, int64_t np, int lg, double h,
                                                        uint32_t rmask, size_t T, uint32_t *__restrict__ key,
                                                        uint32_t *__restrict__ rank, uint32_t *__restrict__ count)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint32_t rep = (uint32_t)(p >> 6) & rmask;  // wave-uniform
    const int lane = threadIdx.x & 63;
    const bool live = p < np;
    const uint32_t k = live ? tile_key(pos, p, lg, h, 1.0 / h) : 0u;
    if (live) key[p] = k;
    uint64_t todo = __ballot(live), grp = 0;
    int lead = lane;
    while (todo) {  // wave-uniform: one pass per distinct tile among the live lanes
        const int l = __builtin_ctzll(todo);
        const uint32_t kl = __builtin_amdgcn_readlane(k, l);
        const uint64_t m = __ballot(live && k == kl);
        if (live && k == kl) {
            grp = m;
            lead = l;
        }
        todo &= ~m;
    }
    uint32_t base = 0;
    if (live && lane == lead) base = atomicAdd(&count[(size_t)rep * T + k], (uint32_t)__popcll(grp));
    base = __shfl(base, lead, 64);
    if (live) rank[p] = base + (uint32_t)__popcll(grp & ((1ull << lane) - 1ull));
}

// start is tile-major: start[t S + s] = first slot of replica s of tile t
__global__ __launch_bounds__(kBlock) void k_bin_scatter(const uint32_t *__restrict__ key,
                                                          const uint32_t *__restrict__ rank,
                                                          const uint32_t *__restrict__ start, int64_t np,
                                                          uint32_t rmask, uint32_t *__restrict__ perm)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= np) return;
    const uint32_t rep = (uint32_t)(p >> 6) & rmask;
    perm[start[(size_t)key[p] * (rmask + 1) + rep] + rank[p]] = (uint32_t)p;
}

// slots [b, e) of tile t: from its first replica to the next tile's
__device__ __forceinline__ void tile_slots(const uint32_t *__restrict__ start, uint32_t t, uint32_t T, uint32_t S,
                                           uint32_t np, uint32_t &b, uint32_t &e)
{
    b = start[(size_t)t * S];
    e = t + 1 < T ? start[(size_t)(t + 1) * S] : np;
}

__global__ __launch_bounds__(kBlock) void k_unit_count(const uint32_t *__restrict__ start, uint32_t T, uint32_t S,
                                                         uint32_t np, uint32_t *__restrict__ nu)
{
    const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= T) return;
    uint32_t b, e;
    tile_slots(start, t, T, S, np, b, e);
    nu[t] = (e - b + kUnit - 1) / kUnit;
}

__global__ __launch_bounds__(kBlock) void k_unit_fill(const uint32_t *__restrict__ start,
                                                        const uint32_t *__restrict__ nu,
                                                        const uint32_t *__restrict__ uoff, uint32_t T, uint32_t S,
                                                        uint32_t np, uint4 *__restrict__ units,
                                                        uint32_t *__restrict__ total)
{
    const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= T) return;
    uint32_t b, e;
    tile_slots(start, t, T, S, np, b, e);
    const uint32_t o = uoff[t], n = nu[t];
    for (uint32_t k = 0; k < n; ++k)
        units[o + k] = make_uint4(t, b + k * kUnit, min(b + (k + 1) * kUnit, e), 0u);
    if (t == T - 1) *total = o + n;
}

__global__ __launch_bounds__(kBlock) void k_zero_u32(uint32_t *__restrict__ x, size_t n)
{
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (size_t)gridDim.x * kBlock) x[t] = 0u;
}

inline size_t n_tiles(const mgfr_ctx *c) { return (size_t)1 << (3 * (c->lev[0].lg - kBinLg)); }
// replicas per tile count: 64, fewer above 2^18 tiles (at most 2^24 counters)
inline size_t n_reps(size_t T) { return std::max<size_t>(1, std::min<size_t>(64, ((size_t)1 << 24) / T)); }

// the replica counts in scan order: element u = t S + s reads count[s T + t]
struct TileMajor {
    const uint32_t *count;
    uint32_t T, lgS;
    __host__ __device__ uint32_t operator()(uint32_t u) const
    {
        return count[(size_t)(u & ((1u << lgS) - 1u)) * T + (u >> lgS)];
    }
};

inline auto tile_major(const uint32_t *count, size_t T, size_t S)
{
    uint32_t lgS = 0;
    while (((size_t)1 << lgS) < S) ++lgS;
    return rocprim::make_transform_iterator(rocprim::make_counting_iterator<uint32_t>(0u),
                                            TileMajor{count, (uint32_t)T, lgS});
}

unsigned grid_for(size_t n) { return (unsigned)std::min<size_t>((n + kBlock - 1) / kBlock, 4096); }

// at most one unit per tile plus one per kUnit particles
inline size_t max_units(size_t T, int64_t np) { return T + (size_t)((np + kUnit - 1) / kUnit); }

}  // namespace

void bin_free(mgfr_ctx *c)
{
    (void)hipFree(c->bkey);
    (void)hipFree(c->bidx);
    (void)hipFree(c->perm);
    (void)hipFree(c->tcount);
    (void)hipFree(c->tstart);
    (void)hipFree(c->unit_n);
    (void)hipFree(c->unit_off);
    (void)hipFree(c->units);
    (void)hipFree(c->unit_total);
    (void)hipFree(c->sort_tmp);
    c->bkey = c->bidx = c->perm = c->tcount = c->tstart = c->unit_n = c->unit_off = nullptr;
    c->unit_total = nullptr;
    c->units = nullptr;
    c->unit_grid = 0;
    c->sort_tmp = nullptr;
    c->sort_tmp_bytes = 0;
    c->bin_cap = 0;
    c->perm_np = 0;
}

int bin_reserve(mgfr_ctx *c, int64_t np)
{
    if (np <= c->bin_cap) return MGFR_OK;
    if (np > (int64_t)0x7fffffff) return set_error(MGFR_ERR_ARG, "binning holds at most 2^31 - 1 particles");
    MGFR_HIP(hipStreamSynchronize(c->stream));
    bin_free(c);
    const size_t T = n_tiles(c), TS = T * n_reps(T), U = max_units(T, np);
    size_t tmp = 0, tmp2 = 0;
    MGFR_HIP(rocprim::exclusive_scan(nullptr, tmp, tile_major(nullptr, T, n_reps(T)), (uint32_t *)nullptr, 0u, TS,
                                     rocprim::plus<uint32_t>(), c->stream));
    MGFR_HIP(rocprim::exclusive_scan(nullptr, tmp2, (const uint32_t *)nullptr, (uint32_t *)nullptr, 0u, T,
                                     rocprim::plus<uint32_t>(), c->stream));
    tmp = std::max(tmp, tmp2);
    const size_t b = (size_t)np * sizeof(uint32_t);
    if (hipMalloc(&c->bkey, b) != hipSuccess || hipMalloc(&c->bidx, b) != hipSuccess ||
        hipMalloc(&c->perm, b) != hipSuccess || hipMalloc(&c->tcount, TS * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&c->tstart, TS * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&c->unit_n, T * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&c->unit_off, T * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&c->units, U * sizeof(uint4)) != hipSuccess ||
        hipMalloc(&c->unit_total, sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&c->sort_tmp, std::max<size_t>(tmp, 256)) != hipSuccess) {
        (void)hipGetLastError();
        bin_free(c);
        return set_error(MGFR_ERR_OOM, "binning workspace for %lld particles", (long long)np);
    }
    c->sort_tmp_bytes = std::max<size_t>(tmp, 256);
    c->bin_cap = np;
    // the unit kernels loop over units: enough workgroups to fill the chip a few times over
    c->unit_grid = (unsigned)std::min<size_t>(U, 16384);
    return MGFR_OK;
}

// Digit width of the radix sort (the adaptive solver's block keys): 9 bits
// sort keys of 17 or 18 bits in two passes instead of rocPRIM's default three
// of 8 bits
#ifndef MGFR_SORT_RADIX_BITS
#define MGFR_SORT_RADIX_BITS 9
#endif

hipError_t sort_pairs_u32(void *tmp, size_t *tmp_bytes, const uint32_t *kin, uint32_t *kout, const uint32_t *vin,
                          uint32_t *vout, size_t n, unsigned bits, hipStream_t stream)
{
#if MGFR_SORT_RADIX_BITS != 8
    // wider digits: ceil(bits / radix) passes over the pairs instead of ceil(bits / 8)
    using cfg = rocprim::radix_sort_config<
        rocprim::default_config, rocprim::default_config,
        rocprim::radix_sort_onesweep_config<rocprim::kernel_config<512, 32>, rocprim::kernel_config<512, 12>,
                                            MGFR_SORT_RADIX_BITS, rocprim::block_radix_rank_algorithm::match>>;
    return rocprim::radix_sort_pairs<cfg>(tmp, *tmp_bytes, kin, kout, vin, vout, n, 0u, bits, stream);
#else
    return rocprim::radix_sort_pairs(tmp, *tmp_bytes, kin, kout, vin, vout, n, 0u, bits, stream);
#endif
}

int bin_particles(mgfr_ctx *c, const float *pos, int64_t np)
{
    c->perm_np = 0;
    if (np > c->bin_cap) return set_error(MGFR_ERR_ARG, "binning workspace holds %lld particles, got %lld",
                                          (long long)c->bin_cap, (long long)np);
    if (np == 0) return MGFR_OK;
    const Level &L0 = c->lev[0];
    const size_t T = n_tiles(c), S = n_reps(T);
    const uint32_t rmask = (uint32_t)S - 1u;
    const unsigned gp = (unsigned)((np + kBlock - 1) / kBlock);
    k_zero_u32<<<grid_for(T * S), kBlock, 0, c->stream>>>(c->tcount, T * S);
    k_bin_count<<<gp, kBlock, 0, c->stream>>>(pos, np, L0.lg, L0.h, rmask, T, c->bkey, c->bidx, c->tcount);
    MGFR_HIP(hipGetLastError());
    size_t tmp = c->sort_tmp_bytes;
    MGFR_HIP(rocprim::exclusive_scan(c->sort_tmp, tmp, tile_major(c->tcount, T, S), c->tstart, 0u, T * S,
                                     rocprim::plus<uint32_t>(), c->stream));
    k_bin_scatter<<<gp, kBlock, 0, c->stream>>>(c->bkey, c->bidx, c->tstart, np, rmask, c->perm);
    const unsigned gt = (unsigned)((T + kBlock - 1) / kBlock);
    k_unit_count<<<gt, kBlock, 0, c->stream>>>(c->tstart, (uint32_t)T, (uint32_t)S, (uint32_t)np, c->unit_n);
    MGFR_HIP(hipGetLastError());
    tmp = c->sort_tmp_bytes;
    MGFR_HIP(rocprim::exclusive_scan(c->sort_tmp, tmp, (const uint32_t *)c->unit_n, c->unit_off, 0u, T,
                                     rocprim::plus<uint32_t>(), c->stream));
    k_unit_fill<<<gt, kBlock, 0, c->stream>>>(c->tstart, c->unit_n, c->unit_off, (uint32_t)T, (uint32_t)S,
                                              (uint32_t)np, c->units, c->unit_total);
    MGFR_HIP(hipGetLastError());
    c->perm_np = np;
    return MGFR_OK;
}

}  // namespace mgfr
