// Particle binning for the particle <-> mesh steps (Sec. 3.1, Sec. 2).
//
// The cloud-in-cell assignment adds eight weights per particle to the mesh.
// Done in the caller's particle order, each weight is a float64 atomic add
// to a line that is usually not in any cache.  Binning sorts the particle
// indices by the 8^3-cell tile that holds their lower CIC corner, so that one
// workgroup can accumulate a run of particles of one tile in LDS and write
// the 9^3 window once, and the force gather reads the mesh in tile order.
//
// The sort is rocPRIM's device radix sort over the tile key's 3 (lg - 3) bits
// (stable: equal keys keep ascending particle index), with 9-bit digits.
#include "mgfr_internal.h"

#include <rocprim/device/device_radix_sort.hpp>

namespace mgfr {

namespace {

// key[p] = tile of the lower CIC corner of particle p, idx[p] = p.  A particle
// with a non-finite position gets key 0; the assignment kernel skips it and
// reports it.
__global__ __launch_bounds__(kBlock) void k_bin_keys(const float *__restrict__ pos, int64_t np, int lg, double h,
                                                       uint32_t *__restrict__ key, uint32_t *__restrict__ idx)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= np) return;
    const int mask = (1 << lg) - 1, tl = lg - kBinLg;
    int i0, j0, k0;
    double t;
    uint32_t k = 0;
    if (cic_axis(pos[3 * p + 0], h, mask, i0, t) && cic_axis(pos[3 * p + 1], h, mask, j0, t) &&
        cic_axis(pos[3 * p + 2], h, mask, k0, t))
        k = ((((uint32_t)(i0 >> kBinLg) << tl) | (uint32_t)(j0 >> kBinLg)) << tl) | (uint32_t)(k0 >> kBinLg);
    key[p] = k;
    idx[p] = (uint32_t)p;
}

inline unsigned key_bits(const mgfr_ctx *c) { return (unsigned)std::max(1, 3 * (c->lev[0].lg - kBinLg)); }

}  // namespace

void bin_free(mgfr_ctx *c)
{
    (void)hipFree(c->bkey);
    (void)hipFree(c->bkey_s);
    (void)hipFree(c->bidx);
    (void)hipFree(c->perm);
    (void)hipFree(c->sort_tmp);
    c->bkey = c->bkey_s = c->bidx = c->perm = nullptr;
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
    size_t tmp = 0;
    MGFR_HIP(sort_pairs_u32(nullptr, &tmp, nullptr, nullptr, nullptr, nullptr, (size_t)np, key_bits(c), c->stream));
    const size_t b = (size_t)np * sizeof(uint32_t);
    if (hipMalloc(&c->bkey, b) != hipSuccess || hipMalloc(&c->bkey_s, b) != hipSuccess ||
        hipMalloc(&c->bidx, b) != hipSuccess || hipMalloc(&c->perm, b) != hipSuccess ||
        hipMalloc(&c->sort_tmp, std::max<size_t>(tmp, 256)) != hipSuccess) {
        (void)hipGetLastError();
        bin_free(c);
        return set_error(MGFR_ERR_OOM, "binning workspace for %lld particles", (long long)np);
    }
    c->sort_tmp_bytes = std::max<size_t>(tmp, 256);
    c->bin_cap = np;
    return MGFR_OK;
}

// Digit width of the radix sort: 9 bits sort the 18-bit tile keys of a 512^3
// mesh in two passes instead of rocPRIM's default three of 8 bits (0.9 ms less
// per assignment of 512^3 particles)
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
    const Level &L0 = c->lev[0];
    k_bin_keys<<<(unsigned)((np + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(pos, np, L0.lg, L0.h, c->bkey,
                                                                                 c->bidx);
    MGFR_HIP(hipGetLastError());
    size_t tmp = c->sort_tmp_bytes;
    MGFR_HIP(sort_pairs_u32(c->sort_tmp, &tmp, c->bkey, c->bkey_s, c->bidx, c->perm, (size_t)np, key_bits(c),
                            c->stream));
    c->perm_np = np;
    return MGFR_OK;
}

}  // namespace mgfr
