// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <string>
#include <vector>

#include "mgfr.h"

namespace mgfr {

constexpr double kCOverH0 = 2997.92458;  // c/H0 in Mpc/h
constexpr double kCkms = 299792.458;     // c in km/s
constexpr int kTailN = 16;               // levels with N <= kTailN run inside one workgroup
constexpr int kBlock = 256;
constexpr int kTailThreads = 1024;
constexpr int kMaxLevels = 12;

// Constants of the dimensionless operator on one level.
struct OpConst {
    double ih2;     // 1/h^2 of the level
    double bC;      // beta * C
    double q;       // 1/(n+1)
    double max_du;  // Newton step limit (<= 0: none)
    const double *tab;  // 2^(j/64), j = 0..63 (table-driven exponential; global or LDS copy)
};

struct Level {
    int N = 0, lg = 0;
    double h = 0;
    double *u = nullptr, *f = nullptr, *ubar = nullptr;
    double *alt = nullptr;  // second buffer of out-of-place sweeps (current iterate is u)
    // float32 mirrors for the mixed-precision inner cycle
    float *e32 = nullptr, *r32 = nullptr, *u32 = nullptr, *ebar32 = nullptr;
    float *e32alt = nullptr;  // second e buffer of the fused float32 sweep (levels with N >= 128)
};

struct Timer {
    std::vector<hipEvent_t> ev;
    int used = 0;
};

}  // namespace mgfr

struct mgfr_ctx {
    mgfr_params p{};
    hipStream_t stream = nullptr;
    int device = 0;
    double fbar = 0, beta = 0, C = 0, bC = 0, q = 0;
    int nlev = 0;
    mgfr::Level lev[mgfr::kMaxLevels];
    double *alt0 = nullptr;  // level-0 second buffer (owned)
    int fused_min_n = 512;   // levels with N >= this use the fused out-of-place sweep (0: never)
    int colour32_min_n = 128; // float32 sweeps on levels with N >= this by one-colour pass kernels (0: never)
    int fused32 = 0;          // those sweeps as one fused red-black kernel per sweep instead
    double omega32 = 1.0;     // relaxation factor of the float32 correction sweeps (mixed solve)
    double omega_now = 1.0;   // the factor in use (set to 1 once the outer residual grows)
    int inner_max = 1;        // float32 correction V-cycles per float64 residual check, at most
    int smooth_max = 0;       // adaptive smoothing: sweeps double up to this when the residual stalls (0: off)
    bool e32_zero = false;    // level-0 e32 is zero but not cleared: its first colour pass writes it
    // reduction scratch
    double *partial = nullptr;  // [2 * nparts]
    int nparts = 0;
    double *dscal = nullptr;    // device scalars [8]
    double *hscal = nullptr;    // pinned host scalars [8]
    int *dflag = nullptr;       // device flag
    // mixed precision float64 scratch
    double *r64 = nullptr;
    double *exp2tab = nullptr;  // 2^(j/64), j = 0..63, for the table-driven float64 exponential
    // timing
    bool timing = false;
    mgfr::Timer sweep_timer;
    hipEvent_t ev_a = nullptr, ev_b = nullptr, ev_c = nullptr;
    // learned warm start: the attached network (mgfr_set_net: the caller's;
    // mgfr_nn_init: the context's own, destroyed with it)
    void *nn = nullptr;
    bool nn_owned = false;
    // particle binning by 8^3 tiles of CIC lower-corner cells (mgfr_bin.hip)
    int binning = 1;           // 0: assign by direct global atomics
    int64_t bin_cap = 0;       // particles the binning workspace holds
    int64_t perm_np = 0;       // particle count of the last binning (0: none)
    uint32_t *bkey = nullptr, *bidx = nullptr, *perm = nullptr;  // tile and rank of each particle, sorted order
    uint32_t *tcount = nullptr, *tstart = nullptr;  // particles per tile, first sorted slot of each tile
    uint32_t *unit_n = nullptr, *unit_off = nullptr; // work units per tile and the first of each tile
    uint4 *units = nullptr;                          // (tile, first slot, end slot, 0) of each work unit
    uint32_t *unit_total = nullptr;                  // number of work units of the last binning
    uint32_t unit_grid = 0;                          // workgroups of the unit kernels
    void *sort_tmp = nullptr;                        // workspace of the scans
    size_t sort_tmp_bytes = 0;
    // particle-mesh potential (mgfr_pm_accel): FFT plans and the half spectrum, made on first use
    void *pm_fwd = nullptr, *pm_inv = nullptr;
    double2 *pm_spec = nullptr;
};

namespace mgfr {

int set_error(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what, const char *file, int line);

#define MGFR_HIP(call)                                                     \
    do {                                                                   \
        hipError_t _e = (call);                                            \
        if (_e != hipSuccess) return mgfr::hip_fail(_e, #call, __FILE__, __LINE__); \
    } while (0)

inline OpConst level_const(const mgfr_ctx *c, int l)
{
    OpConst k;
    k.ih2 = 1.0 / (c->lev[l].h * c->lev[l].h);
    k.bC = c->bC;
    k.q = c->q;
    k.max_du = c->p.max_du;
    k.tab = c->exp2tab;
    return k;
}

// launch helpers implemented in mgfr_solver.hip
int launch_sweep64(mgfr_ctx *c, int l, double *u, const double *f, int sweeps, bool timed);
int launch_residual_norm64(mgfr_ctx *c, int l, const double *u, const double *f, double *rmax,
                           double *rsumsq);
int vcycle64(mgfr_ctx *c, int l);
int solve_fp64_from(mgfr_ctx *c, double *u, mgfr_stats *st, double D);  // V-cycles from the current u
// adaptive smoothing: after a residual check, res (this check) against res2
// (two checks back, < 0 if none); doubles the sweeps when it has not fallen
void adapt_smoothing(mgfr_ctx *c, double res, double res2);
int collect_timing(mgfr_ctx *c, mgfr_stats *st);

// mixed precision (mgfr_mixed.hip)
int mixed_alloc(mgfr_ctx *c);
int solve_mixed(mgfr_ctx *c, double *u, mgfr_stats *st, double D);

// particle binning (mgfr_bin.hip)
constexpr int kBinLg = 3;  // tile edge 2^kBinLg cells
constexpr int kCicPer = 8;                        // particles per thread and workgroup chunk of a binned assignment
constexpr int kCicChunk = kBlock * kCicPer;
constexpr int kWin = (1 << kBinLg) + 1;           // LDS window edge: a tile plus one cell
constexpr int kWin3 = kWin * kWin * kWin;
// The binned particle kernels work on units: up to kUnit sorted slots of one
// tile (a tile with more particles is split), kUnit / kBlock per thread.
#ifndef MGFR_UNIT
#define MGFR_UNIT 1024
#endif
constexpr int kUnit = MGFR_UNIT;
constexpr int kUnitPer = kUnit / kBlock;
int bin_reserve(mgfr_ctx *c, int64_t np);
int bin_particles(mgfr_ctx *c, const float *pos, int64_t np);  // counting sort by tile; sets perm_np
void bin_free(mgfr_ctx *c);
// Stable radix sort of (key, value) uint32 pairs on the low `bits` key bits.
// With tmp == nullptr only *tmp_bytes is set (the workspace the sort needs).
hipError_t sort_pairs_u32(void *tmp, size_t *tmp_bytes, const uint32_t *kin, uint32_t *kout, const uint32_t *vin,
                          uint32_t *vout, size_t n, unsigned bits, hipStream_t stream);

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

// cic_axis with the reciprocal r = 1/h given: x/h as x r plus one FMA
// correction, which by Markstein's theorem is the correctly rounded quotient
// (r correctly rounded, x r within an ulp), so i0 and t are those of
// cic_axis.  An int32 conversion serves every position within 2^31 cells.
__device__ __forceinline__ bool cic_axis_r(float x, double h, double r, int mask, int &i0, double &t)
{
    const double xd = (double)x;
    double q = xd * r;
    q = fma(fma(-q, h, xd), r, q);
    const double xi = q - 0.5;
    if (!(fabs(xi) < 4.0e18)) return false;
    const double fl = floor(xi);
    t = xi - fl;
    if (fabs(fl) < 2147483648.0)
        i0 = (int)fl & mask;
    else
        i0 = (int)((long long)fl & (long long)mask);
    return true;
}

// particle-mesh potential (mgfr_spectrum.hip): phi with lap phi = (3/2) Omega_m H0^2 delta / a
// by FFT of the 7-point Laplacian; delta and phi may not alias
int pm_potential(mgfr_ctx *c, const double *delta, double *phi);
void pm_free(mgfr_ctx *c);

// learned warm start (mgfr_nn.hip)
int nn_warm_start(mgfr_ctx *c, const double *delta, double *u, double *t_ms);
void nn_free(mgfr_ctx *c);

}  // namespace mgfr
