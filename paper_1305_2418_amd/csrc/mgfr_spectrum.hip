// Power-spectrum diagnostic of the effective-mass formulation (Sec. 3.4):
// the ratio of the power spectrum of delta + delta_eff to that of delta in
// shells of |k|.  Where the fifth force acts unscreened delta_eff = delta / 3
// and the ratio is (4/3)^2; where the field is screened delta_eff -> 0 and
// the ratio -> 1.  This is the quantity behind the paper's power-spectrum
// comparison (Sec. 5), evaluated on one field instead of two simulations.
//
// A library primitive is used for the transforms (hipFFT, real-to-complex,
// float64); the shell sums are a kernel of this file.  Normalisation:
// P(k_i) = L^3 / N^6 * mean over the modes of shell i of |sum_x f(x) e^{-i k.x}|^2,
// shell i = the modes whose integer wave vector n has i - 1/2 <= |n| < i + 1/2,
// k_i = 2 pi i / L, i = 1 .. nbins (nbins <= N/2).
#include "mgfr_internal.h"

#include <hipfft/hipfft.h>

#include <vector>

namespace mgfr {

namespace {

constexpr int kSpecMaxBins = 1024;

// out = a + b (b may be NULL: out = a); the transforms read this copy, never
// the caller's arrays
__global__ __launch_bounds__(kBlock) void k_add(const double *__restrict__ a, const double *__restrict__ b, size_t n,
                                                double *__restrict__ out)
{
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (size_t)gridDim.x * kBlock)
        out[t] = b ? a[t] + b[t] : a[t];
}

// Shell sums of |F1|^2, |F2|^2 and the mode counts over the half-spectrum of a
// real transform (the modes with 0 < kz < N/2 stand for themselves and their
// conjugates: weight 2).  Per-block LDS histograms, then float64 atomics.
__global__ __launch_bounds__(kBlock) void k_shells(const double2 *__restrict__ F1, const double2 *__restrict__ F2,
                                                   int lg, int nbins, double *__restrict__ sum1,
                                                   double *__restrict__ sum2, double *__restrict__ cnt)
{
    __shared__ double h1[kSpecMaxBins + 1], h2[kSpecMaxBins + 1], hc[kSpecMaxBins + 1];
    for (int i = threadIdx.x; i <= nbins; i += kBlock) h1[i] = h2[i] = hc[i] = 0.0;
    __syncthreads();
    const int N = 1 << lg, Nz = N / 2 + 1;
    const size_t n = (size_t)N * N * Nz;
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (size_t)gridDim.x * kBlock) {
        const int iz = (int)(t % Nz);
        const size_t r = t / Nz;
        const int iy = (int)(r & (N - 1)), ix = (int)(r >> lg);
        const int nx = ix < N / 2 ? ix : ix - N, ny = iy < N / 2 ? iy : iy - N;
        const long n2 = (long)nx * nx + (long)ny * ny + (long)iz * iz;
        // no |n| lies on a shell edge (edges are half-integers, n2 is an integer)
        const int bin = (int)floor(sqrt((double)n2) + 0.5);
        if (bin < 1 || bin > nbins) continue;
        const double w = (iz == 0 || iz == N / 2) ? 1.0 : 2.0;
        const double2 a = F1[t], b = F2[t];
        atomicAdd(&h1[bin], w * (a.x * a.x + a.y * a.y));
        atomicAdd(&h2[bin], w * (b.x * b.x + b.y * b.y));
        atomicAdd(&hc[bin], w);
    }
    __syncthreads();
    for (int i = 1 + threadIdx.x; i <= nbins; i += kBlock) {
        if (hc[i] != 0.0) {
            unsafeAtomicAdd(&sum1[i], h1[i]);
            unsafeAtomicAdd(&sum2[i], h2[i]);
            unsafeAtomicAdd(&cnt[i], hc[i]);
        }
    }
}

const char *fft_err(hipfftResult r)
{
    switch (r) {
    case HIPFFT_ALLOC_FAILED: return "hipFFT: allocation failed";
    case HIPFFT_INVALID_VALUE: return "hipFFT: invalid value";
    case HIPFFT_EXEC_FAILED: return "hipFFT: execution failed";
    default: return "hipFFT error";
    }
}

}  // namespace

}  // namespace mgfr

using namespace mgfr;

extern "C" int mgfr_power_ratio(mgfr_ctx *c, const double *delta, const double *delta_eff, int nbins, double *k,
                                double *ratio, double *p_delta, double *counts)
{
    if (!c || !delta || !delta_eff || !k || !ratio) return set_error(MGFR_ERR_ARG, "null argument");
    const Level &L0 = c->lev[0];
    const int N = L0.N;
    if (nbins < 1 || nbins > N / 2 || nbins > kSpecMaxBins)
        return set_error(MGFR_ERR_ARG, "nbins must be in [1, min(N/2, %d)]", kSpecMaxBins);
    const size_t n = (size_t)N * N * N, nc = (size_t)N * N * (N / 2 + 1);
    double *sum = nullptr, *acc = nullptr;
    double2 *F1 = nullptr, *F2 = nullptr;
    hipfftHandle plan = 0;
    bool have_plan = false;
    int rc = MGFR_OK;
    auto fail = [&](int code) {
        rc = code;
        return code;
    };
    do {
        if (hipMalloc(&sum, n * sizeof(double)) != hipSuccess || hipMalloc(&F1, nc * sizeof(double2)) != hipSuccess ||
            hipMalloc(&F2, nc * sizeof(double2)) != hipSuccess ||
            hipMalloc(&acc, 3 * (size_t)(nbins + 1) * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            fail(set_error(MGFR_ERR_OOM, "power-spectrum workspace for N = %d", N));
            break;
        }
        hipfftResult fr = hipfftPlan3d(&plan, N, N, N, HIPFFT_D2Z);
        if (fr != HIPFFT_SUCCESS) {
            fail(set_error(MGFR_ERR_HIP, "%s (plan)", fft_err(fr)));
            break;
        }
        have_plan = true;
        if ((fr = hipfftSetStream(plan, c->stream)) != HIPFFT_SUCCESS) {
            fail(set_error(MGFR_ERR_HIP, "%s (stream)", fft_err(fr)));
            break;
        }
        const unsigned g = (unsigned)std::min<size_t>((n + kBlock - 1) / kBlock, 16384);
        k_add<<<g, kBlock, 0, c->stream>>>(delta, nullptr, n, sum);
        if (hipGetLastError() != hipSuccess) {
            fail(set_error(MGFR_ERR_HIP, "launch failed"));
            break;
        }
        if ((fr = hipfftExecD2Z(plan, sum, (hipfftDoubleComplex *)F1)) != HIPFFT_SUCCESS) {
            fail(set_error(MGFR_ERR_HIP, "%s (transform)", fft_err(fr)));
            break;
        }
        k_add<<<g, kBlock, 0, c->stream>>>(delta, delta_eff, n, sum);
        if (hipGetLastError() != hipSuccess) {
            fail(set_error(MGFR_ERR_HIP, "launch failed"));
            break;
        }
        if ((fr = hipfftExecD2Z(plan, sum, (hipfftDoubleComplex *)F2)) != HIPFFT_SUCCESS) {
            fail(set_error(MGFR_ERR_HIP, "%s (transform)", fft_err(fr)));
            break;
        }
        if (hipMemsetAsync(acc, 0, 3 * (size_t)(nbins + 1) * sizeof(double), c->stream) != hipSuccess) {
            fail(set_error(MGFR_ERR_HIP, "memset failed"));
            break;
        }
        const unsigned gs = (unsigned)std::min<size_t>((nc + kBlock - 1) / kBlock, 4096);
        k_shells<<<gs, kBlock, 0, c->stream>>>(F1, F2, L0.lg, nbins, acc, acc + (nbins + 1), acc + 2 * (nbins + 1));
        std::vector<double> h(3 * (size_t)(nbins + 1));
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(h.data(), acc, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess) {
            fail(set_error(MGFR_ERR_HIP, "shell sums failed"));
            break;
        }
        const double box = c->p.box, norm = box * box * box / ((double)n * (double)n);
        for (int i = 1; i <= nbins; ++i) {
            const double s1 = h[i], s2 = h[(nbins + 1) + i], cn = h[2 * (nbins + 1) + i];
            k[i - 1] = 2.0 * 3.141592653589793 * i / box;
            ratio[i - 1] = s1 > 0.0 ? s2 / s1 : 0.0;
            if (p_delta) p_delta[i - 1] = cn > 0.0 ? norm * s1 / cn : 0.0;
            if (counts) counts[i - 1] = cn;
        }
    } while (false);
    if (have_plan) (void)hipfftDestroy(plan);
    (void)hipFree(sum);
    (void)hipFree(F1);
    (void)hipFree(F2);
    (void)hipFree(acc);
    return rc;
}

// ------------------------------------------------------------------------
// Particle-mesh potential for chained steps: lap_x phi = (3/2) Omega_m H0^2
// delta / a with the periodic 7-point Laplacian (the operator's own
// discretisation), inverted exactly in Fourier space: its eigenvalue at
// integer wave vector n is -(4/h^2) sum_d sin^2(pi n_d / N).  H0 = 100 in
// km/s per Mpc/h, so phi is in (km/s)^2.  The k = 0 mode of phi is zero.
namespace mgfr {
namespace {

__global__ __launch_bounds__(kBlock) void k_pm_green(double2 *__restrict__ F, int lg, double ih2, double pref)
{
    const int N = 1 << lg, Nz = N / 2 + 1;
    const size_t n = (size_t)N * N * Nz;
    const double pN = M_PI / (double)N;
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (size_t)gridDim.x * kBlock) {
        const int iz = (int)(t % Nz);
        const size_t r = t / Nz;
        const int iy = (int)(r & (N - 1)), ix = (int)(r >> lg);
        const double sx = sin(pN * ix), sy = sin(pN * iy), sz = sin(pN * iz);
        const double lam = 4.0 * ih2 * (sx * sx + sy * sy + sz * sz);  // minus the Laplacian's eigenvalue
        const double g = (ix | iy | iz) ? -pref / lam : 0.0;
        F[t].x *= g;
        F[t].y *= g;
    }
}

}  // namespace

void pm_free(mgfr_ctx *c)
{
    if (c->pm_fwd) (void)hipfftDestroy((hipfftHandle)c->pm_fwd);
    if (c->pm_inv) (void)hipfftDestroy((hipfftHandle)c->pm_inv);
    (void)hipFree(c->pm_spec);
    c->pm_fwd = c->pm_inv = nullptr;
    c->pm_spec = nullptr;
}

int pm_potential(mgfr_ctx *c, const double *delta, double *phi)
{
    const Level &L0 = c->lev[0];
    const int N = L0.N;
    const size_t n = (size_t)N * N * N, nc = (size_t)N * N * (N / 2 + 1);
    hipfftResult fr;
    if (!c->pm_spec) {
        if (hipMalloc(&c->pm_spec, nc * sizeof(double2)) != hipSuccess) {
            (void)hipGetLastError();
            c->pm_spec = nullptr;
            return set_error(MGFR_ERR_OOM, "particle-mesh spectrum for N = %d", N);
        }
        hipfftHandle a = 0, b = 0;
        if ((fr = hipfftPlan3d(&a, N, N, N, HIPFFT_D2Z)) != HIPFFT_SUCCESS) {
            pm_free(c);
            return set_error(MGFR_ERR_HIP, "%s (particle-mesh plan)", fft_err(fr));
        }
        c->pm_fwd = (void *)a;
        if ((fr = hipfftPlan3d(&b, N, N, N, HIPFFT_Z2D)) != HIPFFT_SUCCESS) {
            pm_free(c);
            return set_error(MGFR_ERR_HIP, "%s (particle-mesh plan)", fft_err(fr));
        }
        c->pm_inv = (void *)b;
    }
    const hipfftHandle a = (hipfftHandle)c->pm_fwd, b = (hipfftHandle)c->pm_inv;
    if ((fr = hipfftSetStream(a, c->stream)) != HIPFFT_SUCCESS || (fr = hipfftSetStream(b, c->stream)) != HIPFFT_SUCCESS)
        return set_error(MGFR_ERR_HIP, "%s (stream)", fft_err(fr));
    const unsigned g = (unsigned)std::min<size_t>((n + kBlock - 1) / kBlock, 16384);
    k_add<<<g, kBlock, 0, c->stream>>>(delta, nullptr, n, phi);  // the transform may overwrite its input
    MGFR_HIP(hipGetLastError());
    if ((fr = hipfftExecD2Z(a, phi, (hipfftDoubleComplex *)c->pm_spec)) != HIPFFT_SUCCESS)
        return set_error(MGFR_ERR_HIP, "%s (transform)", fft_err(fr));
    const double H0 = 100.0;
    const double pref = 1.5 * c->p.omega_m * H0 * H0 / c->p.a / (double)n;  // with the 1/N^3 of the inverse
    const unsigned gc = (unsigned)std::min<size_t>((nc + kBlock - 1) / kBlock, 16384);
    k_pm_green<<<gc, kBlock, 0, c->stream>>>(c->pm_spec, L0.lg, 1.0 / (L0.h * L0.h), pref);
    MGFR_HIP(hipGetLastError());
    if ((fr = hipfftExecZ2D(b, (hipfftDoubleComplex *)c->pm_spec, phi)) != HIPFFT_SUCCESS)
        return set_error(MGFR_ERR_HIP, "%s (inverse transform)", fft_err(fr));
    return MGFR_OK;
}

}  // namespace mgfr
