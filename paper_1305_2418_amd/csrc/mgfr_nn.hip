// Learned warm start: a small 3D U-Net in bfloat16 with float32 accumulation,
// built from hand-written MFMA convolution kernels (forward, backward-data,
// backward-weight), an Adam optimiser and the element-wise glue, all on the
// device.  The network maps the density contrast of a periodic S^3 mesh (plus
// the scale factor and |f_R0| as constant channels) to the solution u of the
// field equation on that mesh.  The solver uses it at the N/4 level of an N^3
// problem and prolongs the prediction to the finest level as the initial
// guess of the multigrid solve (Sec. 3.3 step 2 takes the initial guess from
// outside; multigrid still iterates to the same tolerance).
//
// Architecture (channels): 16 -> [16,16] -> pool -> [32,32] -> pool -> [64,64]
// -> up, concat(64+32) -> [32,32] -> up, concat(32+16) -> [16,16] -> 1x1 -> 1,
// every bracketed entry a 3^3 periodic convolution with bias and ReLU; pool is
// the 2^3 mean, up the 2^3 nearest-neighbour copy.  Activations are
// channels-last ([voxel][channel], voxel = ((b S + z) S + y) S + x).
//
// Convolution as an implicit GEMM on v_mfma_f32_16x16x32_bf16: rows are
// voxels, columns output channels, and the reduction runs over chunks of the
// input channels staged in LDS with their halo, and within a chunk over the
// 27 taps and its channels in steps of 32 (8 consecutive channels of one tap
// per lane).  The backward-data pass is the same kernel on
// the output gradient with the taps mirrored and the weight matrix transposed;
// the backward-weight pass reduces over voxels with LDS-transposed tiles and
// float32 atomics.
#include "mgfr_internal.h"
#include "mgfr_ops.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace mgfr {

namespace {

#ifndef MGFR_CONV_WAVES
#define MGFR_CONV_WAVES 4
#endif
#ifndef MGFR_CONV_MT
#define MGFR_CONV_MT 4
#endif
constexpr int kConvWaves = MGFR_CONV_WAVES;  // waves per workgroup in the forward kernel
constexpr int kConvMT = MGFR_CONV_MT;        // 16-voxel row tiles per wave (256 voxels per workgroup)
// LDS stride of a staged voxel: 32-channel chunks get 8 bf16 of padding (the
// 16-byte A-fragment reads of 16 consecutive voxels then spread over the
// banks: 1.4x faster on those layers; 16-channel chunks are faster without)
__host__ __device__ constexpr int conv_stride(int CC) { return CC == 32 ? CC + 8 : CC; }
constexpr float kUScale = 5.0f; // network output = u / kUScale

__device__ __forceinline__ float bf2f(__bf16 x) { return (float)x; }
__device__ __forceinline__ __bf16 f2bf(float x) { return (__bf16)x; }

// -------------------------------------------------------------- convolution

// Y[v][o] = act(sum_{t,c} X[v + off(t)][c] W[t][o][c] + bias[o]) on B periodic S^3
// volumes.  W layout [27][Cout][Cin].  Cin % 8 == 0, Cout % 16 == 0, Cout <= 96, S >= 8.
//
// A workgroup owns a tile of 256 output voxels, TX x 8 x TZ with TX = min(S, 16)
// and TZ = 256 / (8 TX); it stages the tile and a one-voxel periodic halo of
// the input in LDS, CC channels at a time (CC = 32, 16 or 8, dividing Cin),
// so that the 27 taps read the activations from LDS instead of gathering them
// 27 times from global memory.  Each wave computes 4 row tiles of 16 voxels
// against all Cout columns; the weights come from global memory (L2/L1 hits:
// every workgroup reads the same few KB), each k-step's fragments loaded
// while the previous step's MFMAs run.

// NT column tiles of 16 output channels per workgroup, starting at channel
// 16 NT blockIdx.y (a template parameter: the accumulators of the 16-channel
// layers then take 16 registers, not 96; small grids split Cout over
// blockIdx.y to fill the chip)
template <int NT>
__global__ __launch_bounds__(64 * kConvWaves) void k_conv3d(const __bf16 *__restrict__ X, int lgS, int Cin,
                                                             const __bf16 *__restrict__ W,
                                                             const float *__restrict__ bias, int Cout, int relu,
                                                             __bf16 *__restrict__ Y, float *__restrict__ Y32)
{
    extern __shared__ __attribute__((aligned(16))) __bf16 sX[];  // [halo voxels][CC], sized at launch
    __shared__ int sTap[32];  // LDS offset (in voxels) of each tap's neighbour
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int S = 1 << lgS, sm = S - 1;
    const int lgX = lgS < 4 ? lgS : 4;
    const int TX = 1 << lgX, TY = 8, TZ = (16 * kConvMT * kConvWaves) / (TX * TY);
    const int HX = TX + 2, HY = TY + 2, HZ = TZ + 2, HV = HX * HY * HZ;
    unsigned bi = blockIdx.x;
    const int ntx = S / TX, nty = S / TY, ntz = S / TZ;
    const int x0 = (int)(bi % ntx) * TX;
    bi /= ntx;
    const int y0 = (int)(bi % nty) * TY;
    bi /= nty;
    const int z0 = (int)(bi % ntz) * TZ;
    const size_t vol = bi / ntz;
    const int g = lane >> 4, r16 = lane & 15;
    const int ocol0 = 16 * NT * (int)blockIdx.y;
    if (threadIdx.x < 32) {
        const int t = threadIdx.x < 27 ? threadIdx.x : 0;
        sTap[threadIdx.x] = ((t / 9 - 1) * HY + ((t / 3) % 3 - 1)) * HX + (t % 3 - 1);
    }
    // halo-tile voxel of each row this lane feeds to the A operand
    int hb[kConvMT];
#pragma unroll
    for (int mt = 0; mt < kConvMT; ++mt) {
        const int lv = 16 * (w * kConvMT + mt) + r16;
        const int lx = lv & (TX - 1), ly = (lv >> lgX) & (TY - 1), lz = lv >> (lgX + 3);
        hb[mt] = ((lz + 1) * HY + (ly + 1)) * HX + (lx + 1);
    }
    f32x4 acc[kConvMT][NT];
#pragma unroll
    for (int mt = 0; mt < kConvMT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int lgC = (Cin % 32 == 0) ? 5 : ((Cin % 16 == 0) ? 4 : 3);  // chunk CC = 2^lgC channels
    const int CC = 1 << lgC;
    const int q8 = CC >> 3, KC = 27 * CC, CS = conv_stride(CC);
    for (int cc0 = 0; cc0 < Cin; cc0 += CC) {
        __syncthreads();  // the previous chunk's readers are done
        for (int idx = threadIdx.x; idx < HV * q8; idx += 64 * kConvWaves) {
            const int hv = idx / q8, q = idx - hv * q8;
            const int hx = hv % HX, t = hv / HX, hy = t % HY, hz = t / HY;
            const size_t src = ((((vol << lgS) + (size_t)((z0 + hz - 1) & sm)) << (2 * lgS)) +
                                ((size_t)((y0 + hy - 1) & sm) << lgS) + (size_t)((x0 + hx - 1) & sm));
            *(bf16x8 *)(sX + hv * CS + 8 * q) = *(const bf16x8 *)(X + src * Cin + cc0 + 8 * q);
        }
        __syncthreads();
        // weight fragments from global memory, loaded one k-step ahead
        auto loadB = [&](int k0, bf16x8 *b) {
            const int kk = k0 + 8 * g;
            const bool valid = kk < KC;
            const int tap = valid ? kk >> lgC : 0;
            const int c = valid ? kk & (CC - 1) : 0;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                b[nt] = valid ? *(const bf16x8 *)(W + ((size_t)tap * Cout + ocol0 + 16 * nt + r16) * Cin + cc0 + c)
                              : bf16x8{};
        };
        bf16x8 bcur[NT], bnxt[NT] = {};
        loadB(0, bcur);
        for (int k0 = 0; k0 < KC; k0 += 32) {
            if (k0 + 32 < KC) loadB(k0 + 32, bnxt);
            const int kk = k0 + 8 * g;
            const bool valid = kk < KC;
            const int tap = valid ? kk >> lgC : 0;
            const int c = valid ? kk & (CC - 1) : 0;
            const int toff = sTap[tap];
            bf16x8 a[kConvMT];
#pragma unroll
            for (int mt = 0; mt < kConvMT; ++mt)
                a[mt] = valid ? *(const bf16x8 *)(sX + (hb[mt] + toff) * CS + c) : bf16x8{};
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int mt = 0; mt < kConvMT; ++mt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], bcur[nt], acc[mt][nt], 0, 0, 0);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) bcur[nt] = bnxt[nt];
        }
    }
#pragma unroll
    for (int mt = 0; mt < kConvMT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            {
                const int o = ocol0 + 16 * nt + r16;
                const float bo = bias ? bias[o] : 0.f;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int lv = 16 * (w * kConvMT + mt) + 4 * g + j;
                    const int lx = lv & (TX - 1), ly = (lv >> lgX) & (TY - 1), lz = lv >> (lgX + 3);
                    const size_t v = ((((vol << lgS) + (size_t)(z0 + lz)) << lgS) + (size_t)(y0 + ly)) * (size_t)S +
                                      (size_t)(x0 + lx);
                    float val = acc[mt][nt][j] + bo;
                    if (relu) val = fmaxf(val, 0.f);
                    if (Y) Y[v * Cout + o] = f2bf(val);
                    if (Y32) Y32[v * Cout + o] = val;
                }
            }
        }
}

// Launch k_conv3d over nvox = B S^3 voxels (S >= 8, Cout a multiple of 16 up to 96).
void launch_conv3d(const __bf16 *X, size_t nvox, int lgS, int Cin, const __bf16 *W, const float *bias, int Cout,
                   int relu, __bf16 *Y, float *Y32, hipStream_t s)
{
    const unsigned blocks = (unsigned)(nvox / (16 * kConvMT * kConvWaves));
    // LDS: the halo tile ((TX+2) x 10 x (TZ+2) voxels) times the channel chunk (bf16)
    const int TX = lgS < 4 ? (1 << lgS) : 16, TZ = (16 * kConvMT * kConvWaves) / (TX * 8);
    const int CC = (Cin % 32 == 0) ? 32 : ((Cin % 16 == 0) ? 16 : 8);
    const size_t lds = (size_t)(TX + 2) * 10 * (TZ + 2) * conv_stride(CC) * sizeof(__bf16);
    int nt = Cout >> 4, groups = 1;
    // fewer than two workgroups per CU: split the output channels
    while (blocks * groups < 512 && nt % 2 == 0) {
        nt /= 2;
        groups *= 2;
    }
    const dim3 grid(blocks, groups);
    switch (nt) {
    case 1: k_conv3d<1><<<grid, 64 * kConvWaves, lds, s>>>(X, lgS, Cin, W, bias, Cout, relu, Y, Y32); break;
    case 2: k_conv3d<2><<<grid, 64 * kConvWaves, lds, s>>>(X, lgS, Cin, W, bias, Cout, relu, Y, Y32); break;
    case 3: k_conv3d<3><<<grid, 64 * kConvWaves, lds, s>>>(X, lgS, Cin, W, bias, Cout, relu, Y, Y32); break;
    case 4: k_conv3d<4><<<grid, 64 * kConvWaves, lds, s>>>(X, lgS, Cin, W, bias, Cout, relu, Y, Y32); break;
    case 5: k_conv3d<5><<<grid, 64 * kConvWaves, lds, s>>>(X, lgS, Cin, W, bias, Cout, relu, Y, Y32); break;
    default: k_conv3d<6><<<grid, 64 * kConvWaves, lds, s>>>(X, lgS, Cin, W, bias, Cout, relu, Y, Y32); break;
    }
}

// dW[t][o][c] += sum_v dZ[v][o] X[v + off(t)][c];  Cin, Cout % 16 == 0.
// Grid (27, chunks); each workgroup reduces kWChunk voxels for one tap.
constexpr int kWChunk = 2048, kWStage = 64;

__global__ __launch_bounds__(256) void k_conv3d_wgrad(const __bf16 *__restrict__ X, const __bf16 *__restrict__ dZ,
                                                       int lgS, int Cin, int Cout, size_t nvox,
                                                       float *__restrict__ dW)
{
    __shared__ __bf16 sA[96][kWStage + 8];
    __shared__ __bf16 sB[96][kWStage + 8];
    const int tap = blockIdx.x;
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const int S = 1 << lgS, sm = S - 1;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int OT = Cout >> 4, CT = Cin >> 4, ntiles = OT * CT;
    f32x4 acc[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    const size_t vbeg = (size_t)blockIdx.y * kWChunk;
    for (size_t vs = vbeg; vs < vbeg + kWChunk && vs < nvox; vs += kWStage) {
        __syncthreads();
        // stage dZ[vs..vs+63][0..Cout) -> sA[o][v] and X[shifted][0..Cin) -> sB[c][v]
        for (int idx = threadIdx.x; idx < kWStage * Cout; idx += 256) {
            const int v = idx / Cout, o = idx - v * Cout;
            sA[o][v] = dZ[(vs + v) * Cout + o];
        }
        for (int idx = threadIdx.x; idx < kWStage * Cin; idx += 256) {
            const int v = idx / Cin, c = idx - v * Cin;
            const size_t vv = vs + v;
            const int x = (int)(vv & sm), y = (int)((vv >> lgS) & sm), z = (int)((vv >> (2 * lgS)) & sm);
            const size_t b = vv >> (3 * lgS);
            const size_t src = (((b << lgS) + ((z + dz) & sm)) << (2 * lgS)) + ((size_t)((y + dy) & sm) << lgS) +
                               ((x + dx) & sm);
            sB[c][v] = X[src * Cin + c];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int tile = w + 4 * q;
            if (tile < ntiles) {
                const int ot = tile / CT, ct = tile - ot * CT;
#pragma unroll
                for (int kk = 0; kk < kWStage; kk += 32) {
                    bf16x8 a, b;
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        a[j] = sA[16 * ot + r16][kk + 8 * g + j];
                        b[j] = sB[16 * ct + r16][kk + 8 * g + j];
                    }
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[q], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const int tile = w + 4 * q;
        if (tile < ntiles) {
            const int ot = tile / CT, ct = tile - ot * CT;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int o = 16 * ot + 4 * g + j, c = 16 * ct + r16;
                unsafeAtomicAdd(&dW[((size_t)tap * Cout + o) * Cin + c], acc[q][j]);
            }
        }
    }
}

// db[o] += sum_v dZ[v][o]
__global__ __launch_bounds__(256) void k_bias_grad(const __bf16 *__restrict__ dZ, int C, size_t nvox, float *__restrict__ db)
{
    const int o = threadIdx.x % C;
    const int lanes = 256 / C;
    const int sub = threadIdx.x / C;
    if (sub >= lanes) return;
    float s = 0.f;
    for (size_t v = (size_t)blockIdx.x * lanes + sub; v < nvox; v += (size_t)gridDim.x * lanes) s += bf2f(dZ[v * C + o]);
    unsafeAtomicAdd(&db[o], s);
}

// Wt[t'][c][o] = W[26 - t'][o][c]: weights of the backward-data convolution
__global__ void k_wt_transpose(const __bf16 *__restrict__ W, int Cin, int Cout, __bf16 *__restrict__ Wt)
{
    const size_t n = (size_t)27 * Cin * Cout;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int o = (int)(i % Cout);
        const int c = (int)((i / Cout) % Cin);
        const int t = (int)(i / ((size_t)Cout * Cin));
        Wt[i] = W[((size_t)(26 - t) * Cout + o) * Cin + c];
    }
}

// ---------------------------------------------------------------- glue

__global__ void k_features(const double *__restrict__ delta, size_t nvox, int lgS, const float *__restrict__ cond,
                           __bf16 *__restrict__ x0)
{
    for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += (size_t)gridDim.x * blockDim.x) {
        const size_t b = v >> (3 * lgS);
        bf16x8 lo = bf16x8{}, hi = bf16x8{};
        lo[0] = f2bf((float)(asinh(delta[v]) * 0.25));
        lo[1] = f2bf(cond[2 * b + 0]);
        lo[2] = f2bf(cond[2 * b + 1]);
        *(bf16x8 *)(x0 + v * 16) = lo;
        *(bf16x8 *)(x0 + v * 16 + 8) = hi;
    }
}

// 2^3 mean: out has side S/2 (lgS of the output)
__global__ void k_pool(const __bf16 *__restrict__ in, int lgSo, int C, size_t nout, __bf16 *__restrict__ out)
{
    const int So = 1 << lgSo, sm = So - 1, lgSi = lgSo + 1;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nout * C; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const size_t v = i / C;
        const int x = (int)(v & sm), y = (int)((v >> lgSo) & sm), z = (int)((v >> (2 * lgSo)) & sm);
        const size_t b = v >> (3 * lgSo);
        float s = 0.f;
        for (int a = 0; a < 8; ++a) {
            const size_t src = (((b << lgSi) + (2 * z + (a >> 2))) << (2 * lgSi)) + ((size_t)(2 * y + ((a >> 1) & 1)) << lgSi) +
                               (2 * x + (a & 1));
            s += bf2f(in[src * C + c]);
        }
        out[i] = f2bf(0.125f * s);
    }
}

// out[v] = concat(in[parent(v)] (Cu channels), skip[v] (Cs channels)): the
// nearest-neighbour upsampling and the skip connection of one decoder level in
// one pass, 8 channels (16 bytes) per thread; Cu, Cs multiples of 8
__global__ void k_concat_up(const __bf16 *__restrict__ in, int Cu, const __bf16 *__restrict__ skip, int Cs,
                            int lgSo, size_t nout, __bf16 *__restrict__ out)
{
    const int sm = (1 << lgSo) - 1, lgSi = lgSo - 1, q8 = (Cu + Cs) >> 3, qu = Cu >> 3;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nout * q8; i += (size_t)gridDim.x * blockDim.x) {
        const size_t v = i / q8;
        const int q = (int)(i - v * q8);
        bf16x8 val;
        if (q < qu) {
            const int x = (int)(v & sm), y = (int)((v >> lgSo) & sm), z = (int)((v >> (2 * lgSo)) & sm);
            const size_t b = v >> (3 * lgSo);
            const size_t src = (((b << lgSi) + (z >> 1)) << (2 * lgSi)) + ((size_t)(y >> 1) << lgSi) + (x >> 1);
            val = *(const bf16x8 *)(in + src * Cu + 8 * q);
        } else {
            val = *(const bf16x8 *)(skip + v * Cs + 8 * (q - qu));
        }
        *(bf16x8 *)(out + i * 8) = val;
    }
}

// d_in[parent][c] = sum_children d_out[child][off + c]
__global__ void k_upsample_bwd(const __bf16 *__restrict__ dout, int lgSi, int C, size_t nin, int Ctot, int off,
                               __bf16 *__restrict__ din)
{
    const int Si = 1 << lgSi, sm = Si - 1, lgSo = lgSi + 1;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nin * C; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const size_t v = i / C;
        const int x = (int)(v & sm), y = (int)((v >> lgSi) & sm), z = (int)((v >> (2 * lgSi)) & sm);
        const size_t b = v >> (3 * lgSi);
        float s = 0.f;
        for (int a = 0; a < 8; ++a) {
            const size_t src = (((b << lgSo) + (2 * z + (a >> 2))) << (2 * lgSo)) + ((size_t)(2 * y + ((a >> 1) & 1)) << lgSo) +
                               (2 * x + (a & 1));
            s += bf2f(dout[src * Ctot + off + c]);
        }
        din[i] = f2bf(s);
    }
}

// skip-connection gradient: d_skip[v][c] = d_cat[v][off + c] + d_pool[parent(v)][c] / 8
__global__ void k_skip_grad(const __bf16 *__restrict__ dcat, int Ctot, int off, const __bf16 *__restrict__ dpool,
                            int lgS, int C, size_t nvox, __bf16 *__restrict__ dskip)
{
    const int S = 1 << lgS, sm = S - 1, lgP = lgS - 1;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvox * C; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const size_t v = i / C;
        const int x = (int)(v & sm), y = (int)((v >> lgS) & sm), z = (int)((v >> (2 * lgS)) & sm);
        const size_t b = v >> (3 * lgS);
        const size_t par = (((b << lgP) + (z >> 1)) << (2 * lgP)) + ((size_t)(y >> 1) << lgP) + (x >> 1);
        dskip[i] = f2bf(bf2f(dcat[v * Ctot + off + c]) + 0.125f * bf2f(dpool[par * C + c]));
    }
}

// dz = dy * (y > 0), reading dy from channels [off, off + C) of a Ctot-channel tensor
__global__ void k_relu_bwd(const __bf16 *__restrict__ dy, int Ctot, int off, const __bf16 *__restrict__ y, size_t nvox,
                           int C, __bf16 *__restrict__ dz)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvox * C; i += (size_t)gridDim.x * blockDim.x) {
        const size_t v = i / C;
        const int c = (int)(i % C);
        dz[i] = bf2f(y[i]) > 0.f ? dy[v * Ctot + off + c] : f2bf(0.f);
    }
}

// 1x1 head: y[v] = sum_c h[v][c] wh[c] + bh
__global__ void k_head(const __bf16 *__restrict__ h, size_t nvox, const float *__restrict__ wh, float *__restrict__ y)
{
    for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += (size_t)gridDim.x * blockDim.x) {
        float s = wh[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) s += bf2f(h[v * 16 + c]) * wh[c];
        y[v] = s;
    }
}

// loss = mean (y - u/kUScale)^2 accumulated into loss[0]; dy = 2 (y - t) / n
__global__ __launch_bounds__(256) void k_loss(const float *__restrict__ y, const double *__restrict__ u, size_t n,
                                               float *__restrict__ dy, float *__restrict__ loss)
{
    float s = 0.f;
    for (size_t v = (size_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (size_t)gridDim.x * 256) {
        const float d = y[v] - (float)u[v] / kUScale;
        dy[v] = 2.f * d / (float)n;
        s += d * d;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) unsafeAtomicAdd(loss, s / (float)n);
}

// head backward: dh[v][c] = dy[v] wh[c]; dwh[c] += sum_v dy[v] h[v][c]; dbh += sum dy
__global__ __launch_bounds__(256) void k_head_bwd(const __bf16 *__restrict__ h, const float *__restrict__ dy, size_t n,
                                                   const float *__restrict__ wh, __bf16 *__restrict__ dh,
                                                   float *__restrict__ dwh)
{
    float s[17];
#pragma unroll
    for (int c = 0; c < 17; ++c) s[c] = 0.f;
    for (size_t v = (size_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (size_t)gridDim.x * 256) {
        const float d = dy[v];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            s[c] += d * bf2f(h[v * 16 + c]);
            dh[v * 16 + c] = f2bf(d * wh[c]);
        }
        s[16] += d;
    }
#pragma unroll
    for (int c = 0; c < 17; ++c) {
        float x = s[c];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if ((threadIdx.x & 63) == 0) unsafeAtomicAdd(&dwh[c], x);
    }
}

__global__ void k_to_u(const float *__restrict__ y, size_t n, double *__restrict__ u)
{
    for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x)
        u[v] = (double)(y[v] * kUScale);
}

// Adam on float32 master weights (bias-corrected; t = step count >= 1)
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ gr, float *__restrict__ m, float *__restrict__ v,
                       size_t n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = gr[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

__global__ void k_to_bf16(const float *__restrict__ p, size_t n, __bf16 *__restrict__ o)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        o[i] = f2bf(p[i]);
}

__global__ void k_restrict4(const double *__restrict__ fine, int lgc, double *__restrict__ coarse)
{
    const int Nc = 1 << lgc, lgf = lgc + 2;
    const size_t n = (size_t)Nc * Nc * Nc;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const int K = (int)(t & (Nc - 1)), J = (int)((t >> lgc) & (Nc - 1)), I = (int)(t >> (2 * lgc));
        double s = 0.0;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                for (int c = 0; c < 4; ++c) s += fine[cidx(4 * I + a, 4 * J + b, 4 * K + c, lgf)];
        coarse[t] = s / 64.0;
    }
}

// coarse = mean of the 8 daughters (the restriction of Sec. 3.3) of a float64 field
__global__ void k_restrict_mean(const double *__restrict__ fine, int lgc, double *__restrict__ coarse)
{
    const int Nc = 1 << lgc, lgf = lgc + 1;
    const size_t n = (size_t)Nc * Nc * Nc;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const int K = (int)(t & (Nc - 1)), J = (int)((t >> lgc) & (Nc - 1)), I = (int)(t >> (2 * lgc));
        double s = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c) s += fine[cidx(2 * I + a, 2 * J + b, 2 * K + c, lgf)];
        coarse[t] = s * 0.125;
    }
}

// u = P(uc) on the finer mesh: the linear reconstruction (parent value plus
// the central-difference gradient, Sec. 3.3), stored (no clearing pass)
__global__ __launch_bounds__(kBlock) void k_prolong_field_set(double *__restrict__ u, const double *__restrict__ uc,
                                                                int lgc)
{
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int K = (int)(t & ((1u << lgc) - 1)), J = (int)((t >> lgc) & ((1u << lgc) - 1)), I = (int)(t >> (2 * lgc));
    const int m = (1 << lgc) - 1, lg = lgc + 1;
    const double v0 = uc[cidx(I, J, K, lgc)];
    const double gx = uc[cidx((I + 1) & m, J, K, lgc)] - uc[cidx((I - 1) & m, J, K, lgc)];
    const double gy = uc[cidx(I, (J + 1) & m, K, lgc)] - uc[cidx(I, (J - 1) & m, K, lgc)];
    const double gz = uc[cidx(I, J, (K + 1) & m, lgc)] - uc[cidx(I, J, (K - 1) & m, lgc)];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                double v = v0;
                v += (a ? 0.125 : -0.125) * gx;
                v += (b ? 0.125 : -0.125) * gy;
                v += (c ? 0.125 : -0.125) * gz;
                u[cidx(2 * I + a, 2 * J + b, 2 * K + c, lg)] = v;
            }
}

inline unsigned gridn(size_t n, unsigned cap = 16384) { return (unsigned)std::min<size_t>((n + 255) / 256, cap); }

}  // namespace

}  // namespace mgfr

using namespace mgfr;

// ================================================================ network

namespace {

struct ConvSpec {
    int cin, cout;
    size_t woff, boff;  // offsets into the parameter vector
};

// layer order: c1a c1b c2a c2b c3a c3b c4a c4b c5a c5b, then the head (16 weights + bias)
const int kLayerCin[10] = {16, 16, 16, 32, 32, 64, 96, 32, 48, 16};
const int kLayerCout[10] = {16, 16, 32, 32, 64, 64, 32, 32, 16, 16};

}  // namespace

struct mgfr_net {
    hipStream_t stream = nullptr;
    size_t maxvox = 0;
    ConvSpec L[10];
    size_t nparam = 0, head_off = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // master, grad, Adam moments
    __bf16 *wbf = nullptr;   // bf16 copy of every parameter (conv weights used in [t][o][c] layout)
    __bf16 *wt = nullptr;    // transposed, mirrored conv weights for backward-data (same offsets)
    int step = 0;
    int fwd_B = 0, fwd_lg = 0;  // shape of the last forward pass (0: none yet)
    // activations
    __bf16 *x0, *h1a, *s1, *p1, *h2a, *s2, *p2, *h3a, *h3, *cat4, *h4a, *h4, *cat5, *h5a, *h5;
    float *y32, *dy32, *cond, *loss;
    // gradient scratch
    __bf16 *gA, *gB, *gC, *gD;
    float *hcond = nullptr, *hloss = nullptr;
};

namespace {

int net_alloc(mgfr_net *n)
{
    size_t off = 0;
    for (int i = 0; i < 10; ++i) {
        n->L[i].cin = kLayerCin[i];
        n->L[i].cout = kLayerCout[i];
        n->L[i].woff = off;
        off += (size_t)27 * kLayerCin[i] * kLayerCout[i];
        n->L[i].boff = off;
        off += kLayerCout[i];
    }
    n->head_off = off;
    off += 17;
    n->nparam = off;
    const size_t P = n->nparam;
    MGFR_HIP(hipMalloc(&n->p, P * sizeof(float)));
    MGFR_HIP(hipMalloc(&n->g, P * sizeof(float)));
    MGFR_HIP(hipMalloc(&n->m, P * sizeof(float)));
    MGFR_HIP(hipMalloc(&n->v, P * sizeof(float)));
    MGFR_HIP(hipMalloc(&n->wbf, P * sizeof(__bf16)));
    MGFR_HIP(hipMalloc(&n->wt, P * sizeof(__bf16)));
    const size_t V = n->maxvox, V2 = V / 8, V3 = V / 64;
    auto A = [&](__bf16 **ptr, size_t elems) -> int {
        MGFR_HIP(hipMalloc(ptr, elems * sizeof(__bf16)));
        return MGFR_OK;
    };
    int rc;
    if ((rc = A(&n->x0, V * 16)) || (rc = A(&n->h1a, V * 16)) || (rc = A(&n->s1, V * 16)) ||
        (rc = A(&n->p1, V2 * 16)) || (rc = A(&n->h2a, V2 * 32)) || (rc = A(&n->s2, V2 * 32)) ||
        (rc = A(&n->p2, V3 * 32)) || (rc = A(&n->h3a, V3 * 64)) || (rc = A(&n->h3, V3 * 64)) ||
        (rc = A(&n->cat4, V2 * 96)) || (rc = A(&n->h4a, V2 * 32)) || (rc = A(&n->h4, V2 * 32)) ||
        (rc = A(&n->cat5, V * 48)) || (rc = A(&n->h5a, V * 16)) || (rc = A(&n->h5, V * 16)) ||
        (rc = A(&n->gA, V * 48)) || (rc = A(&n->gB, V * 48)) || (rc = A(&n->gC, V * 16)) || (rc = A(&n->gD, V * 16)))
        return rc;
    MGFR_HIP(hipMalloc(&n->y32, V * sizeof(float)));
    MGFR_HIP(hipMalloc(&n->dy32, V * sizeof(float)));
    MGFR_HIP(hipMalloc(&n->cond, 2 * 4096 * sizeof(float)));
    MGFR_HIP(hipMalloc(&n->loss, sizeof(float)));
    MGFR_HIP(hipHostMalloc(&n->hcond, 2 * 4096 * sizeof(float), hipHostMallocDefault));
    MGFR_HIP(hipHostMalloc(&n->hloss, sizeof(float), hipHostMallocDefault));
    return MGFR_OK;
}

void net_free(mgfr_net *n)
{
    if (!n) return;
    void *ptrs[] = {n->p, n->g, n->m, n->v, n->wbf, n->wt, n->x0, n->h1a, n->s1, n->p1, n->h2a, n->s2, n->p2,
                    n->h3a, n->h3, n->cat4, n->h4a, n->h4, n->cat5, n->h5a, n->h5, n->gA, n->gB, n->gC, n->gD,
                    n->y32, n->dy32, n->cond, n->loss};
    for (void *q : ptrs) (void)hipFree(q);
    if (n->hcond) (void)hipHostFree(n->hcond);
    if (n->hloss) (void)hipHostFree(n->hloss);
    delete n;
}

// refresh the bf16 weights and the backward-data copies from the master weights
int net_refresh(mgfr_net *n)
{
    k_to_bf16<<<gridn(n->nparam), 256, 0, n->stream>>>(n->p, n->nparam, n->wbf);
    for (int i = 0; i < 10; ++i)
        k_wt_transpose<<<gridn((size_t)27 * n->L[i].cin * n->L[i].cout), 256, 0, n->stream>>>(
            n->wbf + n->L[i].woff, n->L[i].cin, n->L[i].cout, n->wt + n->L[i].woff);
    MGFR_HIP(hipGetLastError());
    return MGFR_OK;
}

int conv(mgfr_net *n, const __bf16 *x, size_t nvox, int lgS, int layer, bool relu, __bf16 *y)
{
    const ConvSpec &L = n->L[layer];
    launch_conv3d(x, nvox, lgS, L.cin, n->wbf + L.woff, n->p + L.boff, L.cout, relu ? 1 : 0, y, nullptr, n->stream);
    MGFR_HIP(hipGetLastError());
    return MGFR_OK;
}

// Backward through one conv+ReLU layer: dy (channels [off, off+Cout) of a Ctot tensor),
// its output y and input x; accumulates weight/bias gradients, writes dx if non-null.
int conv_bwd(mgfr_net *n, const __bf16 *dy, int Ctot, int off, const __bf16 *y, const __bf16 *x, size_t nvox, int lgS,
             int layer, __bf16 *dz_scratch, __bf16 *dx)
{
    const ConvSpec &L = n->L[layer];
    k_relu_bwd<<<gridn(nvox * L.cout), 256, 0, n->stream>>>(dy, Ctot, off, y, nvox, L.cout, dz_scratch);
    const unsigned chunks = (unsigned)((nvox + kWChunk - 1) / kWChunk);
    k_conv3d_wgrad<<<dim3(27, chunks), 256, 0, n->stream>>>(x, dz_scratch, lgS, L.cin, L.cout, nvox, n->g + L.woff);
    k_bias_grad<<<gridn(nvox, 1024), 256, 0, n->stream>>>(dz_scratch, L.cout, nvox, n->g + L.boff);
    if (dx) {
        launch_conv3d(dz_scratch, nvox, lgS, L.cout, n->wt + L.woff, nullptr, L.cin, 0, dx, nullptr, n->stream);
    }
    MGFR_HIP(hipGetLastError());
    return MGFR_OK;
}

int net_forward(mgfr_net *n, const double *delta, int B, int lgS)
{
    const size_t V = (size_t)B << (3 * lgS), V2 = V / 8, V3 = V / 64;
    int rc;
    n->fwd_B = B;
    n->fwd_lg = lgS;
    MGFR_HIP(hipMemcpyAsync(n->cond, n->hcond, 2 * B * sizeof(float), hipMemcpyHostToDevice, n->stream));
    k_features<<<gridn(V), 256, 0, n->stream>>>(delta, V, lgS, n->cond, n->x0);
    if ((rc = conv(n, n->x0, V, lgS, 0, true, n->h1a)) || (rc = conv(n, n->h1a, V, lgS, 1, true, n->s1))) return rc;
    k_pool<<<gridn(V2 * 16), 256, 0, n->stream>>>(n->s1, lgS - 1, 16, V2, n->p1);
    if ((rc = conv(n, n->p1, V2, lgS - 1, 2, true, n->h2a)) || (rc = conv(n, n->h2a, V2, lgS - 1, 3, true, n->s2)))
        return rc;
    k_pool<<<gridn(V3 * 32), 256, 0, n->stream>>>(n->s2, lgS - 2, 32, V3, n->p2);
    if ((rc = conv(n, n->p2, V3, lgS - 2, 4, true, n->h3a)) || (rc = conv(n, n->h3a, V3, lgS - 2, 5, true, n->h3)))
        return rc;
    k_concat_up<<<gridn(V2 * 12), 256, 0, n->stream>>>(n->h3, 64, n->s2, 32, lgS - 1, V2, n->cat4);
    if ((rc = conv(n, n->cat4, V2, lgS - 1, 6, true, n->h4a)) || (rc = conv(n, n->h4a, V2, lgS - 1, 7, true, n->h4)))
        return rc;
    k_concat_up<<<gridn(V * 6), 256, 0, n->stream>>>(n->h4, 32, n->s1, 16, lgS, V, n->cat5);
    if ((rc = conv(n, n->cat5, V, lgS, 8, true, n->h5a)) || (rc = conv(n, n->h5a, V, lgS, 9, true, n->h5))) return rc;
    k_head<<<gridn(V), 256, 0, n->stream>>>(n->h5, V, n->p + n->head_off, n->y32);
    MGFR_HIP(hipGetLastError());
    return MGFR_OK;
}

int net_backward(mgfr_net *n, int B, int lgS)
{
    const size_t V = (size_t)B << (3 * lgS), V2 = V / 8, V3 = V / 64;
    int rc;
    MGFR_HIP(hipMemsetAsync(n->g, 0, n->nparam * sizeof(float), n->stream));
    // head
    k_head_bwd<<<gridn(V, 2048), 256, 0, n->stream>>>(n->h5, n->dy32, V, n->p + n->head_off, n->gC, n->g + n->head_off);
    // level 1 decoder: c5b (dy = gC) -> d(h5a) in gD; c5a -> d(cat5) in gA [V][48]
    if ((rc = conv_bwd(n, n->gC, 16, 0, n->h5, n->h5a, V, lgS, 9, n->gB, n->gD))) return rc;
    if ((rc = conv_bwd(n, n->gD, 16, 0, n->h5a, n->cat5, V, lgS, 8, n->gB, n->gA))) return rc;
    // d(h4) = sum over children of d(cat5)[:, 0:32]  -> gB [V2][32]
    k_upsample_bwd<<<gridn(V2 * 32), 256, 0, n->stream>>>(n->gA, lgS - 1, 32, V2, 48, 0, n->gB);
    // keep d(cat5)[:, 32:48] (the s1 part): copy into gD [V][16]
    // (k_skip_grad below combines it with the pooled gradient later)
    // level 2 decoder: c4b (dy = gB) -> d(h4a) in gC ; c4a -> d(cat4) in gB?  use separate buffers
    // gC holds [V2][32]; d(cat4) [V2][96] goes to gD? gD is [V][16] >= V2*96 when V >= 48 V2 ... use gB region after
    if ((rc = conv_bwd(n, n->gB, 32, 0, n->h4, n->h4a, V2, lgS - 1, 7, n->gC + 0, n->gD))) return rc;  // dz in gC, d(h4a) in gD
    // c4a: dy = gD [V2][32]; dz scratch gC; d(cat4) -> gB [V2][96] (gB has V*48 >= V2*96 elements)
    if ((rc = conv_bwd(n, n->gD, 32, 0, n->h4a, n->cat4, V2, lgS - 1, 6, n->gC, n->gB))) return rc;
    // d(h3) = sum over children of d(cat4)[:, 0:64] -> gC [V3][64]
    k_upsample_bwd<<<gridn(V3 * 64), 256, 0, n->stream>>>(n->gB, lgS - 2, 64, V3, 96, 0, n->gC);
    // level 3: c3b (dy = gC) -> d(h3a) in gD ; c3a -> d(p2) in gC
    __bf16 *dz3 = n->gD + V3 * 64;  // scratch after d(h3a)
    if ((rc = conv_bwd(n, n->gC, 64, 0, n->h3, n->h3a, V3, lgS - 2, 5, dz3, n->gD))) return rc;
    if ((rc = conv_bwd(n, n->gD, 64, 0, n->h3a, n->p2, V3, lgS - 2, 4, dz3, n->gC))) return rc;
    // d(s2) = d(cat4)[:, 64:96] + d(p2)/8 -> gD [V2][32]
    k_skip_grad<<<gridn(V2 * 32), 256, 0, n->stream>>>(n->gB, 96, 64, n->gC, lgS - 1, 32, V2, n->gD);
    // level 2 encoder: c2b (dy = gD) -> d(h2a) in gC ; c2a -> d(p1) in gD
    __bf16 *dz2 = n->gB;  // d(cat4) no longer needed
    if ((rc = conv_bwd(n, n->gD, 32, 0, n->s2, n->h2a, V2, lgS - 1, 3, dz2, n->gC))) return rc;
    if ((rc = conv_bwd(n, n->gC, 32, 0, n->h2a, n->p1, V2, lgS - 1, 2, dz2, n->gD))) return rc;
    // d(s1) = d(cat5)[:, 32:48] + d(p1)/8 -> gC [V][16]
    k_skip_grad<<<gridn(V * 16), 256, 0, n->stream>>>(n->gA, 48, 32, n->gD, lgS, 16, V, n->gC);
    // level 1 encoder: c1b (dy = gC) -> d(h1a) in gD ; c1a (no input gradient)
    if ((rc = conv_bwd(n, n->gC, 16, 0, n->s1, n->h1a, V, lgS, 1, n->gB, n->gD))) return rc;
    if ((rc = conv_bwd(n, n->gD, 16, 0, n->h1a, n->x0, V, lgS, 0, n->gB, nullptr))) return rc;
    MGFR_HIP(hipGetLastError());
    return MGFR_OK;
}

int check_shape(const mgfr_net *n, int B, int S, int *lgS)
{
    if (B < 1 || S < 32 || S > 1024 || (S & (S - 1)))
        return set_error(MGFR_ERR_ARG, "network inputs need B >= 1 and a power-of-two side 32 <= S <= 1024");
    int lg = 0;
    while ((1 << lg) < S) ++lg;
    if (((size_t)B << (3 * lg)) > n->maxvox) return set_error(MGFR_ERR_ARG, "B * S^3 exceeds the network's capacity");
    if (B > 4096) return set_error(MGFR_ERR_ARG, "B must be <= 4096");
    *lgS = lg;
    return MGFR_OK;
}

void set_cond(mgfr_net *n, const double *cond, int B)
{
    for (int b = 0; b < B; ++b) {
        n->hcond[2 * b + 0] = (float)((cond[2 * b + 0] - 0.75) * 4.0);
        n->hcond[2 * b + 1] = (float)((std::log10(cond[2 * b + 1]) + 5.5) / 1.5);
    }
}

}  // namespace

extern "C" int mgfr_net_create(int seed, int64_t max_voxels, void *stream, mgfr_net **out)
{
    if (!out) return set_error(MGFR_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (max_voxels < 4096 || max_voxels % 4096) return set_error(MGFR_ERR_ARG, "max_voxels must be a positive multiple of 4096");
    mgfr_net *n = new (std::nothrow) mgfr_net();
    if (!n) return set_error(MGFR_ERR_OOM, "host allocation failed");
    n->stream = (hipStream_t)stream;
    n->maxvox = (size_t)max_voxels;
    int rc = net_alloc(n);
    if (rc) {
        net_free(n);
        return rc;
    }
    // He-normal initialisation from a seeded generator, zero biases
    std::vector<float> h(n->nparam, 0.f);
    std::mt19937_64 gen((uint64_t)seed);
    for (int i = 0; i < 10; ++i) {
        std::normal_distribution<float> d(0.f, std::sqrt(2.f / (27.f * n->L[i].cin)));
        for (size_t k = 0; k < (size_t)27 * n->L[i].cin * n->L[i].cout; ++k) h[n->L[i].woff + k] = d(gen);
    }
    std::normal_distribution<float> dh(0.f, std::sqrt(1.f / 16.f));
    for (int c = 0; c < 16; ++c) h[n->head_off + c] = dh(gen);
    hipError_t e = hipMemcpy(n->p, h.data(), n->nparam * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(n->m, 0, n->nparam * sizeof(float));
    if (e == hipSuccess) e = hipMemset(n->v, 0, n->nparam * sizeof(float));
    if (e != hipSuccess) {
        net_free(n);
        return hip_fail(e, "network initialisation", __FILE__, __LINE__);
    }
    if ((rc = net_refresh(n))) {
        net_free(n);
        return rc;
    }
    *out = n;
    return MGFR_OK;
}

extern "C" void mgfr_net_destroy(mgfr_net *n) { net_free(n); }

extern "C" int mgfr_net_set_stream(mgfr_net *n, void *stream)
{
    if (!n) return set_error(MGFR_ERR_ARG, "net is NULL");
    n->stream = (hipStream_t)stream;
    return MGFR_OK;
}

extern "C" int64_t mgfr_net_num_params(const mgfr_net *n) { return n ? (int64_t)n->nparam : -1; }

extern "C" int mgfr_net_get_params(mgfr_net *n, float *host)
{
    if (!n || !host) return set_error(MGFR_ERR_ARG, "net and host must be non-NULL");
    MGFR_HIP(hipMemcpyAsync(host, n->p, n->nparam * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    MGFR_HIP(hipStreamSynchronize(n->stream));
    return MGFR_OK;
}

extern "C" int mgfr_net_set_params(mgfr_net *n, const float *host)
{
    if (!n || !host) return set_error(MGFR_ERR_ARG, "net and host must be non-NULL");
    MGFR_HIP(hipMemcpyAsync(n->p, host, n->nparam * sizeof(float), hipMemcpyHostToDevice, n->stream));
    MGFR_HIP(hipMemsetAsync(n->m, 0, n->nparam * sizeof(float), n->stream));
    MGFR_HIP(hipMemsetAsync(n->v, 0, n->nparam * sizeof(float), n->stream));
    n->step = 0;
    int rc = net_refresh(n);
    if (rc) return rc;
    MGFR_HIP(hipStreamSynchronize(n->stream));
    return MGFR_OK;
}

// Checkpoint file: 8-byte tag "MGFRNET1", int64 parameter count, int32 Adam
// step, int32 layer count (10) and each layer's (Cin, Cout) as int32, then the
// float32 master parameters, Adam first and second moments (native byte order).
namespace {
constexpr char kNetTag[8] = {'M', 'G', 'F', 'R', 'N', 'E', 'T', '1'};
}

extern "C" int mgfr_net_save(mgfr_net *n, const char *path)
{
    if (!n || !path) return set_error(MGFR_ERR_ARG, "net and path must be non-NULL");
    const size_t P = n->nparam;
    std::vector<float> buf(3 * P);
    MGFR_HIP(hipMemcpyAsync(buf.data(), n->p, P * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    MGFR_HIP(hipMemcpyAsync(buf.data() + P, n->m, P * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    MGFR_HIP(hipMemcpyAsync(buf.data() + 2 * P, n->v, P * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    MGFR_HIP(hipStreamSynchronize(n->stream));
    FILE *f = fopen(path, "wb");
    if (!f) return set_error(MGFR_ERR_ARG, "cannot open %s for writing", path);
    const int64_t np = (int64_t)P;
    int32_t hdr[2 + 20];
    hdr[0] = n->step;
    hdr[1] = 10;
    for (int i = 0; i < 10; ++i) {
        hdr[2 + 2 * i] = n->L[i].cin;
        hdr[3 + 2 * i] = n->L[i].cout;
    }
    const bool ok = fwrite(kNetTag, 1, 8, f) == 8 && fwrite(&np, sizeof np, 1, f) == 1 &&
                    fwrite(hdr, sizeof hdr, 1, f) == 1 && fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    if (fclose(f) != 0 || !ok) return set_error(MGFR_ERR_ARG, "writing %s failed", path);
    return MGFR_OK;
}

extern "C" int mgfr_net_load(mgfr_net *n, const char *path)
{
    if (!n || !path) return set_error(MGFR_ERR_ARG, "net and path must be non-NULL");
    FILE *f = fopen(path, "rb");
    if (!f) return set_error(MGFR_ERR_ARG, "cannot open %s", path);
    char tag[8];
    int64_t np = 0;
    int32_t hdr[2 + 20];
    const size_t P = n->nparam;
    std::vector<float> buf(3 * P);
    bool ok = fread(tag, 1, 8, f) == 8 && memcmp(tag, kNetTag, 8) == 0 && fread(&np, sizeof np, 1, f) == 1 &&
              np == (int64_t)P && fread(hdr, sizeof hdr, 1, f) == 1 && hdr[1] == 10;
    for (int i = 0; ok && i < 10; ++i) ok = hdr[2 + 2 * i] == n->L[i].cin && hdr[3 + 2 * i] == n->L[i].cout;
    ok = ok && fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    fclose(f);
    if (!ok) return set_error(MGFR_ERR_ARG, "%s is not a checkpoint of this network", path);
    MGFR_HIP(hipMemcpyAsync(n->p, buf.data(), P * sizeof(float), hipMemcpyHostToDevice, n->stream));
    MGFR_HIP(hipMemcpyAsync(n->m, buf.data() + P, P * sizeof(float), hipMemcpyHostToDevice, n->stream));
    MGFR_HIP(hipMemcpyAsync(n->v, buf.data() + 2 * P, P * sizeof(float), hipMemcpyHostToDevice, n->stream));
    n->step = hdr[0];
    int rc = net_refresh(n);
    if (rc) return rc;
    MGFR_HIP(hipStreamSynchronize(n->stream));
    return MGFR_OK;
}

extern "C" int mgfr_net_predict(mgfr_net *n, const double *delta, int B, int S, const double *cond, double *u)
{
    if (!n || !delta || !cond || !u) return set_error(MGFR_ERR_ARG, "net, delta, cond and u must be non-NULL");
    int lgS, rc;
    if ((rc = check_shape(n, B, S, &lgS))) return rc;
    set_cond(n, cond, B);
    if ((rc = net_forward(n, delta, B, lgS))) return rc;
    const size_t V = (size_t)B << (3 * lgS);
    k_to_u<<<gridn(V), 256, 0, n->stream>>>(n->y32, V, u);
    MGFR_HIP(hipGetLastError());
    MGFR_HIP(hipStreamSynchronize(n->stream));
    return MGFR_OK;
}

extern "C" int mgfr_net_activation(mgfr_net *n, int index, void *dst, int64_t count)
{
    if (!n || !dst) return set_error(MGFR_ERR_ARG, "net and dst must be non-NULL");
    if (index < 0 || index > 15) return set_error(MGFR_ERR_ARG, "activation index must be in [0, 15]");
    if (n->fwd_B == 0) return set_error(MGFR_ERR_ARG, "no forward pass has run on this network yet");
    // buffer, channels and pooling depth (0: S^3, 1: (S/2)^3, 2: (S/4)^3) in forward order
    const __bf16 *buf[15] = {n->x0, n->h1a, n->s1, n->p1, n->h2a, n->s2, n->p2, n->h3a,
                             n->h3, n->cat4, n->h4a, n->h4, n->cat5, n->h5a, n->h5};
    static const int ch[16] = {16, 16, 16, 16, 32, 32, 32, 64, 64, 96, 32, 32, 48, 16, 16, 1};
    static const int depth[16] = {0, 0, 0, 1, 1, 1, 2, 2, 2, 1, 1, 1, 0, 0, 0, 0};
    const size_t vox = ((size_t)n->fwd_B << (3 * n->fwd_lg)) >> (3 * depth[index]);
    const size_t elems = vox * ch[index];
    if (count != (int64_t)elems) return set_error(MGFR_ERR_ARG, "count does not match the activation's size");
    const void *src = index == 15 ? (const void *)n->y32 : (const void *)buf[index];
    const size_t esz = index == 15 ? sizeof(float) : sizeof(__bf16);
    MGFR_HIP(hipMemcpyAsync(dst, src, elems * esz, hipMemcpyDeviceToDevice, n->stream));
    MGFR_HIP(hipStreamSynchronize(n->stream));
    return MGFR_OK;
}

extern "C" int mgfr_net_train_step(mgfr_net *n, const double *delta, const double *u_target, int B, int S,
                                   const double *cond, float lr, float *loss)
{
    if (!n || !delta || !u_target || !cond) return set_error(MGFR_ERR_ARG, "net, delta, u_target and cond must be non-NULL");
    if (!(lr > 0.f)) return set_error(MGFR_ERR_ARG, "lr must be > 0");
    int lgS, rc;
    if ((rc = check_shape(n, B, S, &lgS))) return rc;
    set_cond(n, cond, B);
    if ((rc = net_forward(n, delta, B, lgS))) return rc;
    const size_t V = (size_t)B << (3 * lgS);
    MGFR_HIP(hipMemsetAsync(n->loss, 0, sizeof(float), n->stream));
    k_loss<<<gridn(V, 2048), 256, 0, n->stream>>>(n->y32, u_target, V, n->dy32, n->loss);
    if ((rc = net_backward(n, B, lgS))) return rc;
    n->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)n->step), c2 = 1.f - std::pow(b2, (float)n->step);
    k_adam<<<gridn(n->nparam), 256, 0, n->stream>>>(n->p, n->g, n->m, n->v, n->nparam, lr, b1, b2, 1e-8f, c1, c2);
    if ((rc = net_refresh(n))) return rc;
    MGFR_HIP(hipMemcpyAsync(n->hloss, n->loss, sizeof(float), hipMemcpyDeviceToHost, n->stream));
    MGFR_HIP(hipStreamSynchronize(n->stream));
    if (loss) *loss = *n->hloss;
    if (!std::isfinite(*n->hloss)) return set_error(MGFR_ERR_NONFINITE, "training loss is not finite");
    return MGFR_OK;
}

extern "C" int mgfr_net_grads(mgfr_net *n, const double *delta, const double *u_target, int B, int S,
                              const double *cond, float *loss, float *grad_host)
{
    if (!n || !delta || !u_target || !cond || !grad_host) return set_error(MGFR_ERR_ARG, "null argument");
    int lgS, rc;
    if ((rc = check_shape(n, B, S, &lgS))) return rc;
    set_cond(n, cond, B);
    if ((rc = net_forward(n, delta, B, lgS))) return rc;
    const size_t V = (size_t)B << (3 * lgS);
    MGFR_HIP(hipMemsetAsync(n->loss, 0, sizeof(float), n->stream));
    k_loss<<<gridn(V, 2048), 256, 0, n->stream>>>(n->y32, u_target, V, n->dy32, n->loss);
    if ((rc = net_backward(n, B, lgS))) return rc;
    MGFR_HIP(hipMemcpyAsync(grad_host, n->g, n->nparam * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    MGFR_HIP(hipMemcpyAsync(n->hloss, n->loss, sizeof(float), hipMemcpyDeviceToHost, n->stream));
    MGFR_HIP(hipStreamSynchronize(n->stream));
    if (loss) *loss = *n->hloss;
    return MGFR_OK;
}

// ----------------------------------------------------- single-layer entry points

static int conv_args(int B, int S, int Cin, int Cout, int *lgS)
{
    if (B < 1 || S < 8 || (S & (S - 1))) return set_error(MGFR_ERR_ARG, "B >= 1 and power-of-two S >= 8 required");
    if (Cin < 8 || Cin % 8 || Cin > 96) return set_error(MGFR_ERR_ARG, "Cin must be a multiple of 8 in [8, 96]");
    if (Cout < 16 || Cout % 16 || Cout > 96) return set_error(MGFR_ERR_ARG, "Cout must be a multiple of 16 in [16, 96]");
    int lg = 0;
    while ((1 << lg) < S) ++lg;
    *lgS = lg;
    return MGFR_OK;
}

extern "C" int mgfr_conv3d_fwd(const void *x, int B, int S, int Cin, const void *w, const float *bias, int Cout,
                               int relu, void *y, float *y32, void *stream)
{
    int lgS, rc;
    if ((rc = conv_args(B, S, Cin, Cout, &lgS))) return rc;
    if (!x || !w || (!y && !y32)) return set_error(MGFR_ERR_ARG, "x, w and an output must be non-NULL");
    const size_t V = (size_t)B << (3 * lgS);
    launch_conv3d((const __bf16 *)x, V, lgS, Cin, (const __bf16 *)w, bias, Cout, relu, (__bf16 *)y, y32,
                  (hipStream_t)stream);
    MGFR_HIP(hipGetLastError());
    return MGFR_OK;
}

extern "C" int mgfr_conv3d_bwd_data(const void *dz, int B, int S, int Cout, const void *w, int Cin, void *wt_work,
                                    void *dx, void *stream)
{
    int lgS, rc;
    if ((rc = conv_args(B, S, Cout, Cin, &lgS))) return rc;
    if (Cin % 16 || Cout % 8) return set_error(MGFR_ERR_ARG, "backward-data needs Cin % 16 == 0");
    if (!dz || !w || !wt_work || !dx) return set_error(MGFR_ERR_ARG, "null argument");
    hipStream_t s = (hipStream_t)stream;
    k_wt_transpose<<<gridn((size_t)27 * Cin * Cout), 256, 0, s>>>((const __bf16 *)w, Cin, Cout, (__bf16 *)wt_work);
    const size_t V = (size_t)B << (3 * lgS);
    launch_conv3d((const __bf16 *)dz, V, lgS, Cout, (const __bf16 *)wt_work, nullptr, Cin, 0, (__bf16 *)dx, nullptr,
                  s);
    MGFR_HIP(hipGetLastError());
    return MGFR_OK;
}

extern "C" int mgfr_conv3d_bwd_weight(const void *x, const void *dz, int B, int S, int Cin, int Cout, float *dw,
                                      float *db, void *stream)
{
    int lgS, rc;
    if ((rc = conv_args(B, S, Cin, Cout, &lgS))) return rc;
    if (Cin % 16) return set_error(MGFR_ERR_ARG, "backward-weight needs Cin % 16 == 0");
    if (!x || !dz || !dw) return set_error(MGFR_ERR_ARG, "null argument");
    hipStream_t s = (hipStream_t)stream;
    const size_t V = (size_t)B << (3 * lgS);
    k_conv3d_wgrad<<<dim3(27, (unsigned)((V + kWChunk - 1) / kWChunk)), 256, 0, s>>>(
        (const __bf16 *)x, (const __bf16 *)dz, lgS, Cin, Cout, V, dw);
    if (db) k_bias_grad<<<gridn(V, 1024), 256, 0, s>>>((const __bf16 *)dz, Cout, V, db);
    MGFR_HIP(hipGetLastError());
    return MGFR_OK;
}

// ------------------------------------------------------------ solver hook

extern "C" int mgfr_set_net(mgfr_ctx *c, mgfr_net *n)
{
    if (!c) return set_error(MGFR_ERR_ARG, "ctx is NULL");
    nn_free(c);
    c->nn = n;
    return MGFR_OK;
}

// The context's own network (the mgfr_nn_* calls): capacity for the N/4 mesh
// and for training batches of eight 64^3 volumes.
extern "C" int mgfr_nn_init(mgfr_ctx *c, int seed)
{
    if (!c) return set_error(MGFR_ERR_ARG, "ctx is NULL");
    const int64_t n4 = (int64_t)(c->lev[0].N / 4) * (c->lev[0].N / 4) * (c->lev[0].N / 4);
    const int64_t cap = std::max<int64_t>({n4, (int64_t)8 * 64 * 64 * 64});
    mgfr_net *n = nullptr;
    int rc = mgfr_net_create(seed, (cap + 4095) / 4096 * 4096, c->stream, &n);
    if (rc) return rc;
    nn_free(c);
    c->nn = n;
    c->nn_owned = true;
    return MGFR_OK;
}

namespace {
mgfr_net *ctx_net(mgfr_ctx *c)
{
    if (!c) {
        set_error(MGFR_ERR_ARG, "ctx is NULL");
        return nullptr;
    }
    if (!c->nn) set_error(MGFR_ERR_ARG, "no network: call mgfr_nn_init or mgfr_set_net first");
    return (mgfr_net *)c->nn;
}
}  // namespace

extern "C" int mgfr_nn_train_step(mgfr_ctx *c, const double *delta, const double *u_target, int B, int S,
                                  const double *cond, float lr, float *loss)
{
    mgfr_net *n = ctx_net(c);
    if (!n) return MGFR_ERR_ARG;
    int rc = mgfr_net_set_stream(n, c->stream);
    return rc ? rc : mgfr_net_train_step(n, delta, u_target, B, S, cond, lr, loss);
}

extern "C" int mgfr_nn_predict(mgfr_ctx *c, const double *delta, double *u0)
{
    mgfr_net *n = ctx_net(c);
    if (!n) return MGFR_ERR_ARG;
    if (!delta || !u0) return set_error(MGFR_ERR_ARG, "delta and u0 must be non-NULL");
    const int cc = c->p.coarse_cycles;
    c->p.coarse_cycles = 0;  // the guess itself, without the coarse-level V-cycles of a solve
    double ms = 0.0;
    const int rc = nn_warm_start(c, delta, u0, &ms);
    c->p.coarse_cycles = cc;
    return rc;
}

extern "C" int mgfr_nn_save(mgfr_ctx *c, const char *path)
{
    mgfr_net *n = ctx_net(c);
    return n ? mgfr_net_save(n, path) : MGFR_ERR_ARG;
}

extern "C" int mgfr_nn_load(mgfr_ctx *c, const char *path)
{
    mgfr_net *n = ctx_net(c);
    return n ? mgfr_net_load(n, path) : MGFR_ERR_ARG;
}

namespace mgfr {

int nn_warm_start(mgfr_ctx *c, const double *delta, double *u, double *t_ms)
{
    mgfr_net *n = (mgfr_net *)c->nn;
    if (!n) return set_error(MGFR_ERR_ARG, "nn_mode needs a network attached with mgfr_set_net");
    if (c->nlev < 3 || c->lev[2].N < 32)
        return set_error(MGFR_ERR_ARG, "the network warm start needs N >= 128 (prediction on the N/4 mesh)");
    Level &L1 = c->lev[1], &L2 = c->lev[2];
    const int lg2 = L2.lg;
    const size_t n2 = (size_t)1 << (3 * lg2), n1 = (size_t)1 << (3 * L1.lg);
    if (n2 > n->maxvox) return set_error(MGFR_ERR_ARG, "the network's capacity is smaller than the N/4 mesh");
    hipStream_t saved = n->stream;
    n->stream = c->stream;
    MGFR_HIP(hipEventRecord(c->ev_c, c->stream));
    // delta on the N/4 mesh (means of 4^3 cells), network prediction of u there
    k_restrict4<<<gridn(n2), 256, 0, c->stream>>>(delta, lg2, L2.f);
    const double cond[2] = {c->p.a, c->p.fr0_abs};
    set_cond(n, cond, 1);
    int rc = net_forward(n, L2.f, 1, lg2);
    n->stream = saved;
    if (rc) return rc;
    k_to_u<<<gridn(n2), 256, 0, c->stream>>>(n->y32, n2, L2.u);
    // Coarse correction (nested iteration): the prediction is the initial guess
    // of the N/4 problem L(u) = R R f, which gets coarse_cycles V-cycles; its
    // solution, prolonged, starts coarse_cycles V-cycles of the N/2 problem
    // L(u) = R f, whose solution prolonged is the initial guess at N.  With
    // coarse_cycles = 0 the prediction is prolonged directly.
    const int cc = c->p.coarse_cycles;
    if (cc > 0) {
        k_restrict_mean<<<gridn(n1), 256, 0, c->stream>>>(c->lev[0].f, L1.lg, L1.f);
        k_restrict_mean<<<gridn(n2), 256, 0, c->stream>>>(L1.f, lg2, L2.f);
        MGFR_HIP(hipGetLastError());
        for (int k = 0; k < cc; ++k)
            if ((rc = vcycle64(c, 2))) return rc;
    }
    // prolong twice with the linear reconstruction (Sec. 3.3)
    k_prolong_field_set<<<(unsigned)((n2 + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(L1.u, L2.u, lg2);
    for (int k = 0; k < cc; ++k)
        if ((rc = vcycle64(c, 1))) return rc;
    k_prolong_field_set<<<(unsigned)((n1 + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(u, L1.u, L1.lg);
    MGFR_HIP(hipGetLastError());
    MGFR_HIP(hipEventRecord(c->ev_b, c->stream));
    MGFR_HIP(hipEventSynchronize(c->ev_b));
    float ms = 0.f;
    MGFR_HIP(hipEventElapsedTime(&ms, c->ev_c, c->ev_b));
    *t_ms = ms;
    return MGFR_OK;
}

// detach the network; destroy it if the context created it (mgfr_nn_init)
void nn_free(mgfr_ctx *c)
{
    if (c->nn_owned && c->nn) mgfr_net_destroy((mgfr_net *)c->nn);
    c->nn = nullptr;
    c->nn_owned = false;
}

}  // namespace mgfr
