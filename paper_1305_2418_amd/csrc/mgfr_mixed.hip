// Mixed-precision solve: float64 defect correction around float32 FAS V-cycles.
//
// Outer loop (float64, finest level only):
//   r = f - L(u)                      residual of the float64 iterate
//   stop when max|r| / D <= tol       (Sec. 3.3 step 8)
//   solve N_u(e) = r approximately    one float32 FAS V-cycle, e = 0 initially
//   u <- u + e
// where N_u(e) = L(u + e) - L(u) is evaluated without cancellation:
//   N_c = (1/h^2) sum_nb [ (w_n X_n + w_c X_c)/2 (u_n - u_c)
//                          + (w_n (1 + X_n) + w_c (1 + X_c))/2 (e_n - e_c) ]
//         + bC s_c expm1(-q e_c)
// with w = e^u, s = e^{-q u}, X = expm1(e).  The float32 unknown is the small
// correction, so float32 keeps its relative precision and the float64
// residual can still reach 1e-8.  The inner cycle is the same FAS V-cycle as
// the float64 solve (Sec. 3.3): restriction by daughter means of e and of the
// linearisation point u, coarse source N_2h(R e) + R(r - N(e)), correction
// e += P(e_2h - R e), red-black Newton-Gauss-Seidel on e.  In exact
// arithmetic one such cycle from e = 0 reproduces one float64 V-cycle, so the
// float64 residual follows the float64 solve's history to rounding.  If it
// grows for three consecutive outer iterations (the float64 solve itself shows
// two-step transients from a cold start in deep screening) or turns
// non-finite, the solve restarts as the plain float64 solve from u = 0.
#include "mgfr_internal.h"
#include "mgfr_ops.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

namespace mgfr {

namespace {


__device__ __forceinline__ size_t ix(int i, int j, int k, int lg)
{
    return (((((size_t)i) << lg) + (size_t)j) << lg) + (size_t)k;
}

// Index of cell (i,j,k) in a float32 correction-cycle array e, r or ebar of a
// level: natural order, or (split) every (i,j) row holding its cells with
// i + j + k even first (in k order), then the odd ones, so that a one-colour
// pass reads and writes its half of a row contiguously.  u32 is always natural.
__device__ __forceinline__ size_t sx(int i, int j, int k, int lg, bool split)
{
    const size_t row = ((((size_t)i) << lg) + (size_t)j) << lg;
    return split ? row + ((size_t)((i + j + k) & 1) << (lg - 1)) + (size_t)(k >> 1) : row + (size_t)k;
}

__device__ __forceinline__ double nanmax_d(double a, double b) { return (a != a || a > b) ? a : b; }

// gather the cell and its six periodic neighbours and their exponentials
struct MxCell {
    float ec, Xc, uc, wc;
    float en[6], Xn[6], un[6], wn[6];
};

__device__ __forceinline__ void mx_gather(const float *__restrict__ e, const float *__restrict__ u, int i, int j,
                                          int k, int lg, MxCell &c, bool split = false)
{
    const int m = (1 << lg) - 1;
    const int ni[6] = {(i + 1) & m, (i - 1) & m, i, i, i, i}, nj[6] = {j, j, (j + 1) & m, (j - 1) & m, j, j},
              nk[6] = {k, k, k, k, (k + 1) & m, (k - 1) & m};
    c.ec = e[sx(i, j, k, lg, split)];
    c.uc = u[ix(i, j, k, lg)];
    c.Xc = fexpm1(c.ec);
    c.wc = fexp(c.uc);
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        c.en[t] = e[sx(ni[t], nj[t], nk[t], lg, split)];
        c.un[t] = u[ix(ni[t], nj[t], nk[t], lg)];
        c.Xn[t] = fexpm1(c.en[t]);
        c.wn[t] = fexp(c.un[t]);
    }
}

__device__ __forceinline__ void mx_sweep_cell(float *__restrict__ e, const float *__restrict__ u,
                                              const float *__restrict__ r, size_t t, int lg, int colour,
                                              const MxConst &kc)
{
    const int m = (1 << lg) - 1;
    const int mh = (int)(t & (size_t)((1 << (lg - 1)) - 1));
    const size_t row = t >> (lg - 1);
    const int j = (int)(row & m), i = (int)(row >> lg);
    const int k = 2 * mh + ((i + j + colour) & 1);
    MxCell c;
    mx_gather(e, u, i, j, k, lg, c);
    const size_t cc = ix(i, j, k, lg);
    e[cc] = c.ec + mx_step(c.ec, c.Xc, c.uc, c.wc, c.en, c.Xn, c.un, c.wn, r[cc], kc);
}

__device__ __forceinline__ float mx_value_at(const float *__restrict__ e, const float *__restrict__ u, int i, int j,
                                             int k, int lg, const MxConst &kc, bool split = false)
{
    MxCell c;
    mx_gather(e, u, i, j, k, lg, c, split);
    return mx_value(c.ec, c.Xc, c.uc, c.wc, c.en, c.Xn, c.un, c.wn, kc);
}

// Daughter means of e, u and of the residual r - N(e) for coarse cell (I,J,K):
// the 2x2x2 block and its 24 face neighbours are loaded and exponentiated once.
__device__ __forceinline__ void mx_restrict_block(const float *__restrict__ e, const float *__restrict__ u,
                                                  const float *__restrict__ r, int I, int J, int K, int lg,
                                                  const MxConst &kc, float &em, float &um, float &rm, bool split)
{
    const int m = (1 << lg) - 1;
    const int i0 = 2 * I, j0 = 2 * J, k0 = 2 * K;
    // index 0..7: block cell (a,b,c) -> a*4+b*2+c; faces: [face][p][q]
    float Be[8], Bu[8], BX[8], Bw[8];
    float Fe[6][4], Fu[6][4], FX[6][4], Fw[6][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                Be[a * 4 + b * 2 + c] = e[sx(i0 + a, j0 + b, k0 + c, lg, split)];
                Bu[a * 4 + b * 2 + c] = u[ix(i0 + a, j0 + b, k0 + c, lg)];
            }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int fi[6] = {(i0 + 2) & m, (i0 - 1) & m, i0 + p, i0 + p, i0 + p, i0 + p};
            const int fj[6] = {j0 + p, j0 + p, (j0 + 2) & m, (j0 - 1) & m, j0 + q, j0 + q};
            const int fk[6] = {k0 + q, k0 + q, k0 + q, k0 + q, (k0 + 2) & m, (k0 - 1) & m};
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                Fe[f][p * 2 + q] = e[sx(fi[f], fj[f], fk[f], lg, split)];
                Fu[f][p * 2 + q] = u[ix(fi[f], fj[f], fk[f], lg)];
            }
        }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        BX[t] = fexpm1(Be[t]);
        Bw[t] = fexp(Bu[t]);
    }
#pragma unroll
    for (int f = 0; f < 6; ++f)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            FX[f][t] = fexpm1(Fe[f][t]);
            Fw[f][t] = fexp(Fu[f][t]);
        }
    float se = 0.f, su = 0.f, sr = 0.f;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int t = a * 4 + b * 2 + c;
                // neighbours +x, -x, +y, -y, +z, -z: inside the block or on a face
                const int nx0 = (a ^ 1) * 4 + b * 2 + c;
                const int ny0 = a * 4 + (b ^ 1) * 2 + c;
                const int nz0 = a * 4 + b * 2 + (c ^ 1);
                float en[6], Xn[6], un[6], wn[6];
#define MX_NB(slot, inblock, bi, face, fi)                                                  \
    if (inblock) { en[slot] = Be[bi]; Xn[slot] = BX[bi]; un[slot] = Bu[bi]; wn[slot] = Bw[bi]; } \
    else { en[slot] = Fe[face][fi]; Xn[slot] = FX[face][fi]; un[slot] = Fu[face][fi]; wn[slot] = Fw[face][fi]; }
                MX_NB(0, a == 0, nx0, 0, b * 2 + c)
                MX_NB(1, a == 1, nx0, 1, b * 2 + c)
                MX_NB(2, b == 0, ny0, 2, a * 2 + c)
                MX_NB(3, b == 1, ny0, 3, a * 2 + c)
                MX_NB(4, c == 0, nz0, 4, a * 2 + b)
                MX_NB(5, c == 1, nz0, 5, a * 2 + b)
#undef MX_NB
                const float N = mx_value(Be[t], BX[t], Bu[t], Bw[t], en, Xn, un, wn, kc);
                se += Be[t];
                su += Bu[t];
                sr += r[sx(i0 + a, j0 + b, k0 + c, lg, split)] - N;
            }
    em = 0.125f * se;
    um = 0.125f * su;
    rm = 0.125f * sr;
}

// daughter means of e, u and of the residual r - N(e) for coarse cell (I,J,K)
__device__ __forceinline__ void mx_restrict_cell(const float *__restrict__ e, const float *__restrict__ u,
                                                 const float *__restrict__ r, int I, int J, int K, int lg,
                                                 const MxConst &kc, float &em, float &um, float &rm)
{
    float se = 0.f, su = 0.f, sr = 0.f;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int i = 2 * I + a, j = 2 * J + b, k = 2 * K + c;
                const size_t cc = ix(i, j, k, lg);
                se += e[cc];
                su += u[cc];
                sr += r[cc] - mx_value_at(e, u, i, j, k, lg, kc);
            }
    em = 0.125f * se;
    um = 0.125f * su;
    rm = 0.125f * sr;
}

__device__ __forceinline__ float mx_prolong(const float *__restrict__ ec, const float *__restrict__ eb, int i,
                                            int j, int k, int lgc, int mode)
{
    const int m = (1 << lgc) - 1;
    const int I = i >> 1, J = j >> 1, K = k >> 1;
    const size_t P = ix(I, J, K, lgc);
    float v = ec[P] - eb[P];
    if (mode == 0) {
        const size_t xp = ix((I + 1) & m, J, K, lgc), xm = ix((I - 1) & m, J, K, lgc);
        const size_t yp = ix(I, (J + 1) & m, K, lgc), ym = ix(I, (J - 1) & m, K, lgc);
        const size_t zp = ix(I, J, (K + 1) & m, lgc), zm = ix(I, J, (K - 1) & m, lgc);
        const float gx = (ec[xp] - eb[xp]) - (ec[xm] - eb[xm]);
        const float gy = (ec[yp] - eb[yp]) - (ec[ym] - eb[ym]);
        const float gz = (ec[zp] - eb[zp]) - (ec[zm] - eb[zm]);
        v += ((i & 1) ? 0.125f : -0.125f) * gx;
        v += ((j & 1) ? 0.125f : -0.125f) * gy;
        v += ((k & 1) ? 0.125f : -0.125f) * gz;
    }
    return v;
}

// Element at a wave-uniform row pointer plus a 32-bit byte offset (lets the
// compiler address with a scalar base and one 32-bit lane offset).
template <typename T>
__device__ __forceinline__ const T &at_off(const float *base, uint32_t byte_off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ T &at_off(float *base, uint32_t byte_off)
{
    return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off);
}

// ---------------------------------------------------------- colour pass (N >= 128)
//
// One colour of the float32 correction sweep on a level with N >= 128: the
// cells with (i + j + k) & 1 == colour are updated in place; all six
// neighbours of such a cell have the other colour and are only read.
// Workgroup: CTJ rows of a 128-cell row tile plus one halo row on each side,
// one wave per row, marching over `chunk` planes.  Lane l holds the pair
// k = k0 + 2l, k0 + 2l + 1 of its row; in each plane one of the two is updated
// (column s, the same for the whole wave) and the other is published in LDS
// for the rows above and below and the neighbouring lanes.  s alternates from
// plane to plane, so the plane loop is written out for both parities.  e^u and
// expm1(e) of a cell are evaluated once, when its plane is loaded, and kept as
// P = e^u expm1(e) and W = e^(u+e); the cells beyond the tile's ends in k come
// from the first lanes of the upper halo wave.
// e, r and ebar of such a level are stored split by colour (see sx), so the
// pass reads r and writes e of its half only: 12 B per cell.

#ifndef MGFR_CTJ
#define MGFR_CTJ 8
#endif
constexpr int CTJ = MGFR_CTJ;  // updated rows per workgroup (the last row tile may be partial)
#ifndef MGFR_COLOUR_PF
#define MGFR_COLOUR_PF 3
#endif
constexpr int kColourPf = MGFR_COLOUR_PF;  // planes between a raw load and its use (1, 2 or 3)
static_assert(kColourPf >= 1 && kColourPf <= 3, "prefetch distance 1, 2 or 3");
#ifndef MGFR_CHUNKS
#define MGFR_CHUNKS 8
#endif
constexpr int kChunks = MGFR_CHUNKS;  // plane chunks along i per pass (N / kChunks planes each)
constexpr int CKW = 128;  // cells per row tile
constexpr int CLW = 66;   // LDS row: 64 lanes and one halo slot on each side

struct Cell4 {
    float u, e, P, W;
};

__device__ __forceinline__ Cell4 mx_cell(float u, float e)
{
    const float w = fexp(u);
    const float P = w * fexpm1(e);
    return Cell4{u, e, P, w + P};
}

__device__ __forceinline__ float4 pack(const Cell4 &c) { return make_float4(c.u, c.e, c.P, c.W); }
__device__ __forceinline__ Cell4 unpack(const float4 &v) { return Cell4{v.x, v.y, v.z, v.w}; }

// New e at a cell from the cell, its residual target r and its six neighbours
// (the same Newton step as mx_step, on the P/W form).
__device__ __forceinline__ float mx_update(const Cell4 &c, float r, const Cell4 &n0, const Cell4 &n1,
                                           const Cell4 &n2, const Cell4 &n3, const Cell4 &n4, const Cell4 &n5,
                                           const MxConst &k)
{
    float Su = 0.f, Se = 0.f, A = 0.f, B = 0.f, SW = 0.f;
    auto add = [&](const Cell4 &n) {
        const float du = n.u - c.u, de = n.e - c.e;
        Su += du;
        Se += de;
        A = fmaf(n.P, du, A);
        B = fmaf(n.W, de, B);
        SW += n.W;
    };
    add(n0);
    add(n1);
    add(n2);
    add(n3);
    add(n4);
    add(n5);
    const float flux = 0.5f * ((A + c.P * Su) + (B + c.W * Se));
    const float dflux = 0.5f * (c.W * (Su + Se - 6.0f) - SW);
    const float sc = fexp(-k.q * c.u);
    const float cm = fexpm1(-k.q * c.e);
    const float N = k.ih2 * flux + k.bC * sc * cm;
    const float J = k.ih2 * dflux - k.q * k.bC * sc * (1.0f + cm);
    float d = -(N - r) * __builtin_amdgcn_rcpf(J) * k.omega;
    if (k.max_du > 0.f) d = fminf(fmaxf(d, -k.max_du), k.max_du);
    return c.e + d;
}

struct ColourArgs {
    float *e;
    const float *u, *r;
    int lg, colour, chunk;
    MxConst kc;
};

// The plane loop of one wave whose updated column in the first plane is S0.
// ZERO: e is zero everywhere (the first pass of a correction cycle): nothing
// of e is read, and the cells of the other colour are written as 0, so that
// the array need not be cleared beforehand.
template <int S0, bool ZERO>
__device__ __forceinline__ void mx_colour_rows(const ColourArgs &A, int i0, int j0, int k0, int wv, int lane,
                                               float4 *sB)
{
    const int lg = A.lg, m = (1 << lg) - 1;
    const size_t hN = (size_t)1 << (lg - 1);
    const int row = wv - 1;                      // -1 and CTJ: halo rows
    const bool upd = row >= 0 && row < CTJ && j0 + row <= m;  // uniform over the wave
    const int jg = (j0 + row) & m;
    const size_t plane = (size_t)1 << (2 * lg);
    const size_t rowbase = (size_t)jg << lg;
    // rows that update nothing load r of the tile's first row (already fetched)
    const size_t rrowbase = upd ? rowbase : (size_t)j0 << lg;
    // addresses: a wave-uniform row pointer (scalar arithmetic) plus a 32-bit lane offset
    const uint32_t kk = 4u * (uint32_t)(k0 + 2 * lane), kh2 = 4u * (uint32_t)(k0 / 2 + lane);  // byte offsets
    auto pb = [&](int pl) { return (size_t)(pl & m) * plane + rowbase; };
    // u in natural order; e and r split by colour (column 0 of plane pl lies in half (pl + jg) & 1)
    auto ldu = [&](int pl) { return at_off<float2>(A.u + pb(pl), kk); };
    auto lde = [&](int pl) {
        if constexpr (ZERO) return make_float2(0.0f, 0.0f);
        const bool odd = ((pl + jg) & 1) != 0;
        const float *h0 = A.e + pb(pl) + (odd ? hN : 0), *h1 = A.e + pb(pl) + (odd ? 0 : hN);
        return make_float2(at_off<float>(h0, kh2), at_off<float>(h1, kh2));
    };
    auto row_c = [&](int pl) { return A.e + pb(pl) + (size_t)A.colour * hN; };  // half of the updated cells
    auto row_r = [&](int pl) { return A.r + (size_t)(pl & m) * plane + rrowbase + (size_t)A.colour * hN; };
    // k-halo duty: lanes 0..CTJ-1 of the upper halo wave serve row `lane`.  Every
    // lane of every wave issues the same loads in every plane (lane mod CTJ), so
    // that no load sits under a branch and the prefetch waits stay exact.
    const bool kh = wv == 0 && lane < CTJ;
    const int khq = lane % CTJ;
    const size_t khrow = (size_t)((j0 + khq) & m) << lg;
    const int khpar = (A.colour + j0 + khq) & 1;  // updated column of that row in even planes
    auto kh_k = [&](int pl) { return (khpar ^ (pl & 1)) ? ((k0 + CKW) & m) : ((k0 - 1) & m); };
    auto kh_u = [&](int pl) { return (size_t)(pl & m) * plane + khrow + (size_t)kh_k(pl); };
    // the halo cell has the other colour
    auto kh_e = [&](int pl) {
        return (size_t)(pl & m) * plane + khrow + (size_t)(1 - A.colour) * hN + (size_t)(kh_k(pl) >> 1);
    };
    auto kh_slot = [&](int pl) { return (lane + 1) * CLW + ((khpar ^ (pl & 1)) ? CLW - 1 : 0); };

    // prologue: plane i0 (both columns), plane i0 - 1 (column S0), raw plane i0 + 1
    Cell4 c0, c1, prev;
    {
        const float2 u0 = ldu(i0), e0 = lde(i0);
        const float2 um = ldu(i0 - 1), em = lde(i0 - 1);
        c0 = mx_cell(u0.x, e0.x);
        c1 = mx_cell(u0.y, e0.y);
        prev = S0 ? mx_cell(um.y, em.y) : mx_cell(um.x, em.x);
    }
    // raw loads of step p: u, e of plane p + 1, r of plane p, the k-halo cell of plane p.
    // They are issued kColourPf steps ahead; four register sets rotate with the
    // four-plane loop body, so that no register holding a load in flight is copied.
    struct Raw {
        float2 u, e;
        float r, khu, khe;
    };
    auto load = [&](int p) {
        Raw w;
        w.u = ldu(p + 1);
        w.e = lde(p + 1);
        w.r = at_off<float>(row_r(p), kh2);
        w.khu = A.u[kh_u(p)];
        w.khe = ZERO ? 0.0f : A.e[kh_e(p)];
        return w;
    };
    Raw ra = load(i0), rb = kColourPf >= 2 ? load(i0 + 1) : Raw{}, rc = kColourPf == 3 ? load(i0 + 2) : Raw{}, rd;
    int buf = 0;

    // one plane with updated column S: consume cur (step p), load nxt (step p + kColourPf)
    auto step = [&](int p, auto Sc, const Raw &cur, Raw &nxt) {
        constexpr int S = decltype(Sc)::value;
        nxt = load(p + kColourPf);
        // plane p + 1 from the raw values loaded kColourPf planes ago
        const Cell4 n0 = mx_cell(cur.u.x, cur.e.x), n1 = mx_cell(cur.u.y, cur.e.y);
        float4 *B = sB + buf * (CTJ + 2) * CLW;
        B[(row + 1) * CLW + lane + 1] = pack(S ? c0 : c1);
        if (kh) B[kh_slot(p)] = pack(mx_cell(cur.khu, cur.khe));
        __syncthreads();
        if (upd) {
            const Cell4 up = unpack(B[row * CLW + lane + 1]);
            const Cell4 dn = unpack(B[(row + 2) * CLW + lane + 1]);
            const Cell4 sd = unpack(B[(row + 1) * CLW + lane + (S ? 2 : 0)]);
            const float en = S ? mx_update(c1, cur.r, c0, sd, up, dn, prev, n1, A.kc)
                               : mx_update(c0, cur.r, c1, sd, up, dn, prev, n0, A.kc);
            at_off<float>(row_c(p), kh2) = en;
            if constexpr (ZERO) at_off<float>(A.e + pb(p) + (size_t)(1 - A.colour) * hN, kh2) = 0.0f;
        }
        prev = S ? c0 : c1;
        c0 = n0;
        c1 = n1;
        buf ^= 1;
    };
    using Z0 = std::integral_constant<int, S0>;
    using Z1 = std::integral_constant<int, 1 - S0>;
    if constexpr (kColourPf == 3) {
        for (int p = i0; p < i0 + A.chunk; p += 4) {  // chunk is a multiple of 4
            step(p, Z0{}, ra, rd);
            step(p + 1, Z1{}, rb, ra);
            step(p + 2, Z0{}, rc, rb);
            step(p + 3, Z1{}, rd, rc);
        }
    } else if constexpr (kColourPf == 2) {
        for (int p = i0; p < i0 + A.chunk; p += 4) {
            step(p, Z0{}, ra, rc);
            step(p + 1, Z1{}, rb, rd);
            step(p + 2, Z0{}, rc, ra);
            step(p + 3, Z1{}, rd, rb);
        }
    } else {
        for (int p = i0; p < i0 + A.chunk; p += 2) {
            step(p, Z0{}, ra, rb);
            step(p + 1, Z1{}, rb, ra);
        }
    }
}

// grid: 1-D, (N / CKW) ceil(N / CTJ) (N / chunk) workgroups, spread so that
// workgroups adjacent in j run on the same XCD (they share halo rows)
template <bool ZERO>
__device__ __forceinline__ void mx_colour_pass(const ColourArgs &A, float4 *sB)
{
    const int lg = A.lg;
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned L = (b & 7u) * (nb >> 3) + (b >> 3);  // nb is a multiple of 8
    const int nkt = (1 << lg) / CKW, njt = ((1 << lg) + CTJ - 1) / CTJ;
    const int kt = (int)(L % (unsigned)nkt), jt = (int)((L / (unsigned)nkt) % (unsigned)njt),
              it = (int)(L / ((unsigned)nkt * (unsigned)njt));
    const int k0 = kt * CKW, j0 = jt * CTJ, i0 = it * A.chunk;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int s0 = (A.colour + i0 + j0 + wv - 1) & 1;  // updated column of this wave's row in plane i0
    if (s0)
        mx_colour_rows<1, ZERO>(A, i0, j0, k0, wv, lane, sB);
    else
        mx_colour_rows<0, ZERO>(A, i0, j0, k0, wv, lane, sB);
}

__global__ __launch_bounds__(64 * (CTJ + 2)) void k_mx_colour(ColourArgs A)
{
    __shared__ float4 sB[2 * (CTJ + 2) * CLW];
    mx_colour_pass<false>(A, sB);
}

// the first pass of a correction cycle, from e = 0
__global__ __launch_bounds__(64 * (CTJ + 2)) void k_mx_colour_zero(ColourArgs A)
{
    __shared__ float4 sB[2 * (CTJ + 2) * CLW];
    mx_colour_pass<true>(A, sB);
}

// ------------------------------------------- fused red-black sweep (N >= 128)
//
// One whole float32 correction sweep (red cells, then black cells) in one
// launch, out of place: eout = sweep(ein) on a split level (see sx).  A
// workgroup owns FI = FW - 4 rows of a 128-cell row tile and marches over
// `chunk` planes; in step p it updates the red cells of plane p + 1 and then
// the black cells of plane p, which by then have all six red neighbours new.
// The black update of an edge row needs red updates one row beyond the tile,
// which need the old black values of the row after that, so the workgroup has
// one wave per row for FI + 4 rows: the outer two only load, the next two
// update their red cells as well (results kept in LDS, not stored).  In k the
// same holds for the cells k0 - 1 and k0 + 128: the first wave (an outer row)
// also loads the cells k0 - 2, k0 - 1, k0 + 128, k0 + 129 of every row (one
// lane each) and updates the red ones of the inner rows.  The chunk starts two
// planes early for the same reason in i.
//
// Lane l of a row wave holds the cells k0 + 2l, k0 + 2l + 1; on plane p + 1
// the red one is column s = (p + 1 + j) & 1, and on plane p that same column
// is black, so each lane does one red and one black update per step.  LDS
// holds three planes (p, p + 1 and the one being filled) as P/W cells by row,
// column parity and pair slot (slot 0 and 65: the k-halo cells).  Every cell
// of ein, u and r is read once and every cell of eout written once (16 B per
// cell and sweep) apart from the halo rows, which come mostly from L2.

#ifndef MGFR_FW
#define MGFR_FW 16
#endif
constexpr int FW = MGFR_FW;  // waves (rows) per workgroup
constexpr int FI = FW - 4;   // rows updated and stored
constexpr int FS = 66;       // LDS slots per row and column parity
static_assert(4 * FW <= 64, "the k-halo cells of all rows are served by one wave");

struct Sweep2Args {
    const float *ein;
    float *eout;
    const float *u, *r;
    int lg, chunk;
    MxConst kc;
};

// (u, e, P = w X, W = w E) of a cell, w = e^u, X = e^e - 1 (fexpm1), E = e^e
__device__ __forceinline__ float4 mx_cell4(float u, float e, float w)
{
    const float E = fexp(e);
    const float X = fabsf(e) < 0x1p-10f ? fmaf(0.5f * e, e, e) : E - 1.0f;
    return make_float4(u, e, w * X, w * E);
}

// New e at a cell c = (u, e, P, W) from its residual target r and six
// neighbours (u, e, P, W): the Newton step of mx_update.
__device__ __forceinline__ float own_update(const float4 &c, float r, const float4 &n0, const float4 &n1,
                                            const float4 &n2, const float4 &n3, const float4 &n4, const float4 &n5,
                                            const MxConst &k)
{
    float Su = 0.f, Se = 0.f, A = 0.f, B = 0.f, SW = 0.f;
    auto add = [&](const float4 &n) {
        const float du = n.x - c.x, de = n.y - c.y;
        Su += du;
        Se += de;
        A = fmaf(n.z, du, A);
        B = fmaf(n.w, de, B);
        SW += n.w;
    };
    add(n0);
    add(n1);
    add(n2);
    add(n3);
    add(n4);
    add(n5);
    const float flux = 0.5f * ((A + c.z * Su) + (B + c.w * Se));
    const float dflux = 0.5f * (c.w * (Su + Se - 6.0f) - SW);
    const float sc = fexp(-k.q * c.x);
    const float cm = fexpm1(-k.q * c.y);
    const float bs = k.bC * sc;
    const float N = k.ih2 * flux + bs * cm;
    const float J = k.ih2 * dflux - k.q * bs * (1.0f + cm);
    float d = -(N - r) * __builtin_amdgcn_rcpf(J) * k.omega;
    if (k.max_du > 0.f) d = fminf(fmaxf(d, -k.max_du), k.max_du);
    return c.y + d;
}

template <int S0>
__device__ __forceinline__ void mx_sweep2_rows(const Sweep2Args &A, int i0, int j0, int k0, int w, int lane,
                                               float4 *sX)
{
    const int lg = A.lg, m = (1 << lg) - 1;
    const size_t hN = (size_t)1 << (lg - 1), plane = (size_t)1 << (2 * lg);
    const int jg = (j0 + w - 2) & m;
    const bool red_row = w >= 1 && w <= FW - 2;                          // uniform over the wave
    const bool blk_row = w >= 2 && w <= FW - 3 && j0 + w - 2 <= m;      // rows stored
    const size_t rowb = (size_t)jg << lg;
    // addresses: a wave-uniform row pointer plus a 32-bit lane byte offset
    const uint32_t kk = 4u * (uint32_t)(k0 + 2 * lane), kh2 = 4u * (uint32_t)(k0 / 2 + lane);
    auto pb = [&](int pl) { return (size_t)(pl & m) * plane + rowb; };
    auto ldu = [&](int pl) { return at_off<float2>(A.u + pb(pl), kk); };
    // cell k0 + 2l lies in half (pl + jg) & 1 of its row (k0 is even)
    auto lde = [&](int pl) {
        const bool odd = ((pl + jg) & 1) != 0;
        return make_float2(at_off<float>(A.ein + pb(pl) + (odd ? hN : 0), kh2),
                           at_off<float>(A.ein + pb(pl) + (odd ? 0 : hN), kh2));
    };
    // k-halo duty of the first wave: lane = 4 row + c, c -> k0 - 2, k0 - 1, k0 + 128, k0 + 129
    const bool hv = w == 0 && lane < 4 * FW;
    const int hl = lane % (4 * FW), hw = hl >> 2, hc = hl & 3;
    const int hjg = (j0 + hw - 2) & m;
    const int hk = (hc < 2 ? k0 - 2 + hc : k0 + 126 + hc) & m;
    const int hpar = hc & 1, hslot = hc < 2 ? 0 : FS - 1;
    const bool hin = hv && (hc == 1 || hc == 2) && hw >= 2 && hw <= FW - 3;
    const size_t hrow = (size_t)hjg << lg;
    auto hb = [&](int pl) { return (size_t)(pl & m) * plane + hrow; };
    auto hle = [&](int pl) { return A.ein[hb(pl) + ((size_t)((pl + hjg + hk) & 1) << (lg - 1)) + (size_t)(hk >> 1)]; };
    auto cell = [&](float u, float e) { return mx_cell4(u, e, fexp(u)); };
    auto at = [&](int buf, int row, int par, int slot) { return ((buf * FW + row) * 2 + par) * FS + slot; };

    // raw loads of step p, issued one step ahead in two alternating register sets
    struct Raw {
        float2 u, e;       // plane p + 2
        float rr, rb;      // r of the red cell of plane p + 1, of the black cell of plane p
        float hu, he, hr;  // k-halo cell: u, e of plane p + 2, r of plane p + 1 (red half)
    };
    auto load = [&](int p) {
        Raw x;
        x.u = ldu(p + 2);
        x.e = lde(p + 2);
        x.rr = at_off<float>(A.r + pb(p + 1), kh2);
        x.rb = at_off<float>(A.r + pb(p) + hN, kh2);
        x.hu = A.u[hb(p + 2) + (size_t)hk];
        x.he = hle(p + 2);
        x.hr = A.r[hb(p + 1) + (size_t)(hk >> 1)];
        return x;
    };

    // planes i0 - 2 (P0) and i0 - 1 (P1), old values; the k-halo cell of plane
    // p is read back from LDS, that of plane p + 1 is kept in H1
    float4 P0[2], P1[2], H1, prev;
    {
        const float2 ua = ldu(i0 - 2), ea = lde(i0 - 2), ub = ldu(i0 - 1), eb = lde(i0 - 1);
        P0[0] = cell(ua.x, ea.x);
        P0[1] = cell(ua.y, ea.y);
        P1[0] = cell(ub.x, eb.x);
        P1[1] = cell(ub.y, eb.y);
        prev = P0[0];
        const float4 H0 = cell(A.u[hb(i0 - 2) + (size_t)hk], hle(i0 - 2));
        if (hv) sX[at(0, hw, hpar, hslot)] = H0;  // ordered by the first step's barrier
        H1 = cell(A.u[hb(i0 - 1) + (size_t)hk], hle(i0 - 1));
    }
    Raw ra = load(i0 - 2), rb;
    int x0 = 0, x1 = 1, x2 = 2;  // LDS buffers of planes p, p + 1, p + 2
    const int iend = i0 + A.chunk;

    auto step = [&](int p, auto Sc, auto Bc, const Raw &cur, Raw &nxt) {
        constexpr int S = decltype(Sc)::value;
        constexpr bool BLACK = decltype(Bc)::value;
        nxt = load(p + 1);
        const float4 Q0 = cell(cur.u.x, cur.e.x), Q1 = cell(cur.u.y, cur.e.y);
        const float4 &QS = S ? Q1 : Q0;
        float4 HQ = H1;
        if (w == 0) HQ = cell(cur.hu, cur.he);
        // publish the old black cell of plane p + 1 (and the k-halo cells)
        sX[at(x1, w, 1 - S, lane + 1)] = P1[1 - S];
        if (hv) sX[at(x1, hw, hpar, hslot)] = H1;
        __syncthreads();
        // red cell of plane p + 1: neighbours black and old
        if (red_row) {
            const float4 sd = S ? sX[at(x1, w, 0, lane + 2)] : sX[at(x1, w, 1, lane)];
            const float4 up = sX[at(x1, w - 1, S, lane + 1)];
            const float4 dn = sX[at(x1, w + 1, S, lane + 1)];
            const float wr = fexp(P1[S].x);
            const float en = own_update(P1[S], cur.rr, P1[1 - S], sd, up, dn, P0[S], QS, A.kc);
            P1[S] = mx_cell4(P1[S].x, en, wr);
            sX[at(x1, w, S, lane + 1)] = P1[S];
            if (blk_row && p + 1 >= i0 && p + 1 < iend) at_off<float>(A.eout + pb(p + 1), kh2) = en;
        }
        if (w == 0) {
            // red k-halo cells of the stored rows
            if (hin && (((p + 1) + hjg + hk) & 1) == 0) {
                const float4 na = hc == 1 ? sX[at(x1, hw, 0, 0)] : sX[at(x1, hw, 1, FS - 1)];
                const float4 nb = hc == 1 ? sX[at(x1, hw, 0, 1)] : sX[at(x1, hw, 1, FS - 2)];
                const float4 up = sX[at(x1, hw - 1, hpar, hslot)];
                const float4 dn = sX[at(x1, hw + 1, hpar, hslot)];
                const float4 H0 = sX[at(x0, hw, hpar, hslot)];
                const float wh = fexp(H1.x);
                const float en = own_update(H1, cur.hr, na, nb, up, dn, H0, HQ, A.kc);
                H1 = mx_cell4(H1.x, en, wh);
                sX[at(x1, hw, hpar, hslot)] = H1;
            }
        }
        // black cell of plane p: neighbours red and new (plane p's buffer was
        // completed in the previous step)
        if (BLACK && blk_row) {
            const float4 sd = S ? sX[at(x0, w, 0, lane + 2)] : sX[at(x0, w, 1, lane)];
            const float4 up = sX[at(x0, w - 1, S, lane + 1)];
            const float4 dn = sX[at(x0, w + 1, S, lane + 1)];
            at_off<float>(A.eout + pb(p) + hN, kh2) =
                own_update(P0[S], cur.rb, P0[1 - S], sd, up, dn, prev, P1[S], A.kc);
        }
        prev = P0[1 - S];
        P0[0] = P1[0];
        P0[1] = P1[1];
        P1[0] = Q0;
        P1[1] = Q1;
        H1 = HQ;
        const int t = x0;
        x0 = x1;
        x1 = x2;
        x2 = t;
    };
    using Z0 = std::integral_constant<int, S0>;
    using Z1 = std::integral_constant<int, 1 - S0>;
    using NB = std::integral_constant<bool, false>;
    using YB = std::integral_constant<bool, true>;
    step(i0 - 2, Z0{}, NB{}, ra, rb);
    step(i0 - 1, Z1{}, NB{}, rb, ra);
    for (int p = i0; p < iend; p += 2) {  // chunk is even
        step(p, Z0{}, YB{}, ra, rb);
        step(p + 1, Z1{}, YB{}, rb, ra);
    }
}

// grid: 1-D, (N / 128) ceil(N / FI) (N / chunk) workgroups, spread over the
// XCDs as in the colour pass
__global__ __launch_bounds__(64 * FW) void k_mx_sweep2(Sweep2Args A)
{
    __shared__ float4 sX[3 * FW * 2 * FS];
    const int lg = A.lg;
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned L = (b & 7u) * (nb >> 3) + (b >> 3);  // nb is a multiple of 8
    const int nkt = (1 << lg) / CKW, njt = ((1 << lg) + FI - 1) / FI;
    const int kt = (int)(L % (unsigned)nkt), jt = (int)((L / (unsigned)nkt) % (unsigned)njt),
              it = (int)(L / ((unsigned)nkt * (unsigned)njt));
    const int k0 = kt * CKW, j0 = jt * FI, i0 = it * A.chunk;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    // red column of this wave's row on plane i0 - 1 (step i0 - 2)
    const int s0 = (i0 - 1 + j0 + w - 2) & 1;
    if (s0)
        mx_sweep2_rows<1>(A, i0, j0, k0, w, lane, sX);
    else
        mx_sweep2_rows<0>(A, i0, j0, k0, w, lane, sX);
}

// ------------------------------------------------- restriction pass (N >= 128)
//
// Residual restriction from a split level with N >= 128 to the next coarser
// level: for every coarse cell the means of e, u and r - N(e) over its eight
// daughters.  Same workgroups and plane march as the colour pass, but both
// cells of a lane's pair need N(e), so both are published in LDS and the
// k-halo holds both ends of every row.  The daughter sums run over the pair
// (lane), the row pair (adjacent waves, combined in LDS) and the plane pair
// (two consecutive steps).

__device__ __forceinline__ float mx_nval(const Cell4 &c, const Cell4 &n0, const Cell4 &n1, const Cell4 &n2,
                                         const Cell4 &n3, const Cell4 &n4, const Cell4 &n5, const MxConst &k)
{
    float Su = 0.f, Se = 0.f, A = 0.f, B = 0.f;
    auto add = [&](const Cell4 &n) {
        const float du = n.u - c.u, de = n.e - c.e;
        Su += du;
        Se += de;
        A = fmaf(n.P, du, A);
        B = fmaf(n.W, de, B);
    };
    add(n0);
    add(n1);
    add(n2);
    add(n3);
    add(n4);
    add(n5);
    const float flux = 0.5f * ((A + c.P * Su) + (B + c.W * Se));
    return k.ih2 * flux + k.bC * fexp(-k.q * c.u) * fexpm1(-k.q * c.e);
}

constexpr int PTJ = 8;  // fine rows per workgroup (even: rows pair up)

struct RestrictArgs {
    const float *e, *u, *r;
    float *ebc, *uc, *rc;
    int lg, chunk;
    bool split_c;
    MxConst kc;
};

__global__ __launch_bounds__(64 * (PTJ + 2)) void k_mx_restrict_pass(RestrictArgs A)
{
    __shared__ float4 sB[2 * (PTJ + 2) * CLW * 2];  // [buffer][row][slot][column]
    __shared__ float4 sR[PTJ / 2][64];               // odd rows' daughter sums
    const int lg = A.lg, m = (1 << lg) - 1, lgc = lg - 1;
    const size_t hN = (size_t)1 << (lg - 1);
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned L = (b & 7u) * (nb >> 3) + (b >> 3);
    const int nkt = (1 << lg) / CKW, njt = (1 << lg) / PTJ;
    const int kt = (int)(L % (unsigned)nkt), jt = (int)((L / (unsigned)nkt) % (unsigned)njt),
              it = (int)(L / ((unsigned)nkt * (unsigned)njt));
    const int k0 = kt * CKW, j0 = jt * PTJ, i0 = it * A.chunk;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int row = wv - 1;
    const bool upd = row >= 0 && row < PTJ;
    const int jg = (j0 + row) & m;
    const size_t plane = (size_t)1 << (2 * lg);
    const size_t rowbase = (size_t)jg << lg;
    const size_t kk = (size_t)(k0 + 2 * lane), kh2 = (size_t)(k0 / 2 + lane);
    auto pb = [&](int pl) { return (size_t)(pl & m) * plane + rowbase; };
    auto ld_split = [&](const float *a, int pl) {  // both cells of the pair from the two colour halves
        const size_t q = pb(pl) + kh2;
        const bool odd = ((pl + jg) & 1) != 0;
        return make_float2(a[q + (odd ? hN : 0)], a[q + (odd ? 0 : hN)]);
    };
    // k-halo: lanes 0..2 PTJ - 1 of wave 0 serve row lane / 2, end lane & 1 (0: k0 - 1, 1: k0 + CKW)
    const bool kh = wv == 0 && lane < 2 * PTJ;
    const int khq = (lane & (2 * PTJ - 1)) >> 1, khs = lane & 1;
    const int khj = (j0 + khq) & m, khk = khs ? ((k0 + CKW) & m) : ((k0 - 1) & m);
    auto kh_u = [&](int pl) { return (size_t)(pl & m) * plane + ((size_t)khj << lg) + (size_t)khk; };
    auto kh_e = [&](int pl) {
        return (size_t)(pl & m) * plane + ((size_t)khj << lg) + ((size_t)(((pl & m) + khj + khk) & 1) << (lg - 1)) +
               (size_t)(khk >> 1);
    };
    auto slot = [&](int r, int l, int col) { return ((r + 1) * CLW + l + 1) * 2 + col; };

    Cell4 p0, p1, c0, c1;
    {
        const float2 um = *reinterpret_cast<const float2 *>(A.u + pb(i0 - 1) + kk), em = ld_split(A.e, i0 - 1);
        const float2 u0 = *reinterpret_cast<const float2 *>(A.u + pb(i0) + kk), e0 = ld_split(A.e, i0);
        p0 = mx_cell(um.x, em.x);
        p1 = mx_cell(um.y, em.y);
        c0 = mx_cell(u0.x, e0.x);
        c1 = mx_cell(u0.y, e0.y);
    }
    // raw loads of step p: u, e of plane p + 1; r and the k-halo cell of plane p
    struct Raw {
        float2 u, e, r;
        float khu, khe;
    };
    auto load = [&](int p) {
        Raw w;
        w.u = *reinterpret_cast<const float2 *>(A.u + pb(p + 1) + kk);
        w.e = ld_split(A.e, p + 1);
        w.r = ld_split(A.r, p);  // halo rows: loaded, not used
        w.khu = A.u[kh_u(p)];
        w.khe = A.e[kh_e(p)];
        return w;
    };
    Raw ra = load(i0), rb;  // issued one step ahead (more would cost occupancy here)
    int buf = 0;
    float se = 0.f, su = 0.f, sr = 0.f;
    auto step = [&](int p, bool second, const Raw &cur, Raw &nxt) {
        nxt = load(p + 1);
        const Cell4 n0 = mx_cell(cur.u.x, cur.e.x), n1 = mx_cell(cur.u.y, cur.e.y);
        float4 *B = sB + buf * (PTJ + 2) * CLW * 2;
        B[slot(row, lane, 0)] = pack(c0);
        B[slot(row, lane, 1)] = pack(c1);
        if (kh) B[khs ? slot(khq, CKW / 2, 0) : slot(khq, -1, 1)] = pack(mx_cell(cur.khu, cur.khe));
        __syncthreads();
        if (upd) {
            const Cell4 up0 = unpack(B[slot(row - 1, lane, 0)]), up1 = unpack(B[slot(row - 1, lane, 1)]);
            const Cell4 dn0 = unpack(B[slot(row + 1, lane, 0)]), dn1 = unpack(B[slot(row + 1, lane, 1)]);
            const Cell4 lf = unpack(B[slot(row, lane - 1, 1)]), rt = unpack(B[slot(row, lane + 1, 0)]);
            const float N0 = mx_nval(c0, p0, n0, up0, dn0, lf, c1, A.kc);
            const float N1 = mx_nval(c1, p1, n1, up1, dn1, c0, rt, A.kc);
            se += c0.e + c1.e;
            su += c0.u + c1.u;
            sr += (cur.r.x - N0) + (cur.r.y - N1);
        }
        if (second) {
            if (upd && (row & 1)) sR[row >> 1][lane] = make_float4(se, su, sr, 0.f);
            __syncthreads();
            if (upd && !(row & 1)) {
                const float4 o = sR[row >> 1][lane];
                const int I = (p & m) >> 1, J = jg >> 1, K = k0 / 2 + lane;
                const size_t nat = ((((size_t)I << lgc) + (size_t)J) << lgc) + (size_t)K;
                const size_t spl = A.split_c ? ((((size_t)I << lgc) + (size_t)J) << lgc) +
                                                   ((size_t)((I + J + K) & 1) << (lgc - 1)) + (size_t)(K >> 1)
                                             : nat;
                A.ebc[spl] = 0.125f * (se + o.x);
                A.uc[nat] = 0.125f * (su + o.y);
                A.rc[spl] = 0.125f * (sr + o.z);
            }
            se = su = sr = 0.f;
        }
        p0 = c0;
        p1 = c1;
        c0 = n0;
        c1 = n1;
        buf ^= 1;
    };
    for (int p = i0; p < i0 + A.chunk; p += 2) {
        step(p, false, ra, rb);
        step(p + 1, true, rb, ra);
    }
}

// ------------------------------------------------------------------- kernels

__global__ __launch_bounds__(kBlock) void k_mx_sweep_half(float *__restrict__ e, const float *__restrict__ u,
                                                            const float *__restrict__ r, int lg, int colour,
                                                            MxConst kc)
{
    mx_sweep_cell(e, u, r, (size_t)blockIdx.x * kBlock + threadIdx.x, lg, colour, kc);
}

__global__ __launch_bounds__(kBlock) void k_mx_residual_restrict(const float *__restrict__ e,
                                                                   const float *__restrict__ u,
                                                                   const float *__restrict__ r, int lg, MxConst kc,
                                                                   float *__restrict__ eb_c, float *__restrict__ u_c,
                                                                   float *__restrict__ r_c, bool split, bool split_c)
{
    const int lgc = lg - 1;
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int K = (int)(t & ((1u << lgc) - 1)), J = (int)((t >> lgc) & ((1u << lgc) - 1)), I = (int)(t >> (2 * lgc));
    float em, um, rm;
    mx_restrict_block(e, u, r, I, J, K, lg, kc, em, um, rm, split);
    const size_t tc = sx(I, J, K, lgc, split_c);
    eb_c[tc] = em;
    u_c[t] = um;
    r_c[tc] = rm;
}

// r_c += N_c(eb); e_c = eb
__global__ __launch_bounds__(kBlock) void k_mx_coarse_rhs(const float *__restrict__ eb, const float *__restrict__ u,
                                                            int lg, MxConst kc, float *__restrict__ rc,
                                                            float *__restrict__ ec, bool split)
{
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int m = (1 << lg) - 1;
    const int k = (int)(t & m), j = (int)((t >> lg) & m), i = (int)(t >> (2 * lg));
    const size_t ts = sx(i, j, k, lg, split);
    rc[ts] += mx_value_at(eb, u, i, j, k, lg, kc, split);
    ec[ts] = eb[ts];
}

// one thread per coarse cell: its 8 daughters of the 2^lg mesh
__global__ __launch_bounds__(kBlock) void k_mx_prolong_add(float *__restrict__ e, const float *__restrict__ ec,
                                                             const float *__restrict__ eb, int lg, int mode, bool split,
                                                             bool split_c)
{
    const int lgc = lg - 1, m = (1 << lgc) - 1;
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int K = (int)(t & ((1u << lgc) - 1)), J = (int)((t >> lgc) & ((1u << lgc) - 1)), I = (int)(t >> (2 * lgc));
    auto d = [&](int i, int j, int k) {
        const size_t q = sx(i, j, k, lgc, split_c);
        return ec[q] - eb[q];
    };
    const float v0 = d(I, J, K);
    float gx = 0.f, gy = 0.f, gz = 0.f;
    if (mode == 0) {
        gx = d((I + 1) & m, J, K) - d((I - 1) & m, J, K);
        gy = d(I, (J + 1) & m, K) - d(I, (J - 1) & m, K);
        gz = d(I, J, (K + 1) & m) - d(I, J, (K - 1) & m);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                float v = v0;
                if (mode == 0) {
                    v += (a ? 0.125f : -0.125f) * gx;
                    v += (b ? 0.125f : -0.125f) * gy;
                    v += (c ? 0.125f : -0.125f) * gz;
                }
                e[sx(2 * I + a, 2 * J + b, 2 * K + c, lg, split)] += v;
            }
}

struct MxTail {
    float *e[kMaxLevels];
    float *u[kMaxLevels];
    float *r[kMaxLevels];
    float *eb[kMaxLevels];
    float ih2[kMaxLevels];
    int lg[kMaxLevels];
    int l0, nlev, pre, post, coarse, mode;
    float bC, q, max_du, omega;
};

// The tail (levels with N <= kTailN: 16^3, 8^3, 4^3) runs in one workgroup
// with every array in LDS: e, u and r of its top level are copied in and e is
// copied out at the end; the coarser levels' arrays (e, u, r and the restricted
// e) live only here.  Level l0 + k holds 2^(3 (lg0 - k)) cells; its arrays sit
// after those of the finer levels (three at l0, four below).
constexpr int kTailLdsFloats = 3 * (1 << 12) + 4 * (1 << 9) + 4 * (1 << 6);
static_assert(kTailN <= 16, "the tail's LDS holds levels up to 16^3");

struct TailLds {
    float *lds;
    int l0, lg0;
    __device__ int cells(int l) const { return 1 << (3 * (lg0 - (l - l0))); }
    __device__ float *base(int l) const
    {
        int off = 0;
        if (l > l0) {
            off = 3 * cells(l0);
            for (int k = l0 + 1; k < l; ++k) off += 4 * cells(k);
        }
        return lds + off;
    }
    __device__ float *e(int l) const { return base(l); }
    __device__ float *u(int l) const { return base(l) + cells(l); }
    __device__ float *r(int l) const { return base(l) + 2 * cells(l); }
    __device__ float *eb(int l) const { return base(l) + 3 * cells(l); }  // l > l0
};

// Red-black sweeps of one tail level.  The 4^3 level (32 cells per colour) is
// swept by the first wave alone: within one wave the LDS accesses of a
// half-sweep are done before the next one's, and the fences keep the compiler
// from moving them, so no workgroup barrier is needed per half-sweep.
__device__ void mx_tail_sweeps(const MxTail &A, const TailLds &T, int l, int sweeps)
{
    const MxConst kc{A.ih2[l], A.bC, A.q, A.max_du, A.omega};
    const int lg = A.lg[l];
    const int half = 1 << (3 * lg - 1);
    float *e = T.e(l);
    const float *u = T.u(l), *r = T.r(l);
    if (half <= 32) {  // uniform
        if (threadIdx.x < 64)
            for (int s = 0; s < sweeps; ++s)
                for (int colour = 0; colour < 2; ++colour) {
                    if ((int)threadIdx.x < half) mx_sweep_cell(e, u, r, threadIdx.x, lg, colour, kc);
                    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                }
        __syncthreads();
        return;
    }
    for (int s = 0; s < sweeps; ++s)
        for (int colour = 0; colour < 2; ++colour) {
            for (int t = threadIdx.x; t < half; t += kTailThreads) mx_sweep_cell(e, u, r, t, lg, colour, kc);
            __syncthreads();
        }
}

__global__ __launch_bounds__(kTailThreads) void k_mx_tail(MxTail A)
{
    __shared__ float lds[kTailLdsFloats];
    const TailLds T{lds, A.l0, A.lg[A.l0]};
    const int n0 = T.cells(A.l0);
    for (int t = threadIdx.x; t < n0; t += kTailThreads) {
        T.e(A.l0)[t] = A.e[A.l0][t];
        T.u(A.l0)[t] = A.u[A.l0][t];
        T.r(A.l0)[t] = A.r[A.l0][t];
    }
    __syncthreads();
    for (int l = A.l0; l < A.nlev - 1; ++l) {
        mx_tail_sweeps(A, T, l, A.pre);
        const MxConst kc{A.ih2[l], A.bC, A.q, A.max_du};
        const int lg = A.lg[l], lgc = lg - 1;
        const int nc = 1 << (3 * lgc);
        for (int t = threadIdx.x; t < nc; t += kTailThreads) {
            const int K = t & ((1 << lgc) - 1), J = (t >> lgc) & ((1 << lgc) - 1), I = t >> (2 * lgc);
            float em, um, rm;
            mx_restrict_cell(T.e(l), T.u(l), T.r(l), I, J, K, lg, kc, em, um, rm);
            T.eb(l + 1)[t] = em;
            T.u(l + 1)[t] = um;
            T.r(l + 1)[t] = rm;
        }
        __syncthreads();
        const MxConst kcc{A.ih2[l + 1], A.bC, A.q, A.max_du};
        const int mc = (1 << lgc) - 1;
        for (int t = threadIdx.x; t < nc; t += kTailThreads) {
            const int k = t & mc, j = (t >> lgc) & mc, i = t >> (2 * lgc);
            T.r(l + 1)[t] += mx_value_at(T.eb(l + 1), T.u(l + 1), i, j, k, lgc, kcc);
        }
        __syncthreads();
        for (int t = threadIdx.x; t < nc; t += kTailThreads) T.e(l + 1)[t] = T.eb(l + 1)[t];
        __syncthreads();
    }
    mx_tail_sweeps(A, T, A.nlev - 1, A.coarse);
    for (int l = A.nlev - 2; l >= A.l0; --l) {
        const int lg = A.lg[l];
        const int n = 1 << (3 * lg);
        const int m = (1 << lg) - 1;
        for (int t = threadIdx.x; t < n; t += kTailThreads) {
            const int k = t & m, j = (t >> lg) & m, i = t >> (2 * lg);
            T.e(l)[t] += mx_prolong(T.e(l + 1), T.eb(l + 1), i, j, k, lg - 1, A.mode);
        }
        __syncthreads();
        mx_tail_sweeps(A, T, l, A.post);
    }
    for (int t = threadIdx.x; t < n0; t += kTailThreads) A.e[A.l0][t] = T.e(A.l0)[t];
}

// float64 residual of u on the finest level, its float32 copies for the inner
// cycle, and per-block max / sum of squares (thread per 2x2x2 block)
__global__ __launch_bounds__(kBlock) void k_mx_outer_residual(const double *__restrict__ u,
                                                                const double *__restrict__ f, int lg, OpConst kc,
                                                                float *__restrict__ r32, float *__restrict__ u32,
                                                                float *__restrict__ e32,
                                                                double *__restrict__ partial, int nparts, bool split)
{
    __shared__ double sh[2 * kBlock / 64];
    const int lgc = lg - 1;
    const size_t nblk = (size_t)1 << (3 * lgc);
    double mx = 0.0, sm = 0.0;
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < nblk; t += (size_t)gridDim.x * kBlock) {
        const int K = (int)(t & ((1u << lgc) - 1)), J = (int)((t >> lgc) & ((1u << lgc) - 1)),
                  I = (int)(t >> (2 * lgc));
        BlockRes br;
        block_residuals(u, f, I, J, K, lg, kc, br);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const size_t cc = ix(2 * I + a, 2 * J + b, 2 * K + c, lg);
                    const double r = br.r[(a * 2 + b) * 2 + c];
                    const size_t cs = sx(2 * I + a, 2 * J + b, 2 * K + c, lg, split);
                    r32[cs] = (float)r;
                    u32[cc] = (float)u[cc];
                    e32[cs] = 0.0f;
                    mx = nanmax_d(mx, fabs(r));
                    sm += r * r;
                }
    }
    for (int o = 32; o > 0; o >>= 1) {
        mx = nanmax_d(mx, __shfl_xor(mx, o, 64));
        sm += __shfl_xor(sm, o, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[w] = mx;
        sh[kBlock / 64 + w] = sm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kBlock / 64; ++i) {
            mx = nanmax_d(mx, sh[i]);
            sm += sh[kBlock / 64 + i];
        }
        partial[blockIdx.x] = mx;
        partial[nparts + blockIdx.x] = sm;
    }
}

// Float64 outer step of the mixed solve on a level-0 mesh with N >= 64:
// v = u + e (ADD_E) or v = u, then r = f - L(v) at every cell.  Same plane
// march as the colour pass: workgroups of RTJ rows of a 64-cell row tile plus
// a halo row on each side (one wave per row, one cell per lane); v and e^v of
// a plane are staged in LDS, so every exponential is evaluated once per cell
// (plus the halo).  Writes v (ADD_E: into the second buffer uout), r and v as
// float32 for the inner cycle, and per-workgroup max|r| and sum r^2.  Every
// wave issues the same loads in every plane (see k_mx_colour).
constexpr int RTJ = 8, RTK = 64, RLW = RTK + 2;

struct CorrArgs {
    const double *u, *f;
    const float *e;
    double *uout;
    float *r32, *u32;
    int lg, chunk, nunits;
    bool split;
    OpConst kc;
    double *partial;
    int nparts;
    const double *exp2tab;
};

template <bool ADD_E>
__global__ __launch_bounds__(64 * (RTJ + 2)) void k_mx_correct_residual(CorrArgs A)
{
    __shared__ double2 sB[2 * (RTJ + 2) * RLW];
    __shared__ double red[2 * (RTJ + 2)];
    __shared__ double tab[64];
    if (threadIdx.x < 64) tab[threadIdx.x] = A.exp2tab[threadIdx.x];
    __syncthreads();
    const int lg = A.lg, m = (1 << lg) - 1;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int row = wv - 1;
    const bool upd = row >= 0 && row < RTJ;
    const size_t plane = (size_t)1 << (2 * lg);
    const int nkt = (1 << lg) / RTK, njt = (1 << lg) / RTJ;
    // k-halo duty: lanes 0..2 RTJ - 1 of wave 0 serve row lane / 2, side lane & 1
    const bool kh = wv == 0 && lane < 2 * RTJ;
    const int khq = (lane & (2 * RTJ - 1)) >> 1, khs = lane & 1;
    double mx = 0.0, sm = 0.0;
    for (int unit = blockIdx.x; unit < A.nunits; unit += gridDim.x) {
        const int kt = unit % nkt, jt = (unit / nkt) % njt, it = unit / (nkt * njt);
        const int k0 = kt * RTK, j0 = jt * RTJ, i0 = it * A.chunk;
        const int jg = (j0 + row) & m, k = k0 + lane;
        const size_t rowoff = ((size_t)jg << lg) + (size_t)k;
        const int khj = (j0 + khq) & m, khk = khs ? ((k0 + RTK) & m) : ((k0 - 1) & m);
        const size_t khoff = ((size_t)khj << lg) + (size_t)khk;
        auto eidx = [&](int pl, size_t off, int j, int kk) {
            return (size_t)(pl & m) * plane +
                   (A.split ? (((size_t)j << lg) + ((size_t)(((pl & m) + j + kk) & 1) << (lg - 1)) + (size_t)(kk >> 1))
                            : off);
        };
        auto vload = [&](int pl, size_t off, int j, int kk) {
            double v = A.u[(size_t)(pl & m) * plane + off];
            if (ADD_E) v += (double)A.e[eidx(pl, off, j, kk)];
            return v;
        };
        // raw loads of step p (u and e kept apart: they are summed where used,
        // so that no arithmetic on a load in flight sits at the loop latch)
        struct Raw {
            double u, f, ku;
            float e, ke;
        };
        auto load = [&](int p) {
            Raw w;
            w.u = A.u[(size_t)((p + 1) & m) * plane + rowoff];
            w.e = ADD_E ? A.e[eidx(p + 1, rowoff, jg, k)] : 0.f;
            w.f = A.f[(size_t)(p & m) * plane + rowoff];  // halo rows: loaded, not used
            w.ku = A.u[(size_t)(p & m) * plane + khoff];
            w.ke = ADD_E ? A.e[eidx(p, khoff, khj, khk)] : 0.f;
            return w;
        };
        double vm = vload(i0 - 1, rowoff, jg, k), vc = vload(i0, rowoff, jg, k);
        double Em = exp64(vm, tab), Ec = exp64(vc, tab);
        Raw ra = load(i0), rb = load(i0 + 1), rc, rd;  // issued two steps ahead (see k_mx_colour)
        int buf = 0;
        auto step = [&](int p, const Raw &cur, Raw &nxt) {
            nxt = load(p + 2);
            const double vp = cur.u + (double)cur.e, Ep = exp64(vp, tab);
            double2 *B = sB + buf * (RTJ + 2) * RLW;
            B[(row + 1) * RLW + lane + 1] = make_double2(vc, Ec);
            if (kh) {
                const double kv = cur.ku + (double)cur.ke;
                B[(khq + 1) * RLW + (khs ? RLW - 1 : 0)] = make_double2(kv, exp64(kv, tab));
            }
            __syncthreads();
            if (upd) {
                const double2 a = B[row * RLW + lane + 1], b = B[(row + 2) * RLW + lane + 1];
                const double2 c = B[(row + 1) * RLW + lane], d = B[(row + 1) * RLW + lane + 2];
                const double d0 = vp - vc, d1 = vm - vc, d2 = b.x - vc, d3 = a.x - vc, d4 = d.x - vc, d5 = c.x - vc;
                const double S1 = ((d0 + d1) + (d2 + d3)) + (d4 + d5);
                const double S3 = ((Ep * d0 + Em * d1) + (b.y * d2 + a.y * d3)) + (d.y * d4 + c.y * d5);
                const double L = A.kc.ih2 * 0.5 * (S3 + Ec * S1) + A.kc.bC * expm1_64(-A.kc.q * vc, tab);
                const double r = cur.f - L;
                const size_t o = (size_t)(p & m) * plane + rowoff;
                if (ADD_E) A.uout[o] = vc;
                A.u32[o] = (float)vc;
                A.r32[A.split ? (size_t)(p & m) * plane + ((size_t)jg << lg) + ((size_t)(((p & m) + jg + k) & 1) << (lg - 1)) + (size_t)(k >> 1) : o] = (float)r;
                mx = nanmax_d(mx, fabs(r));
                sm += r * r;
            }
            vm = vc;
            Em = Ec;
            vc = vp;
            Ec = Ep;
            buf ^= 1;
        };
        for (int p = i0; p < i0 + A.chunk; p += 4) {
            step(p, ra, rc);
            step(p + 1, rb, rd);
            step(p + 2, rc, ra);
            step(p + 3, rd, rb);
        }
        __syncthreads();  // the next unit reuses the LDS buffers
    }
    for (int o = 32; o > 0; o >>= 1) {
        mx = nanmax_d(mx, __shfl_xor(mx, o, 64));
        sm += __shfl_xor(sm, o, 64);
    }
    if (lane == 0) {
        red[wv] = mx;
        red[RTJ + 2 + wv] = sm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < RTJ + 2; ++w) {
            mx = nanmax_d(mx, red[w]);
            sm += red[RTJ + 2 + w];
        }
        A.partial[blockIdx.x] = mx;
        A.partial[A.nparts + blockIdx.x] = sm;
    }
}

__global__ __launch_bounds__(kBlock) void k_mx_update(double *__restrict__ u, const float *__restrict__ e, int lg,
                                                        bool split)
{
    const size_t n = (size_t)1 << (3 * lg);
    const int m = (1 << lg) - 1;
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (size_t)gridDim.x * kBlock) {
        const int k = (int)(t & m), j = (int)((t >> lg) & m), i = (int)(t >> (2 * lg));
        u[t] += (double)e[sx(i, j, k, lg, split)];
    }
}

__global__ __launch_bounds__(1024) void k_mx_final(const double *__restrict__ partial, int nparts,
                                                    double *__restrict__ out)
{
    __shared__ double sh[32];
    double mx = 0.0, sm = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 1024) {
        mx = nanmax_d(mx, partial[i]);
        sm += partial[nparts + i];
    }
    for (int o = 32; o > 0; o >>= 1) {
        mx = nanmax_d(mx, __shfl_xor(mx, o, 64));
        sm += __shfl_xor(sm, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[threadIdx.x >> 6] = mx;
        sh[16 + (threadIdx.x >> 6)] = sm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 16; ++i) {
            mx = nanmax_d(mx, sh[i]);
            sm += sh[16 + i];
        }
        out[0] = mx;
        out[1] = sm;
    }
}

inline unsigned nb(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

MxConst mx_const(const mgfr_ctx *c, int l)
{
    return MxConst{(float)(1.0 / (c->lev[l].h * c->lev[l].h)), (float)c->bC, (float)c->q, (float)c->p.max_du,
                   (float)c->omega_now};
}

// Levels swept by the one-colour pass kernel store e, r and ebar split by colour.
static bool split_level(const mgfr_ctx *c, int l) { return c->colour32_min_n > 0 && c->lev[l].N >= c->colour32_min_n; }

// Per-launch timing of the finest level's sweep kernels: a pair of events
// around each launch (read back by collect_timing).
static int timer_slot(mgfr_ctx *c, bool timed, int &slot)
{
    slot = -1;
    if (!timed) return MGFR_OK;
    Timer &T = c->sweep_timer;
    if (T.used + 2 > (int)T.ev.size())
        for (int q = 0; q < 16; ++q) {
            hipEvent_t ev;
            MGFR_HIP(hipEventCreate(&ev));
            T.ev.push_back(ev);
        }
    slot = T.used;
    T.used += 2;
    MGFR_HIP(hipEventRecord(T.ev[slot], c->stream));
    return MGFR_OK;
}

static int timer_end(mgfr_ctx *c, int slot)
{
    if (slot >= 0) MGFR_HIP(hipEventRecord(c->sweep_timer.ev[slot + 1], c->stream));
    return MGFR_OK;
}

int mx_launch_sweeps(mgfr_ctx *c, int l, int sweeps, bool timed)
{
    Level &L = c->lev[l];
    const MxConst kc = mx_const(c, l);
    const size_t half = (size_t)1 << (3 * L.lg - 1);
    const bool colour_pass = split_level(c, l);
    int slot, rc;
    for (int s = 0; s < sweeps; ++s) {
        if (colour_pass && c->fused32 && L.e32alt) {
            const int chunk = L.N / kChunks;
            const unsigned nbf = (unsigned)((L.N / CKW) * ((L.N + FI - 1) / FI) * kChunks);
            if ((rc = timer_slot(c, timed, slot))) return rc;
            k_mx_sweep2<<<nbf, 64 * FW, 0, c->stream>>>(Sweep2Args{L.e32, L.e32alt, L.u32, L.r32, L.lg, chunk, kc});
            if ((rc = timer_end(c, slot))) return rc;
            std::swap(L.e32, L.e32alt);
        } else if (colour_pass) {
            const int chunk = L.N / kChunks;
            const unsigned nb = (unsigned)((L.N / CKW) * ((L.N + CTJ - 1) / CTJ) * kChunks);
            for (int colour = 0; colour < 2; ++colour) {
                const ColourArgs A{L.e32, L.u32, L.r32, L.lg, colour, chunk, kc};
                if (l == 0 && c->e32_zero) {  // first pass after a float64 check; not timed
                    k_mx_colour_zero<<<nb, 64 * (CTJ + 2), 0, c->stream>>>(A);
                    c->e32_zero = false;
                    continue;
                }
                if ((rc = timer_slot(c, timed, slot))) return rc;
                k_mx_colour<<<nb, 64 * (CTJ + 2), 0, c->stream>>>(A);
                if ((rc = timer_end(c, slot))) return rc;
            }
        } else {
            for (int colour = 0; colour < 2; ++colour) {
                if ((rc = timer_slot(c, timed, slot))) return rc;
                k_mx_sweep_half<<<nb(half), kBlock, 0, c->stream>>>(L.e32, L.u32, L.r32, L.lg, colour, kc);
                if ((rc = timer_end(c, slot))) return rc;
            }
        }
    }
    MGFR_HIP(hipGetLastError());
    return MGFR_OK;
}

int mx_launch_tail(mgfr_ctx *c, int l0)
{
    MxTail A;
    memset(&A, 0, sizeof A);
    for (int l = 0; l < c->nlev; ++l) {
        A.e[l] = c->lev[l].e32;
        A.u[l] = c->lev[l].u32;
        A.r[l] = c->lev[l].r32;
        A.eb[l] = c->lev[l].ebar32;
        A.ih2[l] = (float)(1.0 / (c->lev[l].h * c->lev[l].h));
        A.lg[l] = c->lev[l].lg;
    }
    A.l0 = l0;
    A.nlev = c->nlev;
    A.pre = c->p.pre_smooth;
    A.post = c->p.post_smooth;
    A.coarse = c->p.coarse_sweeps;
    A.mode = c->p.prolong;
    A.bC = (float)c->bC;
    A.q = (float)c->q;
    A.max_du = (float)c->p.max_du;
    A.omega = (float)c->omega_now;
    k_mx_tail<<<1, kTailThreads, 0, c->stream>>>(A);
    MGFR_HIP(hipGetLastError());
    return MGFR_OK;
}

int mx_vcycle(mgfr_ctx *c, int l)
{
    Level &L = c->lev[l];
    if (L.N <= kTailN) return mx_launch_tail(c, l);
    int rc;
    if ((rc = mx_launch_sweeps(c, l, c->p.pre_smooth, l == 0 && c->timing))) return rc;
    Level &Lc = c->lev[l + 1];
    const size_t nc = (size_t)1 << (3 * Lc.lg);
    const bool sf = split_level(c, l), sc = split_level(c, l + 1);
    if (sf && L.N >= CKW) {
        const int chunk = L.N / 8;
        const unsigned nbk = (unsigned)((L.N / CKW) * (L.N / PTJ) * (L.N / chunk));
        k_mx_restrict_pass<<<nbk, 64 * (PTJ + 2), 0, c->stream>>>(
            RestrictArgs{L.e32, L.u32, L.r32, Lc.ebar32, Lc.u32, Lc.r32, L.lg, chunk, sc, mx_const(c, l)});
    } else {
        k_mx_residual_restrict<<<nb(nc), kBlock, 0, c->stream>>>(L.e32, L.u32, L.r32, L.lg, mx_const(c, l),
                                                                 Lc.ebar32, Lc.u32, Lc.r32, sf, sc);
    }
    k_mx_coarse_rhs<<<nb(nc), kBlock, 0, c->stream>>>(Lc.ebar32, Lc.u32, Lc.lg, mx_const(c, l + 1), Lc.r32, Lc.e32,
                                                      sc);
    MGFR_HIP(hipGetLastError());
    if ((rc = mx_vcycle(c, l + 1))) return rc;
    k_mx_prolong_add<<<nb(nc), kBlock, 0, c->stream>>>(L.e32, Lc.e32, Lc.ebar32, L.lg, c->p.prolong, sf, sc);
    MGFR_HIP(hipGetLastError());
    return mx_launch_sweeps(c, l, c->p.post_smooth, l == 0 && c->timing);
}

}  // namespace

int mixed_alloc(mgfr_ctx *c)
{
    for (int l = 0; l < c->nlev; ++l) {
        Level &L = c->lev[l];
        const size_t bytes = sizeof(float) * (size_t)L.N * L.N * L.N;
        MGFR_HIP(hipMalloc(&L.e32, bytes));
        MGFR_HIP(hipMalloc(&L.r32, bytes));
        MGFR_HIP(hipMalloc(&L.u32, bytes));
        if (l > 0) MGFR_HIP(hipMalloc(&L.ebar32, bytes));
        if (L.N >= CKW) MGFR_HIP(hipMalloc(&L.e32alt, bytes));
    }
    return MGFR_OK;
}

// Float64 residual of the level-0 iterate (also prepares the float32 inner
// problem); returns max|r| and sum r^2 on the host.
static int outer_residual(mgfr_ctx *c, double *rmax, double *rsq)
{
    Level &L0 = c->lev[0];
    const size_t nblk = (size_t)1 << (3 * (L0.lg - 1));
    const unsigned g = (unsigned)std::min<size_t>(nb(nblk), (size_t)c->nparts);
    k_mx_outer_residual<<<g, kBlock, 0, c->stream>>>(L0.u, L0.f, L0.lg, level_const(c, 0), L0.r32, L0.u32, L0.e32,
                                                      c->partial, (int)g, split_level(c, 0));
    k_mx_final<<<1, 1024, 0, c->stream>>>(c->partial, (int)g, c->dscal);
    MGFR_HIP(hipGetLastError());
    MGFR_HIP(hipMemcpyAsync(c->hscal, c->dscal, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    MGFR_HIP(hipStreamSynchronize(c->stream));
    *rmax = c->hscal[0];
    *rsq = c->hscal[1];
    return MGFR_OK;
}

// Outer step: (add_e) u <- u + e, then the float64 residual of u, the inner
// problem's float32 arrays and e = 0; returns max|r| and sum r^2 on the host.
// On meshes with N >= 64 one plane-marching kernel does both (the new iterate
// goes to the second level-0 buffer, which then becomes the current one).
static int outer_step(mgfr_ctx *c, bool add_e, double *rmax, double *rsq)
{
    Level &L0 = c->lev[0];
    const size_t n = (size_t)L0.N * L0.N * L0.N;
    if (L0.N < RTK || L0.alt == nullptr) {
        if (add_e)
            k_mx_update<<<(unsigned)std::min<size_t>(nb(n), 8192), kBlock, 0, c->stream>>>(L0.u, L0.e32, L0.lg,
                                                                                            split_level(c, 0));
        MGFR_HIP(hipGetLastError());
        return outer_residual(c, rmax, rsq);
    }
    CorrArgs A;
    A.u = L0.u;
    A.f = L0.f;
    A.e = L0.e32;
    A.uout = add_e ? L0.alt : nullptr;
    A.r32 = L0.r32;
    A.u32 = L0.u32;
    A.lg = L0.lg;
    A.chunk = L0.N / 8;
    A.nunits = (L0.N / RTK) * (L0.N / RTJ) * 8;
    A.split = split_level(c, 0);
    A.kc = level_const(c, 0);
    A.partial = c->partial;
    A.exp2tab = c->exp2tab;
    const int g = std::min(A.nunits, c->nparts);
    A.nparts = g;
    if (add_e)
        k_mx_correct_residual<true><<<g, 64 * (RTJ + 2), 0, c->stream>>>(A);
    else
        k_mx_correct_residual<false><<<g, 64 * (RTJ + 2), 0, c->stream>>>(A);
    if (add_e) std::swap(L0.u, L0.alt);
    // e = 0: cleared here, or by the first colour pass of the next cycle, which
    // then reads no e and writes the cells it does not update as 0
    c->e32_zero = split_level(c, 0) && c->p.pre_smooth >= 1 && !(c->fused32 && L0.e32alt);
    if (!c->e32_zero) MGFR_HIP(hipMemsetAsync(L0.e32, 0, n * sizeof(float), c->stream));
    k_mx_final<<<1, 1024, 0, c->stream>>>(c->partial, g, c->dscal);
    MGFR_HIP(hipGetLastError());
    MGFR_HIP(hipMemcpyAsync(c->hscal, c->dscal, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    MGFR_HIP(hipStreamSynchronize(c->stream));
    *rmax = c->hscal[0];
    *rsq = c->hscal[1];
    return MGFR_OK;
}

int solve_mixed(mgfr_ctx *c, double *u, mgfr_stats *st, double D)
{
    Level &L0 = c->lev[0];
    const size_t n = (size_t)L0.N * L0.N * L0.N;
    const double ncell = (double)n;
    double rmax, rsq;
    int rc = outer_step(c, false, &rmax, &rsq);
    if (rc) return rc;
    double res = rmax / D, prev = res, prev2 = -1.0;  // prev, prev2: one and two checks back
    st->res0 = res;
    int it = 0, outer = 0, grow = 0, status;
    double rate = 0.5;  // residual reduction per correction cycle, from the last outer step
    c->omega_now = c->omega32;
    for (;;) {
        if (!std::isfinite(res) || grow >= 3) {
            // fall back: plain float64 solve from u = 0 (in the caller's array)
            L0.u = u;
            L0.alt = c->alt0;
            MGFR_HIP(hipMemsetAsync(u, 0, n * sizeof(double), c->stream));
            st->fell_back = 1;
            const int done = it;
            status = solve_fp64_from(c, u, st, D);
            st->outer_iters = done + st->vcycles;
            return status;
        }
        if (res <= c->p.tol) { status = MGFR_OK; break; }
        if (it >= c->p.max_vcycles) { status = MGFR_NOT_CONVERGED; break; }
        // Run up to inner_max correction cycles before the next float64
        // residual, but not past the cycle before the one the measured rate
        // predicts to reach the tolerance: each cycle is a full FAS V-cycle
        // of N_u(e) = r, so only the checks are skipped, and the last cycles
        // are checked one by one.
        int k = 1;
        if (c->inner_max > 1 && rate < 1.0) {
            const double need = std::ceil(std::log(c->p.tol / res) / std::log(rate));
            if (need > 2.0) k = (int)std::min<double>({(double)c->inner_max, need - 1.0, (double)(c->p.max_vcycles - it)});
        }
        for (int j = 0; j < k; ++j)
            if ((rc = mx_vcycle(c, 0))) return rc;
        if ((rc = outer_step(c, true, &rmax, &rsq))) return rc;
        if (c->timing && (rc = collect_timing(c, st))) return rc;
        prev2 = outer >= 1 ? prev : -1.0;
        prev = res;
        res = rmax / D;
        adapt_smoothing(c, res, prev2);
        if (res > 0.0 && prev > 0.0) rate = std::min(1.0, std::pow(res / prev, 1.0 / k));
        grow = (res > prev) ? grow + 1 : 0;
        if (grow) c->omega_now = 1.0;  // over-relaxation off for the rest of the solve once the residual grows
        if (outer < MGFR_MAX_HIST) st->res_hist[outer] = res;
        it += k;
        ++outer;
    }
    st->vcycles = it;
    st->outer_iters = outer;
    st->res = res;
    st->l2res = std::sqrt(rsq / ncell) / D;
    return status;
}

}  // namespace mgfr
