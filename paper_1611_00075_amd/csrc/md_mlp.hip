// Steps a8/a9: the learned descriptor-MLP potential (model in md.h).
//
// Forces, two passes (the shape of the embedded-atom kernels):
//   pass 1a (k_mlp_desc): per atom, the 16 radial descriptors over its list
//     row (8 lanes per atom, as in the pair kernels), evaluated only for
//     the pairs within rc, which are also written out as a compact list;
//   pass 1b (k_mlp_net): per tile of 16 atoms, the network and its backward
//     pass to dE_i/dG_i on the BF16 matrix cores (dE_i/dG_i overwrites G_i);
//   pass 2 (k_mlp_force): per pair of the compact list,
//     s_ij = sum_k (dE_i/dG_ik + dE_j/dG_jk) g_k'(r), F_i -= s_ij R / r.
// Training: k_mlp_grad (forward, loss, backward, weight gradients as
// matrix-core products over atoms, one partial row per wavefront) and
// k_mlp_update (fixed-order sum of the rows, then Adam on FP32 masters).
//
// Matrix-core layout (v_mfma_f32_16x16x32_bf16: A 16x32, B 32x16, D 16x16;
// A row = lane % 16, B column = lane % 16, K slots 8 (lane / 16) + item;
// D column = lane % 16, rows 4 (lane / 16) + r).  Every product is taken
// transposed: weights are the A operand (16 output features by 32 inputs),
// activations the B operand (32 inputs by 16 atoms).  A layer's result in
// lane l is then atom l % 16, features 16 t + 4 g + r (g = l / 16, tile t,
// r < 4), and it packs in registers into the next B operand when the K slot
// (g, item j) of K-step s carries feature 32 s + 4 g + j (j < 4) or
// 32 s + 16 + 4 g + j - 4 (j >= 4); the weight operands are laid out with
// the same order of their input index.  The 22 weight operands (layer 1:
// 4, layer 2: 8, and the transposed ones of the backward pass: 8 + 2) are
// staged once per block in LDS in operand order.
//
// The 16 Gaussians of a pair come from three exponentials: with t = r - c8
// (c8 the centre of Gaussian 8) e_8 = exp(-t^2 / 2w^2), and neighbouring
// Gaussians differ by the factor exp(t dmu / w^2) exp(-(m + 1/2) dmu^2 / w^2)
// going up (its inverse form going down).  The cutoff function is
// cos^2(pi r / 2 rc), with cos and sin from their Taylor series on
// [0, pi/2] (truncation below 1e-8).
#include <cmath>

#include "md_pair.h"

namespace md {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x8 __attribute__((ext_vector_type(8)));

constexpr int kIn = MD_MLP_IN, kHid = MD_MLP_HID, kNP = MD_MLP_NPARAM;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kHid;
static_assert(oB3 + 1 == kNP, "parameter layout");
constexpr int kRow = 5320;                          // partial-gradient row stride (floats)
constexpr int kOpL1 = 0, kOpL2 = 4, kOpB2 = 12, kOpB1 = 20, kOps = 22;
constexpr int kTile = 16;                           // atoms per matrix-core tile
constexpr int kChunk = kTile * (kBlock / kWave);    // atoms per block iteration
constexpr float kLog2e = 1.4426950408889634f;
constexpr int kMaxAtomBlocks = 2048;                // persistent grid of pass 1
constexpr int kMaxGradWaves = 1024;

__device__ __forceinline__ f32x4 mfma(const bf16x8 &a, const bf16x8 &b, const f32x4 &c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }
__device__ __forceinline__ uint16_t f_to_bf16(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }

// Float -> bfloat16 (round to nearest even, v_cvt_pk_bf16_f32).  Vectors of
// bf16 are only ever built whole by a vector conversion: element-wise
// reads and writes of bf16 vectors are avoided (this compiler folds such
// sequences wrongly).
__device__ __forceinline__ bf16x8 pack(const f32x4 &lo, const f32x4 &hi)
{
    const f32x8 v = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    return __builtin_convertvector(v, bf16x8);
}

__device__ __forceinline__ bf16x8 pack8(const float (&u)[8])
{
    const f32x8 v = {u[0], u[1], u[2], u[3], u[4], u[5], u[6], u[7]};
    return __builtin_convertvector(v, bf16x8);
}

// v rounded to bfloat16 (nearest even), as a float: the value pack() stores.
__device__ __forceinline__ float bf16_round(float v)
{
    uint32_t u = __float_as_uint(v);
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

// A matrix-core B operand of NS bfloat16 terms whose sum is the FP32 vector
// it was made from: NS = 1 rounds the activations to bfloat16 (the BF16
// form); NS = 3 splits each value exactly into hi + mid + lo terms (each
// residual is exact in FP32, and 3 x 8 significant bits carry the FP32
// significand), so the product of bfloat16 weights and the split operand,
// accumulated in FP32, is the product with FP32 activations (the
// FP32-activation form).
template <int NS>
struct Opd {
    bf16x8 p[NS];
};

template <int NS>
__device__ __forceinline__ Opd<NS> split8(const float (&u)[8])
{
    Opd<NS> o;
    float r[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) r[j] = u[j];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        o.p[k] = pack8(r);
        if (k + 1 < NS)
#pragma unroll
            for (int j = 0; j < 8; ++j) r[j] -= bf16_round(r[j]);
    }
    return o;
}

template <int NS>
__device__ __forceinline__ Opd<NS> split(const f32x4 &lo, const f32x4 &hi)
{
    const float u[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    return split8<NS>(u);
}

template <int NS>
__device__ __forceinline__ f32x4 mfma_s(const bf16x8 &a, const Opd<NS> &b, f32x4 c)
{
#pragma unroll
    for (int k = 0; k < NS; ++k) c = mfma(a, b.p[k], c);
    return c;
}

__device__ __forceinline__ float sigm(float a)
{
    return __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(-a * kLog2e));
}

// feature carried by K slot (g, j) of K-step s
__device__ __forceinline__ int kslot(int s, int g, int j) { return 32 * s + (j < 4 ? 4 * g + j : 12 + 4 * g + j); }

struct MlpArgs {
    float ax, ay, az;       // L_a / 2^32: displacement per scaled unit (A)
    float rc2;              // rc^2
    float c8;               // mu_8 = mu0 + 8 dmu
    float ka;               // log2(e) / (2 w^2)
    float alpha;            // log2(e) dmu / w^2
    float q[8];             // exp(-(m + 1/2) dmu^2 / w^2)
    float phi;              // pi / (2 rc)
    float iw2, cw;          // 1 / w^2, dmu / w^2
    float mean[kIn], inv_std[kIn];
    Gate gate;
};

MlpArgs make_args(const md_box_t *box, const md_mlp_t *m)
{
    MlpArgs a{};
    const double two32 = 4294967296.0;
    if (box) {
        a.ax = float(box->L[0] / two32);
        a.ay = float(box->L[1] / two32);
        a.az = float(box->L[2] / two32);
    }
    const double w2 = m->width * m->width, l2e = 1.4426950408889634;
    a.rc2 = float(m->rc * m->rc);
    a.c8 = float(m->mu0 + 8.0 * m->dmu);
    a.ka = float(l2e / (2.0 * w2));
    a.alpha = float(l2e * m->dmu / w2);
    for (int k = 0; k < 8; ++k) a.q[k] = float(std::exp(-(k + 0.5) * m->dmu * m->dmu / w2));
    a.phi = float(3.14159265358979323846 / (2.0 * m->rc));
    a.iw2 = float(1.0 / w2);
    a.cw = float(m->dmu / w2);
    for (int k = 0; k < kIn; ++k) {
        a.mean[k] = m->mean[k];
        a.inv_std[k] = m->inv_std[k];
    }
    return a;
}

// ---- pair basis -----------------------------------------------------------

__device__ __forceinline__ void gaussians(const MlpArgs &p, float t, float (&e)[kIn])
{
    e[8] = __builtin_amdgcn_exp2f(-p.ka * t * t);
    const float up = __builtin_amdgcn_exp2f(p.alpha * t), dn = __builtin_amdgcn_exp2f(-p.alpha * t);
#pragma unroll
    for (int m = 0; m < 7; ++m) e[9 + m] = e[8 + m] * (up * p.q[m]);
#pragma unroll
    for (int m = 0; m < 8; ++m) e[7 - m] = e[8 - m] * (dn * p.q[m]);
}

// cos(phi), z = phi^2, 0 <= phi <= pi/2: Taylor series to phi^12
__device__ __forceinline__ float cos_z(float z)
{
    float c = 1.f / 479001600.f;
    c = __builtin_fmaf(c, z, -1.f / 3628800.f);
    c = __builtin_fmaf(c, z, 1.f / 40320.f);
    c = __builtin_fmaf(c, z, -1.f / 720.f);
    c = __builtin_fmaf(c, z, 1.f / 24.f);
    c = __builtin_fmaf(c, z, -0.5f);
    return __builtin_fmaf(c, z, 1.f);
}

// sin(phi), same range: Taylor series to phi^15
__device__ __forceinline__ float sin_z(float ph, float z)
{
    float s = -1.f / 1307674368000.f;
    s = __builtin_fmaf(s, z, 1.f / 6227020800.f);
    s = __builtin_fmaf(s, z, -1.f / 39916800.f);
    s = __builtin_fmaf(s, z, 1.f / 362880.f);
    s = __builtin_fmaf(s, z, -1.f / 5040.f);
    s = __builtin_fmaf(s, z, 1.f / 120.f);
    s = __builtin_fmaf(s, z, -1.f / 6.f);
    return ph * __builtin_fmaf(s, z, 1.f);
}

// ---- weights in LDS -------------------------------------------------------

struct WeightsLds {
    uint16_t ops[kOps][kWave][8];
    float b1[kHid], b2[kHid], w3[kHid];
    float mean[kIn], inv_std[kIn];
    float b3;
};

__device__ void stage_weights(WeightsLds &L, const uint16_t *__restrict__ w, const MlpArgs &p)
{
    for (int e = threadIdx.x; e < kOps * kWave * 8; e += blockDim.x) {
        const int o = e >> 9, lane = (e >> 3) & (kWave - 1), j = e & 7, g = lane >> 4, li = lane & 15;
        uint16_t v = 0;
        if (o < kOpL2) {
            if (g < 2) v = w[oW1 + (16 * o + li) * kIn + 8 * g + j];
        } else if (o < kOpB2) {
            const int t = (o - kOpL2) >> 1, s = (o - kOpL2) & 1;
            v = w[oW2 + (16 * t + li) * kHid + kslot(s, g, j)];
        } else if (o < kOpB1) {
            const int t = (o - kOpB2) >> 1, s = (o - kOpB2) & 1;
            v = w[oW2 + kslot(s, g, j) * kHid + 16 * t + li];
        } else {
            v = w[oW1 + kslot(o - kOpB1, g, j) * kIn + li];
        }
        L.ops[o][lane][j] = v;
    }
    for (int e = threadIdx.x; e < kHid; e += blockDim.x) {
        L.b1[e] = bf16_to_f(w[oB1 + e]);
        L.b2[e] = bf16_to_f(w[oB2 + e]);
        L.w3[e] = bf16_to_f(w[oW3 + e]);
    }
    if (threadIdx.x < kIn) {
        L.mean[threadIdx.x] = p.mean[threadIdx.x];
        L.inv_std[threadIdx.x] = p.inv_std[threadIdx.x];
    }
    if (threadIdx.x == 0) L.b3 = bf16_to_f(w[oB3]);
    __syncthreads();
}

__device__ __forceinline__ bf16x8 op(const WeightsLds &L, int o, int lane)
{
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(L.ops[o][lane]));
}

// ---- the network on one tile of 16 atoms (one wavefront) --------------------

template <int NS>
struct Fwd {
    f32x4 ds1[4], ds2[4];   // silu'(a1), silu'(a2) of lane's atom, features 16t + 4g + r
    f32x4 h[4], h2[4];      // silu(a1) before rounding, silu(a2)
    Opd<NS> h1[2];          // layer-2 B operand
    float E;                // energy of atom lane % 16
};

// silu(a) = a s and silu'(a) = s (1 + a (1 - s)), s = 1 / (1 + exp(-a))
__device__ __forceinline__ float2 silu2(float a)
{
    const float s = sigm(a);
    return make_float2(a * s, s * __builtin_fmaf(a, 1.f - s, 1.f));
}

template <int NS>
__device__ __forceinline__ void forward(const WeightsLds &L, int lane, const Opd<NS> &X, Fwd<NS> &F)
{
    const int g = lane >> 4;
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const f32x4 a = mfma_s<NS>(op(L, kOpL1 + t, lane), X, z);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float2 v = silu2(a[r] + L.b1[16 * t + 4 * g + r]);
            F.h[t][r] = v.x;
            F.ds1[t][r] = v.y;
        }
    }
    F.h1[0] = split<NS>(F.h[0], F.h[1]);
    F.h1[1] = split<NS>(F.h[2], F.h[3]);
    float e = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 a = mfma_s<NS>(op(L, kOpL2 + 2 * t, lane), F.h1[0], z);
        a = mfma_s<NS>(op(L, kOpL2 + 2 * t + 1, lane), F.h1[1], a);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int f = 16 * t + 4 * g + r;
            const float2 v = silu2(a[r] + L.b2[f]);
            F.h2[t][r] = v.x;
            F.ds2[t][r] = v.y;
            e = __builtin_fmaf(L.w3[f], F.h2[t][r], e);
        }
    }
    e += __shfl_xor(e, 16, kWave);
    e += __shfl_xor(e, 32, kWave);
    F.E = e + L.b3;
}

// dE/dx for the tile: lane's atom, input features 4g + r
template <int NS>
__device__ __forceinline__ f32x4 backward_input(const WeightsLds &L, int lane, const Fwd<NS> &F)
{
    const int g = lane >> 4;
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
    f32x4 d[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) d[t][r] = L.w3[16 * t + 4 * g + r] * F.ds2[t][r];
    const Opd<NS> D2[2] = {split<NS>(d[0], d[1]), split<NS>(d[2], d[3])};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 p = mfma_s<NS>(op(L, kOpB2 + 2 * t, lane), D2[0], z);
        p = mfma_s<NS>(op(L, kOpB2 + 2 * t + 1, lane), D2[1], p);
#pragma unroll
        for (int r = 0; r < 4; ++r) d[t][r] = p[r] * F.ds1[t][r];
    }
    const Opd<NS> D1[2] = {split<NS>(d[0], d[1]), split<NS>(d[2], d[3])};
    f32x4 dx = mfma_s<NS>(op(L, kOpB1, lane), D1[0], z);
    return mfma_s<NS>(op(L, kOpB1 + 1, lane), D1[1], dx);
}

// ---- pass 1 / descriptors / network ---------------------------------------

// Descriptor sums of one atom (unreduced over its 8 lanes), in two phases.
// (1) The 8 lanes sweep the row; the distances of the pairs within rc are
// packed into the atom's LDS segment `seg` and, if orow is not NULL, their
// indices into the atom's compact row (the list pass 2 walks).  (2) The
// Gaussians of the packed pairs, 8 at a time, so no lane computes a pair
// beyond rc.  Returns the number of pairs within rc (in all 8 lanes).  All
// lanes of the wave call it (cnt = 0 for atoms past the end).
template <int U>
__device__ __forceinline__ int32_t descriptor(const MlpArgs &p, const uint4 *__restrict__ xs,
                                              const int32_t *__restrict__ row, int32_t cnt, const uint4 &pi,
                                              int sub, int lane, float *seg, int32_t *__restrict__ orow,
                                              float (&G)[kIn])
{
    int32_t base = 0;
    for (int32_t t0 = 0; t0 < cnt; t0 += U * kSlice) {
        int32_t j[U];
        uint4 pj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) j[u] = row[ell_pos(min(t0 + u * kSlice + sub, cnt - 1))];
#pragma unroll
        for (int u = 0; u < U; ++u) pj[u] = xs[j[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            float dx, dy, dz;
            disp<false>(pi, pj[u], p.ax, p.ay, p.az, dx, dy, dz);
            const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
            // the wave's mask of pairs within rc, straight from the compares
            const uint64_t inm = __builtin_amdgcn_ballot_w64(t0 + u * kSlice + sub < cnt) &
                                 __builtin_amdgcn_fcmpf(r2, p.rc2, 4);   // ordered less-than
            const uint32_t gm = uint32_t(inm >> (lane & ~(kSlice - 1))) & 0xffu;
            const int32_t pos = base + __popc(gm & ((1u << sub) - 1u));
            if (__builtin_amdgcn_inverse_ballot_w64(inm)) {
                seg[pos] = __builtin_amdgcn_sqrtf(r2);
                if (orow) orow[ell_pos(pos)] = j[u];
            }
            base += __popc(gm);
        }
    }
    wave_sync();
    for (int32_t q = sub; q < base; q += kSlice) {
        const float r = seg[q];
        float e[kIn];
        gaussians(p, r - p.c8, e);
        const float ph = p.phi * r;
        const float c = cos_z(ph * ph);
        const float fc = c * c;
#pragma unroll
        for (int k = 0; k < kIn; ++k) G[k] = __builtin_fmaf(e[k], fc, G[k]);
    }
    return base;
}

// Sum over the 8 lanes of an atom, scattered: lane `sub` ends with the totals
// of features 2 sub and 2 sub + 1 in v0, v1.
__device__ __forceinline__ void reduce_scatter8(float (&G)[kIn], int sub, float &v0, float &v1)
{
    float a[8], b[4];
    const bool h4 = sub & 4, h2 = sub & 2, h1 = sub & 1;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float keep = h4 ? G[k + 8] : G[k], give = h4 ? G[k] : G[k + 8];
        a[k] = keep + __shfl_xor(give, 4, kWave);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float keep = h2 ? a[k + 4] : a[k], give = h2 ? a[k] : a[k + 4];
        b[k] = keep + __shfl_xor(give, 2, kWave);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float keep = h1 ? b[k + 2] : b[k], give = h1 ? b[k] : b[k + 2];
        (k == 0 ? v0 : v1) = keep + __shfl_xor(give, 1, kWave);
    }
}

// Pass 1a: raw descriptors G[n][16] of one slice of 8 atoms per wavefront
// (8 lanes per atom) and, if idx_in is not NULL, the compact list of the
// pairs within rc.  Dynamic LDS: cap floats per atom of the block.
__global__ __launch_bounds__(kBlock) void k_mlp_desc(int64_t n, MlpArgs p, const uint4 *__restrict__ xs, int32_t cap,
                                                     const int32_t *__restrict__ idx,
                                                     const int32_t *__restrict__ count, float *__restrict__ G,
                                                     int32_t *__restrict__ idx_in, int32_t *__restrict__ cnt_in)
{
    if (gated(p.gate)) return;
    extern __shared__ float seg_lds[];
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const SliceLane sl = slice_lane(blk);
    const int64_t i = sl.i;
    const int sub = sl.sub, lane = threadIdx.x % kWave;
    float g[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) g[k] = 0.f;
    const bool live = i < n;
    const int32_t cnt = live ? min(count[i], cap) : 0;
    const uint4 pi = live ? xs[i] : make_uint4(0, 0, 0, 0);
    float *seg = seg_lds + (threadIdx.x / kSlice) * cap;
    const int32_t nin = descriptor<6>(p, xs, live ? ell_row(idx, i, cap) : idx, cnt, pi, sub, lane, seg,
                                      idx_in && live ? idx_in + (ell_row(idx_in, i, cap) - idx_in) : nullptr, g);
    if (cnt_in && live && sub == 0) cnt_in[i] = nin;
    float v0, v1;
    reduce_scatter8(g, sub, v0, v1);
    if (live) *reinterpret_cast<float2 *>(G + i * kIn + 2 * sub) = make_float2(v0, v1);
}

// Pass 1b: the network on raw descriptors, tiles of 16 atoms per wavefront,
// persistent blocks (the weight operands are staged once per block).
// Energies E_i (e_atom, may be NULL; FP64 block partial in part if not NULL)
// and dE/dG (dEdG, may be NULL).  Gin and dEdG may be the same buffer: a
// wavefront reads its 16 rows before it writes them.
// Two waves per SIMD (at most 256 registers: the compiler would otherwise
// keep every weight operand in registers and run one wave per SIMD).
template <int NS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
void k_mlp_net(int64_t n, MlpArgs p, const float *Gin, const uint16_t *__restrict__ w, float *__restrict__ e_atom,
               float *dEdG, double *__restrict__ part)
{
    if (gated(p.gate)) return;
    __shared__ WeightsLds L;
    __shared__ double red[kBlock / kWave];
    stage_weights(L, w, p);

    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int g = lane >> 4, m = lane & 15;
    const int64_t chunks = (n + kChunk - 1) / kChunk;
    const int64_t c0 = chunks * blk / gridDim.x, c1 = chunks * (blk + 1) / gridDim.x;
    double esum = 0.0;

    // the next chunk's inputs are loaded while the current chunk computes
    float4 n0 = {0.f, 0.f, 0.f, 0.f}, n1 = n0;
    auto fetch = [&](int64_t c) {
        const int64_t i = c * kChunk + int64_t(wave) * kTile + m;
        if (g < 2 && i < n) {
            n0 = *reinterpret_cast<const float4 *>(Gin + i * kIn + 8 * g);
            n1 = *reinterpret_cast<const float4 *>(Gin + i * kIn + 8 * g + 4);
        }
    };
    if (c0 < c1) fetch(c0);
    for (int64_t c = c0; c < c1; ++c) {
        const int64_t i = c * kChunk + int64_t(wave) * kTile + m;
        const float4 u0 = n0, u1 = n1;
        if (c + 1 < c1) fetch(c + 1);
        float u[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (g < 2 && i < n) {
            const float v[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
#pragma unroll
            for (int j = 0; j < 8; ++j) u[j] = (v[j] - L.mean[8 * g + j]) * L.inv_std[8 * g + j];
        }
        const Opd<NS> X = split8<NS>(u);
        Fwd<NS> F;
        forward<NS>(L, lane, X, F);
        if (g == 0 && i < n) {
            if (e_atom) e_atom[i] = F.E;
            esum += double(F.E);
        }
        if (dEdG) {
            const f32x4 dx = backward_input<NS>(L, lane, F);
            if (i < n) {
                float4 o;
                o.x = dx[0] * L.inv_std[4 * g + 0];
                o.y = dx[1] * L.inv_std[4 * g + 1];
                o.z = dx[2] * L.inv_std[4 * g + 2];
                o.w = dx[3] * L.inv_std[4 * g + 3];
                *reinterpret_cast<float4 *>(dEdG + i * kIn + 4 * g) = o;
            }
        }
    }
    if (part) {
        double v[1] = {esum};
        block_sum<1>(v, red);
        if (threadIdx.x == 0) {
            part[int64_t(blk) * 8] = v[0];
            for (int q = 1; q < 8; ++q) part[int64_t(blk) * 8 + q] = 0.0;
        }
    }
}

// ---- pass 2: forces ---------------------------------------------------------

template <int U, bool ENERGY, bool COMP>
__global__ __launch_bounds__(kBlock) void k_mlp_force(int64_t n, MlpArgs p, const uint4 *__restrict__ xs,
                                                      int32_t cap, const int32_t *__restrict__ idx,
                                                      const int32_t *__restrict__ count,
                                                      const float4 *__restrict__ dEdG, float *__restrict__ f,
                                                      double *__restrict__ part)
{
    if (gated(p.gate)) return;
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const SliceLane sl = slice_lane(blk);
    const int64_t i = sl.i;
    const int sub = sl.sub;

    float fx = 0.f, fy = 0.f, fz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
    double w[6] = {0, 0, 0, 0, 0, 0};
    if (i < n) {
        const uint4 pi = xs[i];
        float di[kIn];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 v = dEdG[i * 4 + q];
            di[4 * q] = v.x;
            di[4 * q + 1] = v.y;
            di[4 * q + 2] = v.z;
            di[4 * q + 3] = v.w;
        }
        const int32_t cnt = min(count[i], cap);
        const int32_t *row = ell_row(idx, i, cap);
        for (int32_t t0 = sub; t0 < cnt; t0 += U * kSlice) {
            int32_t j[U];
#pragma unroll
            for (int u = 0; u < U; ++u) j[u] = row[ell_pos(min(t0 + u * kSlice, cnt - 1))];
            uint4 pj[U];
            float4 dj[U][4];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                pj[u] = xs[j[u]];
#pragma unroll
                for (int q = 0; q < 4; ++q) dj[u][q] = dEdG[int64_t(j[u]) * 4 + q];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                float dx, dy, dz;
                disp<false>(pi, pj[u], p.ax, p.ay, p.az, dx, dy, dz);
                const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                const bool in = t0 + u * kSlice < cnt && r2 < p.rc2;
                const float ir = __builtin_amdgcn_rsqf(r2);   // 1/r, and r = r2 / r
                const float r = r2 * ir;
                const float t = r - p.c8;
                float e[kIn];
                gaussians(p, t, e);
                const float ph = p.phi * r, zz = ph * ph;
                const float c = cos_z(zz), s = sin_z(ph, zz);
                const float fc = c * c, dfc = -2.f * p.phi * s * c;
                const float dju[kIn] = {dj[u][0].x, dj[u][0].y, dj[u][0].z, dj[u][0].w,
                                        dj[u][1].x, dj[u][1].y, dj[u][1].z, dj[u][1].w,
                                        dj[u][2].x, dj[u][2].y, dj[u][2].z, dj[u][2].w,
                                        dj[u][3].x, dj[u][3].y, dj[u][3].z, dj[u][3].w};
                // s_ij = sum_k c_k e_k (dfc - fc (t - (k - 8) dmu) / w^2)
                float S0 = 0.f, S1 = 0.f;
#pragma unroll
                for (int k = 0; k < kIn; ++k) {
                    const float qk = (di[k] + dju[k]) * e[k];
                    S0 += qk;
                    S1 = __builtin_fmaf(float(k - 8), qk, S1);
                }
                const float sij = __builtin_fmaf(-fc * t, p.iw2, dfc) * S0 + fc * p.cw * S1;
                const float gs = in ? -sij * ir : 0.f;
                acc_add<COMP>(fx, cx, gs, dx);
                acc_add<COMP>(fy, cy, gs, dy);
                acc_add<COMP>(fz, cz, gs, dz);
                if (ENERGY && in) {
                    w[0] += double(gs * dx * dx); w[1] += double(gs * dy * dy); w[2] += double(gs * dz * dz);
                    w[3] += double(gs * dx * dy); w[4] += double(gs * dx * dz); w[5] += double(gs * dy * dz);
                }
            }
        }
    }
    const double gx = combine(fx, cx), gy = combine(fy, cy), gz = combine(fz, cz);
    if (sub == 0 && i < n) {
        f[i] = float(gx);
        f[n + i] = float(gy);
        f[2 * n + i] = float(gz);
    }
    if (ENERGY) {
        __shared__ double lds[8 * (kBlock / kWave)];
        double v[8] = {0.0, 0.0, w[0], w[1], w[2], w[3], w[4], w[5]};
        block_sum<8>(v, lds);
        if (threadIdx.x == 0)
            for (int c = 0; c < 8; ++c) part[int64_t(blk) * 8 + c] = v[c];
    }
}

// ---- training ---------------------------------------------------------------

struct GradLds {
    uint16_t xT[kIn][2 * kTile];     // [feature][atom of the 32-atom group]
    uint16_t h1T[kHid][2 * kTile];
    uint16_t d2T[kHid][2 * kTile];
    uint16_t d1T[kHid][2 * kTile];
};

__device__ __forceinline__ bf16x8 lds8(const uint16_t *p)
{
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(p));
}

// One partial gradient row per wavefront over a contiguous range of 32-atom
// groups of the batch; part[wave][kNP] (float), lpart[wave] = sum of err^2.
__global__ __launch_bounds__(kBlock) void k_mlp_grad(int64_t batch, const int32_t *__restrict__ sel,
                                                     const float *__restrict__ G, const float *__restrict__ target,
                                                     MlpArgs p, const uint16_t *__restrict__ w, int32_t waves,
                                                     float *__restrict__ part, double *__restrict__ lpart)
{
    __shared__ WeightsLds L;
    __shared__ GradLds S[kBlock / kWave];
    stage_weights(L, w, p);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int g = lane >> 4, m = lane & 15;
    const int64_t wg = int64_t(blockIdx.x) * (kBlock / kWave) + wave;
    if (wg >= waves) return;
    GradLds &T = S[wave];
    const int64_t groups = (batch + 2 * kTile - 1) / (2 * kTile);
    const int64_t q0 = groups * wg / waves, q1 = groups * (wg + 1) / waves;
    const float scale = 2.f / float(batch);
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};

    f32x4 gW2[16], gW1[4];
#pragma unroll
    for (int k = 0; k < 16; ++k) gW2[k] = z;
#pragma unroll
    for (int k = 0; k < 4; ++k) gW1[k] = z;
    float gb1[16], gb2[16], gw3[16], gb3 = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) gb1[k] = gb2[k] = gw3[k] = 0.f;
    double loss = 0.0;

    for (int64_t q = q0; q < q1; ++q) {
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            const int64_t a = q * 2 * kTile + h * kTile + m;
            const bool valid = a < batch;
            const int64_t row = valid ? (sel ? int64_t(sel[a]) : a) : 0;
            bf16x8 X = {};
            if (g < 2) {
                float u[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                if (valid) {
                    const float4 u0 = *reinterpret_cast<const float4 *>(G + row * kIn + 8 * g);
                    const float4 u1 = *reinterpret_cast<const float4 *>(G + row * kIn + 8 * g + 4);
                    const float v[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
#pragma unroll
                    for (int j = 0; j < 8; ++j) u[j] = (v[j] - L.mean[8 * g + j]) * L.inv_std[8 * g + j];
                }
                X = pack8(u);
#pragma unroll
                for (int j = 0; j < 8; ++j) T.xT[8 * g + j][h * kTile + m] = f_to_bf16(u[j]);
            }
            Fwd<1> F;
            forward<1>(L, lane, Opd<1>{{X}}, F);
            const float err = valid ? F.E - target[row] : 0.f;
            const float gE = scale * err;
            if (g == 0) {
                loss += double(err) * double(err);
                gb3 += gE;
            }
            f32x4 d[4];
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int f = 16 * t + 4 * g + r;
                    gw3[4 * t + r] = __builtin_fmaf(gE, F.h2[t][r], gw3[4 * t + r]);
                    d[t][r] = gE * L.w3[f] * F.ds2[t][r];
                    gb2[4 * t + r] += d[t][r];
                    T.d2T[f][h * kTile + m] = f_to_bf16(d[t][r]);
                    T.h1T[f][h * kTile + m] = f_to_bf16(F.h[t][r]);
                }
            const bf16x8 D2[2] = {pack(d[0], d[1]), pack(d[2], d[3])};
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                f32x4 pr = mfma(op(L, kOpB2 + 2 * t, lane), D2[0], z);
                pr = mfma(op(L, kOpB2 + 2 * t + 1, lane), D2[1], pr);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float d1 = pr[r] * F.ds1[t][r];
                    gb1[4 * t + r] += d1;
                    T.d1T[16 * t + 4 * g + r][h * kTile + m] = f_to_bf16(d1);
                }
            }
        }
        wave_sync();
#pragma unroll
        for (int tn = 0; tn < 4; ++tn) {
            const bf16x8 A2 = lds8(&T.d2T[16 * tn + m][8 * g]);
#pragma unroll
            for (int tk = 0; tk < 4; ++tk) gW2[4 * tn + tk] = mfma(A2, lds8(&T.h1T[16 * tk + m][8 * g]), gW2[4 * tn + tk]);
            gW1[tn] = mfma(lds8(&T.d1T[16 * tn + m][8 * g]), lds8(&T.xT[m][8 * g]), gW1[tn]);
        }
        wave_sync();
    }

    // sums over the 16 atoms of a lane group
#pragma unroll
    for (int k = 0; k < 16; ++k)
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            gb1[k] += __shfl_xor(gb1[k], o, kWave);
            gb2[k] += __shfl_xor(gb2[k], o, kWave);
            gw3[k] += __shfl_xor(gw3[k], o, kWave);
        }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
        gb3 += __shfl_xor(gb3, o, kWave);
        loss += __shfl_xor(loss, o, kWave);
    }
    float *out = part + wg * kRow;
#pragma unroll
    for (int tn = 0; tn < 4; ++tn)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int fo = 16 * tn + 4 * g + r;
#pragma unroll
            for (int tk = 0; tk < 4; ++tk) out[oW2 + fo * kHid + 16 * tk + m] = gW2[4 * tn + tk][r];
            out[oW1 + fo * kIn + m] = gW1[tn][r];
            if (m == 0) {
                out[oB1 + fo] = gb1[4 * tn + r];
                out[oB2 + fo] = gb2[4 * tn + r];
                out[oW3 + fo] = gw3[4 * tn + r];
            }
        }
    if (lane == 0) {
        out[oB3] = gb3;
        lpart[wg] = loss;
    }
}

// Fixed-order sum of the partial rows; then either the raw gradient or an
// Adam step (c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t)).
__global__ __launch_bounds__(kBlock) void k_mlp_update(int32_t rows, const float *__restrict__ part,
                                                       const double *__restrict__ lpart, double inv_batch,
                                                       float *__restrict__ grad, double *__restrict__ loss,
                                                       float lr, float b1, float b2, float eps, float c1, float c2,
                                                       float *__restrict__ master, float *__restrict__ m1,
                                                       float *__restrict__ m2, uint16_t *__restrict__ w)
{
    const int pi = blockIdx.x * kBlock + threadIdx.x;
    if (loss && pi == 0) {
        double s = 0.0;
        for (int r = 0; r < rows; ++r) s += lpart[r];
        *loss = s * inv_batch;
    }
    if (pi >= kNP) return;
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += double(part[int64_t(r) * kRow + pi]);
    const float gr = float(s);
    if (grad) grad[pi] = gr;
    if (master) {
        const float a = __builtin_fmaf(b1, m1[pi], (1.f - b1) * gr);
        const float v = __builtin_fmaf(b2, m2[pi], (1.f - b2) * gr * gr);
        m1[pi] = a;
        m2[pi] = v;
        const float x = master[pi] - lr * (a * c1) / (__builtin_sqrtf(v * c2) + eps);
        master[pi] = x;
        w[pi] = f_to_bf16(x);
    }
}

// Per-component sums of G and G^2 (FP64) over a contiguous range of rows per
// block; part[b][32].
__global__ __launch_bounds__(kBlock) void k_mlp_moments(int64_t n, const float *__restrict__ G,
                                                        double *__restrict__ part)
{
    __shared__ double red[2][kBlock];
    const int k = threadIdx.x % kIn, r0 = threadIdx.x / kIn;
    const int64_t b0 = n * blockIdx.x / gridDim.x, b1 = n * (blockIdx.x + 1) / gridDim.x;
    double s = 0.0, ss = 0.0;
    for (int64_t i = b0 + r0; i < b1; i += kBlock / kIn) {
        const double v = double(G[i * kIn + k]);
        s += v;
        ss += v * v;
    }
    red[0][threadIdx.x] = s;
    red[1][threadIdx.x] = ss;
    __syncthreads();
    if (threadIdx.x < kIn) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < kBlock / kIn; ++q) {
            a += red[0][q * kIn + k];
            b += red[1][q * kIn + k];
        }
        part[int64_t(blockIdx.x) * 2 * kIn + k] = a;
        part[int64_t(blockIdx.x) * 2 * kIn + kIn + k] = b;
    }
}

__global__ void k_mlp_moments_final(int64_t n, int32_t blocks, const double *__restrict__ part,
                                    double *__restrict__ out)
{
    const int k = threadIdx.x;
    if (k >= kIn) return;
    double a = 0.0, b = 0.0;
    for (int q = 0; q < blocks; ++q) {
        a += part[int64_t(q) * 2 * kIn + k];
        b += part[int64_t(q) * 2 * kIn + kIn + k];
    }
    const double mean = a / double(n);
    const double var = b / double(n) - mean * mean;
    out[k] = mean;
    out[kIn + k] = var > 0.0 ? sqrt(var) : 0.0;
}

size_t seg_bytes(int32_t cap) { return size_t(kBlock / kSlice) * size_t(cap) * sizeof(float); }

uint32_t slice_blocks(int64_t n) { return uint32_t((n * kSlice + kBlock - 1) / kBlock); }

uint32_t atom_grid(int64_t n)
{
    const int64_t chunks = (n + kChunk - 1) / kChunk;
    return uint32_t(chunks < kMaxAtomBlocks ? chunks : kMaxAtomBlocks);
}

constexpr int kMomentBlocks = 1024;

struct TrainWs {
    size_t part, lpart, moments, total;
};

TrainWs train_ws(int64_t batch)
{
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const int64_t groups = (batch + 2 * kTile - 1) / (2 * kTile);
    const int64_t waves = groups < kMaxGradWaves ? (groups > 0 ? groups : 1) : kMaxGradWaves;
    TrainWs t{};
    size_t o = 0;
    t.part = o;    o += up(size_t(waves) * kRow * 4);
    t.lpart = o;   o += up(size_t(waves) * 8);
    t.moments = o; o += up(size_t(kMomentBlocks) * 2 * kIn * 8);
    t.total = o;
    return t;
}

int32_t grad_waves(int64_t batch)
{
    const int64_t groups = (batch + 2 * kTile - 1) / (2 * kTile);
    return int32_t(groups < kMaxGradWaves ? groups : kMaxGradWaves);
}

}  // namespace

// ---- launchers (argument checks are done by the C ABI) -----------------------

int mlp_descriptors(const md_box_t *box, int64_t n, const uint32_t *xs, int32_t cap, const int32_t *idx,
                    const int32_t *count, const md_mlp_t *mlp, float *G, hipStream_t s)
{
    if (n == 0) return MD_OK;
    const MlpArgs a = make_args(box, mlp);
    hipLaunchKernelGGL(k_mlp_desc, dim3(slice_blocks(n)), dim3(kBlock), seg_bytes(cap), s, n, a,
                       reinterpret_cast<const uint4 *>(xs), cap, idx, count, G, nullptr, nullptr);
    MD_HIP_TRY(hipGetLastError());
    return MD_OK;
}

int mlp_eval(int64_t n, const float *G, const md_mlp_t *mlp, const uint16_t *w, float *e_atom, float *dEdG,
             hipStream_t s)
{
    if (n == 0) return MD_OK;
    const MlpArgs a = make_args(nullptr, mlp);
    if (mlp->activations == MD_MLP_ACT_FP32)
        hipLaunchKernelGGL(k_mlp_net<3>, dim3(atom_grid(n)), dim3(kBlock), 0, s, n, a, G, w, e_atom, dEdG, nullptr);
    else
        hipLaunchKernelGGL(k_mlp_net<1>, dim3(atom_grid(n)), dim3(kBlock), 0, s, n, a, G, w, e_atom, dEdG, nullptr);
    MD_HIP_TRY(hipGetLastError());
    return MD_OK;
}

int forces_mlp(const md_box_t *box, int64_t n, const uint32_t *xs, int32_t cap, const int32_t *idx,
               const int32_t *count, const md_mlp_t *mlp, const uint16_t *w, float *dEdG, int32_t *idx_in,
               int32_t *cnt_in, float *e_atom, float *f, double *ev, int32_t flags, void *ws, const WsLayout &wl,
               hipStream_t s, Gate gate)
{
    const bool energy = flags & MD_ENERGY;
    const bool comp = !(flags & MD_NO_COMPENSATE);
    const bool reuse = flags & MD_MLP_REUSE;
    double *part1 = ws_ptr<double>(ws, wl.red1);
    double *part2 = ws_ptr<double>(ws, wl.red2);
    const uint32_t g1 = n > 0 && !reuse ? atom_grid(n) : 0;
    const uint32_t g2 = n > 0 ? slice_blocks(n) : 0;
    if (int64_t(g1) > wl.red_blocks || int64_t(g2) > wl.red_blocks) return MD_ERR_WORKSPACE;
    MlpArgs a = make_args(box, mlp);
    a.gate = gate;
    const uint4 *q = reinterpret_cast<const uint4 *>(xs);
    if (n > 0) {
        if (!reuse) {
            // pass 1a: descriptors into the dEdG buffer and the compact list;
            // pass 1b: the network overwrites each row with dE/dG in place
            hipLaunchKernelGGL(k_mlp_desc, dim3(g2), dim3(kBlock), seg_bytes(cap), s, n, a, q, cap, idx, count,
                               dEdG, idx_in, cnt_in);
            if (mlp->activations == MD_MLP_ACT_FP32)
                hipLaunchKernelGGL(k_mlp_net<3>, dim3(g1), dim3(kBlock), 0, s, n, a, dEdG, w, e_atom, dEdG,
                                   energy ? part1 : nullptr);
            else
                hipLaunchKernelGGL(k_mlp_net<1>, dim3(g1), dim3(kBlock), 0, s, n, a, dEdG, w, e_atom, dEdG,
                                   energy ? part1 : nullptr);
        }
        const float4 *d4 = reinterpret_cast<const float4 *>(dEdG);
        // pass 2 walks the compact list of pairs within rc (the full list when
        // dE/dG is given)
        const int32_t *pidx = reuse ? idx : idx_in;
        const int32_t *pcnt = reuse ? count : cnt_in;
        if (energy && comp)
            hipLaunchKernelGGL((k_mlp_force<2, true, true>), dim3(g2), dim3(kBlock), 0, s, n, a, q, cap, pidx, pcnt,
                               d4, f, part2);
        else if (energy)
            hipLaunchKernelGGL((k_mlp_force<2, true, false>), dim3(g2), dim3(kBlock), 0, s, n, a, q, cap, pidx, pcnt,
                               d4, f, part2);
        else if (comp)
            hipLaunchKernelGGL((k_mlp_force<2, false, true>), dim3(g2), dim3(kBlock), 0, s, n, a, q, cap, pidx, pcnt,
                               d4, f, part2);
        else
            hipLaunchKernelGGL((k_mlp_force<2, false, false>), dim3(g2), dim3(kBlock), 0, s, n, a, q, cap, pidx, pcnt,
                               d4, f, part2);
        MD_HIP_TRY(hipGetLastError());
    }
    if (energy) return launch_reduce_partials(part1, g1, part2, g2, ev, kReduceEAM, 0.0, 0.0, s);
    return MD_OK;
}

size_t mlp_workspace_bytes(int64_t batch) { return train_ws(batch).total; }

int mlp_moments(int64_t n, const float *G, double *moments, void *tws, hipStream_t s)
{
    const TrainWs t = train_ws(0);
    double *part = ws_ptr<double>(tws, t.moments);
    const int32_t nb = int32_t(n < kMomentBlocks ? (n > 0 ? n : 1) : kMomentBlocks);
    hipLaunchKernelGGL(k_mlp_moments, dim3(nb), dim3(kBlock), 0, s, n, G, part);
    hipLaunchKernelGGL(k_mlp_moments_final, dim3(1), dim3(kWave), 0, s, n, nb, part, moments);
    MD_HIP_TRY(hipGetLastError());
    return MD_OK;
}

int mlp_grad_update(int64_t batch, const int32_t *sel, const float *G, const float *target, const md_mlp_t *mlp,
                    const uint16_t *w_in, float *grad, double *loss, const md_adam_t *adam, float *master, float *m1,
                    float *m2, uint16_t *w_out, void *tws, hipStream_t s)
{
    const TrainWs t = train_ws(batch);
    float *part = ws_ptr<float>(tws, t.part);
    double *lpart = ws_ptr<double>(tws, t.lpart);
    const int32_t waves = grad_waves(batch);
    const MlpArgs a = make_args(nullptr, mlp);
    const uint32_t blocks = uint32_t((waves + kBlock / kWave - 1) / (kBlock / kWave));
    hipLaunchKernelGGL(k_mlp_grad, dim3(blocks), dim3(kBlock), 0, s, batch, sel, G, target, a, w_in, waves, part,
                       lpart);
    float lr = 0.f, b1 = 0.f, b2 = 0.f, eps = 0.f, c1 = 0.f, c2 = 0.f;
    if (adam) {
        lr = float(adam->lr);
        b1 = float(adam->beta1);
        b2 = float(adam->beta2);
        eps = float(adam->eps);
        c1 = float(1.0 / (1.0 - std::pow(adam->beta1, double(adam->step))));
        c2 = float(1.0 / (1.0 - std::pow(adam->beta2, double(adam->step))));
    }
    hipLaunchKernelGGL(k_mlp_update, dim3((kNP + kBlock - 1) / kBlock), dim3(kBlock), 0, s, waves, part, lpart,
                       1.0 / double(batch), grad, loss, lr, b1, b2, eps, c1, c2, adam ? master : nullptr,
                       adam ? m1 : nullptr, adam ? m2 : nullptr, adam ? w_out : nullptr);
    MD_HIP_TRY(hipGetLastError());
    return MD_OK;
}

}  // namespace md
