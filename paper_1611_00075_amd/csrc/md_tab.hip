// Tabulated embedded-atom functions (Sec. 3.1's piecewise-defined psi and
// Phi; Sec. 5: an interpolation table is such a piecewise definition).
//
// Table layout (device, FP32, one float4 per interval): the interpolant on
// interval k in powers of s = (u - u_k)/h in [0, 1],
//   f = a0 + a1 s + a2 s^2 + a3 s^3,   df/du = (a1 + 2 a2 s + 3 a3 s^2)/h,
// psi intervals [0, m), Phi intervals [m, 2m), F intervals [2m, 2m + mf).
// The coefficients are formed on the host in FP64 from the knot values and
// slopes (cubic Hermite: a0 = f_k, a1 = h f'_k, a2 = 3 (f_{k+1} - f_k) -
// h (2 f'_k + f'_{k+1}), a3 = 2 (f_k - f_{k+1}) + h (f'_k + f'_{k+1})).
//
// The two passes are those of the analytic forms (density + embedding, then
// pair forces gathering F'), with one difference: the r tables live in LDS,
// where a lane's lookup is one 16-byte LDS read instead of a second
// scattered global gather beside the neighbour's position.  Staging a table
// per block only pays when a block covers many atoms, so the blocks are
// large (16 waves sharing one copy of the table) and each covers a
// contiguous run of slices of 8 atoms, the runs of one XCD forming one
// contiguous Morton range.  The grid is a few times what is resident at
// once: with exactly one resident round the slowest waves set the time;
// with several, the dispatcher fills the CUs that finish first.
#include <cmath>
#include <type_traits>
#include <vector>

#include "md_pair.h"

namespace md {

constexpr int kTabBlock = 1024;
constexpr uint32_t kTabRounds = 4;   // grid = this many times the resident blocks
constexpr int kTabWaves = kTabBlock / kWave;

struct TAB32 {
    float ax, ay, az;   // L_a / 2^32 (non-cubic boxes)
    float len;          // length unit of the displacements (s or 1)
    float cut2u;        // rc^2 in that unit
    float inv_dr;       // 1 / dr
    float top_r;        // m = number of r intervals, as float
    float inv_drho;
    float top_rho;      // number of rho intervals, as float
    int32_t m, mf;      // r intervals, rho intervals
    Gate gate;
};

// Interval and position in it of u (in units of the knot spacing), clamped
// to [0, top]: k in [0, m-1], s in [0, 1].
__device__ __forceinline__ int tab_cell(float x, float top, int m, float &s)
{
    const float xc = fminf(fmaxf(x, 0.f), top);
    const int k = min(int(xc), m - 1);
    s = xc - float(k);
    return k;
}

__device__ __forceinline__ float tab_val(const float4 &c, float s)
{
    return __builtin_fmaf(__builtin_fmaf(__builtin_fmaf(c.w, s, c.z), s, c.y), s, c.x);
}

// d f / d s
__device__ __forceinline__ float tab_ds(const float4 &c, float s)
{
    return __builtin_fmaf(__builtin_fmaf(3.f * c.w, s, 2.f * c.z), s, c.y);
}

// F(rho) and F'(rho) from the global F table, tangent continuation outside
__device__ __forceinline__ void tab_embed(const TAB32 &p, const float4 *__restrict__ Ftab, float rho, float &F,
                                          float &Fp)
{
    const float x = rho * p.inv_drho;
    float s;
    const int k = tab_cell(x, p.top_rho, p.mf, s);
    const float4 c = Ftab[k];
    const float d = tab_ds(c, s);
    const float ex = x - (float(k) + s);   // 0 inside the table
    F = __builtin_fmaf(d, ex, tab_val(c, s));
    Fp = d * p.inv_drho;
}

// The slices of this wave: XCD x (block b runs on XCD b % 8; the grid is a
// multiple of 8 blocks) owns one contiguous range of slices, cut into one
// contiguous run per block of that XCD; the waves of a block interleave
// over its run.
struct SliceRange {
    uint32_t first, end, stride;
};

__device__ __forceinline__ SliceRange wave_slices(uint32_t nslices)
{
    const uint32_t x = blockIdx.x % kXcds, per_xcd = gridDim.x / kXcds;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint32_t chunk = (nslices + kXcds - 1) / kXcds;
    const uint32_t lo = x * chunk;
    const uint32_t hi = min(lo + chunk, nslices);
    const uint32_t run = (chunk + per_xcd - 1) / per_xcd;
    const uint32_t b0 = lo + (blockIdx.x / kXcds) * run;
    return {b0 + wave, min(b0 + run, hi), uint32_t(kTabWaves)};
}

// Sum of NV doubles over the block's waves, fixed order; valid in thread 0.
template <int NV>
__device__ __forceinline__ void tab_block_sum(double (&v)[NV], double *lds)
{
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] = group_sum(v[c], kWave);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) lds[wave * NV + c] = v[c];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            double t = 0.0;
            for (int w = 0; w < kTabWaves; ++w) t += lds[w * NV + c];
            v[c] = t;
        }
}

// pass 1: rho_i = sum psi(r_ij); F(rho_i), F'_i; F'_i into the fourth word
template <int U, bool CUBIC, bool ENERGY, bool COMP>
__global__ __launch_bounds__(kTabBlock) void k_tab_rho(int64_t n, uint4 *__restrict__ xs, int32_t cap,
                                                       const int32_t *__restrict__ idx,
                                                       const int32_t *__restrict__ count, TAB32 p,
                                                       const float4 *__restrict__ table, float *__restrict__ rho,
                                                       float *__restrict__ fprime, double *__restrict__ part,
                                                       uint32_t nslices)
{
    if (gated(p.gate)) return;
    extern __shared__ float4 lds_tab[];   // psi intervals
    for (int k = threadIdx.x; k < p.m; k += kTabBlock) lds_tab[k] = table[k];
    __syncthreads();
    const float4 *Ftab = table + 2 * p.m;
    const int lane = threadIdx.x % kWave, sub = lane % kSlice;
    const __amdgpu_buffer_rsrc_t xs_r = make_rsrc(xs, uint32_t(n) * 16u);
    double Fsum = 0.0;
    const SliceRange sr = wave_slices(nslices);
    for (uint32_t sl = sr.first; sl < sr.end; sl += sr.stride) {
        const int64_t i = int64_t(sl) * kSlice + lane / kSlice;
        const __amdgpu_buffer_rsrc_t row_r = make_rsrc(idx + int64_t(sl) * cap * kSlice, uint32_t(cap) * 32u);
        float s = 0.f, c = 0.f;
        if (i < n) {
            const uint4 pi = xs[i];
            const int32_t cnt = min(count[i], cap);
            walk_split<U, 3>(xs_r, row_r, cnt, sub, [&](const auto &pj, int32_t t0, auto masked) {
                constexpr int K = sizeof(pj) / sizeof(uint4);
                float bs = 0.f;
#pragma unroll
                for (int u = 0; u < K; ++u) {
                    float dx, dy, dz;
                    disp<CUBIC>(pi, pj[u], p.ax, p.ay, p.az, dx, dy, dz);
                    const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                    float q;
                    const int k = tab_cell(__builtin_amdgcn_sqrtf(r2) * p.len * p.inv_dr, p.top_r, p.m, q);
                    const float psi = tab_val(lds_tab[k], q);
                    bs += ((!decltype(masked)::value || t0 + u * kSlice < cnt) && r2 < p.cut2u) ? psi : 0.f;
                }
                acc_sum<COMP>(s, c, bs);
            });
        }
        const double g = combine(s, c);
        if (sub == 0 && i < n) {
            const float r = float(g);
            float F, Fp;
            tab_embed(p, Ftab, r, F, Fp);
            rho[i] = r;
            fprime[i] = Fp;
            xs[i].w = __float_as_uint(Fp);
            Fsum += double(F);
        }
    }
    if (ENERGY) {
        __shared__ double red[kTabWaves];
        double v[1] = {Fsum};
        tab_block_sum<1>(v, red);
        if (threadIdx.x == 0) {
            part[int64_t(blockIdx.x) * 8] = v[0];
            for (int q = 1; q < 8; ++q) part[int64_t(blockIdx.x) * 8 + q] = 0.0;
        }
    }
}

// pass 2: F_i = -sum_j [(F'_i + F'_j) psi'(r) + Phi'(r)] (r_i - r_j) / r
template <int U, bool CUBIC, bool ENERGY, bool COMP>
__global__ __launch_bounds__(kTabBlock) void k_tab_force(int64_t n, const uint4 *__restrict__ xs, int32_t cap,
                                                         const int32_t *__restrict__ idx,
                                                         const int32_t *__restrict__ count, TAB32 p,
                                                         const float4 *__restrict__ table,
                                                         const float *__restrict__ rho, float *__restrict__ f,
                                                         float *__restrict__ e_atom, double *__restrict__ part,
                                                         uint32_t nslices)
{
    if (gated(p.gate)) return;
    extern __shared__ float4 lds_tab[];   // psi intervals, then Phi intervals
    for (int k = threadIdx.x; k < 2 * p.m; k += kTabBlock) lds_tab[k] = table[k];
    __syncthreads();
    const float4 *Ftab = table + 2 * p.m;
    const int lane = threadIdx.x % kWave, sub = lane % kSlice;
    const __amdgpu_buffer_rsrc_t xs_r = make_rsrc(xs, uint32_t(n) * 16u);
    double e = 0.0, w[6] = {0, 0, 0, 0, 0, 0};
    const SliceRange sr = wave_slices(nslices);
    for (uint32_t sl = sr.first; sl < sr.end; sl += sr.stride) {
        const int64_t i = int64_t(sl) * kSlice + lane / kSlice;
        const __amdgpu_buffer_rsrc_t row_r = make_rsrc(idx + int64_t(sl) * cap * kSlice, uint32_t(cap) * 32u);
        float fx = 0.f, fy = 0.f, fz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
        double ei = 0.0;
        if (i < n) {
            const uint4 pi = xs[i];
            const float fpi = __uint_as_float(pi.w);
            const int32_t cnt = min(count[i], cap);
            walk_split<U, 4>(xs_r, row_r, cnt, sub, [&](const auto &pj, int32_t t0, auto masked) {
                constexpr int K = sizeof(pj) / sizeof(uint4);
                float bx = 0.f, by = 0.f, bz = 0.f;
#pragma unroll
                for (int u = 0; u < K; ++u) {
                    float dx, dy, dz;
                    disp<CUBIC>(pi, pj[u], p.ax, p.ay, p.az, dx, dy, dz);
                    const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                    const bool in = (!decltype(masked)::value || t0 + u * kSlice < cnt) && r2 < p.cut2u;
                    const float ir = __builtin_amdgcn_rsqf(r2);   // 1/r and r = r2 / r
                    float q;
                    const int k = tab_cell(r2 * ir * p.len * p.inv_dr, p.top_r, p.m, q);
                    const float4 cp = lds_tab[k], cf = lds_tab[p.m + k];
                    const float fsum = fpi + __uint_as_float(pj[u].w);
                    // dU/dr = [(F'_i + F'_j) dpsi/ds + dPhi/ds] / dr; g = -(dU/dr) / r_u
                    const float dUds = __builtin_fmaf(fsum, tab_ds(cp, q), tab_ds(cf, q));
                    float g = -dUds * p.inv_dr * ir;
                    g = in ? g : 0.f;
                    bx = __builtin_fmaf(g, dx, bx);
                    by = __builtin_fmaf(g, dy, by);
                    bz = __builtin_fmaf(g, dz, bz);
                    if (ENERGY && in) {
                        ei += double(tab_val(cf, q));
                        w[0] += double(g * dx * dx); w[1] += double(g * dy * dy); w[2] += double(g * dz * dz);
                        w[3] += double(g * dx * dy); w[4] += double(g * dx * dz); w[5] += double(g * dy * dz);
                    }
                }
                acc_sum<COMP>(fx, cx, bx);
                acc_sum<COMP>(fy, cy, by);
                acc_sum<COMP>(fz, cz, bz);
            });
        }
        const double gx = combine(fx, cx), gy = combine(fy, cy), gz = combine(fz, cz);
        if (sub == 0 && i < n) {
            f[i] = float(gx);
            f[n + i] = float(gy);
            f[2 * n + i] = float(gz);
        }
        if (ENERGY) {
            e += ei;
            if (e_atom) {
                // site energy F(rho_i) + 1/2 sum_j Phi(r_ij)
                double es = ei;
#pragma unroll
                for (int o = 1; o < kSlice; o <<= 1) es += __shfl_xor(es, o, kWave);
                if (sub == 0 && i < n) {
                    float F, Fp;
                    tab_embed(p, Ftab, rho[i], F, Fp);
                    e_atom[i] = float(double(F) + 0.5 * es);
                }
            }
        }
    }
    if (ENERGY) {
        __shared__ double red[8 * kTabWaves];
        const double u = double(p.len);
        double v[8] = {e, 0.0, w[0] * u, w[1] * u, w[2] * u, w[3] * u, w[4] * u, w[5] * u};
        tab_block_sum<8>(v, red);
        if (threadIdx.x == 0)
            for (int c = 0; c < 8; ++c) part[int64_t(blockIdx.x) * 8 + c] = v[c];
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
constexpr int kTabUnroll = 4;

bool tab_ok(const md_tab_t *t)
{
    return t && t->nr >= 2 && t->nr <= MD_TAB_MAX_KNOTS && t->nrho >= 2 && t->nrho <= MD_TAB_MAX_RHO_KNOTS &&
           std::isfinite(t->dr) && t->dr > 0.0 && std::isfinite(t->drho) && t->drho > 0.0;
}

int64_t tab_bytes(const md_tab_t *t)
{
    return tab_ok(t) ? 32 * int64_t(t->nr - 1) + 16 * int64_t(t->nrho - 1) : 0;
}

int tab_pack(const md_tab_t *t, const double *psi, const double *dpsi, const double *phi, const double *dphi,
             const double *F, const double *dF, void *table, hipStream_t s)
{
    const int64_t m = t->nr - 1, mf = t->nrho - 1;
    std::vector<float> h(size_t(4 * (2 * m + mf)));
    auto fill = [&](float *out, const double *v, const double *dv, int64_t cnt, double step) {
        for (int64_t k = 0; k < cnt; ++k) {
            const double f0 = v[k], f1 = v[k + 1], m0 = step * dv[k], m1 = step * dv[k + 1];
            out[4 * k + 0] = float(f0);
            out[4 * k + 1] = float(m0);
            out[4 * k + 2] = float(3.0 * (f1 - f0) - (2.0 * m0 + m1));
            out[4 * k + 3] = float(2.0 * (f0 - f1) + (m0 + m1));
        }
    };
    for (int64_t k = 0; k <= m; ++k)
        if (!std::isfinite(psi[k]) || !std::isfinite(dpsi[k]) || !std::isfinite(phi[k]) || !std::isfinite(dphi[k]))
            return MD_ERR_ARG;
    for (int64_t k = 0; k <= mf; ++k)
        if (!std::isfinite(F[k]) || !std::isfinite(dF[k])) return MD_ERR_ARG;
    fill(h.data(), psi, dpsi, m, t->dr);
    fill(h.data() + 4 * m, phi, dphi, m, t->dr);
    fill(h.data() + 8 * m, F, dF, mf, t->drho);
    MD_HIP_TRY(hipMemcpyAsync(table, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, s));
    MD_HIP_TRY(hipStreamSynchronize(s));
    return MD_OK;
}

// Blocks of the grid: kTabRounds times as many as fit on the device at once
// for this kernel and LDS size, a multiple of 8, no more than the slices
// need.
static uint32_t tab_grid(const void *kernel, size_t lds, uint32_t nslices)
{
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (cus[dev] == 0) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
        cus[dev] = c;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kTabBlock, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const uint32_t full = uint32_t(cus[dev]) * uint32_t(per_cu) * kTabRounds;
    const uint32_t need = (nslices + kTabWaves - 1) / kTabWaves;
    const uint32_t g = need < full ? need : full;
    return (g + kXcds - 1) / kXcds * kXcds;
}

template <bool CUBIC, bool E, bool C>
static int launch_tab(hipStream_t s, int64_t n, uint4 *q, int32_t cap, const int32_t *idx, const int32_t *cnt,
                      const TAB32 &p, const float4 *table, float *rho, float *fprime, float *f, float *ea,
                      double *part1, double *part2, int64_t max_blocks, uint32_t &g1, uint32_t &g2)
{
    const uint32_t nslices = uint32_t((n + kSlice - 1) / kSlice);
    const size_t lds1 = size_t(p.m) * 16, lds2 = size_t(p.m) * 32;
    g1 = tab_grid(reinterpret_cast<const void *>(&k_tab_rho<kTabUnroll, CUBIC, E, C>), lds1, nslices);
    g2 = tab_grid(reinterpret_cast<const void *>(&k_tab_force<kTabUnroll, CUBIC, E, C>), lds2, nslices);
    if (int64_t(g1) > max_blocks || int64_t(g2) > max_blocks) return MD_ERR_WORKSPACE;
    hipLaunchKernelGGL((k_tab_rho<kTabUnroll, CUBIC, E, C>), dim3(g1), dim3(kTabBlock), lds1, s, n, q, cap, idx, cnt,
                       p, table, rho, fprime, part1, nslices);
    hipLaunchKernelGGL((k_tab_force<kTabUnroll, CUBIC, E, C>), dim3(g2), dim3(kTabBlock), lds2, s, n, q, cap, idx,
                       cnt, p, table, rho, f, ea, part2, nslices);
    MD_HIP_TRY(hipGetLastError());
    return MD_OK;
}

int forces_tab(const md_box_t *box, int64_t n, uint32_t *xs, int32_t cap, const int32_t *idx, const int32_t *cnt,
               const md_tab_t *tab, const void *table, float *rho, float *fprime, float *f, float *e_atom,
               double *ev, int32_t flags, void *ws, const WsLayout &w, hipStream_t s, Gate gate)
{
    const double two32 = 4294967296.0;
    const bool cubic = box->L[0] == box->L[1] && box->L[1] == box->L[2];
    const double u = cubic ? box->L[0] / two32 : 1.0;
    const double rc = (tab->nr - 1) * tab->dr;
    TAB32 p;
    p.ax = float(box->L[0] / two32);
    p.ay = float(box->L[1] / two32);
    p.az = float(box->L[2] / two32);
    p.len = float(u);
    p.cut2u = float(rc * rc / (u * u));
    p.inv_dr = float(1.0 / tab->dr);
    p.m = tab->nr - 1;
    p.top_r = float(p.m);
    p.inv_drho = float(1.0 / tab->drho);
    p.mf = tab->nrho - 1;
    p.top_rho = float(p.mf);
    p.gate = gate;
    const bool energy = flags & MD_ENERGY;
    const bool comp = !(flags & MD_NO_COMPENSATE);
    double *part1 = ws_ptr<double>(ws, w.red1);
    double *part2 = ws_ptr<double>(ws, w.red2);
    uint4 *q = reinterpret_cast<uint4 *>(xs);
    const float4 *t = static_cast<const float4 *>(table);
    uint32_t g1 = 0, g2 = 0;
    if (n > 0) {
        auto go = [&](auto cub, auto en, auto co) {
            return launch_tab<decltype(cub)::value, decltype(en)::value, decltype(co)::value>(
                s, n, q, cap, idx, cnt, p, t, rho, fprime, f, e_atom, part1, part2, w.red_blocks, g1, g2);
        };
        using T = std::true_type;
        using F = std::false_type;
        int rc_;
        if (cubic) rc_ = energy ? (comp ? go(T{}, T{}, T{}) : go(T{}, T{}, F{})) : (comp ? go(T{}, F{}, T{}) : go(T{}, F{}, F{}));
        else rc_ = energy ? (comp ? go(F{}, T{}, T{}) : go(F{}, T{}, F{})) : (comp ? go(F{}, F{}, T{}) : go(F{}, F{}, F{}));
        if (rc_ != MD_OK) return rc_;
    }
    if (energy) return launch_reduce_partials(part1, g1, part2, g2, ev, kReduceEAM, 0.0, 0.0, s);
    return MD_OK;
}

}  // namespace md
