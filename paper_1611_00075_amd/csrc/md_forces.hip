// Steps a4-a6: Lennard-Jones and embedded-atom forces over full Verlet lists
// (the two-pass embedded-atom kernels serve both the Finnis-Sinclair form
// and the exponential second-moment tight-binding form of Sec. 3.1).
//
// The pair loop of the paper (Sec. 2.2) visits each pair once and scatters
// -F into f_j; the paper avoids the resulting write races with its cell-task
// schedule.  Here every atom's row holds all its neighbours, so each pair is
// evaluated from both sides and every force is written once by its owner:
// no atomics and bitwise-reproducible results.
//
// Lists are sliced ELL: slices of 8 atoms whose rows are interleaved in
// blocks of 8 entries.  A wave holds one slice, 8 consecutive lanes per atom,
// so each load of 64 indices reads one contiguous 256-byte run.  Each lane
// fetches U list entries and then U positions before using any, so U
// independent gathers per lane are in flight.  Rows are walked with raw
// buffer loads: a slot past the row's end gets an out-of-range offset,
// which returns zeros without memory traffic, so no load is predicated.
// The 8 partial sums of an atom are combined in FP64 with lane shuffles.
//
// FP32 path: displacements come from 32-bit scaled coordinates (fraction of
// the box times 2^32, Sec. 4.1 "fetch"/"dist"): the integer difference is the
// periodic minimum image.  In a cubic box all lengths are kept in units of
// s = L/2^32 (cutoffs and constants are pre-scaled on the host); the unit
// vector of a pair does not depend on the unit.  Pair arithmetic is FP32;
// per-lane sums are Kahan-compensated unless MD_NO_COMPENSATE.
#include <cmath>

#include "md_pair.h"


namespace md {

// ---------------------------------------------------------------------------
// Lennard-Jones, FP32 pair arithmetic
// ---------------------------------------------------------------------------
struct LJ32 {
    float ax, ay, az;       // L_a / 2^32 (non-cubic boxes)
    float len;              // length unit of the displacements (s or 1)
    float rc2, sig2, eps4, eps24;  // rc^2, sigma^2 in that unit; 4 eps; 24 eps / unit
    Gate gate;
};

template <int TPA, int U, bool CUBIC, bool ENERGY, bool COMP>
__global__ __launch_bounds__(kBlock) void k_lj32(int64_t n, const uint4 *__restrict__ xs,
                                                 int32_t cap, const int32_t *__restrict__ idx,
                                                 const int32_t *__restrict__ count, LJ32 p, float *__restrict__ f,
                                                 double *__restrict__ part, Span sp, const BrickTab *tab)
{
    if (gated(p.gate)) return;
    static_assert(TPA == kSlice, "one slice per wave");
    const uint32_t lblk = xcd_block(blockIdx.x, gridDim.x);   // partial rows by the launch's block
    uint32_t blk = lblk;
    if (tab) {
        const BrickSel e = brick_select(tab, lblk);
        blk = e.blk;
        xs += e.slot0;
        idx += e.slot0 * cap;
        count += e.slot0;
        f += e.atom0;
        n = e.n_end;
        sp.n_xs = e.n_xs;
        sp.slice0 = e.slice0;
    }
    const SliceLane sl = slice_lane(blk, sp.slice0);
    const int64_t i = sl.i;
    const int sub = sl.sub;

    const SliceBufs b = slice_bufs(xs, sp.n_xs, idx, cap, blk, sp.slice0);
    float fx = 0.f, fy = 0.f, fz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
    double e = 0.0, np = 0.0, w[6] = {0, 0, 0, 0, 0, 0};
    if (i < n) {
        const uint4 pi = xs[i];
        const int32_t cnt = min(count[i], cap);
        // a batch's pair forces are summed plainly, the sum added compensated
        walk_split<U, 3>(b.xs, b.row, cnt, sub, [&](const auto &pj, int32_t t, auto masked) {
            constexpr int K = sizeof(pj) / sizeof(uint4);
            float bx = 0.f, by = 0.f, bz = 0.f;
#pragma unroll
            for (int u = 0; u < K; ++u) {
                float dx, dy, dz;
                disp<CUBIC>(pi, pj[u], p.ax, p.ay, p.az, dx, dy, dz);
                const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                const bool in = (!decltype(masked)::value || t + u * TPA < cnt) && r2 < p.rc2;
                const float ir2 = __builtin_amdgcn_rcpf(r2);
                const float s2 = p.sig2 * ir2;
                const float s6 = s2 * s2 * s2;
                // 24 eps s6 (2 s6 - 1) / r^2 with the prefactor folded into the bracket
                float fs = s6 * __builtin_fmaf(2.f * p.eps24, s6, -p.eps24) * ir2;
                fs = in ? fs : 0.f;
                bx = __builtin_fmaf(fs, dx, bx);
                by = __builtin_fmaf(fs, dy, by);
                bz = __builtin_fmaf(fs, dz, bz);
                if (ENERGY && in) {
                    e += double(p.eps4 * (s6 * s6 - s6));
                    np += 1.0;
                    w[0] += double(fs * dx * dx); w[1] += double(fs * dy * dy); w[2] += double(fs * dz * dz);
                    w[3] += double(fs * dx * dy); w[4] += double(fs * dx * dz); w[5] += double(fs * dy * dz);
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
        f[sp.fs + i] = float(gy);
        f[2 * sp.fs + i] = float(gz);
    }
    if (ENERGY) {
        __shared__ double lds[8 * (kBlock / kWave)];
        const double u = double(p.len);   // virial back to physical units
        double v[8] = {e, np, w[0] * u, w[1] * u, w[2] * u, w[3] * u, w[4] * u, w[5] * u};
        block_sum<8>(v, lds);
        if (threadIdx.x == 0)
            for (int c = 0; c < 8; ++c) part[int64_t(lblk) * 8 + c] = v[c];
    }
}

// ---------------------------------------------------------------------------
// Lennard-Jones, FP64 pair arithmetic (minimum image as in the list build)
// ---------------------------------------------------------------------------
struct LJ64 {
    double L[3], hL[3];
    double rc2, sig2, eps4, eps24;
    Gate gate;
};

__device__ __forceinline__ double minimg64(double d, double L, double hL)
{
    if (d > hL)
        d -= L;
    else if (d < -hL)
        d += L;
    return d;
}

template <int TPA, bool ENERGY>
__global__ __launch_bounds__(kBlock) void k_lj64(int64_t n, const double *__restrict__ x,
                                                 int32_t cap, const int32_t *__restrict__ idx,
                                                 const int32_t *__restrict__ count, LJ64 p, double *__restrict__ f,
                                                 double *__restrict__ part)
{
    if (gated(p.gate)) return;
    static_assert(TPA == kSlice, "one slice per wave");
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const SliceLane sl = slice_lane(blk);
    const int64_t i = sl.i;
    const int sub = sl.sub;

    double fx = 0, fy = 0, fz = 0, e = 0, np = 0, w[6] = {0, 0, 0, 0, 0, 0};
    if (i < n) {
        const double xi = x[i], yi = x[n + i], zi = x[2 * n + i];
        const int32_t cnt = min(count[i], cap);
        const int32_t *row = ell_row(idx, i, cap);
        for (int32_t k = sub; k < cnt; k += TPA) {
            const int64_t j = row[ell_pos(k)];
            // displacement i -> j as in the plain definition, then R = -d
            const double dx = minimg64(x[j] - xi, p.L[0], p.hL[0]);
            const double dy = minimg64(x[n + j] - yi, p.L[1], p.hL[1]);
            const double dz = minimg64(x[2 * n + j] - zi, p.L[2], p.hL[2]);
            const double r2 = (dx * dx + dy * dy) + dz * dz;
            if (r2 < p.rc2) {
                const double s2 = p.sig2 / r2;
                const double s6 = s2 * s2 * s2;
                const double fs = p.eps24 * (2.0 * s6 * s6 - s6) / r2;
                fx -= fs * dx;
                fy -= fs * dy;
                fz -= fs * dz;
                if (ENERGY) {
                    e += p.eps4 * (s6 * s6 - s6);
                    np += 1.0;
                    w[0] += fs * dx * dx; w[1] += fs * dy * dy; w[2] += fs * dz * dz;
                    w[3] += fs * dx * dy; w[4] += fs * dx * dz; w[5] += fs * dy * dz;
                }
            }
        }
    }
#pragma unroll
    for (int o = 1; o < kSlice; o <<= 1) {
        fx += __shfl_xor(fx, o, kWave);
        fy += __shfl_xor(fy, o, kWave);
        fz += __shfl_xor(fz, o, kWave);
    }
    if (sub == 0 && i < n) {
        f[i] = fx;
        f[n + i] = fy;
        f[2 * n + i] = fz;
    }
    if (ENERGY) {
        __shared__ double lds[8 * (kBlock / kWave)];
        double v[8] = {e, np, w[0], w[1], w[2], w[3], w[4], w[5]};
        block_sum<8>(v, lds);
        if (threadIdx.x == 0)
            for (int c = 0; c < 8; ++c) part[int64_t(blk) * 8 + c] = v[c];
    }
}

// ---------------------------------------------------------------------------
// embedded-atom method (Finnis-Sinclair), FP32 pair arithmetic
// ---------------------------------------------------------------------------
// The pair polynomial c0 + c1 r + c2 r^2 cancels strongly at first-neighbour
// distances (about 65x for the Cu-like set); it is evaluated in powers of
// t = r - c instead, p0 + p1 t + p2 t^2, with p_k formed on the host in FP64.
struct FS32 {
    float ax, ay, az;       // L_a / 2^32 (non-cubic boxes)
    float len;              // length unit of the displacements (s or 1)
    float d2u, c2u;         // d^2, c^2 in that unit
    float d, c, p0, p1, p2, A;  // physical
    Gate gate;
    static constexpr int kRhoWords = 3;   // words of a neighbour's scaled coordinates pass 1 reads
    static constexpr bool kSplit = true;  // row walk: full batches, then one masked tail batch
    static constexpr int kRhoUnroll = 4;  // row entries per lane per batch in pass 1 (measured)
};

// Second-moment tight-binding form: psi = exp2(cq - kq r) S(r),
// Phi = exp2(cp - kp r) S(r), F = -A sqrt(rho) with A = 1; the constants
// fold xi^2, 2A, r0 and the exponents (kq = 2q log2(e)/r0, lq = 2q/r0, ...).
struct TB32 {
    float ax, ay, az;       // L_a / 2^32 (non-cubic boxes)
    float len;              // length unit of the displacements (s or 1)
    float cut2u;            // rc^2 in that unit
    float rs, iw;           // switch start, 1 / (rc - rs)
    float kq, cq, lq;       // density: exponent slope (base 2), offset, slope (base e)
    float kp, cp, lp;       // pair function, likewise
    float A;                // embedding prefactor (1)
    Gate gate;
    static constexpr int kRhoWords = 3;
    static constexpr bool kSplit = true;
    static constexpr int kRhoUnroll = 6;  // exponentials per pair: deeper batches pay (measured)
};

// Two elements: the tight-binding constants per pair kind k = t_i + t_j
// (0: 0-0, 1: 0-1, 2: 1-1).  The element of atom i is bit 0 of the fourth
// word of its scaled coordinates (on entry the element itself; after pass 1
// F'_i with its lowest mantissa bit replaced by the element).  With
// COMMON_CUT all kinds share the smooth cutoff (kind 0's values are used),
// which leaves four constants to choose per pair; the base-e slopes follow
// from the base-2 ones (l = k ln 2).
template <bool COMMON_CUT>
struct TBM32 {
    float ax, ay, az;       // L_a / 2^32 (non-cubic boxes)
    float len;              // length unit of the displacements (s or 1)
    float cut2u[3], rs[3], iw[3];
    float kq[3], cq[3];
    float kp[3], cp[3];
    float A;                // embedding prefactor (1)
    Gate gate;
    static constexpr int kRhoWords = 4;
    // whole batches without selects, slots past the row end masked in the
    // pair term: the longer pair terms favour fewer selects over fewer slots
    static constexpr bool kSplit = false;
    static constexpr int kRhoUnroll = 6;
};

// ---- pair terms of the forms ------------------------------------------------
// rho_term: psi(r) of a listed pair (0 when not counted); force_term: the
// force factor g = -(dU/dr)/r_u (F_i = g d, d in the displacement unit) and
// the pair energy of the pair.  wi, wj: the fourth words of the two atoms'
// scaled coordinates (F' after pass 1); fprime_word: the word pass 1 stores.

struct PairOut {
    float g, v;
    bool in;
};

__device__ __forceinline__ float rho_term(const FS32 &p, float r2, bool valid, uint32_t, uint32_t)
{
    const float t = __builtin_amdgcn_sqrtf(r2) * p.len - p.d;
    return (valid && r2 < p.d2u) ? t * t : 0.f;
}

__device__ __forceinline__ PairOut force_term(const FS32 &p, float r2, bool valid, uint32_t wi, uint32_t wj)
{
    const float fsum = __uint_as_float(wi) + __uint_as_float(wj);
    const bool in_d = valid && r2 < p.d2u, in_c = valid && r2 < p.c2u;
    // one reciprocal square root gives both r and 1/r
    const float ir = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * ir * p.len;
    const float dpsi = in_d ? fsum * 2.f * (r - p.d) : 0.f;
    const float t = r - p.c;
    const float poly = __builtin_fmaf(__builtin_fmaf(p.p2, t, p.p1), t, p.p0);
    const float dpoly = __builtin_fmaf(2.f * p.p2, t, p.p1);
    const float dV = in_c ? t * __builtin_fmaf(t, dpoly, 2.f * poly) : 0.f;
    float g = -(dpsi + dV) * ir;
    g = in_d || in_c ? g : 0.f;
    return {g, in_c ? t * t * poly : 0.f, in_d || in_c};
}

__device__ __forceinline__ uint32_t fprime_word(const FS32 &, float fp, uint32_t) { return __float_as_uint(fp); }

// S(r) and dS/dr of the smooth cutoff, branch-free (x clamped to [0, 1])
__device__ __forceinline__ void tb_switch(float r, float rs, float iw, float &S, float &dS)
{
    const float x = fminf(fmaxf((r - rs) * iw, 0.f), 1.f);
    const float x2 = x * x, y = 1.f - x;
    S = __builtin_fmaf(-x2 * x, __builtin_fmaf(__builtin_fmaf(6.f, x, -15.f), x, 10.f), 1.f);
    dS = -30.f * iw * x2 * y * y;
}

// the tight-binding pair terms from one kind's constants
__device__ __forceinline__ float tb_psi(float r, float rs, float iw, float kq, float cq)
{
    float S, dS;
    tb_switch(r, rs, iw, S, dS);
    return __builtin_amdgcn_exp2f(__builtin_fmaf(-kq, r, cq)) * S;
}

// (ir = 1 / r in the displacement unit)
__device__ __forceinline__ float2 tb_force(float r, float ir, float fsum, float rs, float iw, float kq, float cq,
                                          float lq, float kp, float cp, float lp)
{
    float S, dS;
    tb_switch(r, rs, iw, S, dS);
    const float eq = __builtin_amdgcn_exp2f(__builtin_fmaf(-kq, r, cq));
    const float ep = __builtin_amdgcn_exp2f(__builtin_fmaf(-kp, r, cp));
    const float dpsi = fsum * eq * __builtin_fmaf(-lq, S, dS);
    const float dPhi = ep * __builtin_fmaf(-lp, S, dS);
    return make_float2(-(dpsi + dPhi) * ir, ep * S);
}

__device__ __forceinline__ float rho_term(const TB32 &p, float r2, bool valid, uint32_t, uint32_t)
{
    const float psi = tb_psi(__builtin_amdgcn_sqrtf(r2) * p.len, p.rs, p.iw, p.kq, p.cq);
    return (valid && r2 < p.cut2u) ? psi : 0.f;
}

__device__ __forceinline__ PairOut force_term(const TB32 &p, float r2, bool valid, uint32_t wi, uint32_t wj)
{
    const bool in = valid && r2 < p.cut2u;
    const float ir = __builtin_amdgcn_rsqf(r2);
    const float2 o = tb_force(r2 * ir * p.len, ir, __uint_as_float(wi) + __uint_as_float(wj), p.rs, p.iw, p.kq,
                              p.cq, p.lq, p.kp, p.cp, p.lp);
    return {in ? o.x : 0.f, in ? o.y : 0.f, in};
}

__device__ __forceinline__ uint32_t fprime_word(const TB32 &, float fp, uint32_t) { return __float_as_uint(fp); }

// per-lane choice among the three pair kinds (branch-free)
__device__ __forceinline__ float sel3(const float (&v)[3], uint32_t k)
{
    return k == 0u ? v[0] : (k == 1u ? v[1] : v[2]);
}

template <bool CC>
__device__ __forceinline__ float cut_sel(const float (&v)[3], uint32_t k)
{
    return CC ? v[0] : sel3(v, k);
}

template <bool CC>
__device__ __forceinline__ float rho_term(const TBM32<CC> &p, float r2, bool valid, uint32_t wi, uint32_t wj)
{
    const uint32_t k = (wi & 1u) + (wj & 1u);
    const float psi = tb_psi(__builtin_amdgcn_sqrtf(r2) * p.len, cut_sel<CC>(p.rs, k), cut_sel<CC>(p.iw, k),
                             sel3(p.kq, k), sel3(p.cq, k));
    return (valid && r2 < cut_sel<CC>(p.cut2u, k)) ? psi : 0.f;
}

template <bool CC>
__device__ __forceinline__ PairOut force_term(const TBM32<CC> &p, float r2, bool valid, uint32_t wi, uint32_t wj)
{
    constexpr float kLn2 = 0.693147180559945309f;
    const uint32_t k = (wi & 1u) + (wj & 1u);
    const bool in = valid && r2 < cut_sel<CC>(p.cut2u, k);
    const float ir = __builtin_amdgcn_rsqf(r2);
    const float fsum = __uint_as_float(wi & ~1u) + __uint_as_float(wj & ~1u);
    const float kq = sel3(p.kq, k), kp = sel3(p.kp, k);
    const float2 o = tb_force(r2 * ir * p.len, ir, fsum, cut_sel<CC>(p.rs, k), cut_sel<CC>(p.iw, k), kq,
                              sel3(p.cq, k), kq * kLn2, kp, sel3(p.cp, k), kp * kLn2);
    return {in ? o.x : 0.f, in ? o.y : 0.f, in};
}

template <bool CC>
__device__ __forceinline__ uint32_t fprime_word(const TBM32<CC> &, float fp, uint32_t wi)
{
    return (__float_as_uint(fp) & ~1u) | (wi & 1u);
}

// pass 1: rho_i = sum psi(r_ij), then F_i = -A sqrt(rho_i), F'_i; F'_i is
// stored in the fourth word of the scaled coordinates for pass 2's gather.
template <class P, int TPA, int U, bool CUBIC, bool ENERGY, bool COMP>
__global__ __launch_bounds__(kBlock) void k_eam_rho(int64_t n, uint4 *__restrict__ xs,
                                                    int32_t cap, const int32_t *__restrict__ idx,
                                                    const int32_t *__restrict__ count, P p,
                                                    float *__restrict__ rho, float *__restrict__ fprime,
                                                    double *__restrict__ part, Span sp, const BrickTab *tab)
{
    if (gated(p.gate)) return;
    static_assert(TPA == kSlice, "one slice per wave");
    const uint32_t lblk = xcd_block(blockIdx.x, gridDim.x);
    uint32_t blk = lblk;
    if (tab) {
        const BrickSel e = brick_select(tab, lblk);
        blk = e.blk;
        xs += e.slot0;
        idx += e.slot0 * cap;
        count += e.slot0;
        rho += e.atom0;
        fprime += e.atom0;
        n = e.n_end;
        sp.n_xs = e.n_xs;
        sp.slice0 = e.slice0;
    }
    const SliceLane sl = slice_lane(blk, sp.slice0);
    const int64_t i = sl.i;
    const int sub = sl.sub;

    const SliceBufs b = slice_bufs(xs, sp.n_xs, idx, cap, blk, sp.slice0);
    float s = 0.f, c = 0.f;
    uint32_t wi = 0;
    if (i < n) {
        const uint4 pi = xs[i];
        wi = pi.w;
        const int32_t cnt = min(count[i], cap);
        walk_form<P::kSplit, U, P::kRhoWords>(b.xs, b.row, cnt, sub, [&](const auto &pj, int32_t t0, auto masked) {
            constexpr int K = sizeof(pj) / sizeof(uint4);
            float bs = 0.f;
#pragma unroll
            for (int u = 0; u < K; ++u) {
                float dx, dy, dz;
                disp<CUBIC>(pi, pj[u], p.ax, p.ay, p.az, dx, dy, dz);
                const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                bs += rho_term(p, r2, !decltype(masked)::value || t0 + u * TPA < cnt, pi.w, pj[u].w);
            }
            acc_sum<COMP>(s, c, bs);
        });
    }
    const double g = combine(s, c);
    double Fi = 0.0;
    if (sub == 0 && i < n) {
        float F = 0.f, Fp = 0.f;
        const float r = float(g);
        if (r > 0.f) {
            const float sq = __builtin_amdgcn_sqrtf(r);
            F = -p.A * sq;
            Fp = -0.5f * p.A * __builtin_amdgcn_rcpf(sq);
        }
        rho[i] = r;
        fprime[i] = Fp;
        xs[i].w = fprime_word(p, Fp, wi);
        Fi = double(F);
    }
    if (ENERGY) {
        __shared__ double lds[1 * (kBlock / kWave)];
        double v[1] = {Fi};
        block_sum<1>(v, lds);
        if (threadIdx.x == 0) {
            part[int64_t(lblk) * 8] = v[0];
            for (int q = 1; q < 8; ++q) part[int64_t(lblk) * 8 + q] = 0.0;
        }
    }
}

// pass 2: F_i = -sum_j [(F'_i + F'_j) psi'(r) + V'(r)] (r_i - r_j) / r
template <class P, int TPA, int U, bool CUBIC, bool ENERGY, bool COMP>
__global__ __launch_bounds__(kBlock) void k_eam_force(int64_t n, const uint4 *__restrict__ xs,
                                                      int32_t cap, const int32_t *__restrict__ idx,
                                                      const int32_t *__restrict__ count, P p,
                                                      const float *__restrict__ rho, float *__restrict__ f,
                                                      float *__restrict__ e_atom, double *__restrict__ part, Span sp,
                                                      const BrickTab *tab)
{
    if (gated(p.gate)) return;
    static_assert(TPA == kSlice, "one slice per wave");
    const uint32_t lblk = xcd_block(blockIdx.x, gridDim.x);
    uint32_t blk = lblk;
    if (tab) {
        const BrickSel e = brick_select(tab, lblk);
        blk = e.blk;
        xs += e.slot0;
        idx += e.slot0 * cap;
        count += e.slot0;
        rho += e.atom0;
        f += e.atom0;
        if (e_atom) e_atom += e.atom0;
        n = e.n_end;
        sp.n_xs = e.n_xs;
        sp.slice0 = e.slice0;
    }
    const SliceLane sl = slice_lane(blk, sp.slice0);
    const int64_t i = sl.i;
    const int sub = sl.sub;

    const SliceBufs b = slice_bufs(xs, sp.n_xs, idx, cap, blk, sp.slice0);
    float fx = 0.f, fy = 0.f, fz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
    double e = 0.0, w[6] = {0, 0, 0, 0, 0, 0};
    if (i < n) {
        const uint4 pi = xs[i];
        const int32_t cnt = min(count[i], cap);
        walk_form<P::kSplit, U, 4>(b.xs, b.row, cnt, sub, [&](const auto &pj, int32_t t0, auto masked) {
            constexpr int K = sizeof(pj) / sizeof(uint4);
            float bx = 0.f, by = 0.f, bz = 0.f;
#pragma unroll
            for (int u = 0; u < K; ++u) {
                float dx, dy, dz;
                disp<CUBIC>(pi, pj[u], p.ax, p.ay, p.az, dx, dy, dz);
                const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                // -(dU/dr) / r in the displacement unit: F = g * (dx, dy, dz)
                const PairOut o = force_term(p, r2, !decltype(masked)::value || t0 + u * TPA < cnt, pi.w, pj[u].w);
                const float g = o.g;
                bx = __builtin_fmaf(g, dx, bx);
                by = __builtin_fmaf(g, dy, by);
                bz = __builtin_fmaf(g, dz, bz);
                if (ENERGY && o.in) {
                    e += double(o.v);
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
        f[sp.fs + i] = float(gy);
        f[2 * sp.fs + i] = float(gz);
    }
    if (ENERGY && e_atom) {
        // site energy F(rho_i) + 1/2 sum_j V(r_ij); F as in the first pass
        double ei = e;
#pragma unroll
        for (int o = 1; o < kSlice; o <<= 1) ei += __shfl_xor(ei, o, kWave);
        if (sub == 0 && i < n) {
            const float r = rho[i];
            const float F = r > 0.f ? -p.A * __builtin_amdgcn_sqrtf(r) : 0.f;
            e_atom[i] = float(double(F) + 0.5 * ei);
        }
    }
    if (ENERGY) {
        __shared__ double lds[8 * (kBlock / kWave)];
        const double u = double(p.len);
        double v[8] = {e, 0.0, w[0] * u, w[1] * u, w[2] * u, w[3] * u, w[4] * u, w[5] * u};
        block_sum<8>(v, lds);
        if (threadIdx.x == 0)
            for (int c = 0; c < 8; ++c) part[int64_t(lblk) * 8 + c] = v[c];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
constexpr int kTPA = kSlice;   // lanes per atom of the FP32 kernels
constexpr int kUnroll = 4;     // row entries per lane per batch (embedded-atom passes)
constexpr int kUnrollLJ = 6;   // LJ: rows of ~70 entries take two batches (measured best of 2-12)

static uint32_t blocks_for(int64_t n, int tpa) { return uint32_t((n * tpa + kBlock - 1) / kBlock); }

static bool is_cubic(const md_box_t *b) { return b->L[0] == b->L[1] && b->L[1] == b->L[2]; }

struct List {
    int32_t cap;
    const int32_t *idx, *cnt;
};

template <int TPA, bool CUBIC, bool E, bool C>
static void launch_lj32(uint32_t gb, hipStream_t s, int64_t n, const uint4 *q, const List &l, const LJ32 &p,
                        float *f, double *part, const Span &sp, const BrickTab *tab)
{
    hipLaunchKernelGGL((k_lj32<TPA, kUnrollLJ, CUBIC, E, C>), dim3(gb), dim3(kBlock), 0, s, n, q, l.cap, l.idx, l.cnt,
                       p, f, part, sp, tab);
}

template <int TPA, bool CUBIC>
static void dispatch_lj32(bool e, bool c, uint32_t gb, hipStream_t s, int64_t n, const uint4 *q, const List &l,
                          const LJ32 &p, float *f, double *part, const Span &sp, const BrickTab *tab = nullptr)
{
    if (e && c) launch_lj32<TPA, CUBIC, true, true>(gb, s, n, q, l, p, f, part, sp, tab);
    else if (e) launch_lj32<TPA, CUBIC, true, false>(gb, s, n, q, l, p, f, part, sp, tab);
    else if (c) launch_lj32<TPA, CUBIC, false, true>(gb, s, n, q, l, p, f, part, sp, tab);
    else launch_lj32<TPA, CUBIC, false, false>(gb, s, n, q, l, p, f, part, sp, tab);
}

// blocks of a launch over the slices from sp.slice0 to the one holding atom n-1
static uint32_t blocks_span(int64_t n, const Span &sp)
{
    const int64_t slices = (n + kSlice - 1) / kSlice - int64_t(sp.slice0);
    return slices > 0 ? uint32_t((slices + kBlock / kWave - 1) / (kBlock / kWave)) : 0u;
}

static LJ32 lj_constants(const md_box_t *box, const md_lj_t *lj, Gate gate)
{
    const double two32 = 4294967296.0;
    const bool cubic = is_cubic(box);
    const double u = cubic ? box->L[0] / two32 : 1.0;   // length unit
    LJ32 p;
    p.ax = float(box->L[0] / two32);
    p.ay = float(box->L[1] / two32);
    p.az = float(box->L[2] / two32);
    p.len = float(u);
    p.rc2 = float(lj->rc * lj->rc / (u * u));
    p.sig2 = float(lj->sigma * lj->sigma / (u * u));
    p.eps4 = float(4.0 * lj->eps);
    p.eps24 = float(24.0 * lj->eps / u);
    p.gate = gate;
    return p;
}

int forces_lj(const md_box_t *box, int64_t n, const double *x, const uint32_t *xs, int32_t cap, const int32_t *idx,
              const int32_t *cnt, const md_lj_t *lj, void *f, double *ev, int32_t flags, void *ws, const WsLayout &w,
              hipStream_t s, Gate gate)
{
    return forces_lj_part(box, n, x, xs, cap, idx, cnt, lj, f, ev, flags, ws_ptr<double>(ws, w.red1), w.red_blocks,
                          s, gate);
}

int forces_lj_part(const md_box_t *box, int64_t n, const double *x, const uint32_t *xs, int32_t cap,
                   const int32_t *idx, const int32_t *cnt, const md_lj_t *lj, void *f, double *ev, int32_t flags,
                   double *part, int64_t part_rows, hipStream_t s, Gate gate)
{
    const List l{cap, idx, cnt};
    const bool energy = flags & MD_ENERGY;
    const double phi_rc = [&] {
        const double s2 = lj->sigma * lj->sigma / (lj->rc * lj->rc);
        const double s6 = s2 * s2 * s2;
        return 4.0 * lj->eps * (s6 * s6 - s6);
    }();
    uint32_t gb = 0;
    if (n > 0) {
        if (flags & MD_PAIR_FP64) {
            gb = blocks_for(n, kTPA);
            if (energy && int64_t(gb) > part_rows) return MD_ERR_WORKSPACE;
            LJ64 p;
            for (int a = 0; a < 3; ++a) {
                p.L[a] = box->L[a];
                p.hL[a] = 0.5 * box->L[a];
            }
            p.rc2 = lj->rc * lj->rc;
            p.sig2 = lj->sigma * lj->sigma;
            p.eps4 = 4.0 * lj->eps;
            p.eps24 = 24.0 * lj->eps;
            p.gate = gate;
            double *fd = static_cast<double *>(f);
            if (energy)
                hipLaunchKernelGGL((k_lj64<kTPA, true>), dim3(gb), dim3(kBlock), 0, s, n, x, cap, idx, cnt, p, fd,
                                   part);
            else
                hipLaunchKernelGGL((k_lj64<kTPA, false>), dim3(gb), dim3(kBlock), 0, s, n, x, cap, idx, cnt, p, fd,
                                   part);
        } else {
            const bool cubic = is_cubic(box);
            gb = blocks_for(n, kTPA);
            if (energy && int64_t(gb) > part_rows) return MD_ERR_WORKSPACE;
            const LJ32 p = lj_constants(box, lj, gate);
            const uint4 *q = reinterpret_cast<const uint4 *>(xs);
            float *ff = static_cast<float *>(f);
            const bool comp = !(flags & MD_NO_COMPENSATE);
            if (cubic) dispatch_lj32<kTPA, true>(energy, comp, gb, s, n, q, l, p, ff, part, whole(n));
            else dispatch_lj32<kTPA, false>(energy, comp, gb, s, n, q, l, p, ff, part, whole(n));
        }
        MD_HIP_TRY(hipGetLastError());
    }
    if (energy) return launch_reduce_partials(part, gb, nullptr, 0, ev, kReduceLJ, phi_rc, 0.0, s);
    return MD_OK;
}

template <class P, int TPA, bool CUBIC, bool E, bool C>
static void launch_eam(int passes, uint32_t gb, hipStream_t s, int64_t n, uint4 *q, const List &l, const P &p,
                       float *rho, float *fprime, float *f, float *ea, double *part1, double *part2, const Span &sp,
                       const BrickTab *tab)
{
    if (passes & 1)
        hipLaunchKernelGGL((k_eam_rho<P, TPA, P::kRhoUnroll, CUBIC, E, C>), dim3(gb), dim3(kBlock), 0, s, n, q, l.cap,
                           l.idx, l.cnt, p, rho, fprime, part1, sp, tab);
    if (passes & 2)
        hipLaunchKernelGGL((k_eam_force<P, TPA, kUnroll, CUBIC, E, C>), dim3(gb), dim3(kBlock), 0, s, n, q, l.cap,
                           l.idx, l.cnt, p, rho, f, ea, part2, sp, tab);
}

template <class P, int TPA, bool CUBIC>
static void dispatch_eam(int passes, bool e, bool c, uint32_t gb, hipStream_t s, int64_t n, uint4 *q,
                         const List &l, const P &p, float *rho, float *fprime, float *f, float *ea, double *p1,
                         double *p2, const Span &sp, const BrickTab *tab = nullptr)
{
    if (e && c) launch_eam<P, TPA, CUBIC, true, true>(passes, gb, s, n, q, l, p, rho, fprime, f, ea, p1, p2, sp, tab);
    else if (e) launch_eam<P, TPA, CUBIC, true, false>(passes, gb, s, n, q, l, p, rho, fprime, f, ea, p1, p2, sp, tab);
    else if (c) launch_eam<P, TPA, CUBIC, false, true>(passes, gb, s, n, q, l, p, rho, fprime, f, ea, p1, p2, sp, tab);
    else launch_eam<P, TPA, CUBIC, false, false>(passes, gb, s, n, q, l, p, rho, fprime, f, ea, p1, p2, sp, tab);
}

// Both passes of an embedded-atom form P (geometry fields set here).
template <class P>
static int forces_two_pass(const md_box_t *box, int64_t n, uint32_t *xs, const List &l, P p, float *rho,
                           float *fprime, float *f, float *e_atom, double *ev, int32_t flags, void *ws,
                           const WsLayout &w, hipStream_t s)
{
    const bool energy = flags & MD_ENERGY;
    const bool comp = !(flags & MD_NO_COMPENSATE);
    double *part1 = ws_ptr<double>(ws, w.red1);
    double *part2 = ws_ptr<double>(ws, w.red2);
    const bool cubic = is_cubic(box);
    const uint32_t gb = n > 0 ? blocks_for(n, kTPA) : 0;
    if (int64_t(gb) > w.red_blocks) return MD_ERR_WORKSPACE;
    uint4 *q = reinterpret_cast<uint4 *>(xs);
    if (n > 0) {
        if (cubic)
            dispatch_eam<P, kTPA, true>(3, energy, comp, gb, s, n, q, l, p, rho, fprime, f, e_atom, part1, part2,
                                        whole(n));
        else
            dispatch_eam<P, kTPA, false>(3, energy, comp, gb, s, n, q, l, p, rho, fprime, f, e_atom, part1, part2,
                                         whole(n));
        MD_HIP_TRY(hipGetLastError());
    }
    if (energy) return launch_reduce_partials(part1, gb, part2, gb, ev, kReduceEAM, 0.0, 0.0, s);
    return MD_OK;
}

// displacement unit of the FP32 pair kernels: L/2^32 in a cubic box, else 1
static double disp_unit(const md_box_t *box) { return is_cubic(box) ? box->L[0] / 4294967296.0 : 1.0; }

static FS32 fs_constants(const md_box_t *box, const md_fs_t *fs, Gate gate)
{
    const double two32 = 4294967296.0;
    const double u = disp_unit(box);
    FS32 p;
    p.ax = float(box->L[0] / two32);
    p.ay = float(box->L[1] / two32);
    p.az = float(box->L[2] / two32);
    p.len = float(u);
    p.d2u = float(fs->d * fs->d / (u * u));
    p.c2u = float(fs->c * fs->c / (u * u));
    p.d = float(fs->d);
    p.c = float(fs->c);
    p.p0 = float(fs->c0 + fs->c1 * fs->c + fs->c2 * fs->c * fs->c);
    p.p1 = float(fs->c1 + 2.0 * fs->c2 * fs->c);
    p.p2 = float(fs->c2);
    p.A = float(fs->A);
    p.gate = gate;
    return p;
}

int forces_eam(const md_box_t *box, int64_t n, uint32_t *xs, int32_t cap, const int32_t *idx, const int32_t *cnt,
               const md_fs_t *fs, float *rho, float *fprime, float *f, float *e_atom, double *ev, int32_t flags,
               void *ws, const WsLayout &w, hipStream_t s, Gate gate)
{
    return forces_two_pass(box, n, xs, List{cap, idx, cnt}, fs_constants(box, fs, gate), rho, fprime, f, e_atom, ev,
                           flags, ws, w, s);
}

int forces_tb(const md_box_t *box, int64_t n, uint32_t *xs, int32_t cap, const int32_t *idx, const int32_t *cnt,
              const md_tb_t *tb, float *rho, float *fprime, float *f, float *e_atom, double *ev, int32_t flags,
              void *ws, const WsLayout &w, hipStream_t s, Gate gate)
{
    const double two32 = 4294967296.0, log2e = 1.4426950408889634;
    const double u = disp_unit(box);
    TB32 p;
    p.ax = float(box->L[0] / two32);
    p.ay = float(box->L[1] / two32);
    p.az = float(box->L[2] / two32);
    p.len = float(u);
    p.cut2u = float(tb->rc * tb->rc / (u * u));
    p.rs = float(tb->rs);
    p.iw = float(1.0 / (tb->rc - tb->rs));
    const double kq = 2.0 * tb->q * log2e / tb->r0, kp = tb->p * log2e / tb->r0;
    p.kq = float(kq);
    p.cq = float(kq * tb->r0 + std::log2(tb->xi * tb->xi));
    p.lq = float(2.0 * tb->q / tb->r0);
    p.kp = float(kp);
    p.cp = float(kp * tb->r0 + std::log2(2.0 * tb->A));
    p.lp = float(tb->p / tb->r0);
    p.A = 1.f;
    p.gate = gate;
    return forces_two_pass(box, n, xs, List{cap, idx, cnt}, p, rho, fprime, f, e_atom, ev, flags, ws, w, s);
}

template <bool CC>
static TBM32<CC> tbm_constants(const md_box_t *box, const md_tbm_t *tb, Gate gate)
{
    const double two32 = 4294967296.0, log2e = 1.4426950408889634;
    const double u = disp_unit(box);
    TBM32<CC> p;
    p.ax = float(box->L[0] / two32);
    p.ay = float(box->L[1] / two32);
    p.az = float(box->L[2] / two32);
    p.len = float(u);
    for (int k = 0; k < 3; ++k) {
        const md_tb_t &t = tb->pair[k];
        p.cut2u[k] = float(t.rc * t.rc / (u * u));
        p.rs[k] = float(t.rs);
        p.iw[k] = float(1.0 / (t.rc - t.rs));
        const double kq = 2.0 * t.q * log2e / t.r0, kp = t.p * log2e / t.r0;
        p.kq[k] = float(kq);
        p.cq[k] = float(kq * t.r0 + std::log2(t.xi * t.xi));
        p.kp[k] = float(kp);
        p.cp[k] = float(kp * t.r0 + std::log2(2.0 * t.A));
    }
    p.A = 1.f;
    p.gate = gate;
    return p;
}

int forces_tbm(const md_box_t *box, int64_t n, uint32_t *xs, int32_t cap, const int32_t *idx, const int32_t *cnt,
               const md_tbm_t *tb, float *rho, float *fprime, float *f, float *e_atom, double *ev, int32_t flags,
               void *ws, const WsLayout &w, hipStream_t s, Gate gate)
{
    const md_tb_t *q = tb->pair;
    const bool common = q[0].rs == q[1].rs && q[0].rs == q[2].rs && q[0].rc == q[1].rc && q[0].rc == q[2].rc;
    const List l{cap, idx, cnt};
    if (common)
        return forces_two_pass(box, n, xs, l, tbm_constants<true>(box, tb, gate), rho, fprime, f, e_atom, ev, flags,
                               ws, w, s);
    return forces_two_pass(box, n, xs, l, tbm_constants<false>(box, tb, gate), rho, fprime, f, e_atom, ev, flags, ws,
                           w, s);
}

// ---- ranges of the bricks of a domain decomposition, one launch ----
// `tab` (device) gives each brick's atom range and bases (BrickTab); gb
// logical blocks in all; xs, idx, count, f, rho, fprime are the arrays of
// all bricks (slot and atom 0); fs the stride of f's components.  Partial
// energy rows (MD_ENERGY) go to part[0 .. gb).

int bricks_forces_lj(const md_box_t *vbox, const BrickTab *tab, uint32_t gb, int64_t fs, const uint32_t *xs,
                     int32_t cap, const int32_t *idx, const int32_t *cnt, const md_lj_t *lj, float *f, int32_t flags,
                     double *part, hipStream_t s, Gate gate)
{
    if (gb == 0) return MD_OK;
    const LJ32 p = lj_constants(vbox, lj, gate);
    const List l{cap, idx, cnt};
    const uint4 *q = reinterpret_cast<const uint4 *>(xs);
    const bool energy = flags & MD_ENERGY, comp = !(flags & MD_NO_COMPENSATE);
    const Span sp{0, fs, 0u};
    if (is_cubic(vbox)) dispatch_lj32<kTPA, true>(energy, comp, gb, s, 0, q, l, p, f, part, sp, tab);
    else dispatch_lj32<kTPA, false>(energy, comp, gb, s, 0, q, l, p, f, part, sp, tab);
    MD_HIP_TRY(hipGetLastError());
    return MD_OK;
}

// pass: 1 = densities and F' (rho, fprime, the fourth words), 2 = forces
int bricks_forces_eam(int pass, const md_box_t *vbox, const BrickTab *tab, uint32_t gb, int64_t fs, uint32_t *xs,
                      int32_t cap, const int32_t *idx, const int32_t *cnt, const md_fs_t *fsp, float *rho,
                      float *fprime, float *f, int32_t flags, double *part, hipStream_t s, Gate gate)
{
    if (gb == 0) return MD_OK;
    const FS32 p = fs_constants(vbox, fsp, gate);
    const List l{cap, idx, cnt};
    uint4 *q = reinterpret_cast<uint4 *>(xs);
    const bool energy = flags & MD_ENERGY, comp = !(flags & MD_NO_COMPENSATE);
    const Span sp{0, fs, 0u};
    if (is_cubic(vbox))
        dispatch_eam<FS32, kTPA, true>(pass, energy, comp, gb, s, 0, q, l, p, rho, fprime, f, nullptr, part, part, sp,
                                       tab);
    else
        dispatch_eam<FS32, kTPA, false>(pass, energy, comp, gb, s, 0, q, l, p, rho, fprime, f, nullptr, part, part,
                                        sp, tab);
    MD_HIP_TRY(hipGetLastError());
    return MD_OK;
}

}  // namespace md
