// Steps a4-a6: Lennard-Jones and embedded-atom forces over full Verlet lists.
//
// The pair loop of the paper (Sec. 2.2) visits each pair once and scatters
// -F into f_j; the paper avoids the resulting write races with its cell-task
// schedule.  Here every atom's row holds all its neighbours, so each pair is
// evaluated from both sides and every force is written once by its owner:
// no atomics and bitwise-reproducible results.
//
// Thread mapping: TPA consecutive lanes share one atom and walk its row with
// stride TPA, so each wave issues coalesced 4*TPA-byte runs of list indices
// and 16-byte gathers of scaled coordinates.  The TPA partial sums are
// combined in FP64 with lane shuffles.
//
// FP32 path: displacements come from 32-bit scaled coordinates (fraction of
// the box times 2^32, Sec. 4.1 "fetch"/"dist"): the integer difference is the
// periodic minimum image, converted to float and scaled by L/2^32.  Pair
// arithmetic is FP32; per-lane sums use Kahan compensation.
#include "md_common.h"

namespace md {

struct LJ32 {
    float sx, sy, sz;      // L / 2^32 per axis
    float rc2, sig2, eps4, eps24;
};

struct LJ64 {
    double L[3], hL[3];
    double rc2, sig2, eps4, eps24;
};

template <bool COMP>
__device__ __forceinline__ void kahan_add(float &s, float &c, float a, float b)
{
    // s += a * b with the product's contribution compensated
    if (COMP) {
        const float y = __builtin_fmaf(a, b, -c);
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    } else {
        s = __builtin_fmaf(a, b, s);
    }
}

__device__ __forceinline__ float idiff(uint32_t a, uint32_t b, float scale)
{
    return float(int32_t(a - b)) * scale;
}

// ---------------------------------------------------------------------------
// Lennard-Jones, FP32 pair arithmetic
// ---------------------------------------------------------------------------
template <int TPA, bool ENERGY, bool COMP>
__global__ __launch_bounds__(kBlock) void k_lj32(int64_t n, const uint4 *__restrict__ xs,
                                                 const int64_t *__restrict__ off, const int32_t *__restrict__ idx,
                                                 LJ32 p, float *__restrict__ f, double *__restrict__ part)
{
    constexpr int APB = kBlock / TPA;  // atoms per block
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int sub = threadIdx.x % TPA;
    const int64_t i = int64_t(blk) * APB + threadIdx.x / TPA;

    float fx = 0.f, fy = 0.f, fz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
    double e = 0.0, np = 0.0, w[6] = {0, 0, 0, 0, 0, 0};
    if (i < n) {
        const uint4 pi = xs[i];
        const int64_t k1 = off[i + 1];
        for (int64_t k = off[i] + sub; k < k1; k += TPA) {
            const uint4 pj = xs[idx[k]];
            const float dx = idiff(pi.x, pj.x, p.sx);
            const float dy = idiff(pi.y, pj.y, p.sy);
            const float dz = idiff(pi.z, pj.z, p.sz);
            const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
            if (r2 < p.rc2) {
                const float ir2 = __builtin_amdgcn_rcpf(r2);
                const float s2 = p.sig2 * ir2;
                const float s6 = s2 * s2 * s2;
                const float fs = p.eps24 * s6 * __builtin_fmaf(2.f, s6, -1.f) * ir2;
                kahan_add<COMP>(fx, cx, fs, dx);
                kahan_add<COMP>(fy, cy, fs, dy);
                kahan_add<COMP>(fz, cz, fs, dz);
                if (ENERGY) {
                    e += double(p.eps4 * (s6 * s6 - s6));
                    np += 1.0;
                    w[0] += double(fs * dx * dx); w[1] += double(fs * dy * dy); w[2] += double(fs * dz * dz);
                    w[3] += double(fs * dx * dy); w[4] += double(fs * dx * dz); w[5] += double(fs * dy * dz);
                }
            }
        }
    }
    double gx = double(fx) - double(cx), gy = double(fy) - double(cy), gz = double(fz) - double(cz);
    if (TPA > 1) {
        gx = group_sum(gx, TPA);
        gy = group_sum(gy, TPA);
        gz = group_sum(gz, TPA);
    }
    if (sub == 0 && i < n) {
        f[i] = float(gx);
        f[n + i] = float(gy);
        f[2 * n + i] = float(gz);
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
// Lennard-Jones, FP64 pair arithmetic (minimum image as in the list build)
// ---------------------------------------------------------------------------
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
                                                 const int64_t *__restrict__ off, const int32_t *__restrict__ idx,
                                                 LJ64 p, double *__restrict__ f, double *__restrict__ part)
{
    constexpr int APB = kBlock / TPA;
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int sub = threadIdx.x % TPA;
    const int64_t i = int64_t(blk) * APB + threadIdx.x / TPA;

    double fx = 0, fy = 0, fz = 0, e = 0, np = 0, w[6] = {0, 0, 0, 0, 0, 0};
    if (i < n) {
        const double xi = x[i], yi = x[n + i], zi = x[2 * n + i];
        const int64_t k1 = off[i + 1];
        for (int64_t k = off[i] + sub; k < k1; k += TPA) {
            const int64_t j = idx[k];
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
    if (TPA > 1) {
        fx = group_sum(fx, TPA);
        fy = group_sum(fy, TPA);
        fz = group_sum(fz, TPA);
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
    float sx, sy, sz;
    float d, d2, c, c2, p0, p1, p2, A;
};

// pass 1: rho_i = sum psi(r_ij), then F_i = -A sqrt(rho_i), F'_i; F'_i is
// stored in the fourth word of the scaled coordinates for pass 2's gather.
template <int TPA, bool ENERGY, bool COMP>
__global__ __launch_bounds__(kBlock) void k_eam_rho(int64_t n, uint4 *__restrict__ xs,
                                                    const int64_t *__restrict__ off, const int32_t *__restrict__ idx,
                                                    FS32 p, float *__restrict__ rho, float *__restrict__ fprime,
                                                    double *__restrict__ part)
{
    constexpr int APB = kBlock / TPA;
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int sub = threadIdx.x % TPA;
    const int64_t i = int64_t(blk) * APB + threadIdx.x / TPA;

    float s = 0.f, c = 0.f;
    if (i < n) {
        const uint4 pi = xs[i];
        const int64_t k1 = off[i + 1];
        for (int64_t k = off[i] + sub; k < k1; k += TPA) {
            const uint4 pj = xs[idx[k]];
            const float dx = idiff(pi.x, pj.x, p.sx);
            const float dy = idiff(pi.y, pj.y, p.sy);
            const float dz = idiff(pi.z, pj.z, p.sz);
            const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
            if (r2 < p.d2) {
                const float t = __builtin_amdgcn_sqrtf(r2) - p.d;
                kahan_add<COMP>(s, c, t, t);
            }
        }
    }
    double g = double(s) - double(c);
    if (TPA > 1) g = group_sum(g, TPA);
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
        xs[i].w = __float_as_uint(Fp);
        Fi = double(F);
    }
    if (ENERGY) {
        __shared__ double lds[1 * (kBlock / kWave)];
        double v[1] = {Fi};
        block_sum<1>(v, lds);
        if (threadIdx.x == 0) {
            part[int64_t(blk) * 8] = v[0];
            for (int q = 1; q < 8; ++q) part[int64_t(blk) * 8 + q] = 0.0;
        }
    }
}

// pass 2: F_i = -sum_j [(F'_i + F'_j) psi'(r) + V'(r)] (r_i - r_j) / r
template <int TPA, bool ENERGY, bool COMP>
__global__ __launch_bounds__(kBlock) void k_eam_force(int64_t n, const uint4 *__restrict__ xs,
                                                      const int64_t *__restrict__ off,
                                                      const int32_t *__restrict__ idx, FS32 p, float *__restrict__ f,
                                                      double *__restrict__ part)
{
    constexpr int APB = kBlock / TPA;
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int sub = threadIdx.x % TPA;
    const int64_t i = int64_t(blk) * APB + threadIdx.x / TPA;

    float fx = 0.f, fy = 0.f, fz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
    double e = 0.0, w[6] = {0, 0, 0, 0, 0, 0};
    if (i < n) {
        const uint4 pi = xs[i];
        const float fpi = __uint_as_float(pi.w);
        const int64_t k1 = off[i + 1];
        for (int64_t k = off[i] + sub; k < k1; k += TPA) {
            const uint4 pj = xs[idx[k]];
            const float dx = idiff(pi.x, pj.x, p.sx);
            const float dy = idiff(pi.y, pj.y, p.sy);
            const float dz = idiff(pi.z, pj.z, p.sz);
            const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
            const bool in_d = r2 < p.d2, in_c = r2 < p.c2;
            if (in_d || in_c) {
                const float r = __builtin_amdgcn_sqrtf(r2);
                const float ir = __builtin_amdgcn_rcpf(r);
                float dUdr = 0.f;
                if (in_d) dUdr = (fpi + __uint_as_float(pj.w)) * 2.f * (r - p.d);
                float V = 0.f;
                if (in_c) {
                    const float t = r - p.c;
                    const float poly = __builtin_fmaf(__builtin_fmaf(p.p2, t, p.p1), t, p.p0);
                    const float dpoly = __builtin_fmaf(2.f * p.p2, t, p.p1);
                    dUdr += t * __builtin_fmaf(t, dpoly, 2.f * poly);
                    V = t * t * poly;
                }
                const float g = -dUdr * ir;
                kahan_add<COMP>(fx, cx, g, dx);
                kahan_add<COMP>(fy, cy, g, dy);
                kahan_add<COMP>(fz, cz, g, dz);
                if (ENERGY) {
                    e += double(V);
                    w[0] += double(g * dx * dx); w[1] += double(g * dy * dy); w[2] += double(g * dz * dz);
                    w[3] += double(g * dx * dy); w[4] += double(g * dx * dz); w[5] += double(g * dy * dz);
                }
            }
        }
    }
    double gx = double(fx) - double(cx), gy = double(fy) - double(cy), gz = double(fz) - double(cz);
    if (TPA > 1) {
        gx = group_sum(gx, TPA);
        gy = group_sum(gy, TPA);
        gz = group_sum(gz, TPA);
    }
    if (sub == 0 && i < n) {
        f[i] = float(gx);
        f[n + i] = float(gy);
        f[2 * n + i] = float(gz);
    }
    if (ENERGY) {
        __shared__ double lds[8 * (kBlock / kWave)];
        double v[8] = {e, 0.0, w[0], w[1], w[2], w[3], w[4], w[5]};
        block_sum<8>(v, lds);
        if (threadIdx.x == 0)
            for (int c = 0; c < 8; ++c) part[int64_t(blk) * 8 + c] = v[c];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
constexpr int kTPA = 8;

static uint32_t blocks_for(int64_t n, int tpa) { return uint32_t((n * tpa + kBlock - 1) / kBlock); }

int forces_lj(const md_box_t *box, int64_t n, const double *x, const uint32_t *xs, const int64_t *off,
              const int32_t *idx, const md_lj_t *lj, void *f, double *ev, int32_t flags, void *ws,
              const WsLayout &w, hipStream_t s)
{
    const bool energy = flags & MD_ENERGY;
    double *part = ws_ptr<double>(ws, w.red1);
    const uint32_t gb = blocks_for(n, kTPA);
    if (int64_t(gb) > w.red_blocks) return MD_ERR_WORKSPACE;
    const double phi_rc = [&] {
        const double s2 = lj->sigma * lj->sigma / (lj->rc * lj->rc);
        const double s6 = s2 * s2 * s2;
        return 4.0 * lj->eps * (s6 * s6 - s6);
    }();
    if (n > 0) {
        if (flags & MD_PAIR_FP64) {
            LJ64 p;
            for (int a = 0; a < 3; ++a) {
                p.L[a] = box->L[a];
                p.hL[a] = 0.5 * box->L[a];
            }
            p.rc2 = lj->rc * lj->rc;
            p.sig2 = lj->sigma * lj->sigma;
            p.eps4 = 4.0 * lj->eps;
            p.eps24 = 24.0 * lj->eps;
            double *fd = static_cast<double *>(f);
            if (energy)
                hipLaunchKernelGGL((k_lj64<kTPA, true>), dim3(gb), dim3(kBlock), 0, s, n, x, off, idx, p, fd, part);
            else
                hipLaunchKernelGGL((k_lj64<kTPA, false>), dim3(gb), dim3(kBlock), 0, s, n, x, off, idx, p, fd, part);
        } else {
            const double two32 = 4294967296.0;
            LJ32 p;
            p.sx = float(box->L[0] / two32);
            p.sy = float(box->L[1] / two32);
            p.sz = float(box->L[2] / two32);
            p.rc2 = float(lj->rc * lj->rc);
            p.sig2 = float(lj->sigma * lj->sigma);
            p.eps4 = float(4.0 * lj->eps);
            p.eps24 = float(24.0 * lj->eps);
            const uint4 *q = reinterpret_cast<const uint4 *>(xs);
            float *ff = static_cast<float *>(f);
            const bool comp = !(flags & MD_NO_COMPENSATE);
            if (energy && comp)
                hipLaunchKernelGGL((k_lj32<kTPA, true, true>), dim3(gb), dim3(kBlock), 0, s, n, q, off, idx, p, ff, part);
            else if (energy)
                hipLaunchKernelGGL((k_lj32<kTPA, true, false>), dim3(gb), dim3(kBlock), 0, s, n, q, off, idx, p, ff, part);
            else if (comp)
                hipLaunchKernelGGL((k_lj32<kTPA, false, true>), dim3(gb), dim3(kBlock), 0, s, n, q, off, idx, p, ff, part);
            else
                hipLaunchKernelGGL((k_lj32<kTPA, false, false>), dim3(gb), dim3(kBlock), 0, s, n, q, off, idx, p, ff, part);
        }
        MD_HIP_TRY(hipGetLastError());
    }
    if (energy) return launch_reduce_partials(part, n > 0 ? gb : 0, nullptr, 0, ev, kReduceLJ, phi_rc, 0.0, s);
    return MD_OK;
}

int forces_eam(const md_box_t *box, int64_t n, uint32_t *xs, const int64_t *off, const int32_t *idx,
               const md_fs_t *fs, float *rho, float *fprime, float *f, double *ev, int32_t flags, void *ws,
               const WsLayout &w, hipStream_t s)
{
    const bool energy = flags & MD_ENERGY;
    const bool comp = !(flags & MD_NO_COMPENSATE);
    double *part1 = ws_ptr<double>(ws, w.red1);
    double *part2 = ws_ptr<double>(ws, w.red2);
    const uint32_t gb = blocks_for(n, kTPA);
    if (int64_t(gb) > w.red_blocks) return MD_ERR_WORKSPACE;
    const double two32 = 4294967296.0;
    FS32 p;
    p.sx = float(box->L[0] / two32);
    p.sy = float(box->L[1] / two32);
    p.sz = float(box->L[2] / two32);
    p.d = float(fs->d);
    p.d2 = float(fs->d * fs->d);
    p.c = float(fs->c);
    p.c2 = float(fs->c * fs->c);
    p.p0 = float(fs->c0 + fs->c1 * fs->c + fs->c2 * fs->c * fs->c);
    p.p1 = float(fs->c1 + 2.0 * fs->c2 * fs->c);
    p.p2 = float(fs->c2);
    p.A = float(fs->A);
    uint4 *q = reinterpret_cast<uint4 *>(xs);
    if (n > 0) {
#define MD_EAM_LAUNCH(E, C)                                                                                   \
    hipLaunchKernelGGL((k_eam_rho<kTPA, E, C>), dim3(gb), dim3(kBlock), 0, s, n, q, off, idx, p, rho, fprime, \
                       part1);                                                                                \
    hipLaunchKernelGGL((k_eam_force<kTPA, E, C>), dim3(gb), dim3(kBlock), 0, s, n, q, off, idx, p, f, part2)
        if (energy && comp) { MD_EAM_LAUNCH(true, true); }
        else if (energy) { MD_EAM_LAUNCH(true, false); }
        else if (comp) { MD_EAM_LAUNCH(false, true); }
        else { MD_EAM_LAUNCH(false, false); }
#undef MD_EAM_LAUNCH
        MD_HIP_TRY(hipGetLastError());
    }
    if (energy)
        return launch_reduce_partials(part1, n > 0 ? gb : 0, part2, n > 0 ? gb : 0, ev, kReduceEAM, 0.0, 0.0, s);
    return MD_OK;
}

}  // namespace md
