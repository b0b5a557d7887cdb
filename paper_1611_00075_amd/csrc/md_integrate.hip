// Step a7: velocity Verlet (Sec. 3.3) in FP64 with the displacement
// rebuild check fused into the drift, and the kinetic-energy reduction fused
// into the second half kick.
#include "md_common.h"

namespace md {

struct DriftArgs {
    double hk, dt;         // hk = dt/2 * accel
    double L[3], hL[3];    // for the minimum image of x - xref
    double k[3];           // 2^32 / L, scaled coordinates
    double half_skin_sq;
    int32_t tag;
};

__device__ __forceinline__ double minimg_d(double d, double L, double hL)
{
    if (d > hL)
        d -= L;
    else if (d < -hL)
        d += L;
    return d;
}

template <typename FT, bool KEEP>
__global__ __launch_bounds__(kBlock) void k_kick_drift(int64_t n, double *__restrict__ x, double *__restrict__ v,
                                                       const FT *__restrict__ f, const double *__restrict__ xref,
                                                       int32_t *__restrict__ status, uint4 *__restrict__ xs,
                                                       DriftArgs a)
{
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    bool moved = false, bad = false;
    if (i < n) {
        double p[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double vc = v[c * n + i] + a.hk * double(f[c * n + i]);
            v[c * n + i] = vc;
            p[c] = x[c * n + i] + a.dt * vc;
            x[c * n + i] = p[c];
            bad |= !isfinite(p[c]);
        }
        if (xref) {
            const double dx = minimg_d(p[0] - xref[i], a.L[0], a.hL[0]);
            const double dy = minimg_d(p[1] - xref[n + i], a.L[1], a.hL[1]);
            const double dz = minimg_d(p[2] - xref[2 * n + i], a.L[2], a.hL[2]);
            moved = ((dx * dx + dy * dy) + dz * dz) > a.half_skin_sq;
        }
        if (xs)   // whole 16-byte words; with KEEP, bit 0 of the fourth word (the element) carried over
            xs[i] = make_uint4(uint32_t(uint64_t(__double2ll_rn(p[0] * a.k[0]))),
                               uint32_t(uint64_t(__double2ll_rn(p[1] * a.k[1]))),
                               uint32_t(uint64_t(__double2ll_rn(p[2] * a.k[2]))), KEEP ? xs[i].w & 1u : 0u);
    }
    // one store per wave that saw the condition (idempotent values)
    if (__ballot(moved) && (threadIdx.x % kWave) == 0) status[0] = a.tag;
    if (__ballot(bad) && (threadIdx.x % kWave) == 0) atomicOr(&status[1], 1);
}

template <typename FT, bool KE>
__global__ __launch_bounds__(kBlock) void k_kick(int64_t n, double *__restrict__ v, const FT *__restrict__ f,
                                                 double hk, double *__restrict__ part)
{
    const uint32_t blk = blockIdx.x;
    const int64_t i = int64_t(blk) * kBlock + threadIdx.x;
    double s = 0.0;
    if (i < n) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double vc = v[c * n + i] + hk * double(f[c * n + i]);
            v[c * n + i] = vc;
            s += vc * vc;
        }
    }
    if (KE) {
        __shared__ double lds[kBlock / kWave];
        double r[1] = {s};
        block_sum<1>(r, lds);
        if (threadIdx.x == 0) {
            part[int64_t(blk) * 8] = r[0];
            for (int c = 1; c < 8; ++c) part[int64_t(blk) * 8 + c] = 0.0;
        }
    }
}

// v += kick * f; x += dt v; rebuild check; scaled coordinates.  kick is
// dt/2 * accel for a half step, dt * accel when the closing half kick of the
// previous step is fused in (same forces).
int kick_drift(const md_box_t *box, int64_t n, double *x, double *v, const void *f, bool f64, double kick, double dt,
               const double *xref, double half_skin_sq, int32_t *status, int32_t tag, uint32_t *xs, hipStream_t s,
               bool keep_element)
{
    const uint32_t gb = uint32_t((n + kBlock - 1) / kBlock);
    if (n <= 0) return MD_OK;
    DriftArgs a;
    a.hk = kick;
    a.dt = dt;
    for (int c = 0; c < 3; ++c) {
        a.L[c] = box->L[c];
        a.hL[c] = 0.5 * box->L[c];
        a.k[c] = 4294967296.0 / box->L[c];
    }
    a.half_skin_sq = half_skin_sq;
    a.tag = tag;
    uint4 *q = reinterpret_cast<uint4 *>(xs);
    if (f64)
        hipLaunchKernelGGL((k_kick_drift<double, false>), dim3(gb), dim3(kBlock), 0, s, n, x, v,
                           static_cast<const double *>(f), xref, status, q, a);
    else if (keep_element)
        hipLaunchKernelGGL((k_kick_drift<float, true>), dim3(gb), dim3(kBlock), 0, s, n, x, v,
                           static_cast<const float *>(f), xref, status, q, a);
    else
        hipLaunchKernelGGL((k_kick_drift<float, false>), dim3(gb), dim3(kBlock), 0, s, n, x, v,
                           static_cast<const float *>(f), xref, status, q, a);
    MD_HIP_TRY(hipGetLastError());
    return MD_OK;
}

int integrate(int32_t phase, const md_box_t *box, int64_t n, double *x, double *v, const void *f, double dt,
              double accel, double mass, const double *xref, double half_skin_sq, int32_t *status, int32_t tag,
              uint32_t *xs, double *ke, int32_t flags, void *ws, const WsLayout &w, hipStream_t s)
{
    const bool f64 = flags & MD_PAIR_FP64;
    const double hk = 0.5 * dt * accel;
    const uint32_t gb = uint32_t((n + kBlock - 1) / kBlock);
    if (phase == MD_KICK_DRIFT)
        return kick_drift(box, n, x, v, f, f64, hk, dt, xref, half_skin_sq, status, tag, xs, s,
                          (flags & MD_XS_ELEMENT) != 0);
    if (phase != MD_KICK) return MD_ERR_ARG;
    double *part = ws_ptr<double>(ws, w.red1);
    if (int64_t(gb) > w.red_blocks) return MD_ERR_WORKSPACE;
    if (n > 0) {
        if (ke) {
            if (f64)
                hipLaunchKernelGGL((k_kick<double, true>), dim3(gb), dim3(kBlock), 0, s, n, v,
                                   static_cast<const double *>(f), hk, part);
            else
                hipLaunchKernelGGL((k_kick<float, true>), dim3(gb), dim3(kBlock), 0, s, n, v,
                                   static_cast<const float *>(f), hk, part);
        } else {
            if (f64)
                hipLaunchKernelGGL((k_kick<double, false>), dim3(gb), dim3(kBlock), 0, s, n, v,
                                   static_cast<const double *>(f), hk, part);
            else
                hipLaunchKernelGGL((k_kick<float, false>), dim3(gb), dim3(kBlock), 0, s, n, v,
                                   static_cast<const float *>(f), hk, part);
        }
        MD_HIP_TRY(hipGetLastError());
    }
    if (ke) return launch_reduce_partials(part, n > 0 ? gb : 0, nullptr, 0, ke, kReduceKE, mass, 0.0, s);
    return MD_OK;
}

}  // namespace md
