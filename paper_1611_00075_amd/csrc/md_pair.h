// Pair-loop building blocks shared by the force kernels: compensated
// accumulation, displacements from scaled coordinates, the sliced-ELL row
// walk and the cross-lane combine of an atom's 8 partial sums.
#pragma once

#include "md_common.h"

namespace md {

template <bool COMP>
__device__ __forceinline__ void acc_add(float &s, float &c, float a, float b)
{
    // s += a * b, with the running error of the sum compensated
    if (COMP) {
        const float y = __builtin_fmaf(a, b, -c);
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    } else {
        s = __builtin_fmaf(a, b, s);
    }
}

// Displacement r_i - r_j from scaled coordinates.  CUBIC: in units of
// L/2^32 (no multiply); otherwise in physical units (ax = L_a / 2^32).
template <bool CUBIC>
__device__ __forceinline__ void disp(const uint4 &pi, const uint4 &pj, float ax, float ay, float az, float &dx,
                                     float &dy, float &dz)
{
    dx = float(int32_t(pi.x - pj.x));
    dy = float(int32_t(pi.y - pj.y));
    dz = float(int32_t(pi.z - pj.z));
    if (!CUBIC) {
        dx *= ax;
        dy *= ay;
        dz *= az;
    }
}

// Sliced-ELL row of atom i: entry e at row[(e / 8) * 64 + e % 8].
__device__ __forceinline__ const int32_t *ell_row(const int32_t *idx, int64_t i, int32_t cap)
{
    return idx + (int64_t(i / kSlice) * cap * kSlice + (i % kSlice) * kSlice);
}

__device__ __forceinline__ int64_t ell_pos(int32_t e) { return int64_t(e / kSlice) * (kSlice * kSlice) + e % kSlice; }

// Walk row entries [0, cnt) with stride U*TPA starting at `sub`;
// body(pj, valid).  With lane = 8 * atom + sub the lanes of a wave read one
// contiguous 256-byte run of the list per load, and each quarter-wave
// gathers 8 consecutive neighbours of one atom.
template <int TPA, int U, typename Body>
__device__ __forceinline__ void walk_row(const uint4 *__restrict__ xs, const int32_t *__restrict__ row, int32_t cnt,
                                         int sub, Body &&body)
{
    for (int32_t t = sub; t < cnt; t += U * TPA) {
        int32_t j[U];
#pragma unroll
        for (int u = 0; u < U; ++u) j[u] = row[ell_pos(min(t + u * TPA, cnt - 1))];
        uint4 pj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) pj[u] = xs[j[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) body(pj[u], t + u * TPA < cnt);
    }
}

// The 8 lanes of one atom are consecutive: combine over them in FP64.
__device__ __forceinline__ double combine(float s, float c)
{
    double g = double(s) - double(c);
#pragma unroll
    for (int o = 1; o < kSlice; o <<= 1) g += __shfl_xor(g, o, kWave);
    return g;
}

// Atom and lane-in-atom of this thread: a wave holds one slice of kSlice
// atoms, lane = kSlice * a + sub.
struct SliceLane {
    int64_t i;
    int sub;
};

__device__ __forceinline__ SliceLane slice_lane(uint32_t blk)
{
    return {int64_t(blk) * (kBlock / kSlice) + threadIdx.x / kSlice, int(threadIdx.x % kSlice)};
}

}  // namespace md
