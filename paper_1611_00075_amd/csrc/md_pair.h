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

// s += v with the running error of the sum compensated (Kahan).
template <bool COMP>
__device__ __forceinline__ void acc_sum(float &s, float &c, float v)
{
    if (COMP) {
        const float y = v - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    } else {
        s += v;
    }
}

// Raw buffer resource over `bytes` bytes at `base` (gfx9 raw buffer
// semantics: a load at a byte offset >= bytes returns zero, so no load
// leaves the range).  base and bytes must be wave-uniform.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, int(bytes), 0x00020000);
}

// Compile-time flag handed to a row walk's body: whether slots of the
// batch may lie past the row's end (the body must then mask them).
template <bool M>
struct Masked {
    static constexpr bool value = M;
};

// Row walk through buffer loads.  The wavefront holds one slice of 8 atoms
// (lane = 8 * atom + sub); the slice's block of the list is one buffer
// (row_r, cap * 32 bytes), in which entry sub + 8 q of the lane's atom sits
// at byte q * 256 + 4 * lane: one lane offset plus an immediate per load.
// Per iteration each lane reads U entries, then their U positions (xs_r,
// 16 bytes per atom, WORDS = 3 or 4 words read), then calls
// body(pj, t, Masked<true>) with the U positions of entries t + 8 u.  For
// entries past the row end both loads are given an offset outside their
// buffer, so they move no data and return zero; the body masks them
// (t + 8 u >= cnt).
//
// MASKED = false drops the two per-slot selects: slots past the row end read
// whatever index the row holds there (or zero past the row's buffer), and
// the position load of any such index stays inside the positions' buffer
// or returns zero; the body masks those slots as before.  Fewer vector
// instructions for more gathered bytes: it pays for the forms whose pair
// terms are longest (the two-element tight-binding form).
template <int U, int WORDS, bool MASKED = true, typename Body>
__device__ __forceinline__ void walk_buf(const __amdgpu_buffer_rsrc_t &xs_r, const __amdgpu_buffer_rsrc_t &row_r,
                                         int32_t cnt, int sub, Body &&body)
{
    constexpr uint32_t kOut = 0xfffffff0u;   // beyond any buffer here
    uint32_t off = (threadIdx.x % kWave) * 4u;
    for (int32_t t = sub; t < cnt; t += U * kSlice, off += U * 256u) {
        bool ok[U];
        uint32_t j[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ok[u] = !MASKED || t + u * kSlice < cnt;
            j[u] = __builtin_amdgcn_raw_buffer_load_b32(row_r, ok[u] ? off + u * 256u : kOut, 0, 0);
        }
        uint4 pj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t o = ok[u] ? j[u] << 4 : kOut;
            if (WORDS == 4) {
                const auto v = __builtin_amdgcn_raw_buffer_load_b128(xs_r, o, 0, 0);
                pj[u] = make_uint4(v[0], v[1], v[2], v[3]);
            } else {
                const auto v = __builtin_amdgcn_raw_buffer_load_b96(xs_r, o, 0, 0);
                pj[u] = make_uint4(v[0], v[1], v[2], 0u);
            }
        }
        body(pj, t, Masked<true>{});
    }
}

// Row walk in two parts.  Full batches: while all U entries t + 8 u of the
// lane are inside the row, U indices then U positions are loaded with no
// per-slot selects and body(pj, t, Masked<false>) gets U positions, all of
// them real neighbours.  Tail (1 to U - 1 entries left): one batch of
// U - 1 slots, body(pj, t, Masked<true>) with pj of length U - 1; the loads
// of slots past the end are switched off in the execution mask (zeros in
// pj).  A lane given an out-of-range offset instead still passes through
// the gather's address processing and issue: masking took the LJ kernel
// from 0.130 to 0.1255 ms.  A lane thus evaluates fewer slots than
// U * ceil(cnt / 8U) and makes no selects in its full batches.  (What
// bounds the pair kernels is the list stream, 4 bytes per entry read once,
// together with the pair arithmetic; the position gathers add little.)
template <int U, int WORDS, typename Body>
__device__ __forceinline__ void walk_split(const __amdgpu_buffer_rsrc_t &xs_r, const __amdgpu_buffer_rsrc_t &row_r,
                                           int32_t cnt, int sub, Body &&body)
{
    static_assert(U > 1, "a tail batch holds U - 1 slots");
    auto pos = [&](uint32_t o) {
        if (WORDS == 4) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b128(xs_r, o, 0, 0);
            return make_uint4(v[0], v[1], v[2], v[3]);
        } else {
            const auto v = __builtin_amdgcn_raw_buffer_load_b96(xs_r, o, 0, 0);
            return make_uint4(v[0], v[1], v[2], 0u);
        }
    };
    uint32_t off = (threadIdx.x % kWave) * 4u;
    int32_t t = sub;
    for (; t + (U - 1) * kSlice < cnt; t += U * kSlice, off += U * 256u) {
        uint32_t j[U];
#pragma unroll
        for (int u = 0; u < U; ++u) j[u] = __builtin_amdgcn_raw_buffer_load_b32(row_r, off + u * 256u, 0, 0);
        uint4 pj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) pj[u] = pos(j[u] << 4);
        body(pj, t, Masked<false>{});
    }
    if (t < cnt) {
        constexpr int V = U - 1;
        bool ok[V];
        uint32_t j[V];
#pragma unroll
        for (int u = 0; u < V; ++u) {
            ok[u] = t + u * kSlice < cnt;
            j[u] = 0u;
            if (ok[u]) j[u] = __builtin_amdgcn_raw_buffer_load_b32(row_r, off + u * 256u, 0, 0);
        }
        uint4 pj[V];
#pragma unroll
        for (int u = 0; u < V; ++u) {
            pj[u] = make_uint4(0u, 0u, 0u, 0u);
            if (ok[u]) pj[u] = pos(j[u] << 4);
        }
        body(pj, t, Masked<true>{});
    }
}

// The row walk of a pair form: split (SPLIT) or whole batches with no
// selects (walk_buf without masking).
template <bool SPLIT, int U, int WORDS, typename Body>
__device__ __forceinline__ void walk_form(const __amdgpu_buffer_rsrc_t &xs_r, const __amdgpu_buffer_rsrc_t &row_r,
                                          int32_t cnt, int sub, Body &&body)
{
    if constexpr (SPLIT) walk_split<U, WORDS>(xs_r, row_r, cnt, sub, body);
    else walk_buf<U, WORDS, false>(xs_r, row_r, cnt, sub, body);
}

// The atoms a force launch covers: the slices from slice0 on, rows and
// outputs of atoms below n (the kernel's n argument); positions of the
// first n_xs atoms may be gathered (atoms from n to n_xs are ghost copies
// whose forces are not computed); force component c of atom i at
// f[c * fs + i].  Whole-system launches: n_xs = fs = n, slice0 = 0.
struct Span {
    int64_t n_xs;
    int64_t fs;
    uint32_t slice0;
};

__host__ __device__ inline Span whole(int64_t n) { return Span{n, n, 0u}; }

// Several bricks of a domain decomposition in one launch.  Logical block b
// belongs to brick e with blk0[e] <= b < blk0[e + 1]; for its blocks the
// kernel's position, list and count arrays start at the brick's first slot
// (slot0[e]) and its per-atom outputs at the brick's first atom (atom0[e]);
// its span is (n_xs[e], the launch's force stride, slice0[e]) over atoms
// below n_end[e] of the brick.
struct BrickTab {
    int32_t nb;
    int64_t blk0[MD_DD_MAX_BRICKS + 1];
    int64_t slot0[MD_DD_MAX_BRICKS], atom0[MD_DD_MAX_BRICKS], n_end[MD_DD_MAX_BRICKS], n_xs[MD_DD_MAX_BRICKS];
    uint32_t slice0[MD_DD_MAX_BRICKS];
};

struct BrickSel {
    uint32_t blk;                    // block within the brick's range
    int64_t slot0, atom0, n_end, n_xs;
    uint32_t slice0;
};

__device__ __forceinline__ BrickSel brick_select(const BrickTab *t, uint32_t b)
{
    int lo = 0, hi = t->nb;   // blk0[lo] <= b < blk0[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (t->blk0[mid] <= b) lo = mid;
        else hi = mid;
    }
    return {uint32_t(b - t->blk0[lo]), t->slot0[lo], t->atom0[lo], t->n_end[lo], t->n_xs[lo], t->slice0[lo]};
}

// Buffers of a force kernel's wavefront: the positions (n_xs < 2^28 atoms)
// and its slice's block of the list.
struct SliceBufs {
    __amdgpu_buffer_rsrc_t xs, row;
};

__device__ __forceinline__ SliceBufs slice_bufs(const void *xs, int64_t n_xs, const int32_t *idx, int32_t cap,
                                                uint32_t blk, uint32_t slice0 = 0)
{
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t slice = int64_t(slice0) + int64_t(blk) * (kBlock / kWave) + wave;
    return {make_rsrc(xs, uint32_t(n_xs) * 16u), make_rsrc(idx + slice * cap * kSlice, uint32_t(cap) * 32u)};
}

// A double from the lane that data-parallel-primitive control CTRL names
// (row and bank masks full): quad_perm 0xB1 = lane ^ 1, 0x4E = lane ^ 2,
// row_half_mirror 0x141 = 7 - lane within each group of 8.
template <int CTRL>
__device__ __forceinline__ double dpp_double(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// The 8 lanes of one atom are consecutive: combine over them in FP64, the
// pairwise order ((g0 + g1) + (g2 + g3)) + ((g4 + g5) + (g6 + g7)) in every
// lane.  All lanes of the wave must be active.
__device__ __forceinline__ double combine(float s, float c)
{
    double g = double(s) - double(c);
    g += dpp_double<0xb1>(g);
    g += dpp_double<0x4e>(g);
    g += dpp_double<0x141>(g);
    return g;
}

// Atom and lane-in-atom of this thread: a wave holds one slice of kSlice
// atoms, lane = kSlice * a + sub.
struct SliceLane {
    int64_t i;
    int sub;
};

__device__ __forceinline__ SliceLane slice_lane(uint32_t blk, uint32_t slice0 = 0)
{
    return {int64_t(slice0) * kSlice + int64_t(blk) * (kBlock / kSlice) + threadIdx.x / kSlice,
            int(threadIdx.x % kSlice)};
}

}  // namespace md
