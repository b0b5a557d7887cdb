// Domain decomposition on one device: bricks with ghost layers, the halo
// exchange (pack, transfer, unpack) and the inner/outer split of the force
// step (Sec. 2.1's hybrid algorithm; its steps pack boundary coordinates,
// send, receive, compute forces inside the domain, wait, compute forces
// across the boundary, wait).
//
// Directions: d = (ex + 1) + 3 (ey + 1) + 9 (ez + 1) for e in {-1, 0, 1}^3,
// d = 13 the brick itself.  A ghost entry of target brick t with direction
// d is a copy of an atom of brick s = t - e (periodically): e_a = +1 puts
// it in t's lower halo cell layer (cell 0), e_a = -1 in the upper one
// (cell k+1).  Frame offsets off[t * 27 + d] take a position of the source
// (wrapped into the box at the last build) to t's frame: periodic shift,
// minus t's origin, plus one cell.
#include <algorithm>
#include <cmath>
#include <vector>

#include "md_pair.h"

namespace md {
namespace {

constexpr int kDirs = 27;
constexpr int kSelf = 13;

struct DdGeom {
    double L[3], B[3], c[3], inv_b[3];
    int32_t p[3], k[3];
};

__device__ __forceinline__ double dd_wrap(double x, double L)
{
    double w = x - L * floor(x / L);
    if (w >= L) w -= L;
    if (w < 0.0) w += L;
    return w;
}

__device__ __forceinline__ int32_t brick_coord(double w, double inv_b, int32_t p)
{
    int32_t b = int32_t(w * inv_b);
    b = b >= p ? p - 1 : b;
    return b < 0 ? 0 : b;
}

// wrap in place; key = brick (bx + px (by + py bz))
__global__ __launch_bounds__(kBlock) void k_dd_keys(int64_t n, double *x, DdGeom g, int32_t *key)
{
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    int32_t b[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double w = dd_wrap(x[a * n + i], g.L[a]);
        x[a * n + i] = w;
        b[a] = brick_coord(w, g.inv_b[a], g.p[a]);
    }
    key[i] = b[0] + g.p[0] * (b[1] + g.p[1] * b[2]);
}

// ---- stable partition by a small integer key ----
// hist[k * nb + blk] = members of key k in block blk
__global__ __launch_bounds__(kBlock) void k_part_hist(int64_t n, const int32_t *key, int32_t K, int32_t *hist)
{
    extern __shared__ int32_t cnt[];
    for (int k = threadIdx.x; k < K; k += kBlock) cnt[k] = 0;
    __syncthreads();
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&cnt[key[i]], 1);
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += kBlock) hist[int64_t(k) * gridDim.x + blockIdx.x] = cnt[k];
}

// members of one key keep their index order: rank in the wave from ballots,
// ranks of earlier waves of the block from per-wave counts in LDS
__global__ __launch_bounds__(kBlock) void k_part_scatter(int64_t n, const int32_t *key, int32_t K,
                                                         const int32_t *offs, int32_t *perm)
{
    extern __shared__ int32_t wc[];   // [kBlock / kWave][K]
    constexpr int kWaves = kBlock / kWave;
    for (int k = threadIdx.x; k < kWaves * K; k += kBlock) wc[k] = 0;
    __syncthreads();
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const bool in = i < n;
    const int32_t r = in ? key[i] : -1;
    int32_t rank = 0;
    uint64_t todo = __ballot(in);
    while (todo) {
        const int leader = __builtin_ctzll(todo);
        const int32_t rc = __builtin_amdgcn_readlane(r, leader);
        const uint64_t same = __ballot(r == rc) & todo;
        if (lane == leader) wc[wave * K + rc] = __popcll(same);
        if (r == rc) rank = __popcll(same & ((uint64_t(1) << lane) - 1));
        todo &= ~same;
    }
    __syncthreads();
    if (in) {
        for (int w = 0; w < wave; ++w) rank += wc[w * K + r];
        perm[offs[int64_t(r) * gridDim.x + blockIdx.x] + rank] = int32_t(i);
    }
}

__global__ void k_part_starts(const int32_t *offs, int32_t K, int32_t nb, int32_t *start)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k <= K) start[k] = offs[int64_t(k) * nb];
}

// ---- ghost selection ----
__device__ __forceinline__ void dir_of(int d, int (&e)[3])
{
    e[0] = d % 3 - 1;
    e[1] = (d / 3) % 3 - 1;
    e[2] = d / 9 - 1;
}

// directions in which atom i is a ghost of a neighbouring brick
__global__ __launch_bounds__(kBlock) void k_dd_mask(int64_t n, const double *x, DdGeom g, uint32_t *mask,
                                                    int32_t *cnt)
{
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    bool lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double w = x[a * n + i];
        const int32_t b = brick_coord(w, g.inv_b[a], g.p[a]);
        const double u = w - b * g.B[a];
        lo[a] = u < g.c[a];
        hi[a] = u >= g.B[a] - g.c[a];
    }
    uint32_t m = 0;
    for (int d = 0; d < kDirs; ++d) {
        if (d == kSelf) continue;
        int e[3];
        dir_of(d, e);
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) ok = ok && (e[a] == 0 || (e[a] > 0 ? hi[a] : lo[a]));
        m |= ok ? (1u << d) : 0u;
    }
    mask[i] = m;
    cnt[i] = __popc(m);
}

// entries (atom, key = target * 27 + d) in atom order
__global__ __launch_bounds__(kBlock) void k_dd_expand(int64_t n, const double *x, DdGeom g, const uint32_t *mask,
                                                      const int32_t *eoff, int32_t *ent_atom, int32_t *ent_key)
{
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    int32_t b[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) b[a] = brick_coord(x[a * n + i], g.inv_b[a], g.p[a]);
    uint32_t m = mask[i];
    int32_t o = eoff[i];
    while (m) {
        const int d = __builtin_ctz(m);
        m &= m - 1;
        int e[3];
        dir_of(d, e);
        int32_t t[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) t[a] = (b[a] + e[a] + g.p[a]) % g.p[a];
        ent_atom[o] = int32_t(i);
        ent_key[o] = (t[0] + g.p[0] * (t[1] + g.p[1] * t[2])) * kDirs + d;
        ++o;
    }
}

__global__ __launch_bounds__(kBlock) void k_dd_gather_entries(int64_t m, const int32_t *order,
                                                              const int32_t *ent_atom, const int32_t *ent_key,
                                                              int32_t *src, int32_t *code)
{
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= m) return;
    const int32_t j = order[k];
    src[k] = ent_atom[j];
    code[k] = ent_key[j];
}

// one brick's atoms and ghosts in its frame: true positions and the
// positions that decide the cell (local axes clamped inside the brick,
// halo axes at the middle of their halo cell)
__global__ __launch_bounds__(kBlock) void k_dd_assemble(int64_t m, int64_t nt, int64_t b0, int64_t g0,
                                                        const double *x, int64_t n, const int32_t *gh_src,
                                                        const int32_t *gh_code, const double *off, int32_t t,
                                                        DdGeom g, double *xt, double *xb)
{
    const int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (j >= m) return;
    int64_t src;
    int32_t code;
    if (j < nt) {
        src = b0 + j;
        code = t * kDirs + kSelf;
    } else {
        src = gh_src[g0 + j - nt];
        code = gh_code[g0 + j - nt];
    }
    int e[3];
    dir_of(code % kDirs, e);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double p = x[a * n + src] + off[code * 3 + a];
        xt[a * m + j] = p;
        const double c = g.c[a];
        const double lo = c * (1.0 + 1e-9), hi = c * (g.k[a] + 1) * (1.0 - 1e-9);
        xb[a * m + j] = e[a] > 0 ? 0.5 * c : (e[a] < 0 ? (g.k[a] + 1.5) * c : fmin(fmax(p, lo), hi));
    }
}

// after a brick's sort: where its atoms came from (gperm) and where its
// ghosts went (gh_slot)
// (the cell order puts a brick's own atoms first; an atom on the wrong side
// of nt would be a broken invariant: it is flagged and not written)
__global__ __launch_bounds__(kBlock) void k_dd_after_sort(int64_t m, int64_t nt, int64_t b0, int64_t g0,
                                                          int64_t slot0, const int32_t *perm, int32_t *gperm,
                                                          int32_t *gh_slot, int32_t *bad)
{
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= m) return;
    const int32_t a = perm[k];
    if ((k < nt) != (a < nt) || a < 0 || a >= m) {
        atomicOr(bad, 1);
        return;
    }
    if (k < nt) gperm[b0 + k] = int32_t(b0 + a);
    else gh_slot[g0 + (a - nt)] = int32_t(slot0 + k);
}

__global__ __launch_bounds__(kBlock) void k_dd_invert(int64_t n, const int32_t *gperm, int32_t *inv)
{
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) inv[gperm[i]] = int32_t(i);
}

__device__ __forceinline__ int brick_of(int64_t i, const int64_t *bstart, int nb)
{
    int lo = 0, hi = nb;   // bstart[lo] <= i < bstart[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (bstart[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_dd_remap(int64_t m, const int32_t *inv, int32_t *gh_src,
                                                     int32_t *gh_src_slot, const int64_t *bstart,
                                                     const int64_t *slot0, int nb)
{
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= m) return;
    const int32_t s = inv[gh_src[k]];
    gh_src[k] = s;
    const int b = brick_of(s, bstart, nb);
    gh_src_slot[k] = int32_t(slot0[b] + (s - bstart[b]));
}

// ---- the per-step exchange ----
__device__ __forceinline__ uint32_t to_fixed(double x, double k)
{
    return uint32_t(uint64_t(__double2ll_rn(x * k)));
}

struct Scale {
    double k[3];   // 2^32 / frame edge
};

__global__ __launch_bounds__(kBlock) void k_dd_scale_local(int64_t n, const double *x, const int64_t *bstart,
                                                           const int64_t *slot0, int nb, const double *off,
                                                           Scale sc, uint4 *xs)
{
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const int b = brick_of(i, bstart, nb);
    const double *o = off + (b * kDirs + kSelf) * 3;
    xs[slot0[b] + (i - bstart[b])] = make_uint4(to_fixed(x[i] + o[0], sc.k[0]), to_fixed(x[n + i] + o[1], sc.k[1]),
                                                to_fixed(x[2 * n + i] + o[2], sc.k[2]), 0u);
}

// velocity-Verlet kick (hk = the half kicks due, dt/2 or dt, times the
// acceleration per unit force) and drift, the displacement rebuild check
// against xref (status[0] = 1), and the new local coordinates written
// straight into the brick frames (what k_dd_scale_local does)
struct DdDrift {
    double hk, dt, hs2, L[3], hL[3];
};

__global__ __launch_bounds__(kBlock) void k_dd_kick_drift(int64_t n, double *x, double *v, const float *f,
                                                          const double *xref, int32_t *status, const int64_t *bstart,
                                                          const int64_t *slot0, int nb, const double *off, Scale sc,
                                                          DdDrift a, uint4 *xs)
{
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    bool moved = false, bad = false;
    if (i < n) {
        double p[3];
        double r2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double vc = v[c * n + i] + a.hk * double(f[c * n + i]);
            v[c * n + i] = vc;
            p[c] = x[c * n + i] + a.dt * vc;
            x[c * n + i] = p[c];
            bad |= !isfinite(p[c]);
            double d = p[c] - xref[c * n + i];
            d = d > a.hL[c] ? d - a.L[c] : (d < -a.hL[c] ? d + a.L[c] : d);
            r2 = c == 0 ? d * d : (c == 1 ? r2 + d * d : r2 + d * d);
        }
        moved = r2 > a.hs2;
        const int b = brick_of(i, bstart, nb);
        const double *o = off + (b * kDirs + kSelf) * 3;
        xs[slot0[b] + (i - bstart[b])] = make_uint4(to_fixed(p[0] + o[0], sc.k[0]), to_fixed(p[1] + o[1], sc.k[1]),
                                                    to_fixed(p[2] + o[2], sc.k[2]), 0u);
    }
    if (__ballot(moved) && (threadIdx.x % kWave) == 0) status[0] = 1;
    if (__ballot(bad) && (threadIdx.x % kWave) == 0) atomicOr(&status[1], 1);
}

__global__ __launch_bounds__(kBlock) void k_dd_pack(int64_t m, const double *x, int64_t n, const int32_t *src,
                                                    double *send)
{
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= m) return;
    const int32_t j = src[k];
    send[k] = x[j];
    send[m + k] = x[n + j];
    send[2 * m + k] = x[2 * n + j];
}

__global__ __launch_bounds__(kBlock) void k_dd_unpack(int64_t m, const double *recv, const int32_t *slot,
                                                      const int32_t *code, const double *off, Scale sc, uint4 *xs)
{
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= m) return;
    const double *o = off + code[k] * 3;
    xs[slot[k]] = make_uint4(to_fixed(recv[k] + o[0], sc.k[0]), to_fixed(recv[m + k] + o[1], sc.k[1]),
                             to_fixed(recv[2 * m + k] + o[2], sc.k[2]), 0u);
}

__global__ __launch_bounds__(kBlock) void k_dd_pack_w(int64_t m, const uint4 *xs, const int32_t *src_slot,
                                                      uint32_t *send)
{
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (k < m) send[k] = xs[src_slot[k]].w;
}

__global__ __launch_bounds__(kBlock) void k_dd_unpack_w(int64_t m, const uint32_t *recv, const int32_t *slot,
                                                        uint4 *xs)
{
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (k < m) xs[slot[k]].w = recv[k];
}

inline uint32_t blocks(int64_t n) { return uint32_t((n + kBlock - 1) / kBlock); }
inline size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

DdGeom geom(const md_dd_t *dd)
{
    DdGeom g;
    for (int a = 0; a < 3; ++a) {
        g.L[a] = dd->box.L[a];
        g.p[a] = dd->p[a];
        g.k[a] = dd->k[a];
        g.B[a] = dd->box.L[a] / dd->p[a];
        g.c[a] = dd->c[a];
        g.inv_b[a] = double(dd->p[a]) / dd->box.L[a];
    }
    return g;
}

// scratch layout in dws
struct DdScratch {
    size_t off, bstart, slot0, key, perm, mask, cnt, eoff, ent_atom, ent_key, order, hist, offs, starts, bsum,
        xt, xb, xsorted, cell, permt, cstart, gperm, inv, part1, part2, word, tab_in, tab_out, total;
    int64_t rows, hist_len;
};

DdScratch scratch_layout(const md_dd_t *dd)
{
    DdScratch l{};
    const int64_t n = std::max<int64_t>(dd->n, 1), gc = std::max<int64_t>(dd->ghost_cap, 1);
    const int64_t sc = std::max<int64_t>(dd->slot_cap, 1), P = std::max(dd->n_bricks, 1);
    const int64_t nbn = (n + kBlock - 1) / kBlock, nbg = (gc + kBlock - 1) / kBlock;
    l.hist_len = std::max(P * nbn, P * kDirs * nbg);
    const int64_t scan_len = std::max(l.hist_len, n) + 1;
    l.rows = n / 32 + 4 * P + 64;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o += up256(bytes);
        return r;
    };
    l.off = take(size_t(P) * kDirs * 3 * 8);
    l.bstart = take(size_t(P + 1) * 8);
    l.slot0 = take(size_t(P + 1) * 8);
    l.key = take(size_t(n) * 4);
    l.perm = take(size_t(n) * 4);
    l.mask = take(size_t(n) * 4);
    l.cnt = take(size_t(n) * 4);
    l.eoff = take(size_t(n + 1) * 4);
    l.ent_atom = take(size_t(gc) * 4);
    l.ent_key = take(size_t(gc) * 4);
    l.order = take(size_t(gc) * 4);
    l.hist = take(size_t(l.hist_len) * 4);
    l.offs = take(size_t(l.hist_len + 1) * 4);
    l.starts = take(size_t(P * kDirs + 1) * 4);
    l.bsum = take(size_t(scan_len / kScanTile + 2) * 8);
    l.xt = take(size_t(3 * sc) * 8);
    l.xb = take(size_t(3 * sc) * 8);
    l.xsorted = take(size_t(3 * sc) * 8);
    l.cell = take(size_t(sc) * 4);
    l.permt = take(size_t(sc) * 4);
    l.cstart = take(size_t(dd->vgrid.n_cells + 1) * 4);
    l.gperm = take(size_t(n) * 4);
    l.inv = take(size_t(n) * 4);
    l.part1 = take(size_t(l.rows) * 8 * 8);
    l.part2 = take(size_t(l.rows) * 8 * 8);
    l.word = take(64);
    l.tab_in = take(sizeof(BrickTab));
    l.tab_out = take(sizeof(BrickTab));
    l.total = o;
    return l;
}

// The inner (or outer) atoms of every brick as one launch: per brick the
// slices of its inner atoms (whole slices only) or the rest of its atoms.
// Returns the launch's logical blocks.
uint32_t fill_tab(const md_dd_t *dd, bool inner, BrickTab &t)
{
    t = BrickTab{};
    t.nb = dd->n_bricks;
    int64_t blk = 0;
    for (int e = 0; e < dd->n_bricks; ++e) {
        const int64_t nt = dd->brick_start[e + 1] - dd->brick_start[e];
        const int64_t gt = dd->ghost_start[e + 1] - dd->ghost_start[e];
        const uint32_t split = uint32_t(dd->n_inner[e] / kSlice);
        t.blk0[e] = blk;
        t.slot0[e] = dd->slot0[e];
        t.atom0[e] = dd->brick_start[e];
        t.n_xs[e] = nt + gt;
        t.slice0[e] = inner ? 0u : split;
        t.n_end[e] = inner ? int64_t(split) * kSlice : nt;
        const int64_t slices = (t.n_end[e] + kSlice - 1) / kSlice - int64_t(t.slice0[e]);
        blk += slices > 0 ? (slices + kBlock / kWave - 1) / (kBlock / kWave) : 0;
    }
    t.blk0[dd->n_bricks] = blk;
    return uint32_t(blk);
}

// stable partition of m keys in [0, K): perm and start[K + 1] (device)
int partition(int64_t m, const int32_t *key, int32_t K, int32_t *perm, int32_t *start, void *dws,
              const DdScratch &l, hipStream_t s)
{
    const uint32_t nb = std::max<uint32_t>(blocks(m), 1);
    if (int64_t(K) * nb > l.hist_len) return MD_ERR_WORKSPACE;
    int32_t *hist = ws_ptr<int32_t>(dws, l.hist), *offs = ws_ptr<int32_t>(dws, l.offs);
    hipLaunchKernelGGL(k_part_hist, dim3(nb), dim3(kBlock), size_t(K) * 4, s, m, key, K, hist);
    MD_HIP_TRY(hipGetLastError());
    if (int rc = launch_scan_i32_to_i32(hist, offs, int64_t(K) * nb, ws_ptr<int64_t>(dws, l.bsum), s)) return rc;
    if (m > 0) {
        hipLaunchKernelGGL(k_part_scatter, dim3(nb), dim3(kBlock), size_t(K) * 4 * (kBlock / kWave), s, m, key, K,
                           offs, perm);
        MD_HIP_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(k_part_starts, dim3((K + 1 + 255) / 256), dim3(256), 0, s, offs, K, int32_t(nb), start);
    MD_HIP_TRY(hipGetLastError());
    return MD_OK;
}

Scale frame_scale(const md_dd_t *dd)
{
    Scale sc;
    for (int a = 0; a < 3; ++a) sc.k[a] = 4294967296.0 / dd->vbox.L[a];
    return sc;
}

int get_events(md_dd_t *dd)
{
    for (int q = 0; q < 4; ++q)
        if (!dd->events[q]) {
            hipEvent_t e;
            MD_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            dd->events[q] = e;
        }
    return MD_OK;
}

}  // namespace
}  // namespace md

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace md;

extern "C" {

int md_dd_init(md_dd_t *dd, const md_box_t *box, const int32_t p[3], double r_list)
{
    if (!dd || !box || !p || !(r_list > 0.0) || !std::isfinite(r_list)) return MD_ERR_ARG;
    md_dd_t d = *dd;
    d.box = *box;
    d.n_bricks = 1;
    d.vgrid = md_grid_t{};
    d.vgrid.n_cells = 1;
    for (int a = 0; a < 3; ++a) {
        if (!(box->L[a] > 0.0) || !std::isfinite(box->L[a]) || p[a] < 1) return MD_ERR_BOX;
        d.p[a] = p[a];
        d.n_bricks *= p[a];
        const double B = box->L[a] / p[a];
        const double k = std::floor(B / (r_list * (1.0 + 1e-6)));
        if (k < 3.0 || k > 1000.0) return MD_ERR_BOX;
        d.k[a] = int32_t(k);
        d.c[a] = B / k;
        d.vbox.L[a] = (k + 3.0) * d.c[a];
        d.vgrid.L[a] = d.vbox.L[a];
        d.vgrid.nc[a] = d.k[a] + 3;
        d.vgrid.inv_cell[a] = double(d.vgrid.nc[a]) / d.vbox.L[a];
        d.vgrid.n_cells *= d.vgrid.nc[a];
    }
    if (d.n_bricks > MD_DD_MAX_BRICKS) return MD_ERR_BOX;
    d.vgrid.r_list = r_list;
    d.vgrid.reach = 1;
    d.inner_cells = int64_t(d.k[0] - 2) * (d.k[1] - 2) * (d.k[2] - 2);
    *dd = d;
    return MD_OK;
}

size_t md_dd_scratch_bytes(const md_dd_t *dd) { return dd ? scratch_layout(dd).total : 0; }

int md_dd_workspace_init(md_dd_t *dd, void *stream)
{
    if (!dd || !dd->vws || !dd->dws || dd->n_bricks < 1) return MD_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const DdScratch l = scratch_layout(dd);
    if (dd->dws_bytes < l.total) return MD_ERR_WORKSPACE;
    const md_grid_t &g = dd->vgrid;
    std::vector<int32_t> morton(size_t(g.n_cells)), rank(size_t(g.n_cells));
    if (int rc = md_grid_cell_ranks(&g, morton.data())) return rc;
    // class-major order: inner cells, outer cells, ghost and gap cells
    std::vector<std::pair<std::pair<int, int32_t>, int64_t>> v;
    v.reserve(size_t(g.n_cells));
    for (int64_t z = 0; z < g.nc[2]; ++z)
        for (int64_t y = 0; y < g.nc[1]; ++y)
            for (int64_t x = 0; x < g.nc[0]; ++x) {
                const int64_t c[3] = {x, y, z};
                int cls = 0;
                for (int a = 0; a < 3; ++a) {
                    if (c[a] < 1 || c[a] > dd->k[a]) cls = 2;
                    else if ((c[a] == 1 || c[a] == dd->k[a]) && cls < 1) cls = 1;
                }
                const int64_t lin = x + g.nc[0] * (y + g.nc[1] * z);
                v.push_back({{cls, morton[size_t(lin)]}, lin});
            }
    std::sort(v.begin(), v.end());
    for (size_t r = 0; r < v.size(); ++r) rank[size_t(v[r].second)] = int32_t(r);
    if (int rc = workspace_upload(&g, dd->slot_cap, rank.data(), dd->vws, dd->vws_bytes, s)) return rc;
    // frame offsets
    const DdGeom ge = geom(dd);
    std::vector<double> off(size_t(dd->n_bricks) * kDirs * 3);
    for (int t = 0; t < dd->n_bricks; ++t) {
        const int tc[3] = {t % dd->p[0], (t / dd->p[0]) % dd->p[1], t / (dd->p[0] * dd->p[1])};
        for (int d = 0; d < kDirs; ++d) {
            const int e[3] = {d % 3 - 1, (d / 3) % 3 - 1, d / 9 - 1};
            for (int a = 0; a < 3; ++a) {
                const int sa = ((tc[a] - e[a]) % dd->p[a] + dd->p[a]) % dd->p[a];
                const int raw = sa + e[a];
                const double shift = raw >= dd->p[a] ? -ge.L[a] : (raw < 0 ? ge.L[a] : 0.0);
                off[(size_t(t) * kDirs + d) * 3 + a] = shift - tc[a] * ge.B[a] + ge.c[a];
            }
        }
    }
    MD_HIP_TRY(hipMemcpyAsync(ws_ptr<double>(dd->dws, l.off), off.data(), off.size() * 8, hipMemcpyHostToDevice, s));
    MD_HIP_TRY(hipStreamSynchronize(s));
    return MD_OK;
}

int md_dd_rebuild(md_dd_t *dd, void *stream)
{
    if (!dd || dd->n < 1 || !dd->x || !dd->v || !dd->xref || !dd->ids || !dd->x2 || !dd->v2 || !dd->ids2 ||
        !dd->xs || !dd->count || !dd->idx || !dd->gh_src || !dd->gh_slot || !dd->gh_code || !dd->gh_src_slot ||
        !dd->vws || !dd->dws || dd->row_cap < 8 || dd->row_cap % 8 || dd->row_cap > MD_MAX_ROW_CAP ||
        dd->n > MD_MAX_ATOMS_FP32 || dd->slot_cap > MD_MAX_ATOMS_FP32)
        return MD_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const DdScratch l = scratch_layout(dd);
    if (dd->dws_bytes < l.total) return MD_ERR_WORKSPACE;
    const WsLayout wl = ws_layout(dd->vgrid.n_cells, dd->slot_cap);
    if (dd->vws_bytes < wl.total) return MD_ERR_WORKSPACE;
    const int64_t n = dd->n;
    const int P = dd->n_bricks;
    const DdGeom g = geom(dd);
    void *ws = dd->dws;
    int32_t *key = ws_ptr<int32_t>(ws, l.key), *perm = ws_ptr<int32_t>(ws, l.perm);
    int32_t *starts = ws_ptr<int32_t>(ws, l.starts);

    // 1. wrap, brick keys, stable regrouping by brick
    hipLaunchKernelGGL(k_dd_keys, dim3(blocks(n)), dim3(kBlock), 0, s, n, dd->x, g, key);
    MD_HIP_TRY(hipGetLastError());
    if (int rc = partition(n, key, P, perm, starts, ws, l, s)) return rc;
    std::vector<int32_t> hs(size_t(P) * kDirs + 1);
    MD_HIP_TRY(hipMemcpyAsync(hs.data(), starts, size_t(P + 1) * 4, hipMemcpyDeviceToHost, s));
    if (int rc = permute(n, 3, perm, dd->x, dd->x2, 8, s)) return rc;
    if (int rc = permute(n, 3, perm, dd->v, dd->v2, 8, s)) return rc;
    if (int rc = permute(n, 1, perm, dd->ids, dd->ids2, 4, s)) return rc;
    MD_HIP_TRY(hipMemcpyAsync(dd->x, dd->x2, size_t(3 * n) * 8, hipMemcpyDeviceToDevice, s));
    MD_HIP_TRY(hipMemcpyAsync(dd->v, dd->v2, size_t(3 * n) * 8, hipMemcpyDeviceToDevice, s));
    MD_HIP_TRY(hipMemcpyAsync(dd->ids, dd->ids2, size_t(n) * 4, hipMemcpyDeviceToDevice, s));
    MD_HIP_TRY(hipStreamSynchronize(s));
    for (int t = 0; t <= P; ++t) dd->brick_start[t] = hs[size_t(t)];

    // 2. ghost entries: directions per atom, expanded in atom order, grouped
    //    by (target brick, direction) keeping atom order
    uint32_t *mask = ws_ptr<uint32_t>(ws, l.mask);
    int32_t *cnt = ws_ptr<int32_t>(ws, l.cnt), *eoff = ws_ptr<int32_t>(ws, l.eoff);
    hipLaunchKernelGGL(k_dd_mask, dim3(blocks(n)), dim3(kBlock), 0, s, n, dd->x, g, mask, cnt);
    MD_HIP_TRY(hipGetLastError());
    if (int rc = launch_scan_i32_to_i32(cnt, eoff, n, ws_ptr<int64_t>(ws, l.bsum), s)) return rc;
    int32_t G = 0;
    MD_HIP_TRY(hipMemcpyAsync(&G, eoff + n, 4, hipMemcpyDeviceToHost, s));
    MD_HIP_TRY(hipStreamSynchronize(s));
    if (G > dd->ghost_cap) {
        dd->ghost_needed = G;
        return MD_ERR_CAPACITY;
    }
    int32_t *ent_atom = ws_ptr<int32_t>(ws, l.ent_atom), *ent_key = ws_ptr<int32_t>(ws, l.ent_key);
    int32_t *order = ws_ptr<int32_t>(ws, l.order);
    hipLaunchKernelGGL(k_dd_expand, dim3(blocks(n)), dim3(kBlock), 0, s, n, dd->x, g, mask, eoff, ent_atom, ent_key);
    MD_HIP_TRY(hipGetLastError());
    if (int rc = partition(G, ent_key, P * kDirs, order, starts, ws, l, s)) return rc;
    if (G > 0) {
        hipLaunchKernelGGL(k_dd_gather_entries, dim3(blocks(G)), dim3(kBlock), 0, s, G, order, ent_atom, ent_key,
                           dd->gh_src, dd->gh_code);
        MD_HIP_TRY(hipGetLastError());
    }
    MD_HIP_TRY(hipMemcpyAsync(hs.data(), starts, hs.size() * 4, hipMemcpyDeviceToHost, s));
    MD_HIP_TRY(hipStreamSynchronize(s));
    dd->n_ghost = G;
    for (int t = 0; t <= P; ++t) dd->ghost_start[t] = hs[size_t(t) * kDirs];
    // slots: each brick's atoms then ghosts, 8-aligned
    int64_t o = 0;
    for (int t = 0; t < P; ++t) {
        dd->slot0[t] = o;
        const int64_t m = (dd->brick_start[t + 1] - dd->brick_start[t]) + (dd->ghost_start[t + 1] - dd->ghost_start[t]);
        o += (m + 7) / 8 * 8;
    }
    dd->slot0[P] = o;
    if (o > dd->slot_cap) {
        dd->slot_needed = o;
        return MD_ERR_CAPACITY;
    }

    // 3. per brick: frame positions, cell sort, lists
    double *xt = ws_ptr<double>(ws, l.xt), *xb = ws_ptr<double>(ws, l.xb), *xsorted = ws_ptr<double>(ws, l.xsorted);
    int32_t *cell = ws_ptr<int32_t>(ws, l.cell), *permt = ws_ptr<int32_t>(ws, l.permt);
    int32_t *cstart = ws_ptr<int32_t>(ws, l.cstart), *gperm = ws_ptr<int32_t>(ws, l.gperm);
    int32_t *word = ws_ptr<int32_t>(ws, l.word);
    const double *off = ws_ptr<double>(ws, l.off);
    int32_t longest_all = 0;
    int32_t *bad = word + 8;
    if (int rc = launch_fill_i32(bad, 1, 0, s)) return rc;
    for (int t = 0; t < P; ++t) {
        const int64_t nt = dd->brick_start[t + 1] - dd->brick_start[t];
        const int64_t gt = dd->ghost_start[t + 1] - dd->ghost_start[t];
        const int64_t m = nt + gt;
        dd->n_inner[t] = 0;
        if (m == 0) continue;
        hipLaunchKernelGGL(k_dd_assemble, dim3(blocks(m)), dim3(kBlock), 0, s, m, nt, dd->brick_start[t],
                           dd->ghost_start[t], dd->x, n, dd->gh_src, dd->gh_code, off, t, g, xt, xb);
        MD_HIP_TRY(hipGetLastError());
        if (int rc = bin_cells(&dd->vgrid, m, xb, cell, permt, cstart, dd->vws, wl, s)) return rc;
        if (int rc = permute(m, 3, permt, xt, xsorted, 8, s)) return rc;
        int32_t needed = 0;
        const int rc = build_neighbors(&dd->vgrid, m, xsorted, cstart, dd->row_cap, dd->idx + dd->slot0[t] * dd->row_cap,
                                       dd->count + dd->slot0[t], word, &needed, dd->vws, wl, s);
        if (rc != MD_OK && rc != MD_ERR_CAPACITY) return rc;
        longest_all = std::max(longest_all, needed);
        int32_t ni = 0;
        MD_HIP_TRY(hipMemcpyAsync(&ni, cstart + dd->inner_cells, 4, hipMemcpyDeviceToHost, s));
        hipLaunchKernelGGL(k_dd_after_sort, dim3(blocks(m)), dim3(kBlock), 0, s, m, nt, dd->brick_start[t],
                           dd->ghost_start[t], dd->slot0[t], permt, gperm, dd->gh_slot, bad);
        MD_HIP_TRY(hipGetLastError());
        MD_HIP_TRY(hipStreamSynchronize(s));
        dd->n_inner[t] = ni;
    }
    int32_t broken = 0;
    MD_HIP_TRY(hipMemcpyAsync(&broken, bad, 4, hipMemcpyDeviceToHost, s));
    MD_HIP_TRY(hipStreamSynchronize(s));
    if (broken) return MD_ERR_ARG;
    if (longest_all > dd->row_cap) {
        dd->row_cap_needed = longest_all;
        return MD_ERR_CAPACITY;
    }

    // 4. atoms into each brick's sorted order; ghost sources follow them
    if (int rc = permute(n, 3, gperm, dd->x, dd->x2, 8, s)) return rc;
    if (int rc = permute(n, 3, gperm, dd->v, dd->v2, 8, s)) return rc;
    if (int rc = permute(n, 1, gperm, dd->ids, dd->ids2, 4, s)) return rc;
    MD_HIP_TRY(hipMemcpyAsync(dd->x, dd->x2, size_t(3 * n) * 8, hipMemcpyDeviceToDevice, s));
    MD_HIP_TRY(hipMemcpyAsync(dd->v, dd->v2, size_t(3 * n) * 8, hipMemcpyDeviceToDevice, s));
    MD_HIP_TRY(hipMemcpyAsync(dd->ids, dd->ids2, size_t(n) * 4, hipMemcpyDeviceToDevice, s));
    MD_HIP_TRY(hipMemcpyAsync(dd->xref, dd->x, size_t(3 * n) * 8, hipMemcpyDeviceToDevice, s));
    int32_t *inv = ws_ptr<int32_t>(ws, l.inv);
    hipLaunchKernelGGL(k_dd_invert, dim3(blocks(n)), dim3(kBlock), 0, s, n, gperm, inv);
    MD_HIP_TRY(hipMemcpyAsync(ws_ptr<int64_t>(ws, l.bstart), dd->brick_start, size_t(P + 1) * 8,
                              hipMemcpyHostToDevice, s));
    MD_HIP_TRY(hipMemcpyAsync(ws_ptr<int64_t>(ws, l.slot0), dd->slot0, size_t(P + 1) * 8, hipMemcpyHostToDevice, s));
    if (G > 0) {
        hipLaunchKernelGGL(k_dd_remap, dim3(blocks(G)), dim3(kBlock), 0, s, int64_t(G), inv, dd->gh_src,
                           dd->gh_src_slot, ws_ptr<int64_t>(ws, l.bstart), ws_ptr<int64_t>(ws, l.slot0), P);
    }
    MD_HIP_TRY(hipGetLastError());
    BrickTab tin, tout;
    fill_tab(dd, true, tin);
    fill_tab(dd, false, tout);
    MD_HIP_TRY(hipMemcpyAsync(ws_ptr<char>(ws, l.tab_in), &tin, sizeof(BrickTab), hipMemcpyHostToDevice, s));
    MD_HIP_TRY(hipMemcpyAsync(ws_ptr<char>(ws, l.tab_out), &tout, sizeof(BrickTab), hipMemcpyHostToDevice, s));
    MD_HIP_TRY(hipStreamSynchronize(s));
    ++dd->builds;
    return MD_OK;
}

namespace {
int dd_forces(md_dd_t *dd, double *ev, int32_t flags, void *stream, void *comm, bool scale_local);
}

int md_dd_forces(md_dd_t *dd, double *ev, int32_t flags, void *stream, void *comm)
{
    return dd_forces(dd, ev, flags, stream, comm, true);
}

namespace {
int dd_forces(md_dd_t *dd, double *ev, int32_t flags, void *stream, void *comm, bool scale_local)
{
    if (!dd || dd->n < 1 || !dd->f || (dd->potential != MD_POT_LJ && dd->potential != MD_POT_EAM)) return MD_ERR_ARG;
    if (dd->potential == MD_POT_EAM && (!dd->rho || !dd->fprime)) return MD_ERR_ARG;
    if (flags & ~(MD_ENERGY | MD_NO_COMPENSATE)) return MD_ERR_ARG;
    if ((flags & MD_ENERGY) && !ev) return MD_ERR_ARG;
    if (dd->builds < 1) return MD_ERR_ARG;
    const DdScratch l = scratch_layout(dd);
    if (dd->dws_bytes < l.total) return MD_ERR_WORKSPACE;
    if (int rc = get_events(dd)) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream), sc = comm ? static_cast<hipStream_t>(comm) : s;
    hipEvent_t eL = static_cast<hipEvent_t>(dd->events[0]), eH = static_cast<hipEvent_t>(dd->events[1]);
    hipEvent_t eR = static_cast<hipEvent_t>(dd->events[2]), eF = static_cast<hipEvent_t>(dd->events[3]);
    const int64_t n = dd->n, G = dd->n_ghost;
    const int P = dd->n_bricks;
    const Scale scl = frame_scale(dd);
    void *ws = dd->dws;
    const double *off = ws_ptr<double>(ws, l.off);
    uint4 *xs = reinterpret_cast<uint4 *>(dd->xs);
    const int32_t fl = (flags | dd->flags) & (MD_ENERGY | MD_NO_COMPENSATE);

    // local coordinates into the brick frames (unless the drift wrote them)
    if (scale_local) {
        hipLaunchKernelGGL(k_dd_scale_local, dim3(blocks(n)), dim3(kBlock), 0, s, n, dd->x,
                           ws_ptr<int64_t>(ws, l.bstart), ws_ptr<int64_t>(ws, l.slot0), P, off, scl, xs);
        MD_HIP_TRY(hipGetLastError());
    }
    MD_HIP_TRY(hipEventRecord(eL, s));
    // halo positions: pack, transfer, unpack on the communication stream
    MD_HIP_TRY(hipStreamWaitEvent(sc, eL, 0));
    if (G > 0) {
        hipLaunchKernelGGL(k_dd_pack, dim3(blocks(G)), dim3(kBlock), 0, sc, G, dd->x, n, dd->gh_src, dd->send);
        MD_HIP_TRY(hipMemcpyAsync(dd->recv, dd->send, size_t(3 * G) * 8, hipMemcpyDeviceToDevice, sc));
        hipLaunchKernelGGL(k_dd_unpack, dim3(blocks(G)), dim3(kBlock), 0, sc, G, dd->recv, dd->gh_slot, dd->gh_code,
                           off, scl, xs);
        MD_HIP_TRY(hipGetLastError());
    }
    MD_HIP_TRY(hipEventRecord(eH, sc));

    double *part1 = ws_ptr<double>(ws, l.part1), *part2 = ws_ptr<double>(ws, l.part2);
    int64_t rows1 = 0, rows2 = 0;
    BrickTab host_tab;
    const uint32_t gb_in = fill_tab(dd, true, host_tab), gb_out = fill_tab(dd, false, host_tab);
    if (int64_t(gb_in) + gb_out > l.rows) return MD_ERR_WORKSPACE;
    const BrickTab *tab_in = ws_ptr<BrickTab>(ws, l.tab_in), *tab_out = ws_ptr<BrickTab>(ws, l.tab_out);
    // one phase (inner or outer atoms of every brick) of one pass, one launch
    auto phase = [&](int pass, bool inner) -> int {
        const BrickTab *tab = inner ? tab_in : tab_out;
        const uint32_t gb = inner ? gb_in : gb_out;
        int64_t &rows = pass == 2 ? rows2 : rows1;
        double *part = (pass == 2 ? part2 : part1) + rows * 8;
        int rc;
        if (dd->potential == MD_POT_LJ)
            rc = bricks_forces_lj(&dd->vbox, tab, gb, n, dd->xs, dd->row_cap, dd->idx, dd->count, &dd->lj, dd->f, fl,
                                  part, s);
        else
            rc = bricks_forces_eam(pass, &dd->vbox, tab, gb, n, dd->xs, dd->row_cap, dd->idx, dd->count, &dd->fs,
                                   dd->rho, dd->fprime, dd->f, fl, part, s);
        rows += gb;
        return rc;
    };
    if (dd->potential == MD_POT_LJ) {
        if (int rc = phase(1, true)) return rc;
        MD_HIP_TRY(hipStreamWaitEvent(s, eH, 0));
        if (int rc = phase(1, false)) return rc;
        if (fl & MD_ENERGY) {
            const double s2 = dd->lj.sigma * dd->lj.sigma / (dd->lj.rc * dd->lj.rc), s6 = s2 * s2 * s2;
            return launch_reduce_partials(part1, rows1, nullptr, 0, ev, kReduceLJ, 4.0 * dd->lj.eps * (s6 * s6 - s6),
                                          0.0, s);
        }
        return MD_OK;
    }
    // FS: densities (inner, then outer once the halo is in), F' of the atoms
    // others hold as ghosts exchanged while the inner pair forces run
    if (int rc = phase(1, true)) return rc;
    MD_HIP_TRY(hipStreamWaitEvent(s, eH, 0));
    if (int rc = phase(1, false)) return rc;
    MD_HIP_TRY(hipEventRecord(eR, s));
    MD_HIP_TRY(hipStreamWaitEvent(sc, eR, 0));
    if (G > 0) {
        hipLaunchKernelGGL(k_dd_pack_w, dim3(blocks(G)), dim3(kBlock), 0, sc, G, xs, dd->gh_src_slot, dd->send_w);
        MD_HIP_TRY(hipMemcpyAsync(dd->recv_w, dd->send_w, size_t(G) * 4, hipMemcpyDeviceToDevice, sc));
        hipLaunchKernelGGL(k_dd_unpack_w, dim3(blocks(G)), dim3(kBlock), 0, sc, G, dd->recv_w, dd->gh_slot, xs);
        MD_HIP_TRY(hipGetLastError());
    }
    MD_HIP_TRY(hipEventRecord(eF, sc));
    if (int rc = phase(2, true)) return rc;
    MD_HIP_TRY(hipStreamWaitEvent(s, eF, 0));
    if (int rc = phase(2, false)) return rc;
    if (fl & MD_ENERGY) return launch_reduce_partials(part1, rows1, part2, rows2, ev, kReduceEAM, 0.0, 0.0, s);
    return MD_OK;
}

}  // namespace

// Steps with the closing half kick of a step fused into the next step's
// kick-drift (one kick of dt), which also writes the brick-frame
// coordinates; the last step's closing kick is applied on return.
int md_dd_run(md_dd_t *dd, int64_t steps, double dt, double accel, double skin, void *stream, void *comm)
{
    if (!dd || steps < 0 || !dd->status || !(dt > 0.0) || !(skin > 0.0)) return MD_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dd->builds < 1) {
        if (int rc = md_dd_rebuild(dd, stream)) return rc;
        if (int rc = dd_forces(dd, nullptr, 0, stream, comm, true)) return rc;
    }
    const DdScratch l = scratch_layout(dd);
    if (dd->dws_bytes < l.total) return MD_ERR_WORKSPACE;
    DdDrift a;
    a.dt = dt;
    a.hs2 = 0.25 * skin * skin;
    for (int c = 0; c < 3; ++c) {
        a.L[c] = dd->box.L[c];
        a.hL[c] = 0.5 * dd->box.L[c];
    }
    const double hk = 0.5 * dt * accel;
    bool pending = false;   // the closing half kick of the last completed step
    for (int64_t k = 0; k < steps; ++k) {
        bool scaled = false;
        if (dd->phase == 0) {
            if (int rc = launch_fill_i32(dd->status, 2, 0, s)) return rc;
            a.hk = pending ? 2.0 * hk : hk;
            hipLaunchKernelGGL(k_dd_kick_drift, dim3(blocks(dd->n)), dim3(kBlock), 0, s, dd->n, dd->x, dd->v, dd->f,
                               dd->xref, dd->status, ws_ptr<int64_t>(dd->dws, l.bstart),
                               ws_ptr<int64_t>(dd->dws, l.slot0), dd->n_bricks, ws_ptr<double>(dd->dws, l.off),
                               frame_scale(dd), a, reinterpret_cast<uint4 *>(dd->xs));
            MD_HIP_TRY(hipGetLastError());
            pending = false;
            int32_t st[2] = {0, 0};
            MD_HIP_TRY(hipMemcpyAsync(st, dd->status, 8, hipMemcpyDeviceToHost, s));
            MD_HIP_TRY(hipStreamSynchronize(s));
            if (st[1]) return MD_ERR_NONFINITE;
            dd->phase = st[0] ? 2 : 1;
            scaled = !st[0];
        }
        if (dd->phase == 2) {
            if (int rc = md_dd_rebuild(dd, stream)) return rc;
            dd->phase = 1;
        }
        if (int rc = dd_forces(dd, nullptr, 0, stream, comm, !scaled)) return rc;
        pending = true;
        dd->phase = 0;
        ++dd->steps;
    }
    if (pending)
        if (int rc = md_integrate(MD_KICK, &dd->box, dd->n, dd->x, dd->v, dd->f, dt, accel, 1.0, nullptr, 0.0,
                                  nullptr, 0, nullptr, nullptr, 0, dd->vws, dd->vws_bytes, stream))
            return rc;
    return MD_OK;
}

int md_dd_release(md_dd_t *dd)
{
    if (!dd) return MD_ERR_ARG;
    int rc = MD_OK;
    for (int q = 0; q < 4; ++q)
        if (dd->events[q]) {
            if (hipEventDestroy(static_cast<hipEvent_t>(dd->events[q])) != hipSuccess) rc = MD_ERR_HIP;
            dd->events[q] = nullptr;
        }
    return rc;
}

}  // extern "C"
