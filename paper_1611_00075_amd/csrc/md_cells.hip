// Steps a1-a3: wrap + cell assignment, stable counting sort into
// Morton-ordered cells, permutation of per-atom arrays, scaled coordinates,
// and full Verlet neighbour lists from LDS-staged neighbour-cell tiles.
//
// Every floating-point decision here (wrap, cell index, r^2 < r_list^2) is
// taken in FP64 with the operation order of the plain definition and no FMA
// contraction (the library is built with -ffp-contract=off), so cell
// assignments and neighbour sets are reproducible bit for bit.
#include "md_common.h"
#include "md_pair.h"

namespace md {

struct GridArgs {
    double L[3], hL[3], inv_cell[3];
    int32_t nc[3], reach;
};

__device__ __forceinline__ double wrap1(double x, double L)
{
    double w = x - L * floor(x / L);
    if (w >= L) w -= L;
    if (w < 0.0) w += L;
    return w;
}

__device__ __forceinline__ int32_t cell1(double w, double inv, int32_t nc)
{
    int32_t c = int32_t(w * inv);
    c = c >= nc ? nc - 1 : c;
    return c < 0 ? 0 : c;
}

// ---------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_bin_assign(int64_t n, double *x, GridArgs g, const int32_t *lin2rank,
                                                       int32_t *cell, int32_t *cnt, int32_t *slot)
{
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    int32_t c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double w = wrap1(x[a * n + i], g.L[a]);
        x[a * n + i] = w;
        c[a] = cell1(w, g.inv_cell[a], g.nc[a]);
    }
    const int64_t lin = c[0] + int64_t(g.nc[0]) * (c[1] + int64_t(g.nc[1]) * c[2]);
    const int32_t r = lin2rank[lin];
    cell[i] = r;
    // one atomic per distinct cell of the wave (atoms arrive nearly sorted):
    // the first remaining lane claims a run of slots for all lanes of its
    // cell, which take consecutive slots in lane order
    uint64_t todo = __ballot(true);
    while (todo) {
        const int leader = __builtin_ctzll(todo);
        const int32_t rc = __builtin_amdgcn_readlane(r, leader);
        const uint64_t same = __ballot(r == rc) & todo;
        int32_t base = 0;
        if ((threadIdx.x % kWave) == leader) base = atomicAdd(&cnt[rc], __popcll(same));
        base = __builtin_amdgcn_readlane(base, leader);
        if (r == rc && ((todo >> (threadIdx.x % kWave)) & 1u))
            slot[i] = base + __builtin_amdgcn_mbcnt_hi(uint32_t(same >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(same), 0u));
        todo &= ~same;
    }
}

__global__ __launch_bounds__(kBlock) void k_bin_scatter(int64_t n, const int32_t *cell, const int32_t *slot,
                                                        const int32_t *cell_start, int32_t *tmp)
{
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    tmp[cell_start[cell[i]] + slot[i]] = int32_t(i);
}

// The atomic slots give an arbitrary order inside each cell; restore input
// order (stability) by ranking each atom among the members of its cell.
__global__ __launch_bounds__(kBlock) void k_bin_stable(int64_t n, const int32_t *cell, const int32_t *tmp,
                                                       const int32_t *cell_start, int32_t *perm)
{
    const int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (p >= n) return;
    const int32_t i = tmp[p];
    const int32_t c = cell[i];
    const int32_t s0 = cell_start[c], s1 = cell_start[c + 1];
    int32_t rank = 0;
    for (int32_t q = s0; q < s1; ++q) rank += tmp[q] < i;
    perm[s0 + rank] = i;
}

int bin_cells(const md_grid_t *grid, int64_t n, double *x, int32_t *cell, int32_t *perm, int32_t *cell_start,
              void *ws, const WsLayout &w, hipStream_t s)
{
    GridArgs g;
    for (int a = 0; a < 3; ++a) {
        g.L[a] = grid->L[a];
        g.hL[a] = 0.5 * grid->L[a];
        g.inv_cell[a] = grid->inv_cell[a];
        g.nc[a] = grid->nc[a];
    }
    g.reach = grid->reach;
    int32_t *cnt = ws_ptr<int32_t>(ws, w.cell_cnt);
    int32_t *slot = ws_ptr<int32_t>(ws, w.slot);
    int32_t *tmp = ws_ptr<int32_t>(ws, w.tmp);
    int rc = launch_fill_i32(cnt, grid->n_cells + 1, 0, s);
    if (rc) return rc;
    if (n > 0) {
        const uint32_t gb = uint32_t((n + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_bin_assign, dim3(gb), dim3(kBlock), 0, s, n, x, g, ws_ptr<int32_t>(ws, w.lin2rank), cell,
                           cnt, slot);
        MD_HIP_TRY(hipGetLastError());
    }
    rc = launch_scan_i32_to_i32(cnt, cell_start, grid->n_cells, ws_ptr<int64_t>(ws, w.scan), s);
    if (rc) return rc;
    if (n > 0) {
        const uint32_t gb = uint32_t((n + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_bin_scatter, dim3(gb), dim3(kBlock), 0, s, n, cell, slot, cell_start, tmp);
        hipLaunchKernelGGL(k_bin_stable, dim3(gb), dim3(kBlock), 0, s, n, cell, tmp, cell_start, perm);
        MD_HIP_TRY(hipGetLastError());
    }
    return MD_OK;
}

// ---------------------------------------------------------------------------
// permutation and scaled coordinates
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kBlock) void k_permute(int64_t n, int32_t ncomp, const int32_t *perm, const T *src,
                                                    T *dst)
{
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= n) return;
    const int64_t j = perm[k];
    for (int32_t c = 0; c < ncomp; ++c) dst[c * n + k] = src[c * n + j];
}

int permute(int64_t n, int32_t ncomp, const int32_t *perm, const void *src, void *dst, int32_t eb, hipStream_t s)
{
    if (n <= 0) return MD_OK;
    const uint32_t gb = uint32_t((n + kBlock - 1) / kBlock);
    switch (eb) {
    case 4:
        hipLaunchKernelGGL(k_permute<uint32_t>, dim3(gb), dim3(kBlock), 0, s, n, ncomp, perm,
                           static_cast<const uint32_t *>(src), static_cast<uint32_t *>(dst));
        break;
    case 8:
        hipLaunchKernelGGL(k_permute<uint64_t>, dim3(gb), dim3(kBlock), 0, s, n, ncomp, perm,
                           static_cast<const uint64_t *>(src), static_cast<uint64_t *>(dst));
        break;
    case 16:
        hipLaunchKernelGGL(k_permute<uint4>, dim3(gb), dim3(kBlock), 0, s, n, ncomp, perm,
                           static_cast<const uint4 *>(src), static_cast<uint4 *>(dst));
        break;
    default:
        return MD_ERR_ARG;
    }
    MD_HIP_TRY(hipGetLastError());
    return MD_OK;
}

// fixed-point fraction of the box, modulo 2^32 (negative and >= L positions
// wrap by the integer conversion)
__device__ __forceinline__ uint32_t scale1(double x, double k)
{
    return uint32_t(uint64_t(__double2ll_rn(x * k)));
}

__global__ __launch_bounds__(kBlock) void k_scale(int64_t n, const double *x, double k0, double k1, double k2,
                                                  uint4 *xs)
{
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    xs[i] = make_uint4(scale1(x[i], k0), scale1(x[n + i], k1), scale1(x[2 * n + i], k2), 0u);
}

int scale_positions(const md_box_t *box, int64_t n, const double *x, uint32_t *xs, hipStream_t s)
{
    if (n <= 0) return MD_OK;
    const double two32 = 4294967296.0;
    const uint32_t gb = uint32_t((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_scale, dim3(gb), dim3(kBlock), 0, s, n, x, two32 / box->L[0], two32 / box->L[1],
                       two32 / box->L[2], reinterpret_cast<uint4 *>(xs));
    MD_HIP_TRY(hipGetLastError());
    return MD_OK;
}

// Positions, velocities and input indices into the sorted order in two
// passes: gather from the old order into xr (the new reference positions),
// vt and it; then copy vt, it and xr back into the state arrays and, with
// xs, write the scaled coordinates of the new positions.
__global__ __launch_bounds__(kBlock) void k_reorder_gather(int64_t n, const int32_t *__restrict__ perm,
                                                           const double *__restrict__ x,
                                                           const double *__restrict__ v,
                                                           const int32_t *__restrict__ ids, double *__restrict__ xr,
                                                           double *__restrict__ vt, int32_t *__restrict__ it)
{
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= n) return;
    const int64_t j = perm[k];
    for (int c = 0; c < 3; ++c) {
        xr[c * n + k] = x[c * n + j];
        vt[c * n + k] = v[c * n + j];
    }
    it[k] = ids[j];
}

__global__ __launch_bounds__(kBlock) void k_reorder_put(int64_t n, const double *__restrict__ xr,
                                                        const double *__restrict__ vt,
                                                        const int32_t *__restrict__ it, double *__restrict__ x,
                                                        double *__restrict__ v, int32_t *__restrict__ ids, double k0,
                                                        double k1, double k2, uint4 *__restrict__ xs)
{
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= n) return;
    double p[3];
    for (int c = 0; c < 3; ++c) {
        p[c] = xr[c * n + k];
        x[c * n + k] = p[c];
        v[c * n + k] = vt[c * n + k];
    }
    ids[k] = it[k];
    if (xs) xs[k] = make_uint4(scale1(p[0], k0), scale1(p[1], k1), scale1(p[2], k2), 0u);
}

int reorder_state(int64_t n, const int32_t *perm, double *x, double *v, int32_t *ids, double *xref, double *vtmp,
                  int32_t *itmp, const md_box_t *box, uint32_t *xs, hipStream_t s)
{
    if (n <= 0) return MD_OK;
    const double two32 = 4294967296.0;
    const uint32_t gb = uint32_t((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_reorder_gather, dim3(gb), dim3(kBlock), 0, s, n, perm, x, v, ids, xref, vtmp, itmp);
    hipLaunchKernelGGL(k_reorder_put, dim3(gb), dim3(kBlock), 0, s, n, xref, vtmp, itmp, x, v, ids,
                       two32 / box->L[0], two32 / box->L[1], two32 / box->L[2], reinterpret_cast<uint4 *>(xs));
    MD_HIP_TRY(hipGetLastError());
    return MD_OK;
}

// The element of each atom (0 or 1; only bit 0 is used) into the fourth word
// of its scaled coordinates.
__global__ __launch_bounds__(kBlock) void k_set_elements(int64_t n, const int32_t *types, uint4 *xs)
{
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) xs[i].w = uint32_t(types[i]) & 1u;
}

int set_elements(int64_t n, const int32_t *types, uint32_t *xs, hipStream_t s)
{
    if (n <= 0) return MD_OK;
    const uint32_t gb = uint32_t((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_set_elements, dim3(gb), dim3(kBlock), 0, s, n, types, reinterpret_cast<uint4 *>(xs));
    MD_HIP_TRY(hipGetLastError());
    return MD_OK;
}

// ---------------------------------------------------------------------------
// neighbour lists
// ---------------------------------------------------------------------------

constexpr int kMaxStencil = 125;       // (2*reach+1)^3, reach <= 2

// Distinct values of (c + o) mod nc, o in [-reach, reach], in increasing o;
// img[k] = floor((c + o) / nc) of the value's first offset: the periodic
// image of that stencil cell (the only one when no value was de-duplicated).
__device__ __forceinline__ int stencil_axis(int32_t c, int32_t nc, int32_t reach, int32_t *out, int32_t *img)
{
    int m = 0;
    for (int o = -reach; o <= reach; ++o) {
        int32_t v = c + o, k = 0;
        while (v < 0) {
            v += nc;
            --k;
        }
        while (v >= nc) {
            v -= nc;
            ++k;
        }
        bool dup = false;
        for (int q = 0; q < m; ++q) dup |= (out[q] == v);
        if (!dup) {
            img[m] = k;
            out[m++] = v;
        }
    }
    return m;
}

// Wave-uniform copies of values the compiler cannot prove uniform.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// The definition's minimum image without branches: subtracting 0, L or -L
// gives the same bits as leaving d alone, d - L or d + L.
__device__ __forceinline__ double minimg_sel(double d, double L, double hL)
{
    const double t = d > hL ? L : (d < -hL ? -L : 0.0);
    return d - t;
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

constexpr int kNbChunks = 4;                   // 64-candidate chunks held in registers at once
constexpr int kNbTile = kNbChunks * kWave;     // candidates per register tile
constexpr int kNbStage = 2 * kNbTile;          // staged candidates: a tile plus one raw tile's survivors
constexpr int kNbWaves = 1;                    // wavefronts (cells) per block
constexpr int kNbMap = 1024;                   // candidates whose stencil cell is tabulated in LDS
constexpr int kNbCellsPerWave = 1;             // consecutive cells (Morton ranks) per wavefront
constexpr uint32_t kNbXcdChunk = 256;          // consecutive blocks (cells) an XCD takes at a time
constexpr int kNbBlock = kNbWaves * kWave;

// Per-wave LDS state: the home atoms' positions (read back as broadcasts),
// the stencil's cell ranges with their periodic images, and the candidates
// that passed the bounding-box test, waiting for a register tile.
struct NbWaveLds {
    double hx[kWave], hy[kWave], hz[kWave];
    double box[6];                            // homes' bounding box: lo x, y, z, hi x, y, z
    int32_t rstart[kMaxStencil], rbase[kMaxStencil + 1], rimg[kMaxStencil];
    int32_t stage[kNbStage];
    uint8_t cmap[kNbMap];                     // stencil cell of each candidate (up to kNbMap)
};

// A tile of candidates in registers: lane l holds candidates l, 64 + l, ...
struct NbTile {
    double x[kNbChunks], y[kNbChunks], z[kNbChunks];
    int32_t j[kNbChunks];
};

// Home atom i (position xi, yi, zi; r entries so far) against the first NC
// chunks of the tile: every hit is appended to the row at r in candidate
// order; returns the new row length.  All chunks are tested before any is
// stored, so the NC chains are independent; only lanes with a hit store,
// through a buffer whose range ends at the row capacity (stores past it are
// dropped).
template <int NC, bool INTERIOR>
__device__ __forceinline__ uint32_t nb_home(const NbTile &T, double xi, double yi, double zi, int32_t i, uint32_t r,
                                            __amdgpu_buffer_rsrc_t row, double rl2, const GridArgs &g)
{
    uint64_t mk[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double dx = T.x[c] - xi, dy = T.y[c] - yi, dz = T.z[c] - zi;
        if (!INTERIOR) {
            dx = minimg_sel(dx, g.L[0], g.hL[0]);
            dy = minimg_sel(dy, g.L[1], g.hL[1]);
            dz = minimg_sel(dz, g.L[2], g.hL[2]);
        }
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        // the wave's hit mask straight from the two compares (r2 < rl2 as an
        // ordered less-than, so a +inf padding candidate never hits)
        mk[c] = __builtin_amdgcn_fcmp(r2, rl2, 4) & __builtin_amdgcn_ballot_w64(T.j[c] != i);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (!mk[c]) continue;   // no hit in this chunk (wave-uniform)
        const uint32_t e = __builtin_amdgcn_mbcnt_hi(uint32_t(mk[c] >> 32),
                                                     __builtin_amdgcn_mbcnt_lo(uint32_t(mk[c]), r));
        // entry e of the row at byte (e / 8) * 256 + (e % 8) * 4
        if (__builtin_amdgcn_inverse_ballot_w64(mk[c]))   // this lane's bit of the mask
            __builtin_amdgcn_raw_buffer_store_b32(T.j[c], row, (e << 2) + __umul24(e >> 3, 224u), 0, 0);
        r += uint32_t(__popcll(mk[c]));
    }
    return r;
}

// The home batches of one cell against its stencil's candidates; returns the
// longest row of the cell.
//
// Candidates are streamed 256 at a time from the stencil's cell ranges.  With
// `filter`, a candidate is kept only if it lies within r_list of the
// bounding box of the batch's home atoms (in its periodic image of the
// stencil; with a margin of 1e-9 of r_list^2, far above the rounding of
// either test, so no candidate that the exact test accepts is dropped).
// Kept candidates are staged in LDS; every 256 of them fill a register
// tile, against which each home atom is tested with the exact FP64 test.
template <bool INTERIOR>
__device__ __forceinline__ int32_t nb_cell(NbWaveLds &L, int64_t n, const double *x, const GridArgs &g, double rl2,
                                           double keep2, bool filter, int32_t h0, int32_t h1, int32_t m,
                                           int32_t total, int32_t row_cap, int32_t *idx, int32_t *count)
{
    const int lane = threadIdx.x % kWave;
    int top = 1;                              // highest power of two <= m
    while (2 * top <= m) top *= 2;
    int32_t longest = 0;
    const double inf = __builtin_inf();
    // bytes of one row seen as a buffer: its last entry (row_cap - 1) ends there
    const uint32_t row_bytes = uint32_t(row_cap) * 32u - 224u;

    for (int32_t hb = h0; hb < h1; hb += kWave) {
        const int32_t hn = min(kWave, h1 - hb);
        const int32_t hl = hb + min(lane, hn - 1);
        const double xh = x[hl], yh = x[n + hl], zh = x[2 * n + hl];
        L.hx[lane] = xh;
        L.hy[lane] = yh;
        L.hz[lane] = zh;
        // bounding box of the batch's homes (lanes past hn repeat the last home)
        if (filter) {
            const double b0 = wave_min(xh), b1 = wave_min(yh), b2 = wave_min(zh);
            const double b3 = wave_max(xh), b4 = wave_max(yh), b5 = wave_max(zh);
            if (lane == 0) {
                L.box[0] = b0, L.box[1] = b1, L.box[2] = b2;
                L.box[3] = b3, L.box[4] = b4, L.box[5] = b5;
            }
        }
        // first int32 of the lane's home row (slice block + position in the slice)
        const int64_t row_l = int64_t(hl >> 3) * row_cap * 8 + (hl & 7) * 8;
        wave_sync();
        int32_t run_l = 0;                                // row length of home atom `lane`
        int32_t fill = 0;                                 // staged candidates (wave-uniform)
        for (int32_t t0 = 0; t0 < total; t0 += kNbTile) {
            // a raw tile of up to 256 candidates, four independent chunks
            bool keep[kNbChunks];
            int32_t jr[kNbChunks];
#pragma unroll
            for (int c = 0; c < kNbChunks; ++c) {
                const int32_t gq = t0 + c * kWave + lane;
                keep[c] = false;
                jr[c] = 0;
                if (gq < total) {
                    // the stencil cell k of candidate gq: tabulated, or the last
                    // range with rbase[k] <= gq (rbase[m] = total never is)
                    int k = 0;
                    if (total <= kNbMap) {
                        k = L.cmap[gq];
                    } else {
                        for (int s = top; s > 0; s >>= 1) {
                            const int t = min(k + s, m);
                            k = L.rbase[t] <= gq ? t : k;
                        }
                    }
                    const int32_t j = L.rstart[k] + (gq - L.rbase[k]);
                    jr[c] = j;
                    keep[c] = true;
                    if (filter) {
                        double cx = x[j], cy = x[n + j], cz = x[2 * n + j];
                        if (!INTERIOR) {
                            const int32_t im = L.rimg[k];
                            cx += double((im & 3) - 1) * g.L[0];
                            cy += double(((im >> 2) & 3) - 1) * g.L[1];
                            cz += double(((im >> 4) & 3) - 1) * g.L[2];
                        }
                        const double dx = fmax(fmax(L.box[0] - cx, cx - L.box[3]), 0.0);
                        const double dy = fmax(fmax(L.box[1] - cy, cy - L.box[4]), 0.0);
                        const double dz = fmax(fmax(L.box[2] - cz, cz - L.box[5]), 0.0);
                        keep[c] = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx)) < keep2;
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < kNbChunks; ++c) {
                const uint64_t mk = __builtin_amdgcn_ballot_w64(keep[c]);
                if (keep[c])
                    L.stage[fill + int32_t(__builtin_amdgcn_mbcnt_hi(uint32_t(mk >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo(uint32_t(mk), 0u)))] =
                        jr[c];
                fill += __popcll(mk);
            }
            const bool last = t0 + kNbTile >= total;
            while (fill >= kNbTile || (last && fill > 0)) {
                wave_sync();
                const int32_t nt = min(fill, kNbTile);
                const int nch = (nt + kWave - 1) / kWave;
                NbTile T;
#pragma unroll
                for (int c = 0; c < kNbChunks; ++c) {
                    const int32_t q = c * kWave + lane;
                    T.j[c] = -1;
                    T.x[c] = T.y[c] = T.z[c] = inf;
                    if (q < nt) {
                        const int32_t jj = L.stage[q];
                        T.j[c] = jj;
                        T.x[c] = x[jj];
                        T.y[c] = x[n + jj];
                        T.z[c] = x[2 * n + jj];
                    }
                }
                for (int32_t h = 0; h < hn; ++h) {
                    const int32_t i = hb + h;
                    const uint32_t r = uint32_t(__builtin_amdgcn_readlane(run_l, h));
                    const int64_t ro = int64_t(uint32_t(__builtin_amdgcn_readlane(int32_t(row_l), h))) |
                                       (int64_t(__builtin_amdgcn_readlane(int32_t(row_l >> 32), h)) << 32);
                    const auto row = make_rsrc(idx + ro, row_bytes);
                    const double xi = L.hx[h], yi = L.hy[h], zi = L.hz[h];
                    uint32_t rn;
                    switch (nch) {
                    case 4: rn = nb_home<4, INTERIOR>(T, xi, yi, zi, i, r, row, rl2, g); break;
                    case 3: rn = nb_home<3, INTERIOR>(T, xi, yi, zi, i, r, row, rl2, g); break;
                    case 2: rn = nb_home<2, INTERIOR>(T, xi, yi, zi, i, r, row, rl2, g); break;
                    default: rn = nb_home<1, INTERIOR>(T, xi, yi, zi, i, r, row, rl2, g); break;
                    }
                    if (lane == h) run_l = int32_t(rn);
                }
                // candidates staged past the tile move to the front
                const int32_t left = fill - nt;
                int32_t v[kNbChunks];
#pragma unroll
                for (int c = 0; c < kNbChunks; ++c)
                    if (c * kWave + lane < left) v[c] = L.stage[nt + c * kWave + lane];
                wave_sync();
#pragma unroll
                for (int c = 0; c < kNbChunks; ++c)
                    if (c * kWave + lane < left) L.stage[c * kWave + lane] = v[c];
                fill = left;
                wave_sync();
            }
        }
        if (lane < hn) count[hb + lane] = run_l;
        longest = max(longest, lane < hn ? run_l : 0);
        wave_sync();
    }
    return longest;
}

// One wavefront per cell (Morton rank) in one-wave blocks, no block-wide
// barriers.  The atoms of the up to 27 (125) neighbouring cells are
// contiguous runs of the sorted arrays; the wave streams them, keeps those
// within reach of its homes' bounding box, and tests each home atom against
// 64 kept candidates at a time, compacting hits with a ballot straight into
// the sliced-ELL rows (entry e of atom i at
// idx[(i/8 * row_cap/8 + e/8) * 64 + (i%8) * 8 + e%8]).  Row order: stencil
// cell (x fastest), then sorted index.  Rows longer than row_cap are counted
// but truncated (the row is written through a buffer whose range ends at
// entry row_cap, so stores past it are dropped); the longest row length is
// folded into *max_count.
//
// Interior cells (no stencil cell wraps around the box and nc >= 2 reach + 2
// on every axis) use the plain difference x_j - x_i: every candidate is then
// closer than half a box, so the minimum-image correction of the definition
// never applies and the result is bitwise the same.  A padding candidate
// gives +inf in every branch, so it never passes r^2 < r_list^2.  The
// bounding-box filter runs when no stencil offset was de-duplicated on any
// axis (nc >= 2 reach + 1): each stencil cell is then one periodic image,
// the only one that can lie within r_list of a home.
// The rows of the atoms of cell `rank`; returns the cell's longest row.
__device__ __forceinline__ int32_t nb_one_cell(NbWaveLds &L, int64_t rank, int64_t n, const double *x,
                                               const GridArgs &g, double rl2, double keep2,
                                               const int32_t *cell_start, const int32_t *rank_xyz,
                                               const int32_t *lin2rank, int32_t row_cap, int32_t *idx,
                                               int32_t *count)
{
    const int lane = threadIdx.x % kWave;
    const int32_t h0 = uni(cell_start[rank]), h1 = uni(cell_start[rank + 1]);
    if (h0 == h1) return 0;

    const int32_t pk = uni(rank_xyz[rank]);   // packed cell coordinates
    const int32_t c3[3] = {pk & 1023, (pk >> 10) & 1023, pk >> 20};
    bool interior = true, nodup = true;
    for (int a = 0; a < 3; ++a) {
        interior &= (g.nc[a] >= 2 * g.reach + 2) && (c3[a] - g.reach >= 0) && (c3[a] + g.reach < g.nc[a]);
        nodup &= g.nc[a] >= 2 * g.reach + 1;
    }
    int32_t ax[5], ay[5], az[5], ix[5], iy[5], iz[5];
    const int mx = stencil_axis(c3[0], g.nc[0], g.reach, ax, ix);
    const int my = stencil_axis(c3[1], g.nc[1], g.reach, ay, iy);
    const int mz = stencil_axis(c3[2], g.nc[2], g.reach, az, iz);
    const int m = mx * my * mz;
    // stencil cells: lane t takes cells t and t + 64 (x-fastest order), reads
    // their ranges, and a shuffle scan forms the range prefix
    int32_t carry = 0;
    for (int t0 = 0; t0 < m; t0 += kWave) {
        const int t = t0 + lane;
        int32_t len = 0;
        if (t < m) {
            // t = a + mx (b + my c) for small mx, my: exact reciprocal multiplies
            const int q1 = (t * ((65536 + mx - 1) / mx)) >> 16;
            const int a = t - q1 * mx;
            const int c = (q1 * ((65536 + my - 1) / my)) >> 16;
            const int b = q1 - c * my;
            const int64_t l = ax[a] + int64_t(g.nc[0]) * (ay[b] + int64_t(g.nc[1]) * az[c]);
            const int32_t r = lin2rank[l];
            const int32_t st = cell_start[r];
            len = cell_start[r + 1] - st;
            L.rstart[t] = st;
            L.rimg[t] = (ix[a] + 1) | ((iy[b] + 1) << 2) | ((iz[c] + 1) << 4);
        }
        int32_t v = len;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int32_t u = __shfl_up(v, o, kWave);
            if (lane >= o) v += u;
        }
        if (t < m) L.rbase[t + 1] = carry + v;
        carry += __builtin_amdgcn_readlane(v, kWave - 1);
    }
    if (lane == 0) L.rbase[0] = 0;
    wave_sync();
    if (carry <= kNbMap)   // tabulate the stencil cell of every candidate: lane t writes cell t's run
        for (int t = lane; t < m; t += kWave)
            for (int32_t q = L.rbase[t], e = L.rbase[t + 1]; q < e; ++q) L.cmap[q] = uint8_t(t);
    wave_sync();
    return interior ? nb_cell<true>(L, n, x, g, rl2, keep2, nodup, h0, h1, m, carry, row_cap, idx, count)
                               : nb_cell<false>(L, n, x, g, rl2, keep2, nodup, h0, h1, m, carry, row_cap, idx, count);
}

// The per-wave LDS (about 6 KB) lets a CU hold 26 waves, 6 per SIMD; the
// register budget is set to match (80 VGPRs instead of the 83 the compiler
// would take, which allow only 5): the candidate gathers and the dependent
// loads of the stencil set-up need the waves to hide their latency.
__global__ __launch_bounds__(kNbBlock) __attribute__((amdgpu_waves_per_eu(6)))
void k_neighbors(int64_t n, const double *x, GridArgs g, double rl2, double keep2, int64_t n_cells,
                 const int32_t *cell_start, const int32_t *rank_xyz, const int32_t *lin2rank, int32_t row_cap,
                 int32_t *idx, int32_t *count, int32_t *max_count)
{
    __shared__ NbWaveLds lds_all[kNbWaves];
    const int lane = threadIdx.x % kWave, wave = uni(threadIdx.x / kWave);
    NbWaveLds &L = lds_all[wave];
    const int64_t first = (int64_t(xcd_chunked(blockIdx.x, gridDim.x, kNbXcdChunk)) * kNbWaves + wave) *
                          kNbCellsPerWave;
    int32_t longest = 0;
    for (int c = 0; c < kNbCellsPerWave && first + c < n_cells; ++c) {
        longest = max(longest, nb_one_cell(L, first + c, n, x, g, rl2, keep2, cell_start, rank_xyz, lin2rank,
                                           row_cap, idx, count));
        wave_sync();
    }
    for (int o = kWave / 2; o > 0; o >>= 1) longest = max(longest, __shfl_xor(longest, o, kWave));
    // *max_count only grows, so a wave whose longest row does not exceed a
    // value already there has nothing to add: the check keeps the atomics on
    // this one word (which the L2 serialises) to a few per launch
    if (lane == 0 && longest > __hip_atomic_load(max_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(max_count, longest);
}

int build_neighbors(const md_grid_t *grid, int64_t n, const double *x, const int32_t *cell_start, int32_t row_cap,
                    int32_t *idx, int32_t *count, int32_t *max_count, int32_t *needed, void *ws, const WsLayout &w,
                    hipStream_t s)
{
    GridArgs g;
    for (int a = 0; a < 3; ++a) {
        g.L[a] = grid->L[a];
        g.hL[a] = 0.5 * grid->L[a];
        g.inv_cell[a] = grid->inv_cell[a];
        g.nc[a] = grid->nc[a];
    }
    g.reach = grid->reach;
    const double rl2 = grid->r_list * grid->r_list;
    const double keep2 = rl2 * (1.0 + 1e-9);
    int rc = launch_fill_i32(max_count, 1, 0, s);
    if (rc) return rc;
    const int64_t per_block = int64_t(kNbWaves) * kNbCellsPerWave;
    const uint32_t nb = uint32_t((grid->n_cells + per_block - 1) / per_block);
    if (n > 0) {
        hipLaunchKernelGGL(k_neighbors, dim3(nb), dim3(kNbBlock), 0, s, n, x, g, rl2, keep2, grid->n_cells,
                           cell_start, ws_ptr<int32_t>(ws, w.rank2lin), ws_ptr<int32_t>(ws, w.lin2rank), row_cap, idx,
                           count, max_count);
        MD_HIP_TRY(hipGetLastError());
    }
    if (needed) {
        int32_t mc = 0;
        MD_HIP_TRY(hipMemcpyAsync(&mc, max_count, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        MD_HIP_TRY(hipStreamSynchronize(s));
        *needed = mc;
        if (mc > row_cap) return MD_ERR_CAPACITY;
    }
    return MD_OK;
}

}  // namespace md
