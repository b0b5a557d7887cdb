// Steps a1-a3: wrap + cell assignment, stable counting sort into
// Morton-ordered cells, permutation of per-atom arrays, scaled coordinates,
// and full Verlet neighbour lists from LDS-staged neighbour-cell tiles.
//
// Every floating-point decision here (wrap, cell index, r^2 < r_list^2) is
// taken in FP64 with the operation order of the plain definition and no FMA
// contraction (the library is built with -ffp-contract=off), so cell
// assignments and neighbour sets are reproducible bit for bit.
#include "md_common.h"

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

// ---------------------------------------------------------------------------
// neighbour lists
// ---------------------------------------------------------------------------

constexpr int kMaxStencil = 125;       // (2*reach+1)^3, reach <= 2

// distinct values of (c + o) mod nc, o in [-reach, reach], in increasing o
__device__ __forceinline__ int stencil_axis(int32_t c, int32_t nc, int32_t reach, int32_t *out)
{
    int m = 0;
    for (int o = -reach; o <= reach; ++o) {
        int32_t v = c + o;
        while (v < 0) v += nc;
        while (v >= nc) v -= nc;
        bool dup = false;
        for (int k = 0; k < m; ++k) dup |= (out[k] == v);
        if (!dup) out[m++] = v;
    }
    return m;
}

// Wave-uniform copies of values the compiler cannot prove uniform.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double lane_f64(double v, int l)
{
    const int64_t b = __double_as_longlong(v);
    const int32_t lo = __builtin_amdgcn_readlane(int32_t(b), l), hi = __builtin_amdgcn_readlane(int32_t(b >> 32), l);
    return __longlong_as_double((int64_t(hi) << 32) | int64_t(uint32_t(lo)));
}

// The definition's minimum image without branches: subtracting 0, L or -L
// gives the same bits as leaving d alone, d - L or d + L.
__device__ __forceinline__ double minimg_sel(double d, double L, double hL)
{
    const double t = d > hL ? L : (d < -hL ? -L : 0.0);
    return d - t;
}

constexpr int kNbWaveTile = 128;       // candidates staged per wave at once
constexpr int kNbWaves = kBlock / kWave;

// Per-wave LDS state.
struct NbWaveLds {
    double sx[kNbWaveTile], sy[kNbWaveTile], sz[kNbWaveTile];
    int32_t sj[kNbWaveTile];
    int32_t rstart[kMaxStencil], rbase[kMaxStencil + 1];
};

// One wavefront per cell (Morton rank), four cells per block, no block-wide
// barriers.  The atoms of the up to 27 (125) neighbouring cells are
// contiguous runs of the sorted arrays; the wave stages them in LDS tiles of
// 128 and tests one home atom against 64 candidates at a time, compacting
// hits with a ballot straight into the sliced-ELL rows (entry e of atom i at
// idx[(i/8 * row_cap/8 + e/8) * 64 + (i%8) * 8 + e%8]).  Row order: stencil
// cell, then sorted
// index.  Rows longer than row_cap are counted but truncated; the longest
// row length is folded into *max_count.
//
// Interior cells (no stencil cell wraps around the box and nc >= 2 reach + 2
// on every axis) use the plain difference x_j - x_i: every candidate is then
// closer than half a box, so the minimum-image correction of the definition
// never applies and the result is bitwise the same.
__global__ __launch_bounds__(kBlock) void k_neighbors(int64_t n, const double *x, GridArgs g, double rl2,
                                                      int64_t n_cells, const int32_t *cell_start,
                                                      const int32_t *rank_xyz, const int32_t *lin2rank,
                                                      int32_t row_cap, int32_t *idx, int32_t *count,
                                                      int32_t *max_count)
{
    __shared__ NbWaveLds lds_all[kNbWaves];
    const int lane = threadIdx.x % kWave, wave = uni(threadIdx.x / kWave);
    NbWaveLds &L = lds_all[wave];
    const int64_t rank = int64_t(xcd_block(blockIdx.x, gridDim.x)) * kNbWaves + wave;
    if (rank >= n_cells) return;
    const int32_t h0 = uni(cell_start[rank]), h1 = uni(cell_start[rank + 1]);
    if (h0 == h1) return;

    // stencil cells: lane t takes cells t and t + 64 (x-fastest order), reads
    // their ranges, and a shuffle scan forms the range prefix
    const int32_t pk = uni(rank_xyz[rank]);   // packed cell coordinates
    const int32_t c3[3] = {pk & 1023, (pk >> 10) & 1023, pk >> 20};
    bool interior = true;
    for (int a = 0; a < 3; ++a)
        interior &= (g.nc[a] >= 2 * g.reach + 2) && (c3[a] - g.reach >= 0) && (c3[a] + g.reach < g.nc[a]);
    int32_t ax[5], ay[5], az[5];
    const int mx = stencil_axis(c3[0], g.nc[0], g.reach, ax);
    const int my = stencil_axis(c3[1], g.nc[1], g.reach, ay);
    const int mz = stencil_axis(c3[2], g.nc[2], g.reach, az);
    const int m = mx * my * mz;
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
    const int32_t total = carry;
    int32_t longest = 0;

    for (int32_t hb = h0; hb < h1; hb += kWave) {
        const int32_t hn = min(kWave, h1 - hb);
        // home positions, fetched once and broadcast with shuffles
        const int32_t hl = hb + min(lane, hn - 1);
        const double xl = x[hl], yl = x[n + hl], zl = x[2 * n + hl];
        int32_t run_l = 0;                                // row length of home atom `lane`
        for (int32_t t0 = 0; t0 < total; t0 += kNbWaveTile) {
            const int32_t tn = min(kNbWaveTile, total - t0);
            wave_sync();
            for (int32_t q = lane; q < tn; q += kWave) {
                const int32_t gq = t0 + q;
                int lo = 0, hi = m - 1;           // last range with rbase <= gq
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (L.rbase[mid] <= gq) lo = mid; else hi = mid - 1;
                }
                const int32_t j = L.rstart[lo] + (gq - L.rbase[lo]);
                L.sj[q] = j;
                L.sx[q] = x[j];
                L.sy[q] = x[n + j];
                L.sz[q] = x[2 * n + j];
            }
            wave_sync();
            for (int32_t h = 0; h < hn; ++h) {
                const int32_t i = hb + h;
                const double xi = lane_f64(xl, h), yi = lane_f64(yl, h), zi = lane_f64(zl, h);
                int32_t r = __builtin_amdgcn_readlane(run_l, h);
                int32_t *row = idx + (int64_t(i >> 3) * row_cap * 8 + (i & 7) * 8);
                for (int32_t c0 = 0; c0 < tn; c0 += kWave) {
                    const int32_t q = c0 + lane;
                    bool hit = false;
                    if (q < tn) {
                        double dx = L.sx[q] - xi, dy = L.sy[q] - yi, dz = L.sz[q] - zi;
                        if (!interior) {
                            dx = minimg_sel(dx, g.L[0], g.hL[0]);
                            dy = minimg_sel(dy, g.L[1], g.hL[1]);
                            dz = minimg_sel(dz, g.L[2], g.hL[2]);
                        }
                        const double r2 = (dx * dx + dy * dy) + dz * dz;
                        hit = (L.sj[q] != i) && (r2 < rl2);
                    }
                    const uint64_t mask = __ballot(hit);
                    if (hit) {
                        const int e = r + __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
                        if (e < row_cap) row[int64_t(e >> 3) * 64 + (e & 7)] = L.sj[q];
                    }
                    r += __popcll(mask);
                }
                if (lane == h) run_l = r;
            }
        }
        if (lane < hn) count[hb + lane] = run_l;
        longest = max(longest, lane < hn ? run_l : 0);
    }
    for (int o = kWave / 2; o > 0; o >>= 1) longest = max(longest, __shfl_xor(longest, o, kWave));
    if (lane == 0) atomicMax(max_count, longest);
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
    int rc = launch_fill_i32(max_count, 1, 0, s);
    if (rc) return rc;
    const uint32_t nb = uint32_t((grid->n_cells + kNbWaves - 1) / kNbWaves);
    if (n > 0) {
        hipLaunchKernelGGL(k_neighbors, dim3(nb), dim3(kBlock), 0, s, n, x, g, rl2, grid->n_cells, cell_start,
                           ws_ptr<int32_t>(ws, w.rank2lin), ws_ptr<int32_t>(ws, w.lin2rank), row_cap, idx, count,
                           max_count);
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
