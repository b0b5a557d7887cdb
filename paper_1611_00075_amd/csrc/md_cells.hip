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
    slot[i] = atomicAdd(&cnt[r], 1);
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

constexpr int kNbTile = 1024;          // candidates staged in LDS at once
constexpr int kNbHome = 64;            // home atoms per pass
constexpr int kMaxStencil = 125;       // (2*reach+1)^3, reach <= 2

// distinct values of (c + o) mod nc, o in [-reach, reach], in increasing o
__device__ __forceinline__ int stencil_axis(int32_t c, int32_t nc, int32_t reach, int32_t *out)
{
    int m = 0;
    for (int o = -reach; o <= reach; ++o) {
        int32_t v = ((c + o) % nc + nc) % nc;
        bool dup = false;
        for (int k = 0; k < m; ++k) dup |= (out[k] == v);
        if (!dup) out[m++] = v;
    }
    return m;
}

__device__ __forceinline__ double minimg(double d, double L, double hL)
{
    if (d > hL)
        d -= L;
    else if (d < -hL)
        d += L;
    return d;
}

// One block per cell (Morton rank).  The atoms of the up to 27 (125)
// neighbouring cells are contiguous runs of the sorted arrays; they are
// staged in LDS tiles, and each wave tests one home atom against 64
// candidates at a time, compacting hits with a ballot.  COUNT writes the row
// lengths, FILL the rows (candidate order: stencil cell, then sorted index).
template <bool FILL>
__global__ __launch_bounds__(kBlock) void k_neighbors(int64_t n, const double *x, GridArgs g, double rl2,
                                                      const int32_t *cell_start, const int32_t *rank2lin,
                                                      const int32_t *lin2rank, int32_t *count,
                                                      const int64_t *offsets, int32_t *idx)
{
    __shared__ double sx[kNbTile], sy[kNbTile], sz[kNbTile];
    __shared__ int32_t sj[kNbTile];
    __shared__ int32_t rstart[kMaxStencil], rbase[kMaxStencil + 1];
    __shared__ int32_t run[kNbHome];
    __shared__ int32_t nst;

    const uint32_t rank = xcd_block(blockIdx.x, gridDim.x);
    const int32_t h0 = cell_start[rank], h1 = cell_start[rank + 1];
    if (h0 == h1) return;

    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    if (threadIdx.x == 0) {
        const int32_t lin = rank2lin[rank];
        const int32_t cx = lin % g.nc[0], cy = (lin / g.nc[0]) % g.nc[1], cz = lin / (g.nc[0] * g.nc[1]);
        int32_t ax[5], ay[5], az[5];
        const int mx = stencil_axis(cx, g.nc[0], g.reach, ax);
        const int my = stencil_axis(cy, g.nc[1], g.reach, ay);
        const int mz = stencil_axis(cz, g.nc[2], g.reach, az);
        int m = 0, base = 0;
        for (int c = 0; c < mz; ++c)
            for (int b = 0; b < my; ++b)
                for (int a = 0; a < mx; ++a) {
                    const int64_t l = ax[a] + int64_t(g.nc[0]) * (ay[b] + int64_t(g.nc[1]) * az[c]);
                    const int32_t r = lin2rank[l];
                    rstart[m] = cell_start[r];
                    rbase[m] = base;
                    base += cell_start[r + 1] - cell_start[r];
                    ++m;
                }
        rbase[m] = base;
        nst = m;
    }
    __syncthreads();
    const int m = nst;
    const int32_t total = rbase[m];

    for (int32_t hb = h0; hb < h1; hb += kNbHome) {
        const int32_t hn = min(kNbHome, h1 - hb);
        if (threadIdx.x < hn) run[threadIdx.x] = 0;
        __syncthreads();
        for (int32_t t0 = 0; t0 < total; t0 += kNbTile) {
            const int32_t tn = min(kNbTile, total - t0);
            for (int32_t q = threadIdx.x; q < tn; q += kBlock) {
                const int32_t gq = t0 + q;
                int lo = 0, hi = m - 1;           // last range with rbase <= gq
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (rbase[mid] <= gq) lo = mid; else hi = mid - 1;
                }
                const int32_t j = rstart[lo] + (gq - rbase[lo]);
                sj[q] = j;
                sx[q] = x[j];
                sy[q] = x[n + j];
                sz[q] = x[2 * n + j];
            }
            __syncthreads();
            for (int32_t h = wave; h < hn; h += kBlock / kWave) {
                const int32_t i = hb + h;
                const double xi = x[i], yi = x[n + i], zi = x[2 * n + i];
                int32_t r = run[h];
                const int64_t rowb = FILL ? offsets[i] : 0;
                for (int32_t c0 = 0; c0 < tn; c0 += kWave) {
                    const int32_t q = c0 + lane;
                    bool hit = false;
                    int32_t j = -1;
                    if (q < tn) {
                        j = sj[q];
                        const double dx = minimg(sx[q] - xi, g.L[0], g.hL[0]);
                        const double dy = minimg(sy[q] - yi, g.L[1], g.hL[1]);
                        const double dz = minimg(sz[q] - zi, g.L[2], g.hL[2]);
                        const double r2 = (dx * dx + dy * dy) + dz * dz;
                        hit = (j != i) && (r2 < rl2);
                    }
                    const uint64_t mask = __ballot(hit);
                    if (FILL && hit) {
                        const int pos = __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
                        idx[rowb + r + pos] = j;
                    }
                    r += __popcll(mask);
                }
                if (lane == 0) run[h] = r;
            }
            __syncthreads();
        }
        if (!FILL && threadIdx.x < hn) count[hb + threadIdx.x] = run[threadIdx.x];
        __syncthreads();
    }
}

int build_neighbors(const md_grid_t *grid, int64_t n, const double *x, const int32_t *cell_start, int64_t *offsets,
                    int32_t *idx, int64_t capacity, int64_t *needed, void *ws, const WsLayout &w, hipStream_t s)
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
    int32_t *cnt = ws_ptr<int32_t>(ws, w.nbcnt);
    const uint32_t nb = uint32_t(grid->n_cells);
    if (n > 0) {
        hipLaunchKernelGGL(k_neighbors<false>, dim3(nb), dim3(kBlock), 0, s, n, x, g, rl2, cell_start,
                           ws_ptr<int32_t>(ws, w.rank2lin), ws_ptr<int32_t>(ws, w.lin2rank), cnt,
                           (const int64_t *)nullptr, (int32_t *)nullptr);
        MD_HIP_TRY(hipGetLastError());
    }
    int rc = launch_scan_i32_to_i64(cnt, offsets, n, ws_ptr<int64_t>(ws, w.scan), s);
    if (rc) return rc;
    int64_t total = 0;
    MD_HIP_TRY(hipMemcpyAsync(&total, offsets + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MD_HIP_TRY(hipStreamSynchronize(s));
    *needed = total;
    if (total > capacity) return MD_ERR_CAPACITY;
    if (n > 0 && total > 0) {
        hipLaunchKernelGGL(k_neighbors<true>, dim3(nb), dim3(kBlock), 0, s, n, x, g, rl2, cell_start,
                           ws_ptr<int32_t>(ws, w.rank2lin), ws_ptr<int32_t>(ws, w.lin2rank), (int32_t *)nullptr,
                           offsets, idx);
        MD_HIP_TRY(hipGetLastError());
    }
    return MD_OK;
}

}  // namespace md
