// Internal helpers shared by the HIP translation units of libmd.so.
// gfx950 only: wave64, 8 XCDs, no portability layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "md.h"

namespace md {

constexpr int kWave = 64;
constexpr int kXcds = 8;          // MI355X: 8 accelerator complex dies
constexpr int kBlock = 256;       // threads per block for the streaming kernels

#define MD_HIP_TRY(expr)                                   \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return MD_ERR_HIP;           \
    } while (0)

// Workgroups are dispatched to the XCDs round-robin (block b runs on XCD
// b % 8).  xcd_chunked remaps so that each XCD processes chunks of C
// consecutive logical blocks, the chunks dealt to the XCDs in turn (XCD x
// takes chunks x, x + 8, x + 16, ...): with Morton-ordered atoms,
// neighbouring blocks share an XCD's L2 within a chunk, and work that is
// uneven along the order (a box half empty, a dense cluster) is spread over
// all XCDs.  (One contiguous range per XCD left the 32 M-atom slab's list
// build at 20 ms with half the CUs idle; chunks of 256 cells: 10.7 ms.)  A
// bijection on [0, G): blocks past the last whole round of 8 chunks keep
// their index.
__device__ __forceinline__ uint32_t xcd_chunked(uint32_t b, uint32_t G, uint32_t C)
{
    const uint32_t round = kXcds * C, full = G / round * round;
    if (b >= full) return b;
    const uint32_t x = b % kXcds, k = b / kXcds;   // k-th block dispatched to XCD x
    return ((k / C) * kXcds + x) * C + k % C;
}

// The mapping of the streaming and pair kernels: chunks of 512 blocks.
constexpr uint32_t kXcdChunk = 512;
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t G) { return xcd_chunked(b, G, kXcdChunk); }

// Device-side skip of a speculative launch: a gated kernel returns at once
// when *flag == tag or *over > limit (words written earlier on the same
// stream).
struct Gate {
    const int32_t *flag = nullptr;
    int32_t tag = 0;
    const int32_t *over = nullptr;
    int32_t limit = 0;
};
__device__ __forceinline__ bool gated(const Gate &g)
{
    return (g.flag && *g.flag == g.tag) || (g.over && *g.over > g.limit);
}

// Orders the LDS accesses of one wavefront around this point (the lanes of a
// wave exchange data through LDS without a block barrier).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T group_sum(T v, int width)
{
    for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sum of NV doubles over a block of kBlock threads in a fixed order; the
// result is valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds /* NV * kBlock/kWave */)
{
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] = group_sum(v[c], kWave);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) lds[wave * NV + c] = v[c];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            double s = 0.0;
            for (int w = 0; w < kBlock / kWave; ++w) s += lds[w * NV + c];
            v[c] = s;
        }
    }
}

// Workspace layout (bytes from the start of ws).  Every region is 256-byte
// aligned.
struct WsLayout {
    size_t status;    // int32[64]: [0] = init magic, [1] = grid n_cells check
    size_t lin2rank;  // int32[n_cells]
    size_t rank2lin;  // int32[n_cells]: packed cell coordinates of each rank
    size_t cell_cnt;  // int32[n_cells + 1]
    size_t slot;      // int32[n]
    size_t tmp;       // int32[n]
    size_t scan;      // int64[scan_blocks]
    size_t red1;      // double[red_blocks * 8]
    size_t red2;      // double[red_blocks * 8]
    size_t total;
    int64_t red_blocks;
};

constexpr int kScanItems = 8;                     // per thread
constexpr int kScanTile = kBlock * kScanItems;    // per block
constexpr int32_t kWsMagic = 0x4d443535;          // "MD55"
constexpr int kSlice = 8;                         // atoms per sliced-ELL slice

// The regions that depend only on n come first, so the force and kick calls
// can locate their reduction partials without the cell count.
inline WsLayout ws_layout(int64_t n_cells, int64_t n)
{
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    WsLayout w{};
    size_t o = 0;
    const int64_t nn = n > 0 ? n : 1;
    const int64_t m = (n_cells + 1 > nn + 1 ? n_cells + 1 : nn + 1);
    const int64_t scan_blocks = (m + kScanTile - 1) / kScanTile + 1;
    w.red_blocks = nn / 16 + 64;
    w.status = o;   o += up(64 * 4);
    w.red1 = o;     o += up(size_t(w.red_blocks) * 8 * 8);
    w.red2 = o;     o += up(size_t(w.red_blocks) * 8 * 8);
    w.slot = o;     o += up(size_t(nn) * 4);
    w.tmp = o;      o += up(size_t(nn) * 4);
    w.lin2rank = o; o += up(size_t(n_cells) * 4);
    w.rank2lin = o; o += up(size_t(n_cells) * 4);
    w.cell_cnt = o; o += up(size_t(n_cells + 1) * 4);
    w.scan = o;     o += up(size_t(scan_blocks) * 8);
    w.total = o;
    return w;
}

template <typename T>
inline T *ws_ptr(void *ws, size_t off) { return reinterpret_cast<T *>(static_cast<char *>(ws) + off); }

// ---- launchers implemented in the kernel translation units ----
int launch_fill_i32(int32_t *p, int64_t count, int32_t value, hipStream_t s);
// out[0] = 0, out[k+1] = sum_{q<=k} in[q], k < m.  OutT = int32_t or int64_t.
int launch_scan_i32_to_i32(const int32_t *in, int32_t *out, int64_t m, int64_t *bsum, hipStream_t s);
// out[c] = sum over nb partial rows of part[b*8 + c], fixed order; then the
// combination selected by `mode` (see md_reduce.hip).
int launch_reduce_partials(const double *part1, int64_t nb1, const double *part2, int64_t nb2,
                           double *out, int mode, double a0, double a1, hipStream_t s);

enum ReduceMode { kReduceLJ = 0, kReduceEAM = 1, kReduceKE = 2 };

// ---- the path's steps (argument checks are done by the C ABI) ----
int bin_cells(const md_grid_t *, int64_t, double *, int32_t *, int32_t *, int32_t *, void *, const WsLayout &,
              hipStream_t);
int permute(int64_t, int32_t, const int32_t *, const void *, void *, int32_t, hipStream_t);
int scale_positions(const md_box_t *, int64_t, const double *, uint32_t *, hipStream_t);
int reorder_state(int64_t n, const int32_t *perm, double *x, double *v, int32_t *ids, double *xref, double *vtmp,
                  int32_t *itmp, const md_box_t *box, uint32_t *xs, hipStream_t s);
int build_neighbors(const md_grid_t *, int64_t, const double *, const int32_t *, int32_t, int32_t *, int32_t *,
                    int32_t *, int32_t *, void *, const WsLayout &, hipStream_t);
int forces_lj(const md_box_t *, int64_t, const double *, const uint32_t *, int32_t, const int32_t *, const int32_t *,
              const md_lj_t *, void *, double *, int32_t, void *, const WsLayout &, hipStream_t, Gate = {});
// forces_lj with its per-block energy partials (8 doubles per block of
// kBlock / kSlice atoms, part_rows blocks at most) at `part`
int forces_lj_part(const md_box_t *, int64_t, const double *, const uint32_t *, int32_t, const int32_t *,
                   const int32_t *, const md_lj_t *, void *, double *, int32_t, double *, int64_t, hipStream_t,
                   Gate = {});
// argument checks of md_forces_lj (everything but the workspace)
int lj_args_check(const md_box_t *, int64_t, const double *, const uint32_t *, int32_t, const int32_t *,
                  const int32_t *, const md_lj_t *, const void *, const double *, int32_t);
int forces_eam(const md_box_t *, int64_t, uint32_t *, int32_t, const int32_t *, const int32_t *, const md_fs_t *,
               float *, float *, float *, float *, double *, int32_t, void *, const WsLayout &, hipStream_t,
               Gate = {});
int forces_tb(const md_box_t *, int64_t, uint32_t *, int32_t, const int32_t *, const int32_t *, const md_tb_t *,
              float *, float *, float *, float *, double *, int32_t, void *, const WsLayout &, hipStream_t,
              Gate = {});
int forces_tbm(const md_box_t *, int64_t, uint32_t *, int32_t, const int32_t *, const int32_t *, const md_tbm_t *,
               float *, float *, float *, float *, double *, int32_t, void *, const WsLayout &, hipStream_t,
               Gate = {});
int set_elements(int64_t, const int32_t *, uint32_t *, hipStream_t);
int workspace_upload(const md_grid_t *, int64_t, const int32_t *, void *, size_t, hipStream_t);
struct BrickTab;
int bricks_forces_lj(const md_box_t *, const BrickTab *, uint32_t, int64_t, const uint32_t *, int32_t, const int32_t *,
                     const int32_t *, const md_lj_t *, float *, int32_t, double *, hipStream_t, Gate = {});
int bricks_forces_eam(int, const md_box_t *, const BrickTab *, uint32_t, int64_t, uint32_t *, int32_t,
                      const int32_t *, const int32_t *, const md_fs_t *, float *, float *, float *, int32_t, double *,
                      hipStream_t, Gate = {});
bool tab_ok(const md_tab_t *);
int64_t tab_bytes(const md_tab_t *);
int tab_pack(const md_tab_t *, const double *, const double *, const double *, const double *, const double *,
             const double *, void *, hipStream_t);
int forces_tab(const md_box_t *, int64_t, uint32_t *, int32_t, const int32_t *, const int32_t *, const md_tab_t *,
               const void *, float *, float *, float *, float *, double *, int32_t, void *, const WsLayout &,
               hipStream_t, Gate = {});
int integrate(int32_t, const md_box_t *, int64_t, double *, double *, const void *, double, double, double,
              const double *, double, int32_t *, int32_t, uint32_t *, double *, int32_t, void *, const WsLayout &,
              hipStream_t);
int mlp_descriptors(const md_box_t *, int64_t, const uint32_t *, int32_t, const int32_t *, const int32_t *,
                    const md_mlp_t *, float *, hipStream_t);
int mlp_eval(int64_t, const float *, const md_mlp_t *, const uint16_t *, float *, float *, hipStream_t);
int forces_mlp(const md_box_t *, int64_t, const uint32_t *, int32_t, const int32_t *, const int32_t *,
               const md_mlp_t *, const uint16_t *, float *, int32_t *, int32_t *, float *, float *, double *, int32_t,
               void *, const WsLayout &, hipStream_t, Gate = {});
size_t mlp_workspace_bytes(int64_t batch);
int mlp_moments(int64_t, const float *, double *, void *, hipStream_t);
// gradient of the batch loss (grad, loss may be NULL); with adam, an Adam
// step on master/m1/m2 and the refreshed bfloat16 copy w_out
int mlp_grad_update(int64_t, const int32_t *, const float *, const float *, const md_mlp_t *, const uint16_t *,
                    float *, double *, const md_adam_t *, float *, float *, float *, uint16_t *, void *, hipStream_t);
int run(md_system_t *sys, int64_t steps, hipStream_t s);
int kick_drift(const md_box_t *box, int64_t n, double *x, double *v, const void *f, bool f64, double kick, double dt,
               const double *xref, double half_skin_sq, int32_t *status, int32_t tag, uint32_t *xs, hipStream_t s,
               bool keep_element = false);

}  // namespace md
