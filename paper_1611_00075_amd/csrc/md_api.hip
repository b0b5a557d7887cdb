// C ABI façade of libmd.so: argument checks, workspace layout, Morton
// tables, and dispatch to the kernel launchers.  See include/md.h.
#include <algorithm>
#include <cmath>
#include <vector>

#include "md_common.h"

using namespace md;

namespace {

inline hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

constexpr int64_t kMaxAtoms = 2147483646;  // int32 atom indices
// the FP32 pair kernels address the scaled coordinates (16 B per atom)
// through one 32-bit buffer range
constexpr int64_t kMaxAtomsXs = MD_MAX_ATOMS_FP32;

bool box_ok(const md_box_t *b)
{
    if (!b) return false;
    for (int a = 0; a < 3; ++a)
        if (!(b->L[a] > 0.0) || !std::isfinite(b->L[a])) return false;
    return true;
}

bool grid_ok(const md_grid_t *g)
{
    if (!g || g->n_cells <= 0 || (g->reach != 1 && g->reach != 2)) return false;
    int64_t c = 1;
    for (int a = 0; a < 3; ++a) {
        if (g->nc[a] < 1) return false;
        c *= g->nc[a];
    }
    return c == g->n_cells;
}

// Workspace validation: big enough for (grid, n) and initialised for a grid
// with the same number of cells.
int ws_check(const md_grid_t *g, int64_t n, void *ws, size_t bytes, WsLayout &w)
{
    if (!ws) return MD_ERR_WORKSPACE;
    w = ws_layout(g ? g->n_cells : 0, n);
    if (bytes < w.total) return MD_ERR_WORKSPACE;
    return MD_OK;
}

// workspace for the force and kick calls: only the n-dependent prefix
// (status words and reduction partials) is used
int ws_check_n(int64_t n, void *ws, size_t bytes, WsLayout &w)
{
    if (!ws) return MD_ERR_WORKSPACE;
    w = ws_layout(0, n);
    if (bytes < w.lin2rank) return MD_ERR_WORKSPACE;
    return MD_OK;
}

// descriptor geometry: positive width and spacing, 0 < rc, finite
// normalisation, a known activation form
bool mlp_ok(const md_mlp_t *m)
{
    if (!m || !(m->rc > 0.0) || !(m->width > 0.0) || !(m->dmu > 0.0) || !std::isfinite(m->mu0)) return false;
    if (!std::isfinite(m->rc) || !std::isfinite(m->width) || !std::isfinite(m->dmu)) return false;
    for (int k = 0; k < MD_MLP_IN; ++k)
        if (!std::isfinite(m->mean[k]) || !std::isfinite(m->inv_std[k])) return false;
    return m->activations == MD_MLP_ACT_BF16 || m->activations == MD_MLP_ACT_FP32;
}

uint64_t spread3(uint64_t v)
{
    uint64_t r = 0;
    for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (3 * b);
    return r;
}

}  // namespace

int md::lj_args_check(const md_box_t *box, int64_t n, const double *x, const uint32_t *xs, int32_t row_cap,
                      const int32_t *idx, const int32_t *count, const md_lj_t *lj, const void *f, const double *ev,
                      int32_t flags)
{
    if (!box_ok(box)) return MD_ERR_BOX;
    if (!lj || !(lj->rc > 0.0) || !(lj->sigma > 0.0) || n < 0 || n > kMaxAtoms || row_cap < 1 || row_cap % 8 ||
        row_cap > MD_MAX_ROW_CAP)
        return MD_ERR_ARG;
    if (flags & ~(MD_ENERGY | MD_PAIR_FP64 | MD_NO_COMPENSATE)) return MD_ERR_ARG;
    if (n > 0 && (!idx || !count || !f)) return MD_ERR_ARG;
    if (n > 0 && (flags & MD_PAIR_FP64) && !x) return MD_ERR_ARG;
    if (n > 0 && !(flags & MD_PAIR_FP64) && !xs) return MD_ERR_ARG;
    if (!(flags & MD_PAIR_FP64) && n > kMaxAtomsXs) return MD_ERR_ARG;
    if ((flags & MD_ENERGY) && !ev) return MD_ERR_ARG;
    return MD_OK;
}

extern "C" {

const char *md_error_string(int status)
{
    switch (status) {
    case MD_OK: return "ok";
    case MD_ERR_ARG: return "invalid argument";
    case MD_ERR_BOX: return "box too small for the list cutoff (need 0 < r_list < L/2 on every axis)";
    case MD_ERR_CAPACITY: return "neighbour list exceeds its buffer; reallocate to *needed and retry";
    case MD_ERR_NONFINITE: return "non-finite position detected";
    case MD_ERR_HIP: return "HIP runtime error";
    case MD_ERR_WORKSPACE: return "workspace too small or not initialised";
    default: return "unknown status";
    }
}

int md_grid_init(const md_box_t *box, double r_list, int32_t reach, md_grid_t *grid)
{
    if (!box || !grid || (reach != 1 && reach != 2) || !(r_list > 0.0)) return MD_ERR_ARG;
    if (!box_ok(box)) return MD_ERR_BOX;
    md_grid_t g{};
    g.n_cells = 1;
    for (int a = 0; a < 3; ++a) {
        if (!(r_list < 0.5 * box->L[a])) return MD_ERR_BOX;
        g.L[a] = box->L[a];
        const double nc = std::floor(reach * box->L[a] / r_list);
        if (nc < 1.0 || nc > 1024.0) return MD_ERR_BOX;   // cell coordinates pack into 10 bits
        g.nc[a] = int32_t(nc);
        g.inv_cell[a] = double(g.nc[a]) / box->L[a];
        g.n_cells *= g.nc[a];
    }
    if (g.n_cells > 2147483647) return MD_ERR_BOX;
    g.r_list = r_list;
    g.reach = reach;
    *grid = g;
    return MD_OK;
}

int md_grid_cell_ranks(const md_grid_t *grid, int32_t *rank)
{
    if (!grid_ok(grid) || !rank) return MD_ERR_ARG;
    // walk the Morton codes of the enclosing power-of-two cube in order and
    // number the codes that fall inside the grid
    int32_t p = 1;
    const int32_t mx = std::max(grid->nc[0], std::max(grid->nc[1], grid->nc[2]));
    while (p < mx) p <<= 1;
    const int64_t nc0 = grid->nc[0], nc1 = grid->nc[1];
    if (int64_t(p) * p * p <= 4 * grid->n_cells + 4096) {
        int32_t r = 0;
        const uint64_t ncode = uint64_t(p) * p * p;
        for (uint64_t code = 0; code < ncode; ++code) {
            uint32_t c[3] = {0, 0, 0};
            for (int b = 0; 3 * b < 63 && (code >> (3 * b)); ++b)
                for (int a = 0; a < 3; ++a) c[a] |= uint32_t((code >> (3 * b + a)) & 1u) << b;
            if (int32_t(c[0]) < grid->nc[0] && int32_t(c[1]) < grid->nc[1] && int32_t(c[2]) < grid->nc[2])
                rank[c[0] + nc0 * (c[1] + nc1 * c[2])] = r++;
        }
        return MD_OK;
    }
    // elongated grids: sort the codes of the cells
    std::vector<std::pair<uint64_t, int64_t>> v;
    v.reserve(size_t(grid->n_cells));
    for (int64_t z = 0; z < grid->nc[2]; ++z)
        for (int64_t y = 0; y < nc1; ++y)
            for (int64_t x = 0; x < nc0; ++x)
                v.emplace_back(spread3(x) | (spread3(y) << 1) | (spread3(z) << 2), x + nc0 * (y + nc1 * z));
    std::sort(v.begin(), v.end());
    for (size_t r = 0; r < v.size(); ++r) rank[v[r].second] = int32_t(r);
    return MD_OK;
}

size_t md_workspace_bytes(const md_grid_t *grid, int64_t n)
{
    if (!grid_ok(grid) || n < 0 || n > kMaxAtoms) return 0;
    return ws_layout(grid->n_cells, n).total;
}

// Cell tables of `grid` under the cell order lin2rank (a permutation of the
// cells) into a workspace laid out for n atoms, status words cleared;
// synchronises s.
extern "C++" int md::workspace_upload(const md_grid_t *grid, int64_t n, const int32_t *l2r, void *ws,
                                      size_t ws_bytes, hipStream_t s)
{
    WsLayout w;
    if (int rc = ws_check(grid, n, ws, ws_bytes, w)) return rc;
    const int64_t nc0 = grid->nc[0], nc1 = grid->nc[1];
    std::vector<int32_t> r2l(size_t(grid->n_cells), -1);
    for (int64_t l = 0; l < grid->n_cells; ++l) {
        const int32_t r = l2r[size_t(l)];
        if (r < 0 || r >= grid->n_cells || r2l[size_t(r)] != -1) return MD_ERR_ARG;
        // rank -> packed cell coordinates cx | cy << 10 | cz << 20
        const int32_t cx = int32_t(l % nc0), cy = int32_t((l / nc0) % nc1), cz = int32_t(l / (nc0 * nc1));
        r2l[size_t(r)] = cx | (cy << 10) | (cz << 20);
    }
    int32_t hdr[64] = {};
    hdr[0] = kWsMagic;
    hdr[1] = int32_t(uint32_t(uint64_t(grid->n_cells) & 0xffffffffu));
    hdr[2] = int32_t(uint32_t(uint64_t(grid->n_cells) >> 32));
    MD_HIP_TRY(hipMemcpyAsync(ws_ptr<char>(ws, w.lin2rank), l2r, size_t(grid->n_cells) * 4, hipMemcpyHostToDevice, s));
    MD_HIP_TRY(hipMemcpyAsync(ws_ptr<char>(ws, w.rank2lin), r2l.data(), r2l.size() * 4, hipMemcpyHostToDevice, s));
    MD_HIP_TRY(hipMemcpyAsync(ws_ptr<char>(ws, w.status), hdr, sizeof(hdr), hipMemcpyHostToDevice, s));
    MD_HIP_TRY(hipStreamSynchronize(s));
    return MD_OK;
}

int md_workspace_init(const md_grid_t *grid, int64_t n, void *ws, size_t ws_bytes, void *stream)
{
    if (!grid_ok(grid) || n < 0 || n > kMaxAtoms) return MD_ERR_ARG;
    WsLayout w;
    if (int rc = ws_check(grid, n, ws, ws_bytes, w)) return rc;
    std::vector<int32_t> l2r(size_t(grid->n_cells));
    if (int rc = md_grid_cell_ranks(grid, l2r.data())) return rc;
    return workspace_upload(grid, n, l2r.data(), ws, ws_bytes, as_stream(stream));
}

int md_bin_cells(const md_grid_t *grid, int64_t n, double *x, int32_t *cell, int32_t *perm, int32_t *cell_start,
                 void *ws, size_t ws_bytes, void *stream)
{
    if (!grid_ok(grid) || n < 0 || n > kMaxAtoms || !cell_start) return MD_ERR_ARG;
    if (n > 0 && (!x || !cell || !perm)) return MD_ERR_ARG;
    WsLayout w;
    if (int rc = ws_check(grid, n, ws, ws_bytes, w)) return rc;
    return bin_cells(grid, n, x, cell, perm, cell_start, ws, w, as_stream(stream));
}

int md_permute(int64_t n, int32_t ncomp, const int32_t *perm, const void *src, void *dst, int32_t elem_bytes,
               void *stream)
{
    if (n < 0 || n > kMaxAtoms || ncomp < 1 || ncomp > 16) return MD_ERR_ARG;
    if (elem_bytes != 4 && elem_bytes != 8 && elem_bytes != 16) return MD_ERR_ARG;
    if (n > 0 && (!perm || !src || !dst || src == dst)) return MD_ERR_ARG;
    return permute(n, ncomp, perm, src, dst, elem_bytes, as_stream(stream));
}

int md_scale_positions(const md_box_t *box, int64_t n, const double *x, uint32_t *xs, void *stream)
{
    if (!box_ok(box)) return MD_ERR_BOX;
    if (n < 0 || n > kMaxAtoms || (n > 0 && (!x || !xs))) return MD_ERR_ARG;
    return scale_positions(box, n, x, xs, as_stream(stream));
}

int md_build_neighbors(const md_grid_t *grid, int64_t n, const double *x, const int32_t *cell_start,
                       int32_t row_cap, int32_t *idx, int32_t *count, int32_t *max_count, int32_t *needed, void *ws,
                       size_t ws_bytes, void *stream)
{
    if (!grid_ok(grid) || n < 0 || n > kMaxAtoms || !cell_start || !max_count || row_cap < 1 || row_cap % 8 ||
        row_cap > MD_MAX_ROW_CAP)
        return MD_ERR_ARG;
    if (n > 0 && (!x || !idx || !count)) return MD_ERR_ARG;
    WsLayout w;
    if (int rc = ws_check(grid, n, ws, ws_bytes, w)) return rc;
    return build_neighbors(grid, n, x, cell_start, row_cap, idx, count, max_count, needed, ws, w, as_stream(stream));
}

int md_forces_lj(const md_box_t *box, int64_t n, const double *x, const uint32_t *xs, int32_t row_cap,
                 const int32_t *idx, const int32_t *count, const md_lj_t *lj, void *f, double *ev, int32_t flags,
                 void *ws, size_t ws_bytes, void *stream)
{
    if (int rc = lj_args_check(box, n, x, xs, row_cap, idx, count, lj, f, ev, flags)) return rc;
    WsLayout w;
    if (int rc = ws_check_n(n, ws, ws_bytes, w)) return rc;
    return forces_lj(box, n, x, xs, row_cap, idx, count, lj, f, ev, flags, ws, w, as_stream(stream));
}

int md_forces_eam(const md_box_t *box, int64_t n, uint32_t *xs, int32_t row_cap, const int32_t *idx,
                  const int32_t *count, const md_fs_t *fs, float *rho, float *fprime, float *f, float *e_atom,
                  double *ev, int32_t flags, void *ws, size_t ws_bytes, void *stream)
{
    if (!box_ok(box)) return MD_ERR_BOX;
    if (!fs || !(fs->d > 0.0) || !(fs->c > 0.0) || n < 0 || n > kMaxAtomsXs || row_cap < 1 || row_cap % 8 ||
        row_cap > MD_MAX_ROW_CAP)
        return MD_ERR_ARG;
    if (flags & ~(MD_ENERGY | MD_NO_COMPENSATE)) return MD_ERR_ARG;
    if (n > 0 && (!xs || !idx || !count || !rho || !fprime || !f)) return MD_ERR_ARG;
    if ((flags & MD_ENERGY) && !ev) return MD_ERR_ARG;
    if (e_atom && !(flags & MD_ENERGY)) return MD_ERR_ARG;
    WsLayout w;
    if (int rc = ws_check_n(n, ws, ws_bytes, w)) return rc;
    return forces_eam(box, n, xs, row_cap, idx, count, fs, rho, fprime, f, e_atom, ev, flags, ws, w,
                      as_stream(stream));
}

static bool tb_ok(const md_tb_t *tb)
{
    return tb && tb->A > 0.0 && tb->xi > 0.0 && tb->p > 0.0 && tb->q > 0.0 && tb->r0 > 0.0 && tb->rs > 0.0 &&
           tb->rc > tb->rs && std::isfinite(tb->A) && std::isfinite(tb->xi) && std::isfinite(tb->p) &&
           std::isfinite(tb->q) && std::isfinite(tb->r0) && std::isfinite(tb->rc);
}

int md_forces_tb(const md_box_t *box, int64_t n, uint32_t *xs, int32_t row_cap, const int32_t *idx,
                 const int32_t *count, const md_tb_t *tb, float *rho, float *fprime, float *f, float *e_atom,
                 double *ev, int32_t flags, void *ws, size_t ws_bytes, void *stream)
{
    if (!box_ok(box)) return MD_ERR_BOX;
    if (!tb_ok(tb) || n < 0 || n > kMaxAtomsXs || row_cap < 1 || row_cap % 8 || row_cap > MD_MAX_ROW_CAP)
        return MD_ERR_ARG;
    if (flags & ~(MD_ENERGY | MD_NO_COMPENSATE)) return MD_ERR_ARG;
    if (n > 0 && (!xs || !idx || !count || !rho || !fprime || !f)) return MD_ERR_ARG;
    if ((flags & MD_ENERGY) && !ev) return MD_ERR_ARG;
    if (e_atom && !(flags & MD_ENERGY)) return MD_ERR_ARG;
    WsLayout w;
    if (int rc = ws_check_n(n, ws, ws_bytes, w)) return rc;
    return forces_tb(box, n, xs, row_cap, idx, count, tb, rho, fprime, f, e_atom, ev, flags, ws, w,
                     as_stream(stream));
}

int md_forces_tbm(const md_box_t *box, int64_t n, uint32_t *xs, int32_t row_cap, const int32_t *idx,
                  const int32_t *count, const md_tbm_t *tbm, float *rho, float *fprime, float *f, float *e_atom,
                  double *ev, int32_t flags, void *ws, size_t ws_bytes, void *stream)
{
    if (!box_ok(box)) return MD_ERR_BOX;
    if (!tbm || !tb_ok(&tbm->pair[0]) || !tb_ok(&tbm->pair[1]) || !tb_ok(&tbm->pair[2])) return MD_ERR_ARG;
    if (n < 0 || n > kMaxAtomsXs || row_cap < 1 || row_cap % 8 || row_cap > MD_MAX_ROW_CAP) return MD_ERR_ARG;
    if (flags & ~(MD_ENERGY | MD_NO_COMPENSATE)) return MD_ERR_ARG;
    if (n > 0 && (!xs || !idx || !count || !rho || !fprime || !f)) return MD_ERR_ARG;
    if ((flags & MD_ENERGY) && !ev) return MD_ERR_ARG;
    if (e_atom && !(flags & MD_ENERGY)) return MD_ERR_ARG;
    WsLayout w;
    if (int rc = ws_check_n(n, ws, ws_bytes, w)) return rc;
    return forces_tbm(box, n, xs, row_cap, idx, count, tbm, rho, fprime, f, e_atom, ev, flags, ws, w,
                      as_stream(stream));
}

int md_set_elements(int64_t n, const int32_t *types, uint32_t *xs, void *stream)
{
    if (n < 0 || n > kMaxAtomsXs || (n > 0 && (!types || !xs))) return MD_ERR_ARG;
    return set_elements(n, types, xs, as_stream(stream));
}

int64_t md_tab_bytes(const md_tab_t *tab) { return tab_bytes(tab); }

int md_tab_pack(const md_tab_t *tab, const double *psi, const double *dpsi, const double *phi, const double *dphi,
                const double *F, const double *dF, void *table, void *stream)
{
    if (!tab_ok(tab) || !psi || !dpsi || !phi || !dphi || !F || !dF || !table) return MD_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(table) % 16) return MD_ERR_ARG;
    return tab_pack(tab, psi, dpsi, phi, dphi, F, dF, table, as_stream(stream));
}

int md_forces_tab(const md_box_t *box, int64_t n, uint32_t *xs, int32_t row_cap, const int32_t *idx,
                  const int32_t *count, const md_tab_t *tab, const void *table, float *rho, float *fprime, float *f,
                  float *e_atom, double *ev, int32_t flags, void *ws, size_t ws_bytes, void *stream)
{
    if (!box_ok(box)) return MD_ERR_BOX;
    if (!tab_ok(tab)) return MD_ERR_ARG;
    if (n < 0 || n > kMaxAtomsXs || row_cap < 1 || row_cap % 8 || row_cap > MD_MAX_ROW_CAP) return MD_ERR_ARG;
    if (flags & ~(MD_ENERGY | MD_NO_COMPENSATE)) return MD_ERR_ARG;
    if (n > 0 && (!xs || !idx || !count || !rho || !fprime || !f || !table)) return MD_ERR_ARG;
    if (table && reinterpret_cast<uintptr_t>(table) % 16) return MD_ERR_ARG;
    if ((flags & MD_ENERGY) && !ev) return MD_ERR_ARG;
    if (e_atom && !(flags & MD_ENERGY)) return MD_ERR_ARG;
    WsLayout w;
    if (int rc = ws_check_n(n, ws, ws_bytes, w)) return rc;
    return forces_tab(box, n, xs, row_cap, idx, count, tab, table, rho, fprime, f, e_atom, ev, flags, ws, w,
                      as_stream(stream));
}

int md_mlp_descriptors(const md_box_t *box, int64_t n, const uint32_t *xs, int32_t row_cap, const int32_t *idx,
                       const int32_t *count, const md_mlp_t *mlp, float *G, void *stream)
{
    if (!box_ok(box)) return MD_ERR_BOX;
    if (!mlp_ok(mlp) || n < 0 || n > kMaxAtomsXs || row_cap < 1 || row_cap % 8 || row_cap > MD_MLP_MAX_ROW)
        return MD_ERR_ARG;
    if (n > 0 && (!xs || !idx || !count || !G)) return MD_ERR_ARG;
    return mlp_descriptors(box, n, xs, row_cap, idx, count, mlp, G, as_stream(stream));
}

int md_mlp_eval(int64_t n, const float *G, const md_mlp_t *mlp, const uint16_t *w, float *e_atom, float *dEdG,
                void *stream)
{
    if (!mlp_ok(mlp) || n < 0 || n > kMaxAtoms) return MD_ERR_ARG;
    if (n > 0 && (!G || !w || !e_atom)) return MD_ERR_ARG;
    return mlp_eval(n, G, mlp, w, e_atom, dEdG, as_stream(stream));
}

int md_forces_mlp(const md_box_t *box, int64_t n, const uint32_t *xs, int32_t row_cap, const int32_t *idx,
                  const int32_t *count, const md_mlp_t *mlp, const uint16_t *w, float *dEdG, int32_t *idx_in,
                  int32_t *cnt_in, float *e_atom, float *f, double *ev, int32_t flags, void *ws, size_t ws_bytes,
                  void *stream)
{
    if (!box_ok(box)) return MD_ERR_BOX;
    if (!mlp_ok(mlp) || n < 0 || n > kMaxAtomsXs || row_cap < 1 || row_cap % 8 || row_cap > MD_MAX_ROW_CAP)
        return MD_ERR_ARG;
    if (flags & ~(MD_ENERGY | MD_NO_COMPENSATE | MD_MLP_REUSE)) return MD_ERR_ARG;
    const bool reuse = flags & MD_MLP_REUSE;
    if (!reuse && row_cap > MD_MLP_MAX_ROW) return MD_ERR_ARG;
    if (n > 0 && (!xs || !idx || !count || !dEdG || !f)) return MD_ERR_ARG;
    if (n > 0 && !reuse && (!w || !idx_in || !cnt_in)) return MD_ERR_ARG;
    if ((flags & MD_ENERGY) && !ev) return MD_ERR_ARG;
    WsLayout wl;
    if (int rc = ws_check_n(n, ws, ws_bytes, wl)) return rc;
    return forces_mlp(box, n, xs, row_cap, idx, count, mlp, w, dEdG, idx_in, cnt_in, e_atom, f, ev, flags, ws, wl,
                      as_stream(stream));
}

size_t md_mlp_workspace_bytes(int64_t batch)
{
    if (batch < 0 || batch > kMaxAtoms) return 0;
    return mlp_workspace_bytes(batch);
}

int md_mlp_moments(int64_t n, const float *G, double *moments, void *tws, size_t tws_bytes, void *stream)
{
    if (n < 1 || n > kMaxAtoms || !G || !moments) return MD_ERR_ARG;
    if (!tws || tws_bytes < mlp_workspace_bytes(0)) return MD_ERR_WORKSPACE;
    return mlp_moments(n, G, moments, tws, as_stream(stream));
}

int md_mlp_grad(int64_t batch, const int32_t *sel, const float *G, const float *target, const md_mlp_t *mlp,
                const uint16_t *w, float *grad, double *loss, void *tws, size_t tws_bytes, void *stream)
{
    if (!mlp_ok(mlp) || batch < 1 || batch > kMaxAtoms || !G || !target || !w || !grad) return MD_ERR_ARG;
    if (!tws || tws_bytes < mlp_workspace_bytes(batch)) return MD_ERR_WORKSPACE;
    return mlp_grad_update(batch, sel, G, target, mlp, w, grad, loss, nullptr, nullptr, nullptr, nullptr, nullptr,
                           tws, as_stream(stream));
}

int md_mlp_train_step(int64_t batch, const int32_t *sel, const float *G, const float *target, const md_mlp_t *mlp,
                      const md_adam_t *adam, float *master, float *m1, float *m2, uint16_t *w, double *loss,
                      void *tws, size_t tws_bytes, void *stream)
{
    if (!mlp_ok(mlp) || batch < 1 || batch > kMaxAtoms || !G || !target || !w) return MD_ERR_ARG;
    if (!adam || !master || !m1 || !m2 || adam->step < 1 || !(adam->lr >= 0.0) || !(adam->eps > 0.0) ||
        !(adam->beta1 >= 0.0 && adam->beta1 < 1.0) || !(adam->beta2 >= 0.0 && adam->beta2 < 1.0))
        return MD_ERR_ARG;
    if (!tws || tws_bytes < mlp_workspace_bytes(batch)) return MD_ERR_WORKSPACE;
    return mlp_grad_update(batch, sel, G, target, mlp, w, nullptr, loss, adam, master, m1, m2, w, tws,
                           as_stream(stream));
}

int md_integrate(int32_t phase, const md_box_t *box, int64_t n, double *x, double *v, const void *f, double dt,
                 double accel, double mass, const double *xref, double half_skin_sq, int32_t *status, int32_t tag,
                 uint32_t *xs, double *ke, int32_t flags, void *ws, size_t ws_bytes, void *stream)
{
    if (!box_ok(box)) return MD_ERR_BOX;
    if (n < 0 || n > kMaxAtoms || (flags & ~(MD_PAIR_FP64 | MD_XS_ELEMENT))) return MD_ERR_ARG;
    if ((flags & MD_XS_ELEMENT) && (flags & MD_PAIR_FP64)) return MD_ERR_ARG;
    if (phase != MD_KICK_DRIFT && phase != MD_KICK) return MD_ERR_ARG;
    if (n > 0 && (!v || !f)) return MD_ERR_ARG;
    if (phase == MD_KICK_DRIFT && n > 0 && (!x || !status)) return MD_ERR_ARG;
    WsLayout w{};
    if (phase == MD_KICK) {
        if (int rc = ws_check_n(n, ws, ws_bytes, w)) return rc;
    }
    return integrate(phase, box, n, x, v, f, dt, accel, mass, xref, half_skin_sq, status, tag, xs, ke, flags, ws, w,
                     as_stream(stream));
}

int md_run(md_system_t *sys, int64_t steps, void *stream)
{
    if (!sys || steps < 0 || !box_ok(&sys->box) || !grid_ok(&sys->grid) || sys->n < 0 || sys->n > kMaxAtoms)
        return MD_ERR_ARG;
    if (sys->potential != MD_POT_LJ && sys->potential != MD_POT_EAM && sys->potential != MD_POT_MLP &&
        sys->potential != MD_POT_TB && sys->potential != MD_POT_TBM && sys->potential != MD_POT_TAB)
        return MD_ERR_ARG;
    if (sys->potential == MD_POT_TAB &&
        (!tab_ok(&sys->tab) || !sys->tab_table || reinterpret_cast<uintptr_t>(sys->tab_table) % 16))
        return MD_ERR_ARG;
    if (sys->potential == MD_POT_TB && !tb_ok(&sys->tb)) return MD_ERR_ARG;
    if (sys->potential == MD_POT_TBM &&
        (!tb_ok(&sys->tbm.pair[0]) || !tb_ok(&sys->tbm.pair[1]) || !tb_ok(&sys->tbm.pair[2])))
        return MD_ERR_ARG;
    if (sys->flags & ~(MD_PAIR_FP64 | MD_NO_COMPENSATE)) return MD_ERR_ARG;
    if (sys->potential != MD_POT_LJ && (sys->flags & MD_PAIR_FP64)) return MD_ERR_ARG;
    if (sys->potential == MD_POT_MLP && !mlp_ok(&sys->mlp)) return MD_ERR_ARG;
    if (sys->row_cap < 8 || sys->row_cap % 8 || sys->row_cap > MD_MAX_ROW_CAP || (sys->phase != 0 && sys->phase != 1))
        return MD_ERR_ARG;
    for (int a = 0; a < 3; ++a)
        if (sys->grid.L[a] != sys->box.L[a]) return MD_ERR_ARG;
    const bool f64 = sys->flags & MD_PAIR_FP64;
    if (!f64 && sys->n > kMaxAtomsXs) return MD_ERR_ARG;
    if (sys->n > 0) {
        if (!sys->x || !sys->v || !sys->xref || !sys->scratch || !sys->ids || !sys->ids_scratch || !sys->f ||
            !sys->cell || !sys->perm || !sys->cell_start || !sys->idx || !sys->count || !sys->max_count ||
            !sys->status)
            return MD_ERR_ARG;
        if (!f64 && !sys->xs) return MD_ERR_ARG;
        if ((sys->potential == MD_POT_EAM || sys->potential == MD_POT_TB || sys->potential == MD_POT_TBM ||
             sys->potential == MD_POT_TAB) &&
            (!sys->rho || !sys->fprime))
            return MD_ERR_ARG;
        if (sys->potential == MD_POT_TBM && (!sys->types || !sys->types_scratch)) return MD_ERR_ARG;
        if (sys->potential == MD_POT_MLP && (!sys->mlp_w || !sys->dEdG || !sys->idx_in || !sys->cnt_in))
            return MD_ERR_ARG;
    }
    WsLayout w;
    if (int rc = ws_check(&sys->grid, sys->n, sys->ws, sys->ws_bytes, w)) return rc;
    return run(sys, steps, as_stream(stream));
}

}  // extern "C"
