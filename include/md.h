/*
 * md.h -- C ABI of the MI355X (gfx950) short-range molecular-dynamics hot
 * path after Mangiardi & Meyer, "A hybrid algorithm for parallel molecular
 * dynamics simulations" (arXiv:1611.00075).
 *
 * The path: cell binning with a counting sort into Morton-ordered cells,
 * Verlet neighbour lists over the neighbouring cells within cutoff + skin,
 * Lennard-Jones and embedded-atom (Finnis-Sinclair) forces, velocity-Verlet
 * update with the displacement rebuild rule.
 *
 * Conventions shared by every entry point
 *   - Pointers named x, v, xref, f are device pointers to structure-of-arrays
 *     blocks of 3*n elements: component a of atom i is at [a*n + i].
 *   - The caller owns every buffer, including the workspace `ws`; the library
 *     never allocates or frees device memory.  `ws` must be at least
 *     md_workspace_bytes() long and initialised once with md_workspace_init()
 *     for the grid it is used with.
 *   - Every device call enqueues its kernels on `stream` (a hipStream_t
 *     passed as void*; NULL is the default stream) and returns without
 *     waiting, except where a call says it synchronises.
 *   - Return value: MD_OK (0) or a negative md_status code.  No exception or
 *     abort crosses the ABI.  Argument errors are detected on the host before
 *     anything is enqueued; kernel-detected conditions (non-finite
 *     positions) are reported through the status words of md_integrate.
 *   - Calls that share one workspace must not run concurrently.
 *   - Atom counts are limited to n < 2^31 - 1; list positions are 64-bit.
 */
#ifndef MD_H
#define MD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
typedef enum md_status {
    MD_OK = 0,
    MD_ERR_ARG = -1,        /* null pointer, bad size or flag */
    MD_ERR_BOX = -2,        /* r_list >= L/2 on some axis, or L <= 0 */
    MD_ERR_CAPACITY = -3,   /* neighbour list larger than its buffer */
    MD_ERR_NONFINITE = -4,  /* a kernel saw a non-finite position */
    MD_ERR_HIP = -5,        /* a HIP runtime call failed */
    MD_ERR_WORKSPACE = -6   /* workspace too small or not initialised */
} md_status;

/* Message for a status code (static storage, never NULL). */
const char *md_error_string(int status);

/* ---- flags ---- */
#define MD_ENERGY        0x1  /* forces: also write energy and virial to ev */
#define MD_PAIR_FP64     0x2  /* forces: FP64 pair arithmetic, FP64 forces */
#define MD_NO_COMPENSATE 0x4  /* forces: plain FP32 accumulation (timing aid) */
#define MD_MLP_REUSE     0x8  /* md_forces_mlp: dEdG already holds dE_i/dG_i */
#define MD_XS_ELEMENT    0x10 /* md_integrate: keep bit 0 of xs[4i+3] (the element) */

/* ---- geometry ---- */

/* Orthorhombic box, periodic on every axis (Sec. 3.3).  Open boundaries are
 * not supported. */
typedef struct md_box {
    double L[3];
} md_box_t;

/* Cell grid used for binning and neighbour search (Sec. 2.1: the volume is
 * divided into small cells).  Cells have edge >= r_list / reach, so every
 * pair closer than r_list lies within `reach` cells along each axis. */
typedef struct md_grid {
    double L[3];
    double r_list;
    double inv_cell[3];   /* nc[a] / L[a], computed on the host */
    int32_t nc[3];        /* cells per axis: floor(reach * L / r_list) */
    int32_t reach;        /* stencil half-width in cells (1 or 2) */
    int64_t n_cells;
} md_grid_t;

/* Host only.  Fills *grid for a box and list cutoff r_list.  reach = 1 gives
 * cells of edge >= r_list and the 27-cell stencil; reach = 2 gives cells of
 * edge >= r_list/2 and the 125-cell stencil.  Stencil offsets that coincide
 * modulo nc are visited once.  Returns MD_ERR_BOX unless
 * 0 < r_list < L[a]/2 and nc[a] <= 1024 on every axis. */
int md_grid_init(const md_box_t *box, double r_list, int32_t reach,
                 md_grid_t *grid);

/* Host only.  Dense Morton rank of every cell: rank[cx + nc0*(cy + nc1*cz)]
 * is the position of the cell when all cells are sorted by the Morton
 * (bit-interleaved) code of (cx, cy, cz).  `rank` holds n_cells entries. */
int md_grid_cell_ranks(const md_grid_t *grid, int32_t *rank);

/* ---- workspace ---- */

/* Host only.  Bytes of workspace needed for up to n atoms on `grid`. */
size_t md_workspace_bytes(const md_grid_t *grid, int64_t n);

/* Uploads the Morton tables of `grid` into ws and clears the status words.
 * Synchronises `stream` once (a host-to-device copy). */
int md_workspace_init(const md_grid_t *grid, int64_t n, void *ws,
                      size_t ws_bytes, void *stream);

/* ---- step a1/a2: binning ---- */

/* Wraps x in place into [0, L) (w = x - L floor(x/L), one correction each
 * way, FP64), assigns each atom its cell c = (int)(w * inv_cell) clamped to
 * nc-1, and sorts the atoms by the Morton rank of their cell with a stable
 * counting sort.
 * Outputs (device, caller-owned):
 *   cell[n]                Morton rank of each atom's cell, in input order;
 *   perm[n]                perm[k] = input index of the k-th sorted atom;
 *                          atoms of one cell keep their input order;
 *   cell_start[n_cells+1]  sorted atoms of the cell of rank r are
 *                          [cell_start[r], cell_start[r+1]).
 * Reorder per-atom arrays with md_permute afterwards. */
int md_bin_cells(const md_grid_t *grid, int64_t n, double *x, int32_t *cell,
                 int32_t *perm, int32_t *cell_start, void *ws, size_t ws_bytes,
                 void *stream);

/* dst[c*n + k] = src[c*n + perm[k]] for c < ncomp, k < n; elements of
 * elem_bytes = 4, 8 or 16 bytes.  src and dst must not overlap. */
int md_permute(int64_t n, int32_t ncomp, const int32_t *perm, const void *src,
               void *dst, int32_t elem_bytes, void *stream);

/* Scaled coordinates for the FP32 force kernels (the fractional position of
 * Sec. 4.1, "fetch" and "dist"): xs[4i+a] = round(x[a*n+i] * 2^32 / L[a])
 * modulo 2^32, so that the 32-bit difference of two atoms is their periodic
 * minimum-image displacement in units of L[a]/2^32.  xs[4i+3] is set to 0;
 * md_forces_eam stores F'(rho_i) there between its passes. */
int md_scale_positions(const md_box_t *box, int64_t n, const double *x,
                       uint32_t *xs, void *stream);

/* ---- step a3: neighbour lists ---- */

/* List layout (sliced ELL).  Atoms are grouped in slices of 8 consecutive
 * (sorted) atoms; row i has capacity row_cap (a multiple of 8) and its
 * entry e < count[i] <= row_cap is stored at
 *     idx[(i/8 * row_cap/8 + e/8) * 64 + (i%8) * 8 + e%8],
 * i.e. the rows of a slice are interleaved in blocks of 8 entries, so idx
 * holds ceil(n / 8) * 8 * row_cap int32 (sorted atom indices).  row_cap is
 * at most MD_MAX_ROW_CAP. */
#define MD_SLICE 8
#define MD_MAX_ROW_CAP (1 << 24)

/* Largest n the FP32 pair paths (md_forces_lj without MD_PAIR_FP64,
 * md_forces_eam, the MLP entry points, md_run without MD_PAIR_FP64) accept:
 * they read the scaled coordinates through one 32-bit byte range. */
#define MD_MAX_ATOMS_FP32 ((1 << 28) - 1)

/* Full Verlet lists (Sec. 3.3): row i holds every j != i with
 * r_ij^2 < r_list^2, r_ij^2 = (dx*dx + dy*dy) + dz*dz of the minimum-image
 * displacement dx = x_j - x_i (shifted by L when |dx| > L/2), in FP64 with
 * no contraction.  j in N(i) iff i in N(j).  Positions must be the wrapped,
 * sorted output of md_bin_cells + md_permute, cell_start its output.
 * Outputs: count[n], the rows in idx (order within a row unspecified but
 * deterministic), and *max_count (device int32) = the longest row.  Rows
 * longer than row_cap are truncated; the list is then invalid.  If `needed`
 * (host) is not NULL the call synchronises `stream` once, stores the longest
 * row there and returns MD_ERR_CAPACITY when it exceeds row_cap (the caller
 * grows idx and repeats the call); with needed == NULL it does not wait and
 * the caller must check *max_count before using the list. */
int md_build_neighbors(const md_grid_t *grid, int64_t n, const double *x,
                       const int32_t *cell_start, int32_t row_cap,
                       int32_t *idx, int32_t *count, int32_t *max_count,
                       int32_t *needed, void *ws, size_t ws_bytes,
                       void *stream);

/* ---- step a4: Lennard-Jones ---- */

typedef struct md_lj {
    double eps, sigma, rc;
} md_lj_t;

/* Lennard-Jones forces from a full list (the pair loop of Sec. 2.2, with
 * every pair visited from both sides so that no force is scattered):
 *   F_i = sum_{j in N(i), r < rc} 24 eps s6 (2 s6 - 1) / r^2 (r_i - r_j),
 *   s6 = (sigma/r)^6, truncated at rc.
 * The list (row_cap, idx, count) is the output of md_build_neighbors.
 * Default: displacements from the scaled coordinates xs, pair arithmetic in
 * FP32, per-lane sums compensated (Kahan) in FP32 and combined across lanes
 * in FP64; f is float[3n].  With MD_PAIR_FP64: displacements from x in
 * FP64 (minimum image as in md_build_neighbors), all arithmetic FP64, f is
 * double[3n]; xs may be NULL.  f is overwritten.
 * With MD_ENERGY, ev[8] (device) receives E = 1/2 sum 4 eps (s12 - s6),
 * E_shift (each pair shifted by -Phi(rc)) and the virial
 * W_ab = 1/2 sum_i sum_j f_s R_a R_b in the order xx, yy, zz, xy, xz, yz,
 * reduced in FP64 in a fixed order. */
int md_forces_lj(const md_box_t *box, int64_t n, const double *x,
                 const uint32_t *xs, int32_t row_cap, const int32_t *idx,
                 const int32_t *count, const md_lj_t *lj, void *f, double *ev,
                 int32_t flags, void *ws, size_t ws_bytes, void *stream);

/* ---- allocation-free variant ----
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * kernels, arguments, outputs and errors as md_forces_lj, without the
 * workspace: the per-block energy and virial partials (MD_ENERGY) live in a
 * device array of the library, MD_NOALLOC_MAX_ATOMS / 32 rows of 8 doubles
 * (8 MiB), one copy per GPU held until the process ends.  With MD_ENERGY,
 * n > MD_NOALLOC_MAX_ATOMS is rejected with MD_ERR_ARG; without it any n
 * md_forces_lj takes is accepted (the array is then not touched).  The call
 * allocates and frees nothing; its first call on a device looks up that
 * device's copy of the array.  `stream` must belong to the current device.
 * All calls on one GPU share its array: calls with MD_ENERGY whose
 * execution overlaps on that GPU (different streams, threads) race on it
 * and must be serialised by the caller.  Nothing in the array needs to start
 * at zero: each call writes every row it reads. */
#define MD_NOALLOC_MAX_ATOMS (1 << 22)

int md_forces_lj_noalloc(const md_box_t *box, int64_t n, const double *x,
                         const uint32_t *xs, int32_t row_cap,
                         const int32_t *idx, const int32_t *count,
                         const md_lj_t *lj, void *f, double *ev,
                         int32_t flags, void *stream);

/* ---- steps a5/a6: embedded-atom method ---- */

/* Finnis-Sinclair form of Eqs. (1)-(2): psi(r) = (r-d)^2 for r < d,
 * F(rho) = -A sqrt(rho) (F = F' = 0 at rho = 0), V(r) = (r-c)^2
 * (c0 + c1 r + c2 r^2) for r < c. */
typedef struct md_fs {
    double A, d, c, c0, c1, c2;
} md_fs_t;

/* The three steps of Sec. 3.1: (1) rho_i = sum_j psi(r_ij) over the full
 * list; (2) F_i, F'_i per atom (fused into the first kernel's epilogue);
 * (3) F_i = -sum_j [(F'_i + F'_j) psi'(r) + V'(r)] (r_i - r_j)/r.
 * FP32 pair arithmetic from the scaled coordinates xs (written by
 * md_scale_positions; xs[4i+3] is overwritten with F'_i), compensated FP32
 * sums.  Outputs: rho[n], fprime[n] (float), f float[3n] (overwritten); with
 * MD_ENERGY, ev[8] = E_total, E_embed, W_xx, W_yy, W_zz, W_xy, W_xz, W_yz,
 * and, if e_atom is not NULL, the site energies
 * e_atom[i] = F(rho_i) + 1/2 sum_j V(r_ij) (float; needs MD_ENERGY). */
int md_forces_eam(const md_box_t *box, int64_t n, uint32_t *xs,
                  int32_t row_cap, const int32_t *idx, const int32_t *count,
                  const md_fs_t *fs, float *rho, float *fprime, float *f,
                  float *e_atom, double *ev, int32_t flags, void *ws,
                  size_t ws_bytes, void *stream);

/* Second-moment tight-binding potential in the form of Eqs. (1)-(2) with
 * the exponential density and pair functions and square-root embedding
 * that Sec. 3.1 names for its copper potential:
 *   psi(r) = xi^2 exp(-2q (r/r0 - 1)) S(r),  Phi(r) = 2A exp(-p (r/r0 - 1)) S(r),
 *   F(rho) = -sqrt(rho)  (F = F' = 0 at rho = 0),
 * S = 1 for r <= rs, 0 for r >= rc, 1 - x^3 (10 - 15 x + 6 x^2) with
 * x = (r - rs)/(rc - rs) in between (0 < rs < rc).  Energies in the unit of
 * A and xi, lengths in the unit of r0. */
typedef struct md_tb {
    double A, xi, p, q, r0, rs, rc;
} md_tb_t;

/* The same three steps, kernels and outputs as md_forces_eam, with psi,
 * Phi and F of md_tb_t (Phi in place of V; e_atom[i] = F(rho_i) +
 * 1/2 sum_j Phi(r_ij)).  The list must reach rc. */
int md_forces_tb(const md_box_t *box, int64_t n, uint32_t *xs,
                 int32_t row_cap, const int32_t *idx, const int32_t *count,
                 const md_tb_t *tb, float *rho, float *fprime, float *f,
                 float *e_atom, double *ev, int32_t flags, void *ws,
                 size_t ws_bytes, void *stream);

/* Two elements (the Cu-Au systems of Sec. 3.1): the same form with the
 * parameters of each pair's kind, pair[t_i + t_j] (0: 0-0, 1: 0-1, 2: 1-1),
 * F(rho) = -sqrt(rho) for both.  The element t_i (0 or 1) of atom i travels
 * as bit 0 of xs[4i+3]: on entry that word must hold the element
 * (md_set_elements; md_integrate with MD_XS_ELEMENT keeps it); on return it
 * holds F'_i with its lowest mantissa bit replaced by the element.
 * Otherwise as md_forces_tb. */
typedef struct md_tbm {
    md_tb_t pair[3];
} md_tbm_t;

int md_forces_tbm(const md_box_t *box, int64_t n, uint32_t *xs,
                  int32_t row_cap, const int32_t *idx, const int32_t *count,
                  const md_tbm_t *tbm, float *rho, float *fprime, float *f,
                  float *e_atom, double *ev, int32_t flags, void *ws,
                  size_t ws_bytes, void *stream);

/* xs[4i+3] = types[i] & 1 for i < n (the element word md_forces_tbm reads;
 * xs from md_scale_positions). */
int md_set_elements(int64_t n, const int32_t *types, uint32_t *xs,
                    void *stream);

/* ---- tabulated embedded-atom functions ----
 *
 * Sec. 3.1 names piecewise-defined psi and Phi for its iron potential, and
 * Sec. 5 takes an interpolation table to be such a piecewise definition.
 * One element, the form of Eqs. (1)-(2) with psi, Phi and F given as
 * tables:
 *   psi, Phi at r_k = k dr (k = 0 .. nr-1) by value and slope,
 *   F at rho_k = k drho (k = 0 .. nrho-1) by value and slope;
 * between two knots a function is the cubic Hermite interpolant of the
 * values and slopes at the two knots; psi = Phi = 0 for r >= rc =
 * (nr-1) dr; below rho = 0 and above rho_{nrho-1}, F continues along the
 * tangent at that end knot. */
#define MD_TAB_MAX_KNOTS 2001   /* knots of psi and Phi (rc / dr <= 2000) */
#define MD_TAB_MAX_RHO_KNOTS (1 << 24)

typedef struct md_tab {
    int32_t nr;      /* knots of psi and Phi, 2 .. MD_TAB_MAX_KNOTS */
    int32_t nrho;    /* knots of F, 2 .. MD_TAB_MAX_RHO_KNOTS */
    double dr;       /* knot spacing in r (> 0) */
    double drho;     /* knot spacing in rho (> 0) */
} md_tab_t;

/* Bytes of the device table of `tab`: 32 (nr-1) + 16 (nrho-1); 0 for an
 * invalid tab. */
int64_t md_tab_bytes(const md_tab_t *tab);

/* Fills the device table (caller-owned, md_tab_bytes bytes, 16-byte
 * aligned) from host FP64 arrays: psi, dpsi, phi, dphi [nr] (values and
 * slopes at r_k), F, dF [nrho] (at rho_k).  The table holds per interval
 * the FP32 coefficients of the interpolant in powers of the position in
 * the interval (psi intervals, then Phi intervals, then F intervals).  The
 * copy is enqueued on `stream` and waited for before returning.
 * MD_ERR_ARG for a bad tab, a null pointer or a non-finite value. */
int md_tab_pack(const md_tab_t *tab, const double *psi, const double *dpsi,
                const double *phi, const double *dphi, const double *F,
                const double *dF, void *table, void *stream);

/* The three steps of Sec. 3.1 with tabulated psi, Phi and F (table from
 * md_tab_pack for the same tab).  Same outputs as md_forces_eam, with Phi
 * in place of V (e_atom[i] = F(rho_i) + 1/2 sum_j Phi(r_ij)).  The list
 * must reach rc = (nr-1) dr. */
int md_forces_tab(const md_box_t *box, int64_t n, uint32_t *xs,
                  int32_t row_cap, const int32_t *idx, const int32_t *count,
                  const md_tab_t *tab, const void *table, float *rho,
                  float *fprime, float *f, float *e_atom, double *ev,
                  int32_t flags, void *ws, size_t ws_bytes, void *stream);

/* ---- steps a8/a9: learned descriptor-MLP potential ----
 *
 * A learned stand-in for the embedded-atom energy of Eqs. (1)-(2): like
 * F(rho_i) + 1/2 sum_j V(r_ij), the energy of atom i is a function of the
 * distances to its neighbours only.
 *   pair basis  g_k(r) = exp(-(r - mu_k)^2 / (2 w^2)) fc(r) for r < rc,
 *               fc(r) = (cos(pi r / rc) + 1) / 2, mu_k = mu0 + k dmu, k < 16;
 *   descriptor  G_ik = sum_{j in N(i), r_ij < rc} g_k(r_ij);
 *   network     x = (G_i - mean) * inv_std, h1 = silu(W1 x + b1),
 *               h2 = silu(W2 h1 + b2), E_i = w3 . h2 + b3 (16 -> 64 -> 64
 *               -> 1, silu(a) = a / (1 + exp(-a)));
 *   forces      F_i = -dE/dx_i, E = sum_i E_i.
 * Parameters: MD_MLP_NPARAM bfloat16 values (uint16 bit patterns), row-major
 * matrices with the output index first: W1[64][16], b1[64], W2[64][64],
 * b2[64], w3[64], b3.  The matrix products run on the BF16 matrix cores with
 * FP32 accumulation: every vector entering a product (x, h1, and the
 * back-propagated vectors dE/da2, dE/da1) is rounded to bfloat16 (round to
 * nearest even); pre-activations, SiLU and its derivative, biases, the last
 * layer and all sums over neighbours are FP32. */
#define MD_MLP_IN     16
#define MD_MLP_HID    64
#define MD_MLP_NPARAM 5313

/* Activation form of the network's matrix products (md_mlp_t.activations):
 *   MD_MLP_ACT_BF16  every vector entering a product is rounded to bfloat16
 *                    (the form above; the default);
 *   MD_MLP_ACT_FP32  every such vector is split exactly into three bfloat16
 *                    terms (hi + mid + lo, together the FP32 significand) and
 *                    the products of the three are summed on the matrix
 *                    cores in FP32: the network with FP32 activations and
 *                    the same bfloat16 parameters (three times the matrix
 *                    work).  Training (md_mlp_grad, md_mlp_train_step) always
 *                    uses the BF16 form. */
#define MD_MLP_ACT_BF16 0
#define MD_MLP_ACT_FP32 1

typedef struct md_mlp {
    double rc;                  /* descriptor cutoff */
    double mu0, dmu;            /* Gaussian centres mu_k = mu0 + k dmu */
    double width;               /* Gaussian width w */
    float mean[MD_MLP_IN];      /* input normalisation */
    float inv_std[MD_MLP_IN];
    int32_t activations;        /* MD_MLP_ACT_BF16 or MD_MLP_ACT_FP32 */
    int32_t reserved;           /* 0 */
} md_mlp_t;

/* Longest list row (row_cap) the descriptor passes accept: the in-range
 * distances of a row are staged in LDS. */
#define MD_MLP_MAX_ROW 256

/* Raw descriptors G[n][16] (float, row i contiguous) from a full list at
 * any list cutoff >= rc (the output of md_build_neighbors, row_cap <=
 * MD_MLP_MAX_ROW) and the scaled coordinates xs of md_scale_positions.
 * FP32; the 16 Gaussians of a pair are formed from three exponentials by
 * their ratio recurrence (exact up to rounding for r > 1 A with the default
 * centres and width). */
int md_mlp_descriptors(const md_box_t *box, int64_t n, const uint32_t *xs,
                       int32_t row_cap, const int32_t *idx,
                       const int32_t *count, const md_mlp_t *mlp, float *G,
                       void *stream);

/* The network alone on given raw descriptors G[n][16]: per-atom energies
 * e_atom[n] and, if dEdG is not NULL, dE_i/dG_i [n][16] (float). */
int md_mlp_eval(int64_t n, const float *G, const md_mlp_t *mlp,
                const uint16_t *w, float *e_atom, float *dEdG, void *stream);

/* Forces of the learned potential in two passes (the same two-pass shape
 * as md_forces_eam):
 *   pass 1: over the full list (row_cap <= MD_MLP_MAX_ROW): G_i, the network
 *           and its backward pass to dE_i/dG_i, stored in dEdG[n][16]
 *           (caller-owned float scratch); the pairs within rc are written as
 *           a compact list in the same sliced-ELL layout, idx_in (as large
 *           as idx) and cnt_in[n] (caller-owned int32 scratch);
 *   pass 2: over the compact list, F_i = -sum_{j, r_ij < rc} s_ij
 *           (r_i - r_j) / r_ij with s_ij = sum_k (dE_i/dG_ik + dE_j/dG_jk)
 *           g_k'(r_ij).
 * f is float[3n], overwritten; compensated FP32 sums.  e_atom (may be NULL)
 * receives E_i.  With MD_ENERGY, ev[8] = E, E, W_xx, W_yy, W_zz, W_xy, W_xz,
 * W_yz (W_ab = -1/2 sum_i sum_j s_ij R_a R_b / r_ij), FP64 in fixed order.
 * With MD_MLP_REUSE, pass 1 is skipped, dEdG is taken as given (the stored
 * result of an earlier call on the same positions, or the caller's own) and
 * pass 2 walks (row_cap, idx, count) as passed: the full list, or the
 * compact list idx_in/cnt_in of an earlier call on the same positions; w,
 * idx_in, cnt_in and e_atom are then unused (may be NULL), any row_cap is
 * accepted, and E in ev is 0.
 * ws as for md_forces_lj. */
int md_forces_mlp(const md_box_t *box, int64_t n, const uint32_t *xs,
                  int32_t row_cap, const int32_t *idx, const int32_t *count,
                  const md_mlp_t *mlp, const uint16_t *w, float *dEdG,
                  int32_t *idx_in, int32_t *cnt_in, float *e_atom, float *f,
                  double *ev, int32_t flags, void *ws, size_t ws_bytes,
                  void *stream);

/* Host only.  Bytes of training workspace for batches of up to `batch`
 * atoms (md_mlp_moments, md_mlp_grad, md_mlp_train_step). */
size_t md_mlp_workspace_bytes(int64_t batch);

/* Per-component mean and standard deviation (population) of G[n][16]:
 * moments[0..15] = mean, moments[16..31] = std (device double[32]), FP64
 * sums in a fixed order. */
int md_mlp_moments(int64_t n, const float *G, double *moments, void *tws,
                   size_t tws_bytes, void *stream);

/* Per-atom energy loss of a batch, L = (1/B) sum_b (E(G[sel[b]]) -
 * target[sel[b]])^2 (sel may be NULL: rows 0..B-1; its entries must index
 * rows of G and target, which the library cannot check), and its gradient with
 * respect to the parameters (float[MD_MLP_NPARAM], the layout of w) by back
 * propagation: BF16 matrix-core products for dL/dW1, dL/dW2 and the
 * backward pass, FP32 sums for the biases and w3, per-block partials summed
 * in FP64 in a fixed order.  *loss (device double, may be NULL) = L. */
int md_mlp_grad(int64_t batch, const int32_t *sel, const float *G,
                const float *target, const md_mlp_t *mlp, const uint16_t *w,
                float *grad, double *loss, void *tws, size_t tws_bytes,
                void *stream);

/* Adam (Kingma & Ba) on FP32 master weights. */
typedef struct md_adam {
    double lr, beta1, beta2, eps;
    int64_t step;               /* 1 for the first update */
} md_adam_t;

/* One optimiser step: the gradient of md_mlp_grad, then per parameter
 * m1 = b1 m1 + (1-b1) g, m2 = b2 m2 + (1-b2) g^2,
 * master -= lr (m1 / (1-b1^step)) / (sqrt(m2 / (1-b2^step)) + eps)   (FP32)
 * and w = bfloat16(master) (round to nearest even).  master, m1, m2 are
 * float[MD_MLP_NPARAM]; w is both the network used for the gradient and the
 * refreshed copy.  *loss (may be NULL) = the batch loss before the step. */
int md_mlp_train_step(int64_t batch, const int32_t *sel, const float *G,
                      const float *target, const md_mlp_t *mlp,
                      const md_adam_t *adam, float *master, float *m1,
                      float *m2, uint16_t *w, double *loss, void *tws,
                      size_t tws_bytes, void *stream);

/* ---- domain decomposition on one device ----
 *
 * Sec. 2.1's spatial decomposition with the asynchronous force step of its
 * hybrid algorithm (pack the boundary coordinates, send, receive, forces
 * inside the domain while the messages travel, wait, forces across the
 * domain boundary), for the LJ and FS forms.  The periodic box is cut into
 * p[0] x p[1] x p[2] equal bricks, all on this device (each the share one
 * device of a multi-device run would hold).  Each brick holds its own
 * atoms and ghost copies of the atoms of the neighbouring bricks (periodic
 * images included) within one halo layer of width c >= r_list of its
 * faces.  A brick is computed in its own frame, a periodic box of k+3
 * cells of edge c per axis (c = brick edge / k): cells 1..k cover the
 * brick, cells 0 and k+1 the halo, cell k+2 is an empty gap so that no pair
 * forms across the frame's periodic boundary.  Cells are ranked inner cells
 * first (at least one cell inside the brick faces), then the brick's face
 * layer (outer cells), then ghost cells, so a brick's sorted atoms are its
 * inner atoms (no ghost within r_list at a build), its outer atoms, and
 * its ghosts.
 *
 * State after md_dd_rebuild: the atoms in x, v, ids are grouped by brick
 * (brick t holds [brick_start[t], brick_start[t+1]), in its sorted order);
 * brick t's atoms and ghosts own the slots [slot0[t], slot0[t] + n_t + g_t)
 * of xs, count, and of the sliced-ELL list (at idx + slot0[t] * row_cap);
 * ghost entry k (k < n_ghost, grouped by brick) is a copy of atom
 * gh_src[k] in slot gh_slot[k]. */
#define MD_DD_MAX_BRICKS 64

typedef struct md_dd {
    /* geometry: md_dd_init */
    md_box_t box;                /* the periodic box */
    int32_t p[3];                /* bricks per axis, >= 1 */
    int32_t n_bricks;
    int32_t k[3];                /* cells per brick edge, >= 3 */
    double c[3];                 /* cell edge (halo width), >= r_list */
    md_box_t vbox;               /* a brick's frame: (k + 3) c per axis */
    md_grid_t vgrid;             /* its cells */
    int64_t inner_cells;         /* cells ranked first */
    /* set by the caller */
    int32_t potential;           /* MD_POT_LJ or MD_POT_EAM */
    int32_t flags;               /* MD_NO_COMPENSATE */
    md_lj_t lj;
    md_fs_t fs;
    int64_t n;                   /* atoms */
    double *x, *v, *xref;        /* device [3][n] */
    int32_t *ids;                /* device [n] */
    double *x2, *v2;             /* device [3][n] scratch */
    int32_t *ids2;               /* device [n] scratch */
    float *f;                    /* device [3][n] */
    float *rho, *fprime;         /* device [n] (MD_POT_EAM) */
    int32_t row_cap;             /* list row capacity (multiple of 8) */
    int64_t slot_cap;            /* capacity of xs, count (slots) */
    uint32_t *xs;                /* device [slot_cap][4] */
    int32_t *count;              /* device [slot_cap] */
    int32_t *idx;                /* device [slot_cap * row_cap] */
    int64_t ghost_cap;           /* capacity of the ghost entry arrays */
    int32_t *gh_src, *gh_slot, *gh_code, *gh_src_slot;   /* device [ghost_cap] */
    double *send, *recv;         /* device [3 * ghost_cap] */
    uint32_t *send_w, *recv_w;   /* device [ghost_cap] */
    void *vws;                   /* workspace of vgrid for slot_cap atoms (md_dd_workspace_init) */
    size_t vws_bytes;
    void *dws;                   /* scratch of md_dd_scratch_bytes */
    size_t dws_bytes;
    int32_t *status;             /* device int32[2], zero-initialised */
    /* set by md_dd_rebuild */
    int64_t n_ghost;
    int64_t brick_start[MD_DD_MAX_BRICKS + 1];
    int64_t slot0[MD_DD_MAX_BRICKS + 1];
    int64_t ghost_start[MD_DD_MAX_BRICKS + 1];
    int64_t n_inner[MD_DD_MAX_BRICKS];   /* atoms in inner cells per brick */
    int64_t ghost_needed, slot_needed;   /* out: set with MD_ERR_CAPACITY */
    int32_t row_cap_needed;
    int32_t phase;               /* md_dd_run: 0 at a step boundary; 1 forces and
                                    the closing kick pending; 2 a build first */
    int64_t builds, steps;
    void *events[4];             /* created on first use, md_dd_release */
} md_dd_t;

/* Host only.  Fills the geometry of *dd (box, p, n_bricks, k, c, vbox,
 * vgrid, inner_cells) for lists of cutoff r_list: k[a] =
 * floor(brick edge / (r_list (1 + 1e-6))), which must be >= 3.
 * MD_ERR_BOX otherwise or for more than MD_DD_MAX_BRICKS bricks. */
int md_dd_init(md_dd_t *dd, const md_box_t *box, const int32_t p[3],
               double r_list);

/* Host only.  Bytes of dws for dd->n, dd->ghost_cap, dd->slot_cap. */
size_t md_dd_scratch_bytes(const md_dd_t *dd);

/* Uploads the cell ranks of dd->vgrid (inner, outer, ghost classes, Morton
 * order inside each) into dd->vws (md_workspace_bytes(&dd->vgrid,
 * dd->slot_cap) bytes) and the frame offsets into dd->dws.  Synchronises
 * `stream`. */
int md_dd_workspace_init(md_dd_t *dd, void *stream);

/* Wraps the positions, regroups the atoms by brick (stable), selects the
 * ghosts of every brick, sorts each brick's atoms and ghosts by cell and
 * builds its lists, orders each brick's atoms as sorted, and sets
 * xref = x.  Synchronises `stream` (it reads sizes back).
 * MD_ERR_CAPACITY with ghost_needed, slot_needed or row_cap_needed set when
 * a buffer is too small (grow it and call again). */
int md_dd_rebuild(md_dd_t *dd, void *stream);

/* Forces of the current positions in the asynchronous order: local
 * coordinates scaled into the brick frames, ghost coordinates packed,
 * copied and unpacked on `comm` while the inner atoms' forces run on
 * `stream`, then the outer atoms' (FS: both passes so split, with the F'
 * of ghosts exchanged on `comm` between them).  f, rho, fprime are indexed
 * like x.  With MD_ENERGY in flags, ev[8] as md_forces_lj / md_forces_eam
 * over all atoms.  `comm` may equal `stream`. */
int md_dd_forces(md_dd_t *dd, double *ev, int32_t flags, void *stream,
                 void *comm);

/* `steps` velocity-Verlet steps (dt, accel as md_integrate) with the
 * displacement rebuild rule (skin/2) checked after every drift (the flag
 * is read back each step), md_dd_rebuild when it fires, md_dd_forces.
 * A build that reports MD_ERR_CAPACITY returns at once with phase = 2:
 * grow the buffers and call again; the pending step is completed first. */
int md_dd_run(md_dd_t *dd, int64_t steps, double dt, double accel,
              double skin, void *stream, void *comm);

/* Destroys the events md_dd_forces created; MD_ERR_HIP if the runtime
 * reports a failure (every event handle is cleared either way). */
int md_dd_release(md_dd_t *dd);

/* ---- step a7: velocity Verlet ---- */

#define MD_KICK_DRIFT 1   /* v += dt/2 a f; x += dt v; rebuild check */
#define MD_KICK       2   /* v += dt/2 a f; optional kinetic energy */

/* One half of a velocity-Verlet step (Sec. 3.3), a = accel per unit force
 * (force_to_accel / mass), FP64 state.
 * f is float[3n], or double[3n] when flags has MD_PAIR_FP64.
 * MD_KICK_DRIFT: x is not re-wrapped.  If xref is not NULL, status[0] is set
 *   to `tag` when some atom has |minimg(x - xref)|^2 > half_skin_sq (the
 *   rebuild rule: moved more than half the skin since the last build);
 *   status[1] gets bit 0 set when a new position is not finite.  status is
 *   never cleared by the library.  If xs is not NULL, the scaled
 *   coordinates are rewritten from the new positions (xs[4i+3] set to 0,
 *   or to its own bit 0 with MD_XS_ELEMENT in flags).
 * MD_KICK: if ke is not NULL, *ke (device) = 1/2 mass sum |v|^2 over the
 *   updated velocities, reduced in FP64 in a fixed order. */
int md_integrate(int32_t phase, const md_box_t *box, int64_t n, double *x,
                 double *v, const void *f, double dt, double accel,
                 double mass, const double *xref, double half_skin_sq,
                 int32_t *status, int32_t tag, uint32_t *xs, double *ke,
                 int32_t flags, void *ws, size_t ws_bytes, void *stream);

/* ---- native step driver ---- */

#define MD_POT_LJ  0
#define MD_POT_EAM 1
#define MD_POT_MLP 2
#define MD_POT_TB  3
#define MD_POT_TBM 4
#define MD_POT_TAB 5

/* One system for md_run.  The caller fills every field (device buffers are
 * caller-owned; sizes as for the calls above) and keeps the struct between
 * calls: md_run updates step, builds, phase, need_build, row_cap_needed. */
typedef struct md_system {
    md_box_t box;
    md_grid_t grid;
    md_lj_t lj;                 /* MD_POT_LJ */
    md_fs_t fs;                 /* MD_POT_EAM */
    double dt;
    double accel;               /* force_to_accel / mass */
    double half_skin_sq;        /* (skin / 2)^2 */
    int64_t n;
    int64_t step;               /* completed steps; step + 1 tags the rebuild check */
    int64_t builds;             /* list builds so far */
    double *x, *v, *xref;       /* [3n] FP64 */
    double *scratch;            /* [3n] permutation scratch */
    int32_t *ids, *ids_scratch; /* [n]: input index of each sorted atom */
    uint32_t *xs;               /* [4n] scaled coordinates (FP32 path) */
    void *f;                    /* float[3n], double[3n] with MD_PAIR_FP64 */
    float *rho, *fprime;        /* [n], MD_POT_EAM */
    int32_t *cell, *perm, *cell_start;
    int32_t *idx, *count, *max_count;   /* sliced-ELL list, row_cap */
    int32_t *status;            /* device int32[2], zero-initialised */
    int32_t *host_status;       /* pinned host int32[4] (hipHostMalloc), or NULL */
    void *ws;
    size_t ws_bytes;
    int32_t row_cap;
    int32_t row_cap_needed;     /* out: set with MD_ERR_CAPACITY */
    int32_t potential;          /* MD_POT_LJ, MD_POT_EAM, MD_POT_MLP, MD_POT_TB, MD_POT_TBM or MD_POT_TAB */
    int32_t flags;              /* MD_PAIR_FP64 (LJ only), MD_NO_COMPENSATE */
    int32_t need_build;         /* 1: build lists (and forces) before stepping */
    int32_t phase;              /* 0: at a step boundary; 1: a step is in flight */
    int32_t timing;             /* 1: time each force evaluation with HIP events */
    int32_t pad_;
    double force_ms;            /* out (timing): summed force-kernel time */
    int64_t force_calls;        /* out (timing): force evaluations timed */
    md_mlp_t mlp;               /* MD_POT_MLP */
    const uint16_t *mlp_w;      /* MD_POT_MLP: MD_MLP_NPARAM bfloat16 parameters */
    float *dEdG;                /* MD_POT_MLP: [16n] scratch */
    int32_t *idx_in, *cnt_in;   /* MD_POT_MLP: compact list scratch, sized as idx, count */
    md_tb_t tb;                 /* MD_POT_TB (rho, fprime as for MD_POT_EAM) */
    md_tbm_t tbm;               /* MD_POT_TBM (rho, fprime as for MD_POT_EAM) */
    int32_t *types, *types_scratch;   /* MD_POT_TBM: [n] element of each sorted atom, permuted at builds */
    md_tab_t tab;               /* MD_POT_TAB (rho, fprime as for MD_POT_EAM) */
    const void *tab_table;      /* MD_POT_TAB: device table from md_tab_pack */
} md_system_t;

/* Runs `steps` velocity-Verlet steps (Sec. 3.3) of the path: kick + drift
 * with the rebuild check, md_bin_cells + md_permute + md_scale_positions +
 * md_build_neighbors whenever some atom moved more than skin/2 since the
 * last build, forces (md_forces_lj, md_forces_eam, md_forces_mlp,
 * md_forces_tb, md_forces_tbm or md_forces_tab), kick.  Between two
 * steps the closing half kick and the next opening half kick are applied as
 * one kick with the same forces.  On entry with need_build set (a new
 * system) the lists and forces are built first; otherwise f must hold the
 * forces of x.  Per-atom arrays stay in the library's sorted order; ids maps
 * them to input order.
 * The host waits once per step for the 4-byte rebuild flag, and once per
 * build for the longest list row: when host_status is pinned host memory
 * the device publishes them there (words 0-2: flag, word 3: longest row) and
 * the host polls them, otherwise it copies them and synchronises the stream.
 * Each step's force evaluation is queued before the host has read the flag
 * (and after a build, before it has read the longest row); the kernels skip
 * themselves on the device when the flag is set or a row overflowed.
 * Returns MD_OK when all steps are done and the state is at a step boundary.
 * MD_ERR_CAPACITY: a list row exceeded row_cap; row_cap_needed holds the
 * longest row, a step is in flight (phase 1); grow idx, set row_cap and call
 * again with the remaining steps (target - step).  MD_ERR_NONFINITE: a
 * position became non-finite.  With timing set, each force evaluation is
 * bracketed by HIP events on `stream` and their elapsed times are added to
 * force_ms / force_calls. */
int md_run(md_system_t *sys, int64_t steps, void *stream);

/* ---- measurement aid ----
 *
 * The achievable peaks of this GPU are measured, not assumed: md_probe runs
 * `blocks` blocks of 256 threads, each thread `iters` iterations of one kind
 * of arithmetic on independent chains, and writes nothing the caller needs
 * (out: a device word of the kind's type, written only in an impossible
 * case).  Time it with events on `stream`; work per launch:
 *   MD_PROBE_FMA_F32:   blocks * 256 * iters * 8 FP32 fused multiply-adds
 *   MD_PROBE_FMA_F64:   blocks * 256 * iters * 8 FP64 fused multiply-adds
 *   MD_PROBE_MFMA_BF16: blocks * 4 * iters * 8 v_mfma_f32_16x16x32_bf16
 *                       (16,384 operations each). */
#define MD_PROBE_FMA_F32   0
#define MD_PROBE_FMA_F64   1
#define MD_PROBE_MFMA_BF16 2

int md_probe(int32_t kind, int64_t iters, int32_t blocks, void *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MD_H */
