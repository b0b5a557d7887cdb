/*
 * FP64 CPU oracle for the short-range molecular-dynamics hot path of
 * Mangiardi & Meyer, "A hybrid algorithm for parallel molecular dynamics
 * simulations" (arXiv:1611.00075).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously
 * correct statement of what the GPU path computes.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it.  It
 * shares no code, header, table or helper with the HIP library, and the HIP
 * library never calls it.
 *
 * Conventions (all functions):
 *   - positions, velocities, forces are FP64 structure-of-arrays in the
 *     caller's atom order;
 *   - the box is orthorhombic and periodic on every axis, edge lengths L[3];
 *   - every cutoff test is strict (r^2 < rc^2);
 *   - no function allocates memory that outlives the call; outputs are
 *     caller-owned.
 *
 * Parity pins: every function here is checked by the CPU tests against
 * brute force, closed-form lattice sums, finite differences of the energy,
 * conservation laws or published constants.  No function is "parity
 * unpinned".
 */
#ifndef MD_ORACLE_H
#define MD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- periodic geometry (Sec. 3.3: periodic boundaries on every axis) ---- */

/* Wrap each coordinate into [0, L): w = x - L*floor(x/L), then one
 * correction step each way.  FP64, correctly rounded division, no FMA. */
void or_wrap(int64_t n, const double L[3], double *x, double *y, double *z);

/* Cell coordinates of wrapped positions on an nc[0] x nc[1] x nc[2] grid:
 * c = (int)(w * (nc/L)), clamped to nc-1.  (Sec. 2.1: the volume is divided
 * into small cells.) */
void or_cell_coords(int64_t n, const double L[3], const int32_t nc[3],
                    const double *x, const double *y, const double *z,
                    int32_t *cx, int32_t *cy, int32_t *cz);

/* Minimum-image displacement component: dx = b - a, shifted by one box
 * length when it exceeds half a box. */
double or_minimg(double a, double b, double L);

/* ---- Verlet neighbour sets (Sec. 3.3: list cutoff larger than the
 * potential cutoff) ---- */

/* Full neighbour set N(i) = { j != i : r_ij^2 < r_list^2 } by the O(N^2)
 * definition.  Row i lists j in ascending order.  offsets has n+1 entries.
 * Returns the total number of entries; idx is written only if the total fits
 * in cap. */
int64_t or_neighbors_brute(int64_t n, const double L[3], double r_list,
                           const double *x, const double *y, const double *z,
                           int64_t *offsets, int32_t *idx, int64_t cap);

/* The same set through a cell list (cells of edge >= r_list, 27 neighbour
 * cells with duplicates removed when a box holds fewer than three cells).
 * Rows are sorted ascending so that the result is comparable entry by entry
 * with or_neighbors_brute.  Positions must already be wrapped. */
int64_t or_neighbors_cells(int64_t n, const double L[3], double r_list,
                           const double *x, const double *y, const double *z,
                           int64_t *offsets, int32_t *idx, int64_t cap);

/* ---- potentials ---- */

typedef struct {
    double eps, sigma, rc;
} or_lj_t;

/* Finnis-Sinclair form used for the metal benchmark:
 *   psi(r) = (r-d)^2 for r<d, F(rho) = -A sqrt(rho),
 *   V(r)   = (r-c)^2 (c0 + c1 r + c2 r^2) for r<c. */
typedef struct {
    double A, d, c, c0, c1, c2;
} or_fs_t;

/* or_neighbors_cells with the rows shared among `threads` OpenMP threads
 * (counted, summed, then filled and sorted row by row): the same output;
 * for timing the oracle on all cores. */
int64_t or_neighbors_cells_omp(int64_t n, const double L[3], double r_list,
                               const double *x, const double *y, const double *z,
                               int64_t *offsets, int32_t *idx, int64_t cap, int32_t threads);

/* Lennard-Jones forces as the gradient of the pair energy (the pair force
 * of Sec. 2.2): with U = 1/2 sum_i sum_{j != i, r_ij < rc} Phi(r_ij),
 *   F_i = -dU/dr_i = sum_{j in N(i), r_ij < rc} -(1/r) dPhi/dr (r_i - r_j),
 * summed over atom i's own row of a full list (every j != i within the
 * list cutoff, each pair in both rows; any superset of the pairs within rc).
 * ev[8] receives: E (truncated), E_shift (each pair shifted by -Phi(rc)),
 * virial W_xx, W_yy, W_zz, W_xy, W_xz, W_yz (sum over pairs of f_s R_a R_b),
 * each pair's share taken half from each of its two rows. */
void or_forces_lj(int64_t n, const double L[3], const double *x,
                  const double *y, const double *z, const int64_t *offsets,
                  const int32_t *idx, const or_lj_t *p, double *fx,
                  double *fy, double *fz, double ev[8]);

/* The same computation with the rows shared among `threads` OpenMP threads
 * (each force written by the thread of its row: no races); forces are the
 * same bits as or_forces_lj, the energy and virial sums differ only in the
 * order of their terms.  For timing the oracle on all cores. */
void or_forces_lj_omp(int64_t n, const double L[3], const double *x,
                      const double *y, const double *z, const int64_t *offsets,
                      const int32_t *idx, const or_lj_t *p, double *fx,
                      double *fy, double *fz, double ev[8], int32_t threads);

/* Embedded-atom forces in the three steps of Sec. 3.1 (after Eqs. 1-2):
 * (1) rho_i = sum_j psi(r_ij) by the pair loop, (2) F_i(rho_i) per atom,
 * (3) the pair interaction and the forces by the pair loop.
 * Outputs rho[n], fprime[n] (= F'(rho_i)), forces, e_atom[n] (per-atom
 * energy F(rho_i) + 1/2 sum_j V(r_ij); may be NULL) and ev[8]:
 * E_total, E_embed, then the six virial components. */
void or_forces_eam(int64_t n, const double L[3], const double *x,
                   const double *y, const double *z, const int64_t *offsets,
                   const int32_t *idx, const or_fs_t *p, double *rho,
                   double *fprime, double *fx, double *fy, double *fz,
                   double *e_atom, double ev[8]);

/* Second-moment tight-binding potential in the form of Eqs. (1)-(2): the
 * exponential density and pair functions and square-root embedding that
 * Sec. 3.1 names for its copper potential,
 *   psi(r) = xi^2 exp(-2q (r/r0 - 1)) S(r),  Phi(r) = 2A exp(-p (r/r0 - 1)) S(r),
 *   F(rho) = -sqrt(rho)  (F = F' = 0 at rho = 0),
 * with the smooth cutoff S = 1 for r <= rs, S = 0 for r >= rc and
 * S = 1 - x^3 (10 - 15 x + 6 x^2), x = (r - rs)/(rc - rs), in between.
 * (The factor 2 in Phi makes the paper's 1/2 sum_{i != j} Phi the sum over
 * atoms of sum_j A exp(...).)  Same three steps and outputs as
 * or_forces_eam; e_atom = F(rho_i) + 1/2 sum_j Phi(r_ij). */
typedef struct {
    double A, xi, p, q, r0, rs, rc;
} or_tb_t;

void or_forces_tb(int64_t n, const double L[3], const double *x,
                  const double *y, const double *z, const int64_t *offsets,
                  const int32_t *idx, const or_tb_t *p, double *rho,
                  double *fprime, double *fx, double *fy, double *fz,
                  double *e_atom, double ev[8]);

/* Two elements (types[i] = 0 or 1): the same form with the parameters of
 * the pair's kind, pair[types[i] + types[j]] (0: 0-0, 1: 0-1, 2: 1-1);
 * F(rho) = -sqrt(rho) for both elements.  Outputs as or_forces_tb. */
void or_forces_tbm(int64_t n, const double L[3], const double *x,
                   const double *y, const double *z, const int32_t *types,
                   const int64_t *offsets, const int32_t *idx,
                   const or_tb_t pair[3], double *rho, double *fprime,
                   double *fx, double *fy, double *fz, double *e_atom,
                   double ev[8]);

/* Tabulated functions (Sec. 3.1 names piecewise-defined psi and Phi for its
 * iron potential; Sec. 5 equates an interpolation table with such a
 * piecewise definition).  One element, the form of Eqs. (1)-(2):
 *   psi, Phi given at r_k = k dr (k = 0 .. nr-1) by value and slope;
 *   F given at rho_k = k drho (k = 0 .. nrho-1) by value and slope.
 * Between two knots a function is the cubic Hermite interpolant of the
 * values and slopes at the two knots.  psi = Phi = 0 for r >= rc =
 * (nr-1) dr (strict: a pair counts when r < rc).  Below rho_0 = 0 and above
 * rho_{nrho-1}, F continues along its tangent at that end knot.
 * Same three steps and outputs as or_forces_eam;
 * e_atom = F(rho_i) + 1/2 sum_j Phi(r_ij). */
typedef struct {
    int32_t nr, nrho;
    double dr, drho;
    const double *psi, *dpsi, *phi, *dphi, *F, *dF;
} or_tab_t;

void or_forces_tab(int64_t n, const double L[3], const double *x,
                   const double *y, const double *z, const int64_t *offsets,
                   const int32_t *idx, const or_tab_t *p, double *rho,
                   double *fprime, double *fx, double *fy, double *fz,
                   double *e_atom, double ev[8]);

/* One tabulated function (values f[m], slopes df[m] at u_k = k h) at u:
 * *val and *slope of its interpolant (the F rule outside [0, (m-1) h]). */
void or_tab_eval(int32_t m, double h, const double *f, const double *df,
                 double u, double *val, double *slope);

/* ---- velocity-Verlet molecular dynamics (Sec. 3.3) ---- */

enum { OR_POT_LJ = 0, OR_POT_EAM = 1 };

typedef struct {
    int32_t potential;      /* OR_POT_LJ or OR_POT_EAM */
    or_lj_t lj;
    or_fs_t fs;
    double r_list;          /* potential cutoff + skin */
    double skin;
    double dt;
    double mass;
    double force_to_accel;  /* 1 in reduced units; 1/103.6427 for eV, A, amu, fs */
    int32_t reverse_order;  /* 1: visit each neighbour row in reverse order */
    int32_t threads;        /* > 1: LJ forces and the per-atom loops on this many OpenMP threads */
} or_md_params_t;

/* Runs `steps` velocity-Verlet steps in place.  Before the first step the
 * positions are wrapped, the list is built and the forces are evaluated.
 * Each step: half kick, drift, rebuild (wrap + new list) iff some atom has
 * moved more than skin/2 since the last build, forces, half kick.
 * Per step k (0 = the initial state, k = 1..steps after step k) the arrays
 * epot[k], ekin[k] (may be NULL) receive the potential energy (E_shift for
 * LJ, E_total for EAM) and the kinetic energy.  If loop_seconds is not
 * NULL it receives the wall time of the step loop alone (the initial build
 * and force evaluation excluded, as in the paper's timing, Sec. 3.3).
 * Returns the number of list builds including the first, or a negative
 * value on allocation failure. */
int64_t or_md_run(int64_t n, const double L[3], double *x, double *y,
                  double *z, double *vx, double *vy, double *vz,
                  const or_md_params_t *p, int64_t steps, double *epot,
                  double *ekin, double *loop_seconds);

#ifdef __cplusplus
}
#endif
#endif
