/*
 * FP64 CPU oracle of the learned descriptor-MLP potential.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h): loaded by the tests, the smoke
 * check and the benchmark's CPU-baseline leg, never by the product path.
 *
 * The learned form stands in for the embedded-atom energy of Eqs. (1)-(2):
 * the energy of atom i is a function of its radial environment only, as
 * F(rho_i) + 1/2 sum_j V(r_ij) is.  The model:
 *
 *   pair basis   g_k(r) = exp(-(r - mu_k)^2 / (2 w^2)) fc(r),  r < rc,
 *                fc(r)  = (cos(pi r / rc) + 1) / 2,  mu_k = mu0 + k dmu,
 *   descriptor   G_ik = sum_{j != i, r_ij < rc} g_k(r_ij),       k < 16,
 *   input        x_i  = (G_i - mean) * inv_std            (per component),
 *   network      h1 = silu(W1 x + b1)   (64),  h2 = silu(W2 h1 + b2)  (64),
 *                E_i = w3 . h2 + b3,    silu(a) = a / (1 + exp(-a)),
 *   energy       E = sum_i E_i,   forces F_i = -dE/dx_i.
 *
 * Parameter vector (OR_MLP_NPARAM doubles, row-major matrices, output index
 * first): W1[64][16], b1[64], W2[64][64], b2[64], w3[64], b3.
 *
 * Mixed precision: with bf16 != 0 every vector that enters a matrix product
 * is rounded to bfloat16 (round to nearest even) first -- x before W1, h1
 * before W2, and in the backward pass the vectors before W2^T, W1^T and the
 * weight-gradient products -- exactly where a BF16 matrix-core evaluation
 * rounds.  Weights are taken as given (the caller rounds them).  With
 * bf16 == 0 everything is plain FP64 and the forces are the exact negative
 * gradient of the energy.
 */
#ifndef MD_ORACLE_MLP_H
#define MD_ORACLE_MLP_H
#include <stdint.h>

#include "oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MLP_IN 16
#define OR_MLP_HID 64
#define OR_MLP_NPARAM (OR_MLP_HID * OR_MLP_IN + OR_MLP_HID + OR_MLP_HID * OR_MLP_HID + OR_MLP_HID + OR_MLP_HID + 1)

typedef struct {
    double rc;              /* descriptor cutoff */
    double mu0, dmu;        /* Gaussian centres mu_k = mu0 + k dmu */
    double width;           /* Gaussian width w */
    double mean[OR_MLP_IN];
    double inv_std[OR_MLP_IN];
} or_mlp_t;

/* Nearest bfloat16 value (ties to even) of v after rounding v to FP32. */
double or_bf16_round(double v);

/* Raw descriptors G[n][16] from a full neighbour list (any superset of the
 * pairs within rc; positions need not be wrapped). */
void or_mlp_descriptors(int64_t n, const double L[3], const double *x,
                        const double *y, const double *z,
                        const int64_t *offsets, const int32_t *idx,
                        const or_mlp_t *m, double *G);

/* Per-atom energies e_atom[n] and, if dEdG is not NULL, dE_i/dG_i [n][16]. */
void or_mlp_energy(int64_t n, const double *G, const or_mlp_t *m,
                   const double *params, int32_t bf16, double *e_atom,
                   double *dEdG);

/* Forces F_i = -sum_{j in N(i), r < rc} sum_k (dEdG_ik + dEdG_jk)
 * g_k'(r_ij) (x_i - x_j) / r_ij from a full list, and, if w6 is not NULL,
 * the virial W_ab = -1/2 sum_i sum_j s_ij R_a R_b / r_ij (xx, yy, zz, xy,
 * xz, yz), s_ij the scalar factor above. */
void or_mlp_forces(int64_t n, const double L[3], const double *x,
                   const double *y, const double *z, const int64_t *offsets,
                   const int32_t *idx, const or_mlp_t *m, const double *dEdG,
                   double *fx, double *fy, double *fz, double *w6);

/* Per-atom energy loss  (1/n) sum_i (E_i - target_i)^2  and, if grad is not
 * NULL, its gradient with respect to the parameter vector. */
double or_mlp_loss_grad(int64_t n, const double *G, const double *target,
                        const or_mlp_t *m, const double *params, int32_t bf16,
                        double *grad);

/* Training snapshots from a Finnis-Sinclair trajectory (Sec. 3.3 MD).
 * Equilibration: equil_steps velocity-Verlet steps in chunks of
 * rescale_every steps, the velocities rescaled to temperature T_kelvin after
 * each chunk (T = m e_unit sum v^2 / ((3n - 3) kB)).  Sampling: n_samples
 * times, sample_every NVE steps, then the wrapped positions pos[s][n][3],
 * the per-atom energies e_atom[s][n] and (if forces is not NULL) the forces
 * forces[s][n][3].  Returns the number of list builds, or -1 on allocation
 * failure. */
int64_t or_eam_samples(int64_t n, const double L[3], double *x, double *y,
                       double *z, double *vx, double *vy, double *vz,
                       const or_md_params_t *p, double T_kelvin, double kB,
                       double e_unit, int64_t equil_steps,
                       int64_t rescale_every, int64_t n_samples,
                       int64_t sample_every, double *pos, double *e_atom,
                       double *forces);

#ifdef __cplusplus
}
#endif
#endif
