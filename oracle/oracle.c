/*
 * FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Written from the definitions of arXiv:1611.00075: the pair-force loop with
 * Newton's third law (Sec. 2.2), the embedded-atom energy (Eqs. 1 and 2) and
 * its three-step evaluation (Sec. 3.1), velocity-Verlet dynamics with a
 * Verlet list whose cutoff exceeds the potential cutoff and the
 * displacement rebuild rule (Sec. 3.3).  Nothing here is blocked, fused or
 * reordered for speed.
 *
 * Compile with -ffp-contract=off: cell and neighbour decisions are compared
 * bit for bit with the GPU library.
 */
#include "oracle.h"

#include <math.h>
#include <time.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* periodic geometry                                                   */
/* ------------------------------------------------------------------ */

static double wrap1(double x, double L)
{
    double w = x - L * floor(x / L);
    if (w >= L) w -= L;
    if (w < 0.0) w += L;
    return w;
}

void or_wrap(int64_t n, const double L[3], double *x, double *y, double *z)
{
    for (int64_t i = 0; i < n; ++i) {
        x[i] = wrap1(x[i], L[0]);
        y[i] = wrap1(y[i], L[1]);
        z[i] = wrap1(z[i], L[2]);
    }
}

static int32_t cell1(double w, double inv_cell, int32_t nc)
{
    int32_t c = (int32_t)(w * inv_cell);
    if (c >= nc) c = nc - 1;
    if (c < 0) c = 0;
    return c;
}

void or_cell_coords(int64_t n, const double L[3], const int32_t nc[3],
                    const double *x, const double *y, const double *z,
                    int32_t *cx, int32_t *cy, int32_t *cz)
{
    double inv[3];
    for (int a = 0; a < 3; ++a) inv[a] = (double)nc[a] / L[a];
    for (int64_t i = 0; i < n; ++i) {
        cx[i] = cell1(x[i], inv[0], nc[0]);
        cy[i] = cell1(y[i], inv[1], nc[1]);
        cz[i] = cell1(z[i], inv[2], nc[2]);
    }
}

double or_minimg(double a, double b, double L)
{
    double d = b - a;
    if (d > 0.5 * L)
        d -= L;
    else if (d < -0.5 * L)
        d += L;
    return d;
}

/* squared minimum-image distance, summed left to right */
static double dist2(const double L[3], const double *x, const double *y,
                    const double *z, int64_t i, int64_t j, double d[3])
{
    d[0] = or_minimg(x[i], x[j], L[0]);
    d[1] = or_minimg(y[i], y[j], L[1]);
    d[2] = or_minimg(z[i], z[j], L[2]);
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

/* ------------------------------------------------------------------ */
/* neighbour sets                                                      */
/* ------------------------------------------------------------------ */

int64_t or_neighbors_brute(int64_t n, const double L[3], double r_list,
                           const double *x, const double *y, const double *z,
                           int64_t *offsets, int32_t *idx, int64_t cap)
{
    const double rl2 = r_list * r_list;
    double d[3];
    int64_t total = 0;
    offsets[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            if (dist2(L, x, y, z, i, j, d) < rl2) {
                if (total < cap) idx[total] = (int32_t)j;
                ++total;
            }
        }
        offsets[i + 1] = total;
    }
    return total;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t u = *(const int32_t *)a, v = *(const int32_t *)b;
    return (u > v) - (u < v);
}

/* distinct values of (c + o) mod nc for o in {-1, 0, 1} */
static int stencil_axis(int32_t c, int32_t nc, int32_t out[3])
{
    int m = 0;
    for (int o = -1; o <= 1; ++o) {
        int32_t v = ((c + o) % nc + nc) % nc;
        int dup = 0;
        for (int k = 0; k < m; ++k) dup |= (out[k] == v);
        if (!dup) out[m++] = v;
    }
    return m;
}

int64_t or_neighbors_cells(int64_t n, const double L[3], double r_list,
                           const double *x, const double *y, const double *z,
                           int64_t *offsets, int32_t *idx, int64_t cap)
{
    int32_t nc[3];
    for (int a = 0; a < 3; ++a) {
        nc[a] = (int32_t)floor(L[a] / r_list);
        if (nc[a] < 1) nc[a] = 1;
    }
    const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int32_t *cx = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *cy = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *cz = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *head = malloc(sizeof(int64_t) * (size_t)ncell);
    int64_t *next = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    or_cell_coords(n, L, nc, x, y, z, cx, cy, cz);
    for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
    for (int64_t i = n - 1; i >= 0; --i) {
        int64_t c = cx[i] + (int64_t)nc[0] * (cy[i] + (int64_t)nc[1] * cz[i]);
        next[i] = head[c];
        head[c] = i;
    }
    const double rl2 = r_list * r_list;
    double d[3];
    int64_t total = 0;
    offsets[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t sx[3], sy[3], sz[3];
        int mx = stencil_axis(cx[i], nc[0], sx);
        int my = stencil_axis(cy[i], nc[1], sy);
        int mz = stencil_axis(cz[i], nc[2], sz);
        int64_t row = total;
        for (int a = 0; a < mx; ++a)
            for (int b = 0; b < my; ++b)
                for (int e = 0; e < mz; ++e) {
                    int64_t c = sx[a] + (int64_t)nc[0] * (sy[b] + (int64_t)nc[1] * sz[e]);
                    for (int64_t j = head[c]; j >= 0; j = next[j]) {
                        if (j == i) continue;
                        if (dist2(L, x, y, z, i, j, d) < rl2) {
                            if (total < cap) idx[total] = (int32_t)j;
                            ++total;
                        }
                    }
                }
        if (total <= cap) qsort(idx + row, (size_t)(total - row), sizeof(int32_t), cmp_i32);
        offsets[i + 1] = total;
    }
    free(cx); free(cy); free(cz); free(head); free(next);
    return total;
}

/* The same list with the rows shared among `threads` OpenMP threads: each
 * row counted, the offsets summed, each row filled and sorted by its own
 * thread.  The same output as or_neighbors_cells; for timing only. */
static int64_t cell_row(int64_t i, const int32_t nc[3], const int32_t *cx, const int32_t *cy, const int32_t *cz,
                        const int64_t *head, const int64_t *next, const double L[3], double rl2, const double *x,
                        const double *y, const double *z, int32_t *out)
{
    int32_t sx[3], sy[3], sz[3];
    int mx = stencil_axis(cx[i], nc[0], sx);
    int my = stencil_axis(cy[i], nc[1], sy);
    int mz = stencil_axis(cz[i], nc[2], sz);
    double d[3];
    int64_t m = 0;
    for (int a = 0; a < mx; ++a)
        for (int b = 0; b < my; ++b)
            for (int e = 0; e < mz; ++e) {
                int64_t c = sx[a] + (int64_t)nc[0] * (sy[b] + (int64_t)nc[1] * sz[e]);
                for (int64_t j = head[c]; j >= 0; j = next[j]) {
                    if (j == i) continue;
                    if (dist2(L, x, y, z, i, j, d) < rl2) {
                        if (out) out[m] = (int32_t)j;
                        ++m;
                    }
                }
            }
    if (out) qsort(out, (size_t)m, sizeof(int32_t), cmp_i32);
    return m;
}

int64_t or_neighbors_cells_omp(int64_t n, const double L[3], double r_list,
                               const double *x, const double *y, const double *z,
                               int64_t *offsets, int32_t *idx, int64_t cap, int32_t threads)
{
    int32_t nc[3];
    for (int a = 0; a < 3; ++a) {
        nc[a] = (int32_t)floor(L[a] / r_list);
        if (nc[a] < 1) nc[a] = 1;
    }
    const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int32_t *cx = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *cy = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *cz = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *head = malloc(sizeof(int64_t) * (size_t)ncell);
    int64_t *next = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    or_cell_coords(n, L, nc, x, y, z, cx, cy, cz);
    for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
    for (int64_t i = n - 1; i >= 0; --i) {
        int64_t c = cx[i] + (int64_t)nc[0] * (cy[i] + (int64_t)nc[1] * cz[i]);
        next[i] = head[c];
        head[c] = i;
    }
    const double rl2 = r_list * r_list;
    offsets[0] = 0;
#pragma omp parallel for num_threads(threads) schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i)
        offsets[i + 1] = cell_row(i, nc, cx, cy, cz, head, next, L, rl2, x, y, z, NULL);
    for (int64_t i = 0; i < n; ++i) offsets[i + 1] += offsets[i];
    const int64_t total = offsets[n];
    if (total <= cap) {
#pragma omp parallel for num_threads(threads) schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i)
            cell_row(i, nc, cx, cy, cz, head, next, L, rl2, x, y, z, idx + offsets[i]);
    }
    free(cx); free(cy); free(cz); free(head); free(next);
    return total;
}

/* ------------------------------------------------------------------ */
/* Lennard-Jones: forces as the gradient of the pair energy            */
/* ------------------------------------------------------------------ */

static double lj_phi(const or_lj_t *p, double r2)
{
    double s2 = p->sigma * p->sigma / r2;
    double s6 = s2 * s2 * s2;
    return 4.0 * p->eps * (s6 * s6 - s6);
}

/* The contribution of atom i's row: its force, and its half of the energy
 * and virial of each of its pairs (every pair appears in both rows). */
static void lj_row(int64_t i, const double L[3], const double *x, const double *y, const double *z,
                   const int64_t *offsets, const int32_t *idx, const or_lj_t *p, double rc2, double phi_rc,
                   double f[3], double *E, double *Es, double W[6])
{
    f[0] = f[1] = f[2] = 0.0;
    for (int64_t k = offsets[i]; k < offsets[i + 1]; ++k) {
        int64_t j = idx[k];
        if (j == i) continue;
        double d[3];
        double r2 = dist2(L, x, y, z, i, j, d);
        if (!(r2 < rc2)) continue;
        /* R = r_i - r_j is minus the displacement i -> j */
        double R[3] = {-d[0], -d[1], -d[2]};
        double s2 = p->sigma * p->sigma / r2;
        double s6 = s2 * s2 * s2;
        /* -dPhi(r_ij)/dr_i = -(1/r) dPhi/dr R */
        double fs = 24.0 * p->eps * (2.0 * s6 * s6 - s6) / r2;
        f[0] += fs * R[0]; f[1] += fs * R[1]; f[2] += fs * R[2];
        double phi = 4.0 * p->eps * (s6 * s6 - s6);
        *E += 0.5 * phi;
        *Es += 0.5 * (phi - phi_rc);
        W[0] += 0.5 * fs * R[0] * R[0]; W[1] += 0.5 * fs * R[1] * R[1];
        W[2] += 0.5 * fs * R[2] * R[2]; W[3] += 0.5 * fs * R[0] * R[1];
        W[4] += 0.5 * fs * R[0] * R[2]; W[5] += 0.5 * fs * R[1] * R[2];
    }
}

void or_forces_lj(int64_t n, const double L[3], const double *x,
                  const double *y, const double *z, const int64_t *offsets,
                  const int32_t *idx, const or_lj_t *p, double *fx,
                  double *fy, double *fz, double ev[8])
{
    const double rc2 = p->rc * p->rc;
    const double phi_rc = lj_phi(p, rc2);
    double E = 0.0, Es = 0.0, W[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        double f[3];
        lj_row(i, L, x, y, z, offsets, idx, p, rc2, phi_rc, f, &E, &Es, W);
        fx[i] = f[0]; fy[i] = f[1]; fz[i] = f[2];
    }
    ev[0] = E; ev[1] = Es;
    for (int a = 0; a < 6; ++a) ev[2 + a] = W[a];
}

void or_forces_lj_omp(int64_t n, const double L[3], const double *x,
                      const double *y, const double *z, const int64_t *offsets,
                      const int32_t *idx, const or_lj_t *p, double *fx,
                      double *fy, double *fz, double ev[8], int32_t threads)
{
    const double rc2 = p->rc * p->rc;
    const double phi_rc = lj_phi(p, rc2);
    double E = 0.0, Es = 0.0, W0 = 0, W1 = 0, W2 = 0, W3 = 0, W4 = 0, W5 = 0;
#pragma omp parallel for num_threads(threads) schedule(static) reduction(+ : E, Es, W0, W1, W2, W3, W4, W5)
    for (int64_t i = 0; i < n; ++i) {
        double f[3], W[6] = {0, 0, 0, 0, 0, 0};
        lj_row(i, L, x, y, z, offsets, idx, p, rc2, phi_rc, f, &E, &Es, W);
        fx[i] = f[0]; fy[i] = f[1]; fz[i] = f[2];
        W0 += W[0]; W1 += W[1]; W2 += W[2]; W3 += W[3]; W4 += W[4]; W5 += W[5];
    }
    ev[0] = E; ev[1] = Es;
    ev[2] = W0; ev[3] = W1; ev[4] = W2; ev[5] = W3; ev[6] = W4; ev[7] = W5;
}

/* ------------------------------------------------------------------ */
/* Embedded-atom method, Finnis-Sinclair form, three steps             */
/* ------------------------------------------------------------------ */

static double fs_V(const or_fs_t *p, double r)
{
    double t = r - p->c;
    return t * t * (p->c0 + p->c1 * r + p->c2 * r * r);
}

static double fs_dV(const or_fs_t *p, double r)
{
    double t = r - p->c;
    return 2.0 * t * (p->c0 + p->c1 * r + p->c2 * r * r) +
           t * t * (p->c1 + 2.0 * p->c2 * r);
}

void or_forces_eam(int64_t n, const double L[3], const double *x,
                   const double *y, const double *z, const int64_t *offsets,
                   const int32_t *idx, const or_fs_t *p, double *rho,
                   double *fprime, double *fx, double *fy, double *fz,
                   double *e_atom, double ev[8])
{
    const double d2 = p->d * p->d, c2 = p->c * p->c;
    double d[3];
    /* step 1: localization function rho_i = sum_{j != i} psi(r_ij) */
    for (int64_t i = 0; i < n; ++i) rho[i] = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = offsets[i]; k < offsets[i + 1]; ++k) {
            int64_t j = idx[k];
            if (j <= i) continue;
            double r2 = dist2(L, x, y, z, i, j, d);
            if (!(r2 < d2)) continue;
            double t = sqrt(r2) - p->d;
            rho[i] += t * t;
            rho[j] += t * t;
        }
    /* step 2: embedding energy F_i(rho_i) and its derivative */
    double Eemb = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double F = 0.0, Fp = 0.0;
        if (rho[i] > 0.0) {
            double s = sqrt(rho[i]);
            F = -p->A * s;
            Fp = -p->A / (2.0 * s);
        }
        fprime[i] = Fp;
        Eemb += F;
        if (e_atom) e_atom[i] = F;
        fx[i] = fy[i] = fz[i] = 0.0;
    }
    /* step 3: pair interaction and forces */
    double Epair = 0.0, W[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = offsets[i]; k < offsets[i + 1]; ++k) {
            int64_t j = idx[k];
            if (j <= i) continue;
            double r2 = dist2(L, x, y, z, i, j, d);
            if (!(r2 < d2) && !(r2 < c2)) continue;
            double r = sqrt(r2);
            double dUdr = 0.0; /* dU/dr_ij with rho_i, rho_j frozen */
            if (r2 < d2) dUdr += (fprime[i] + fprime[j]) * 2.0 * (r - p->d);
            if (r2 < c2) {
                double V = fs_V(p, r);
                dUdr += fs_dV(p, r);
                Epair += V;
                if (e_atom) {
                    e_atom[i] += 0.5 * V;
                    e_atom[j] += 0.5 * V;
                }
            }
            double R[3] = {-d[0], -d[1], -d[2]};
            double g = -dUdr / r; /* F_i = g R */
            fx[i] += g * R[0]; fy[i] += g * R[1]; fz[i] += g * R[2];
            fx[j] -= g * R[0]; fy[j] -= g * R[1]; fz[j] -= g * R[2];
            W[0] += g * R[0] * R[0]; W[1] += g * R[1] * R[1];
            W[2] += g * R[2] * R[2]; W[3] += g * R[0] * R[1];
            W[4] += g * R[0] * R[2]; W[5] += g * R[1] * R[2];
        }
    ev[0] = Eemb + Epair;
    ev[1] = Eemb;
    for (int a = 0; a < 6; ++a) ev[2 + a] = W[a];
}

/* ------------------------------------------------------------------ */
/* second-moment tight-binding potential                              */
/* ------------------------------------------------------------------ */

/* smooth cutoff S(r) and dS/dr */
static void tb_switch(const or_tb_t *p, double r, double *S, double *dS)
{
    if (r <= p->rs) {
        *S = 1.0;
        *dS = 0.0;
        return;
    }
    if (r >= p->rc) {
        *S = 0.0;
        *dS = 0.0;
        return;
    }
    double w = p->rc - p->rs, x = (r - p->rs) / w;
    *S = 1.0 - x * x * x * (10.0 - 15.0 * x + 6.0 * x * x);
    *dS = -30.0 * x * x * (1.0 - x) * (1.0 - x) / w;
}

void or_forces_tb(int64_t n, const double L[3], const double *x,
                  const double *y, const double *z, const int64_t *offsets,
                  const int32_t *idx, const or_tb_t *p, double *rho,
                  double *fprime, double *fx, double *fy, double *fz,
                  double *e_atom, double ev[8])
{
    const double rc2 = p->rc * p->rc;
    double d[3];
    /* step 1: rho_i = sum_{j != i} psi(r_ij) */
    for (int64_t i = 0; i < n; ++i) rho[i] = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = offsets[i]; k < offsets[i + 1]; ++k) {
            int64_t j = idx[k];
            if (j <= i) continue;
            double r2 = dist2(L, x, y, z, i, j, d);
            if (!(r2 < rc2)) continue;
            double r = sqrt(r2), S, dS;
            tb_switch(p, r, &S, &dS);
            double psi = p->xi * p->xi * exp(-2.0 * p->q * (r / p->r0 - 1.0)) * S;
            rho[i] += psi;
            rho[j] += psi;
        }
    /* step 2: embedding F_i = -sqrt(rho_i) and F'_i */
    double Eemb = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double F = 0.0, Fp = 0.0;
        if (rho[i] > 0.0) {
            double s = sqrt(rho[i]);
            F = -s;
            Fp = -1.0 / (2.0 * s);
        }
        fprime[i] = Fp;
        Eemb += F;
        if (e_atom) e_atom[i] = F;
        fx[i] = fy[i] = fz[i] = 0.0;
    }
    /* step 3: pair interaction and forces */
    double Epair = 0.0, W[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = offsets[i]; k < offsets[i + 1]; ++k) {
            int64_t j = idx[k];
            if (j <= i) continue;
            double r2 = dist2(L, x, y, z, i, j, d);
            if (!(r2 < rc2)) continue;
            double r = sqrt(r2), S, dS;
            tb_switch(p, r, &S, &dS);
            double eq = p->xi * p->xi * exp(-2.0 * p->q * (r / p->r0 - 1.0));
            double ep = 2.0 * p->A * exp(-p->p * (r / p->r0 - 1.0));
            double dpsi = eq * (dS - 2.0 * p->q / p->r0 * S);
            double Phi = ep * S, dPhi = ep * (dS - p->p / p->r0 * S);
            double dUdr = (fprime[i] + fprime[j]) * dpsi + dPhi;
            Epair += Phi;
            if (e_atom) {
                e_atom[i] += 0.5 * Phi;
                e_atom[j] += 0.5 * Phi;
            }
            double R[3] = {-d[0], -d[1], -d[2]};
            double g = -dUdr / r; /* F_i = g R */
            fx[i] += g * R[0]; fy[i] += g * R[1]; fz[i] += g * R[2];
            fx[j] -= g * R[0]; fy[j] -= g * R[1]; fz[j] -= g * R[2];
            W[0] += g * R[0] * R[0]; W[1] += g * R[1] * R[1];
            W[2] += g * R[2] * R[2]; W[3] += g * R[0] * R[1];
            W[4] += g * R[0] * R[2]; W[5] += g * R[1] * R[2];
        }
    ev[0] = Eemb + Epair;
    ev[1] = Eemb;
    for (int a = 0; a < 6; ++a) ev[2 + a] = W[a];
}

/* ------------------------------------------------------------------ */
/* tabulated functions: cubic Hermite interpolation between knots       */
/* ------------------------------------------------------------------ */

/* The interpolant on [u_k, u_k + h] with s = (u - u_k)/h:
 *   f = H00(s) f_k + H10(s) h f'_k + H01(s) f_{k+1} + H11(s) h f'_{k+1},
 * H00 = 2s^3 - 3s^2 + 1, H10 = s^3 - 2s^2 + s, H01 = -2s^3 + 3s^2,
 * H11 = s^3 - s^2 (the textbook cubic Hermite basis); its slope is the
 * derivative of the same expression in u.  Outside [u_0, u_{m-1}] the
 * tangent line at the end knot. */
void or_tab_eval(int32_t m, double h, const double *f, const double *df,
                 double u, double *val, double *slope)
{
    const double umax = (m - 1) * h;
    if (u < 0.0) {
        *val = f[0] + df[0] * u;
        *slope = df[0];
        return;
    }
    if (u > umax) {
        *val = f[m - 1] + df[m - 1] * (u - umax);
        *slope = df[m - 1];
        return;
    }
    int32_t k = (int32_t)floor(u / h);
    if (k > m - 2) k = m - 2;
    const double s = (u - k * h) / h;
    const double s2 = s * s, s3 = s2 * s;
    const double H00 = 2.0 * s3 - 3.0 * s2 + 1.0, H10 = s3 - 2.0 * s2 + s;
    const double H01 = -2.0 * s3 + 3.0 * s2, H11 = s3 - s2;
    const double dH00 = 6.0 * s2 - 6.0 * s, dH10 = 3.0 * s2 - 4.0 * s + 1.0;
    const double dH01 = -6.0 * s2 + 6.0 * s, dH11 = 3.0 * s2 - 2.0 * s;
    *val = H00 * f[k] + H10 * h * df[k] + H01 * f[k + 1] + H11 * h * df[k + 1];
    *slope = (dH00 * f[k] + dH01 * f[k + 1]) / h + dH10 * df[k] + dH11 * df[k + 1];
}

void or_forces_tab(int64_t n, const double L[3], const double *x,
                   const double *y, const double *z, const int64_t *offsets,
                   const int32_t *idx, const or_tab_t *p, double *rho,
                   double *fprime, double *fx, double *fy, double *fz,
                   double *e_atom, double ev[8])
{
    const double rc = (p->nr - 1) * p->dr, rc2 = rc * rc;
    double d[3];
    /* step 1: rho_i = sum_{j != i} psi(r_ij) */
    for (int64_t i = 0; i < n; ++i) rho[i] = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = offsets[i]; k < offsets[i + 1]; ++k) {
            int64_t j = idx[k];
            if (j <= i) continue;
            double r2 = dist2(L, x, y, z, i, j, d);
            if (!(r2 < rc2)) continue;
            double r = sqrt(r2), psi, dpsi;
            if (!(r < rc)) continue;
            or_tab_eval(p->nr, p->dr, p->psi, p->dpsi, r, &psi, &dpsi);
            rho[i] += psi;
            rho[j] += psi;
        }
    /* step 2: embedding F(rho_i) and F'(rho_i) */
    double Eemb = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double F, Fp;
        or_tab_eval(p->nrho, p->drho, p->F, p->dF, rho[i], &F, &Fp);
        fprime[i] = Fp;
        Eemb += F;
        if (e_atom) e_atom[i] = F;
        fx[i] = fy[i] = fz[i] = 0.0;
    }
    /* step 3: pair interaction and forces */
    double Epair = 0.0, W[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = offsets[i]; k < offsets[i + 1]; ++k) {
            int64_t j = idx[k];
            if (j <= i) continue;
            double r2 = dist2(L, x, y, z, i, j, d);
            if (!(r2 < rc2)) continue;
            double r = sqrt(r2), psi, dpsi, Phi, dPhi;
            if (!(r < rc)) continue;
            or_tab_eval(p->nr, p->dr, p->psi, p->dpsi, r, &psi, &dpsi);
            or_tab_eval(p->nr, p->dr, p->phi, p->dphi, r, &Phi, &dPhi);
            double dUdr = (fprime[i] + fprime[j]) * dpsi + dPhi;
            Epair += Phi;
            if (e_atom) {
                e_atom[i] += 0.5 * Phi;
                e_atom[j] += 0.5 * Phi;
            }
            double R[3] = {-d[0], -d[1], -d[2]};
            double g = -dUdr / r; /* F_i = g R */
            fx[i] += g * R[0]; fy[i] += g * R[1]; fz[i] += g * R[2];
            fx[j] -= g * R[0]; fy[j] -= g * R[1]; fz[j] -= g * R[2];
            W[0] += g * R[0] * R[0]; W[1] += g * R[1] * R[1];
            W[2] += g * R[2] * R[2]; W[3] += g * R[0] * R[1];
            W[4] += g * R[0] * R[2]; W[5] += g * R[1] * R[2];
        }
    ev[0] = Eemb + Epair;
    ev[1] = Eemb;
    for (int a = 0; a < 6; ++a) ev[2 + a] = W[a];
}

void or_forces_tbm(int64_t n, const double L[3], const double *x,
                   const double *y, const double *z, const int32_t *types,
                   const int64_t *offsets, const int32_t *idx,
                   const or_tb_t pair[3], double *rho, double *fprime,
                   double *fx, double *fy, double *fz, double *e_atom,
                   double ev[8])
{
    double d[3];
    /* step 1: rho_i = sum_{j != i} psi_{t_i t_j}(r_ij) */
    for (int64_t i = 0; i < n; ++i) rho[i] = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = offsets[i]; k < offsets[i + 1]; ++k) {
            int64_t j = idx[k];
            if (j <= i) continue;
            const or_tb_t *p = &pair[types[i] + types[j]];
            double r2 = dist2(L, x, y, z, i, j, d);
            if (!(r2 < p->rc * p->rc)) continue;
            double r = sqrt(r2), S, dS;
            tb_switch(p, r, &S, &dS);
            double psi = p->xi * p->xi * exp(-2.0 * p->q * (r / p->r0 - 1.0)) * S;
            rho[i] += psi;
            rho[j] += psi;
        }
    /* step 2: embedding F_i = -sqrt(rho_i) and F'_i */
    double Eemb = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double F = 0.0, Fp = 0.0;
        if (rho[i] > 0.0) {
            double s = sqrt(rho[i]);
            F = -s;
            Fp = -1.0 / (2.0 * s);
        }
        fprime[i] = Fp;
        Eemb += F;
        if (e_atom) e_atom[i] = F;
        fx[i] = fy[i] = fz[i] = 0.0;
    }
    /* step 3: pair interaction and forces */
    double Epair = 0.0, W[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = offsets[i]; k < offsets[i + 1]; ++k) {
            int64_t j = idx[k];
            if (j <= i) continue;
            const or_tb_t *p = &pair[types[i] + types[j]];
            double r2 = dist2(L, x, y, z, i, j, d);
            if (!(r2 < p->rc * p->rc)) continue;
            double r = sqrt(r2), S, dS;
            tb_switch(p, r, &S, &dS);
            double eq = p->xi * p->xi * exp(-2.0 * p->q * (r / p->r0 - 1.0));
            double ep = 2.0 * p->A * exp(-p->p * (r / p->r0 - 1.0));
            double dpsi = eq * (dS - 2.0 * p->q / p->r0 * S);
            double Phi = ep * S, dPhi = ep * (dS - p->p / p->r0 * S);
            double dUdr = (fprime[i] + fprime[j]) * dpsi + dPhi;
            Epair += Phi;
            if (e_atom) {
                e_atom[i] += 0.5 * Phi;
                e_atom[j] += 0.5 * Phi;
            }
            double R[3] = {-d[0], -d[1], -d[2]};
            double g = -dUdr / r; /* F_i = g R */
            fx[i] += g * R[0]; fy[i] += g * R[1]; fz[i] += g * R[2];
            fx[j] -= g * R[0]; fy[j] -= g * R[1]; fz[j] -= g * R[2];
            W[0] += g * R[0] * R[0]; W[1] += g * R[1] * R[1];
            W[2] += g * R[2] * R[2]; W[3] += g * R[0] * R[1];
            W[4] += g * R[0] * R[2]; W[5] += g * R[1] * R[2];
        }
    ev[0] = Eemb + Epair;
    ev[1] = Eemb;
    for (int a = 0; a < 6; ++a) ev[2 + a] = W[a];
}

/* ------------------------------------------------------------------ */
/* velocity Verlet with the displacement rebuild rule                  */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t *off;
    int32_t *idx;
    int64_t cap;
} list_t;

static int64_t cells_list(int64_t n, const double L[3], double r_list, const double *x, const double *y,
                          const double *z, list_t *l, int32_t threads)
{
    if (threads > 1) return or_neighbors_cells_omp(n, L, r_list, x, y, z, l->off, l->idx, l->cap, threads);
    return or_neighbors_cells(n, L, r_list, x, y, z, l->off, l->idx, l->cap);
}

static int build_list(int64_t n, const double L[3], double r_list,
                      const double *x, const double *y, const double *z,
                      list_t *l, int reverse, int32_t threads)
{
    int64_t need = cells_list(n, L, r_list, x, y, z, l, threads);
    if (need > l->cap) {
        free(l->idx);
        l->cap = need + need / 4 + 16;
        l->idx = malloc(sizeof(int32_t) * (size_t)l->cap);
        if (!l->idx) return -1;
        cells_list(n, L, r_list, x, y, z, l, threads);
    }
    if (reverse) {
        for (int64_t i = 0; i < n; ++i) {
            int64_t a = l->off[i], b = l->off[i + 1] - 1;
            while (a < b) {
                int32_t t = l->idx[a]; l->idx[a] = l->idx[b]; l->idx[b] = t;
                ++a; --b;
            }
        }
    }
    return 0;
}

/* forces on the current list; returns the potential energy that the
 * energy-conservation checks follow (E_shift for LJ, E_total for EAM) */
static double eval_forces(int64_t n, const double L[3], const double *x,
                          const double *y, const double *z, const list_t *l,
                          const or_md_params_t *p, double *fx, double *fy,
                          double *fz, double *rho, double *fp)
{
    double ev[8];
    if (p->potential == OR_POT_LJ) {
        if (p->threads > 1)
            or_forces_lj_omp(n, L, x, y, z, l->off, l->idx, &p->lj, fx, fy, fz, ev, p->threads);
        else
            or_forces_lj(n, L, x, y, z, l->off, l->idx, &p->lj, fx, fy, fz, ev);
        return ev[1];
    }
    or_forces_eam(n, L, x, y, z, l->off, l->idx, &p->fs, rho, fp, fx, fy, fz, NULL, ev);
    return ev[0];
}

static double kinetic(int64_t n, const double *vx, const double *vy,
                      const double *vz, double mass, int32_t threads)
{
    double s = 0.0;
#pragma omp parallel for if (threads > 1) num_threads(threads) schedule(static) reduction(+ : s)
    for (int64_t i = 0; i < n; ++i) s += vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i];
    return 0.5 * mass * s;
}

int64_t or_md_run(int64_t n, const double L[3], double *x, double *y,
                  double *z, double *vx, double *vy, double *vz,
                  const or_md_params_t *p, int64_t steps, double *epot,
                  double *ekin, double *loop_seconds)
{
    size_t nb = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *fx = malloc(nb), *fy = malloc(nb), *fz = malloc(nb);
    double *xr = malloc(nb), *yr = malloc(nb), *zr = malloc(nb);
    double *rho = malloc(nb), *fp = malloc(nb);
    list_t l;
    l.off = malloc(sizeof(int64_t) * (size_t)(n + 1));
    l.cap = 64 * n + 16;
    l.idx = malloc(sizeof(int32_t) * (size_t)l.cap);
    int64_t builds = -1;
    if (!fx || !fy || !fz || !xr || !yr || !zr || !rho || !fp || !l.off || !l.idx) goto out;

    const double half_skin2 = 0.25 * p->skin * p->skin;
    const double hk = 0.5 * p->dt * p->force_to_accel / p->mass;

    or_wrap(n, L, x, y, z);
    if (build_list(n, L, p->r_list, x, y, z, &l, p->reverse_order, p->threads)) goto out;
    builds = 1;
    memcpy(xr, x, nb); memcpy(yr, y, nb); memcpy(zr, z, nb);
    double ep = eval_forces(n, L, x, y, z, &l, p, fx, fy, fz, rho, fp);
    if (epot) epot[0] = ep;
    const int32_t th = p->threads > 1 ? p->threads : 1;
    if (ekin) ekin[0] = kinetic(n, vx, vy, vz, p->mass, th);

    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    for (int64_t s = 1; s <= steps; ++s) {
        double maxd2 = 0.0;
#pragma omp parallel for if (th > 1) num_threads(th) schedule(static) reduction(max : maxd2)
        for (int64_t i = 0; i < n; ++i) {
            vx[i] += hk * fx[i]; vy[i] += hk * fy[i]; vz[i] += hk * fz[i];
            x[i] += p->dt * vx[i]; y[i] += p->dt * vy[i]; z[i] += p->dt * vz[i];
            double dx = or_minimg(xr[i], x[i], L[0]);
            double dy = or_minimg(yr[i], y[i], L[1]);
            double dz = or_minimg(zr[i], z[i], L[2]);
            double d2 = (dx * dx + dy * dy) + dz * dz;
            if (d2 > maxd2) maxd2 = d2;
        }
        if (maxd2 > half_skin2) {
            or_wrap(n, L, x, y, z);
            if (build_list(n, L, p->r_list, x, y, z, &l, p->reverse_order, p->threads)) { builds = -1; goto out; }
            ++builds;
            memcpy(xr, x, nb); memcpy(yr, y, nb); memcpy(zr, z, nb);
        }
        ep = eval_forces(n, L, x, y, z, &l, p, fx, fy, fz, rho, fp);
#pragma omp parallel for if (th > 1) num_threads(th) schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            vx[i] += hk * fx[i]; vy[i] += hk * fy[i]; vz[i] += hk * fz[i];
        }
        if (epot) epot[s] = ep;
        if (ekin) ekin[s] = kinetic(n, vx, vy, vz, p->mass, th);
    }
    clock_gettime(CLOCK_MONOTONIC, &t1);
    if (loop_seconds)
        *loop_seconds = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
out:
    free(fx); free(fy); free(fz); free(xr); free(yr); free(zr);
    free(rho); free(fp); free(l.off); free(l.idx);
    return builds;
}
