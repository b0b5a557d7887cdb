/*
 * FP64 oracle of the learned descriptor-MLP potential -- TEST
 * INFRASTRUCTURE ONLY.  The model and its rounding points are stated in
 * mlp.h.  Everything here is the plain definition: sums in atom and
 * neighbour order, the chain rule written out, no blocking or reuse.
 */
#include "mlp.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NI OR_MLP_IN
#define NH OR_MLP_HID
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + NH * NI)
#define OFF_W2 (OFF_B1 + NH)
#define OFF_B2 (OFF_W2 + NH * NH)
#define OFF_W3 (OFF_B2 + NH)
#define OFF_B3 (OFF_W3 + NH)

double or_bf16_round(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (double)f; /* inf / nan */
    u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double rnd(double v, int bf16) { return bf16 ? or_bf16_round(v) : v; }

static double sigmoid(double a) { return 1.0 / (1.0 + exp(-a)); }

/* d silu / da = s (1 + a (1 - s)), s = sigmoid(a) */
static double dsilu(double a)
{
    double s = sigmoid(a);
    return s * (1.0 + a * (1.0 - s));
}

/* g_k(r) and, if dg is not NULL, dg_k/dr, for r < rc */
static void basis(const or_mlp_t *m, double r, double *g, double *dg)
{
    double fc = 0.5 * (cos(M_PI * r / m->rc) + 1.0);
    double dfc = -0.5 * (M_PI / m->rc) * sin(M_PI * r / m->rc);
    double w2 = m->width * m->width;
    for (int k = 0; k < NI; ++k) {
        double t = r - (m->mu0 + k * m->dmu);
        double e = exp(-t * t / (2.0 * w2));
        g[k] = e * fc;
        if (dg) dg[k] = e * (dfc - fc * t / w2);
    }
}

/* r_ij and R = x_i - x_j under the minimum image */
static double pair(const double L[3], const double *x, const double *y,
                   const double *z, int64_t i, int64_t j, double R[3])
{
    R[0] = -or_minimg(x[i], x[j], L[0]);
    R[1] = -or_minimg(y[i], y[j], L[1]);
    R[2] = -or_minimg(z[i], z[j], L[2]);
    return sqrt((R[0] * R[0] + R[1] * R[1]) + R[2] * R[2]);
}

void or_mlp_descriptors(int64_t n, const double L[3], const double *x,
                        const double *y, const double *z,
                        const int64_t *offsets, const int32_t *idx,
                        const or_mlp_t *m, double *G)
{
    double R[3], g[NI];
    for (int64_t i = 0; i < n; ++i) {
        double *Gi = G + i * NI;
        for (int k = 0; k < NI; ++k) Gi[k] = 0.0;
        for (int64_t q = offsets[i]; q < offsets[i + 1]; ++q) {
            double r = pair(L, x, y, z, i, idx[q], R);
            if (!(r < m->rc)) continue;
            basis(m, r, g, NULL);
            for (int k = 0; k < NI; ++k) Gi[k] += g[k];
        }
    }
}

/* Forward pass of one atom; keeps what the backward passes need. */
typedef struct {
    double x[NI], a1[NH], h1[NH], a2[NH], h2[NH], E;
} fwd_t;

static void forward(const or_mlp_t *m, const double *p, const double *G,
                    int bf16, fwd_t *f)
{
    for (int k = 0; k < NI; ++k) f->x[k] = rnd((G[k] - m->mean[k]) * m->inv_std[k], bf16);
    for (int u = 0; u < NH; ++u) {
        double s = p[OFF_B1 + u];
        for (int k = 0; k < NI; ++k) s += p[OFF_W1 + u * NI + k] * f->x[k];
        f->a1[u] = s;
        f->h1[u] = rnd(s * sigmoid(s), bf16);
    }
    for (int u = 0; u < NH; ++u) {
        double s = p[OFF_B2 + u];
        for (int v = 0; v < NH; ++v) s += p[OFF_W2 + u * NH + v] * f->h1[v];
        f->a2[u] = s;
        f->h2[u] = s * sigmoid(s);
    }
    double E = p[OFF_B3];
    for (int u = 0; u < NH; ++u) E += p[OFF_W3 + u] * f->h2[u];
    f->E = E;
}

void or_mlp_energy(int64_t n, const double *G, const or_mlp_t *m,
                   const double *p, int32_t bf16, double *e_atom,
                   double *dEdG)
{
    fwd_t f;
    double d2[NH], d1[NH];
    for (int64_t i = 0; i < n; ++i) {
        forward(m, p, G + i * NI, bf16, &f);
        e_atom[i] = f.E;
        if (!dEdG) continue;
        /* dE/da2 = w3 * silu'(a2); dE/da1 = (W2^T dE/da2) * silu'(a1);
         * dE/dG = (W1^T dE/da1) * inv_std */
        for (int u = 0; u < NH; ++u) d2[u] = rnd(p[OFF_W3 + u] * dsilu(f.a2[u]), bf16);
        for (int v = 0; v < NH; ++v) {
            double s = 0.0;
            for (int u = 0; u < NH; ++u) s += p[OFF_W2 + u * NH + v] * d2[u];
            d1[v] = rnd(s * dsilu(f.a1[v]), bf16);
        }
        for (int k = 0; k < NI; ++k) {
            double s = 0.0;
            for (int u = 0; u < NH; ++u) s += p[OFF_W1 + u * NI + k] * d1[u];
            dEdG[i * NI + k] = s * m->inv_std[k];
        }
    }
}

void or_mlp_forces(int64_t n, const double L[3], const double *x,
                   const double *y, const double *z, const int64_t *offsets,
                   const int32_t *idx, const or_mlp_t *m, const double *dEdG,
                   double *fx, double *fy, double *fz, double *w6)
{
    double R[3], g[NI], dg[NI];
    if (w6)
        for (int a = 0; a < 6; ++a) w6[a] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double f[3] = {0.0, 0.0, 0.0};
        for (int64_t q = offsets[i]; q < offsets[i + 1]; ++q) {
            int64_t j = idx[q];
            double r = pair(L, x, y, z, i, j, R);
            if (!(r < m->rc)) continue;
            basis(m, r, g, dg);
            /* s_ij = dE/dr_ij: r_ij enters G_i and G_j alike */
            double s = 0.0;
            for (int k = 0; k < NI; ++k) s += (dEdG[i * NI + k] + dEdG[j * NI + k]) * dg[k];
            for (int a = 0; a < 3; ++a) f[a] -= s * R[a] / r;
            if (w6) {
                w6[0] -= 0.5 * s * R[0] * R[0] / r;
                w6[1] -= 0.5 * s * R[1] * R[1] / r;
                w6[2] -= 0.5 * s * R[2] * R[2] / r;
                w6[3] -= 0.5 * s * R[0] * R[1] / r;
                w6[4] -= 0.5 * s * R[0] * R[2] / r;
                w6[5] -= 0.5 * s * R[1] * R[2] / r;
            }
        }
        fx[i] = f[0];
        fy[i] = f[1];
        fz[i] = f[2];
    }
}

double or_mlp_loss_grad(int64_t n, const double *G, const double *target,
                        const or_mlp_t *m, const double *p, int32_t bf16,
                        double *grad)
{
    fwd_t f;
    double d2[NH], d2r[NH], d1[NH], d1r[NH];
    double loss = 0.0;
    if (grad) memset(grad, 0, sizeof(double) * OR_MLP_NPARAM);
    for (int64_t i = 0; i < n; ++i) {
        forward(m, p, G + i * NI, bf16, &f);
        double err = f.E - target[i];
        loss += err * err;
        if (!grad) continue;
        double gE = 2.0 * err / (double)n; /* dLoss/dE_i */
        grad[OFF_B3] += gE;
        for (int u = 0; u < NH; ++u) {
            grad[OFF_W3 + u] += gE * f.h2[u];
            d2[u] = gE * p[OFF_W3 + u] * dsilu(f.a2[u]);
            d2r[u] = rnd(d2[u], bf16);
            grad[OFF_B2 + u] += d2[u];
            for (int v = 0; v < NH; ++v) grad[OFF_W2 + u * NH + v] += d2r[u] * f.h1[v];
        }
        for (int v = 0; v < NH; ++v) {
            double s = 0.0;
            for (int u = 0; u < NH; ++u) s += p[OFF_W2 + u * NH + v] * d2r[u];
            d1[v] = s * dsilu(f.a1[v]);
            d1r[v] = rnd(d1[v], bf16);
            grad[OFF_B1 + v] += d1[v];
            for (int k = 0; k < NI; ++k) grad[OFF_W1 + v * NI + k] += d1r[v] * f.x[k];
        }
    }
    return loss / (double)n;
}

/* ---- training trajectories ---- */

static double temperature(int64_t n, const double *vx, const double *vy,
                          const double *vz, double mass, double kB,
                          double e_unit)
{
    double s2 = 0.0;
    for (int64_t i = 0; i < n; ++i) s2 += (vx[i] * vx[i] + vy[i] * vy[i]) + vz[i] * vz[i];
    return mass * e_unit * s2 / ((double)(3 * n - 3) * kB);
}

int64_t or_eam_samples(int64_t n, const double L[3], double *x, double *y,
                       double *z, double *vx, double *vy, double *vz,
                       const or_md_params_t *p, double T_kelvin, double kB,
                       double e_unit, int64_t equil_steps,
                       int64_t rescale_every, int64_t n_samples,
                       int64_t sample_every, double *pos, double *e_atom,
                       double *forces)
{
    int64_t builds = 0;
    for (int64_t done = 0; done < equil_steps;) {
        int64_t k = equil_steps - done < rescale_every ? equil_steps - done : rescale_every;
        int64_t b = or_md_run(n, L, x, y, z, vx, vy, vz, p, k, NULL, NULL, NULL);
        if (b < 0) return -1;
        builds += b;
        double T = temperature(n, vx, vy, vz, p->mass, kB, e_unit);
        double s = T > 0.0 ? sqrt(T_kelvin / T) : 1.0;
        for (int64_t i = 0; i < n; ++i) {
            vx[i] *= s;
            vy[i] *= s;
            vz[i] *= s;
        }
        done += k;
    }
    int64_t cap = 256 * n;
    int64_t *off = malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *idx = malloc(sizeof(int32_t) * (size_t)cap);
    double *buf = malloc(sizeof(double) * (size_t)(8 * n));
    if (!off || !idx || !buf) {
        free(off);
        free(idx);
        free(buf);
        return -1;
    }
    double *rho = buf, *fp = buf + n, *fx = buf + 2 * n, *fy = buf + 3 * n, *fz = buf + 4 * n;
    double *wx = buf + 5 * n, *wy = buf + 6 * n, *wz = buf + 7 * n;
    int64_t rc = builds;
    for (int64_t s = 0; s < n_samples; ++s) {
        int64_t b = or_md_run(n, L, x, y, z, vx, vy, vz, p, sample_every, NULL, NULL, NULL);
        if (b < 0) {
            rc = -1;
            break;
        }
        rc += b;
        memcpy(wx, x, sizeof(double) * (size_t)n);
        memcpy(wy, y, sizeof(double) * (size_t)n);
        memcpy(wz, z, sizeof(double) * (size_t)n);
        or_wrap(n, L, wx, wy, wz);
        if (or_neighbors_brute(n, L, p->r_list, wx, wy, wz, off, idx, cap) > cap) {
            rc = -1;
            break;
        }
        double ev[8];
        or_forces_eam(n, L, wx, wy, wz, off, idx, &p->fs, rho, fp, fx, fy, fz, e_atom + s * n, ev);
        for (int64_t i = 0; i < n; ++i) {
            double *q = pos + (s * n + i) * 3;
            q[0] = wx[i];
            q[1] = wy[i];
            q[2] = wz[i];
            if (forces) {
                double *g = forces + (s * n + i) * 3;
                g[0] = fx[i];
                g[1] = fy[i];
                g[2] = fz[i];
            }
        }
    }
    free(off);
    free(idx);
    free(buf);
    return rc;
}
