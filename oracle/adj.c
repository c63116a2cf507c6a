/*
 * Oracle reverse mode of the particle-mesh step (test infrastructure only;
 * see orc.h).
 *
 * Differentiable model.  The step of pm.c paints each particle's fixed-point
 * mass quantum; that rounding has zero derivative almost everywhere, so the
 * model differentiated here paints the exact segment mass with the same
 * cloud-in-cell weights (the fixed-point mesh equals it to 2^-S per cell):
 *   rho(c) = sum_j m_j W(x_j, c),  delta = rho - 1,
 *   Phi_d = L_d delta,  L_d = F^-1 diag(1.5 Omega_m0 i k_d / k^2) F / M
 *           (zero at k = 0 and on the Nyquist plane of component d),
 *   acc_{i,d} = sum_c W(x_i, c) Phi_d(c),
 *   p' = p + K acc(x),  x' = wrap(x + D p').
 * W(x, c) = prod_e w_e with w_e = 1 - (u_e - floor u_e) on cell floor(u_e) and
 * u_e - floor u_e on the next cell; its derivative along e is -1 / +1 times the
 * other two factors (the right derivative at cell faces).  The wrap has unit
 * derivative.  L_d is a real convolution with an odd kernel, so L_d^T = -L_d.
 *
 * Reverse mode of one step (cotangents xbar, pbar of x', p'):
 *   pbar += D xbar;  g = K pbar;
 *   xbar_i += sum_d g_{i,d} sum_c dW(x_i, c)/dx_i Phi_d(c)          (readout)
 *   psi = sum_d L_d^T G_d = -sum_d L_d G_d,  G_d(c) = sum_i g_{i,d} W(x_i, c)
 *   xbar_j += m_j sum_c psi(c) dW(x_j, c)/dx_j                        (paint)
 * (the initial-condition transpose is orc_ic_vjp in ic.c).
 */
#include "orc.h"
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static void cic_w(const double *x, long P, long i, int n, long cell[3][2], double w[3][2])
{
    for (int d = 0; d < 3; d++) {
        double u = x[d * P + i];
        double f = floor(u);
        long i0 = (long)f;
        w[d][1] = u - f;
        w[d][0] = 1.0 - w[d][1];
        cell[d][0] = ((i0 % n) + n) % n;
        cell[d][1] = (((i0 + 1) % n) + n) % n;
    }
}

/* Segment mass of every particle (mean density 1 per cell). */
static double *particle_masses(const orc_sim *s, long P)
{
    long off[66];
    double mass[65];
    int64_t q[65];
    int nseg = orc_segments(s, off, mass, q);
    if (nseg < 1) return NULL;
    double *m = malloc(sizeof(double) * P);
    for (int g = 0; g < nseg; g++)
        for (long i = off[g]; i < off[g + 1]; i++) m[i] = mass[g];
    return m;
}

/* delta(c) = sum_j m_j W(x_j, c) - 1 with unquantised masses. */
int orc_density_cont(const orc_sim *s, const double *x, double *delta)
{
    long P = orc_num_particles(s, NULL, NULL);
    int n = s->n_mesh;
    long M = (long)n * n * n;
    long off[66];
    double mass[65];
    int64_t q[65];
    int nseg = orc_segments(s, off, mass, q);
    if (nseg < 1) return -1;
    memset(delta, 0, sizeof(double) * M);
    for (int g = 0; g < nseg; g++) orc_paint_d(x, P, off[g], off[g + 1] - off[g], mass[g], n, delta);
    for (long t = 0; t < M; t++) delta[t] -= 1.0;
    return 0;
}

/* Force with the unquantised paint. */
int orc_force_cont(const orc_sim *s, const double *x, double *acc)
{
    long P = orc_num_particles(s, NULL, NULL);
    int n = s->n_mesh;
    long M = (long)n * n * n;
    double *delta = malloc(sizeof(double) * M), *F = malloc(sizeof(double) * 3 * M);
    int rc = orc_density_cont(s, x, delta);
    if (rc == 0) {
        orc_force_mesh_from_delta(delta, n, s->cosmo.omega_m, F);
        orc_readout(F, n, x, P, acc);
    }
    free(delta);
    free(F);
    return rc;
}

/* One step of the differentiable model (same factors as orc_step). */
int orc_step_cont(const orc_sim *s, double *x, double *p, double kick, double drift)
{
    long P = orc_num_particles(s, NULL, NULL);
    double *acc = malloc(sizeof(double) * 3 * P);
    if (orc_force_cont(s, x, acc)) { free(acc); return -1; }
    double n = s->n_mesh;
    for (long i = 0; i < 3 * P; i++) {
        p[i] += kick * acc[i];
        double u = fmod(x[i] + drift * p[i], n);
        if (u < 0) u += n;
        if (u >= n) u -= n;
        x[i] = u;
    }
    free(acc);
    return 0;
}

/* xbar_{i,e} += sum_d coef_i g_{i,d} sum_c dW(x_i, c)/dx_e mesh_d(c) for nd
 * meshes (g = NULL: one mesh, weight coef_i). */
static void readout_grad(const double *mesh, int nd, int n, const double *x, long P, const double *g,
                         const double *coef, double *xbar)
{
    long M = (long)n * n * n;
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < P; i++) {
        long cell[3][2];
        double w[3][2];
        cic_w(x, P, i, n, cell, w);
        double out[3] = {0, 0, 0};
        for (int c0 = 0; c0 < 2; c0++)
            for (int c1 = 0; c1 < 2; c1++)
                for (int c2 = 0; c2 < 2; c2++) {
                    long idx = (cell[0][c0] * n + cell[1][c1]) * n + cell[2][c2];
                    double v = 0;
                    for (int d = 0; d < nd; d++) v += (g ? g[d * P + i] : 1.0) * mesh[d * M + idx];
                    const double s0 = c0 ? 1.0 : -1.0, s1 = c1 ? 1.0 : -1.0, s2 = c2 ? 1.0 : -1.0;
                    out[0] += s0 * w[1][c1] * w[2][c2] * v;
                    out[1] += w[0][c0] * s1 * w[2][c2] * v;
                    out[2] += w[0][c0] * w[1][c1] * s2 * v;
                }
        double cf = coef ? coef[i] : 1.0;
        for (int e = 0; e < 3; e++) xbar[e * P + i] += cf * out[e];
    }
}

/* psi = sum_d L_d^T G_d = -sum_d L_d G_d. */
static void green_transpose(const double *G, int n, double omega_m, double *psi)
{
    long M = (long)n * n * n;
    cplx *acc = calloc(M, sizeof(cplx)), *f = malloc(sizeof(cplx) * M);
    for (int d = 0; d < 3; d++) {
        for (long t = 0; t < M; t++) f[t] = G[d * M + t];
        orc_fft3d((double *)f, n, -1);
        for (long t = 0; t < M; t++) {
            long k[3] = {t / ((long)n * n), (t / n) % n, t % n};
            double kv[3], k2 = 0;
            for (int e = 0; e < 3; e++) {
                long sm = k[e] <= n / 2 ? k[e] : k[e] - n;
                kv[e] = 2.0 * M_PI * sm / n;
                k2 += kv[e] * kv[e];
            }
            if (k2 == 0 || k[d] == n / 2) continue;
            acc[t] -= 1.5 * omega_m * I * kv[d] / k2 * f[t];
        }
    }
    orc_fft3d((double *)acc, n, +1);
    for (long t = 0; t < M; t++) psi[t] = creal(acc[t]) / (double)M;
    free(acc);
    free(f);
}

/* xbar += (d acc / d x)^T g for the force of the differentiable model. */
int orc_force_vjp(const orc_sim *s, const double *x, const double *g, double *xbar)
{
    long P = orc_num_particles(s, NULL, NULL);
    int n = s->n_mesh;
    long M = (long)n * n * n;
    double *delta = malloc(sizeof(double) * M), *F = malloc(sizeof(double) * 3 * M);
    if (orc_density_cont(s, x, delta)) { free(delta); free(F); return -1; }
    orc_force_mesh_from_delta(delta, n, s->cosmo.omega_m, F);
    readout_grad(F, 3, n, x, P, g, NULL, xbar);
    /* paint the cotangents with the readout weights, then the Green transpose */
    memset(F, 0, sizeof(double) * 3 * M);
    for (int d = 0; d < 3; d++) {
        double *Gd = F + d * M;
        for (long i = 0; i < P; i++) {
            long cell[3][2];
            double w[3][2];
            cic_w(x, P, i, n, cell, w);
            for (int c0 = 0; c0 < 2; c0++)
                for (int c1 = 0; c1 < 2; c1++)
                    for (int c2 = 0; c2 < 2; c2++)
                        Gd[(cell[0][c0] * n + cell[1][c1]) * n + cell[2][c2]] +=
                            ((w[0][c0] * w[1][c1]) * w[2][c2]) * g[d * P + i];
        }
    }
    green_transpose(F, n, s->cosmo.omega_m, delta);
    double *m = particle_masses(s, P);
    readout_grad(delta, 1, n, x, P, NULL, m, xbar);
    free(m);
    free(delta);
    free(F);
    return 0;
}

/* Reverse mode of one step at checkpoint x (positions before the step):
 * (xbar, pbar) are the cotangents of (x', p') on entry and of (x, p) on exit. */
int orc_step_vjp(const orc_sim *s, const double *x, double kick, double drift, double *xbar, double *pbar)
{
    long P = orc_num_particles(s, NULL, NULL);
    double *g = malloc(sizeof(double) * 3 * P);
    for (long i = 0; i < 3 * P; i++) {
        pbar[i] += drift * xbar[i];
        g[i] = kick * pbar[i];
    }
    int rc = orc_force_vjp(s, x, g, xbar);
    free(g);
    return rc;
}

/* xbar_j += m_j sum_c dmesh(c) dW(x_j, c)/dx_j: the transpose of the density
 * delta(x) for a cotangent mesh dmesh. */
int orc_density_vjp(const orc_sim *s, const double *x, const double *dmesh, double *xbar)
{
    long P = orc_num_particles(s, NULL, NULL);
    double *m = particle_masses(s, P);
    if (!m) return -1;
    readout_grad(dmesh, 1, s->n_mesh, x, P, NULL, m, xbar);
    free(m);
    return 0;
}
