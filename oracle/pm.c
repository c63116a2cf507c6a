/*
 * Oracle particle-mesh force and kick-drift-kick step
 * (test infrastructure only; see orc.h).
 *
 * FastPM evolves particles with a particle-mesh force (Sec. 1 and Sec. 2.3):
 * mass is assigned to the mesh with cloud-in-cell weights, Poisson's equation
 * lap phi = 1.5 Omega_m0 delta (matter-only source, Sec. 2.2 "Om_pois") is
 * solved in Fourier space, the force F = -grad phi is interpolated back with
 * the same weights, and the kick and drift use the modified factors of
 * Sec. 2.3.  Readings: the exact spectral kernel F_d(k) = 1.5 Omega_m0 i k_d /
 * k^2 delta(k) with no window deconvolution, zero at k = 0 and on the Nyquist
 * plane of component d; the density mesh is accumulated in fixed point with
 * quantum 2^-S per mass unit, corner weights evaluated in double precision in
 * the fixed order below and the last corner taking the remainder, so that each
 * particle deposits exactly its quantised mass.
 */
#include "orc.h"
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static void cic(const double *x, long P, long i, int n, long cell[3][2], double w[3][2])
{
    for (int d = 0; d < 3; d++) {
        double u = x[d * P + i];
        double f = floor(u);
        double dd = u - f;
        long i0 = (long)f;
        w[d][0] = 1.0 - dd;
        w[d][1] = dd;
        cell[d][0] = ((i0 % n) + n) % n;
        cell[d][1] = (((i0 + 1) % n) + n) % n;
    }
}

/* Add particles [off, off+cnt) of mass quantum Qm to the int64 mesh. */
void orc_paint_q(const double *x, long P, long off, long cnt, int64_t Qm, int n, int64_t *mesh)
{
    #pragma omp parallel for schedule(static)
    for (long i = off; i < off + cnt; i++) {
        long cell[3][2];
        double w[3][2];
        cic(x, P, i, n, cell, w);
        int64_t acc = 0;
        int t = 0;
        for (int c0 = 0; c0 < 2; c0++)
            for (int c1 = 0; c1 < 2; c1++)
                for (int c2 = 0; c2 < 2; c2++, t++) {
                    int64_t q;
                    if (t < 7) {
                        double wq = ((w[0][c0] * w[1][c1]) * w[2][c2]) * (double)Qm;
                        q = llrint(wq);
                        acc += q;
                    } else {
                        q = Qm - acc;
                    }
                    long idx = (cell[0][c0] * n + cell[1][c1]) * n + cell[2][c2];
                    #pragma omp atomic
                    mesh[idx] += q;
                }
    }
}

/* Same assignment with unquantised double weights (used for analysis). */
void orc_paint_d(const double *x, long P, long off, long cnt, double m, int n, double *mesh)
{
    #pragma omp parallel for schedule(static)
    for (long i = off; i < off + cnt; i++) {
        long cell[3][2];
        double w[3][2];
        cic(x, P, i, n, cell, w);
        for (int c0 = 0; c0 < 2; c0++)
            for (int c1 = 0; c1 < 2; c1++)
                for (int c2 = 0; c2 < 2; c2++) {
                    long idx = (cell[0][c0] * n + cell[1][c1]) * n + cell[2][c2];
                    double v = ((w[0][c0] * w[1][c1]) * w[2][c2]) * m;
                    #pragma omp atomic
                    mesh[idx] += v;
                }
    }
}

/* F[d][cell], d = 0..2, from the density contrast on an n^3 mesh. */
void orc_force_mesh_from_delta(const double *delta, int n, double omega_m, double *F)
{
    long m = (long)n * n * n;
    cplx *dk = malloc(sizeof(cplx) * m), *f = malloc(sizeof(cplx) * m);
    for (long t = 0; t < m; t++) dk[t] = delta[t];
    orc_fft3d((double *)dk, n, -1);
    for (int d = 0; d < 3; d++) {
        for (long t = 0; t < m; t++) {
            long k[3] = {t / ((long)n * n), (t / n) % n, t % n};
            double kv[3], k2 = 0;
            for (int e = 0; e < 3; e++) {
                long s = k[e] <= n / 2 ? k[e] : k[e] - n;
                kv[e] = 2.0 * M_PI * s / n;
                k2 += kv[e] * kv[e];
            }
            if (k2 == 0 || k[d] == n / 2) { f[t] = 0; continue; }
            f[t] = 1.5 * omega_m * I * kv[d] / k2 * dk[t];
        }
        orc_fft3d((double *)f, n, +1);
        for (long t = 0; t < m; t++) F[d * m + t] = creal(f[t]) / (double)m;
    }
    free(dk);
    free(f);
}

/* delta = Q 2^-S - 1 from the fixed-point mesh, then the force mesh. */
void orc_force_mesh(const int64_t *q, int n, int S, double omega_m, double *F)
{
    long m = (long)n * n * n;
    double *delta = malloc(sizeof(double) * m);
    for (long t = 0; t < m; t++) delta[t] = ldexp((double)q[t], -S) - 1.0;
    orc_force_mesh_from_delta(delta, n, omega_m, F);
    free(delta);
}

void orc_readout(const double *F, int n, const double *x, long P, double *acc)
{
    long m = (long)n * n * n;
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < P; i++) {
        long cell[3][2];
        double w[3][2];
        cic(x, P, i, n, cell, w);
        double s[3] = {0, 0, 0};
        for (int c0 = 0; c0 < 2; c0++)
            for (int c1 = 0; c1 < 2; c1++)
                for (int c2 = 0; c2 < 2; c2++) {
                    long idx = (cell[0][c0] * n + cell[1][c1]) * n + cell[2][c2];
                    double w8 = (w[0][c0] * w[1][c1]) * w[2][c2];
                    for (int d = 0; d < 3; d++) s[d] += w8 * F[d * m + idx];
                }
        for (int d = 0; d < 3; d++) acc[d * P + i] = s[d];
    }
}

/* Force on every particle at positions x (all segments painted). */
int orc_force(const orc_sim *s, const double *x, double *acc)
{
    long off[66];
    double mass[65];
    int64_t q[65];
    int nseg = orc_segments(s, off, mass, q);
    if (nseg < 1) return -1;
    long P = orc_num_particles(s, NULL, NULL);
    int n = s->n_mesh;
    long m = (long)n * n * n;
    int64_t *mesh = calloc(m, sizeof(int64_t));
    double *F = malloc(sizeof(double) * 3 * m);
    for (int g = 0; g < nseg; g++) orc_paint_q(x, P, off[g], off[g + 1] - off[g], q[g], n, mesh);
    orc_force_mesh(mesh, n, s->shift, s->cosmo.omega_m, F);
    orc_readout(F, n, x, P, acc);
    free(mesh);
    free(F);
    return 0;
}

/* One call of the kick-drift-kick loop: force at x, p += kick F, x += drift p
 * (periodic).  acc_out (optional) receives the force. */
int orc_step(const orc_sim *s, double *x, double *p, double kick, double drift, double *acc_out)
{
    long P = orc_num_particles(s, NULL, NULL);
    double *acc = acc_out ? acc_out : malloc(sizeof(double) * 3 * P);
    if (orc_force(s, x, acc)) { if (!acc_out) free(acc); return -1; }
    double n = s->n_mesh;
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < 3 * P; i++) {
        p[i] += kick * acc[i];
        double u = fmod(x[i] + drift * p[i], n);
        if (u < 0) u += n;
        if (u >= n) u -= n;
        x[i] = u;
    }
    if (!acc_out) free(acc);
    return 0;
}
