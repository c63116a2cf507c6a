/*
 * Oracle of the learned force correction (test infrastructure only; see
 * orc.h).  Plain FP64 loops, forward and reverse mode.
 *
 * The correction is an addition of this library to the method (the paper's
 * introduction motivates learned and differentiable extensions of fast
 * particle-mesh codes; it prescribes no network).  Definition:
 *   radial filter: g(k, a) = 1 + h(kt, a), kt = |k| / k_Nyq (k_Nyq = pi per
 *     cell), h an MLP 2 -> 96 -> 96 -> 96 -> 1 with SiLU activations,
 *     tabulated at NET_NB bins kt_b = b sqrt(3) / (NET_NB - 1) and linearly
 *     interpolated in between;
 *   filtered potential: phi_f = F^-1 [ g(k, a) (-1.5 Omega_m0 / k^2) F delta ] / M
 *     (zero at k = 0), delta the painted density contrast;
 *   CNN on the density contrast delta: periodic 3^3 cross-correlations
 *     1 -> 16 (SiLU) -> 16 (SiLU) -> 1, out[co](v) = b[co] + sum_{ci, t}
 *     W[co][ci][t] in[ci](v + o(t)), tap t = (t0 3 + t1) 3 + t2 with offsets
 *     o_e = t_e - 1 along mesh axes (0, 1, 2);
 *   potential phi = phi_f + cnn(delta); force F_d = F^-1 [ -i k_d F phi ] / M
 *     (zero on the Nyquist plane of d), read out with cloud-in-cell weights.
 * The CNN sees the local mass distribution, not the potential: its output
 * then changes the force at wavenumber k in proportion to k^2 relative to
 * the Newtonian force, so it cannot rescale the large-scale force.
 * With the last layers of the MLP and of the CNN at zero this is the plain
 * force of pm.c.  Parameters are one flat array (offsets in orc.h).
 */
#include "orc.h"
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static double silu(double z) { return z / (1.0 + exp(-z)); }
static double dsilu(double z)
{
    double s = 1.0 / (1.0 + exp(-z));
    return s + z * s * (1.0 - s);
}

double orc_net_kt(int b) { return b * sqrt(3.0) / (NET_NB - 1); }

/* MLP value h(kt, a); z (optional) receives the three hidden pre-activations. */
static double mlp(const double *th, double kt, double a, double z[3][NET_H])
{
    double in[2] = {kt, a}, h0[NET_H], h1[NET_H], h2[NET_H];
    for (int j = 0; j < NET_H; j++) {
        double s = th[NET_B0 + j];
        for (int i = 0; i < 2; i++) s += th[NET_W0 + j * 2 + i] * in[i];
        if (z) z[0][j] = s;
        h0[j] = silu(s);
    }
    for (int j = 0; j < NET_H; j++) {
        double s = th[NET_B1 + j];
        for (int i = 0; i < NET_H; i++) s += th[NET_W1 + j * NET_H + i] * h0[i];
        if (z) z[1][j] = s;
        h1[j] = silu(s);
    }
    for (int j = 0; j < NET_H; j++) {
        double s = th[NET_B2 + j];
        for (int i = 0; i < NET_H; i++) s += th[NET_W2 + j * NET_H + i] * h1[i];
        if (z) z[2][j] = s;
        h2[j] = silu(s);
    }
    double s = th[NET_B3];
    for (int i = 0; i < NET_H; i++) s += th[NET_W3 + i] * h2[i];
    return s;
}

void orc_net_table(const double *th, double a, double *table)
{
    for (int b = 0; b < NET_NB; b++) table[b] = 1.0 + mlp(th, orc_net_kt(b), a, NULL);
}

/* dth += sum_b tbar[b] d table[b] / d th. */
void orc_net_table_vjp(const double *th, double a, const double *tbar, double *dth)
{
    for (int b = 0; b < NET_NB; b++) {
        if (tbar[b] == 0) continue;
        double z[3][NET_H], in[2] = {orc_net_kt(b), a};
        mlp(th, in[0], a, z);
        double h[3][NET_H];
        for (int l = 0; l < 3; l++)
            for (int j = 0; j < NET_H; j++) h[l][j] = silu(z[l][j]);
        double g = tbar[b];
        double d2[NET_H], d1[NET_H], d0[NET_H];
        dth[NET_B3] += g;
        for (int i = 0; i < NET_H; i++) {
            dth[NET_W3 + i] += g * h[2][i];
            d2[i] = g * th[NET_W3 + i] * dsilu(z[2][i]);
        }
        for (int i = 0; i < NET_H; i++) d1[i] = 0;
        for (int j = 0; j < NET_H; j++) {
            dth[NET_B2 + j] += d2[j];
            for (int i = 0; i < NET_H; i++) {
                dth[NET_W2 + j * NET_H + i] += d2[j] * h[1][i];
                d1[i] += d2[j] * th[NET_W2 + j * NET_H + i];
            }
        }
        for (int i = 0; i < NET_H; i++) d1[i] *= dsilu(z[1][i]);
        for (int i = 0; i < NET_H; i++) d0[i] = 0;
        for (int j = 0; j < NET_H; j++) {
            dth[NET_B1 + j] += d1[j];
            for (int i = 0; i < NET_H; i++) {
                dth[NET_W1 + j * NET_H + i] += d1[j] * h[0][i];
                d0[i] += d1[j] * th[NET_W1 + j * NET_H + i];
            }
        }
        for (int j = 0; j < NET_H; j++) {
            double dz = d0[j] * dsilu(z[0][j]);
            dth[NET_B0 + j] += dz;
            for (int i = 0; i < 2; i++) dth[NET_W0 + j * 2 + i] += dz * in[i];
        }
    }
}

static long wrapi(long i, long n) { return ((i % n) + n) % n; }

/* out[co][v] = b[co] + sum_{ci,t} W[co][ci][t] in[ci][v + o(t)]. */
void orc_conv3(const double *in, int ci_n, const double *W, const double *bias, int co_n, int n, double *out)
{
    long M = (long)n * n * n;
    #pragma omp parallel for schedule(static)
    for (long v = 0; v < M; v++) {
        long i0 = v / ((long)n * n), i1 = (v / n) % n, i2 = v % n;
        for (int co = 0; co < co_n; co++) {
            double s = bias[co];
            for (int ci = 0; ci < ci_n; ci++)
                for (int t = 0; t < 27; t++) {
                    long u = (wrapi(i0 + t / 9 - 1, n) * n + wrapi(i1 + (t / 3) % 3 - 1, n)) * n +
                             wrapi(i2 + t % 3 - 1, n);
                    s += W[(co * ci_n + ci) * 27 + t] * in[ci * M + u];
                }
            out[co * M + v] = s;
        }
    }
}

/* Reverse mode: din += W^T dout (shifted back), dW += in (x) dout, db += sum dout. */
void orc_conv3_vjp(const double *in, int ci_n, const double *W, int co_n, int n, const double *dout, double *din,
                   double *dW, double *db)
{
    long M = (long)n * n * n;
    for (int co = 0; co < co_n; co++) {
        double s = 0;
        for (long v = 0; v < M; v++) s += dout[co * M + v];
        db[co] += s;
    }
    for (long v = 0; v < M; v++) {
        long i0 = v / ((long)n * n), i1 = (v / n) % n, i2 = v % n;
        for (int t = 0; t < 27; t++) {
            long u = (wrapi(i0 + t / 9 - 1, n) * n + wrapi(i1 + (t / 3) % 3 - 1, n)) * n + wrapi(i2 + t % 3 - 1, n);
            for (int co = 0; co < co_n; co++) {
                double d = dout[co * M + v];
                if (d == 0) continue;
                for (int ci = 0; ci < ci_n; ci++) {
                    if (din) din[ci * M + u] += W[(co * ci_n + ci) * 27 + t] * d;
                    dW[(co * ci_n + ci) * 27 + t] += in[ci * M + u] * d;
                }
            }
        }
    }
}

static void kvec(long t, int n, double kv[3], int nyq[3])
{
    long k[3] = {t / ((long)n * n), (t / n) % n, t % n};
    for (int e = 0; e < 3; e++) {
        long s = k[e] <= n / 2 ? k[e] : k[e] - n;
        kv[e] = 2.0 * M_PI * s / n;
        nyq[e] = (k[e] == n / 2);
    }
}

/* Table value at kt by linear interpolation; *b0, *f receive the bin and weight. */
static double interp(const double *table, double kt, int *b0, double *f)
{
    double tt = kt / orc_net_kt(1);
    int b = (int)floor(tt);
    if (b > NET_NB - 2) b = NET_NB - 2;
    double w = tt - b;
    *b0 = b;
    *f = w;
    return (1.0 - w) * table[b] + w * table[b + 1];
}

typedef struct {
    int n;
    long M;
    double omega_m;
    double table[NET_NB];
    double *delta; /* density contrast (the CNN input) */
    cplx *dk;      /* F delta */
    double *phif;  /* filtered potential */
    double *z1, *a1, *z2, *a2, *dphi;  /* CNN pre-activations / activations / output */
    double *F;     /* 3 force meshes */
} fwd_state;

static void free_state(fwd_state *st)
{
    free(st->delta); free(st->dk); free(st->phif); free(st->z1); free(st->a1); free(st->z2); free(st->a2); free(st->dphi);
    free(st->F);
}

static int forward(const orc_sim *s, const double *th, double a, const double *x, fwd_state *st)
{
    int n = s->n_mesh;
    long M = (long)n * n * n, P = orc_num_particles(s, NULL, NULL);
    st->n = n;
    st->M = M;
    st->omega_m = s->cosmo.omega_m;
    orc_net_table(th, a, st->table);
    st->delta = malloc(sizeof(double) * M);
    if (orc_density_cont(s, x, st->delta)) { free(st->delta); st->delta = NULL; return -1; }
    st->dk = malloc(sizeof(cplx) * M);
    for (long t = 0; t < M; t++) st->dk[t] = st->delta[t];
    orc_fft3d((double *)st->dk, n, -1);
    cplx *f = malloc(sizeof(cplx) * M);
    for (long t = 0; t < M; t++) {
        double kv[3];
        int nyq[3];
        kvec(t, n, kv, nyq);
        double k2 = kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2];
        if (k2 == 0) { f[t] = 0; continue; }
        int b0;
        double w;
        double g = interp(st->table, sqrt(k2) / M_PI, &b0, &w);
        f[t] = g * (-1.5 * st->omega_m / k2) * st->dk[t];
    }
    orc_fft3d((double *)f, n, +1);
    st->phif = malloc(sizeof(double) * M);
    for (long t = 0; t < M; t++) st->phif[t] = creal(f[t]) / (double)M;
    /* CNN on delta */
    st->z1 = malloc(sizeof(double) * NET_C * M);
    st->a1 = malloc(sizeof(double) * NET_C * M);
    st->z2 = malloc(sizeof(double) * NET_C * M);
    st->a2 = malloc(sizeof(double) * NET_C * M);
    st->dphi = malloc(sizeof(double) * M);
    orc_conv3(st->delta, 1, th + NET_C1W, th + NET_C1B, NET_C, n, st->z1);
    for (long t = 0; t < NET_C * M; t++) st->a1[t] = silu(st->z1[t]);
    orc_conv3(st->a1, NET_C, th + NET_C2W, th + NET_C2B, NET_C, n, st->z2);
    for (long t = 0; t < NET_C * M; t++) st->a2[t] = silu(st->z2[t]);
    orc_conv3(st->a2, NET_C, th + NET_C3W, th + NET_C3B, 1, n, st->dphi);
    /* force */
    for (long t = 0; t < M; t++) f[t] = st->phif[t] + st->dphi[t];
    orc_fft3d((double *)f, n, -1);
    st->F = malloc(sizeof(double) * 3 * M);
    cplx *g = malloc(sizeof(cplx) * M);
    for (int d = 0; d < 3; d++) {
        for (long t = 0; t < M; t++) {
            double kv[3];
            int nyq[3];
            kvec(t, n, kv, nyq);
            g[t] = nyq[d] ? 0 : -I * kv[d] * f[t];
        }
        orc_fft3d((double *)g, n, +1);
        for (long t = 0; t < M; t++) st->F[d * M + t] = creal(g[t]) / (double)M;
    }
    free(f);
    free(g);
    (void)P;
    return 0;
}

int orc_learned_force(const orc_sim *s, const double *th, double a, const double *x, double *acc)
{
    fwd_state st;
    memset(&st, 0, sizeof(st));
    if (forward(s, th, a, x, &st)) return -1;
    long P = orc_num_particles(s, NULL, NULL);
    orc_readout(st.F, s->n_mesh, x, P, acc);
    free_state(&st);
    return 0;
}

/* L = sum |acc - target|^2 / sum |target|^2 and dth += dL/dth. */
int orc_learned_loss(const orc_sim *s, const double *th, double a, const double *x, const double *target,
                     double *loss, double *dth)
{
    fwd_state st;
    memset(&st, 0, sizeof(st));
    if (forward(s, th, a, x, &st)) return -1;
    int n = st.n;
    long M = st.M, P = orc_num_particles(s, NULL, NULL);
    double *acc = malloc(sizeof(double) * 3 * P);
    orc_readout(st.F, n, x, P, acc);
    double num = 0, den = 0;
    for (long i = 0; i < 3 * P; i++) {
        num += (acc[i] - target[i]) * (acc[i] - target[i]);
        den += target[i] * target[i];
    }
    *loss = num / den;
    if (!dth) { free(acc); free_state(&st); return 0; }
    /* readout transpose: Fbar_d(c) = sum_i abar_{i,d} W(x_i, c) */
    double *Fbar = calloc(3 * M, sizeof(double));
    for (long i = 0; i < P; i++) {
        double w[3][2];
        long cell[3][2];
        for (int d = 0; d < 3; d++) {
            double u = x[d * P + i], fl = floor(u);
            long i0 = (long)fl;
            w[d][1] = u - fl;
            w[d][0] = 1.0 - w[d][1];
            cell[d][0] = wrapi(i0, n);
            cell[d][1] = wrapi(i0 + 1, n);
        }
        for (int c0 = 0; c0 < 2; c0++)
            for (int c1 = 0; c1 < 2; c1++)
                for (int c2 = 0; c2 < 2; c2++) {
                    long idx = (cell[0][c0] * n + cell[1][c1]) * n + cell[2][c2];
                    double ww = (w[0][c0] * w[1][c1]) * w[2][c2];
                    for (int d = 0; d < 3; d++) Fbar[d * M + idx] += ww * 2.0 * (acc[d * P + i] - target[d * P + i]) / den;
                }
    }
    /* gradient transpose: F_d = F^-1 (-i k_d) F phi / M, a real odd convolution:
     * phibar = -sum_d F^-1 (-i k_d) F Fbar_d / M */
    cplx *pb = calloc(M, sizeof(cplx)), *h = malloc(sizeof(cplx) * M);
    for (int d = 0; d < 3; d++) {
        for (long t = 0; t < M; t++) h[t] = Fbar[d * M + t];
        orc_fft3d((double *)h, n, -1);
        for (long t = 0; t < M; t++) {
            double kv[3];
            int nyq[3];
            kvec(t, n, kv, nyq);
            if (!nyq[d]) pb[t] -= -I * kv[d] * h[t];
        }
    }
    orc_fft3d((double *)pb, n, +1);
    double *phibar = malloc(sizeof(double) * M);
    for (long t = 0; t < M; t++) phibar[t] = creal(pb[t]) / (double)M;
    free(Fbar);
    /* phi = phif + cnn(delta); delta does not depend on the parameters */
    double *d2 = malloc(sizeof(double) * NET_C * M), *d1 = malloc(sizeof(double) * NET_C * M);
    double *ddelta = calloc(M, sizeof(double));   /* unused: delta is not a parameter */
    memset(d2, 0, sizeof(double) * NET_C * M);
    orc_conv3_vjp(st.a2, NET_C, th + NET_C3W, 1, n, phibar, d2, dth + NET_C3W, dth + NET_C3B);
    for (long t = 0; t < NET_C * M; t++) d2[t] *= dsilu(st.z2[t]);
    memset(d1, 0, sizeof(double) * NET_C * M);
    orc_conv3_vjp(st.a1, NET_C, th + NET_C2W, NET_C, n, d2, d1, dth + NET_C2W, dth + NET_C2B);
    for (long t = 0; t < NET_C * M; t++) d1[t] *= dsilu(st.z1[t]);
    orc_conv3_vjp(st.delta, 1, th + NET_C1W, NET_C, n, d1, ddelta, dth + NET_C1W, dth + NET_C1B);
    /* phif = F^-1 [g G F delta] / M:  dL/dg(k) = Re[G_k dk_k conj(F phibar)_k] / M
     * per mode of the full spectrum, distributed to the two table bins */
    for (long t = 0; t < M; t++) h[t] = phibar[t];
    orc_fft3d((double *)h, n, -1);
    double tbar[NET_NB];
    memset(tbar, 0, sizeof(tbar));
    for (long t = 0; t < M; t++) {
        double kv[3];
        int nyq[3];
        kvec(t, n, kv, nyq);
        double k2 = kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2];
        if (k2 == 0) continue;
        int b0;
        double w;
        interp(st.table, sqrt(k2) / M_PI, &b0, &w);
        double dg = creal((-1.5 * st.omega_m / k2) * st.dk[t] * conj(h[t])) / (double)M;
        tbar[b0] += (1.0 - w) * dg;
        tbar[b0 + 1] += w * dg;
    }
    orc_net_table_vjp(th, a, tbar, dth);
    free(pb); free(h); free(phibar); free(d2); free(d1); free(ddelta); free(acc);
    free_state(&st);
    return 0;
}
