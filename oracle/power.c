/*
 * Oracle power spectrum estimator (test infrastructure only; see orc.h).
 *
 * The paper's observables are the CDM, total-matter, neutrino and CDM x
 * neutrino power spectra (Sec. 3, computed there with nbodykit).  Reading: the
 * auto (cross) power of a mode is Re(delta_a conj delta_b) V / M^2 with the
 * unnormalised forward DFT; modes are binned by the integer part of |n|
 * (n the integer wave vector, bin width the fundamental 2 pi / L), every mode
 * of the full mesh except k = 0 is counted once, k_mean is the mode-weighted
 * mean |k|; optionally each field is divided by the cloud-in-cell window
 * prod_d sinc^2(pi n_d / N).  No shot-noise subtraction.
 */
#include "orc.h"
#include <complex.h>
#include <math.h>
#include <stdlib.h>

typedef double complex cplx;

static long isqrt_l(long v)
{
    long b = (long)floor(sqrt((double)v));
    while (b * b > v) b--;
    while ((b + 1) * (b + 1) <= v) b++;
    return b;
}

static double sinc(double x) { return x == 0 ? 1.0 : sin(x) / x; }

void orc_power(const double *da, const double *db, int n, double box, int nbins, int compensate,
               double *k_mean, double *pk, double *n_modes)
{
    long m = (long)n * n * n;
    cplx *A = malloc(sizeof(cplx) * m), *B = NULL;
    for (long t = 0; t < m; t++) A[t] = da[t];
    orc_fft3d((double *)A, n, -1);
    if (db && db != da) {
        B = malloc(sizeof(cplx) * m);
        for (long t = 0; t < m; t++) B[t] = db[t];
        orc_fft3d((double *)B, n, -1);
    } else {
        B = A;
    }
    for (int b = 0; b < nbins; b++) k_mean[b] = pk[b] = n_modes[b] = 0;
    double V = box * box * box, norm = V / ((double)m * (double)m);
    for (long t = 1; t < m; t++) {
        long k[3] = {t / ((long)n * n), (t / n) % n, t % n};
        long s[3], n2 = 0;
        for (int e = 0; e < 3; e++) { s[e] = k[e] < n / 2 ? k[e] : k[e] - n; n2 += s[e] * s[e]; }
        long b = isqrt_l(n2);
        if (b >= nbins) continue;
        double v = creal(A[t] * conj(B[t])) * norm;
        if (compensate) {
            double w = 1.0;
            for (int e = 0; e < 3; e++) { double sc = sinc(M_PI * s[e] / n); w *= sc * sc; }
            v /= w * w;
        }
        pk[b] += v;
        k_mean[b] += 2.0 * M_PI / box * sqrt((double)n2);
        n_modes[b] += 1.0;
    }
    for (int b = 0; b < nbins; b++)
        if (n_modes[b] > 0) { pk[b] /= n_modes[b]; k_mean[b] /= n_modes[b]; }
    free(A);
    if (B != A) free(B);
}
