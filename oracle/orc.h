/*
 * Oracle for the particle-mesh step of FastPM with massive-neutrino particles
 * (Bayer, Banerjee & Feng, arXiv:2007.13394).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 CPU implementation of
 * what the GPU path computes, written from the paper so that the GPU results
 * can be checked against it.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product library never does.
 * It shares no code with the GPU library (its own FFT, cosmology, sampling).
 *
 * Conventions
 *   mesh[i0][i1][i2], i2 fastest; particle coordinate d lives on mesh axis d.
 *   positions/momenta are in mesh-cell units, SoA: x[d*P + i].
 *   forward DFT  X_k = sum_j x_j exp(-2 pi i j k / N), no scaling;
 *   inverse DFT  x_j = sum_k X_k exp(+2 pi i j k / N), no scaling (callers
 *   divide by N^3 where a normalised inverse is meant).
 *   complex arrays are interleaved (re, im) doubles.
 *
 * Pins: tests/test_oracle_*.py check every function against closed forms,
 * the paper's printed values, independent quadrature or brute force, and the
 * reverse mode (adj.c, orc_ic_vjp) against central finite differences of the
 * forward model.
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------- FFT (fft.c) ---------------- */
void orc_fft1d(double *c, long n, int sign);
void orc_fft3d(double *c, long n, int sign);
void orc_dft3d_naive(const double *in, double *out, long n, int sign);
void orc_rfft3d(const double *real, double *half, long n);
void orc_irfft3d(const double *half, double *real, long n);

/* ---------------- background + growth (cosmo.c) ---------------- */
typedef struct {
    /* inputs */
    double omega_m;   /* total matter today, CDM + neutrinos */
    double h;
    double T_cmb;     /* K */
    double N_eff;
    int    n_nu;      /* number of massive eigenstates in the sum (0..3) */
    double m_nu[3];   /* eV */
    /* derived by orc_cosmo_init */
    double omega_g;   /* photons today */
    double omega_nu0; /* M_nu / (93.14 h^2) */
    double omega_c;   /* omega_m - omega_nu0 */
    double omega_L;   /* flat closure with the exact neutrino density today */
    double gamma_nu;  /* T_nu / T_gamma */
    double kT_nu;     /* k_B T_nu0 in eV */
    double a_ini;     /* start of the growth integration */
} orc_cosmo;

int    orc_cosmo_init(orc_cosmo *c);
double orc_fd_F(double y);
double orc_fd_dF(double y);
double orc_omega_nu_E2(const orc_cosmo *c, double a);
double orc_E(const orc_cosmo *c, double a);
double orc_dlnE_dlna(const orc_cosmo *c, double a);
int    orc_growth(const orc_cosmo *c, int n, const double *a, double *D, double *G, double dlna_max);
int    orc_kdk_factors(const orc_cosmo *c, int n, const double *a_force, const double *a_k0,
                       const double *a_k1, const double *a_d1, double *kick, double *drift);

/* ---------------- neutrino sampling (nu.c) ---------------- */
double orc_fd_tilde(int n_nu, const double *alpha, double q);
double orc_integrate(double (*f)(double, void *), void *ctx, double a, double b, double tol);
int    orc_fd_shells(int n_nu, const double *alpha, int n_shell, double q_max,
                     double *edges, double *q_shell, double *m_shell);
void   orc_fibonacci(int n_fib, double *dirs);
double orc_fd_qinv(int n_nu, const double *alpha, double u);

/* ---------------- simulation set-up (ic.c) ---------------- */
typedef struct {
    orc_cosmo cosmo;
    double box;        /* Mpc/h */
    int    n_mesh;     /* force mesh cells per side */
    int    n_cdm;      /* CDM lattice per side */
    int    n_sites;    /* neutrino sites per side (0 = no neutrino particles) */
    int    n_shell;
    int    n_fib;
    double sigma8;
    double n_s;
    double a0;
    int    flip_odd;   /* reverse the direction set on sites with odd i+j+k */
    int    shift;      /* fixed-point shift S */
} orc_sim;

long   orc_num_particles(const orc_sim *s, long *n_cdm, long *n_nu);
int    orc_segments(const orc_sim *s, long *seg_off /*n_seg+1*/, double *seg_mass, int64_t *seg_q);
double orc_bbks_T(double q);
double orc_pk_unnorm(const orc_sim *s, double k);
double orc_sigma_R(const orc_sim *s, double amp, double R);
double orc_pk_amplitude(const orc_sim *s);
int    orc_ic(const orc_sim *s, const float *white, double *x, double *p, double *disp_cdm, double *disp_nu);
int    orc_ic_w64(const orc_sim *s, const double *white, double *x, double *p);
/* Pseudo-random neutrino velocities (one particle per site: n_shell 1,
 * n_fib 0): u [3][n_sites^3] uniforms in [0, 1) give the speed q = C^-1(u0)
 * and the direction cos(theta) = 2 u1 - 1, phi = 2 pi u2 about mesh axis 2. */
int    orc_ic_pseudo(const orc_sim *s, const float *white, const double *u, double *x, double *p);
int    orc_ic_vjp(const orc_sim *s, const double *xbar, const double *pbar, double *wbar);

/* ---------------- PM force and step (pm.c) ---------------- */
void orc_paint_q(const double *x, long P, long off, long cnt, int64_t Qm, int n, int64_t *mesh);
void orc_paint_d(const double *x, long P, long off, long cnt, double m, int n, double *mesh);
void orc_force_mesh(const int64_t *q, int n, int S, double omega_m, double *F);
void orc_force_mesh_from_delta(const double *delta, int n, double omega_m, double *F);
void orc_readout(const double *F, int n, const double *x, long P, double *acc);
int  orc_force(const orc_sim *s, const double *x, double *acc);
int  orc_step(const orc_sim *s, double *x, double *p, double kick, double drift, double *acc_out);

/* ---------------- reverse mode (adj.c; ic.c for orc_ic_vjp) ---------------- */
int  orc_density_cont(const orc_sim *s, const double *x, double *delta);
int  orc_force_cont(const orc_sim *s, const double *x, double *acc);
int  orc_step_cont(const orc_sim *s, double *x, double *p, double kick, double drift);
int  orc_force_vjp(const orc_sim *s, const double *x, const double *g, double *xbar);
int  orc_step_vjp(const orc_sim *s, const double *x, double kick, double drift, double *xbar, double *pbar);
int  orc_density_vjp(const orc_sim *s, const double *x, const double *dmesh, double *xbar);

/* ---------------- learned force correction (net.c) ---------------- */
#define NET_H 96      /* MLP hidden width */
#define NET_NB 256    /* radial table bins */
#define NET_C 16      /* CNN channels */
enum {
    NET_W0 = 0, NET_B0 = NET_W0 + NET_H * 2, NET_W1 = NET_B0 + NET_H, NET_B1 = NET_W1 + NET_H * NET_H,
    NET_W2 = NET_B1 + NET_H, NET_B2 = NET_W2 + NET_H * NET_H, NET_W3 = NET_B2 + NET_H, NET_B3 = NET_W3 + NET_H,
    NET_C1W = NET_B3 + 1, NET_C1B = NET_C1W + NET_C * 27, NET_C2W = NET_C1B + NET_C,
    NET_C2B = NET_C2W + NET_C * NET_C * 27, NET_C3W = NET_C2B + NET_C, NET_C3B = NET_C3W + NET_C * 27,
    NET_NPARAM = NET_C3B + 1
};
double orc_net_kt(int b);
void   orc_net_table(const double *th, double a, double *table);
void   orc_net_table_vjp(const double *th, double a, const double *tbar, double *dth);
void   orc_conv3(const double *in, int ci_n, const double *W, const double *bias, int co_n, int n, double *out);
void   orc_conv3_vjp(const double *in, int ci_n, const double *W, int co_n, int n, const double *dout, double *din,
                     double *dW, double *db);
int    orc_learned_force(const orc_sim *s, const double *th, double a, const double *x, double *acc);
int    orc_learned_loss(const orc_sim *s, const double *th, double a, const double *x, const double *target,
                        double *loss, double *dth);

/* ---------------- power spectrum (power.c) ---------------- */
void orc_power(const double *da, const double *db, int n, double box, int nbins, int compensate,
               double *k_mean, double *pk, double *n_modes);

#ifdef __cplusplus
}
#endif
#endif
