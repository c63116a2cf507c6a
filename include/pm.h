/*
 * libpm: particle-mesh step of FastPM with massive-neutrino particles on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Bayer, Banerjee & Feng, "A fast particle-mesh simulation of
 * non-linear cosmological structure formation with massive neutrinos"
 * (arXiv:2007.13394).  CDM particles sit on a lattice; neutrino particles sit
 * on a coarser staggered lattice of sites, N_shell x (2 N_fib + 1) per site,
 * with quasi-randomly sampled Fermi-Dirac speeds (Sec. 2.1).  Each step paints
 * all particles to a mesh with cloud-in-cell weights, solves Poisson's
 * equation with the matter-only source (Sec. 2.2, "Om_pois" eq.) by FFT,
 * reads the force back at the particles and applies FastPM's modified kick and
 * drift, which keep the Zel'dovich trajectory x = q + D(a) s exact (Sec. 2.3).
 *
 * Conventions used by every entry point
 *   - Mesh index (i0, i1, i2), i2 fastest; particle coordinate d lies along
 *     mesh axis d.  Positions are float32 in mesh-cell units, in [0, N).
 *   - Particle arrays are structure-of-arrays: x[d * stride + i].  For the
 *     calls that take a context, stride = P, the particle count of the
 *     configuration (pm_sizes).
 *   - Particle order: segment 0 holds the N_c CDM particles in lattice order
 *     ((i0 * n + i1) * n + i2); segment 1 + s holds neutrino shell s, ordered
 *     by site (row-major) then direction.  Each segment has one particle mass.
 *     This canonical order holds after pm_ic (or pm_reset_order).  Unless
 *     PM_FLAG_NO_SORT is set (or N < 32 or P >= 2^31), pm_step sorts the
 *     particles by 16^3-cell mesh tile and leaves x and p in that order; the
 *     context then tracks each particle's segment (pm_segment_tags) and
 *     carries an attached id array along (pm_attach_ids).  Every call taking
 *     particles expects them in the context's current order.
 *   - Momenta are canonical, p = a^2 dx/dt / H0, in mesh-cell units, so that
 *     dx/da = p / (a^3 E) and dp/da = F / (a^2 E).
 *   - The force is F = -grad phi with lap phi = 1.5 Omega_m delta in mesh
 *     units; masses are normalised to a mean of one unit per cell.
 *   - Mass is accumulated in fixed point: one unit of mass is 2^shift, and a
 *     cell holds at most 2^(63 - shift) units (mean-cell masses) before its
 *     int64 sum wraps.  The device guard flags a cell that reads below
 *     -2^36 quanta: a sum that wrapped into [2^63, 2^64 - 2^36) is reported
 *     as PM_ERR_OVERFLOW; a sum that passed 2^64 is not detected.  (A cell
 *     with no other mass may legitimately hold a few negative quanta: each
 *     particle's last corner takes its quantum minus seven rounded corners.)
 *   - "device" pointers are HIP device memory owned by the caller; "host"
 *     pointers are ordinary host memory owned by the caller.  The library
 *     never allocates device memory: all scratch lives in the caller's
 *     workspace.  All device work is enqueued on the HIP stream passed in
 *     (a hipStream_t; NULL is the null stream).
 *   - Every call returns a pm_status.  Argument errors are detected before
 *     any device work is enqueued.  pm_last_error() describes the most
 *     recent failure on the calling thread.
 */
#ifndef PM_H
#define PM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PM_OK = 0,
    PM_ERR_ARG = -1,      /* invalid argument or configuration */
    PM_ERR_SIZE = -2,     /* workspace too small */
    PM_ERR_DEVICE = -3,   /* a HIP call failed */
    PM_ERR_OVERFLOW = -4, /* a density cell left the fixed-point range */
    PM_ERR_NAN = -5,      /* a particle position or momentum became non-finite, or a
                             cotangent passed to a reverse-mode call is */
    PM_ERR_STATE = -6     /* call not valid for this context */
} pm_status;

/* pm_config.flags */
enum {
    PM_FLAG_NO_FLIP = 1,   /* keep one direction set on every neutrino site */
    PM_FLAG_NO_GUARDS = 2, /* skip the end-of-call device flag check (no host sync) */
    PM_FLAG_NO_SORT = 4,   /* keep particles in segment order (pm_step paints with
                              global atomics and gathers the force: slower) */
    PM_FLAG_LEARNED = 8,   /* reserve the workspace of the learned force correction
                              (pm_learned_*; N a power of two >= 16) */
    PM_FLAG_NU_PSEUDO = 16, /* pseudo-random neutrino velocities, one particle per
                               site (n_shell 1, n_fib 0): initial conditions by
                               pm_ic_pseudo instead of pm_ic */
    PM_FLAG_DEFER_GUARDS = 32 /* check each call's device flags without waiting for
                                 it: the copy is queued at the end of the call and
                                 read by the next guarded call after that call has
                                 queued its own work, or by pm_sync.  The next call
                                 (or pm_sync) returns the error; the failing call
                                 returns PM_OK.  No host wait per call. */
};

/* Simulation parameters (Table 1 of the paper names the counts).  All
 * fields are read by pm_sizes and copied by pm_init. */
typedef struct {
    int32_t n_mesh;   /* N: force mesh cells per side, power of two, 16..2048 */
    int32_t n_cdm;    /* CDM lattice sites per side; power of two, 8..N */
    int32_t n_sites;  /* neutrino sites per side; 0 = no neutrino particles,
                         otherwise a power of two dividing n_cdm */
    int32_t n_shell;  /* Fermi-Dirac speed shells, 1..64 */
    int32_t n_fib;    /* 2 n_fib + 1 directions per shell, 0..1000 */
    int32_t n_nu;     /* neutrino eigenstates in the background, 0..3 */
    int32_t shift;    /* fixed-point shift S, 16..52 */
    int32_t flags;    /* PM_FLAG_* */
    double box;       /* side length, Mpc/h */
    double omega_m;   /* total matter today (CDM + neutrinos) */
    double h;
    double n_s;
    double sigma8;    /* normalises the linear CDM spectrum at z = 0 */
    double T_cmb;     /* K */
    double N_eff;
    double m_nu[3];   /* eigenstate masses, eV (first n_nu used) */
    double a0;        /* initial scale factor of the initial conditions */
} pm_config;

typedef struct pm_ctx pm_ctx;

/* Sizes implied by a configuration.  Any output pointer may be NULL.
 *   n_particles : P = n_cdm^3 + n_sites^3 n_shell (2 n_fib + 1)
 *   n_segments  : 1 + n_shell (1 when n_sites = 0)
 *   workspace   : bytes of device workspace pm_init needs
 * Errors: PM_ERR_ARG for an invalid configuration. */
pm_status pm_sizes(const pm_config *cfg, int64_t *n_particles, int32_t *n_segments,
                   size_t *workspace_bytes);

/* Create a context.  Computes the background, growth and neutrino shell
 * tables on the host (Sec. 2.1, 2.3), uploads FFT tables into the workspace
 * on `stream` and waits for that upload.  workspace: device, at least
 * pm_sizes' bytes, 256-byte aligned, owned by the caller, must outlive the
 * context.  Errors: PM_ERR_ARG, PM_ERR_SIZE, PM_ERR_DEVICE. */
pm_status pm_init(const pm_config *cfg, void *workspace, size_t workspace_bytes, void *stream,
                  pm_ctx **out);

/* Release the host-side context (the workspace is the caller's). */
void pm_free(pm_ctx *ctx);

/* Human-readable description of the last error on this thread. */
const char *pm_last_error(void);

/* Segment table (host outputs, each may be NULL):
 *   offsets[n_segments + 1] particle index ranges, mass[n_segments] particle
 *   masses in mean-cell units (Sec. 2.1 "m_shell" eq.), quantum[n_segments]
 *   = llrint(mass 2^shift). */
pm_status pm_segments(const pm_ctx *ctx, int64_t *offsets, double *mass, int64_t *quantum);

/* Neutrino shell table (host outputs, n_shell entries each, may be NULL):
 * speeds q_shell and mass fractions m_shell (Sec. 2.1 eqs. "q_shell",
 * "m_shell"), edges[n_shell + 1] with equal area under q f(q) ("N_shell" eq.,
 * effective distribution of the "FD_deg" eq. for unequal masses). */
pm_status pm_shells(const pm_ctx *ctx, double *edges, double *q_shell, double *m_shell);

/* Linear growth (Sec. 2.3, "growthDE" eq.): D(a) and G(a) = a^2 E dD/dlna for
 * n host values a[i] >= 1/160.  Host arrays.  Errors: PM_ERR_ARG. */
pm_status pm_growth(const pm_ctx *ctx, int32_t n, const double *a, double *D, double *G);

/* FastPM factors of one KDK call (Sec. 2.3): kick from a_kick0 to a_kick1
 * with the force at a_force, drift from a_force to a_drift1 with the
 * momentum at a_kick1.  Host outputs. */
pm_status pm_kdk_factors(const pm_ctx *ctx, double a_force, double a_kick0, double a_kick1,
                         double a_drift1, double *kick, double *drift);

/* Zel'dovich initial conditions at a0 (Sec. 2.1, 2.2).
 *   white : device float32 [n_cdm]^3 unit Gaussian white noise (the random
 *           numbers of the realisation; the caller draws them)
 *   x, p  : device float32 [3][P] outputs
 * CDM: lattice plus displacement, p = (G/D)(a0) s.  Neutrinos: staggered
 * sites, shells of radius proportional to speed, Fibonacci directions (set
 * reversed on odd sites unless PM_FLAG_NO_FLIP), bulk displacement from the
 * same noise with free-streaming suppression. */
pm_status pm_ic(pm_ctx *ctx, const float *white, float *x, float *p, void *stream);

/* The same initial conditions with pseudo-random thermal velocities, the
 * sampling the paper compares its quasi-random shells with (Sec. 3, the
 * neutrino power spectrum figure): one neutrino per site at the site plus the
 * bulk displacement; speed q = C^-1(u0), C the cumulative of q^2 f~(q) on
 * [0, 30 / min alpha] (tabulated at 4097 points of q, inverted by search and
 * linear interpolation); direction cos(theta) = 2 u1 - 1, phi = 2 pi u2 about
 * mesh axis 2.  u: device float32 [3][n_sites^3] uniforms in [0, 1), drawn by
 * the caller.  Needs PM_FLAG_NU_PSEUDO (PM_ERR_STATE otherwise; pm_ic returns
 * PM_ERR_STATE for such a context). */
pm_status pm_ic_pseudo(pm_ctx *ctx, const float *white, const float *u, float *x, float *p, void *stream);

/* Cloud-in-cell assignment of particles [first, first + count) with one mass
 * quantum, ADDED to the int64 mesh (caller zeroes it).  This is the mass
 * assignment of the particle-mesh method FastPM is built on (Sec. 1 and
 * 2.3); the density it builds is the source of Poisson's equation, to which
 * CDM and neutrino particles both contribute (Sec. 2.2, "Om_pois" eq.).
 *   x      : device float32, coordinate d of particle i at x[d * stride + i],
 *            every value in [0, N)
 *   mesh_q : device int64 [N]^3
 * Corner weights are products of (1 - d, d) per axis in double precision,
 * rounded to nearest integer quanta, the last corner taking the remainder, so
 * each particle adds exactly `quantum` and the result does not depend on the
 * order of the particles. */
pm_status pm_paint_q(pm_ctx *ctx, const float *x, int64_t stride, int64_t first, int64_t count,
                     int64_t quantum, int64_t *mesh_q, void *stream);

/* pm_paint_q over segments [seg_lo, seg_hi) of a [3][P] particle array, each
 * with its own quantum; added to mesh_q (device int64 [N]^3).  Segment 0 is
 * the CDM, segment 1 + s neutrino shell s with the shell's mass fraction
 * (Sec. 2.1, "m_shell" eq.); painting all of them gives the total-matter
 * density of the Poisson source (Sec. 2.2, "Om_pois" eq.).  On a sorting
 * context the particles are tile-sorted into the workspace and painted tile
 * by tile (the same integers as pm_paint_q); otherwise with global atomics.
 * Errors: PM_ERR_ARG for a bad segment range or NULL pointer. */
pm_status pm_paint(pm_ctx *ctx, const float *x, int32_t seg_lo, int32_t seg_hi, int64_t *mesh_q,
                   void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): pm_paint's
 * tile-sorted path, the same integers added to mesh_q, with the sort's
 * scratch (per-key counts and offsets, the scan's block sums, the sorted
 * position records) in a fixed device array of the library instead of the
 * context's workspace.  The array is about 50 MiB per device, held until the
 * process ends; every call on a device uses that device's one array (the
 * counts are cleared by a kernel at the start of each call), so calls that
 * overlap on one device race and must be ordered by the caller (one stream,
 * or events).  The call allocates nothing and issues no memset.
 * Limits: N <= PM_STATIC_MAX_MESH and P <= PM_STATIC_MAX_PARTICLES, else
 * PM_ERR_SIZE; a context that cannot tile-sort (N < 32) gives PM_ERR_STATE;
 * PM_ERR_ARG for a bad segment range or NULL pointer. */
#define PM_STATIC_MAX_MESH 512
#define PM_STATIC_MAX_PARTICLES 3145728
pm_status pm_paint_static(pm_ctx *ctx, const float *x, int32_t seg_lo, int32_t seg_hi, int64_t *mesh_q,
                          void *stream);

/* Forward 3D real-to-complex transform, unnormalised, X_k = sum_j x_j
 * exp(-2 pi i j.k / N).  real: device float32 [N]^3; out: device interleaved
 * complex64 [N][N][N/2 + 1].  Uses the workspace. */
pm_status pm_fft_r2c(pm_ctx *ctx, const float *real, float *out, void *stream);

/* Inverse 3D complex-to-real transform, unnormalised (returns N^3 times the
 * field whose forward transform is `spec`).  spec: device complex64
 * [N][N][N/2 + 1] (planes k2 = 0 and N/2 must be Hermitian); real: device
 * float32 [N]^3. */
pm_status pm_fft_c2r(pm_ctx *ctx, const float *spec, float *real, void *stream);

/* Force meshes from a fixed-point density: delta = Q 2^-shift - 1, F_d(k) =
 * 1.5 Omega_m i k_d / k^2 delta(k) (zero at k = 0 and on the Nyquist plane of
 * component d): Poisson's equation with the matter source of Sec. 2.2
 * ("Om_pois" eq., Omega_m = Omega_c0 + Omega_nu0) solved by FFT, and minus
 * its gradient.  mesh_q: device int64 [N]^3; out: device float32 [3][N]^3.
 * mesh_q is consumed completely before out is written, so it may lie inside
 * out's memory (a caller short of memory can build the density there). */
pm_status pm_force_mesh(pm_ctx *ctx, const int64_t *mesh_q, float *out, void *stream);

/* Force on every particle at positions x: paint all segments, solve, read
 * back with cloud-in-cell weights (the force of the particle-mesh step,
 * Sec. 2.2 "Om_pois" eq. and Sec. 2.3).  x: device [3][P] in the context's
 * current order; acc: device [3][P], same order.  Errors: PM_ERR_OVERFLOW as
 * for pm_step (unless PM_FLAG_NO_GUARDS). */
pm_status pm_force(pm_ctx *ctx, const float *x, float *acc, void *stream);

/* One call of the kick-drift-kick loop (Sec. 2.3): force at x (time
 * a_force), p += K F with K the kick from a_kick0 to a_kick1, then
 * x += D p with D the drift from a_force to a_drift1 (momentum at a_kick1),
 * wrapped into [0, N).  A run of n steps is n + 1 calls with merged kicks;
 * the last call has a_kick1 = a_drift1 = a_force.  x, p: device [3][P],
 * updated in place.  Errors: PM_ERR_NAN if a result is non-finite,
 * PM_ERR_OVERFLOW if a density cell overflowed (checked at the end of the
 * call, which then waits for the stream, unless PM_FLAG_NO_GUARDS; with
 * PM_FLAG_DEFER_GUARDS reported by the next guarded call or pm_sync).
 * On a sorting context the readout also counts the tile keys of the
 * positions it writes; the next call on the same x array sorts with those
 * counts and checks them after its scatter.  The check (a 4-byte copy) is
 * read back just before the readout, the paint and the force solve having
 * been queued behind it: if the caller changed x in between, the sort is
 * redone from a fresh count and the paint and the solve are queued again.
 * With PM_FLAG_NO_GUARDS every call counts afresh instead. */
pm_status pm_step(pm_ctx *ctx, float *x, float *p, double a_force, double a_kick0, double a_kick1,
                  double a_drift1, void *stream);

/* Binned power spectrum of the particles (Sec. 3): painted density contrast
 * of segments [a_lo, a_hi) crossed with that of [b_lo, b_hi) (auto power if
 * the ranges are equal).  Bins are [b, b+1) in units of 2 pi / L by |k|; k = 0
 * is excluded; each mode of the full mesh counts once.  compensate != 0
 * divides each field by the cloud-in-cell window prod_d sinc^2(pi n_d / N).
 * Host outputs k_mean (h/Mpc), pk ((Mpc/h)^3), n_modes, each nbins long,
 * nbins in 1..2048.  Waits for the stream before returning. */
pm_status pm_power(pm_ctx *ctx, const float *x, int32_t a_lo, int32_t a_hi, int32_t b_lo,
                   int32_t b_hi, int32_t nbins, int32_t compensate, double *k_mean, double *pk,
                   double *n_modes, void *stream);

/* The same estimator on two given density-contrast meshes da, db (device
 * float32 [N]^3, equal for an auto spectrum): cross power Re(da(k) db(k)*).
 * Used to compare runs painted on one mesh (spectra ratios, r(k)). */
pm_status pm_power_mesh(pm_ctx *ctx, const float *da, const float *db, int32_t nbins, int32_t compensate,
                        double *k_mean, double *pk, double *n_modes, void *stream);

/* Attach a caller-owned device array of P uint32 ids (or NULL to detach)
 * that pm_step permutes together with the particles; its initial content is
 * the caller's (for instance 0..P-1 in canonical order).  Errors: PM_ERR_STATE
 * when the configuration cannot sort (N < 32 or P >= 2^31). */
pm_status pm_attach_ids(pm_ctx *ctx, uint32_t *ids);

/* Segment of every particle in the context's current order: tags is a
 * device uint8 array of P entries, written on `stream`. */
pm_status pm_segment_tags(pm_ctx *ctx, uint8_t *tags, void *stream);

/* Declare that the particle arrays passed from now on are in canonical
 * segment order again (as written by pm_ic). */
pm_status pm_reset_order(pm_ctx *ctx);

/* With PM_FLAG_DEFER_GUARDS: wait for the last guarded call's device flags
 * and return its status (PM_ERR_NAN, PM_ERR_OVERFLOW or PM_OK); PM_OK when
 * no check is pending or without the flag.  Waits only for that call's end. */
pm_status pm_sync(pm_ctx *ctx);

/* Launch trace, for measuring kernel durations on the stream they run on.
 * pm_trace_begin makes every later kernel launch of this context record a
 * HIP event before and after it on the launch stream (no host waits are
 * added); at most `capacity` launches are recorded, later ones are not.
 * pm_trace_end stops recording, waits for the recorded launches, and writes
 * up to `max` records: kind[i] (see pm_kernel_name) and ms[i], the elapsed
 * time between the two events of launch i, in launch order; *count receives
 * the number recorded.  Host arrays.  Errors: PM_ERR_ARG, PM_ERR_STATE (no
 * trace in progress), PM_ERR_DEVICE. */
pm_status pm_trace_begin(pm_ctx *ctx, int32_t capacity);
pm_status pm_trace_end(pm_ctx *ctx, int32_t max, int32_t *kind, float *ms, int32_t *count);

/* Name of a kernel kind reported by pm_trace_end ("paint", "axis0", ...). */
const char *pm_kernel_name(int32_t kind);

/* ---- Reverse mode (reconstruction of the initial modes, the application the
 * paper's introduction and conclusions point to).  The differentiated model is
 * the step above with every particle depositing its exact segment mass with
 * cloud-in-cell weights (the fixed-point mesh agrees with it to 2^-shift per
 * cell; the rounding has zero derivative).  The derivative of a weight at a
 * cell face is the right derivative.  All arrays are device float32, SoA
 * [3][P] for particle quantities, in the context's particle order; cotangent
 * outputs are accumulated (+=) unless stated.  The reverse mode needs the
 * particles to keep their order between the forward steps and the reverse
 * pass: configure with PM_FLAG_NO_SORT (pm_step_vjp returns PM_ERR_STATE
 * otherwise). */

/* delta = sum_j m_j W(x_j, c) - 1 (the painted density contrast, from the
 * fixed-point mesh) into a dense float32 [N]^3 mesh. */
pm_status pm_density(pm_ctx *ctx, const float *x, float *delta, void *stream);

/* xbar_j += m_j sum_c dmesh(c) dW(x_j, c)/dx_j: the transpose of pm_density
 * for a cotangent mesh dmesh (dense float32 [N]^3). */
pm_status pm_density_vjp(pm_ctx *ctx, const float *x, const float *dmesh, float *xbar, void *stream);

/* xbar += (d acc / d x)^T g, acc the force of pm_force at x and g [3][P] its
 * cotangent: the readout-derivative term plus the paint-derivative term
 * through the transpose of the gradient of the inverse Laplacian (which is
 * minus itself).  Uses the workspace mesh regions; where the configuration
 * tile-sorts (N >= 32, P < 2^31) it also sorts x and g into the workspace's
 * record arrays and paints the density and the cotangent by tile (the
 * caller's arrays keep their order).  The cotangent is painted in int64 fixed
 * point (a power-of-two unit set by max |g|), so the result is the same on
 * every run and for any order of the particles.
 * PM_ERR_NAN if any value of g is NaN or infinite; xbar is then untouched. */
pm_status pm_force_vjp(pm_ctx *ctx, const float *x, const float *g, float *xbar, void *stream);

/* Reverse mode of pm_step taken at positions x (the checkpoint: positions
 * before the step) with the same four scale factors.  On entry xbar, pbar
 * hold the cotangents of the positions and momenta after the step; on exit,
 * those of the positions and momenta before it (updated in place):
 * pbar += drift xbar, then xbar += kick (dF/dx)^T pbar.  PM_ERR_NAN if a
 * resulting pbar value is NaN or infinite (pbar then holds the drift term
 * and xbar is untouched). */
pm_status pm_step_vjp(pm_ctx *ctx, const float *x, double a_force, double a_kick0, double a_kick1,
                      double a_drift1, float *xbar, float *pbar, void *stream);

/* Transpose of pm_ic with respect to the white noise: wbar (float32
 * [n_cdm]^3, overwritten) = (d(x, p)/d white)^T (xbar, pbar).  The initial
 * conditions are linear in the white noise: each displacement field is
 * F^-1 diag(M) F white, whose transpose is F^-1 diag(conj M) F.  Cotangents in
 * canonical order (PM_ERR_STATE after a sorted step). */
pm_status pm_ic_vjp(pm_ctx *ctx, const float *xbar, const float *pbar, float *wbar, void *stream);

/* ---- Learned force correction (an addition to the method for the
 * coarse-mesh use the paper's introduction motivates; configure with
 * PM_FLAG_LEARNED).  Model: the potential spectrum -1.5 Omega_m0 delta(k) / k^2
 * is multiplied by a radial filter g(k, a) = 1 + MLP(|k| / k_Nyq, a) (two
 * inputs, three hidden layers of 96 SiLU units, tabulated at 256 radial bins
 * and interpolated linearly); a periodic 3^3 CNN (1 -> 16 -> 16 -> 1
 * channels, SiLU; BF16 activations and weights, FP32 accumulation) maps the
 * painted density contrast to a potential correction, phi = phi_f + cnn(delta);
 * the force is minus its spectral gradient, read out with cloud-in-cell
 * weights.
 * With the output layers at zero it is the plain force.  theta: device
 * float32 [pm_net_nparam()], the flat parameter array (MLP W0 [96][2], b0,
 * W1 [96][96], b1, W2 [96][96], b2, W3 [96], b3; conv W [co][ci][27] and b for
 * the three layers, taps (t0 3 + t1) 3 + t2 at offsets t_e - 1). */
int32_t pm_net_nparam(void);

/* Learned force on every particle at x (a: scale factor for the filter and
 * D(a)).  acc: device [3][P]. */
pm_status pm_learned_force(pm_ctx *ctx, const float *theta, double a, const float *x, float *acc, void *stream);

/* pm_step with the learned force: same factors and semantics, including the
 * tile sort (particles come back in sorted order) unless PM_FLAG_NO_SORT. */
pm_status pm_learned_step(pm_ctx *ctx, const float *theta, float *x, float *p, double a_force, double a_kick0,
                          double a_kick1, double a_drift1, void *stream);

/* Force-matching loss L = sum |acc - target|^2 / sum |target|^2 of the learned
 * force at x against target [3][P] (device), written to *loss (host; the
 * call waits for the stream), and dL/dtheta accumulated into dtheta (device
 * float32, or NULL for the loss alone) by the hand-written reverse mode. */
pm_status pm_learned_loss(pm_ctx *ctx, const float *theta, double a, const float *x, const float *target,
                          double *loss, float *dtheta, void *stream);

/* The radial filter table g(k_b, a) = 1 + MLP(kt_b, a) at the NET_NB = 256 bins
 * kt_b = b sqrt(3) / 255 (|k| in units of the Nyquist wavenumber), as the
 * learned force applies it.  theta, table: device float32 [pm_net_nparam()],
 * [256]. */
pm_status pm_net_table(const float *theta, double a, float *table, void *stream);

/* dtheta += sum_b tbar[b] d table[b] / d theta (reverse mode of
 * pm_net_table).  tbar: device float64 [256]; dtheta: device float32. */
pm_status pm_net_table_vjp(const float *theta, double a, const double *tbar, float *dtheta, void *stream);

/* One Adam step (bias-corrected, step t >= 1) on n FP32 master weights theta
 * with moments m, v and gradient g, all device arrays. */
pm_status pm_adam(float *theta, float *m, float *v, const float *g, int64_t n, double lr, double beta1,
                  double beta2, double eps, int32_t t, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PM_H */
