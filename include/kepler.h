/*
 * kepler.h -- C ABI of the MI355X (gfx950) Keplerian radial-velocity library.
 *
 * The library evaluates, for a batch of planetary-system models, the radial
 * velocity of a star perturbed by n_pl planets on independent Keplerian
 * orbits and the chi-square of each model against one set of observations,
 * following Ford (2008), "Parallel Algorithm for Solving Kepler's Equation on
 * Graphics Processing Units" (arXiv:0812.2976):
 *
 *   mean anomaly   M_ijk = 2 pi frac((t_k - t0) / P_ij) + M0_ij        Sec. 2.1 Eq. 4, Sec. 4.2 Eq. 6
 *   Kepler         M = E - e sin E, solved by Danby's quartic iteration Sec. 4.3, Eq. 1
 *   velocity       v_ijk = K [cos(omega + f) + e cos omega]             Sec. 2.1 Eq. 3 (standard form)
 *   planet sum     model_ik = sum_j v_ijk + gamma_i                     Sec. 2.1 Eq. 2
 *   chi-square     chi2_i = sum_k (model_ik - v_k)^2 / (sigma_k^2 + s_i^2)   Sec. 2.2 Eq. 5
 *
 * Conventions that the paper leaves open and this library fixes:
 *   - M0 enters with a plus sign (Eq. 4; Eq. 6 prints a minus) and the epoch
 *     t0 is an argument (the paper uses t0 = 0).
 *   - omega is the argument of pericentre and K the usual semi-amplitude; the
 *     printed Eq. 3 mixes conventions and is read as the standard velocity.
 *   - s_i is one jitter per system (Eq. 5 writes sigma_j); gamma_i is an
 *     optional per-system velocity offset.  Both default to 0 (NULL pointer).
 *
 * Memory.  Every array pointer is a DEVICE pointer owned by the caller; the
 * library never frees or retains one beyond the call (ragged plans keep the
 * pointers they were built with, see below).  Arrays are binary64, densely
 * packed, naturally aligned.
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the default
 * stream).  The batch calls enqueue their kernels on it and return without
 * waiting for them; they allocate nothing and never synchronise.
 *
 * Errors.  Argument and shape errors detected on the host return a non-zero
 * kep_status before anything is launched and set a message readable with
 * kep_last_error().  A launch failure returns KEP_ERR_LAUNCH.  Data outside
 * the model's domain is NOT an error: e outside [0, 1), P <= 0, a non-finite
 * parameter, t, v or sigma, sigma < 0 or sigma^2 + s^2 = 0 make that system's
 * chi-square (and gradient, and model velocities) NaN, without affecting any
 * other system.  Accuracy is stated for e <= 0.99 (the paper's range, Sec. 4.3).
 *
 * Precision (kep_prec):
 *   KEP_FP64  plain binary64 everywhere: IEEE-rounded quotient (t - t0)/P,
 *             Danby iteration with a fixed 30 steps by default, binary64 sums.
 *   KEP_MIXED the paper's mixed precision (Sec. 5.1): the orbital phase
 *             (t - t0)/P reduced modulo one orbit is computed in binary64,
 *             Kepler's equation, the velocity and the planet sum in binary32
 *             (compensated, Sec. 4.4), chi-square accumulated in binary32 with
 *             Kahan compensation and finished in binary64.
 */
#ifndef KEPLER_MI355X_H
#define KEPLER_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KEP_MAX_PL 8          /* planets per system accepted by every entry point */
#define KEP_ABI_VERSION 1

typedef enum kep_status {
    KEP_OK = 0,
    KEP_ERR_ARG = 1,          /* null pointer, negative size, bad enum or option */
    KEP_ERR_SHAPE = 2,        /* sizes inconsistent with each other (n_pl, CSR offsets) */
    KEP_ERR_DEVICE = 3,       /* no usable HIP device or a HIP runtime call failed */
    KEP_ERR_LAUNCH = 4,       /* a kernel launch was rejected */
    KEP_ERR_UNSUPPORTED = 5   /* valid request the library does not implement */
} kep_status;

typedef enum kep_prec {
    KEP_FP64 = 0,
    KEP_MIXED = 1
} kep_prec;

/* Observations shared by every system (Sec. 4.1): times t [d], velocities v
   [m/s] and uncertainties sigma [m/s], each of length n_obs >= 0; t0 is the
   epoch of the mean anomaly. */
typedef struct kep_obs {
    const double *t, *v, *sigma;
    int64_t n_obs;
    double t0;
} kep_obs;

/* Model parameters (Sec. 4.1: n_sys x n_pl x 5 values).  Each of P [d],
   K [m/s], e, omega [rad], M0 [rad] is a plane of n_pl * n_sys values laid out
   [n_pl][n_sys] (system index fastest, so consecutive systems are adjacent in
   memory).  offset (gamma, m/s) and jitter (s, m/s) are [n_sys] or NULL.
   1 <= n_pl <= KEP_MAX_PL, n_sys >= 0. */
typedef struct kep_params {
    const double *P, *K, *e, *omega, *M0;
    const double *offset, *jitter;
    int64_t n_sys, n_pl;
} kep_params;

/* Options; pass NULL for the defaults.  A zero field means "default".
   fixed_iter  > 0: exactly this many Danby iterations for every solve.
               = 0: KEP_FP64 uses 30 (the plain kernel); KEP_MIXED uses the
                    eccentricity schedule (2 iterations for e <= 0.8525, 3 up to
                    0.975, 4 up to 0.9955, 5 up to 0.999, then a convergence
                    test), derived offline for a 1e-9 rad worst-case error.
                    Every KEP_MIXED path starts a planet (or a kepler_solve
                    pair) with e <= 0.9 from a tabulated E(e, M) (bilinear, within
                    2e-3 rad; the tabulated guess of Sec. 5.4) and takes one
                    step: Halley's correction (the second-order member of
                    Danby's family) for e < 0.85 in the kernels that evaluate
                    one planet across a wavefront, Danby's quartic one
                    otherwise (worst error 1e-9 rad in float64).
               < 0: early exit in both precisions (schedule, then convergence test).
   max_iter    cap of the convergence-tested iteration (default 10, Sec. 4.3).
   block_threads, blocks_per_cu: launch shape (multiples of 64 / >= 1); 0 = tuned or built-in default. */
typedef struct kep_options {
    int32_t fixed_iter;
    int32_t max_iter;
    int32_t block_threads;
    int32_t blocks_per_cu;
} kep_options;

/* Kepler's equation (Eq. 1; the paper's Kepler-only mode, Sec. 5.2): for
   i < n, E[i] is the real root of E - e[i] sin E = M[i].  M may be any finite
   value (E is returned on the same branch, E(M + 2 pi) = E(M) + 2 pi); e[i]
   outside [0, 1) or a non-finite input gives NaN.  M, e, E are device arrays of
   n >= 0 doubles; E may alias neither input. */
kep_status kepler_solve(const double *M, const double *e, double *E, int64_t n,
                        kep_prec prec, const kep_options *opts, void *stream);

/* Model velocities (Eq. 2 plus offset): v_model[i * n_obs + k] = model_ik for
   every system i and observation k.  obs->v and obs->sigma are not read and
   may be NULL. */
kep_status rv_model(const kep_obs *obs, const kep_params *par, double *v_model,
                    kep_prec prec, const kep_options *opts, void *stream);

/* Chi-square of every system (Eq. 5): chi2[i], i < n_sys. */
kep_status rv_chisq(const kep_obs *obs, const kep_params *par, double *chi2,
                    kep_prec prec, const kep_options *opts, void *stream);

/* Chi-square and its gradient (the parallel partial derivatives asked for in
   Sec. 6), by the implicit-function adjoint of Kepler's equation:
   dE/dM = 1/(1 - e cos E), dE/de = sin E/(1 - e cos E); no iteration is
   differentiated.  grad is [(5 * n_pl + 1)][n_sys]: rows 5j..5j+4 are
   d chi2 / d(P_j, K_j, e_j, omega_j, M0_j), the last row d chi2 / d gamma.
   The jitter is an input, not differentiated. */
kep_status rv_chisq_grad(const kep_obs *obs, const kep_params *par, double *chi2, double *grad,
                         kep_prec prec, const kep_options *opts, void *stream);

/* Gaussian likelihood with jitter and its gradient.  Eq. 5 weights each
   residual by 1/(sigma_k^2 + s_i^2); with s_i free, the chi-square alone is
   not the quantity to maximise, and the normalisation of the Gaussian enters:
   nll[i] = -2 ln L_i - n_obs ln(2 pi) = chi2_i + sum_k ln(sigma_k^2 + s_i^2).
   grad is [(5 * n_pl + 2)][n_sys]: the rows of rv_chisq_grad (the normalisation
   does not depend on them), then d nll / d s_i = 2 s_i sum_k (w_k - w_k^2 r_k^2)
   with w_k = 1/(sigma_k^2 + s_i^2) and r_k the residual.  A NULL jitter means
   s_i = 0 (the last row is then 0).  Domain and errors as rv_chisq_grad. */
kep_status rv_nll_grad(const kep_obs *obs, const kep_params *par, double *nll, double *grad,
                       kep_prec prec, const kep_options *opts, void *stream);

/* Gauss-Newton products for Levenberg-Marquardt / Newton-type optimisers (the
   paper asks for derivatives to feed optimisers, Sec. 6).  With J the
   Jacobian of the model velocities (rows: observations; columns: the
   np = 5 n_pl + 1 parameters in rv_chisq_grad's order) and
   W = diag(1/(sigma_k^2 + s_i^2)):
     chi2[i]                      = r^T W r (Eq. 5),
     jtwr[a * n_sys + i]          = (J^T W r)_a  (half the chi-square gradient),
     jtwj[idx(a, b) * n_sys + i]  = (J^T W J)_ab for a <= b, packed upper
                                    triangle, idx(a, b) = a np - a (a - 1)/2 + (b - a),
                                    np (np + 1)/2 rows.
   The jitter is a fixed input.  J is formed from the same implicit-function
   derivative terms as rv_chisq_grad and the products run on the matrix cores:
   KEP_FP64 with binary64 terms and binary64 products; KEP_MIXED with binary32
   terms and binary32 products over each group of 64 observations, the groups
   summed in binary64 (each entry within 64 x 2^-24 of the Cauchy-Schwarz
   bound sqrt((J^T W J)_aa (J^T W J)_bb) from the product rounding).
   Domain and errors as rv_chisq_grad. */
kep_status rv_chisq_gn(const kep_obs *obs, const kep_params *par, double *chi2, double *jtwr, double *jtwj,
                       kep_prec prec, const kep_options *opts, void *stream);

/* The paper's separate-function form (Sec. 4.4, first of its two
   implementations; Sec. 5.3 measures it against the fused one): one call
   writes the velocity of every planet at every observation, a second forms
   the planet sums and the chi-square from them.  Binary32 velocities, mixed
   precision arithmetic as KEP_MIXED.
   rv_planet_velocities: dv[(j * n_sys + i) * n_obs + k] = v_ijk (Eq. 3), a
   caller-owned device array of n_pl * n_sys * n_obs floats (observations
   contiguous, so each (planet, system) row is written and read coalesced);
   obs->v and obs->sigma are not read.  A system outside the domain gets NaN
   velocities.
   rv_chisq_from_velocities: chi2[i] (Eq. 5) from dv; par supplies n_sys, n_pl,
   offset and jitter (the planes are not read and may be NULL).  n_obs <= 1024. */
kep_status rv_planet_velocities(const kep_obs *obs, const kep_params *par, float *dv,
                                const kep_options *opts, void *stream);
kep_status rv_chisq_from_velocities(const kep_obs *obs, const kep_params *par, const float *dv, double *chi2,
                                    const kep_options *opts, void *stream);

/* Kepler's equation only, for every (system, planet, observation): the
   paper's first mixed-precision use of the GPU (Sec. 5.2), which returned
   the n_sys x n_pl x n_obs solutions instead of the chi-square.
   E[(j * n_sys + i) * n_obs + k] (binary32, caller-owned device array of
   n_pl * n_sys * n_obs floats, observations contiguous) is the eccentric
   anomaly of planet j of system i at t_k: the mean anomaly of Eq. 4 formed in
   binary64 and reduced to [-pi, pi) (Eq. 6 with the binary64 bracket of
   Sec. 5.1), then the binary32 Danby iteration of KEP_MIXED, so
   E lies in [-pi, pi] and differs by a multiple of 2 pi from the root for the
   mean anomaly taken in [0, 2 pi).  obs->v and obs->sigma are not read; K
   and omega only enter the domain check.  A system outside the domain gets
   NaN, as does an observation with a non-finite time.  Mixed precision only;
   errors as rv_chisq. */
kep_status rv_eccentric_anomalies(const kep_obs *obs, const kep_params *par, float *E, const kep_options *opts,
                                  void *stream);

/* ---- astrometric Keplerian model (Thiele-Innes form) ----
   The star's reflex offset on the sky from the same phase (Eq. 4) and Kepler
   solve (Eq. 1): per planet X = cos E - e, Y = sqrt(1 - e^2) sin E and
     dRA* = B X + G Y,   dDec = A X + F Y,
   summed over planets, plus per-system offsets x0 (RA*cos Dec) and y0 (Dec).
   A, B, F, G are the Thiele-Innes constants of the star's orbit (linear
   parameters; any angular unit, the same for positions and uncertainties).
   chi2 = sum_k (dRA*_k - x_k)^2 / sigma_x,k^2 + (dDec_k - y_k)^2 / sigma_y,k^2.
   This is the larger dynamic range for which Sec. 5.1 notes that binary32 is
   not enough: KEP_MIXED keeps the binary64 phase and the binary32 Danby
   iteration and adds one binary64 Newton step against the binary64 mean
   anomaly (E to ~1e-11 rad), then forms the positions, residuals and sums in
   binary64.  KEP_FP64 is the plain binary64 path (30 Danby steps by default).
   Domain: P > 0, 0 <= e < 1, finite parameters, sigma > 0, else NaN for that
   system.  Planes [n_pl][n_sys] as for kep_params; x0, y0 [n_sys] or NULL. */
typedef struct kep_astro_obs {
    const double *t, *x, *y, *sigma_x, *sigma_y;
    int64_t n_obs;
    double t0;
} kep_astro_obs;

typedef struct kep_astro_params {
    const double *P, *e, *M0, *A, *B, *F, *G;
    const double *x0, *y0;
    int64_t n_sys, n_pl;
} kep_astro_params;

/* Model offsets xy[(i * 2 + 0) * n_obs + k] = dRA*_ik + x0_i and
   xy[(i * 2 + 1) * n_obs + k] = dDec_ik + y0_i.  x, y and the sigmas are not read. */
kep_status astro_model(const kep_astro_obs *obs, const kep_astro_params *par, double *xy,
                       kep_prec prec, const kep_options *opts, void *stream);

/* chi2[i], i < n_sys. */
kep_status astro_chisq(const kep_astro_obs *obs, const kep_astro_params *par, double *chi2,
                       kep_prec prec, const kep_options *opts, void *stream);

/* ---- ragged batches (systems of uneven n_pl and n_obs, CSR-packed) ----
   System i owns observations obs_off[i] .. obs_off[i+1]-1 of t, v, sigma and
   planets pl_off[i] .. pl_off[i+1]-1 of P, K, e, omega, M0 (flat arrays of
   n_pl_total values).  obs_off and pl_off are device arrays of n_sys + 1
   non-decreasing int64 starting at 0 and ending at n_obs_total / n_pl_total;
   every system needs 1 <= n_pl <= KEP_MAX_PL planets and n_obs >= 0. */
typedef struct kep_obs_csr {
    const double *t, *v, *sigma;
    const int64_t *obs_off;
    int64_t n_obs_total;
    double t0;
} kep_obs_csr;

typedef struct kep_params_csr {
    const double *P, *K, *e, *omega, *M0;
    const int64_t *pl_off;
    const double *offset, *jitter;
    int64_t n_sys, n_pl_total;
} kep_params_csr;

typedef struct kep_plan kep_plan;   /* opaque; owned by the library */

/* Build a plan for one ragged batch: copies the CSR offsets to the host,
   checks them and keeps device copies of the checked offsets (later changes
   to obs->obs_off and par->pl_off have no effect on the plan), orders the
   systems by work (n_pl * n_obs, largest first; by planet count within
   windows of 256 systems),
   picks the launch shape (the autotuner times block size x systems per work
   item x observation group size on this batch unless opts fixes
   block_threads; results are cached per device and shape class, and kept in
   the text file named by the environment variable KEP_TUNE_CACHE if set), and
   records the persistent kernel as a HIP graph (the kernel leaves its
   work-queue counters at zero for the next launch, so no reset is
   recorded).  May allocate and synchronises `stream`.  The plan keeps the
   other input pointers: their contents may change between calls, their
   addresses and sizes may not.  KEP_FP64 plans (the plain binary64 path of
   rv_chisq, Sec. 5.1: IEEE quotient, 30 Danby steps by default) skip the
   autotuner and the graph: one wavefront per system over the work order,
   launched directly by both calls below; block_threads at most 256. */
kep_status kep_plan_ragged(const kep_obs_csr *obs, const kep_params_csr *par, kep_prec prec,
                           const kep_options *opts, void *stream, kep_plan **out);

/* Chi-square of every system of the plan's batch into chi2[n_sys] (one graph
   launch on `stream`, a direct launch for KEP_FP64 plans; does not allocate
   or synchronise).  Calls on one plan must not overlap in time (they share
   the plan's work-queue counters). */
kep_status rv_chisq_ragged(kep_plan *plan, double *chi2, void *stream);

/* Same work launched directly, without the graph (for comparison). */
kep_status rv_chisq_ragged_direct(kep_plan *plan, double *chi2, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid allocation): the
   chi-square of a ragged batch in one call, without a plan.  Allocates
   nothing (no hipMalloc, hipFree or allocating library call) and does not
   synchronise: two kernels on `stream`.  The first checks each system's
   offsets on the device and writes the work order (systems by decreasing
   planet count, index order within a count, so results are the same on every
   call) into a static device work area of the library; the second is the
   plan's persistent kernel at a fixed launch shape (256-thread blocks or
   opts->block_threads, 16 systems per work item).
   Arguments as kep_plan_ragged plus chi2[n_sys] (caller-owned device array).
   Limit: n_sys <= 2,097,152 (the work area holds a 32-bit order entry per
   system after 2 KiB of work-queue counters; 8 MiB + 2 KiB per GPU, held
   until the process ends); larger
   batches return KEP_ERR_SHAPE.  Offsets are not read on the host: a system
   whose offsets fall outside [0, n_obs_total] / [0, n_pl_total], decrease, or
   give n_pl outside [1, KEP_MAX_PL] gets a NaN chi-square (other systems are
   unaffected).  Every call on one GPU shares the work area: calls that
   overlap in time on the same GPU (different streams, threads) race and
   must not be made.  KEP_FP64: one kernel, the binary64 path of the plans,
   in system order with every system's offsets checked by the wavefront that
   evaluates it (same NaN rule); it uses no work area, so neither the n_sys
   limit nor the sharing between calls applies to it. */
kep_status rv_chisq_ragged_static(const kep_obs_csr *obs, const kep_params_csr *par, double *chi2, kep_prec prec,
                                  const kep_options *opts, void *stream);

typedef struct kep_plan_info {
    int64_t n_sys, n_obs_total, n_pl_total, triples;
    int32_t block_threads, blocks, sys_per_batch, tuned;
    double tuned_ms;          /* best candidate's time during tuning, 0 if not tuned */
    int32_t group_chunks;     /* largest observation group, in 64-lane chunks */
    int32_t reserved;
} kep_plan_info;

kep_status kep_plan_get_info(const kep_plan *plan, kep_plan_info *info);

void kep_plan_destroy(kep_plan *plan);

/* ---- population sampler: differential-evolution MCMC (DE-MC) ----
   The many-chain MCMC that the batched chi-square serves (Sec. 6 names
   population MCMC and DEMCMC with hundreds to thousands of chains): DE-MC of
   ter Braak (2006) with target exp(-chi2/2) (Eq. 5, jitter fixed per chain)
   and a flat prior on P > 0, K >= 0, 0 <= e < 1, omega, M0 and gamma finite.
   The population is two halves of n_half chains; a generation updates half 0
   using differences of half-1 chains, then half 1 using differences of the
   updated half 0, so no chain's proposal depends on a chain moving with it:
     y = x_i + gam (x_r1 - x_r2) + eps z,  r1 != r2 uniform in the other half,
     z_r standard normal (Box-Muller), accepted iff 2 ln u < chi2(x_i) - chi2(y).
   gam = options->gamma, or 2.38/sqrt(2 d) when gamma <= 0; gam = 1 on every
   generation g with (g + 1) % jump_every == 0 (jump_every > 0).  Random
   numbers: Philox-4x32-10 keyed by the 64-bit seed (low word first), counter
   (chain, draw, g mod 2^32, (g >> 32) | half << 31); draw 0 gives r1, r2 and
   u, draws 1.. give two normals each (rows 2j-2, 2j-1).  A proposal is thus a
   function of (seed, half, chain, generation) only: runs are reproducible and
   independent of launch shape.
   State (device, caller-owned, updated in place):
     x        [2][d][n_half], d = 5 n_pl + 1: each half is a kep_params set of
              planes P[n_pl][n_half], K, e, omega, M0, then the offset row;
     chi2     [2][n_half] chi-square of each chain's state (demc_chisq);
     n_accept [2][n_half] accepted proposals per chain, incremented (or NULL);
     jitter   [2][n_half] fixed jitter of each chain (or NULL = 0).
   2 <= n_half < 2^31, 1 <= n_pl <= KEP_MAX_PL.  A chain whose chi2 is NaN
   (state outside the support) never moves. */
typedef struct kep_demc_state {
    double *x;
    double *chi2;
    int64_t *n_accept;
    const double *jitter;
    int64_t n_half, n_pl;
} kep_demc_state;

typedef struct kep_demc_options {
    double gamma;             /* difference scale; <= 0: 2.38 / sqrt(2 d) */
    int32_t jump_every;       /* > 0: gam = 1 every jump_every-th generation */
    int32_t reserved;
    uint64_t seed;            /* Philox key */
    const double *eps;        /* [d] device: standard deviation of the normal term per row */
} kep_demc_options;

/* chi2 of every chain of the population (both halves; NaN where a K < 0). */
kep_status demc_chisq(const kep_obs *obs, const kep_demc_state *state, kep_prec prec,
                      const kep_options *opts, void *stream);

/* Generations gen0 .. gen0 + n_gen - 1, launched directly (one fused
   propose / chi-square / accept kernel per half).  work: device workspace of
   (d + 1) * n_half doubles, owned by the caller; it receives the last half's
   proposals [d][n_half] and their chi-square [n_half].  Does not allocate or
   synchronise.  prec selects the chi-square kernel (the sampler's own
   arithmetic is binary64 in both). */
kep_status demc_generations(const kep_obs *obs, const kep_demc_state *state, const kep_demc_options *options,
                            uint64_t gen0, int64_t n_gen, double *work, kep_prec prec,
                            const kep_options *opts, void *stream);

/* The same generations recorded as HIP graphs (one of a single generation,
   one of eight): generation k of a graph reads its number as a device
   counter plus k, and the graph's last node advances the counter by the
   graph's generation count; demc_run sets the counter to gen0 and replays the
   graphs until n_gen generations have run.
   Results equal demc_generations bit for bit.  kep_plan_demc
   allocates (the counter) and keeps every pointer of state, options and work;
   calls on one plan must not overlap; synchronise before destroying it. */
typedef struct kep_demc_plan kep_demc_plan;
kep_status kep_plan_demc(const kep_obs *obs, const kep_demc_state *state, const kep_demc_options *options,
                         double *work, kep_prec prec, const kep_options *opts, void *stream,
                         kep_demc_plan **out);
kep_status demc_run(kep_demc_plan *plan, uint64_t gen0, int64_t n_gen, void *stream);
void kep_demc_plan_destroy(kep_demc_plan *plan);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char *kep_last_error(void);

int kep_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KEPLER_MI355X_H */
