/*
 * CPU oracle for batched Keplerian radial-velocity models and their chi-square.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct reference
 * that the GPU library is checked against.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * constant or helper with the GPU library, and the GPU library never calls it.
 *
 * Precision.  Inputs and outputs are IEEE binary64.  The quotient
 * q = (t - t0) / P is rounded to binary64 exactly as the paper prescribes for
 * the bracketed term of the mean anomaly (Sec. 4.2, Eq. 6; Sec. 5.1 stores t and
 * P in double and evaluates the bracket in double).  Every later step (Kepler
 * root, true anomaly, velocity, planet sum, chi-square sum, gradient) runs in
 * x86 extended precision (long double, 64-bit significand) and is rounded to
 * binary64 once at the end, so the oracle is more accurate than any GPU path.
 *
 * Readings of the paper used here (each is listed with its reason in the
 * design notes of the repository):
 *  - Mean anomaly M = 2*pi*frac((t - t0)/P) + M0 with a PLUS sign on M0: Eq. 4
 *    writes +M0 and calls M0 the mean anomaly at the epoch; Eq. 6 prints -M0.
 *    The epoch t0 is an explicit input (the paper fixes t0 = 0, Sec. 2.1).
 *  - Velocity of one planet v = K [cos(omega + f) + e cos(omega)] with K the
 *    usual semi-amplitude, omega the argument of pericentre and f the true
 *    anomaly.  The printed Eq. 3 mixes conventions (its K' and the bracket);
 *    this is the standard Keplerian velocity it stands for.
 *  - Jitter: one value s per system, w_k = 1 / (sigma_k^2 + s^2) (Eq. 5).
 *  - An optional per-system velocity offset gamma is added to the planet sum.
 *  - Domain: e in [0, 1), P > 0 and every input finite, else the system's
 *    chi-square (and gradient) is NaN.
 *
 * Parity pins for each function live in the CPU test suite; none is unpinned.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <float.h>

typedef long double ld;

static const ld PI_L = 3.14159265358979323846264338327950288L;
#define TWO_PI_L (2.0L * PI_L)

static int finite_d(double x) { return isfinite(x) != 0; }

/* ------------------------------------------------------------------ */
/* Kepler's equation, Eq. 1:  M = E - e sin E.                          */
/* g(E) = E - e sin E - M is strictly increasing (g' = 1 - e cos E >=  */
/* 1 - e > 0), so the root is unique and lies in [M - e, M + e].  The  */
/* oracle runs Newton's method on g, kept inside that bracket (a step  */
/* that leaves the bracket is replaced by bisection), started from the */
/* paper's guess E0 = M + 0.85 e sign(sin M) (Sec. 4.3).  It stops     */
/* when the bracket or the Newton step is below the long-double        */
/* resolution; at most 400 steps.  This deliberately differs from the  */
/* GPU's Danby iteration: both must reach the same unique root.        */
/* ------------------------------------------------------------------ */
static ld kepler_root_l(ld M, ld e)
{
    if (e == 0.0L) return M;
    ld lo = M - e, hi = M + e;
    ld E = M + 0.85L * e * (sinl(M) >= 0.0L ? 1.0L : -1.0L);
    if (E < lo) E = lo;
    if (E > hi) E = hi;
    for (int it = 0; it < 400; ++it) {
        ld g = E - e * sinl(E) - M;
        if (g == 0.0L) return E;
        if (g > 0.0L) hi = E; else lo = E;
        ld dg = 1.0L - e * cosl(E);
        ld En = E - g / dg;
        if (!(En > lo && En < hi)) En = 0.5L * (lo + hi);
        ld step = fabsl(En - E);
        E = En;
        ld scale = fabsl(E) > 1.0L ? fabsl(E) : 1.0L;
        if (step <= 4.0L * LDBL_EPSILON * scale) {
            /* one more Newton step from a point this close cannot leave the bracket */
            g = E - e * sinl(E) - M;
            dg = 1.0L - e * cosl(E);
            return E - g / dg;
        }
        if (hi - lo <= 2.0L * LDBL_EPSILON * scale) return 0.5L * (lo + hi);
    }
    return E;
}

double oracle_kepler(double M, double e)
{
    if (!finite_d(M) || !finite_d(e) || !(e >= 0.0 && e < 1.0)) return NAN;
    return (double)kepler_root_l((ld)M, (ld)e);
}

void oracle_kepler_batch(const double *M, const double *e, double *E, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) E[i] = oracle_kepler(M[i], e[i]);
}

/* ------------------------------------------------------------------ */
/* Mean anomaly, Eq. 4 and Eq. 6: q = (t - t0)/P in binary64 (Sec. 5.1),*/
/* phi = q - floor(q) (exact), M = 2 pi phi + M0, brought into [0, 2pi)*/
/* by subtracting whole turns (Sec. 4.2 keeps M in [0, 2pi)).          */
/* ------------------------------------------------------------------ */
static ld mean_anomaly_l(double t, double t0, double P, double M0)
{
    double dt = t - t0;
    double q = dt / P;                 /* IEEE binary64 division, round to nearest */
    double phi = q - floor(q);         /* exact in binary64 */
    ld M = TWO_PI_L * (ld)phi + (ld)M0;
    M -= TWO_PI_L * floorl(M / TWO_PI_L);
    return M;
}

double oracle_mean_anomaly(double t, double t0, double P, double M0)
{
    return (double)mean_anomaly_l(t, t0, P, M0);
}

/* ------------------------------------------------------------------ */
/* True anomaly from E (half-angle form) and the velocity of one planet */
/* (Eq. 3 in its standard reading): v = K [cos(omega + f) + e cos omega]*/
/* ------------------------------------------------------------------ */
static ld true_anomaly_l(ld E, ld e)
{
    return 2.0L * atan2l(sqrtl(1.0L + e) * sinl(0.5L * E), sqrtl(1.0L - e) * cosl(0.5L * E));
}

static int planet_ok(double P, double K, double e, double w, double M0)
{
    return finite_d(P) && P > 0.0 && finite_d(K) && finite_d(e) && e >= 0.0 && e < 1.0 &&
           finite_d(w) && finite_d(M0);
}

static ld planet_rv_l(double t, double t0, double P, double K, double e, double w, double M0)
{
    ld M = mean_anomaly_l(t, t0, P, M0);
    ld E = kepler_root_l(M, (ld)e);
    ld f = true_anomaly_l(E, (ld)e);
    return (ld)K * (cosl((ld)w + f) + (ld)e * cosl((ld)w));
}

double oracle_planet_rv(double t, double t0, double P, double K, double e, double w, double M0)
{
    if (!finite_d(t) || !finite_d(t0) || !planet_ok(P, K, e, w, M0)) return NAN;
    return (double)planet_rv_l(t, t0, P, K, e, w, M0);
}

/* ------------------------------------------------------------------ */
/* Dense batch.  Observations t, v, sigma [n_obs] are shared by every  */
/* system (Sec. 4.1).  Parameter planes P, K, e, w, M0 are [n_pl][n_sys]*/
/* with the system index fastest.  offset and jitter are [n_sys] or   */
/* NULL (zero).  Only systems i in [i0, i1) are evaluated.             */
/* ------------------------------------------------------------------ */
typedef struct {
    const double *t, *v, *sigma;
    int64_t n_obs;
    double t0;
    const double *P, *K, *e, *w, *M0;
    const double *offset, *jitter;
    int64_t n_sys, n_pl;
} oracle_dense;

static int system_ok(const oracle_dense *d, int64_t i)
{
    for (int64_t j = 0; j < d->n_pl; ++j) {
        int64_t p = j * d->n_sys + i;
        if (!planet_ok(d->P[p], d->K[p], d->e[p], d->w[p], d->M0[p])) return 0;
    }
    if (d->offset && !finite_d(d->offset[i])) return 0;
    if (d->jitter && !(finite_d(d->jitter[i]) && d->jitter[i] >= 0.0)) return 0;
    if (!finite_d(d->t0)) return 0;
    return 1;
}

/* Weight of one observation for a system with jitter s (Eq. 5).  Returns 0
   (the caller turns it into NaN) unless sigma >= 0, sigma^2 + s^2 > 0 and
   t, v, sigma are finite. */
static ld weight_l(double sigma, double v, double t, double s)
{
    if (!finite_d(sigma) || !(sigma >= 0.0) || !finite_d(v) || !finite_d(t)) return 0.0L;
    ld var = (ld)sigma * (ld)sigma + (ld)s * (ld)s;
    if (!(var > 0.0L) || !isfinite(var)) return 0.0L;
    return 1.0L / var;
}

/* Eq. 2 plus offset: model velocity of system i at time t. */
static ld model_l(const oracle_dense *d, int64_t i, double t)
{
    ld sum = 0.0L;
    for (int64_t j = 0; j < d->n_pl; ++j) {
        int64_t p = j * d->n_sys + i;
        sum += planet_rv_l(t, d->t0, d->P[p], d->K[p], d->e[p], d->w[p], d->M0[p]);
    }
    if (d->offset) sum += (ld)d->offset[i];
    return sum;
}

void oracle_rv_model(const oracle_dense *d, double *out, int64_t i0, int64_t i1)
{
    for (int64_t i = i0; i < i1; ++i) {
        int ok = system_ok(d, i);
        for (int64_t k = 0; k < d->n_obs; ++k)
            out[i * d->n_obs + k] = (ok && finite_d(d->t[k])) ? (double)model_l(d, i, d->t[k]) : NAN;
    }
}

/* Eq. 5: chi2_i = sum_k (model_ik - v_k)^2 / (sigma_k^2 + s_i^2). */
void oracle_chisq(const oracle_dense *d, double *chi2, int64_t i0, int64_t i1)
{
    for (int64_t i = i0; i < i1; ++i) {
        if (!system_ok(d, i)) { chi2[i] = NAN; continue; }
        double s = d->jitter ? d->jitter[i] : 0.0;
        ld acc = 0.0L;
        int bad = 0;
        for (int64_t k = 0; k < d->n_obs; ++k) {
            ld w = weight_l(d->sigma[k], d->v[k], d->t[k], s);
            if (w == 0.0L) { bad = 1; break; }
            ld r = model_l(d, i, d->t[k]) - (ld)d->v[k];
            acc += w * r * r;
        }
        chi2[i] = bad ? NAN : (double)acc;
    }
}

/* ------------------------------------------------------------------ */
/* Gradient of Eq. 5 with respect to (P, K, e, omega, M0) of every     */
/* planet and the offset gamma; the paper asks for parallel partial    */
/* derivatives of the goodness of fit (Sec. 6).  Analytic, using the   */
/* implicit-function derivatives of Kepler's equation, no iteration   */
/* is differentiated:                                                  */
/*   df/dM = (1 + e cos f)^2 / (1 - e^2)^(3/2)                         */
/*   df/de (M fixed) = sin f (2 + e cos f) / (1 - e^2)                 */
/*   dv/dK = cos(w+f) + e cos w,  dv/dw = -K [sin(w+f) + e sin w]       */
/*   dv/dM0 = -K sin(w+f) df/dM,  dv/dP = dv/dM0 * (-2 pi q / P)       */
/*   dv/de = K cos w - K sin(w+f) df/de                                */
/*   dchi2/dtheta = sum_k 2 w_k r_k dv/dtheta,  dchi2/dgamma = sum 2 w r*/
/* grad layout: [(5*n_pl + 1)][n_sys], planet j uses rows 5j..5j+4 in  */
/* the order P, K, e, omega, M0; the last row is the offset.           */
/* ------------------------------------------------------------------ */
/* Partial derivatives of planet j's velocity at time t with respect to
   (P, K, e, omega, M0) of system i. */
static void planet_dv_l(const oracle_dense *d, int64_t i, int64_t j, double t, ld dv[5])
{
    int64_t p = j * d->n_sys + i;
    ld P = d->P[p], K = d->K[p], e = d->e[p], om = d->w[p];
    ld q = (ld)((t - d->t0) / d->P[p]);
    ld M = mean_anomaly_l(t, d->t0, d->P[p], d->M0[p]);
    ld E = kepler_root_l(M, e);
    ld f = true_anomaly_l(E, e);
    ld one_m_e2 = (1.0L - e) * (1.0L + e);
    ld b = sqrtl(one_m_e2);
    ld ecf = 1.0L + e * cosl(f);
    ld dfdM = ecf * ecf / (one_m_e2 * b);
    ld dfde = sinl(f) * (2.0L + e * cosl(f)) / one_m_e2;
    ld swf = sinl(om + f);
    ld dv_dK = cosl(om + f) + e * cosl(om);
    ld dv_dw = -K * (swf + e * sinl(om));
    ld dv_dM0 = -K * swf * dfdM;
    ld dv_dP = dv_dM0 * (-TWO_PI_L * q / P);
    ld dv_de = K * cosl(om) - K * swf * dfde;
    dv[0] = dv_dP;
    dv[1] = dv_dK;
    dv[2] = dv_de;
    dv[3] = dv_dw;
    dv[4] = dv_dM0;
}

static void chisq_grad_impl(const oracle_dense *d, double *chi2, double *grad, double *scale_r,
                            double *scale_1, int nll, int64_t i0, int64_t i1)
{
    const int64_t npar = 5 * d->n_pl + 1;
    const int64_t nrow = npar + (nll ? 1 : 0);
    ld g[5 * 64 + 1], sr[5 * 64 + 1], s1[5 * 64 + 1];
    for (int64_t i = i0; i < i1; ++i) {
        int ok = system_ok(d, i) && d->n_pl <= 64;
        double s = d->jitter ? d->jitter[i] : 0.0;
        for (int64_t a = 0; a < npar; ++a) g[a] = sr[a] = s1[a] = 0.0L;
        ld acc = 0.0L, sum_logvar = 0.0L, sum_w = 0.0L, sum_w2r2 = 0.0L;
        for (int64_t k = 0; ok && k < d->n_obs; ++k) {
            ld wk = weight_l(d->sigma[k], d->v[k], d->t[k], s);
            if (wk == 0.0L) { ok = 0; break; }
            ld r = model_l(d, i, d->t[k]) - (ld)d->v[k];
            acc += wk * r * r;
            sum_logvar -= logl(wk);
            sum_w += wk;
            sum_w2r2 += wk * wk * r * r;
            ld c = 2.0L * wk * r;
            for (int64_t j = 0; j < d->n_pl; ++j) {
                ld dv[5];
                planet_dv_l(d, i, j, d->t[k], dv);
                for (int a = 0; a < 5; ++a) {
                    g[5 * j + a] += c * dv[a];
                    sr[5 * j + a] += fabsl(c * dv[a]);
                    s1[5 * j + a] += 2.0L * wk * fabsl(dv[a]);
                }
            }
            g[npar - 1] += c;
            sr[npar - 1] += fabsl(c);
            s1[npar - 1] += 2.0L * wk;
        }
        chi2[i] = ok ? (double)(nll ? acc + sum_logvar : acc) : NAN;
        for (int64_t a = 0; a < npar; ++a) {
            grad[a * d->n_sys + i] = ok ? (double)g[a] : NAN;
            if (scale_r) scale_r[a * d->n_sys + i] = ok ? (double)sr[a] : NAN;
            if (scale_1) scale_1[a * d->n_sys + i] = ok ? (double)s1[a] : NAN;
        }
        if (nll) {
            ld s = d->jitter ? (ld)d->jitter[i] : 0.0L;
            grad[(nrow - 1) * d->n_sys + i] = ok ? (double)(2.0L * s * (sum_w - sum_w2r2)) : NAN;
        }
    }
}

void oracle_chisq_grad(const oracle_dense *d, double *chi2, double *grad, int64_t i0, int64_t i1)
{
    chisq_grad_impl(d, chi2, grad, NULL, NULL, 0, i0, i1);
}

/* Gaussian likelihood with jitter (Eq. 5's weights w = 1/(sigma^2 + s^2)):
   -2 ln L = chi2 + sum_k ln(sigma_k^2 + s^2), the constant n_obs ln(2 pi)
   omitted, and its gradient: rows as oracle_chisq_grad, then d/ds =
   2 s (sum_k w_k - sum_k w_k^2 r_k^2).  grad is [(5 n_pl + 2)][n_sys]. */
void oracle_nll_grad(const oracle_dense *d, double *nll, double *grad, int64_t i0, int64_t i1)
{
    chisq_grad_impl(d, nll, grad, NULL, NULL, 1, i0, i1);
}

/* Error scales of the gradient (for stating tolerances): per component,
   scale_r = sum_k |2 w_k r_k dv/dtheta| and scale_1 = sum_k 2 w_k |dv/dtheta|,
   so a residual error dr and a relative error eps in each term move the
   gradient by at most dr * scale_1 + eps * scale_r. */
void oracle_chisq_grad_scales(const oracle_dense *d, double *chi2, double *grad, double *scale_r,
                              double *scale_1, int64_t i0, int64_t i1)
{
    chisq_grad_impl(d, chi2, grad, scale_r, scale_1, 0, i0, i1);
}

/* ------------------------------------------------------------------ */
/* Ragged batch: system i owns observations obs_off[i]..obs_off[i+1]-1 */
/* and planets pl_off[i]..pl_off[i+1]-1 (CSR).  Same chi-square.       */
/* ------------------------------------------------------------------ */
typedef struct {
    const double *t, *v, *sigma;
    const int64_t *obs_off;
    double t0;
    const double *P, *K, *e, *w, *M0;
    const int64_t *pl_off;
    const double *offset, *jitter;
    int64_t n_sys;
} oracle_ragged;

void oracle_chisq_ragged(const oracle_ragged *d, double *chi2, int64_t i0, int64_t i1)
{
    for (int64_t i = i0; i < i1; ++i) {
        int ok = finite_d(d->t0);
        for (int64_t p = d->pl_off[i]; p < d->pl_off[i + 1]; ++p)
            ok = ok && planet_ok(d->P[p], d->K[p], d->e[p], d->w[p], d->M0[p]);
        if (d->offset) ok = ok && finite_d(d->offset[i]);
        if (d->jitter) ok = ok && finite_d(d->jitter[i]) && d->jitter[i] >= 0.0;
        double s = d->jitter ? d->jitter[i] : 0.0;
        ld acc = 0.0L;
        for (int64_t k = d->obs_off[i]; ok && k < d->obs_off[i + 1]; ++k) {
            ld wk = weight_l(d->sigma[k], d->v[k], d->t[k], s);
            if (wk == 0.0L) { ok = 0; break; }
            ld m = 0.0L;
            for (int64_t p = d->pl_off[i]; p < d->pl_off[i + 1]; ++p)
                m += planet_rv_l(d->t[k], d->t0, d->P[p], d->K[p], d->e[p], d->w[p], d->M0[p]);
            if (d->offset) m += (ld)d->offset[i];
            ld r = m - (ld)d->v[k];
            acc += wk * r * r;
        }
        chi2[i] = ok ? (double)acc : NAN;
    }
}

/* ================================================================== */
/* Counter-based random numbers: Philox-4x32-10 (Salmon, Moraes, Dror  */
/* and Shaw, SC'11, "Parallel random numbers: as easy as 1, 2, 3").    */
/* One round maps the counter (c0, c1, c2, c3) under key (k0, k1) to   */
/*   (hi(B c2) ^ c1 ^ k0, lo(B c2), hi(A c0) ^ c3 ^ k1, lo(A c0)),     */
/* A = 0xD2511F53, B = 0xCD9E8D57 (32 x 32 -> 64-bit products); the    */
/* key is advanced by (0x9E3779B9, 0xBB67AE85) before every round but  */
/* the first; ten rounds.                                              */
/* ================================================================== */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)pb;
        uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)pa;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform double in (0, 1] from two 32-bit words: the top 27 bits of a and
   the top 26 bits of b form a 53-bit integer n, u = (n + 1) / 2^53. */
static double unit53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 1.0) * 0x1p-53;
}

/* Integer in [0, m) from one 32-bit word: floor(w m / 2^32). */
static uint32_t below(uint32_t w, uint32_t m)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)m) >> 32);
}

/* ================================================================== */
/* Population MCMC by differential evolution (DE-MC, ter Braak 2006),  */
/* the many-chain sampler the paper names as the target application    */
/* of the batched chi-square (Sec. 6).  Target density exp(-chi2 / 2)  */
/* with a flat prior on P > 0, K >= 0, 0 <= e < 1 and any finite       */
/* omega, M0, gamma.                                                   */
/*                                                                     */
/* The population is split into two halves of n_half chains.  One      */
/* generation updates half 0 with differences of half-1 chains, then   */
/* half 1 with differences of the (updated) half-0 chains, so each     */
/* chain's proposal depends only on chains that do not move while it   */
/* is updated.  For chain i of half h at generation g:                 */
/*   draw 0:  r1, r2 distinct chains of the other half, u in (0, 1]    */
/*   draws 1..: Box-Muller normals z_r, two per draw                   */
/*   y_r = x_r[i] + gam (x_r[r1] - x_r[r2]) + eps_r z_r                */
/*   accept iff 2 ln u < chi2(x) - chi2(y)  (Metropolis, symmetric)    */
/* gam = 2.38 / sqrt(2 d) by default, 1 on every jump_every-th          */
/* generation.  Draw j of (h, i, g) is Philox-4x32-10 at counter       */
/* (i, j, g mod 2^32, floor(g / 2^32) + 2^31 h) under key (seed mod    */
/* 2^32, floor(seed / 2^32)).                                          */
/* Parameter rows (d = 5 n_pl + 1): P_0..P_{n-1}, K.., e.., omega..,   */
/* M0.., gamma, so each half is [d][n_half] in the dense plane layout. */
/* ================================================================== */
typedef struct {
    const double *t, *v, *sigma;
    int64_t n_obs;
    double t0;
    double *x;              /* [2][d][n_half], updated in place */
    double *chi2;           /* [2][n_half], updated in place */
    int64_t *n_accept;      /* [2][n_half], incremented; may be NULL */
    const double *jitter;   /* [2][n_half] or NULL (zero) */
    int64_t n_half, n_pl;
    double gamma;           /* <= 0: 2.38 / sqrt(2 d) */
    int32_t jump_every;     /* > 0: gam = 1 when (g + 1) % jump_every == 0 */
    int32_t reserved;
    uint64_t seed;
    const double *eps;      /* [d] */
    double *margin;         /* [2][n_half] or NULL: (chi2(x) - chi2(y)) - 2 ln u of the last generation */
} oracle_demc;

static void demc_draw(const oracle_demc *s, int h, int64_t i, uint32_t j, uint64_t g, uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)i, j, (uint32_t)g, (uint32_t)(g >> 32) | ((uint32_t)h << 31)};
    uint32_t key[2] = {(uint32_t)s->seed, (uint32_t)(s->seed >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

/* chi-square of one parameter vector y[d] (Eq. 5) through the dense oracle. */
static double demc_chisq(const oracle_demc *s, const double *y, const double *jit)
{
    const int64_t n = s->n_pl;
    for (int64_t j = 0; j < n; ++j)
        if (!(y[n + j] >= 0.0)) return NAN;            /* K >= 0: prior support */
    oracle_dense d = {s->t, s->v, s->sigma, s->n_obs, s->t0,
                      y, y + n, y + 2 * n, y + 3 * n, y + 4 * n, y + 5 * n, jit, 1, n};
    double c = NAN;
    oracle_chisq(&d, &c, 0, 1);
    return c;
}

static const double TWO_PI_D = 6.28318530717958647692528676655900577;

static void demc_half(const oracle_demc *s, int h, uint64_t g)
{
    const int64_t d = 5 * s->n_pl + 1, nh = s->n_half;
    double *xh = s->x + (int64_t)h * d * nh;
    const double *xo = s->x + (int64_t)(1 - h) * d * nh;
    double gam = s->gamma > 0.0 ? s->gamma : 2.38 / sqrt(2.0 * (double)d);
    if (s->jump_every > 0 && (g + 1) % (uint64_t)s->jump_every == 0) gam = 1.0;
    double y[5 * 8 + 1], z[5 * 8 + 2];
    for (int64_t i = 0; i < nh; ++i) {
        uint32_t w[4];
        demc_draw(s, h, i, 0, g, w);
        uint32_t r1 = below(w[0], (uint32_t)nh);
        uint32_t r2 = below(w[1], (uint32_t)nh - 1u);
        if (r2 >= r1) r2 += 1u;
        double u = unit53(w[2], w[3]);
        for (int64_t r = 0; r < d; r += 2) {
            demc_draw(s, h, i, (uint32_t)(1 + r / 2), g, w);
            double u1 = unit53(w[0], w[1]), u2 = unit53(w[2], w[3]);
            double rho = sqrt(-2.0 * log(u1));
            z[r] = rho * cos(TWO_PI_D * u2);
            z[r + 1] = rho * sin(TWO_PI_D * u2);
        }
        for (int64_t r = 0; r < d; ++r)
            y[r] = xh[r * nh + i] + gam * (xo[r * nh + r1] - xo[r * nh + r2]) + s->eps[r] * z[r];
        const double *jit = s->jitter ? s->jitter + (int64_t)h * nh + i : NULL;
        double c_new = demc_chisq(s, y, jit);
        double c_old = s->chi2[(int64_t)h * nh + i];
        if (s->margin) s->margin[(int64_t)h * nh + i] = (c_old - c_new) - 2.0 * log(u);
        if (2.0 * log(u) < c_old - c_new) {            /* false for NaN */
            for (int64_t r = 0; r < d; ++r) xh[r * nh + i] = y[r];
            s->chi2[(int64_t)h * nh + i] = c_new;
            if (s->n_accept) s->n_accept[(int64_t)h * nh + i] += 1;
        }
    }
}

/* Run generations gen0 .. gen0 + n_gen - 1.  n_half >= 2, 1 <= n_pl <= 8. */
void oracle_demc_run(const oracle_demc *s, uint64_t gen0, int64_t n_gen)
{
    if (s->n_half < 2 || s->n_pl < 1 || s->n_pl > 8) return;
    for (int64_t k = 0; k < n_gen; ++k) {
        demc_half(s, 0, gen0 + (uint64_t)k);
        demc_half(s, 1, gen0 + (uint64_t)k);
    }
}

/* ================================================================== */
/* Astrometric Keplerian model: the star's reflex position on the sky, */
/* the larger-dynamic-range application the paper names for the same  */
/* phase and Kepler core (Sec. 5.1).  Thiele-Innes form: with E the    */
/* root of Eq. 1 at the mean anomaly of Eq. 4,                         */
/*   X = cos E - e,  Y = sqrt(1 - e^2) sin E,                          */
/*   dRA* = B X + G Y,  dDec = A X + F Y  (per planet, summed),        */
/* plus per-system offsets (x0, y0).  A, B, F, G and the positions are */
/* in one angular unit (e.g. mas).  chi2 = sum_k (dRA*_k - x_k)^2 /    */
/* sx_k^2 + (dDec_k - y_k)^2 / sy_k^2.  Planes [n_pl][n_sys] as in the */
/* dense batch; model output [n_sys][2][n_obs] (RA row, then Dec row). */
/* ================================================================== */
typedef struct {
    const double *t, *x, *y, *sx, *sy;
    int64_t n_obs;
    double t0;
    const double *P, *e, *M0, *A, *B, *F, *G;
    const double *x0, *y0;
    int64_t n_sys, n_pl;
} oracle_astro;

static int astro_system_ok(const oracle_astro *d, int64_t i)
{
    if (!finite_d(d->t0)) return 0;
    for (int64_t j = 0; j < d->n_pl; ++j) {
        int64_t p = j * d->n_sys + i;
        if (!(finite_d(d->P[p]) && d->P[p] > 0.0 && finite_d(d->e[p]) && d->e[p] >= 0.0 && d->e[p] < 1.0 &&
              finite_d(d->M0[p]) && finite_d(d->A[p]) && finite_d(d->B[p]) && finite_d(d->F[p]) &&
              finite_d(d->G[p])))
            return 0;
    }
    if (d->x0 && !finite_d(d->x0[i])) return 0;
    if (d->y0 && !finite_d(d->y0[i])) return 0;
    return 1;
}

static void astro_xy_l(const oracle_astro *d, int64_t i, double t, ld *ra, ld *dec)
{
    ld sra = d->x0 ? (ld)d->x0[i] : 0.0L, sdec = d->y0 ? (ld)d->y0[i] : 0.0L;
    for (int64_t j = 0; j < d->n_pl; ++j) {
        int64_t p = j * d->n_sys + i;
        ld e = (ld)d->e[p];
        ld E = kepler_root_l(mean_anomaly_l(t, d->t0, d->P[p], d->M0[p]), e);
        ld X = cosl(E) - e;
        ld Y = sqrtl((1.0L - e) * (1.0L + e)) * sinl(E);
        sra += (ld)d->B[p] * X + (ld)d->G[p] * Y;
        sdec += (ld)d->A[p] * X + (ld)d->F[p] * Y;
    }
    *ra = sra;
    *dec = sdec;
}

void oracle_astro_model(const oracle_astro *d, double *out, int64_t i0, int64_t i1)
{
    for (int64_t i = i0; i < i1; ++i) {
        int ok = astro_system_ok(d, i);
        for (int64_t k = 0; k < d->n_obs; ++k) {
            ld ra = 0.0L, dec = 0.0L;
            int okk = ok && finite_d(d->t[k]);
            if (okk) astro_xy_l(d, i, d->t[k], &ra, &dec);
            out[(i * 2 + 0) * d->n_obs + k] = okk ? (double)ra : NAN;
            out[(i * 2 + 1) * d->n_obs + k] = okk ? (double)dec : NAN;
        }
    }
}

void oracle_astro_chisq(const oracle_astro *d, double *chi2, int64_t i0, int64_t i1)
{
    for (int64_t i = i0; i < i1; ++i) {
        if (!astro_system_ok(d, i)) { chi2[i] = NAN; continue; }
        ld acc = 0.0L;
        int bad = 0;
        for (int64_t k = 0; k < d->n_obs; ++k) {
            double t = d->t[k], x = d->x[k], y = d->y[k], sx = d->sx[k], sy = d->sy[k];
            if (!(finite_d(t) && finite_d(x) && finite_d(y) && finite_d(sx) && finite_d(sy) && sx > 0.0 && sy > 0.0)) {
                bad = 1;
                break;
            }
            ld ra, dec;
            astro_xy_l(d, i, t, &ra, &dec);
            ld rx = ra - (ld)x, ry = dec - (ld)y;
            acc += rx * rx / ((ld)sx * (ld)sx) + ry * ry / ((ld)sy * (ld)sy);
        }
        chi2[i] = bad ? NAN : (double)acc;
    }
}


/* ================================================================== */
/* Gauss-Newton products of the chi-square (for Levenberg-Marquardt    */
/* and Newton-type optimisers; the paper asks for derivatives to feed  */
/* optimisers, Sec. 6): with J the Jacobian of the model velocities    */
/* (rows = observations, columns = the 5 n_pl + 1 parameters in the    */
/* gradient's order) and W = diag(w_k), w_k = 1/(sigma_k^2 + s^2):     */
/*   jtwr = J^T W r        (= half the chi-square gradient)            */
/*   jtwj = J^T W J        packed upper triangle, (a, b) with a <= b   */
/*          at a np - a (a - 1) / 2 + (b - a), np = 5 n_pl + 1.        */
/* Layout [row][n_sys] for both.                                       */
/* ================================================================== */
void oracle_gn(const oracle_dense *d, double *chi2, double *jtwr, double *jtwj, int64_t i0, int64_t i1)
{
    const int64_t np = 5 * d->n_pl + 1, npk = np * (np + 1) / 2;
    ld Jr[5 * 8 + 1], JJ[(5 * 8 + 1) * (5 * 8 + 2) / 2], row[5 * 8 + 1];
    for (int64_t i = i0; i < i1; ++i) {
        int ok = system_ok(d, i) && d->n_pl <= 8;
        double s = d->jitter ? d->jitter[i] : 0.0;
        ld acc = 0.0L;
        for (int64_t a = 0; a < np; ++a) Jr[a] = 0.0L;
        for (int64_t a = 0; a < npk; ++a) JJ[a] = 0.0L;
        for (int64_t k = 0; ok && k < d->n_obs; ++k) {
            ld wk = weight_l(d->sigma[k], d->v[k], d->t[k], s);
            if (wk == 0.0L) { ok = 0; break; }
            ld r = model_l(d, i, d->t[k]) - (ld)d->v[k];
            acc += wk * r * r;
            for (int64_t j = 0; j < d->n_pl; ++j) planet_dv_l(d, i, j, d->t[k], row + 5 * j);
            row[np - 1] = 1.0L;
            for (int64_t a = 0; a < np; ++a) {
                Jr[a] += wk * row[a] * r;
                for (int64_t b = a; b < np; ++b) JJ[a * np - a * (a - 1) / 2 + (b - a)] += wk * row[a] * row[b];
            }
        }
        chi2[i] = ok ? (double)acc : NAN;
        for (int64_t a = 0; a < np; ++a) jtwr[a * d->n_sys + i] = ok ? (double)Jr[a] : NAN;
        for (int64_t a = 0; a < npk; ++a) jtwj[a * d->n_sys + i] = ok ? (double)JJ[a] : NAN;
    }
}
