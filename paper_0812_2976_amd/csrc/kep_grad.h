// Per-planet terms of the chi-square gradient and of the Gauss-Newton products:
// the velocity of one planet and its partial derivatives with respect to
// (P, K, e, omega, M0), in binary64 (the plain path) and in the mixed form
// (binary32 Kepler solve, binary64 correction of the root and of the
// velocity, binary32 derivative terms).  Shared by the gradient, likelihood
// and Gauss-Newton kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "kep_device.h"
#include "kep_policy.h"

namespace kep {

// Derivatives use the implicit-function relations of Kepler's equation,
// dE/dM = 1/(1 - e cos E) and dE/de = sin E/(1 - e cos E), in the true-anomaly forms
//   df/dM = b/D^2,  df/de = sin E (2 - e cos E - e^2)/(b D^2),  D = 1 - e cos E,
// so no iteration is differentiated.
template <class T> struct GradPlanet;

template <> struct GradPlanet<double> {
    double P, rP, M0, e, b, K, cw, sw;
};

__device__ __forceinline__ bool grad_setup(double P, double K, double e, double w, double M0, int,
                                           GradPlanet<double> &g)
{
    bool ok = planet_ok(P, K, e, w, M0);
    if (!ok) { P = 1.0; K = 0.0; e = 0.0; w = 0.0; M0 = 0.0; }
    g.P = P;
    g.rP = 1.0 / P;
    g.M0 = M0;
    g.e = e;
    g.b = sqrt((1.0 - e) * (1.0 + e));
    g.K = K;
    sincos(w, &g.sw, &g.cw);
    return ok;
}

// ---------------------------------------------------------------------------
// Mixed-precision adjoint with a binary64 correction of the root.  The binary32
// iteration leaves E with an error of a few 1e-7 rad / (1 - e cos E) (the
// rounding of M to binary32 and of Kepler's residual near |M| ~ pi), and a
// binary32 velocity carries a few ulp of 100 m/s: together about 1e-5 m/s.
// Both enter the gradient through the residual r, which is small near a good
// fit (|r| ~ sigma), so the gradient's error relative to its scale
// sum_k |2 w r dv/dtheta| grows as the fit improves.  Below, one Newton step
// with Danby's second-order term (Sec. 4.3) against the binary64 mean anomaly
// corrects E, and the velocity is formed in binary64 from binary64 sin E and
// cos E; the derivative terms stay binary32 (their relative error enters the
// gradient only relative to that scale).

// sin E and cos E in binary64 of a binary32 value (the knots below):
// E = y + n pi/2 with n the nearest integer to 2E/pi and pi/2 in two parts,
// each product taken inside a fused multiply-add, then the Taylor series of
// sin y and cos y on |y| <= pi/4 (coefficients 1/n!), rotated by the quadrant
// n mod 4: sin to y^17 and cos to y^18 (remainders below 8.4e-20 and
// 3.3e-21), a binary64 result to its last bits.
__device__ __forceinline__ void sincos_root64(float E, double &s, double &c)
{
    const float nf = rintf(E * 0.636619772f);
    const int n = (int)nf;
    const double dn = (double)nf;
    const double y = fma(-dn, 6.123233995736766036e-17, fma(-dn, 1.5707963267948965580, (double)E));
    const double y2 = y * y;
    double ps = 1.0 / 355687428096000.0;             // 1/17!
    ps = fma(ps, y2, -1.0 / 1307674368000.0);        // 1/15!
    ps = fma(ps, y2, 1.0 / 6227020800.0);            // 1/13!
    double pc = -1.0 / 6402373705728000.0;           // 1/18!
    pc = fma(pc, y2, 1.0 / 20922789888000.0);        // 1/16!
    pc = fma(pc, y2, -1.0 / 87178291200.0);          // 1/14!
    pc = fma(pc, y2, 1.0 / 479001600.0);             // 1/12!
    ps = fma(ps, y2, -1.0 / 39916800.0);             // 1/11!
    ps = fma(ps, y2, 1.0 / 362880.0);                // 1/9!
    ps = fma(ps, y2, -1.0 / 5040.0);                 // 1/7!
    ps = fma(ps, y2, 1.0 / 120.0);                   // 1/5!
    ps = fma(ps, y2, -1.0 / 6.0);                    // 1/3!
    const double sy = fma(y * y2, ps, y);
    pc = fma(pc, y2, -1.0 / 3628800.0);              // 1/10!
    pc = fma(pc, y2, 1.0 / 40320.0);                 // 1/8!
    pc = fma(pc, y2, -1.0 / 720.0);                  // 1/6!
    pc = fma(pc, y2, 1.0 / 24.0);                    // 1/4!
    pc = fma(pc, y2, -0.5);                          // 1/2!
    const double cy = fma(y2, pc, 1.0);
    // quadrant q = n mod 4: (sin, cos) = (sy, cy), (cy, -sy), (-sy, -cy), (-cy, sy)
    const int q = n & 3;
    const double s0 = (q & 1) ? cy : sy;
    const double c0 = (q & 1) ? sy : cy;
    s = (q & 2) ? -s0 : s0;
    c = (q == 1 || q == 2) ? -c0 : c0;
}

// Binary64 sin and cos at the knots n/64, |n| <= kSc64Half (|E| <= 3.25: the
// centred range [-pi, pi] and the binary32 rounding of its ends), for the
// binary64 correction of a binary32 root.  A block fills its copy in LDS
// once per launch (16 bytes a knot, 6,672 in all).
constexpr int kSc64Half = 208;
constexpr int kSc64Knots = 2 * kSc64Half + 1;
constexpr size_t kSc64Bytes = (size_t)kSc64Knots * 2 * sizeof(double);

// Every thread of the block calls it; a block barrier must follow before any
// wavefront reads the table.  n/64 is exact in binary32, and the full series
// of sincos_root64 leaves only the rounding of its evaluation.
__device__ __forceinline__ void fill_sincos64_knots(double2 *tab)
{
    for (int q = threadIdx.x; q < kSc64Knots; q += blockDim.x) {
        double sv, cv;
        sincos_root64((float)(q - kSc64Half) * 0.015625f, sv, cv);
        tab[q] = make_double2(sv, cv);
    }
}

// Every root of a centred M (|M| <= pi) lies in [-3.25, 3.25], so moving an
// iterate outside it onto the interval only brings it nearer the root (a NaN
// stays NaN); the knots below cover the interval.
__device__ __forceinline__ float clamp_root(float E) { return fabsf(E) > 3.25f ? copysignf(3.25f, E) : E; }

// sin and cos of the binary32 E, |E| <= 3.25 or NaN, in binary64 from the
// nearest knot, n = rint(64 E): y = E - n/64 is exact in binary32
// (|y| <= 2^-7, and E and n/64 are within a factor two of each other once
// n != 0), sin y to y^5 and cos y to y^6 (remainders 3.5e-19 and 3.4e-22),
// then the rotation by the knot's sin and cos.  A NaN reads knot 0 and
// gives NaN.
__device__ __forceinline__ void sincos_root64_knots(float E, const double2 *tab, double &s, double &c)
{
    const float fn = rintf(E * 64.0f);
    int n;
    __asm__("v_cvt_i32_f32 %0, %1" : "=v"(n) : "v"(fn));    // a NaN converts to 0
    const double y = (double)fmaf(fn, -0.015625f, E);
    const double2 k = tab[n + kSc64Half];
    const double y2 = y * y;
    const double sy = fma(y * y2, fma(y2, 1.0 / 120.0, -1.0 / 6.0), y);
    const double cy = fma(y2, fma(y2, fma(y2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
    s = fma(k.x, cy, k.y * sy);
    c = fma(k.y, cy, -(k.x * sy));
}

// Per-planet record of the mixed adjoint (one per system and planet, in LDS).
struct RecGrad {
    Phase64 ph;                    // P, 1/P, fract(M0/(2 pi) + 1/2)
    double e, A, B;                // binary64 e, K b^2 cos w, -K b sin w  (b = sqrt(1 - e^2))
    double fP, fK;                 // gradient row factors 2 pi K/P, K
    Ecc32 k;                       // binary32 e, 1 - e, e/2, e/6
    float b, rb, b2, c0;           // b, 1/b, 1 - e^2, 2 - 2 e^2
    float cw, sw, bcw, bsw;        // cos w, sin w, b cos w, b sin w
    TabPlace tp;                   // place in the starting-value table (toff -1: the paper's guess)
    int16_t niter;                 // Danby steps from the paper's guess (0: convergence test)
    int8_t check;                  // 1 if the step count is fixed by the caller
    int8_t pad;
};

__device__ __forceinline__ bool grad_setup_rec(int fixed_iter, double P, double K, double e, double w, double M0,
                                               RecGrad &r)
{
    const bool ok = planet_ok(P, K, e, w, M0);
    if (!ok) { P = 1.0; K = 0.0; e = 0.0; w = 0.0; M0 = 0.0; }
    r.ph = make_phase64(P, M0);
    r.k = make_ecc32(e);
    const double b2 = (1.0 - e) * (1.0 + e), b = sqrt(b2);
    double sw, cw;
    sincos_reduced(w, sw, cw);     // to an ulp of w (|w| up to ~1e6 rad); few registers
    r.e = e;
    r.A = K * b2 * cw;
    r.B = -K * b * sw;
    r.fP = kTwoPi * K / P;
    r.fK = K;
    r.b = (float)b;
    r.rb = (float)(1.0 / b);
    r.b2 = (float)b2;
    r.c0 = (float)(2.0 - 2.0 * e * e);
    r.cw = (float)cw;
    r.sw = (float)sw;
    r.bcw = (float)(b * cw);
    r.bsw = (float)(b * sw);
    r.niter = (int16_t)(fixed_iter > 0 ? fixed_iter : sched32(r.k.e));
    r.check = fixed_iter > 0 ? 1 : 0;
    r.pad = 0;
    r.tp = table_place(e, fixed_iter <= 0);
    return ok;
}

// A compiler barrier: the planet records are read from LDS where they are
// used, instead of every planet's record being held in registers across both
// passes of the kernels with the lanes over observations.
__device__ __forceinline__ void lds_reload_barrier() { __asm__ volatile("" ::: "memory"); }

// System assignment of the kernels with the lanes over observations (one
// system per wavefront at a time, many output rows per system).  Runs of
// systems are handed out round-robin, so the whole grid sweeps the batch in
// order (contiguous shares per wavefront or block, which balance the last
// runs better, ran 2-7% slower: the grid then writes all over every output
// row at once).
//   INTERLEAVE: block b takes runs b, b + G, ... of wpb x sb systems (G blocks);
//     wavefront w of the block holds systems run + w + wpb i (i < nb), so the
//     block's wavefronts write neighbouring systems' entries of every output
//     row at about the same time and the L2 merges them into longer pieces
//     (with sb consecutive systems per wavefront each row's line stays partly
//     written for a whole batch and goes back to HBM in pieces).
//   else: wavefront g of W takes runs g, g + W, ... of sb consecutive systems.
struct SysShare {
    int64_t lo, hi;   // first run's start; the number of systems
    int64_t step;     // systems between a wavefront's runs
    int stride, off;  // slot i of the run starting at r is system r + off + stride i
};

template <bool INTERLEAVE>
__device__ __forceinline__ SysShare sys_share(int64_t n_sys, int wpb, int wib, int sb)
{
    SysShare q;
    q.hi = n_sys;
    if constexpr (INTERLEAVE) {
        q.lo = (int64_t)blockIdx.x * wpb * sb;
        q.step = (int64_t)gridDim.x * wpb * sb;
        q.stride = wpb;
        q.off = wib;
    } else {
        q.lo = ((int64_t)blockIdx.x * wpb + wib) * sb;
        q.step = (int64_t)gridDim.x * wpb * sb;
        q.stride = 1;
        q.off = 0;
    }
    return q;
}

// Systems of this wavefront in the run starting at r: first + stride i, i < return value.
__device__ __forceinline__ int share_run(const SysShare &q, int64_t r, int sb, int64_t &first)
{
    first = r + q.off;
    const int64_t left = q.hi - first;
    return left <= 0 ? 0 : (int)min((int64_t)sb, (left + q.stride - 1) / q.stride);
}

// One observation of the kernels with the lanes over observations (the mixed
// adjoint and Gauss-Newton products).
struct ObsG {
    double tt, v;   // t - t0, observed velocity
    float s2;       // sigma^2
    bool in, ok;    // a real observation; t, v, sigma finite and sigma >= 0
};

__device__ __forceinline__ void load_obs_g(const DenseArgs &a, int64_t k, ObsG &o)
{
    o.in = k < a.n_obs;
    const double t = o.in ? a.t[k] : a.t0;
    const double v = o.in ? a.v[k] : 0.0;
    const double s = o.in ? a.sigma[k] : 1.0;
    o.ok = isfinite(t) && isfinite(v) && isfinite(s) && s >= 0.0;
    o.tt = t - a.t0;
    o.v = v;
    o.s2 = (float)(s * s);
}

// Mean anomaly in binary64 for the corrected root, centred on [-pi, pi): the
// quotient q = (t - t0)/P correctly rounded (the product with the correctly
// rounded 1/P, then one correction by its exact remainder, t - t0 - q P by a
// fused multiply-add), as the plain path's IEEE division gives it; fract(q) is
// exact, and the phase offset is added to the fraction, not to q, so that no
// rounding at the magnitude of q (~1e-9 rad at 2.5e6 orbits) enters M.
__device__ __forceinline__ double mean_anomaly64_exact(double tt, const Phase64 &p)
{
    const double q0 = tt * p.rP;
    const double q = fma(fma(-q0, p.P, tt), p.rP, q0);
    const double ph = __builtin_amdgcn_fract(__builtin_amdgcn_fract(q) + p.m0h);
    return fma(ph, kTwoPi, -kPi);
}

// From the binary32 root E of M32 = (float)M64: the binary64 residual
// f = E - e sin E - M64, the corrected step d = d1 / (1 + d1 e sin E / (2 D))
// with d1 = -f / D, D = 1 - e cos E (Danby's second correction; the result is
// within about d^3 e / (6 D) of the root), sin and cos rotated to E + d to
// second order, and the velocity v = (A cos E + B sin E) / (1 - e cos E) in
// binary64 (the reciprocal refined by one Newton step from the binary32 one);
// knots: the block's sin/cos knots (fill_sincos64_knots).  Also returns sin E
// and cos E - e rounded to binary32 for the derivative terms.
__device__ __forceinline__ double refine_velocity(const RecGrad &r, float E, double M64, const double2 *knots,
                                                  float &sE, float &cme)
{
    E = clamp_root(E);
    double s, c;
    sincos_root64_knots(E, knots, s, c);
    const double f = fma(-r.e, s, (double)E - M64);
    const float rD = rcp32((float)fma(-r.e, c, 1.0));
    const float d1 = -(float)f * rD;
    const float d = fmaf(-d1, 0.5f * d1 * r.k.e * (float)s * rD, d1);
    const double dd = (double)d, ph = (double)(0.5f * d * d);
    const double s1 = fma(c, dd, fma(-s, ph, s));        // sin(E + d)
    const double c1 = fma(-s, dd, fma(-c, ph, c));       // cos(E + d)
    const double D = fma(-r.e, c1, 1.0);
    const double r0 = (double)rcp32((float)D);
    const double rD64 = fma(r0, fma(-D, r0, 1.0), r0);
    sE = (float)s1;
    cme = (float)(c1 - r.e);
    return fma(r.A, c1, r.B * s1) * rD64;
}

// The five per-observation terms of planet r's gradient rows from binary32
// sin E and cos E - e; qf = (t - t0)/P.  With D = 1 - e cos E,
// df/dM = b/D^2, df/de = sin E (2 - e cos E - e^2)/(b D^2):
//   x[0] = sin(w+f) df/dM q           dv/dP  = (2 pi K/P) x[0]
//   x[1] = cos(w+f) + e cos w         dv/dK  = x[1]
//   x[2] = cos w - sin(w+f) df/de     dv/de  = K x[2]
//   x[3] = sin(w+f) + e sin w         dv/dw  = -K x[3]
//   x[4] = sin(w+f) df/dM             dv/dM0 = -K x[4]
// x[1] and x[3] in the forms b (b cos w cos E - sin w sin E)/D and
// b (b sin w cos E + cos w sin E)/D: summing cos(w+f) and e cos w (or the
// sines) loses the factor 1 - e near apoapsis (f ~ pi), where they nearly
// cancel, and at e ~ 0.99 that is two decimal digits of the binary32 terms.
__device__ __forceinline__ void grad_terms_ce(const RecGrad &r, float sE, float cme, float qf, float (&x)[5])
{
    const float iD = rcp32(fmaf(-r.k.e, cme, r.b2));       // 1/(1 - e cos E) = 1/((1 - e^2) - e (cos E - e))
    const float cE = cme + r.k.e;
    const float cf = cme * iD;                               // cos f
    const float sf = r.b * sE * iD;                          // sin f
    const float swf = r.sw * cf + r.cw * sf;                 // sin(w + f)
    const float iD2 = iD * iD;
    const float a = swf * (r.b * iD2);                       // sin(w+f) df/dM
    const float bi = r.b * iD;
    x[0] = a * qf;
    x[1] = bi * fmaf(r.bcw, cE, -r.sw * sE);
    x[2] = fmaf(-swf, sE * fmaf(-r.k.e, cme, r.c0) * iD2 * r.rb, r.cw);
    x[3] = bi * fmaf(r.bsw, cE, r.cw * sE);
    x[4] = a;
}

// Sum over the 64 lanes of R per-lane rows (R a power of two <= 64), leaving
// each row's total in the lanes l with l / (64 / R) equal to the row: each
// step halves the rows a lane holds, keeping one half and adding the
// partner's copy of it (R - 1 exchanges in all, instead of R full butterflies).
// (The per-lane choice between the two halves is made by an explicit
// v_cndmask: written as a select of two array elements, the compiler turns it
// into an indexed read of the whole array, a chain of compares and selects.)
__device__ __forceinline__ float lane_select(uint64_t mask, float if_clear, float if_set)
{
    float r;
    __asm__("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(if_clear), "v"(if_set), "s"(mask));
    return r;
}

template <int R>
__device__ __forceinline__ float rows_reduce_scatter(float (&x)[R])
{
#pragma unroll
    for (int h = R / 2, o = 32; h >= 1; h >>= 1, o >>= 1) {
        const uint64_t up = __ballot((__lane_id() & o) != 0);     // lanes keeping the upper half
#pragma unroll
        for (int i = 0; i < h; ++i) {
            const float keep = lane_select(up, x[i], x[i + h]);
            const float send = lane_select(up, x[i + h], x[i]);
            x[i] = keep + __shfl_xor(send, o, 64);
        }
    }
    float v = x[0];
#pragma unroll
    for (int o = 32 / R; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// binary64 plain path: velocity of one planet and its five partial derivatives
// d[0..4] = dv/d(P, K, e, omega, M0) at tt = t - t0.
__device__ __forceinline__ double grad_eval(const GradPlanet<double> &g, double tt, int max_iter, int fixed,
                                            double (&d)[5])
{
    double q = tt / g.P;
    double phi = q - floor(q);
    double M = fma(kTwoPi, phi, g.M0);
    M = M - kTwoPi * floor(M * kInvTwoPi);
    double E = kepler64(M, g.e, M < kPi ? 1.0 : -1.0, fixed, max_iter);
    double s, c;
    sincos(E, &s, &c);
    double D = 1.0 - g.e * c;
    double cf = (c - g.e) / D;
    double sf = g.b * s / D;
    double cwf = g.cw * cf - g.sw * sf;
    double swf = g.sw * cf + g.cw * sf;
    double dvdK = cwf + g.e * g.cw;
    double dfdM = g.b / (D * D);
    double dfde = s * (2.0 - g.e * c - g.e * g.e) / (g.b * D * D);
    double dvdM0 = -g.K * swf * dfdM;
    d[0] = dvdM0 * (-kTwoPi * q / g.P);
    d[1] = dvdK;
    d[2] = g.K * g.cw - g.K * swf * dfde;
    d[3] = -g.K * (swf + g.e * g.sw);
    d[4] = dvdM0;
    return g.K * dvdK;
}

// NLL = true: the Gaussian likelihood with jitter, -2 ln L = chi2 +
// sum_k ln(sigma_k^2 + s^2) (constant dropped), and one more gradient row,
// d/ds = 2 s (sum_k w_k - sum_k w_k^2 r_k^2).

}  // namespace kep
