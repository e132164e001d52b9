// Per-planet terms of the chi-square gradient and of the Gauss-Newton products:
// the velocity of one planet and its partial derivatives with respect to
// (P, K, e, omega, M0).  Shared by the gradient kernels and the Gauss-Newton
// kernel.
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

template <> struct GradPlanet<float> {
    Phase64 ph;                // P, 1/P, fract(M0/(2 pi) + 1/2)
    Ecc32 k;                   // e, 1 - e, e/2, e/6
    float b, K, cw, sw;        // sqrt(1 - e^2), K, cos w, sin w
    float Kecw, c0;            // K e cos w, 2 - e - e^2
    int niter, check;
};

template <> struct GradPlanet<double> {
    double P, rP, M0, e, b, K, cw, sw;
};

__device__ __forceinline__ bool grad_setup(double P, double K, double e, double w, double M0, int fixed_iter,
                                           GradPlanet<float> &g)
{
    bool ok = planet_ok(P, K, e, w, M0);
    if (!ok) { P = 1.0; K = 0.0; e = 0.0; w = 0.0; M0 = 0.0; }
    g.ph = make_phase64(P, M0);
    g.k = make_ecc32(e);
    g.b = (float)sqrt((1.0 - e) * (1.0 + e));
    g.K = (float)K;
    double sw, cw;
    sincos(w, &sw, &cw);
    g.cw = (float)cw;
    g.sw = (float)sw;
    g.Kecw = (float)(K * e * cw);
    g.c0 = (float)(2.0 - e - e * e);
    g.niter = fixed_iter > 0 ? fixed_iter : sched32(g.k.e);
    g.check = fixed_iter > 0 ? 1 : 0;
    return ok;
}

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

// Velocity of one planet at time tt = t - t0 and the five per-observation
// terms whose weighted sums give its gradient (the planet's constant factors
// are applied once per system):
//   x[0] = sin(w+f) df/dM q      dv/dP  = (2 pi K / P) x[0]
//   x[1] = cos(w+f)              dv/dK  = x[1] + e cos w
//   x[2] = sin(w+f) df/de        dv/de  = K cos w - K x[2]
//   x[3] = sin(w+f)              dv/dw  = -K x[3] - K e sin w
//   x[4] = sin(w+f) df/dM        dv/dM0 = -K x[4]
// with q = (t - t0)/P, df/dM = b/D^2, df/de = sin E (2 - e cos E - e^2)/(b D^2).
// tab: the block's LDS copy of the Kepler starting-value table, or null.
__device__ __forceinline__ float grad_terms(const GradPlanet<float> &g, double tt, int max_iter, float (&x)[5],
                                            const uint32_t *tab = nullptr)
{
    const float M = mean_anomaly32(tt, g.ph);
    float sE, omcE;
    kepler32_start(M, g.k, tab, g.niter, max_iter, g.check != 0, sE, omcE);
    const float iD = rcp32(fmaf(g.k.e, omcE, g.k.ome));   // 1 / (1 - e cos E)
    const float cf = (g.k.ome - omcE) * iD;                 // cos f = (cos E - e)/D
    const float sf = g.b * sE * iD;                         // sin f = b sin E / D
    const float cwf = g.cw * cf - g.sw * sf;                // cos(w + f)
    const float swf = g.sw * cf + g.cw * sf;                // sin(w + f)
    const float iD2 = iD * iD;
    const float a = swf * (g.b * iD2);                      // sin(w+f) df/dM
    x[0] = a * (float)(tt * g.ph.rP);
    x[1] = cwf;
    x[2] = swf * (sE * fmaf(g.k.e, omcE, g.c0) * iD2 * rcp32(g.b));
    x[3] = swf;
    x[4] = a;
    return fmaf(g.K, cwf, g.Kecw);
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
