// Device-side arithmetic shared by the gfx950 kernels: orbital phase, Danby's
// iteration for Kepler's equation and the Keplerian velocity, in binary64
// ("plain") and binary32 ("mixed") forms.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kep_tables.h"

namespace kep {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kInvTwoPi = 0.15915494309189533576888376337251;
constexpr double kPi = 3.14159265358979323846264338327950;
// 2 pi as a double-double (hi + lo), for reducing large mean anomalies.
constexpr double kTwoPiHi = 6.283185307179586232;
constexpr double kTwoPiLo = 2.4492935982947064e-16;
constexpr float kHalfPiF = 1.57079637f;

__device__ __forceinline__ int wave_lane() { return __lane_id(); }

__device__ __forceinline__ int uniform_int(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ float uniform_float(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

__device__ __forceinline__ double uniform_double(double x)
{
    int64_t b = __double_as_longlong(x);
    int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
    int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

// Sum over the 64 lanes of a wavefront (butterfly; every lane gets the total).
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ float rcp32(float x) { return __builtin_amdgcn_rcpf(x); }

// Kahan compensated accumulation (Sec. 4.4): the sum is s - c.
struct Kahan32 {
    float s, c;
    __device__ __forceinline__ void init() { s = 0.0f; c = 0.0f; }
    __device__ __forceinline__ void add(float x)
    {
        float y = x - c;
        float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ double value() const { return (double)s - (double)c; }
};

// ----------------------------------------------------------------- binary32
// sin x, 1 - cos x and x - sin x for |x| <= 3 pi / 2.  Arguments beyond pi/2
// are folded with pi - |x| (pi split in two floats, exact subtraction); on
// |y| <= pi/2 the polynomials x - sin x = x^3 p(x^2) and 1 - cos x = x^2 q(x^2)
// keep full relative precision as x -> 0.
struct SinCos32 {
    float s;     // sin x
    float omc;   // 1 - cos x
    float xms;   // x - sin x
};

__device__ __forceinline__ SinCos32 sincos32(float x)
{
    float ax = fabsf(x);
    bool fold = ax > kHalfPiF;
    float yf = (KEP_PI_HI_F - ax) + KEP_PI_LO_F;   // pi - |x|, negative beyond pi
    float y = fold ? (x < 0.0f ? -yf : yf) : x;      // sin x = sin y, cos x = -cos y
    float y2 = y * y;
    float p = fmaf(fmaf(fmaf(fmaf(KEP_P4, y2, KEP_P3), y2, KEP_P2), y2, KEP_P1), y2, KEP_P0);
    float q = fmaf(fmaf(fmaf(fmaf(KEP_Q4, y2, KEP_Q3), y2, KEP_Q2), y2, KEP_Q1), y2, KEP_Q0);
    float yms = (y * y2) * p;
    float s = y - yms;
    float omc_y = y2 * q;
    SinCos32 r;
    r.s = s;
    r.omc = fold ? 2.0f - omc_y : omc_y;
    r.xms = fold ? x - s : yms;
    return r;
}

// Number of Danby iterations for eccentricity e in binary32 (offline schedule,
// worst error 1e-9 rad); 0 means "run the convergence-tested loop".
__device__ __forceinline__ int sched32(float e)
{
    return e <= (float)KEP_S32_E2 ? 2 : e <= (float)KEP_S32_E3 ? 3 : e <= (float)KEP_S32_E4 ? 4
         : e <= (float)KEP_S32_E5 ? 5 : 0;
}

__device__ __forceinline__ int sched64(double e)
{
    return e <= KEP_S64_E2 ? 2 : e <= KEP_S64_E3 ? 3 : e <= KEP_S64_E4 ? 4 : e <= KEP_S64_E5 ? 5 : 0;
}

// One Danby step (Sec. 4.3, quartic; Danby's third correction) on
// f(E) = E - e sin E - M written as (1-e) E + e (E - sin E) - M, with
// f' = (1-e) + e (1 - cos E), f'' = e sin E, f''' = e cos E.  The new iterate
// is kept in the bracket [M - e, M + e] that holds the root.  Returns the step
// and leaves sin E, 1 - cos E of the iterate it started from in `sc`.
__device__ __forceinline__ float danby_step32(float &E, float M, float e, float ome, float lo, float hi,
                                              SinCos32 &sc)
{
    sc = sincos32(E);
    float f = fmaf(ome, E, fmaf(e, sc.xms, -M));
    float f1 = fmaf(e, sc.omc, ome);
    float f2 = e * sc.s;
    float f3 = fmaf(-e, sc.omc, e);
    float d1 = -f * rcp32(f1);
    float d2 = -f * rcp32(fmaf(0.5f * d1, f2, f1));
    float den3 = fmaf(d2, fmaf(d2, f3 * (1.0f / 6.0f), 0.5f * f2), f1);
    float d3 = -f * rcp32(den3);
    float En = __builtin_amdgcn_fmed3f(E + d3, lo, hi);
    float step = En - E;
    E = En;
    return step;
}

// A Danby step for the iterations before the last one: sin and cos from the
// hardware transcendental unit (argument in revolutions) and f in its plain
// form.  Only the last step fixes the accuracy of the root (each step's error
// is the fourth power of the previous one, plus its own rounding), so the
// earlier steps may use cheaper, less accurate arithmetic.
__device__ __forceinline__ void danby_step32_fast(float &E, float M, float e, float lo, float hi)
{
    const float r = E * 0.159154943091895336f;
    const float s = __builtin_amdgcn_sinf(r);
    const float c = __builtin_amdgcn_cosf(r);
    float f = fmaf(-e, s, E - M);
    float f1 = fmaf(-e, c, 1.0f);
    float f2 = e * s;
    float f3 = e * c;
    float d1 = -f * rcp32(f1);
    float d2 = -f * rcp32(fmaf(0.5f * d1, f2, f1));
    float den3 = fmaf(d2, fmaf(d2, f3 * (1.0f / 6.0f), 0.5f * f2), f1);
    float d3 = -f * rcp32(den3);
    E = __builtin_amdgcn_fmed3f(E + d3, lo, hi);
}

// sin and 1 - cos at E + d from their values at E, with sin d and 1 - cos d
// from their Taylor series to d^3 and d^4 (after the first Kepler step |d| is
// below 0.05, so the dropped terms are below 1e-9): replaces a fresh
// evaluation after the last step.
__device__ __forceinline__ void rotate32(float &s, float &omc, float d)
{
    float d2 = d * d;
    float omcd = d2 * fmaf(d2, -1.0f / 24.0f, 0.5f);  // 1 - cos d
    float sd = d * fmaf(d2, -1.0f / 6.0f, 1.0f);       // sin d
    float s_new = fmaf(-s, omcd, fmaf(-omc, sd, s + sd));        // sin E cos d + cos E sin d
    float omc_new = fmaf(s, sd, fmaf(-omc, omcd, omc + omcd));   // 1 - (cos E cos d - sin E sin d)
    s = s_new;
    omc = omc_new;
}

// Kepler solve in binary32 for a centred mean anomaly M in [-pi, pi], from the
// paper's starting guess E0 = M + 0.85 e sign(M) (sign(sin M) on [-pi, pi]).
// niter > 0: that many steps; niter == 0: convergence test
// (|step| <= 2^-22 max(|E|, 1)) capped at max_iter (>= 1).  Returns E and
// sin E, 1 - cos E at the returned E.
__device__ __forceinline__ float kepler32(float M, float e, float ome, int niter, int max_iter, float &sinE,
                                          float &omcE)
{
    float lo = M - e, hi = M + e;
    float E = fmaf(copysignf(0.85f, M), e, M);
    SinCos32 sc;
    float st = 0.0f;
    const int n = niter > 0 ? niter : (max_iter > 0 ? max_iter : 1);
    for (int it = 0; it < n; ++it) {
        if (niter > 0 && it < n - 1) {
            danby_step32_fast(E, M, e, lo, hi);
            continue;
        }
        st = danby_step32(E, M, e, ome, lo, hi, sc);
        if (niter == 0 && fabsf(st) <= 2.384185791e-7f * fmaxf(fabsf(E), 1.0f)) break;
    }
    if (__any(fabsf(st) > 0.0625f)) {   // a large last step (e.g. a single fixed step): evaluate afresh
        sc = sincos32(E);
        st = 0.0f;
    }
    sinE = sc.s;
    omcE = sc.omc;
    rotate32(sinE, omcE, st);
    return E;
}

// Orbital phase in revolutions, centred on [-1/2, 1/2]:
// frac((t - t0)/P + M0/(2 pi)) with the quotient formed from a correctly
// rounded reciprocal and one residual correction (binary64, Sec. 5.1).  The
// integer part of the quotient is removed before M0 is added, so no bits of
// the fraction are lost at large epochs.
__device__ __forceinline__ double phase_rev(double tt, double P, double rP, double m0r)
{
    double q0 = tt * rP;
    double res = fma(-q0, P, tt);
    double q = fma(res, rP, q0);
    double fq = q - rint(q);
    double ph = fq + m0r;
    return ph - rint(ph);
}

// ----------------------------------------------------------------- binary64
// One Danby step in binary64 (the paper's iteration, Sec. 4.3), with IEEE
// divisions and the OCML double sincos; the iterate is kept in [M-e, M+e].
__device__ __forceinline__ double danby_step64(double &E, double M, double e, double lo, double hi)
{
    double s, c;
    sincos(E, &s, &c);
    double f = E - e * s - M;
    double f1 = 1.0 - e * c;
    double f2 = e * s;
    double f3 = e * c;
    double d1 = -f / f1;
    double d2 = -f / (f1 + 0.5 * d1 * f2);
    double d3 = -f / (f1 + 0.5 * d2 * f2 + d2 * d2 * f3 / 6.0);
    double En = fmin(fmax(E + d3, lo), hi);
    double step = En - E;
    E = En;
    return step;
}

// Kepler solve in binary64 for M in [0, 2 pi) (plain kernel) or any reduced M;
// starter E0 = M + 0.85 e sign(sin M) (Sec. 4.3).
// fixed > 0: exactly `fixed` steps; fixed == 0: binary64 schedule then
// convergence test (|step| <= 4 ulp) capped at max_iter.
__device__ __forceinline__ double kepler64(double M, double e, double sgn_sinM, int fixed, int max_iter)
{
    double lo = M - e, hi = M + e;
    double E = M + 0.85 * e * sgn_sinM;
    if (fixed > 0) {
        for (int it = 0; it < fixed; ++it) danby_step64(E, M, e, lo, hi);
    } else {
        int n = sched64(e);
        if (n > 0) {
            for (int it = 0; it < n; ++it) danby_step64(E, M, e, lo, hi);
        } else {
            for (int it = 0; it < max_iter; ++it) {
                double st = danby_step64(E, M, e, lo, hi);
                if (fabs(st) <= 8.9e-16 * fmax(fabs(E), 1.0)) break;
            }
        }
    }
    return E;
}

}  // namespace kep
