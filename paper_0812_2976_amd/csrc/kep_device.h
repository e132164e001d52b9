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

// A binary64 value moved across lanes by a DPP pattern (both halves with the same
// pattern; lanes of rows outside ROWS get 0).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double x)
{
    const int64_t b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
    return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

// Sum over the 64 lanes of a wavefront (every lane must be active), returned
// wave-uniform.  Data-parallel moves instead of LDS permutes: pairs (quad_perm
// 1,0,3,2), quads (2,3,0,1), half rows (row_half_mirror) and rows (row_mirror)
// leave every lane of a row with the row's sum; row_bcast15 adds row 0 into
// row 1 and row 2 into row 3, row_bcast31 rows 0-1 into row 3, so lane 63
// holds the total.
__device__ __forceinline__ double wave_sum(double x)
{
    x += dpp_f64<0xB1, 0xf>(x);    // quad_perm [1, 0, 3, 2]
    x += dpp_f64<0x4E, 0xf>(x);    // quad_perm [2, 3, 0, 1]
    x += dpp_f64<0x141, 0xf>(x);   // row_half_mirror
    x += dpp_f64<0x140, 0xf>(x);   // row_mirror
    x += dpp_f64<0x142, 0xa>(x);   // row_bcast15 into rows 1 and 3
    x += dpp_f64<0x143, 0xc>(x);   // row_bcast31 into rows 2 and 3
    const int64_t b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ float rcp32(float x) { return __builtin_amdgcn_rcpf(x); }

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

// The same three values for |x| <= 3.25 without folding the argument (the
// wider-range polynomials, one degree higher).  Valid for the last step of the
// eccentricity schedule, which starts within 0.015 rad of a root in
// [-pi, pi]; near +-pi, sin x = x - (x - sin x) keeps an absolute error of a
// few ulp of pi (the velocity needs no more).
__device__ __forceinline__ SinCos32 sincos32_wide(float x)
{
    const float x2 = x * x;
    const float p = fmaf(fmaf(fmaf(fmaf(fmaf(KEP_PW5, x2, KEP_PW4), x2, KEP_PW3), x2, KEP_PW2), x2, KEP_PW1), x2, KEP_PW0);
    const float q = fmaf(fmaf(fmaf(fmaf(fmaf(KEP_QW5, x2, KEP_QW4), x2, KEP_QW3), x2, KEP_QW2), x2, KEP_QW1), x2, KEP_QW0);
    const float x3 = x * x2;
    SinCos32 r;
    r.xms = x3 * p;
    r.s = fmaf(-x3, p, x);
    r.omc = x2 * q;
    return r;
}

// sin w and cos w of an angle whose products are rounded to binary32
// afterwards (the planet constants A and B of the mixed chi-square path): w
// reduced by the nearest multiple of 2 pi in binary64, then the binary32
// polynomials of sincos32 (|error| a few 1e-8, the size of the rounding of A
// and B themselves).  Its few registers keep the per-batch setup of the dense
// kernel within the five-wavefront register budget without scratch; the
// general binary64 routine needed 16 more registers there.
__device__ __forceinline__ void sincos_angle32(double w, double &s, double &c)
{
    const double kq = rint(w * kInvTwoPi);
    const float x = (float)fma(-kq, 2.4492935982947064e-16, fma(-kq, 6.283185307179586232, w));
    const SinCos32 r = sincos32(x);
    s = (double)r.s;
    c = (double)(1.0f - r.omc);
}

// Per-planet eccentricity constants of the binary32 Kepler step: e, 1 - e
// (rounded from binary64, so it keeps its relative precision as e -> 1), e/2
// and e/6 (the factors of f'' and f''' in Danby's corrections).
struct Ecc32 {
    float e, ome, eh, e6;
};

__device__ __forceinline__ Ecc32 make_ecc32(double e)
{
    Ecc32 k;
    k.e = (float)e;
    k.ome = (float)(1.0 - e);
    k.eh = (float)(0.5 * e);
    k.e6 = (float)(e * (1.0 / 6.0));
    return k;
}

// Number of Danby steps for eccentricity e in binary32 (offline schedule,
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

// Danby's three corrections (Sec. 4.3: Newton, Halley-like, quartic) from
// f and its derivatives f' = f1, f''/2 = f2h, f'''/6 = f3s.
// One reciprocal instead of three: d1 = -f/f1 makes the second denominator
// f1 + d1 f2h = N/f1 with N = f1^2 - f f2h, so d2 = -f f1/N, and the third
// denominator f1 + d2 (f2h + d2 f3s) = f1 (N^2 - f f2h N + f^2 f1 f3s)/N^2, so
//   d3 = -f N^2 / (f1 (N^2 - f f2h N + f^2 f1 f3s)).
// Same value as the three divisions (and the same vanishing denominator where
// the Halley-like step breaks down); a transcendental takes two binary32
// operations' issue slots and a longer latency, so four more multiply-adds for
// two fewer reciprocals is the cheaper form (measured: fewer cycles per step).
__device__ __forceinline__ float danby_delta(float f, float f1, float f2h, float f3s)
{
    const float g = f * f2h;
    const float N = fmaf(f1, f1, -g);
    const float N2 = N * N;
    const float den = f1 * fmaf(f * f1, f * f3s, fmaf(-g, N, N2));
    return -(f * N2) * rcp32(den);
}

// A Danby step for the iterations before the last one: sin and cos from the
// hardware transcendental unit (argument in revolutions) and f in its plain
// form.  Only the last step fixes the accuracy of the root (each step's error
// is about the fourth power of the previous one, plus its own rounding), so
// the earlier steps may use cheaper, less accurate arithmetic.  Within the
// schedule no clamp to the root's bracket is needed: the worst errors over
// the scanned (e, M) grid are the same with and without it.
__device__ __forceinline__ void danby_step32_fast(float &E, float M, const Ecc32 &k)
{
    const float r = E * 0.159154943091895336f;
    const float s = __builtin_amdgcn_sinf(r);
    const float c = __builtin_amdgcn_cosf(r);
    const float f = fmaf(-k.e, s, E - M);
    const float f1 = fmaf(-k.e, c, 1.0f);
    E += danby_delta(f, f1, k.eh * s, k.e6 * c);
}

// The accurate Danby step on f(E) = (1-e) E + e (E - sin E) - M, with
// f' = (1-e) + e (1 - cos E), f'' = e sin E, f''' = e cos E, all free of
// cancellation near periapsis.  Returns the step and leaves sin E, 1 - cos E
// of the iterate it started from in `sc`.  With CLAMP the new iterate is kept
// in [lo, hi]; the last step of the schedule starts within 0.015 of the root
// and needs no clamp.  WIDE: sin and cos from the unfolded wider-range
// polynomials (only where |E| <= 3.25 is guaranteed: the schedule's last step).
template <bool CLAMP, bool WIDE = false>
__device__ __forceinline__ float danby_step32(float &E, float M, const Ecc32 &k, float lo, float hi, SinCos32 &sc)
{
    sc = WIDE ? sincos32_wide(E) : sincos32(E);
    const float f = fmaf(k.ome, E, fmaf(k.e, sc.xms, -M));
    const float f1 = fmaf(k.e, sc.omc, k.ome);
    const float d3 = danby_delta(f, f1, k.eh * sc.s, fmaf(-k.e6, sc.omc, k.e6));
    const float En = CLAMP ? __builtin_amdgcn_fmed3f(E + d3, lo, hi) : E + d3;
    const float step = En - E;
    E = En;
    return step;
}

// The second-order member of Danby's family (Halley's correction) on the same
// cancellation-free f: d = -f / (f' + d1 f''/2) with d1 = -f/f', which is
// -f f' / (f'^2 - f f''/2).  Its error is about (f''^2/(4 f'^2) - f'''/(6 f')) d0^3
// for a start d0 from the root, so it replaces the quartic step only where the
// start is close enough (the table bands marked for it: within 1e-9 rad after
// the step).  Six operations and one reciprocal where the quartic step takes
// thirteen.  Returns the step (E becomes E + step) and leaves sin E,
// 1 - cos E of the iterate it started from in `sc`.
template <bool WIDE>
__device__ __forceinline__ float halley_step32(float &E, float M, const Ecc32 &k, SinCos32 &sc)
{
    sc = WIDE ? sincos32_wide(E) : sincos32(E);
    const float f = fmaf(k.ome, E, fmaf(k.e, sc.xms, -M));
    const float f1 = fmaf(k.e, sc.omc, k.ome);
    const float N = fmaf(f1, f1, -f * (k.eh * sc.s));
    const float step = -(f * f1) * rcp32(N);
    E += step;
    return step;
}

// rotate32 for steps |d| <= 2e-3 (the Halley bands of the table): sin d = d and
// 1 - cos d = d^2/2, whose dropped terms d^3/6 and d^4/24 are below 1.4e-9.
__device__ __forceinline__ void rotate32_small(float &s, float &omc, float d)
{
    const float omcd = (0.5f * d) * d;
    const float s_new = fmaf(-s, omcd, fmaf(-omc, d, s + d));
    const float omc_new = fmaf(s, d, fmaf(-omc, omcd, omc + omcd));
    s = s_new;
    omc = omc_new;
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
// niter > 0: that many steps (all but the last one cheap); niter == 0:
// accurate, clamped steps until |step| <= 2^-22 max(|E|, 1), at most max_iter.
// check_large: the step count was fixed by the caller rather than the
// schedule.  Returns E and sin E, 1 - cos E at the returned E.
__device__ __forceinline__ float kepler32(float M, const Ecc32 &k, int niter, int max_iter, bool check_large,
                                          float &sinE, float &omcE)
{
    float E = fmaf(copysignf(0.85f, M), k.e, M);
    SinCos32 sc;
    float st = 0.0f;
    if (niter > 0) {
        for (int it = 0; it < niter - 1; ++it) danby_step32_fast(E, M, k);
        // a step count fixed by the caller does not bound the last iterate
        st = check_large ? danby_step32<false>(E, M, k, 0.0f, 0.0f, sc)
                         : danby_step32<false, true>(E, M, k, 0.0f, 0.0f, sc);
    } else {
        check_large = true;
        const float lo = M - k.e, hi = M + k.e;
        const int n = max_iter > 0 ? max_iter : 1;
        for (int it = 0; it < n; ++it) {
            st = danby_step32<true>(E, M, k, lo, hi, sc);
            if (fabsf(st) <= 2.384185791e-7f * fmaxf(fabsf(E), 1.0f)) break;
        }
    }
    // The schedule guarantees a last step below 0.05; a caller-fixed step count
    // or an unconverged loop may not: then evaluate afresh instead of rotating.
    if (check_large && __any(fabsf(st) > 0.0625f)) {
        sc = sincos32(E);
        st = 0.0f;
    }
    sinE = sc.s;
    omcE = sc.omc;
    rotate32(sinE, omcE, st);
    return E;
}

// sin x and cos x in binary64 without the general routine's large-argument
// machinery: x is reduced by the nearest multiple of 2 pi (2 pi in two parts;
// exact for |x| < pi, and within an ulp of x up to |x| ~ 1e6, the precision x
// itself carries there), folded to |y| <= pi / 2 with y = +-(pi - |x|), pi in
// two parts (the first subtraction is exact for pi / 2 <= |x| <= 2 pi), and the
// Taylor series of sin to y^21 and of cos to y^22 are summed by Horner's rule
// (remainders below 2e-17 on |y| <= pi / 2; n! is exact in binary64 up to 22!,
// so each coefficient 1/n! is correctly rounded).  For Kepler roots of a
// centred mean anomaly (the astrometric correction step); the plain binary64
// path keeps the general routine.
__device__ __forceinline__ void sincos_reduced(double x, double &s, double &c)
{
    constexpr double kPiHi = 3.141592653589793116;
    constexpr double kPiLo = 1.2246467991473532e-16;
    const double kq = rint(x * kInvTwoPi);
    x = fma(-kq, 2.0 * kPiLo, fma(-kq, 2.0 * kPiHi, x));
    const double ax = fabs(x);
    const bool fold = ax > 1.5707963267948966;
    const double yf = (kPiHi - ax) + kPiLo;
    const double y = fold ? (x < 0.0 ? -yf : yf) : x;
    const double y2 = y * y;
    double ps = -1.0 / 51090942171709440000.0;               // 1/21!
    ps = fma(ps, y2, 1.0 / 121645100408832000.0);            // 1/19!
    ps = fma(ps, y2, -1.0 / 355687428096000.0);              // 1/17!
    ps = fma(ps, y2, 1.0 / 1307674368000.0);                 // 1/15!
    ps = fma(ps, y2, -1.0 / 6227020800.0);                   // 1/13!
    ps = fma(ps, y2, 1.0 / 39916800.0);                      // 1/11!
    ps = fma(ps, y2, -1.0 / 362880.0);                       // 1/9!
    ps = fma(ps, y2, 1.0 / 5040.0);                          // 1/7!
    ps = fma(ps, y2, -1.0 / 120.0);                          // 1/5!
    ps = fma(ps, y2, 1.0 / 6.0);                             // 1/3!
    double pc = 1.0 / 1124000727777607680000.0;              // 1/22!
    pc = fma(pc, y2, -1.0 / 2432902008176640000.0);          // 1/20!
    pc = fma(pc, y2, 1.0 / 6402373705728000.0);              // 1/18!
    pc = fma(pc, y2, -1.0 / 20922789888000.0);               // 1/16!
    pc = fma(pc, y2, 1.0 / 87178291200.0);                   // 1/14!
    pc = fma(pc, y2, -1.0 / 479001600.0);                    // 1/12!
    pc = fma(pc, y2, 1.0 / 3628800.0);                       // 1/10!
    pc = fma(pc, y2, -1.0 / 40320.0);                        // 1/8!
    pc = fma(pc, y2, 1.0 / 720.0);                           // 1/6!
    pc = fma(pc, y2, -1.0 / 24.0);                           // 1/4!
    pc = fma(pc, y2, 0.5);                                   // 1/2!
    s = fma(-y * y2, ps, y);                                 // y - y^3 (1/3! - y^2/5! + ...)
    const double cy = fma(-y2, pc, 1.0);                     // 1 - y^2 (1/2! - y^2/4! + ...)
    c = fold ? -cy : cy;
}

// Per-planet constants of the binary64 orbital phase: P, 1/P (correctly
// rounded) and fract(M0/(2 pi) + 1/2).
struct Phase64 {
    double P, rP, m0h;
};

__device__ __forceinline__ Phase64 make_phase64(double P, double M0)
{
    Phase64 p;
    p.P = P;
    p.rP = 1.0 / P;
    p.m0h = __builtin_amdgcn_fract(fma(M0, kInvTwoPi, 0.5));
    return p;
}

// Mean anomaly centred on [-pi, pi) (Sec. 4.2, Eq. 6, with the bracket in
// binary64 as in Sec. 5.1), rounded to binary32 only at the end:
// M = 2 pi (fract(q + fract(M0/(2 pi) + 1/2)) - 1/2), q = (t - t0) (1/P) with
// the correctly rounded 1/P.  q carries at most about two ulps of error and
// adding the phase offset one more rounding at the magnitude of q: at the
// largest epochs of the workloads (q ~ 2.5e6 cycles) that is 4.4e-9 rad, well
// below binary32's resolution of M (1.2e-7 rad near pi), so no correction
// step is spent on it.
// The same without P, for records that only need the centred phase.
struct PhaseM {
    double rP, m0h;
};

__device__ __forceinline__ PhaseM make_phasem(double P, double M0)
{
    PhaseM p;
    p.rP = 1.0 / P;
    p.m0h = __builtin_amdgcn_fract(fma(M0, kInvTwoPi, 0.5));
    return p;
}

template <class Ph>
__device__ __forceinline__ float mean_anomaly32(double tt, const Ph &p)
{
    return (float)fma(__builtin_amdgcn_fract(fma(tt, p.rP, p.m0h)), kTwoPi, -kPi);
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
