// Per-precision policies of the dense kernels: the planet record built once
// per (system, planet), the observation record held in registers, and the
// arithmetic of one planet's velocity and of the chi-square accumulation, for
// the mixed-precision path (Sec. 5.1) and the plain binary64 path.  Shared by
// the dense chi-square kernels and the population sampler's fused half-step.
#pragma once

#include <hip/hip_runtime.h>

#include "kep_device.h"
#include "kep_internal.h"
#include "kep_start_tab.h"

namespace kep {

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bool planet_ok(double P, double K, double e, double w, double M0)
{
    return isfinite(P) && P > 0.0 && isfinite(K) && isfinite(e) && e >= 0.0 && e < 1.0 &&
           isfinite(w) && isfinite(M0);
}

// The two binary16 halves of a table word, widened to binary32.
__device__ __forceinline__ float half_lo(uint32_t w) { return (float)__builtin_bit_cast(_Float16, (uint16_t)w); }
__device__ __forceinline__ float half_hi(uint32_t w)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
}

// The starting-value table (Sec. 5.4's interpolated guess; kep_start_tab.h):
// bands of eccentricity, each with its rows, knots in |M| and last step.
constexpr int kTabWords = KEP_TAB_WORDS;
constexpr int kTabBands = KEP_TAB_NBANDS;
constexpr double kTabE0[kTabBands] = KEP_TAB_BAND_E0;
constexpr double kTabE1[kTabBands] = KEP_TAB_BAND_E1;
constexpr int kTabRows[kTabBands] = KEP_TAB_BAND_ROWS;
constexpr int kTabKnots[kTabBands] = KEP_TAB_BAND_KNOTS;
constexpr int kTabOff[kTabBands] = KEP_TAB_BAND_OFF;
constexpr int kTabHalley[kTabBands] = KEP_TAB_BAND_HALLEY;

// A planet's place in the table: the word offset of its row, the weight of the
// next eccentricity row, the band's knots per radian of |M| and its last step.
struct TabPlace {
    float twe;       // weight of the next eccentricity row
    float mscale;    // knots / pi
    int16_t toff;    // word offset of the row; -1: outside the table
    int8_t halley;   // 1: Halley's step from the start, 0: Danby's quartic one
    int8_t pad;
};

// The table place of eccentricity e (binary64, as given); outside the table, or
// when the caller fixes the step count (use = false), toff is -1.
__device__ __forceinline__ TabPlace table_place(double e, bool use)
{
    TabPlace t;
    t.twe = 0.0f;
    t.mscale = 0.0f;
    t.toff = -1;
    t.halley = 0;
    t.pad = 0;
    if (!use || !(e >= 0.0 && e <= KEP_TAB_EMAX)) return t;
    int band = 0;
#pragma unroll
    for (int b = 1; b < kTabBands; ++b) band = e >= kTabE0[b] ? b : band;
#pragma unroll
    for (int b = 0; b < kTabBands; ++b) {
        if (b == band) {
            const double fi = (e - kTabE0[b]) * (kTabRows[b] / (kTabE1[b] - kTabE0[b]));
            const int i = min((int)fi, kTabRows[b] - 1);
            t.twe = (float)(fi - i);
            t.mscale = (float)(kTabKnots[b] / kPi);
            t.toff = (int16_t)(kTabOff[b] + i * (kTabKnots[b] + 2));
            t.halley = (int8_t)kTabHalley[b];
        }
    }
    return t;
}

// Copy of the table into a block's LDS; every thread of the block calls it
// before any wave reads the table (it ends with the block barrier).
__device__ __forceinline__ void load_start_table(uint32_t *dst)
{
    for (int q = threadIdx.x; q < kTabWords; q += blockDim.x) dst[q] = kep_start_tab[q];
    __syncthreads();
}

// Knot of |M| and its fraction for mscale = knots / pi.  M is the centred phase
// (|M| <= binary32 pi, so j <= knots) or NaN; v_cvt_i32_f32 turns a NaN into 0
// (an IEEE-undefined conversion in C++, hence the instruction itself), so the
// two words j, j + 1 read after it stay inside the row of knots + 2 words
// without a clamp.
__device__ __forceinline__ int start_knot(float M, float mscale, float &wm)
{
    const float fj = fabsf(M) * mscale;
    wm = __builtin_amdgcn_fractf(fj);
    int j;
    __asm__("v_cvt_i32_f32 %0, %1" : "=v"(j) : "v"(fj));
    return j;
}

// Bilinear starting value from the words of knots j and j + 1 of a row:
// weight twe towards the next eccentricity row, wm towards knot j + 1, sign of M.
__device__ __forceinline__ float start_value(uint32_t w0, uint32_t w1, float twe, float wm, float M)
{
    const float r0 = fmaf(twe, half_hi(w0), half_lo(w0));
    const float r1 = fmaf(twe, half_hi(w1), half_lo(w1));
    return copysignf(fmaf(wm, r1 - r0, r0), M);
}

// Kepler solve of one lane for kernels whose lanes hold different planets: from
// the LDS starting-value table at the planet's place and one step, else
// kepler32.  The step is Halley's when every lane taking the table start has
// its planet in a Halley band, else Danby's quartic step for all of them (valid
// in every band), so the choice never splits the wavefront.  Returns E and
// sin E, 1 - cos E.
__device__ __forceinline__ float kepler32_start(float M, const Ecc32 &k, const TabPlace &tp, const uint32_t *tab,
                                                int niter, int max_iter, bool check, float &sinE, float &omcE)
{
    if (tab != nullptr && tp.toff >= 0) {
        float wm;
        const uint32_t *q = tab + tp.toff + start_knot(M, tp.mscale, wm);
        float E = start_value(q[0], q[1], tp.twe, wm, M);
        SinCos32 sc;
        if (__all(tp.halley != 0)) {
            const float d = halley_step32<true>(E, M, k, sc);
            sinE = sc.s;
            omcE = sc.omc;
            rotate32_small(sinE, omcE, d);
        } else {
            const float st = danby_step32<false, true>(E, M, k, 0.0f, 0.0f, sc);
            sinE = sc.s;
            omcE = sc.omc;
            rotate32(sinE, omcE, st);
        }
        return E;
    }
    return kepler32(M, k, niter, max_iter, check, sinE, omcE);
}

// ------------------------------------------------------------------ mixed
struct RecMixed {          // 56 bytes, one per (system, planet)
    PhaseM ph;             // 1/P, fract(M0/(2 pi) + 1/2)
    Ecc32 k;               // e, 1 - e, e/2, e/6
    float A, B;            // K b^2 cos w, -K b sin w  (b = sqrt(1 - e^2))
    TabPlace tp;           // place in the starting-value table (toff -1: the paper's guess)
    int16_t niter;         // Danby steps from the paper's guess (0: convergence test)
    int8_t check;          // 1 if the step count is fixed by the caller
    int8_t pad;
};
static_assert(sizeof(RecMixed) == 56, "planet record size");

struct ObsMixed {
    double tt;   // t - t0
    double v;    // observed velocity
    float s2;    // sigma^2
    float w;     // 1 / sigma^2 (no jitter)
    bool in;     // lane holds a real observation
    bool ok;     // t, v, sigma finite and sigma >= 0
};

struct PolMixed {
    static constexpr bool kMixed = true;
    using Rec = RecMixed;
    using Obs = ObsMixed;
    // the planet sum in binary64: each binary32 velocity is added exactly (two
    // instructions a planet, where a Kahan pair takes four), so the sum carries
    // only the rounding of the velocities themselves
    struct ModelAcc {
        double s;
        __device__ __forceinline__ void add(float v) { s += (double)v; }
    };
    // the chi-square terms w r^2 (binary32 weight times the binary64 residual)
    // summed in binary64: no less accurate than the compensated binary32 sum of
    // Sec. 4.4 and two instructions fewer per observation
    struct ChiAcc { double s; };

    static __device__ __forceinline__ bool setup(const DenseArgs &a, double P, double K, double e, double w,
                                                 double M0, Rec &r)
    {
        bool ok = planet_ok(P, K, e, w, M0);
        if (!ok) { P = 1.0; K = 0.0; e = 0.0; w = 0.0; M0 = 0.0; }
        r.ph = make_phasem(P, M0);
        r.k = make_ecc32(e);
        const double b2 = (1.0 - e) * (1.0 + e);
        double sw, cw;
        sincos_angle32(w, sw, cw);
        r.A = (float)(K * b2 * cw);
        r.B = (float)(-K * sqrt(b2) * sw);
        r.niter = (int16_t)(a.fixed_iter > 0 ? a.fixed_iter : sched32(r.k.e));
        r.check = a.fixed_iter > 0 ? 1 : 0;
        r.pad = 0;
        // kernels that hold the table start from it (one step) at e <= KEP_TAB_EMAX
        r.tp = table_place(e, a.fixed_iter <= 0);
        return ok;
    }

    static __device__ __forceinline__ void load_obs(const DenseArgs &a, int64_t k, Obs &o)
    {
        o.in = k < a.n_obs;
        double t = o.in ? a.t[k] : a.t0;
        double v = o.in ? a.v[k] : 0.0;
        double s = o.in ? a.sigma[k] : 1.0;
        o.ok = isfinite(t) && isfinite(v) && isfinite(s) && s >= 0.0;
        o.tt = t - a.t0;
        o.v = v;
        o.s2 = (float)(s * s);
        o.w = (float)(1.0 / (s * s));
    }

    static __device__ __forceinline__ void load_obs_model(const DenseArgs &a, int64_t k, Obs &o)
    {
        o.in = k < a.n_obs;
        double t = o.in ? a.t[k] : a.t0;
        o.ok = isfinite(t);
        o.tt = t - a.t0;
        o.v = 0.0;
        o.s2 = 1.0f;
        o.w = 1.0f;
    }

    // Kepler solve of NCH chunks of one planet (wave-uniform constants): E, and
    // sin E, 1 - cos E at E.  From the starting-value table where the planet has
    // a place in it (one accurate step: Halley's correction in the bands marked
    // for it, Danby's quartic one in the others), else the paper's guess and the
    // eccentricity schedule (or a caller-fixed count, or the convergence-tested
    // loop).  tab: the starting-value table in LDS (the words of kep_start_tab), or null.
    // ROTATE = false: E only (s and omc are left unset).
    template <int NCH, bool ROTATE = true>
    static __device__ __forceinline__ void solve(const Ecc32 &k, int niter, bool check, const TabPlace &tp,
                                                 const float (&M)[NCH], float (&E)[NCH], float (&s)[NCH],
                                                 float (&omc)[NCH], int max_iter, const uint32_t *tab)
    {
        float st[NCH];
        SinCos32 sc[NCH];
        const int toff = uniform_int(tp.toff);
        if (tab != nullptr && toff >= 0) {
            // tabulated starting value (the paper's interpolated initial guess, Sec. 5.4):
            // bilinear in (e, |M|) within 3.7e-3 rad of the root, close enough for the
            // accurate last step alone (4.5e-11 rad in float64; scan in gen_tables.py)
            // (every chunk's reads are issued before any is used)
            const uint32_t *row = tab + toff;
            float wm[NCH];
            uint32_t q0[NCH], q1[NCH];
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const uint32_t *q = row + start_knot(M[c], tp.mscale, wm[c]);
                q0[c] = q[0];                          // binary16 (E_i, E_i+1 - E_i) at knot j
                q1[c] = q[1];
            }
#pragma unroll
            for (int c = 0; c < NCH; ++c) E[c] = start_value(q0[c], q1[c], tp.twe, wm[c], M[c]);
            if (uniform_int(tp.halley) != 0) {
                // bands whose start lies within 1.3e-3 rad: the second-order step
                // suffices (1e-9 rad), and the rotation by it needs two terms
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    const float d = halley_step32<true>(E[c], M[c], k, sc[c]);
                    if constexpr (ROTATE) {
                        s[c] = sc[c].s;
                        omc[c] = sc[c].omc;
                        rotate32_small(s[c], omc[c], d);
                    }
                }
                return;
            }
#pragma unroll
            for (int c = 0; c < NCH; ++c) st[c] = danby_step32<false, true>(E[c], M[c], k, 0.0f, 0.0f, sc[c]);
        } else if (niter > 0) {
#pragma unroll
            for (int c = 0; c < NCH; ++c) E[c] = fmaf(copysignf(0.85f, M[c]), k.e, M[c]);
            for (int it = 0; it < niter - 1; ++it) {   // steps before the last: hardware sin/cos
#pragma unroll
                for (int c = 0; c < NCH; ++c) danby_step32_fast(E[c], M[c], k);
            }
            if (!check) {                              // the schedule bounds the last iterate
#pragma unroll
                for (int c = 0; c < NCH; ++c) st[c] = danby_step32<false, true>(E[c], M[c], k, 0.0f, 0.0f, sc[c]);
            } else {
#pragma unroll
                for (int c = 0; c < NCH; ++c) st[c] = danby_step32<false>(E[c], M[c], k, 0.0f, 0.0f, sc[c]);
            }
        } else {
#pragma unroll
            for (int c = 0; c < NCH; ++c) E[c] = fmaf(copysignf(0.85f, M[c]), k.e, M[c]);
            check = true;
            const int n = max_iter > 0 ? max_iter : 1;
            for (int it = 0; it < n; ++it) {           // convergence-tested (beyond the schedule),
                bool conv = true;                      // clamped to the bracket [M - e, M + e]
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    st[c] = danby_step32<true>(E[c], M[c], k, M[c] - k.e, M[c] + k.e, sc[c]);
                    conv = conv && (fabsf(st[c]) <= 2.384185791e-7f * fmaxf(fabsf(E[c]), 1.0f));
                }
                if (__all(conv)) break;
            }
        }
        if constexpr (!ROTATE) return;
        if (check) {   // a last step the schedule does not bound: evaluate afresh where it is large
            bool large = false;
#pragma unroll
            for (int c = 0; c < NCH; ++c) large = large || fabsf(st[c]) > 0.0625f;
            if (__any(large)) {
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    sc[c] = sincos32(E[c]);
                    st[c] = 0.0f;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            s[c] = sc[c].s;
            omc[c] = sc[c].omc;
            rotate32(s[c], omc[c], st[c]);
        }
    }

    // tab: the starting-value table in LDS (the words of kep_start_tab), or null
    template <int NCH>
    static __device__ __forceinline__ void add_planet(const Rec &rr, const Obs (&o)[NCH], ModelAcc (&m)[NCH],
                                                      int max_iter, int /*fixed: already in rr.niter*/,
                                                      const uint32_t *tab = nullptr)
    {
        // rr comes from an LDS broadcast: every lane holds the same values
        const PhaseM ph = rr.ph;
        const Ecc32 k = rr.k;
        const float A = rr.A, B = rr.B;
        float M[NCH], E[NCH], s[NCH], omc[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) M[c] = mean_anomaly32(o[c].tt, ph);
        solve<NCH>(k, uniform_int(rr.niter), uniform_int(rr.check) != 0, rr.tp, M, E, s, omc, max_iter, tab);
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            float D = fmaf(k.e, omc[c], k.ome);              // 1 - e cos E
            float num = fmaf(B, s[c], fmaf(-A, omc[c], A));  // A cos E + B sin E
            m[c].add(num * rcp32(D));
        }
    }

    static __device__ __forceinline__ void model_init(ModelAcc &m) { m.s = 0.0; }
    static __device__ __forceinline__ double model_value(const ModelAcc &m) { return m.s; }

    static __device__ __forceinline__ void chi_init(ChiAcc &x) { x.s = 0.0; }
    // One observation's contribution; returns false if the weight is invalid.
    static __device__ __forceinline__ bool chi_add(ChiAcc &x, const ModelAcc &m, const Obs &o, double gam,
                                                   double jit, bool has_jit)
    {
        const double r = (m.s + gam) - o.v;   // residual formed in binary64
        float w = o.w;
        bool okw = true;
        if (has_jit) {
            float var = o.s2 + (float)(jit * jit);
            okw = var > 0.0f;
            w = rcp32(var);
        } else {
            okw = o.s2 > 0.0f;
        }
        x.s = fma((double)(w * (float)r), r, x.s);
        return okw;
    }
    static __device__ __forceinline__ double chi_value(const ChiAcc &x) { return x.s; }
};

// ------------------------------------------------------------------ binary64
struct Rec64 {            // 64 bytes
    double P, M0, e, K, b, cw, sw;
    int pad0, pad1;
};

struct Obs64 {
    double tt, v, s2, w;
    bool in, ok;
};

struct Pol64 {
    static constexpr bool kMixed = false;
    using Rec = Rec64;
    using Obs = Obs64;
    struct ModelAcc { double s; };
    using ChiAcc = double;

    static __device__ __forceinline__ bool setup(const DenseArgs &, double P, double K, double e, double w,
                                                 double M0, Rec &r)
    {
        bool ok = planet_ok(P, K, e, w, M0);
        if (!ok) { P = 1.0; K = 0.0; e = 0.0; w = 0.0; M0 = 0.0; }
        r.P = P;
        r.M0 = M0;
        r.e = e;
        r.K = K;
        r.b = sqrt((1.0 - e) * (1.0 + e));
        sincos(w, &r.sw, &r.cw);
        r.pad0 = r.pad1 = 0;
        return ok;
    }

    static __device__ __forceinline__ void load_obs(const DenseArgs &a, int64_t k, Obs &o)
    {
        o.in = k < a.n_obs;
        double t = o.in ? a.t[k] : a.t0;
        double v = o.in ? a.v[k] : 0.0;
        double s = o.in ? a.sigma[k] : 1.0;
        o.ok = isfinite(t) && isfinite(v) && isfinite(s) && s >= 0.0;
        o.tt = t - a.t0;
        o.v = v;
        o.s2 = s * s;
        o.w = 1.0 / (s * s);
    }

    static __device__ __forceinline__ void load_obs_model(const DenseArgs &a, int64_t k, Obs &o)
    {
        o.in = k < a.n_obs;
        double t = o.in ? a.t[k] : a.t0;
        o.ok = isfinite(t);
        o.tt = t - a.t0;
        o.v = 0.0;
        o.s2 = 1.0;
        o.w = 1.0;
    }

    // Plain binary64 (the paper's double-precision variant): IEEE quotient
    // (t - t0)/P, exact fraction, M = 2 pi frac + M0 in [0, 2 pi), Danby's
    // iteration, then v = K b (b cos w cos E - sin w sin E) / (1 - e cos E).
    template <int NCH>
    static __device__ __forceinline__ void add_planet(const Rec &rr, const Obs (&o)[NCH], ModelAcc (&m)[NCH],
                                                      int max_iter, int fixed)
    {
        const double P = uniform_double(rr.P), M0 = uniform_double(rr.M0), e = uniform_double(rr.e);
        const double K = uniform_double(rr.K), b = uniform_double(rr.b);
        const double cw = uniform_double(rr.cw), sw = uniform_double(rr.sw);
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            double q = o[c].tt / P;
            double phi = q - floor(q);
            double M = fma(kTwoPi, phi, M0);
            M = M - kTwoPi * floor(M * kInvTwoPi);
            double E = kepler64(M, e, M < kPi ? 1.0 : -1.0, fixed, max_iter);
            double s, cE;
            sincos(E, &s, &cE);
            m[c].s += K * b * (b * cw * cE - sw * s) / (1.0 - e * cE);
        }
    }

    static __device__ __forceinline__ void model_init(ModelAcc &m) { m.s = 0.0; }
    static __device__ __forceinline__ double model_value(const ModelAcc &m) { return m.s; }
    static __device__ __forceinline__ void chi_init(ChiAcc &x) { x = 0.0; }
    static __device__ __forceinline__ bool chi_add(ChiAcc &x, const ModelAcc &m, const Obs &o, double gam,
                                                   double jit, bool has_jit)
    {
        double r = m.s + gam - o.v;
        double w = o.w;
        bool okw = o.s2 > 0.0;
        if (has_jit) {
            double var = o.s2 + jit * jit;
            okw = var > 0.0;
            w = 1.0 / var;
        }
        x = fma(w * r, r, x);
        return okw;
    }
    static __device__ __forceinline__ double chi_value(const ChiAcc &x) { return x; }
};

// Iteration count of the plain binary64 kernel: fixed_iter > 0 as given,
// 0 -> the fixed 30 steps of the plain kernel, < 0 -> schedule + convergence test.
__device__ __forceinline__ int fixed64(int fixed_iter) { return fixed_iter > 0 ? fixed_iter : (fixed_iter == 0 ? 30 : 0); }

template <class Pol, int NCH>
__device__ __forceinline__ void pol_add_planet(const typename Pol::Rec &r, const typename Pol::Obs (&o)[NCH],
                                               typename Pol::ModelAcc (&m)[NCH], const DenseArgs &a,
                                               const uint32_t *tab = nullptr)
{
    if constexpr (Pol::kMixed) Pol::template add_planet<NCH>(r, o, m, a.max_iter, 0, tab);
    else Pol::template add_planet<NCH>(r, o, m, a.max_iter, fixed64(a.fixed_iter));
}

// Dense kernel.  MODE kChi2: chi-square per system; kModel: model velocities
// [n_sys][n_obs]; kPlanets: every planet's velocity [n_pl][n_sys][n_obs] in
// binary32 (the paper's separate-function form, Sec. 4.4, first implementation);
// kAnomalies: every planet's eccentric anomaly [n_pl][n_sys][n_obs] in binary32
// (the paper's first mixed-precision use of the GPU, Kepler's equation only,
// Sec. 5.2; mixed policy only).
enum { kChi2 = 0, kModel = 1, kPlanets = 2, kAnomalies = 3 };


}  // namespace kep
