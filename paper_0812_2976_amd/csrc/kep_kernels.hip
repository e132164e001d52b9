// gfx950 kernels for batched Keplerian radial-velocity models (Ford 2008).
//
// Dense batches (every system sees the same n_obs observations) use one
// wavefront per system at a time with the 64 lanes spread over observations:
// lane l evaluates observations l, l + 64, ... (NCH chunks held in registers
// for the whole launch), so every parameter a lane needs is wave-uniform and
// the eccentricity schedule of the Kepler solve is uniform across the wave.
// Per-planet constants (reciprocal period, phase offset, amplitudes) are
// computed with the lanes spread over systems instead -- one lane per system
// for a batch of up to 32 systems -- and handed over through the wave's slice
// of LDS, so that setup is paid once per system rather than once per lane.
// The chi-square is reduced across the wave in binary64 (Sec. 4.4's final sum).
#include <hip/hip_runtime.h>

#include "kep_device.h"
#include "kep_internal.h"
#include "kep_philox.h"

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

// ------------------------------------------------------------------ mixed
struct RecMixed {          // 64 bytes, one per (system, planet)
    Phase64 ph;            // P, 1/P, fract(M0/(2 pi) + 1/2)
    Ecc32 k;               // e, 1 - e, e/2, e/6
    float A, B;            // K b^2 cos w, -K b sin w  (b = sqrt(1 - e^2))
    int niter, check;      // Danby steps (0: convergence test); 1 if fixed by the caller
};

struct ObsMixed {
    double tt;   // t - t0
    double v;    // observed velocity
    float s2;    // sigma^2
    float w;     // 1 / sigma^2 (no jitter)
    bool in;     // lane holds a real observation
    bool ok;     // t, v, sigma finite and sigma >= 0
};

struct PolMixed {
    using Rec = RecMixed;
    using Obs = ObsMixed;
    struct ModelAcc { Kahan32 k; };
    using ChiAcc = Kahan32;

    static __device__ __forceinline__ bool setup(const DenseArgs &a, double P, double K, double e, double w,
                                                 double M0, Rec &r)
    {
        bool ok = planet_ok(P, K, e, w, M0);
        if (!ok) { P = 1.0; K = 0.0; e = 0.0; w = 0.0; M0 = 0.0; }
        r.ph = make_phase64(P, M0);
        r.k = make_ecc32(e);
        const double b2 = (1.0 - e) * (1.0 + e);
        double sw, cw;
        sincos(w, &sw, &cw);
        r.A = (float)(K * b2 * cw);
        r.B = (float)(-K * sqrt(b2) * sw);
        r.niter = a.fixed_iter > 0 ? a.fixed_iter : sched32(r.k.e);
        r.check = a.fixed_iter > 0 ? 1 : 0;
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

    template <int NCH>
    static __device__ __forceinline__ void add_planet(const Rec &rr, const Obs (&o)[NCH], ModelAcc (&m)[NCH],
                                                      int max_iter, int /*fixed: already in rr.niter*/)
    {
        // rr comes from an LDS broadcast: every lane holds the same values
        const Phase64 ph = rr.ph;
        const Ecc32 k = rr.k;
        const float A = rr.A, B = rr.B;
        const int niter = uniform_int(rr.niter);
        float M[NCH], E[NCH], st[NCH];
        SinCos32 sc[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            M[c] = mean_anomaly32(o[c].tt, ph);
            E[c] = fmaf(copysignf(0.85f, M[c]), k.e, M[c]);
        }
        bool check = uniform_int(rr.check) != 0;
        if (niter > 0) {
            for (int it = 0; it < niter - 1; ++it) {   // steps before the last: hardware sin/cos
#pragma unroll
                for (int c = 0; c < NCH; ++c) danby_step32_fast(E[c], M[c], k);
            }
#pragma unroll
            for (int c = 0; c < NCH; ++c) st[c] = danby_step32<false>(E[c], M[c], k, 0.0f, 0.0f, sc[c]);
        } else {
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
            float s = sc[c].s, omc = sc[c].omc;
            rotate32(s, omc, st[c]);
            float D = fmaf(k.e, omc, k.ome);           // 1 - e cos E
            float num = fmaf(B, s, fmaf(-A, omc, A));  // A cos E + B sin E
            m[c].k.add(num * rcp32(D));
        }
    }

    static __device__ __forceinline__ void model_init(ModelAcc &m) { m.k.init(); }
    static __device__ __forceinline__ double model_value(const ModelAcc &m) { return m.k.value(); }

    static __device__ __forceinline__ void chi_init(ChiAcc &x) { x.init(); }
    // One observation's contribution; returns false if the weight is invalid.
    static __device__ __forceinline__ bool chi_add(ChiAcc &x, const ModelAcc &m, const Obs &o, double gam,
                                                   double jit, bool has_jit)
    {
        float r = (float)(((double)m.k.s - (double)m.k.c + gam) - o.v);   // residual formed in binary64
        float w = o.w;
        bool okw = true;
        if (has_jit) {
            float var = o.s2 + (float)(jit * jit);
            okw = var > 0.0f;
            w = rcp32(var);
        } else {
            okw = o.s2 > 0.0f;
        }
        x.add(w * r * r);
        return okw;
    }
    static __device__ __forceinline__ double chi_value(const ChiAcc &x) { return x.value(); }
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
                                               typename Pol::ModelAcc (&m)[NCH], const DenseArgs &a)
{
    Pol::template add_planet<NCH>(r, o, m, a.max_iter, fixed64(a.fixed_iter));
}

// Dense kernel.  MODE kChi2: chi-square per system; kModel: model velocities
// [n_sys][n_obs]; kPlanets: every planet's velocity [n_pl][n_sys][n_obs] in
// binary32 (the paper's separate-function form, Sec. 4.4, first implementation).
enum { kChi2 = 0, kModel = 1, kPlanets = 2 };

template <class Pol, int NCH, int MODE>

__global__ void __launch_bounds__(256) k_dense(DenseArgs a)
{
    using Rec = typename Pol::Rec;
    using Obs = typename Pol::Obs;
    using ModelAcc = typename Pol::ModelAcc;
    extern __shared__ __align__(16) unsigned char smem[];

    const int lane = __lane_id();
    const int wpb = blockDim.x >> 6;
    const int wib = uniform_int(threadIdx.x >> 6);
    Rec *recs = reinterpret_cast<Rec *>(smem) + (size_t)wib * a.sb * a.n_pl;
    int *sysbad = reinterpret_cast<int *>(smem + (size_t)wpb * a.sb * a.n_pl * sizeof(Rec)) + wib * a.sb;

    const int64_t gw = (int64_t)blockIdx.x * wpb + wib;
    const int64_t n_waves = (int64_t)gridDim.x * wpb;
    const int64_t n_batches = (a.n_sys + a.sb - 1) / a.sb;
    const int n_groups = (int)((a.n_obs + 64 * NCH - 1) / (64 * NCH));
    const bool has_jit = a.jitter != nullptr;

    Obs o[NCH];
    auto load_group = [&](int g) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            int64_t k = (int64_t)g * 64 * NCH + c * 64 + lane;
            if (MODE != kChi2) Pol::load_obs_model(a, k, o[c]);
            else Pol::load_obs(a, k, o[c]);
        }
    };
    if (n_groups <= 1) load_group(0);

    // Velocities need no reduction over observations, so their work items are
    // (batch, observation group) pairs: a few systems with very many
    // observations still spread over the whole chip.
    constexpr bool MODEL = MODE != kChi2;
    const int64_t n_items = MODEL ? n_batches * n_groups : n_batches;
    int64_t prev_bt = -1;
    for (int64_t item = gw; item < n_items; item += n_waves) {
        const int64_t bt = MODEL ? item / n_groups : item;
        const int g_first = MODEL ? (int)(item - bt * n_groups) : 0;
        const int g_end = MODEL ? g_first + 1 : n_groups;
        const int64_t s0 = bt * a.sb;
        const int nb = (int)min((int64_t)a.sb, a.n_sys - s0);
        if (bt != prev_bt) {
        prev_bt = bt;
        wave_sync_lds();
        if (lane < nb) {
            const int64_t sys = s0 + lane;
            bool ok = isfinite(a.t0);
            for (int j = 0; j < a.n_pl; ++j) {
                const int64_t p = (int64_t)j * a.n_sys + sys;
                Rec r;
                ok = Pol::setup(a, a.P[p], a.K[p], a.e[p], a.w[p], a.M0[p], r) && ok;
                recs[lane * a.n_pl + j] = r;
            }
            if (a.offset) ok = ok && isfinite(a.offset[sys]);
            if (a.jitter) ok = ok && isfinite(a.jitter[sys]) && a.jitter[sys] >= 0.0;
            sysbad[lane] = ok ? 0 : 1;
        }
        wave_sync_lds();
        }

        for (int s = 0; s < nb; ++s) {
            const int64_t sys = s0 + s;
            const double gam = a.offset ? a.offset[sys] : 0.0;
            const double jit = a.jitter ? a.jitter[sys] : 0.0;
            const bool sbad = uniform_int(sysbad[s]) != 0;
            typename Pol::ChiAcc chi;
            Pol::chi_init(chi);
            bool bad_obs = false;
            for (int g = g_first; g < g_end; ++g) {
                if (n_groups > 1) load_group(g);
                ModelAcc m[NCH];
                if (MODE == kPlanets) {
                    for (int j = 0; j < a.n_pl; ++j) {
#pragma unroll
                        for (int c = 0; c < NCH; ++c) Pol::model_init(m[c]);
                        pol_add_planet<Pol, NCH>(recs[s * a.n_pl + j], o, m, a);
                        float *row = a.dv + ((int64_t)j * a.n_sys + sys) * a.n_obs;
#pragma unroll
                        for (int c = 0; c < NCH; ++c) {
                            if (o[c].in) {
                                const int64_t k = (int64_t)g * 64 * NCH + c * 64 + lane;
                                row[k] = (sbad || !o[c].ok) ? __builtin_nanf("") : (float)Pol::model_value(m[c]);
                            }
                        }
                    }
                    continue;
                }
#pragma unroll
                for (int c = 0; c < NCH; ++c) Pol::model_init(m[c]);
                for (int j = 0; j < a.n_pl; ++j) pol_add_planet<Pol, NCH>(recs[s * a.n_pl + j], o, m, a);
                if (MODEL) {
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
                        if (o[c].in) {
                            int64_t k = (int64_t)g * 64 * NCH + c * 64 + lane;
                            double val = Pol::model_value(m[c]) + gam;
                            a.out[sys * a.n_obs + k] = (sbad || !o[c].ok) ? __builtin_nan("") : val;
                        }
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
                        if (o[c].in) {
                            bool okw = Pol::chi_add(chi, m[c], o[c], gam, jit, has_jit);
                            bad_obs = bad_obs || !okw || !o[c].ok;
                        }
                    }
                }
            }
            if (!MODEL) {
                double tot = wave_sum(Pol::chi_value(chi));
                bool bad = sbad || __any(bad_obs);
                if (lane == 0) a.out[sys] = bad ? __builtin_nan("") : tot;
            }
        }
    }
}

// Second kernel of the separate-function form: planet sums (Kahan), residuals
// and the compensated chi-square from the velocities written by kPlanets.
template <int NCH>
__global__ void __launch_bounds__(256) k_chisq_from_dv(DenseArgs a)
{
    const int lane = __lane_id();
    const int wpb = blockDim.x >> 6;
    const int64_t gw = (int64_t)blockIdx.x * wpb + uniform_int(threadIdx.x >> 6);
    const int64_t n_waves = (int64_t)gridDim.x * wpb;
    const bool has_jit = a.jitter != nullptr;
    ObsMixed o[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) PolMixed::load_obs(a, c * 64 + lane, o[c]);
    for (int64_t sys = gw; sys < a.n_sys; sys += n_waves) {
        const double gam = a.offset ? a.offset[sys] : 0.0;
        const double jit = a.jitter ? a.jitter[sys] : 0.0;
        bool bad = !isfinite(a.t0) || (a.offset && !isfinite(gam)) || (has_jit && !(isfinite(jit) && jit >= 0.0));
        PolMixed::ModelAcc m[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) PolMixed::model_init(m[c]);
        for (int j = 0; j < a.n_pl; ++j) {
            const float *row = a.dv + ((int64_t)j * a.n_sys + sys) * a.n_obs;
#pragma unroll
            for (int c = 0; c < NCH; ++c) m[c].k.add(o[c].in ? row[c * 64 + lane] : 0.0f);
        }
        Kahan32 chi;
        chi.init();
        bool bad_obs = false;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            if (o[c].in) {
                bool okw = PolMixed::chi_add(chi, m[c], o[c], gam, jit, has_jit);
                bad_obs = bad_obs || !okw || !o[c].ok;
            }
        }
        const double tot = wave_sum(chi.value());
        bad = bad || __any(bad_obs);
        if (lane == 0) a.out[sys] = bad ? __builtin_nan("") : tot;
    }
}

// ------------------------------------------------------------------ Kepler only
// Standalone Kepler solve (the paper's Kepler-only mode): one lane per pair.
// M is reduced to [-pi, pi] with 2 pi as a double-double; the root is returned
// on the input's branch.
template <bool MIXED>
__device__ __forceinline__ double kepler_one(double M, double e, int fixed, int max_iter)
{
    const bool ok = isfinite(M) && isfinite(e) && e >= 0.0 && e < 1.0;
    if (!ok) { M = 0.0; e = 0.0; }
    const double kq = rint(M * kInvTwoPi);
    double Mr = fma(-kq, kTwoPiHi, M);
    Mr = fma(-kq, kTwoPiLo, Mr);
    double E;
    if (MIXED) {
        const Ecc32 k = make_ecc32(e);
        const int niter = fixed > 0 ? fixed : sched32(k.e);
        float sE, omcE;   // unused here: the standalone solve returns E only
        E = (double)kepler32((float)Mr, k, niter, max_iter, fixed > 0, sE, omcE);
    } else {
        E = kepler64(Mr, e, Mr >= 0.0 ? 1.0 : -1.0, fixed, max_iter);
    }
    E = fma(kq, kTwoPiHi, E);
    E = fma(kq, kTwoPiLo, E);
    return ok ? E : __builtin_nan("");
}

// Each thread takes KU pairs per tile (KU x blockDim consecutive pairs per
// block), issuing all of their loads before solving, so that more memory
// requests are in flight than one pair per thread would allow.
template <bool MIXED, int KU>
__global__ void __launch_bounds__(256) k_kepler(const double *__restrict__ Mv, const double *__restrict__ ev,
                                               double *__restrict__ Ev, int64_t n, int fixed, int max_iter)
{
    const int64_t tile = (int64_t)blockDim.x * KU;
    const int64_t stride = (int64_t)gridDim.x * tile;
    for (int64_t base = (int64_t)blockIdx.x * tile + threadIdx.x; base < n; base += stride) {
        double M[KU], e[KU];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x;
            M[u] = i < n ? Mv[i] : 0.0;
            e[u] = i < n ? ev[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x;
            const double E = kepler_one<MIXED>(M[u], e[u], fixed, max_iter);
            if (i < n) Ev[i] = E;
        }
    }
}

__global__ void k_fill_u32(unsigned int *p, unsigned int value, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

// ------------------------------------------------------------------ gradient
// chi-square and its gradient with one lane per system (the adjoint needs
// 5 n_pl + 1 running sums per system; keeping them in the lane that owns the
// system avoids a cross-lane reduction per sum).  Observations are uniform
// across the wave and arrive through scalar loads.  Derivatives use the
// implicit-function relations of Kepler's equation, dE/dM = 1/(1 - e cos E)
// and dE/de = sin E/(1 - e cos E), in the true-anomaly forms
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
__device__ __forceinline__ float grad_terms(const GradPlanet<float> &g, double tt, int max_iter, float (&x)[5])
{
    const float M = mean_anomaly32(tt, g.ph);
    float sE, omcE;
    kepler32(M, g.k, g.niter, max_iter, g.check != 0, sE, omcE);
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
template <int NPL, bool NLL>
__global__ void __launch_bounds__(256) k_grad_mixed(DenseArgs a)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const bool has_jit = a.jitter != nullptr;
    for (int64_t sys = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; sys < a.n_sys; sys += stride) {
        GradPlanet<float> pl[NPL];
        bool ok = isfinite(a.t0);
#pragma unroll
        for (int j = 0; j < NPL; ++j) {
            const int64_t p = (int64_t)j * a.n_sys + sys;
            ok = grad_setup(a.P[p], a.K[p], a.e[p], a.w[p], a.M0[p], a.fixed_iter, pl[j]) && ok;
        }
        const double gam = a.offset ? a.offset[sys] : 0.0;
        const double jit = a.jitter ? a.jitter[sys] : 0.0;
        if (a.offset) ok = ok && isfinite(gam);
        if (has_jit) ok = ok && isfinite(jit) && jit >= 0.0;
        const float jit2 = (float)(jit * jit);
        Kahan32 chi;
        chi.init();
        double acc[NPL][5], sum_c2 = 0.0;   // binary64 running sums of 2 w r x
        double sum_lv = 0.0, sum_w = 0.0, sum_wr2 = 0.0;
#pragma unroll
        for (int j = 0; j < NPL; ++j) {
#pragma unroll
            for (int i = 0; i < 5; ++i) acc[j][i] = 0.0;
        }
        for (int64_t k = 0; k < a.n_obs; ++k) {
            const double t = a.t[k], vo = a.v[k], sg = a.sigma[k];
            ok = ok && isfinite(t) && isfinite(vo) && isfinite(sg) && sg >= 0.0;
            const double tt = t - a.t0;
            float x[NPL][5];
            Kahan32 msum;
            msum.init();
#pragma unroll
            for (int j = 0; j < NPL; ++j) msum.add(grad_terms(pl[j], tt, a.max_iter, x[j]));
            const float r = (float)(((double)msum.s - (double)msum.c + gam) - vo);
            const float var = (float)(sg * sg) + jit2;
            ok = ok && var > 0.0f;
            const float w = rcp32(var);
            const float wr = w * r;
            chi.add(wr * r);
            if (NLL) {
                sum_lv += (double)logf(var);
                sum_w += (double)w;
                sum_wr2 = fma((double)wr, (double)wr, sum_wr2);
            }
            const double c2 = 2.0 * (double)wr;
            sum_c2 += c2;
#pragma unroll
            for (int j = 0; j < NPL; ++j) {
#pragma unroll
                for (int i = 0; i < 5; ++i) acc[j][i] = fma(c2, (double)x[j][i], acc[j][i]);
            }
        }
        const double nan = __builtin_nan("");
        a.out[sys] = ok ? chi.value() + sum_lv : nan;
        if (NLL) a.grad[(int64_t)(5 * NPL + 1) * a.n_sys + sys] = ok ? 2.0 * jit * (sum_w - sum_wr2) : nan;
#pragma unroll
        for (int j = 0; j < NPL; ++j) {
            const int64_t p = (int64_t)j * a.n_sys + sys;
            const double K = a.K[p], e = a.e[p], P = a.P[p];
            const double cw = pl[j].cw, sw = pl[j].sw;
            double gj[5];
            gj[0] = kTwoPi * K / P * acc[j][0];
            gj[1] = acc[j][1] + e * cw * sum_c2;
            gj[2] = K * cw * sum_c2 - K * acc[j][2];
            gj[3] = -K * acc[j][3] - K * e * sw * sum_c2;
            gj[4] = -K * acc[j][4];
#pragma unroll
            for (int i = 0; i < 5; ++i) a.grad[(int64_t)(5 * j + i) * a.n_sys + sys] = ok ? gj[i] : nan;
        }
        a.grad[(int64_t)(5 * NPL) * a.n_sys + sys] = ok ? sum_c2 : nan;
    }
}

template <int NPL, bool NLL>
__global__ void __launch_bounds__(256) k_grad_f64(DenseArgs a)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const bool has_jit = a.jitter != nullptr;
    const int fixed = fixed64(a.fixed_iter);
    for (int64_t sys = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; sys < a.n_sys; sys += stride) {
        GradPlanet<double> pl[NPL];
        bool ok = isfinite(a.t0);
#pragma unroll
        for (int j = 0; j < NPL; ++j) {
            const int64_t p = (int64_t)j * a.n_sys + sys;
            ok = grad_setup(a.P[p], a.K[p], a.e[p], a.w[p], a.M0[p], a.fixed_iter, pl[j]) && ok;
        }
        const double gam = a.offset ? a.offset[sys] : 0.0;
        const double jit = a.jitter ? a.jitter[sys] : 0.0;
        if (a.offset) ok = ok && isfinite(gam);
        if (has_jit) ok = ok && isfinite(jit) && jit >= 0.0;
        double chi = 0.0, gacc[5 * NPL + 1];
        double sum_lv = 0.0, sum_w = 0.0, sum_wr2 = 0.0;
#pragma unroll
        for (int i = 0; i < 5 * NPL + 1; ++i) gacc[i] = 0.0;
        for (int64_t k = 0; k < a.n_obs; ++k) {
            const double t = a.t[k], vo = a.v[k], sg = a.sigma[k];
            ok = ok && isfinite(t) && isfinite(vo) && isfinite(sg) && sg >= 0.0;
            const double tt = t - a.t0;
            double d[NPL][5];
            double m = 0.0;
#pragma unroll
            for (int j = 0; j < NPL; ++j) m += grad_eval(pl[j], tt, a.max_iter, fixed, d[j]);
            const double r = m + gam - vo;
            const double var = sg * sg + jit * jit;
            ok = ok && var > 0.0;
            const double w = 1.0 / var;
            chi = fma(w * r, r, chi);
            if (NLL) {
                sum_lv += log(var);
                sum_w += w;
                sum_wr2 = fma(w * r, w * r, sum_wr2);
            }
            const double c2 = 2.0 * w * r;
#pragma unroll
            for (int j = 0; j < NPL; ++j) {
#pragma unroll
                for (int i = 0; i < 5; ++i) gacc[5 * j + i] = fma(c2, d[j][i], gacc[5 * j + i]);
            }
            gacc[5 * NPL] += c2;
        }
        const double nan = __builtin_nan("");
        a.out[sys] = ok ? chi + sum_lv : nan;
#pragma unroll
        for (int i = 0; i < 5 * NPL + 1; ++i) a.grad[(int64_t)i * a.n_sys + sys] = ok ? gacc[i] : nan;
        if (NLL) a.grad[(int64_t)(5 * NPL + 1) * a.n_sys + sys] = ok ? 2.0 * jit * (sum_w - sum_wr2) : nan;
    }
}

// ------------------------------------------------------------------ DE-MC
// One half-step of the population sampler, fused: for a batch of sb chains
// of half h the wave
//   A. lanes over chains: draw 0 gives r1 != r2 (other half) and u;
//   B. lanes over (chain, pair of rows): two normals z and the proposal rows
//      y_r = x_ir + gam (x_r1,r - x_r2,r) + eps_r z_r;
//   C. lanes over (chain, planet): the planet records, as the dense kernel's
//      setup does from parameter planes;
//   D. lanes over chains: domain and prior-support flags;
//   then evaluates each proposal's chi-square with the lanes over
//   observations, exactly as the dense chi-square kernel does, and
//   E. lanes over chains: accepts iff 2 ln u < chi2(x) - chi2(y) and K >= 0,
//      copying y into the chain.
// Everything one lane hands to another goes through the wave's slice of LDS;
// the half being updated is read and written only by the lane that owns the
// chain in phase B / E, and the other half is only read.  The proposals and
// their chi-square are also written to the workspace (m.y, m.c_new).
__host__ __device__ inline size_t demc_lds_per_wave(int sb, int n_pl, int d, size_t rec_bytes)
{
    size_t b = (size_t)sb * n_pl * rec_bytes          // planet records
               + (size_t)sb * d * sizeof(double)       // proposals
               + (size_t)sb * 2 * sizeof(double)       // u, chi2 of the proposal
               + (size_t)sb * 2 * sizeof(uint32_t)     // r1, r2
               + (size_t)sb * n_pl * sizeof(int)       // per-planet domain flag
               + (size_t)sb * 2 * sizeof(int);         // per-chain domain and support flags
    return (b + 15) & ~(size_t)15;
}

template <class Pol, int NCH>
__global__ void __launch_bounds__(256) k_demc_half(DenseArgs a, DemcArgs m, int h)
{
    using Rec = typename Pol::Rec;
    using Obs = typename Pol::Obs;
    using ModelAcc = typename Pol::ModelAcc;
    extern __shared__ __align__(16) unsigned char smem[];

    const int lane = __lane_id();
    const int wpb = blockDim.x >> 6;
    const int wib = uniform_int(threadIdx.x >> 6);
    const int sb = a.sb, npl = a.n_pl, d = m.d;
    unsigned char *mine = smem + (size_t)wib * demc_lds_per_wave(sb, npl, d, sizeof(Rec));
    Rec *recs = reinterpret_cast<Rec *>(mine);
    double *y_l = reinterpret_cast<double *>(mine + (size_t)sb * npl * sizeof(Rec));
    double *u_l = y_l + (size_t)sb * d;
    double *cnew_l = u_l + sb;
    uint32_t *r12_l = reinterpret_cast<uint32_t *>(cnew_l + sb);
    int *okpl_l = reinterpret_cast<int *>(r12_l + 2 * sb);
    int *bad_l = okpl_l + sb * npl;
    int *supp_l = bad_l + sb;

    const int64_t nh = m.nh;
    const uint64_t g = m.gen_ptr ? *m.gen_ptr : m.gen;
    const double gde = (m.jump_every > 0 && (g + 1) % (uint64_t)m.jump_every == 0) ? 1.0 : m.gamma;
    double *xh = m.x + (int64_t)h * d * nh;
    const double *xo = m.x + (int64_t)(1 - h) * d * nh;
    const int ndraw = (d + 1) / 2;

    const int64_t gw = (int64_t)blockIdx.x * wpb + wib;
    const int64_t n_waves = (int64_t)gridDim.x * wpb;
    const int64_t n_batches = (nh + sb - 1) / sb;
    const int n_groups = (int)((a.n_obs + 64 * NCH - 1) / (64 * NCH));
    const bool has_jit = a.jitter != nullptr;

    Obs o[NCH];
    auto load_group = [&](int gi) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) Pol::load_obs(a, (int64_t)gi * 64 * NCH + c * 64 + lane, o[c]);
    };
    if (n_groups <= 1) load_group(0);

    for (int64_t bt = gw; bt < n_batches; bt += n_waves) {
        const int64_t s0 = bt * sb;
        const int nb = (int)min((int64_t)sb, nh - s0);
        wave_sync_lds();
        for (int c = lane; c < nb; c += 64) {                                   // A
            const U4 w = demc_draw(m.key0, m.key1, h, (uint32_t)(s0 + c), 0u, g);
            const uint32_t r1 = below(w.w0, (uint32_t)nh);
            uint32_t r2 = below(w.w1, (uint32_t)nh - 1u);
            if (r2 >= r1) r2 += 1u;
            r12_l[2 * c] = r1;
            r12_l[2 * c + 1] = r2;
            u_l[c] = unit53(w.w2, w.w3);
        }
        wave_sync_lds();
        for (int q = lane; q < nb * ndraw; q += 64) {                           // B
            const int c = q / ndraw, p = q - c * ndraw, r = 2 * p;
            const int64_t i = s0 + c;
            const uint32_t r1 = r12_l[2 * c], r2 = r12_l[2 * c + 1];
            const U4 w = demc_draw(m.key0, m.key1, h, (uint32_t)i, (uint32_t)(1 + p), g);
            const double rho = sqrt(-2.0 * log(unit53(w.w0, w.w1)));
            double sn, cs;
            sincos(kTwoPi * unit53(w.w2, w.w3), &sn, &cs);
            {
                // rounded term by term, as written (no contraction)
#pragma clang fp contract(off)
                const int64_t o0 = (int64_t)r * nh;
                const double y0 = xh[o0 + i] + gde * (xo[o0 + r1] - xo[o0 + r2]) + m.eps[r] * (rho * cs);
                y_l[c * d + r] = y0;
                m.y[o0 + i] = y0;
                if (r + 1 < d) {
                    const int64_t o1 = o0 + nh;
                    const double y1 = xh[o1 + i] + gde * (xo[o1 + r1] - xo[o1 + r2]) + m.eps[r + 1] * (rho * sn);
                    y_l[c * d + r + 1] = y1;
                    m.y[o1 + i] = y1;
                }
            }
        }
        wave_sync_lds();
        for (int q = lane; q < nb * npl; q += 64) {                             // C
            const int c = q / npl, j = q - c * npl;
            const double *yc = y_l + c * d;
            Rec rr;
            okpl_l[q] = Pol::setup(a, yc[j], yc[npl + j], yc[2 * npl + j], yc[3 * npl + j], yc[4 * npl + j], rr)
                            ? 1 : 0;
            recs[q] = rr;
        }
        wave_sync_lds();
        for (int c = lane; c < nb; c += 64) {                                   // D
            const double *yc = y_l + c * d;
            bool ok = isfinite(a.t0) && isfinite(yc[5 * npl]);
            bool supp = true;
            for (int j = 0; j < npl; ++j) {
                ok = ok && okpl_l[c * npl + j] != 0;
                supp = supp && yc[npl + j] >= 0.0;
            }
            if (has_jit) ok = ok && isfinite(a.jitter[s0 + c]) && a.jitter[s0 + c] >= 0.0;
            bad_l[c] = ok ? 0 : 1;
            supp_l[c] = supp ? 1 : 0;
        }
        wave_sync_lds();

        for (int s = 0; s < nb; ++s) {
            const double gam = y_l[s * d + 5 * npl];
            const double jit = has_jit ? a.jitter[s0 + s] : 0.0;
            const bool sbad = uniform_int(bad_l[s]) != 0;
            typename Pol::ChiAcc chi;
            Pol::chi_init(chi);
            bool bad_obs = false;
            for (int gi = 0; gi < n_groups; ++gi) {
                if (n_groups > 1) load_group(gi);
                ModelAcc mm[NCH];
#pragma unroll
                for (int c = 0; c < NCH; ++c) Pol::model_init(mm[c]);
                for (int j = 0; j < npl; ++j) pol_add_planet<Pol, NCH>(recs[s * npl + j], o, mm, a);
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    if (o[c].in) {
                        const bool okw = Pol::chi_add(chi, mm[c], o[c], gam, jit, has_jit);
                        bad_obs = bad_obs || !okw || !o[c].ok;
                    }
                }
            }
            const double tot = wave_sum(Pol::chi_value(chi));
            const bool bad = sbad || __any(bad_obs);
            if (lane == 0) cnew_l[s] = bad ? __builtin_nan("") : tot;
        }
        wave_sync_lds();

        for (int c = lane; c < nb; c += 64) {                                   // E
            const int64_t i = s0 + c;
            const double c_new = cnew_l[c];
            double *chi = m.chi2 + (int64_t)h * nh + i;
            m.c_new[i] = c_new;
            if (supp_l[c] != 0 && 2.0 * log(u_l[c]) < *chi - c_new) {
                for (int r = 0; r < d; ++r) xh[(int64_t)r * nh + i] = y_l[c * d + r];
                *chi = c_new;
                if (m.n_accept) m.n_accept[(int64_t)h * nh + i] += 1;
            }
        }
    }
}

template <class Pol>
static hipError_t launch_demc_half_t(DemcArgs m, DenseArgs a, int h, LaunchShape shape, hipStream_t st)
{
    const int block = shape.block > 0 ? shape.block : 256;
    const int wpb = block / 64;
    const size_t rec = sizeof(typename Pol::Rec);
    int sb_cap = kMaxSB;
    while (sb_cap > 1 && (size_t)wpb * demc_lds_per_wave(sb_cap, a.n_pl, m.d, rec) > 48 * 1024) sb_cap /= 2;
    const int nch_needed = (int)((a.n_obs + 63) / 64);
    void (*kern)(DenseArgs, DemcArgs, int);
    if (nch_needed <= 1) kern = k_demc_half<Pol, 1>;
    else if (nch_needed <= 2) kern = k_demc_half<Pol, 2>;
    else if (nch_needed <= 4) kern = k_demc_half<Pol, 4>;
    else kern = k_demc_half<Pol, 8>;
    int per_cu = shape.blocks_per_cu;
    if (per_cu <= 0) {
        int occ = 0;
        const size_t lds = (size_t)wpb * demc_lds_per_wave(sb_cap, a.n_pl, m.d, rec);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, block, lds) != hipSuccess || occ <= 0) occ = 1;
        per_cu = occ;
    }
    const int64_t max_waves = (int64_t)device_cu_count() * per_cu * wpb;
    // ceil: every wave gets at most one batch when the cap allows it, so no wave
    // runs a second batch while the others idle
    const int64_t mw = max_waves > 0 ? max_waves : 1;
    int64_t sb = (m.nh + mw - 1) / mw;
    sb = sb < 1 ? 1 : (sb > sb_cap ? sb_cap : sb);
    a.sb = (int)sb;
    const size_t lds = (size_t)wpb * demc_lds_per_wave(a.sb, a.n_pl, m.d, rec);
    const int64_t n_batches = (m.nh + sb - 1) / sb;
    int64_t grid = (n_batches + wpb - 1) / wpb;
    const int64_t cap = (int64_t)device_cu_count() * per_cu;
    if (grid > cap) grid = cap;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(block), lds, st, a, m, h);
    return hipGetLastError();
}

hipError_t launch_demc_half(DemcArgs m, DenseArgs a, Prec prec, int h, LaunchShape shape, hipStream_t st)
{
    if (m.nh <= 0) return hipSuccess;
    a.n_sys = m.nh;
    a.n_pl = m.n_pl;
    a.jitter = m.jitter ? m.jitter + (int64_t)h * m.nh : nullptr;
    a.out = nullptr;
    a.grad = nullptr;
    a.dv = nullptr;
    return prec == Prec::Mixed ? launch_demc_half_t<PolMixed>(m, a, h, shape, st)
                               : launch_demc_half_t<Pol64>(m, a, h, shape, st);
}

// ------------------------------------------------------------------ ragged
// Persistent kernel over CSR systems.  Work items are runs of `sb` systems in
// decreasing order of work; each wavefront takes the next item from an
// atomic counter until the items run out.  Setup runs one lane per system of
// the item; evaluation runs one system at a time with lanes over that
// system's observations, in groups of up to 4 x 64 loaded with coalesced reads.
struct RecRagged {
    RecMixed pl[kMaxPl];
};

template <int NCH>
__device__ __forceinline__ void ragged_group(const RaggedArgs &a, const RecMixed *recs, int npl, int64_t o0,
                                             int64_t nrem, double gam, double jit, bool has_jit, Kahan32 &chi,
                                             bool &bad_obs)
{
    const int lane = __lane_id();
    ObsMixed o[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int64_t k = c * 64 + lane;
        o[c].in = k < nrem;
        double t = o[c].in ? a.t[o0 + k] : a.t0;
        double v = o[c].in ? a.v[o0 + k] : 0.0;
        double s = o[c].in ? a.sigma[o0 + k] : 1.0;
        o[c].ok = isfinite(t) && isfinite(v) && isfinite(s) && s >= 0.0;
        o[c].tt = t - a.t0;
        o[c].v = v;
        o[c].s2 = (float)(s * s);
        o[c].w = (float)(1.0 / (s * s));
    }
    PolMixed::ModelAcc m[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) PolMixed::model_init(m[c]);
    for (int j = 0; j < npl; ++j) PolMixed::add_planet<NCH>(recs[j], o, m, a.max_iter, 0);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        if (o[c].in) {
            bool okw = PolMixed::chi_add(chi, m[c], o[c], gam, jit, has_jit);
            bad_obs = bad_obs || !okw || !o[c].ok;
        }
    }
}

// GMAX: largest observation group in 64-lane chunks (2 or 4): fewer chunks in
// flight need fewer registers and allow more resident waves; the plan's
// autotuner picks it.
template <int GMAX>
__global__ void __launch_bounds__(256) k_ragged_mixed(RaggedArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = __lane_id();
    const int wpb = blockDim.x >> 6;
    const int wib = uniform_int(threadIdx.x >> 6);
    RecMixed *recs = reinterpret_cast<RecMixed *>(smem) + (size_t)wib * a.sb * kMaxPl;
    int *meta = reinterpret_cast<int *>(smem + (size_t)wpb * a.sb * kMaxPl * sizeof(RecMixed)) + (size_t)wib * a.sb * 2;
    const bool has_jit = a.jitter != nullptr;

    for (;;) {
        unsigned int item = 0;
        if (lane == 0) item = atomicAdd(a.queue, 1u);
        item = (unsigned int)uniform_int((int)__shfl(item, 0, 64));
        if ((int64_t)item >= a.n_items) break;
        const int64_t i0 = (int64_t)item * a.sb;
        const int nb = (int)min((int64_t)a.sb, a.n_sys - i0);
        wave_sync_lds();
        if (lane < nb) {
            const int64_t sys = a.order[i0 + lane];
            const int64_t p0 = a.pl_off[sys];
            const int npl = (int)(a.pl_off[sys + 1] - p0);
            bool ok = isfinite(a.t0) && npl >= 1 && npl <= kMaxPl;
            DenseArgs dummy;
            dummy.fixed_iter = a.fixed_iter;
            for (int j = 0; j < npl && j < kMaxPl; ++j) {
                RecMixed r;
                ok = PolMixed::setup(dummy, a.P[p0 + j], a.K[p0 + j], a.e[p0 + j], a.w[p0 + j], a.M0[p0 + j], r) && ok;
                recs[lane * kMaxPl + j] = r;
            }
            if (a.offset) ok = ok && isfinite(a.offset[sys]);
            if (a.jitter) ok = ok && isfinite(a.jitter[sys]) && a.jitter[sys] >= 0.0;
            meta[2 * lane] = ok ? npl : -npl;
            meta[2 * lane + 1] = (int)sys;
        }
        wave_sync_lds();
        for (int s = 0; s < nb; ++s) {
            const int code = uniform_int(meta[2 * s]);
            const int64_t sys = uniform_int(meta[2 * s + 1]);
            const int npl = code < 0 ? -code : code;
            const int64_t o0 = a.obs_off[sys];
            const int64_t n = a.obs_off[sys + 1] - o0;
            const double gam = a.offset ? a.offset[sys] : 0.0;
            const double jit = a.jitter ? a.jitter[sys] : 0.0;
            Kahan32 chi;
            chi.init();
            bool bad_obs = false;
            for (int64_t g = 0; g < n; g += 64 * GMAX) {
                const int64_t rem = n - g;
                const RecMixed *rs = recs + s * kMaxPl;
                if (rem <= 64) ragged_group<1>(a, rs, npl, o0 + g, rem, gam, jit, has_jit, chi, bad_obs);
                else if (GMAX == 2 || rem <= 128) ragged_group<2>(a, rs, npl, o0 + g, rem, gam, jit, has_jit, chi, bad_obs);
                else if (rem <= 192) ragged_group<3>(a, rs, npl, o0 + g, rem, gam, jit, has_jit, chi, bad_obs);
                else ragged_group<GMAX>(a, rs, npl, o0 + g, rem, gam, jit, has_jit, chi, bad_obs);
            }
            const double tot = wave_sum(chi.value());
            const bool bad = code <= 0 || __any(bad_obs);
            if (lane == 0) a.out[sys] = bad ? __builtin_nan("") : tot;
        }
    }
}

// ------------------------------------------------------------------ launchers
static int g_cu_count = 0;

int device_cu_count()
{
    if (g_cu_count == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 256;
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        g_cu_count = cus;
    }
    return g_cu_count;
}

hipError_t launch_fill_u32(unsigned int *p, unsigned int value, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    int blocks = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, st, p, value, n);
    return hipGetLastError();
}

hipError_t launch_kepler_solve(const double *M, const double *e, double *E, int64_t n, Prec prec, int fixed_iter,
                               int max_iter, LaunchShape shape, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int block = shape.block > 0 ? shape.block : 256;
    const int per_cu = shape.blocks_per_cu > 0 ? shape.blocks_per_cu : 8 * (256 / block);
    constexpr int KU = 4;
    const int64_t need = (n + (int64_t)block * KU - 1) / ((int64_t)block * KU);
    const int64_t cap = (int64_t)device_cu_count() * per_cu;
    const int grid = (int)(need < cap ? need : cap);
    if (prec == Prec::Mixed)
        hipLaunchKernelGGL((k_kepler<true, KU>), dim3(grid), dim3(block), 0, st, M, e, E, n, fixed_iter, max_iter);
    else
        hipLaunchKernelGGL((k_kepler<false, KU>), dim3(grid), dim3(block), 0, st, M, e, E, n,
                           fixed_iter == 0 ? 30 : (fixed_iter < 0 ? 0 : fixed_iter), max_iter);
    return hipGetLastError();
}

template <class Pol, int MODE>
static hipError_t launch_dense_t(DenseArgs a, LaunchShape shape, hipStream_t st)
{
    const int block = shape.block > 0 ? shape.block : 256;
    const int wpb = block / 64;
    const size_t rec_bytes = (size_t)wpb * a.n_pl * sizeof(typename Pol::Rec) + (size_t)wpb * sizeof(int);
    // systems per setup batch: at most kMaxSB and at most 48 KiB of LDS per block
    int64_t sb_cap = (int64_t)(48 * 1024) / (int64_t)rec_bytes;
    sb_cap = sb_cap < 1 ? 1 : (sb_cap > kMaxSB ? kMaxSB : sb_cap);
    size_t lds = rec_bytes * (size_t)sb_cap;
    const int nch_needed = (int)((a.n_obs + 63) / 64);
    void (*kern)(DenseArgs);
    int nch;
    if (nch_needed <= 1) { kern = k_dense<Pol, 1, MODE>; nch = 1; }
    else if (nch_needed <= 2) { kern = k_dense<Pol, 2, MODE>; nch = 2; }
    else if (nch_needed <= 4) { kern = k_dense<Pol, 4, MODE>; nch = 4; }
    else { kern = k_dense<Pol, 8, MODE>; nch = 8; }
    int per_cu = shape.blocks_per_cu;
    if (per_cu <= 0) {
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, block, lds) != hipSuccess || occ <= 0) occ = 1;
        per_cu = occ;
    }
    const int64_t max_waves = (int64_t)device_cu_count() * per_cu * wpb;
    // ceil: every wave gets at most one batch when the cap allows it, so no wave
    // runs a second batch while the others idle
    const int64_t mw = max_waves > 0 ? max_waves : 1;
    int64_t sb = (a.n_sys + mw - 1) / mw;
    sb = sb < 1 ? 1 : (sb > sb_cap ? sb_cap : sb);
    a.sb = (int)sb;
    lds = rec_bytes * (size_t)sb;
    const int64_t n_batches = (a.n_sys + sb - 1) / sb;
    const int64_t n_groups = (a.n_obs + 64 * nch - 1) / (64 * nch);
    const int64_t n_items = MODE != kChi2 ? n_batches * (n_groups > 0 ? n_groups : 1) : n_batches;
    int64_t grid = (n_items + wpb - 1) / wpb;
    const int64_t cap = (int64_t)device_cu_count() * per_cu;
    if (grid > cap) grid = cap;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(block), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_dense(DenseArgs a, Prec prec, bool model, LaunchShape shape, hipStream_t st)
{
    if (a.n_sys <= 0) return hipSuccess;
    if (model && a.n_obs <= 0) return hipSuccess;
    if (prec == Prec::Mixed)
        return model ? launch_dense_t<PolMixed, kModel>(a, shape, st) : launch_dense_t<PolMixed, kChi2>(a, shape, st);
    return model ? launch_dense_t<Pol64, kModel>(a, shape, st) : launch_dense_t<Pol64, kChi2>(a, shape, st);
}

hipError_t launch_planet_velocities(DenseArgs a, LaunchShape shape, hipStream_t st)
{
    if (a.n_sys <= 0 || a.n_obs <= 0) return hipSuccess;
    return launch_dense_t<PolMixed, kPlanets>(a, shape, st);
}

hipError_t launch_chisq_from_velocities(DenseArgs a, LaunchShape shape, hipStream_t st)
{
    if (a.n_sys <= 0) return hipSuccess;
    const int block = shape.block > 0 ? shape.block : 256;
    const int wpb = block / 64;
    const int nch_needed = (int)((a.n_obs + 63) / 64);
    void (*kern)(DenseArgs);
    if (nch_needed <= 1) kern = k_chisq_from_dv<1>;
    else if (nch_needed <= 2) kern = k_chisq_from_dv<2>;
    else if (nch_needed <= 4) kern = k_chisq_from_dv<4>;
    else if (nch_needed <= 8) kern = k_chisq_from_dv<8>;
    else if (nch_needed <= 16) kern = k_chisq_from_dv<16>;
    else return hipErrorInvalidValue;
    const int per_cu = shape.blocks_per_cu > 0 ? shape.blocks_per_cu : 8;
    int64_t grid = (a.n_sys + wpb - 1) / wpb;
    const int64_t cap = (int64_t)device_cu_count() * per_cu;
    if (grid > cap) grid = cap;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(block), 0, st, a);
    return hipGetLastError();
}

}  // namespace kep

namespace kep {

static int grad_grid(int64_t n_sys, int block, int per_cu)
{
    int64_t need = (n_sys + block - 1) / block;
    int64_t cap = (int64_t)device_cu_count() * (per_cu > 0 ? per_cu : 8);
    return (int)(need < cap ? (need > 0 ? need : 1) : cap);
}

hipError_t launch_dense_grad(DenseArgs a, Prec prec, bool nll, LaunchShape shape, hipStream_t st)
{
    if (a.n_sys <= 0) return hipSuccess;
    const int block = shape.block > 0 ? shape.block : 256;
    const int grid = grad_grid(a.n_sys, block, shape.blocks_per_cu);
#define KEP_GRAD_LAUNCH(N, L)                                                                   \
    if (prec == Prec::Mixed) hipLaunchKernelGGL((k_grad_mixed<N, L>), dim3(grid), dim3(block), 0, st, a); \
    else hipLaunchKernelGGL((k_grad_f64<N, L>), dim3(grid), dim3(block), 0, st, a);
#define KEP_GRAD_CASE(N)                                                                     \
    case N:                                                                                  \
        if (nll) { KEP_GRAD_LAUNCH(N, true) } else { KEP_GRAD_LAUNCH(N, false) }              \
        break;
    switch (a.n_pl) {
        KEP_GRAD_CASE(1)
        KEP_GRAD_CASE(2)
        KEP_GRAD_CASE(3)
        KEP_GRAD_CASE(4)
        KEP_GRAD_CASE(5)
        KEP_GRAD_CASE(6)
        KEP_GRAD_CASE(7)
        KEP_GRAD_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef KEP_GRAD_CASE
#undef KEP_GRAD_LAUNCH
    return hipGetLastError();
}

static size_t ragged_lds(int block, int sb)
{
    const int wpb = block / 64;
    return (size_t)wpb * sb * kMaxPl * sizeof(RecMixed) + (size_t)wpb * sb * 2 * sizeof(int);
}

int ragged_max_grid(LaunchShape shape, int sb, int gmax)
{
    const int block = shape.block > 0 ? shape.block : 256;
    int per_cu = shape.blocks_per_cu;
    if (per_cu <= 0) {
        int occ = 0;
        void (*kern)(RaggedArgs) = gmax == 2 ? k_ragged_mixed<2> : k_ragged_mixed<4>;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, block, ragged_lds(block, sb)) != hipSuccess ||
            occ <= 0)
            occ = 1;
        per_cu = occ;
    }
    return device_cu_count() * per_cu;
}

hipError_t launch_ragged(RaggedArgs a, LaunchShape shape, int grid, hipStream_t st)
{
    const int block = shape.block > 0 ? shape.block : 256;
    if (a.gmax == 2)
        hipLaunchKernelGGL(k_ragged_mixed<2>, dim3(grid > 0 ? grid : 1), dim3(block), ragged_lds(block, a.sb), st, a);
    else
        hipLaunchKernelGGL(k_ragged_mixed<4>, dim3(grid > 0 ? grid : 1), dim3(block), ragged_lds(block, a.sb), st, a);
    return hipGetLastError();
}

}  // namespace kep
