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

#include <mutex>
#include <vector>

#include "kep_device.h"
#include "kep_internal.h"
#include "kep_grad.h"
#include "kep_policy.h"

namespace kep {

// Residency target of the dense kernels: the mixed-precision variants with up
// to four chunks per lane are held to five wavefronts per SIMD (at most 102
// VGPRs).  With four chunks the compiler would otherwise use 126 VGPRs (four
// wavefronts); the extra wavefront lets the SIMD issue binary32 arithmetic
// from more wavefronts at once.  At five the four-chunk chi-square keeps 52
// bytes per lane in scratch (its HBM traffic 1.38 of the algorithmic bytes);
// held to four wavefronts it has none but ran 4% slower (c2 1.757 against
// 1.688 ms).
template <class Pol, int NCH>
constexpr int dense_waves_per_simd() { return (Pol::kMixed && NCH <= 4) ? 5 : 1; }

// The mixed kernels start the Kepler solve from the table of kep_start_tab.h,
// copied once into each block's LDS behind the records.
template <class Pol, int MODE>
constexpr bool dense_uses_table() { return Pol::kMixed; }

__host__ __device__ inline size_t dense_table_offset(int wpb, int sb, int n_pl, size_t rec_size)
{
    return ((size_t)wpb * sb * n_pl * rec_size + (size_t)wpb * sb * sizeof(int) + 15) & ~(size_t)15;
}

constexpr size_t kDenseTableBytes = sizeof(kep_start_tab);

template <class Pol, int NCH, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(dense_waves_per_simd<Pol, NCH>())))
k_dense(DenseArgs a)
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
    // mixed velocities: the block's copy of the starting-value table after the records
    const uint32_t *tab = nullptr;
    if constexpr (dense_uses_table<Pol, MODE>()) {
        uint32_t *t = reinterpret_cast<uint32_t *>(smem + dense_table_offset(wpb, a.sb, a.n_pl, sizeof(Rec)));
        load_start_table(t);
        tab = t;
    }

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
            if (a.offset) ok = ok && isfinite(a.offset[sys]);
            if (a.jitter) ok = ok && isfinite(a.jitter[sys]) && a.jitter[sys] >= 0.0;
            sysbad[lane] = ok ? 0 : 1;
        }
        wave_sync_lds();
        // planet records with the lanes over the batch's (planet, system) pairs,
        // planet-major (each parameter plane read in one run)
        for (int q = lane; q < nb * a.n_pl; q += 64) {
            const int j = q / nb, sq = q - j * nb;
            const int64_t p = (int64_t)j * a.n_sys + s0 + sq;
            Rec r;
            if (!Pol::setup(a, a.P[p], a.K[p], a.e[p], a.w[p], a.M0[p], r)) sysbad[sq] = 1;
            recs[sq * a.n_pl + j] = r;
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
                if constexpr (MODE == kAnomalies) {
                    // the same solve as the velocities' (so E is the root the model uses)
                    for (int j = 0; j < a.n_pl; ++j) {
                        const Rec &rr = recs[s * a.n_pl + j];
                        float *row = a.dv + ((int64_t)j * a.n_sys + sys) * a.n_obs;
                        float M[NCH], E[NCH], sv[NCH], omc[NCH];
#pragma unroll
                        for (int c = 0; c < NCH; ++c) M[c] = mean_anomaly32(o[c].tt, rr.ph);
                        PolMixed::solve<NCH, false>(rr.k, uniform_int(rr.niter), uniform_int(rr.check) != 0, rr.tp, M,
                                                    E, sv, omc, a.max_iter, tab);
#pragma unroll
                        for (int c = 0; c < NCH; ++c) {
                            if (o[c].in) {
                                const int64_t k = (int64_t)g * 64 * NCH + c * 64 + lane;
                                // streamed out: nontemporal stores (3.5% at c2)
                                __builtin_nontemporal_store((sbad || !o[c].ok) ? __builtin_nanf("") : E[c], row + k);
                            }
                        }
                    }
                    continue;
                }
                ModelAcc m[NCH];
                if (MODE == kPlanets) {
                    for (int j = 0; j < a.n_pl; ++j) {
#pragma unroll
                        for (int c = 0; c < NCH; ++c) Pol::model_init(m[c]);
                        pol_add_planet<Pol, NCH>(recs[s * a.n_pl + j], o, m, a, tab);
                        float *row = a.dv + ((int64_t)j * a.n_sys + sys) * a.n_obs;
#pragma unroll
                        for (int c = 0; c < NCH; ++c) {
                            if (o[c].in) {
                                const int64_t k = (int64_t)g * 64 * NCH + c * 64 + lane;
                                __builtin_nontemporal_store(
                                    (sbad || !o[c].ok) ? __builtin_nanf("") : (float)Pol::model_value(m[c]), row + k);
                            }
                        }
                    }
                    continue;
                }
#pragma unroll
                for (int c = 0; c < NCH; ++c) Pol::model_init(m[c]);
                for (int j = 0; j < a.n_pl; ++j) pol_add_planet<Pol, NCH>(recs[s * a.n_pl + j], o, m, a, tab);
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

// Second kernel of the separate-function form: planet sums, residuals and the
// chi-square (binary64 sums) from the velocities written by kPlanets.
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
        // every planet's row is requested before the first is summed (one row at a
        // time left too few bytes in flight to fill HBM); the sum keeps planet order
        float dv[kMaxPl][NCH];
#pragma unroll
        for (int j = 0; j < kMaxPl; ++j) {
            if (j < a.n_pl) {
                const float *row = a.dv + ((int64_t)j * a.n_sys + sys) * a.n_obs;
#pragma unroll
                for (int c = 0; c < NCH; ++c)  // read once: nontemporal loads (4% at c2)
                    dv[j][c] = o[c].in ? __builtin_nontemporal_load(row + c * 64 + lane) : 0.0f;
            }
        }
#pragma unroll
        for (int j = 0; j < kMaxPl; ++j) {
            if (j < a.n_pl) {
#pragma unroll
                for (int c = 0; c < NCH; ++c) m[c].add(dv[j][c]);
            }
        }
        PolMixed::ChiAcc chi;
        PolMixed::chi_init(chi);
        bool bad_obs = false;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            if (o[c].in) {
                bool okw = PolMixed::chi_add(chi, m[c], o[c], gam, jit, has_jit);
                bad_obs = bad_obs || !okw || !o[c].ok;
            }
        }
        const double tot = wave_sum(PolMixed::chi_value(chi));
        bad = bad || __any(bad_obs);
        if (lane == 0) a.out[sys] = bad ? __builtin_nan("") : tot;
    }
}

// ------------------------------------------------------------------ Kepler only
// Standalone Kepler solve (the paper's Kepler-only mode): one lane per pair.
// M is reduced to [-pi, pi] with 2 pi as a double-double; the root is returned
// on the input's branch.  Mixed: from the starting-value table (the block's
// LDS copy) and one quartic step where e <= KEP_TAB_EMAX, else the schedule.
template <bool MIXED>
__device__ __forceinline__ double kepler_one(double M, double e, int fixed, int max_iter, const uint32_t *tab)
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
        E = (double)kepler32_start((float)Mr, k, table_place(e, fixed <= 0), tab, niter, max_iter, fixed > 0, sE,
                                   omcE);
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
    const uint32_t *tab = nullptr;
    if constexpr (MIXED) {
        __shared__ uint32_t tab_s[kTabWords];    // Kepler starting values
        load_start_table(tab_s);
        tab = tab_s;
    }
    const int64_t tile = (int64_t)blockDim.x * KU;
    const int64_t stride = (int64_t)gridDim.x * tile;
    for (int64_t base = (int64_t)blockIdx.x * tile + threadIdx.x; base < n; base += stride) {
        double M[KU], e[KU];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x;
            // streamed once: nontemporal loads and stores (2^26 pairs: 4.74 -> 5.07 TB/s)
            M[u] = i < n ? __builtin_nontemporal_load(Mv + i) : 0.0;
            e[u] = i < n ? __builtin_nontemporal_load(ev + i) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x;
            const double E = kepler_one<MIXED>(M[u], e[u], fixed, max_iter, tab);
            if (i < n) __builtin_nontemporal_store(E, Ev + i);
        }
    }
}

// ------------------------------------------------------------------ gradient
// Plain binary64 chi-square and gradient with one lane per system (the
// adjoint needs 5 n_pl + 1 running sums per system; the lane that owns the
// system keeps them).  Observations are uniform across the wave and arrive
// through scalar loads.  The mixed-precision adjoint is in kep_adjoint.hip.
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

// ------------------------------------------------------------------ ragged
// Persistent kernel over CSR systems.  Work items are runs of `sb` systems of
// the plan's work order (decreasing work, grouped by planet count within
// short windows); each wavefront takes the next item from an atomic counter
// until the items run out.  Setup runs with the lanes over the item's (system, planet) pairs.
// Each system's whole groups of 64 observations are evaluated one system at a
// time with the lanes over its observations (uniform planet records, groups
// of up to 4 x 64 loaded with coalesced reads).  The remaining n_obs mod 64
// observations of all the item's systems are then packed back to back into
// one stream of lanes, each lane with its own system's planet records, and a
// segmented scan over each group of 64 lanes returns every system's share: a
// system's last partial group no longer leaves the rest of its wavefront idle.
// Observations of one unit of a system's whole groups (up to G groups of 64),
// as loaded.
template <int G>
struct RawObs {
    double t[G], v[G], s[G];
};

template <int G>
__device__ __forceinline__ void load_unit(const RaggedArgs &a, int64_t k0, int64_t left, RawObs<G> &r)
{
    const int lane = __lane_id();
#pragma unroll
    for (int c = 0; c < G; ++c) {
        const int64_t k = c * 64 + lane;
        const bool in = k < left;
        // read once per launch: nontemporal loads (c3 0.593-0.598 -> 0.588 ms)
        r.t[c] = in ? __builtin_nontemporal_load(a.t + k0 + k) : a.t0;
        r.v[c] = in ? __builtin_nontemporal_load(a.v + k0 + k) : 0.0;
        r.s[c] = in ? __builtin_nontemporal_load(a.sigma + k0 + k) : 1.0;
    }
}

// One unit (the first NCH of its groups) of a system's whole groups, with the
// lanes over its observations and uniform planet records.
template <int NCH, int G>
__device__ __forceinline__ void ragged_unit(const RaggedArgs &a, const RecMixed *recs, int npl, const RawObs<G> &r,
                                            int64_t left, double gam, double jit, bool has_jit, PolMixed::ChiAcc &chi,
                                            bool &bad_obs, const uint32_t *tab)
{
    const int lane = __lane_id();
    ObsMixed o[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        o[c].in = c * 64 + lane < left;
        o[c].ok = isfinite(r.t[c]) && isfinite(r.v[c]) && isfinite(r.s[c]) && r.s[c] >= 0.0;
        o[c].tt = r.t[c] - a.t0;
        o[c].v = r.v[c];
        o[c].s2 = (float)(r.s[c] * r.s[c]);
        o[c].w = rcp32(o[c].s2);
    }
    PolMixed::ModelAcc m[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) PolMixed::model_init(m[c]);
    for (int j = 0; j < npl; ++j) PolMixed::add_planet<NCH>(recs[j], o, m, a.max_iter, 0, tab);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        if (o[c].in) {
            bool okw = PolMixed::chi_add(chi, m[c], o[c], gam, jit, has_jit);
            bad_obs = bad_obs || !okw || !o[c].ok;
        }
    }
}

// One planet's velocity (the arithmetic of PolMixed::add_planet) from this
// lane's own planet record: lanes of different systems differ in step count.
__device__ __forceinline__ float ragged_vel_lane(const RecMixed &r, double tt, int max_iter, const uint32_t *tab)
{
    const float M = mean_anomaly32(tt, r.ph);
    float s, omc;
    kepler32_start(M, r.k, r.tp, tab, r.niter, max_iter, r.check != 0, s, omc);
    const float D = fmaf(r.k.e, omc, r.k.ome);           // 1 - e cos E
    const float num = fmaf(r.B, s, fmaf(-r.A, omc, r.A));  // A cos E + B sin E
    return num * rcp32(D);
}

// LDS of one wavefront for sb systems: planet records [sb][kMaxPl]; per
// system the first planet offset, the global index of its first tail
// observation and its chi-square so far; its first observation and the
// length of its whole groups [sb] each; its offset and jitter [sb][2];
// (code, system) pairs [sb][2], where code is the planet count, negative for
// an invalid system; per-planet domain flags [sb][kMaxPl]; prefix sums of the
// tail lengths [sb + 1]; bad-data flags [sb].
__host__ __device__ inline size_t ragged_lds_per_wave(int sb)
{
    const size_t b = (size_t)sb * kMaxPl * sizeof(RecMixed) + (size_t)sb * 2 * sizeof(int64_t) +
                     (size_t)sb * sizeof(double) + (size_t)sb * 2 * sizeof(int64_t) + (size_t)sb * 2 * sizeof(double) +
                     (size_t)sb * 2 * sizeof(int) + (size_t)sb * kMaxPl * sizeof(int) +
                     (size_t)(sb + 1) * sizeof(int) + (size_t)sb * sizeof(int);
    return (b + 15) & ~(size_t)15;
}

__device__ __forceinline__ int64_t uniform_i64(int64_t x)
{
    const int lo = __builtin_amdgcn_readfirstlane((int)(x & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(x >> 32));
    return ((int64_t)hi << 32) | (uint32_t)lo;
}

// GMAX: largest observation group in 64-lane chunks (2 or 4): fewer chunks in
// flight need fewer registers and allow more resident waves; the plan's
// autotuner picks it.  Five wavefronts per SIMD with two chunks (96 VGPRs, 16
// bytes of scratch), four with four (128 VGPRs, 68 bytes): at c3 the four-chunk
// form at four wavefronts runs 3% faster than the two-chunk one at four.
template <int GMAX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GMAX == 2 ? 5 : 4))) k_ragged_mixed(RaggedArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = __lane_id();
    const int wib = uniform_int(threadIdx.x >> 6);
    const int sb = a.sb;
    unsigned char *mine = smem + (size_t)wib * ragged_lds_per_wave(sb);
    RecMixed *recs = reinterpret_cast<RecMixed *>(mine);
    int64_t *pofs = reinterpret_cast<int64_t *>(recs + sb * kMaxPl);
    int64_t *tail0 = pofs + sb;
    double *acc = reinterpret_cast<double *>(tail0 + sb);
    int64_t *obs0 = reinterpret_cast<int64_t *>(acc + sb);
    int64_t *nfl = obs0 + sb;
    double *gj = reinterpret_cast<double *>(nfl + sb);
    int *meta = reinterpret_cast<int *>(gj + 2 * sb);
    int *okpl = meta + 2 * sb;
    int *tpre = okpl + sb * kMaxPl;
    int *bad = tpre + sb + 1;
    const bool has_jit = a.jitter != nullptr;
    __shared__ uint32_t tab[kTabWords];    // Kepler starting values
    __shared__ unsigned int drained;       // bit q: a wave of this block found queue q drained
    __shared__ unsigned int waves_out;     // the block's waves that have left the item loop
    if (threadIdx.x == 0) {
        drained = 0u;
        waves_out = 0u;
    }
    load_start_table(tab);                 // (its barrier also orders the stores above)

    // this block's XCD queue first (blocks go to the XCDs round-robin), then the
    // others.  Device-scope atomics on one address complete one after another, so
    // probes of a drained queue delay the takes still to come: a wave that finds a
    // queue drained marks it in the block's LDS, and the block's other waves skip it
    // (c3: 0.611 -> 0.599 ms together with the block-level exit count below).
    const int home = (int)(blockIdx.x % kRaggedQueues);
    int tried = 0;
    for (;;) {
        int64_t item = -1;
        while (tried < kRaggedQueues) {               // uniform: every lane takes part in the shuffle
            const int q = (home + tried) % kRaggedQueues;
            // a relaxed read: a mark not yet seen costs one more probe, nothing else
            const unsigned int seen = __hip_atomic_load(&drained, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if ((uniform_int((int)seen) >> q) & 1) {
                ++tried;
                continue;
            }
            unsigned int k = 0;
            if (lane == 0) k = atomicAdd(a.queue + q * kQueueStride, 1u);
            k = (unsigned int)uniform_int(__shfl((int)k, 0, 64));
            const int64_t it = (int64_t)k * kRaggedQueues + q;
            if (it < a.n_items) {
                item = it;
                break;
            }
            if (lane == 0) atomicOr(&drained, 1u << q);
            ++tried;
        }
        if (item < 0) break;
        const int64_t i0 = item * sb;
        const int nb = (int)min((int64_t)sb, a.n_sys - i0);
        wave_sync_lds();
        int rem = 0;
        if (lane < nb) {
            const int32_t code = a.order[i0 + lane];
            if (code >= 0) {
                const int64_t sys = code;
                const int64_t p0 = a.pl_off[sys];
                const int64_t o0 = a.obs_off[sys], n = a.obs_off[sys + 1] - o0;
                // the system's offset and jitter with its offsets, not behind the
                // planet parameters (one dependent round trip fewer per item)
                gj[2 * lane] = a.offset ? a.offset[sys] : 0.0;
                gj[2 * lane + 1] = a.jitter ? a.jitter[sys] : 0.0;
                meta[2 * lane] = (int)(a.pl_off[sys + 1] - p0);
                meta[2 * lane + 1] = (int)sys;
                pofs[lane] = p0;
                rem = (int)(n & 63);
                tail0[lane] = o0 + (n - rem);
                obs0[lane] = o0;
                nfl[lane] = n - rem;
            } else {
                // a system whose offsets failed the on-device check (-1 - index):
                // its offsets are not read again and its chi-square is NaN
                meta[2 * lane] = 0;
                meta[2 * lane + 1] = -1 - code;
                gj[2 * lane] = 0.0;
                gj[2 * lane + 1] = 0.0;
                pofs[lane] = 0;
                tail0[lane] = 0;
                obs0[lane] = 0;
                nfl[lane] = 0;
            }
            acc[lane] = 0.0;
            bad[lane] = 0;
        }
        // prefix sums of the tail lengths over the item's systems
        int incl = rem;
        for (int d = 1; d < 64; d <<= 1) {
            const int u = __shfl_up(incl, d, 64);
            if (lane >= d) incl += u;
        }
        if (lane < nb) tpre[lane + 1] = incl;
        if (lane == 0) tpre[0] = 0;
        const int ntail = uniform_int(__shfl(incl, nb - 1, 64));
        wave_sync_lds();
        DenseArgs dummy;
        dummy.fixed_iter = a.fixed_iter;
        for (int q = lane; q < nb * kMaxPl; q += 64) {
            const int s = q / kMaxPl, j = q - s * kMaxPl;
            if (j < meta[2 * s]) {
                const int64_t p = pofs[s] + j;
                RecMixed r;
                okpl[q] = PolMixed::setup(dummy, a.P[p], a.K[p], a.e[p], a.w[p], a.M0[p], r) ? 1 : 0;
                recs[q] = r;
            }
        }
        wave_sync_lds();
        if (lane < nb) {
            const int npl = meta[2 * lane];
            bool ok = isfinite(a.t0) && npl >= 1 && npl <= kMaxPl;
            for (int j = 0; j < kMaxPl; ++j)
                if (j < npl) ok = ok && okpl[lane * kMaxPl + j] != 0;
            const double g = gj[2 * lane], sj = gj[2 * lane + 1];
            if (a.offset) ok = ok && isfinite(g);
            if (a.jitter) ok = ok && isfinite(sj) && sj >= 0.0;
            meta[2 * lane] = ok ? npl : -npl;
        }
        wave_sync_lds();
        // whole groups of 64 observations, one system at a time, in units of up to
        // GMAX groups.  Each unit's observations are loaded when it starts: the
        // other resident wavefronts cover the wait, and loading the next unit's
        // ahead (registers for two units) cost a wavefront per SIMD, 3% at c3.
        {
            auto has_units = [&](int q) { return uniform_int(meta[2 * q]) > 0 && uniform_i64(nfl[q]) > 0; };
            int us = 0;
            while (us < nb && !has_units(us)) ++us;
            int64_t ug = 0;
            RawObs<GMAX> cur;
            PolMixed::ChiAcc chi;
            PolMixed::chi_init(chi);
            bool bad_obs = false;
            while (us < nb) {
                const int64_t nf = uniform_i64(nfl[us]);
                int ns = us;
                int64_t ng = ug + 64 * GMAX;
                if (ng >= nf) {
                    ns = us + 1;
                    while (ns < nb && !has_units(ns)) ++ns;
                    ng = 0;
                }
                load_unit<GMAX>(a, uniform_i64(obs0[us]) + ug, nf - ug, cur);
                const int64_t left = nf - ug;
                const int code = uniform_int(meta[2 * us]);
                const double gam = gj[2 * us], jit = gj[2 * us + 1];
                const RecMixed *rs = recs + us * kMaxPl;
                if (left <= 64) ragged_unit<1, GMAX>(a, rs, code, cur, left, gam, jit, has_jit, chi, bad_obs, tab);
                else if (GMAX == 2 || left <= 128)
                    ragged_unit<2, GMAX>(a, rs, code, cur, left, gam, jit, has_jit, chi, bad_obs, tab);
                else if (left <= 192) ragged_unit<3, GMAX>(a, rs, code, cur, left, gam, jit, has_jit, chi, bad_obs, tab);
                else ragged_unit<GMAX, GMAX>(a, rs, code, cur, left, gam, jit, has_jit, chi, bad_obs, tab);
                if (ns != us) {
                    const double tot = wave_sum(PolMixed::chi_value(chi));
                    const bool b = __any(bad_obs);
                    if (lane == 0) {
                        acc[us] = tot;
                        bad[us] = b ? 1 : 0;
                    }
                    PolMixed::chi_init(chi);
                    bad_obs = false;
                }
                us = ns;
                ug = ng;
            }
        }
        wave_sync_lds();
        // the packed tails: lane position p of the stream belongs to system s
        // with tpre[s] <= p < tpre[s + 1].  Positions only grow along the
        // stream, so each lane moves its system cursor forward; the next
        // group's observations are loaded before the current group is
        // evaluated.
        if (ntail > 0) {
            int s = 0;
            auto seek = [&](int pos) {
                while (s + 1 < nb && tpre[s + 1] <= pos) ++s;
            };
            auto fetch = [&](int pos, bool in, double &t, double &v, double &sg) {
                t = a.t0;
                v = 0.0;
                sg = 1.0;
                if (in && meta[2 * s] > 0) {
                    const int64_t k = tail0[s] + (pos - tpre[s]);
                    t = __builtin_nontemporal_load(a.t + k);
                    v = __builtin_nontemporal_load(a.v + k);
                    sg = __builtin_nontemporal_load(a.sigma + k);
                }
            };
            bool in = lane < ntail;
            int pp = in ? lane : ntail - 1;
            seek(pp);
            double t, v, sg;
            fetch(pp, in, t, v, sg);
            for (int c0 = 0; c0 < ntail; c0 += 64) {
                const int sc = s;
                const bool inc = in;
                const double tc = t, vc = v, sgc = sg;
                if (c0 + 64 < ntail) {                  // next group: cursor and loads
                    in = c0 + 64 + lane < ntail;
                    pp = in ? c0 + 64 + lane : ntail - 1;
                    seek(pp);
                    fetch(pp, in, t, v, sg);
                }
                const int code = meta[2 * sc];
                const int npl = inc && code > 0 ? code : 0;
                double x = 0.0;
                if (npl > 0) {
                    ObsMixed o;
                    o.in = true;
                    o.ok = isfinite(tc) && isfinite(vc) && isfinite(sgc) && sgc >= 0.0;
                    o.tt = tc - a.t0;
                    o.v = vc;
                    o.s2 = (float)(sgc * sgc);
                    o.w = rcp32(o.s2);
                    PolMixed::ModelAcc m;
                    PolMixed::model_init(m);
                    const RecMixed *rs = recs + sc * kMaxPl;
                    for (int j = 0; j < npl; ++j) m.add(ragged_vel_lane(rs[j], o.tt, a.max_iter, tab));
                    const double gam = gj[2 * sc], jit = gj[2 * sc + 1];
                    PolMixed::ChiAcc cx;
                    PolMixed::chi_init(cx);
                    const bool okw = PolMixed::chi_add(cx, m, o, gam, jit, has_jit);
                    x = PolMixed::chi_value(cx);
                    if (!okw || !o.ok) bad[sc] = 1;     // every writer stores the same value
                }
                // segmented scan: a lane adds only partial sums that start inside
                // its own system's run of lanes (from `head`), so the lane that
                // ends the run holds that system's share of this group, and a
                // non-finite value stays within its own system
                const int head = max(tpre[sc] - c0, 0);
                const int last = min(tpre[sc + 1] - c0, 64) - 1;
                double sum = x;
                for (int d = 1; d < 64; d <<= 1) {
                    const double u = __shfl_up(sum, d, 64);
                    if (lane - d >= head) sum += u;
                }
                if (inc && lane == last && code > 0) acc[sc] += sum;
                wave_sync_lds();
            }
        }
        if (lane < nb) {
            const int code = meta[2 * lane];
            a.out[meta[2 * lane + 1]] = (code <= 0 || bad[lane] != 0) ? __builtin_nan("") : acc[lane];
        }
    }
    // The last wave to leave resets the counters for the next launch, so no
    // reset launch is needed between launches: every wave counts itself out
    // after its last (failed) take from the queue, the last of a block counts
    // the block out (one global atomic per block, not per wave: 0.627 -> 0.611
    // ms at c3), so when the count reaches the number of blocks no wave of this
    // launch touches the queue again.
    if (lane == 0 && atomicAdd(&waves_out, 1u) == (blockDim.x >> 6) - 1) {
        if (atomicAdd(a.queue + kQueueDone, 1u) == gridDim.x - 1) {
            for (int q = 0; q < kRaggedQueues; ++q) atomicExch(a.queue + q * kQueueStride, 0u);
            atomicExch(a.queue + kQueueDone, 0u);
        }
    }
}

// ------------------------------------------------------- ragged, no allocation
// Device memory of the allocation-free ragged entry point: the work-queue
// and exit counters in the first 256 bytes, then the int32 work order of up to
// kStaticMaxSys systems.  One copy per GPU, kept until the process ends; every
// call on a GPU shares it (calls that overlap in time on one GPU race).
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kPrepThreads = 1024;
constexpr int kPrepKeys = kMaxPl + 1;      // planet counts 8 .. 1, then rejected systems

// One block: zeroes the queue counters, checks every system's CSR offsets
// (0 <= o0 <= o1 <= n_obs_total, 0 <= p0 < p1 <= n_pl_total, p1 - p0 <= kMaxPl)
// and writes the work order: systems by decreasing planet count (so that the
// systems of a work item share their planet count), index order within a
// count (a stable counting sort: the order, and so every result, is the same
// on every call), the rejected systems last as -1 - index.  Thread t owns the
// contiguous run of systems [t c, (t + 1) c).
__global__ void __launch_bounds__(kPrepThreads) k_ragged_static_order(const int64_t *__restrict__ obs_off,
                                                                      const int64_t *__restrict__ pl_off,
                                                                      int64_t n_sys, int64_t n_obs_total,
                                                                      int64_t n_pl_total, int32_t *__restrict__ order,
                                                                      unsigned int *__restrict__ queue)
{
    __shared__ int wtot[kPrepKeys][kPrepThreads / 64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int q = t; q < kQueueWords; q += kPrepThreads) queue[q] = 0u;
    const int64_t c = (n_sys + kPrepThreads - 1) / kPrepThreads;
    const int64_t i0 = min(n_sys, (int64_t)t * c), i1 = min(n_sys, i0 + c);
    auto key_of = [&](int64_t i) {
        const int64_t o0 = obs_off[i], o1 = obs_off[i + 1], p0 = pl_off[i], p1 = pl_off[i + 1];
        const bool ok = o0 >= 0 && o0 <= o1 && o1 <= n_obs_total && p0 >= 0 && p0 < p1 && p1 <= n_pl_total &&
                        p1 - p0 <= kMaxPl;
        return ok ? kMaxPl - (int)(p1 - p0) : kMaxPl;      // 0 for 8 planets ... 7 for one, 8 rejected
    };
    int cnt[kPrepKeys];
#pragma unroll
    for (int k = 0; k < kPrepKeys; ++k) cnt[k] = 0;
    for (int64_t i = i0; i < i1; ++i) {
        const int k = key_of(i);
#pragma unroll
        for (int q = 0; q < kPrepKeys; ++q) cnt[q] += (q == k);
    }
    // exclusive prefix of every key's count over the threads (wave scans, then the waves)
    int pre[kPrepKeys];
#pragma unroll
    for (int k = 0; k < kPrepKeys; ++k) {
        int incl = cnt[k];
        for (int d = 1; d < 64; d <<= 1) {
            const int u = __shfl_up(incl, d, 64);
            if (lane >= d) incl += u;
        }
        pre[k] = incl - cnt[k];
        if (lane == 63) wtot[k][w] = incl;
    }
    __syncthreads();
    int64_t base = 0;
#pragma unroll
    for (int k = 0; k < kPrepKeys; ++k) {
        int64_t tot = 0, before = 0;
        for (int q = 0; q < kPrepThreads / 64; ++q) {
            tot += wtot[k][q];
            if (q < w) before += wtot[k][q];
        }
        cnt[k] = (int)(base + before + pre[k]);          // this thread's first slot for key k
        base += tot;
    }
    for (int64_t i = i0; i < i1; ++i) {
        const int k = key_of(i);
        int slot = 0;
#pragma unroll
        for (int q = 0; q < kPrepKeys; ++q) {
            if (q == k) {
                slot = cnt[q];
                cnt[q] += 1;
            }
        }
        order[slot] = k < kMaxPl ? (int32_t)i : (int32_t)(-1 - i);
    }
}

// The scratch array's device address on each GPU (host code must not use the
// array's name: on the host it is a stand-in, not a device address).
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64];

hipError_t static_scratch(void **ptr)
{
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (err != hipSuccess) return err;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_ragged_static(RaggedArgs a, LaunchShape shape, hipStream_t st)
{
    if (a.n_sys <= 0) return hipSuccess;
    if (a.n_sys > kStaticMaxSys) return hipErrorInvalidValue;
    void *base = nullptr;
    hipError_t err = static_scratch(&base);
    if (err != hipSuccess) return err;
    unsigned int *queue = reinterpret_cast<unsigned int *>(base);
    int32_t *order = reinterpret_cast<int32_t *>(reinterpret_cast<unsigned char *>(base) + kStaticQueueBytes);
    hipLaunchKernelGGL(k_ragged_static_order, dim3(1), dim3(kPrepThreads), 0, st, a.obs_off, a.pl_off, a.n_sys,
                       a.n_obs_total, a.n_pl_total, order, queue);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    a.order = order;
    a.queue = queue;
    a.n_items = (a.n_sys + a.sb - 1) / a.sb;
    const int block = shape.block > 0 ? shape.block : 256;
    const int wpb = block / 64;
    const int64_t need = (a.n_items + wpb - 1) / wpb;
    const int64_t cap = ragged_max_grid(shape, a.sb, a.gmax);
    const int grid = (int)(need < cap ? need : cap);
    return launch_ragged(a, shape, grid, st);
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

// Occupancy per (device, kernel, block size, LDS bytes), looked up once: the
// runtime query costs microseconds, as much as a small launch.
int cached_occupancy(const void *kern, int block, size_t lds)
{
    struct Entry { int dev; const void *kern; int block; size_t lds; int occ; };
    static std::mutex mu;
    static std::vector<Entry> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    {
        std::lock_guard<std::mutex> lock(mu);
        for (const Entry &e : cache)
            if (e.dev == dev && e.kern == kern && e.block == block && e.lds == lds) return e.occ;
    }
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, block, lds) != hipSuccess || occ <= 0) occ = 1;
    std::lock_guard<std::mutex> lock(mu);
    if (cache.size() < 4096) cache.push_back(Entry{dev, kern, block, lds, occ});
    return occ;
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
    constexpr bool table = dense_uses_table<Pol, MODE>();
    auto lds_of = [&](int64_t sb) {
        return table ? dense_table_offset(wpb, (int)sb, a.n_pl, sizeof(typename Pol::Rec)) + kDenseTableBytes
                     : rec_bytes * (size_t)sb;
    };
    // systems per setup batch: at most kMaxSB and at most 48 KiB of LDS per block
    // (with the table, 32 KiB: five blocks of four wavefronts share a CU's 160 KiB)
    const int64_t budget = table ? (int64_t)(32 * 1024) - (int64_t)kDenseTableBytes - 16 : (int64_t)(48 * 1024);
    int64_t sb_cap = budget / (int64_t)rec_bytes;
    sb_cap = sb_cap < 1 ? 1 : (sb_cap > kMaxSB ? kMaxSB : sb_cap);
    // a multiple of 16 systems reads whole 128-byte lines of every parameter plane:
    // a line split between two batches may be fetched by two XCDs' L2s
    if (sb_cap > 16) sb_cap &= ~(int64_t)15;
    size_t lds = lds_of(sb_cap);
    const int nch_needed = (int)((a.n_obs + 63) / 64);
    void (*kern)(DenseArgs);
    int nch;
    if (nch_needed <= 1) { kern = k_dense<Pol, 1, MODE>; nch = 1; }
    else if (nch_needed <= 2) { kern = k_dense<Pol, 2, MODE>; nch = 2; }
    else if (nch_needed <= 4) { kern = k_dense<Pol, 4, MODE>; nch = 4; }
    else { kern = k_dense<Pol, 8, MODE>; nch = 8; }
    int per_cu = shape.blocks_per_cu;
    if (per_cu <= 0) {
        per_cu = cached_occupancy((const void *)kern, block, lds);
    }
    const int64_t max_waves = (int64_t)device_cu_count() * per_cu * wpb;
    // ceil: every wave gets at most one batch when the cap allows it, so no wave
    // runs a second batch while the others idle
    const int64_t mw = max_waves > 0 ? max_waves : 1;
    int64_t sb = (a.n_sys + mw - 1) / mw;
    sb = sb < 1 ? 1 : (sb > sb_cap ? sb_cap : sb);
    a.sb = (int)sb;
    lds = lds_of(sb);
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

hipError_t launch_eccentric_anomalies(DenseArgs a, LaunchShape shape, hipStream_t st)
{
    if (a.n_sys <= 0 || a.n_obs <= 0) return hipSuccess;
    return launch_dense_t<PolMixed, kAnomalies>(a, shape, st);
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
    if (prec == Prec::Mixed) return launch_grad_mixed(a, nll, shape, st);
    const int block = shape.block > 0 ? shape.block : 256;
    const int grid = grad_grid(a.n_sys, block, shape.blocks_per_cu);
#define KEP_GRAD_LAUNCH(N, L) hipLaunchKernelGGL((k_grad_f64<N, L>), dim3(grid), dim3(block), 0, st, a);
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
    return (size_t)(block / 64) * ragged_lds_per_wave(sb);
}

// The block's LDS is the waves' dynamic slices plus the static copy of the
// Kepler starting-value table and the block's two queue words (16 bytes
// allowed for them and their alignment).
bool ragged_shape_fits(int block, int sb) { return ragged_lds(block, sb) + sizeof(kep_start_tab) + 16 <= 64 * 1024; }

int ragged_max_grid(LaunchShape shape, int sb, int gmax)
{
    const int block = shape.block > 0 ? shape.block : 256;
    int per_cu = shape.blocks_per_cu;
    if (per_cu <= 0) {
        void (*kern)(RaggedArgs) = gmax == 2 ? k_ragged_mixed<2> : k_ragged_mixed<4>;
        per_cu = cached_occupancy((const void *)kern, block, ragged_lds(block, sb));
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
