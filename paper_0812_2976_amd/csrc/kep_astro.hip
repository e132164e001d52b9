// Astrometric Keplerian model on gfx950: the star's reflex offset on the sky,
// dRA* = B X + G Y and dDec = A X + F Y with X = cos E - e and
// Y = sqrt(1 - e^2) sin E (Thiele-Innes form), summed over planets, and its
// chi-square against measured offsets.  It is the larger-dynamic-range use of
// the same phase and Kepler core (Sec. 5.1 notes that binary32 is not enough
// there): an orbit of 100 mas measured to 0.01 mas needs E to ~1e-7 rad or
// better, below binary32's resolution of E.  The mixed path therefore keeps
// the binary64 phase and the binary32 Danby iteration and adds one Newton
// correction in binary64 against the binary64 mean anomaly (the binary32
// iterate is within ~1e-6 rad, so the corrected E is within ~1e-11 rad), then
// forms X, Y, the positions and the residuals in binary64.
//
// Mapping as in the dense RV kernels: one wavefront per system at a time with
// the lanes over observations (NCH register chunks), per-planet constants
// built with the lanes over systems and handed over through LDS.
#include <hip/hip_runtime.h>

#include "kep_device.h"
#include "kep_grad.h"
#include "kep_internal.h"
#include "kep_policy.h"

namespace kep {

namespace {

struct AstroRec {          // one per (system, planet)
    Phase64 ph;            // P, 1/P, fract(M0/(2 pi) + 1/2)
    double M0, e, b;       // b = sqrt(1 - e^2)
    double A, B, F, G;
    Ecc32 k;
    TabPlace tp;           // place in the starting-value table (toff -1: the paper's guess)
    int niter, check;
};

struct AstroObs {
    double t, x, y, wx, wy;
    bool in, ok;
};

__device__ __forceinline__ bool astro_setup(const AstroArgs &a, int64_t p, AstroRec &r)
{
    double P = a.P[p], e = a.e[p], M0 = a.M0[p], A = a.A[p], B = a.B[p], F = a.F[p], G = a.G[p];
    const bool ok = isfinite(P) && P > 0.0 && isfinite(e) && e >= 0.0 && e < 1.0 && isfinite(M0) &&
                    isfinite(A) && isfinite(B) && isfinite(F) && isfinite(G);
    if (!ok) { P = 1.0; e = 0.0; M0 = 0.0; A = B = F = G = 0.0; }
    r.ph = make_phase64(P, M0);
    r.M0 = M0;
    r.e = e;
    r.b = sqrt((1.0 - e) * (1.0 + e));
    r.A = A;
    r.B = B;
    r.F = F;
    r.G = G;
    r.k = make_ecc32(e);
    r.niter = a.fixed_iter > 0 ? a.fixed_iter : sched32(r.k.e);
    r.check = a.fixed_iter > 0 ? 1 : 0;
    r.tp = table_place(e, a.fixed_iter <= 0);
    return ok;
}

// cos E and sin E of one planet at tt = t - t0, mixed precision: binary64
// centred phase M, binary32 Danby iteration on (float)M (from the starting-value
// table where e <= KEP_TAB_EMAX), one binary64 Newton step against M (binary64
// sin/cos of the binary32 root from the block's knots; 1/(1 - e cos E) from the
// binary32 reciprocal and one Newton step, relative 1e-14 on a step of ~1e-7
// rad), sin/cos carried to the corrected E to second order.
__device__ __forceinline__ void astro_cs_mixed(const AstroRec &r, double tt, int max_iter, const uint32_t *tab,
                                               const double2 *knots, double &cE, double &sE)
{
    const double q0 = tt * r.ph.rP;
    const double res = fma(-q0, r.ph.P, tt);
    const double q = fma(res, r.ph.rP, q0);
    const double u = __builtin_amdgcn_fract(__builtin_amdgcn_fract(q) + r.ph.m0h);
    const double M = fma(u, kTwoPi, -kPi);
    float s32, omc32;
    const float E32 = clamp_root(kepler32_start((float)M, r.k, r.tp, tab, r.niter, max_iter, r.check != 0, s32,
                                                omc32));
    const double E0 = (double)E32;
    double s, c;
    sincos_root64_knots(E32, knots, s, c);
    const double D = fma(-r.e, c, 1.0);
    const double r0 = (double)rcp32((float)D);
    const double d = -fma(-r.e, s, E0 - M) * fma(r0, fma(-D, r0, 1.0), r0);
    const double hd2 = 0.5 * d * d;
    cE = c - d * s - hd2 * c;
    sE = s + d * c - hd2 * s;
}

// Plain binary64: IEEE quotient, M in [0, 2 pi), Danby iteration (kepler64).
__device__ __forceinline__ void astro_cs_f64(const AstroRec &r, double tt, int fixed, int max_iter, double &cE,
                                             double &sE)
{
    const double q = tt / r.ph.P;
    const double phi = q - floor(q);
    double M = fma(kTwoPi, phi, r.M0);
    M = M - kTwoPi * floor(M * kInvTwoPi);
    const double E = kepler64(M, r.e, M < kPi ? 1.0 : -1.0, fixed, max_iter);
    sincos(E, &sE, &cE);
}

template <bool MIXED, int NCH, bool MODEL>
__global__ void __launch_bounds__(256) k_astro(AstroArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = __lane_id();
    const int wpb = blockDim.x >> 6;
    const int wib = uniform_int(threadIdx.x >> 6);
    const int npl = a.n_pl;
    AstroRec *recs = reinterpret_cast<AstroRec *>(smem) + (size_t)wib * a.sb * npl;
    int *sysbad = reinterpret_cast<int *>(smem + (size_t)wpb * a.sb * npl * sizeof(AstroRec)) + wib * a.sb;
    // mixed: the block's copy of the Kepler starting-value table
    const uint32_t *tab = nullptr;
    const double2 *knots = nullptr;
    if constexpr (MIXED) {
        __shared__ uint32_t tab_s[kTabWords];
        __shared__ double2 knots_s[kSc64Knots];
        fill_sincos64_knots(knots_s);
        load_start_table(tab_s);        // ends with the block barrier
        tab = tab_s;
        knots = knots_s;
    }

    const int64_t gw = (int64_t)blockIdx.x * wpb + wib;
    const int64_t n_waves = (int64_t)gridDim.x * wpb;
    const int64_t n_batches = (a.n_sys + a.sb - 1) / a.sb;
    const int n_groups = (int)((a.n_obs + 64 * NCH - 1) / (64 * NCH));
    const int fixed = a.fixed_iter > 0 ? a.fixed_iter : (a.fixed_iter == 0 ? 30 : 0);

    AstroObs o[NCH];
    auto load_group = [&](int g) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int64_t k = (int64_t)g * 64 * NCH + c * 64 + lane;
            o[c].in = k < a.n_obs;
            o[c].ok = true;
            if (!o[c].in) continue;
            o[c].t = a.t[k];
            o[c].ok = isfinite(o[c].t);
            if (!MODEL) {
                o[c].x = a.x[k];
                o[c].y = a.y[k];
                const double sx = a.sx[k], sy = a.sy[k];
                o[c].ok = o[c].ok && isfinite(o[c].x) && isfinite(o[c].y) && isfinite(sx) && isfinite(sy) &&
                          sx > 0.0 && sy > 0.0;
                o[c].wx = 1.0 / (sx * sx);
                o[c].wy = 1.0 / (sy * sy);
            }
        }
    };
    if (n_groups <= 1) load_group(0);

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
                for (int j = 0; j < npl; ++j) {
                    AstroRec r;
                    ok = astro_setup(a, (int64_t)j * a.n_sys + sys, r) && ok;
                    recs[lane * npl + j] = r;
                }
                if (a.x0) ok = ok && isfinite(a.x0[sys]);
                if (a.y0) ok = ok && isfinite(a.y0[sys]);
                sysbad[lane] = ok ? 0 : 1;
            }
            wave_sync_lds();
        }
        for (int s = 0; s < nb; ++s) {
            const int64_t sys = s0 + s;
            const double x0 = a.x0 ? a.x0[sys] : 0.0, y0 = a.y0 ? a.y0[sys] : 0.0;
            const bool sbad = uniform_int(sysbad[s]) != 0;
            double chi = 0.0;
            bool bad_obs = false;
            for (int g = g_first; g < g_end; ++g) {
                if (n_groups > 1) load_group(g);
                double ra[NCH], dec[NCH];
#pragma unroll
                for (int c = 0; c < NCH; ++c) ra[c] = dec[c] = 0.0;
                for (int j = 0; j < npl; ++j) {
                    const AstroRec &r = recs[s * npl + j];
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
                        if (!o[c].in) continue;
                        double cE, sE;
                        if (MIXED) astro_cs_mixed(r, o[c].t - a.t0, a.max_iter, tab, knots, cE, sE);
                        else astro_cs_f64(r, o[c].t - a.t0, fixed, a.max_iter, cE, sE);
                        const double X = cE - r.e, Y = r.b * sE;
                        ra[c] = fma(r.B, X, fma(r.G, Y, ra[c]));
                        dec[c] = fma(r.A, X, fma(r.F, Y, dec[c]));
                    }
                }
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    if (!o[c].in) continue;
                    const int64_t k = (int64_t)g * 64 * NCH + c * 64 + lane;
                    if (MODEL) {
                        const bool bad = sbad || !o[c].ok;
                        a.out[(sys * 2 + 0) * a.n_obs + k] = bad ? __builtin_nan("") : ra[c] + x0;
                        a.out[(sys * 2 + 1) * a.n_obs + k] = bad ? __builtin_nan("") : dec[c] + y0;
                    } else {
                        const double rx = (ra[c] + x0) - o[c].x, ry = (dec[c] + y0) - o[c].y;
                        chi = fma(o[c].wx * rx, rx, fma(o[c].wy * ry, ry, chi));
                        bad_obs = bad_obs || !o[c].ok;
                    }
                }
            }
            if (!MODEL) {
                const double tot = wave_sum(chi);
                const bool bad = sbad || __any(bad_obs);
                if (lane == 0) a.out[sys] = bad ? __builtin_nan("") : tot;
            }
        }
    }
}

template <bool MIXED, bool MODEL>
hipError_t launch_astro_t(AstroArgs a, LaunchShape shape, hipStream_t st)
{
    const int block = shape.block > 0 ? shape.block : 256;
    const int wpb = block / 64;
    const size_t rec_bytes = (size_t)wpb * a.n_pl * sizeof(AstroRec) + (size_t)wpb * sizeof(int);
    // records and (mixed) the block's tables within 32 KiB, so that five blocks
    // of four wavefronts share a CU's 160 KiB (the binary32-iteration kernels
    // fit five wavefronts per SIMD in registers; at 1,048,576 x 2 x 128,
    // 48 KiB and three blocks: 1.15 ms, 40 KiB: 1.08 ms, 32 KiB: 1.06 ms)
    const int64_t tables = MIXED ? (int64_t)(sizeof(kep_start_tab) + kSc64Bytes) : 0;
    int64_t sb_cap = ((int64_t)(32 * 1024) - tables) / (int64_t)rec_bytes;
    sb_cap = sb_cap < 1 ? 1 : (sb_cap > kMaxSB ? kMaxSB : sb_cap);
    const int nch_needed = (int)((a.n_obs + 63) / 64);
    void (*kern)(AstroArgs);
    int nch;
    if (nch_needed <= 1) { kern = k_astro<MIXED, 1, MODEL>; nch = 1; }
    else if (nch_needed <= 2) { kern = k_astro<MIXED, 2, MODEL>; nch = 2; }
    else { kern = k_astro<MIXED, 4, MODEL>; nch = 4; }
    int per_cu = shape.blocks_per_cu;
    if (per_cu <= 0) {
        per_cu = cached_occupancy((const void *)kern, block, rec_bytes * (size_t)sb_cap);
    }
    const int64_t mw = (int64_t)device_cu_count() * per_cu * wpb;
    int64_t sb = (a.n_sys + mw - 1) / (mw > 0 ? mw : 1);
    sb = sb < 1 ? 1 : (sb > sb_cap ? sb_cap : sb);
    a.sb = (int)sb;
    const size_t lds = rec_bytes * (size_t)sb;
    const int64_t n_batches = (a.n_sys + sb - 1) / sb;
    const int64_t n_groups = (a.n_obs + 64 * nch - 1) / (64 * nch);
    const int64_t n_items = MODEL ? n_batches * (n_groups > 0 ? n_groups : 1) : n_batches;
    int64_t grid = (n_items + wpb - 1) / wpb;
    const int64_t cap = (int64_t)device_cu_count() * per_cu;
    if (grid > cap) grid = cap;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(block), lds, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_astro(AstroArgs a, Prec prec, bool model, LaunchShape shape, hipStream_t st)
{
    if (a.n_sys <= 0) return hipSuccess;
    if (model && a.n_obs <= 0) return hipSuccess;
    if (prec == Prec::Mixed)
        return model ? launch_astro_t<true, true>(a, shape, st) : launch_astro_t<true, false>(a, shape, st);
    return model ? launch_astro_t<false, true>(a, shape, st) : launch_astro_t<false, false>(a, shape, st);
}

}  // namespace kep
