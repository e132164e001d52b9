// Plain binary64 chi-square of a ragged (CSR) batch: the paper's
// double-precision variant (Sec. 5.1, Eq. 1-5) over systems that each have
// their own planet and observation counts.  One wavefront per system at a
// time, grid-stride over the positions of the work order (or over the systems
// in their own order when there is none); lanes over the system's
// observations in groups of up to four 64-lane chunks, the planet records
// built by the first n_pl lanes into the wavefront's LDS slice, every planet
// evaluated as in the dense binary64 kernel (IEEE quotient, 30 Danby steps by
// default) and the chi-square summed in binary64.
//
// Every wavefront checks its system's offsets against the CSR totals before
// it reads anything else of the system, so the kernel also runs on offsets
// that no host code has checked: a system whose offsets are inconsistent
// (decreasing, beyond the totals, planet count outside [1, kMaxPl]) gets a NaN
// chi-square and none of its arrays is read.
#include <hip/hip_runtime.h>

#include "kep_device.h"
#include "kep_internal.h"
#include "kep_policy.h"

namespace kep {

namespace {

// One group of up to 64 NC observations of a system (starting at index g0 of
// its n): loads, every planet, and the chi-square terms of the lanes in range.
template <int NC>
__device__ __forceinline__ void ragged64_group(const RaggedArgs &a, const Rec64 *recs, int npl, int64_t o0,
                                               int64_t n, int64_t g0, double gam, double jit, bool has_jit,
                                               int fixed, Pol64::ChiAcc &chi, bool &bad_obs)
{
    const int lane = __lane_id();
    Obs64 o[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int64_t i = g0 + c * 64 + lane;
        o[c].in = i < n;
        const double t = o[c].in ? a.t[o0 + i] : a.t0;
        const double v = o[c].in ? a.v[o0 + i] : 0.0;
        const double s = o[c].in ? a.sigma[o0 + i] : 1.0;
        o[c].ok = isfinite(t) && isfinite(v) && isfinite(s) && s >= 0.0;
        o[c].tt = t - a.t0;
        o[c].v = v;
        o[c].s2 = s * s;
        o[c].w = 1.0 / (s * s);
    }
    Pol64::ModelAcc m[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) Pol64::model_init(m[c]);
    for (int j = 0; j < npl; ++j) Pol64::add_planet<NC>(recs[j], o, m, a.max_iter, fixed);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (o[c].in) {
            const bool okw = Pol64::chi_add(chi, m[c], o[c], gam, jit, has_jit);
            bad_obs = bad_obs || !okw || !o[c].ok;
        }
    }
}

__global__ void __launch_bounds__(256) k_ragged64(RaggedArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = __lane_id();
    const int wpb = blockDim.x >> 6;
    const int wib = uniform_int(threadIdx.x >> 6);
    Rec64 *recs = reinterpret_cast<Rec64 *>(smem) + (size_t)wib * kMaxPl;
    const int64_t n_waves = (int64_t)gridDim.x * wpb;
    const int fixed = fixed64(a.fixed_iter);
    const bool has_jit = a.jitter != nullptr;
    const double nan = __builtin_nan("");
    DenseArgs unused{};                      // Pol64::setup takes the dense arguments and reads none

    for (int64_t pos = (int64_t)blockIdx.x * wpb + wib; pos < a.n_sys; pos += n_waves) {
        int64_t sys = pos;
        bool bad = false;
        if (a.order) {
            const int32_t code = a.order[pos];
            sys = code >= 0 ? (int64_t)code : -1 - (int64_t)code;   // negative: failed an earlier check
            bad = code < 0;
        }
        const int64_t o0 = a.obs_off[sys], o1 = a.obs_off[sys + 1];
        const int64_t p0 = a.pl_off[sys], p1 = a.pl_off[sys + 1];
        const int64_t npl64 = p1 - p0;
        if (bad || !(o0 >= 0 && o0 <= o1 && o1 <= a.n_obs_total && p0 >= 0 && npl64 >= 1 && npl64 <= kMaxPl &&
                     p1 <= a.n_pl_total)) {
            if (lane == 0) a.out[sys] = nan;
            continue;
        }
        const int npl = (int)npl64;
        wave_sync_lds();
        bool pok = true;
        if (lane < npl) {
            const int64_t p = p0 + lane;
            Rec64 r;
            pok = Pol64::setup(unused, a.P[p], a.K[p], a.e[p], a.w[p], a.M0[p], r);
            recs[lane] = r;
        }
        const double gam = a.offset ? a.offset[sys] : 0.0;
        const double jit = has_jit ? a.jitter[sys] : 0.0;
        bad = !isfinite(a.t0) || (a.offset && !isfinite(gam)) || (has_jit && !(isfinite(jit) && jit >= 0.0));
        bad = bad || __any(!pok);
        wave_sync_lds();

        const int64_t n = o1 - o0;
        Pol64::ChiAcc chi;
        Pol64::chi_init(chi);
        bool bad_obs = false;
        // groups of four 64-lane chunks; the last takes only the chunks it needs
        for (int64_t g0 = 0; g0 < n; g0 += 256) {
            const int64_t left = n - g0;
            if (left > 192) ragged64_group<4>(a, recs, npl, o0, n, g0, gam, jit, has_jit, fixed, chi, bad_obs);
            else if (left > 128) ragged64_group<3>(a, recs, npl, o0, n, g0, gam, jit, has_jit, fixed, chi, bad_obs);
            else if (left > 64) ragged64_group<2>(a, recs, npl, o0, n, g0, gam, jit, has_jit, fixed, chi, bad_obs);
            else ragged64_group<1>(a, recs, npl, o0, n, g0, gam, jit, has_jit, fixed, chi, bad_obs);
        }
        const double tot = wave_sum(Pol64::chi_value(chi));
        bad = bad || __any(bad_obs);
        if (lane == 0) a.out[sys] = bad ? nan : tot;
    }
}

}  // namespace

int ragged64_grid(LaunchShape shape, int64_t n_sys)
{
    const int block = shape.block > 0 ? shape.block : 256;
    const int wpb = block / 64;
    int per_cu = shape.blocks_per_cu;
    if (per_cu <= 0) per_cu = cached_occupancy((const void *)k_ragged64, block, (size_t)wpb * kMaxPl * sizeof(Rec64));
    int64_t grid = (n_sys + wpb - 1) / wpb;
    const int64_t cap = (int64_t)device_cu_count() * (per_cu > 0 ? per_cu : 1);
    if (grid > cap) grid = cap;
    return grid < 1 ? 1 : (int)grid;
}

hipError_t launch_ragged64(RaggedArgs a, LaunchShape shape, hipStream_t st)
{
    if (a.n_sys <= 0) return hipSuccess;
    const int block = shape.block > 0 ? shape.block : 256;
    if (block % 64 != 0 || block > 256) return hipErrorInvalidValue;
    const size_t lds = (size_t)(block / 64) * kMaxPl * sizeof(Rec64);
    hipLaunchKernelGGL(k_ragged64, dim3((unsigned)ragged64_grid(shape, a.n_sys)), dim3(block), lds, st, a);
    return hipGetLastError();
}

}  // namespace kep
