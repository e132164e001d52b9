// Mixed-precision chi-square gradient (the implicit-function adjoint; the
// paper asks for parallel partial derivatives for optimisers, Sec. 6) and the
// Gaussian likelihood with jitter, with the lanes over observations.
//
// One wavefront per system at a time, lane l holding observations l, l + 64,
// ... (NCH chunks in registers, streamed in groups beyond 64 NCH), like the
// dense chi-square kernel: every planet constant is wave-uniform (records in
// the wavefront's LDS slice, built with the lanes over the systems of a
// batch), the eccentricity schedule is uniform.  Three wavefronts per SIMD
// (up to 168 VGPRs): at four the compiler spilled up to 220 bytes per lane,
// and the spill slots' write-backs tripled the kernel's HBM writes for the
// same time; at three at most 56 bytes remain (four planets, four chunks).
// Per group of observations:
//   pass 1, per planet: binary64 phase, binary32 Kepler solve (table start or
//     schedule), binary64 correction of E and binary64 velocity (kep_grad.h);
//     sin E and cos E - e kept in binary32;
//   residual r = sum_j v_j + gamma - v_obs in binary64, c = 2 w r;
//   pass 2, per planet: the five derivative terms, c x accumulated per lane;
//   the 5 n_pl + 1 per-lane sums reduced across the wavefront at once
//   (rows_reduce_scatter), each row's total kept in binary64 by one lane.
// The planets' constant factors (K, 2 pi K/P, e cos w, ...) are applied when
// the rows are written.
#include <hip/hip_runtime.h>

#include "kep_device.h"
#include "kep_grad.h"
#include "kep_internal.h"
#include "kep_policy.h"

namespace kep {

namespace {

constexpr int pow2_at_least(int n) { return n <= 1 ? 1 : 2 * pow2_at_least((n + 1) / 2); }

__host__ __device__ inline size_t adj_table_offset(int wpb, int sb, int npl)
{
    return ((size_t)wpb * sb * npl * sizeof(RecGrad) + (size_t)wpb * sb * sizeof(int) + 15) & ~(size_t)15;
}

// The sin/cos knots follow the starting-value table.
__host__ __device__ inline size_t adj_knots_offset(int wpb, int sb, int npl)
{
    return adj_table_offset(wpb, sb, npl) + ((sizeof(kep_start_tab) + 15) & ~(size_t)15);
}

template <int NPL, int NCH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_grad_obs(DenseArgs a, int nll)
{
    constexpr int NROW = 5 * NPL + 1;
    constexpr int R = pow2_at_least(NROW);
    constexpr int SPAN = 64 / R;              // lanes holding one row after the reduction
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = __lane_id();
    const int wpb = blockDim.x >> 6;
    const int wib = uniform_int(threadIdx.x >> 6);
    RecGrad *recs = reinterpret_cast<RecGrad *>(smem) + (size_t)wib * a.sb * NPL;
    int *sysbad = reinterpret_cast<int *>(smem + (size_t)wpb * a.sb * NPL * sizeof(RecGrad)) + wib * a.sb;
    uint32_t *tab = reinterpret_cast<uint32_t *>(smem + adj_table_offset(wpb, a.sb, NPL));
    double2 *knots = reinterpret_cast<double2 *>(smem + adj_knots_offset(wpb, a.sb, NPL));
    fill_sincos64_knots(knots);
    load_start_table(tab);          // ends with the block barrier

    const SysShare share = sys_share<false>(a.n_sys, wpb, wib, a.sb);
    const int n_groups = (int)((a.n_obs + 64 * NCH - 1) / (64 * NCH));
    const bool has_jit = a.jitter != nullptr;
    const int row = lane / SPAN;
    const double nan = __builtin_nan("");

    ObsG o[NCH];
    auto load_group = [&](int g) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) load_obs_g(a, (int64_t)g * 64 * NCH + c * 64 + lane, o[c]);
    };
    if (n_groups <= 1) load_group(0);

    for (int64_t run0 = share.lo; run0 < share.hi; run0 += share.step) {
        int64_t first;
        const int nb = share_run(share, run0, a.sb, first);
        wave_sync_lds();
        if (lane < nb) {
            const int64_t sys = first + (int64_t)share.stride * lane;
            bool ok = isfinite(a.t0);
            if (a.offset) ok = ok && isfinite(a.offset[sys]);
            if (has_jit) ok = ok && isfinite(a.jitter[sys]) && a.jitter[sys] >= 0.0;
            sysbad[lane] = ok ? 0 : 1;
        }
        wave_sync_lds();
        // planet records with the lanes over the run's (planet, system) pairs,
        // planet-major (the block's wavefronts together read whole runs of
        // every parameter plane)
#pragma nounroll
        for (int q = lane; q < nb * NPL; q += 64) {
            const int j = q / nb, sq = q - j * nb;
            const int64_t p = (int64_t)j * a.n_sys + first + (int64_t)share.stride * sq;
            RecGrad r;
            if (!grad_setup_rec(a.fixed_iter, a.P[p], a.K[p], a.e[p], a.w[p], a.M0[p], r)) sysbad[sq] = 1;
            recs[sq * NPL + j] = r;
        }
        wave_sync_lds();

        for (int s = 0; s < nb; ++s) {
            const int64_t sys = first + (int64_t)share.stride * s;
            const double gam = a.offset ? a.offset[sys] : 0.0;
            const double jit = has_jit ? a.jitter[sys] : 0.0;
            const float jit2 = (float)(jit * jit);
            const bool sbad = uniform_int(sysbad[s]) != 0;
            const RecGrad *rs = recs + s * NPL;
            double tot = 0.0;                        // this lane's row, summed over the groups
            double chi = 0.0, sum_lv = 0.0, sum_w = 0.0, sum_wr2 = 0.0;
            bool bad_obs = false;
            for (int g = 0; g < n_groups; ++g) {
                if (n_groups > 1) load_group(g);
                // pass 1: corrected velocities; sin E and cos E - e kept for pass 2.
                // The planet loop is not unrolled (one copy of the Kepler solve in
                // the code); its results go to registers by planet index.
                double model[NCH];
                float sE[NPL][NCH], cme[NPL][NCH];
#pragma unroll
                for (int c = 0; c < NCH; ++c) model[c] = gam;
#pragma nounroll
                for (int j = 0; j < NPL; ++j) {
                    const RecGrad &rr = rs[j];
                    const Phase64 ph = rr.ph;
                    const Ecc32 k = rr.k;
                    double M64[NCH];
                    float M[NCH], E[NCH], sv[NCH], omc[NCH], sj[NCH], cj[NCH];
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
                        M64[c] = mean_anomaly64_exact(o[c].tt, ph);
                        M[c] = (float)M64[c];
                    }
                    PolMixed::solve<NCH, false>(k, uniform_int(rr.niter), uniform_int(rr.check) != 0, rr.tp, M, E,
                                                sv, omc, a.max_iter, tab);
#pragma unroll
                    for (int c = 0; c < NCH; ++c) model[c] += refine_velocity(rr, E[c], M64[c], knots, sj[c], cj[c]);
#pragma unroll
                    for (int jj = 0; jj < NPL; ++jj) {
                        if (jj == j) {
#pragma unroll
                            for (int c = 0; c < NCH; ++c) {
                                sE[jj][c] = sj[c];
                                cme[jj][c] = cj[c];
                            }
                        }
                    }
                }
                // residuals and weights
                float cw2[NCH];
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    const double r = model[c] - o[c].v;
                    const float var = o[c].s2 + jit2;
                    const float w = rcp32(var);
                    const float r32 = (float)r;
                    cw2[c] = 0.0f;
                    if (o[c].in) {
                        bad_obs = bad_obs || !o[c].ok || !(var > 0.0f);
                        const float wr = w * r32;
                        chi = fma((double)wr, r, chi);
                        cw2[c] = 2.0f * wr;
                        if (nll) {
                            sum_lv += (double)logf(var);
                            sum_w += (double)w;
                            sum_wr2 = fma((double)wr, (double)wr, sum_wr2);
                        }
                    }
                }
                // pass 2: derivative terms, weighted per lane
                float acc[R];
#pragma unroll
                for (int i = 0; i < R; ++i) acc[i] = 0.0f;
#pragma unroll
                for (int j = 0; j < NPL; ++j) {
                    lds_reload_barrier();
                    const RecGrad &rr = rs[j];
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
                        float x[5];
                        grad_terms_ce(rr, sE[j][c], cme[j][c], (float)(o[c].tt * rr.ph.rP), x);
#pragma unroll
                        for (int i = 0; i < 5; ++i) acc[5 * j + i] = fmaf(cw2[c], x[i], acc[5 * j + i]);
                    }
                }
#pragma unroll
                for (int c = 0; c < NCH; ++c) acc[5 * NPL] += cw2[c];
                tot += (double)rows_reduce_scatter<R>(acc);
            }
            chi = wave_sum(chi);
            if (nll) {
                sum_lv = wave_sum(sum_lv);
                sum_w = wave_sum(sum_w);
                sum_wr2 = wave_sum(sum_wr2);
            }
            const bool bad = sbad || __any(bad_obs);
            if (lane % SPAN == 0 && row < NROW) {
                double gv = tot;                     // the offset row, and K rows: factor 1
                if (row < 5 * NPL) {
                    const int j = row / 5, i = row - 5 * (row / 5);
                    const RecGrad &rr = rs[j];
                    gv = i == 0 ? rr.fP * tot : i == 1 ? tot : i == 2 ? rr.fK * tot : -rr.fK * tot;
                }
                a.grad[(int64_t)row * a.n_sys + sys] = bad ? nan : gv;
            }
            if (lane == 0) {
                a.out[sys] = bad ? nan : chi + sum_lv;
                if (nll) a.grad[(int64_t)NROW * a.n_sys + sys] = bad ? nan : 2.0 * jit * (sum_w - sum_wr2);
            }
        }
    }
}

template <int NPL, int NCH>
hipError_t launch_grad_obs_t(DenseArgs a, bool nll, LaunchShape shape, hipStream_t st)
{
    const int block = shape.block > 0 ? shape.block : 256;
    const int wpb = block / 64;
    const size_t rec_bytes = (size_t)wpb * (NPL * sizeof(RecGrad) + sizeof(int));
    // systems per setup batch: records and tables within 40 KiB per block (four
    // blocks of four wavefronts on a CU's 160 KiB), at most kMaxSB; a multiple
    // of 8 where possible (whole 64-byte runs of every parameter plane)
    int64_t sb_cap =
        ((int64_t)(40 * 1024) - (int64_t)sizeof(kep_start_tab) - (int64_t)kSc64Bytes - 32) / (int64_t)rec_bytes;
    sb_cap = sb_cap < 1 ? 1 : (sb_cap > kMaxSB ? kMaxSB : sb_cap);
    if (sb_cap > 8) sb_cap &= ~(int64_t)7;
    auto lds_of = [&](int64_t sb) { return adj_knots_offset(wpb, (int)sb, NPL) + kSc64Bytes; };
    void (*kern)(DenseArgs, int) = k_grad_obs<NPL, NCH>;
    int per_cu = shape.blocks_per_cu;
    if (per_cu <= 0) per_cu = cached_occupancy((const void *)kern, block, lds_of(sb_cap));
    const int64_t max_waves = (int64_t)device_cu_count() * per_cu * wpb;
    int64_t sb = (a.n_sys + max_waves - 1) / (max_waves > 0 ? max_waves : 1);
    sb = sb < 1 ? 1 : (sb > sb_cap ? sb_cap : sb);
    a.sb = (int)sb;
    // one block per wpb x sb systems, at most the resident count
    int64_t grid = (a.n_sys + (int64_t)wpb * sb - 1) / ((int64_t)wpb * sb);
    const int64_t cap = (int64_t)device_cu_count() * per_cu;
    if (grid > cap) grid = cap;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(block), lds_of(sb), st, a, nll ? 1 : 0);
    return hipGetLastError();
}

// Observation chunks per lane: enough for n_obs in one group where the
// registers allow (four chunks up to four planets, two beyond).
template <int NPL>
hipError_t launch_grad_obs_npl(DenseArgs a, bool nll, LaunchShape shape, hipStream_t st)
{
    const int64_t need = (a.n_obs + 63) / 64;
    if (need <= 1) return launch_grad_obs_t<NPL, 1>(a, nll, shape, st);
    if (NPL > 4 || need <= 2) return launch_grad_obs_t<NPL, 2>(a, nll, shape, st);
    return launch_grad_obs_t<NPL, (NPL <= 4 ? 4 : 2)>(a, nll, shape, st);
}

}  // namespace

hipError_t launch_grad_mixed(DenseArgs a, bool nll, LaunchShape shape, hipStream_t st)
{
    if (a.n_sys <= 0) return hipSuccess;
    switch (a.n_pl) {
        case 1: return launch_grad_obs_npl<1>(a, nll, shape, st);
        case 2: return launch_grad_obs_npl<2>(a, nll, shape, st);
        case 3: return launch_grad_obs_npl<3>(a, nll, shape, st);
        case 4: return launch_grad_obs_npl<4>(a, nll, shape, st);
        case 5: return launch_grad_obs_npl<5>(a, nll, shape, st);
        case 6: return launch_grad_obs_npl<6>(a, nll, shape, st);
        case 7: return launch_grad_obs_npl<7>(a, nll, shape, st);
        case 8: return launch_grad_obs_npl<8>(a, nll, shape, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace kep
