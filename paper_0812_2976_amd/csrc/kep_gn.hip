// Gauss-Newton products of the chi-square on the matrix cores: for each
// system, with J the Jacobian of the model velocities (one row per
// observation, one column per parameter P, K, e, omega, M0 of each planet and
// the offset) and W = diag(1/(sigma^2 + s^2)),
//   J^T W J (packed upper triangle),  J^T W r,  chi2 = r^T W r.
// These feed Levenberg-Marquardt and Newton-type optimisers (the paper asks
// for derivatives for optimisers, Sec. 6).  J^T W J is a dense contraction
// over the observations, so it runs on MFMA: each lane (one observation)
// forms its row of the augmented matrix sqrt(w) [J | 1 | r] from the
// implicit-function derivative terms of the adjoint (kep_grad.h) and stores it
// in the wavefront's slice of LDS; the wavefront then accumulates the
// upper-triangular 16 x 16 blocks of its Gram matrix, four observations per
// product.  The augmented column gives J^T W r and chi2 from the same products.
//
// binary64 path (k_gn64): rows in binary64, v_mfma_f64_16x16x4_f64.
// Mixed path (k_gn32): rows in binary32 (the derivative terms are binary32
// already), v_mfma_f32_16x16x4_f32 over each group of 64 observations, and
// each group's sums added into binary64 accumulators, so one rounding error
// spans at most 64 terms.  The binary32 tile halves the LDS per wavefront
// (more resident wavefronts) and the binary32 products issue at twice the
// binary64 rate.
#include <hip/hip_runtime.h>

#include "kep_device.h"
#include "kep_grad.h"
#include "kep_internal.h"
#include "kep_policy.h"

namespace kep {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Stores block (bi, bj) of the Gram matrix of sqrt(w) [J | 1 | r]: the packed
// upper triangle of J^T W J, J^T W r from the last column, chi2 from the
// corner.  (i, j) is this lane's entry q of the block.
__device__ __forceinline__ void gn_store(const DenseArgs &a, double *jtwr, double *jtwj, int64_t sys, int np, int i,
                                         int j, double val)
{
    if (i <= j && j < np) jtwj[(int64_t)(i * np - i * (i - 1) / 2 + (j - i)) * a.n_sys + sys] = val;
    else if (j == np && i < np) jtwr[(int64_t)i * a.n_sys + sys] = val;
    else if (i == np && j == np) a.out[sys] = val;
}

// ------------------------------------------------------------------ binary64
template <int NB>
__host__ __device__ constexpr int gn64_stride() { return 16 * NB + 1; }   // odd row length: staggers LDS banks

template <int NB>
__host__ __device__ inline size_t gn64_lds_per_wave()
{
    const size_t b = (size_t)64 * gn64_stride<NB>() * sizeof(double) + (size_t)kMaxPl * sizeof(GradPlanet<double>);
    return (b + 15) & ~(size_t)15;
}

template <int NB>
__global__ void __launch_bounds__(256) k_gn64(DenseArgs a, double *jtwr, double *jtwj)
{
    constexpr int NCOL = 16 * NB;
    constexpr int STRIDE = gn64_stride<NB>();
    constexpr int NPAIR = NB * (NB + 1) / 2;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = __lane_id();
    const int wpb = blockDim.x >> 6;
    const int wib = uniform_int(threadIdx.x >> 6);
    unsigned char *mine = smem + (size_t)wib * gn64_lds_per_wave<NB>();
    double *T = reinterpret_cast<double *>(mine);
    GradPlanet<double> *pl = reinterpret_cast<GradPlanet<double> *>(mine + (size_t)64 * STRIDE * sizeof(double));

    const int npl = a.n_pl;
    const int np = 5 * npl + 1;
    const int fixed = fixed64(a.fixed_iter);
    const bool has_jit = a.jitter != nullptr;
    const int n_chunks = (int)((a.n_obs + 63) / 64);
    const int64_t n_waves = (int64_t)gridDim.x * wpb;
    const double nan = __builtin_nan("");
    double *row = T + lane * STRIDE;
    // padding columns np + 1 .. NCOL - 1 stay zero for the whole launch
    for (int c = np + 1; c < NCOL; ++c) row[c] = 0.0;

    for (int64_t sys = (int64_t)blockIdx.x * wpb + wib; sys < a.n_sys; sys += n_waves) {
        wave_sync_lds();
        bool pok = true;
        if (lane < npl) {
            const int64_t p = (int64_t)lane * a.n_sys + sys;
            GradPlanet<double> q;
            pok = grad_setup(a.P[p], a.K[p], a.e[p], a.w[p], a.M0[p], a.fixed_iter, q);
            pl[lane] = q;
        }
        const double gam = a.offset ? a.offset[sys] : 0.0;
        const double jit = has_jit ? a.jitter[sys] : 0.0;
        bool ok = isfinite(a.t0) && !__any(!pok);
        if (a.offset) ok = ok && isfinite(gam);
        if (has_jit) ok = ok && isfinite(jit) && jit >= 0.0;
        wave_sync_lds();

        d4 acc[NPAIR];
#pragma unroll
        for (int p = 0; p < NPAIR; ++p) acc[p] = d4{0.0, 0.0, 0.0, 0.0};
        bool bad_obs = false;
        for (int ch = 0; ch < n_chunks; ++ch) {
            const int64_t k = (int64_t)ch * 64 + lane;
            if (k < a.n_obs) {
                const double t = a.t[k], vo = a.v[k], sg = a.sigma[k];
                const double var = sg * sg + jit * jit;
                bool ook = isfinite(t) && isfinite(vo) && isfinite(sg) && sg >= 0.0 && var > 0.0;
                const double sw = ook ? sqrt(1.0 / var) : 0.0;   // sqrt(w) = 1 / sqrt(sigma^2 + s^2)
                const double tt = t - a.t0;
                double model = 0.0;
                for (int j = 0; j < npl; ++j) {
                    double d[5];
                    model += grad_eval(pl[j], tt, a.max_iter, fixed, d);
#pragma unroll
                    for (int i = 0; i < 5; ++i) row[5 * j + i] = sw * d[i];
                }
                const double r = (model + gam) - vo;
                row[np - 1] = sw;
                row[np] = sw * r;
                bad_obs = bad_obs || !ook;
            } else {
                for (int c = 0; c <= np; ++c) row[c] = 0.0;    // rows past the last observation
            }
            wave_sync_lds();
            // Gram matrix of the 64 rows: A operand lane l = row (4s + l/16),
            // column (16 bi + l%16); the B operand reads the same pattern for bj.
            const double *src = T + (lane >> 4) * STRIDE + (lane & 15);
#pragma unroll 4
            for (int s = 0; s < 16; ++s) {
                double av[NB];
#pragma unroll
                for (int b = 0; b < NB; ++b) av[b] = src[4 * s * STRIDE + 16 * b];
                int p = 0;
#pragma unroll
                for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
                    for (int bj = bi; bj < NB; ++bj) {
                        acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi], av[bj], acc[p], 0, 0, 0);
                        ++p;
                    }
                }
            }
            wave_sync_lds();
        }
        ok = ok && !__any(bad_obs);

        // lane l holds entry (16 bi + l/16 + 4 q, 16 bj + l%16) of block (bi, bj) in acc[.][q]
        // (the binary64 16x16x4 product interleaves its output rows by four)
        int p = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
            for (int bj = bi; bj < NB; ++bj) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    gn_store(a, jtwr, jtwj, sys, np, 16 * bi + (lane >> 4) + 4 * q, 16 * bj + (lane & 15),
                             ok ? acc[p][q] : nan);
                ++p;
            }
        }
    }
}

// ------------------------------------------------------------------ mixed

// The tile is column-major, T[c * kGn32Col + obs]: a lane writes its row with
// unit stride across the wavefront, and the matrix operands are read as runs
// of four consecutive observations (128-bit loads).  Observation 16 g + s of
// the group feeds step s of lane group g = l/16: the Gram matrix sums over all
// observations, so any fixed assignment of observations to (step, k) slots,
// the same for both operands, gives the same products.
constexpr int kGn32Col = 68;   // 64 observations + 4: consecutive columns start 4 banks apart

template <int NB>
__host__ __device__ inline size_t gn32_lds_per_wave()
{
    const size_t b = (size_t)16 * NB * kGn32Col * sizeof(float) + (size_t)kMaxPl * sizeof(RecGrad);
    return (b + 15) & ~(size_t)15;
}

template <int NB>
__global__ void __launch_bounds__(256) k_gn32(DenseArgs a, double *jtwr, double *jtwj)
{
    constexpr int NCOL = 16 * NB;
    constexpr int NPAIR = NB * (NB + 1) / 2;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = __lane_id();
    const int wpb = blockDim.x >> 6;
    const int wib = uniform_int(threadIdx.x >> 6);
    unsigned char *mine = smem + (size_t)wib * gn32_lds_per_wave<NB>();
    float *T = reinterpret_cast<float *>(mine);
    RecGrad *pl = reinterpret_cast<RecGrad *>(mine + (size_t)NCOL * kGn32Col * sizeof(float));

    const int npl = a.n_pl;
    const int np = 5 * npl + 1;
    const bool has_jit = a.jitter != nullptr;
    const int n_chunks = (int)((a.n_obs + 63) / 64);
    const int64_t n_waves = (int64_t)gridDim.x * wpb;
    const double nan = __builtin_nan("");
    float *col = T + lane;                       // this lane's observation in column 0
    // padding columns np + 1 .. NCOL - 1 stay zero for the whole launch
    for (int c = np + 1; c < NCOL; ++c) col[c * kGn32Col] = 0.0f;

    for (int64_t sys = (int64_t)blockIdx.x * wpb + wib; sys < a.n_sys; sys += n_waves) {
        wave_sync_lds();
        bool pok = true;
        if (lane < npl) {
            const int64_t p = (int64_t)lane * a.n_sys + sys;
            RecGrad q;
            pok = grad_setup_rec(a.fixed_iter, a.P[p], a.K[p], a.e[p], a.w[p], a.M0[p], q);
            pl[lane] = q;
        }
        const double gam = a.offset ? a.offset[sys] : 0.0;
        const double jit = has_jit ? a.jitter[sys] : 0.0;
        bool ok = isfinite(a.t0) && !__any(!pok);
        if (a.offset) ok = ok && isfinite(gam);
        if (has_jit) ok = ok && isfinite(jit) && jit >= 0.0;
        wave_sync_lds();

        d4 acc[NPAIR];
#pragma unroll
        for (int p = 0; p < NPAIR; ++p) acc[p] = d4{0.0, 0.0, 0.0, 0.0};
        bool bad_obs = false;
        for (int ch = 0; ch < n_chunks; ++ch) {
            const int64_t k = (int64_t)ch * 64 + lane;
            if (k < a.n_obs) {
                const double t = a.t[k], vo = a.v[k], sg = a.sigma[k];
                const double var = sg * sg + jit * jit;
                bool ook = isfinite(t) && isfinite(vo) && isfinite(sg) && sg >= 0.0 && var > 0.0;
                const float sw = ook ? __builtin_amdgcn_rsqf((float)var) : 0.0f;   // sqrt(w)
                const double tt = t - a.t0;
                // per planet: the binary32 Kepler solve from the starting-value
                // table (read through the cache) or the schedule, the binary64
                // correction of E and binary64 velocity, the derivative terms of the
                // corrected root (as the mixed adjoint: kep_grad.h)
                double model = 0.0;
                for (int j = 0; j < npl; ++j) {
                    const RecGrad &q = pl[j];
                    const double M64 = mean_anomaly64_exact(tt, q.ph);
                    float M[1] = {(float)M64}, E[1], sv[1], omc[1];
                    PolMixed::solve<1, false>(q.k, uniform_int(q.niter), uniform_int(q.check) != 0, q.tp, M, E, sv,
                                              omc, a.max_iter, kep_start_tab);
                    float sE, cme, x[5];
                    model += refine_velocity(q, E[0], M64, sE, cme);
                    grad_terms_ce(q, sE, cme, (float)(tt * q.ph.rP), x);
                    const float fK = (float)q.fK;
                    float *c = col + 5 * j * kGn32Col;
                    c[0 * kGn32Col] = sw * ((float)q.fP * x[0]);
                    c[1 * kGn32Col] = sw * x[1];
                    c[2 * kGn32Col] = sw * (fK * x[2]);
                    c[3 * kGn32Col] = -sw * (fK * x[3]);
                    c[4 * kGn32Col] = -sw * (fK * x[4]);
                }
                const double r = (model + gam) - vo;   // residual in binary64
                col[(np - 1) * kGn32Col] = sw;
                col[np * kGn32Col] = sw * (float)r;
                bad_obs = bad_obs || !ook;
            } else {
                for (int c = 0; c <= np; ++c) col[c * kGn32Col] = 0.0f;   // rows past the last observation
            }
            wave_sync_lds();
            // A operand of step s, lane l: column 16 bi + l%16, observation 16 (l/16) + s;
            // the B operand reads the same pattern for bj.
            const float *src = T + (lane & 15) * kGn32Col + 16 * (lane >> 4);
            f4 accf[NPAIR];
#pragma unroll
            for (int p = 0; p < NPAIR; ++p) accf[p] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                f4 av[NB];
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    av[b] = *reinterpret_cast<const f4 *>(src + 16 * b * kGn32Col + 4 * s4);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    int p = 0;
#pragma unroll
                    for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
                        for (int bj = bi; bj < NB; ++bj) {
                            accf[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[bi][u], av[bj][u], accf[p], 0, 0, 0);
                            ++p;
                        }
                    }
                }
            }
#pragma unroll
            for (int p = 0; p < NPAIR; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[p][q] += (double)accf[p][q];
            wave_sync_lds();
        }
        ok = ok && !__any(bad_obs);

        // lane l holds entry (16 bi + 4 (l/16) + q, 16 bj + l%16) of block (bi, bj) in acc[.][q]
        // (the binary32 16x16x4 product keeps four consecutive output rows per lane)
        int p = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
            for (int bj = bi; bj < NB; ++bj) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    gn_store(a, jtwr, jtwj, sys, np, 16 * bi + 4 * (lane >> 4) + q, 16 * bj + (lane & 15),
                             ok ? acc[p][q] : nan);
                ++p;
            }
        }
    }
}

template <class KernelFn>
hipError_t launch_gn_k(KernelFn kern, size_t per_wave, DenseArgs a, double *jtwr, double *jtwj, LaunchShape shape,
                       hipStream_t st)
{
    int wpb = shape.block > 0 ? shape.block / 64 : (int)((64 * 1024) / per_wave);
    wpb = wpb < 1 ? 1 : (wpb > 4 ? 4 : wpb);
    if ((size_t)wpb * per_wave > 64 * 1024) return hipErrorInvalidValue;
    const size_t lds = (size_t)wpb * per_wave;
    int per_cu = shape.blocks_per_cu;
    if (per_cu <= 0) {
        per_cu = cached_occupancy((const void *)kern, wpb * 64, lds);
    }
    int64_t grid = (a.n_sys + wpb - 1) / wpb;
    const int64_t cap = (int64_t)device_cu_count() * per_cu;
    if (grid > cap) grid = cap;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(wpb * 64), lds, st, a, jtwr, jtwj);
    return hipGetLastError();
}

template <int NB>
hipError_t launch_gn_t(bool mixed, DenseArgs a, double *jtwr, double *jtwj, LaunchShape shape, hipStream_t st)
{
    return mixed ? launch_gn_k(k_gn32<NB>, gn32_lds_per_wave<NB>(), a, jtwr, jtwj, shape, st)
                 : launch_gn_k(k_gn64<NB>, gn64_lds_per_wave<NB>(), a, jtwr, jtwj, shape, st);
}

}  // namespace

hipError_t launch_gn(DenseArgs a, double *jtwr, double *jtwj, Prec prec, LaunchShape shape, hipStream_t st)
{
    if (a.n_sys <= 0) return hipSuccess;
    const bool mixed = prec == Prec::Mixed;
    const int ncol = 5 * a.n_pl + 2;   // parameters, offset, residual
    if (ncol <= 16) return launch_gn_t<1>(mixed, a, jtwr, jtwj, shape, st);
    if (ncol <= 32) return launch_gn_t<2>(mixed, a, jtwr, jtwj, shape, st);
    if (ncol <= 48) return launch_gn_t<3>(mixed, a, jtwr, jtwj, shape, st);
    return hipErrorInvalidValue;
}

}  // namespace kep
