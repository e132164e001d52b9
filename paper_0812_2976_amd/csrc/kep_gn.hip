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
// in the wavefront's slice of LDS; the wavefront then accumulates 16 x 16
// blocks that cover the upper triangle of its Gram matrix, four observations
// per product.  The augmented column gives J^T W r and chi2 from the same
// products.
//
// binary64 path (k_gn64): rows in binary64, v_mfma_f64_16x16x4_f64.
// Mixed path (k_gn_obs): rows in binary32 (the derivative terms are binary32
// already), v_mfma_f32_16x16x4_f32 over each chunk of 64 observations, and
// each chunk's sums added into binary64 accumulators, so one rounding error
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

// Mixed path (k_gn_obs): the observations of a system in NCH chunks of 64
// per lane, like the mixed adjoint (kep_adjoint.hip): pass 1 over the chunks
// (binary64 phase, binary32 Kepler solve from the starting-value table,
// binary64 correction of E and the velocity) gives every chunk's sin E and
// cos E - e per planet and its binary64 residual; then, one chunk at a time,
// each lane writes its row of sqrt(w) [J | 1 | r] (the derivative terms of the
// corrected root) into the wavefront's tile and the tile's Gram matrix is
// accumulated with v_mfma_f32_16x16x4_f32, each chunk's sums added into
// binary64 accumulators.  The tile is column-major, T[c * kGnCol + obs]: a
// lane writes its row with unit stride across the wavefront, and the matrix
// operands are read as runs of four consecutive observations (128-bit loads).
// Observation 16 g + 4 s + u of the chunk feeds step u of lane group g = l/16
// in the s-th run: the Gram matrix sums over all observations, so any fixed
// assignment of observations to (step, k) slots, the same for both operands,
// gives the same products.  Only the 5 n_pl + 2 live columns are stored.  An
// operand lane past the live columns reads some live column instead: output
// row i of a product depends only on row i of its first operand and output
// column j only on column j of its second, so such lanes change nothing but
// entries that are never stored.
//
// Block products per step of four observations: every pair of 16-column
// blocks, except for 17 to 24 columns (three or four planets), where two
// products cover the upper triangle: with the columns in groups
// X = [0, g), Y = [g, g + 8), Z = [g + 8, NC), g = NC - 16, the product of the
// operands X+Y (rows) and X+Z (columns) holds the pairs XX, XY, XZ and YZ, and
// the square of Y+Z holds YY and ZZ (against three products for two blocks;
// NC <= 24 makes each operand at most 16 columns).
constexpr int kGnCol = 68;   // 64 observations + 4: consecutive columns start 4 banks apart

template <int NPL>
__host__ __device__ constexpr int gn_cols() { return 5 * NPL + 2; }

template <int NPL>
__host__ __device__ inline size_t gn_obs_lds_per_wave(int sb)
{
    const size_t b = (size_t)gn_cols<NPL>() * kGnCol * sizeof(float) + (size_t)sb * NPL * sizeof(RecGrad) +
                     (size_t)sb * sizeof(int);
    return (b + 15) & ~(size_t)15;
}

template <int NPL, int NCH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_gn_obs(DenseArgs a, double *jtwr,
                                                                                       double *jtwj)
{
    constexpr int NC = gn_cols<NPL>();       // parameters, offset, residual
    constexpr int NP = NC - 1;               // parameters and offset
    constexpr int NB = (NC + 15) / 16;       // 16-column blocks
    constexpr bool TWO = NC > 16 && NC <= 24;
    constexpr int GX = NC - 16;              // TWO: group X = [0, GX), Y = [GX, GX + 8), Z = [GX + 8, NC)
    constexpr int NOP = TWO ? 3 : NB;        // operand column sets (TWO: X+Y, X+Z, Y+Z)
    constexpr int NPAIR = TWO ? 2 : NB * (NB + 1) / 2;   // products per step
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = __lane_id();
    const int wpb = blockDim.x >> 6;
    const int wib = uniform_int(threadIdx.x >> 6);
    unsigned char *mine = smem + (size_t)wib * gn_obs_lds_per_wave<NPL>(a.sb);
    float *T = reinterpret_cast<float *>(mine);
    RecGrad *recs = reinterpret_cast<RecGrad *>(mine + (size_t)NC * kGnCol * sizeof(float));
    int *sysbad = reinterpret_cast<int *>(recs + (size_t)a.sb * NPL);
    double2 *knots = reinterpret_cast<double2 *>(smem + (size_t)wpb * gn_obs_lds_per_wave<NPL>(a.sb));
    fill_sincos64_knots(knots);
    __syncthreads();

    const SysShare share = sys_share<true>(a.n_sys, wpb, wib, a.sb);
    const int n_groups = (int)((a.n_obs + 64 * NCH - 1) / (64 * NCH));
    const bool has_jit = a.jitter != nullptr;
    const double nan = __builtin_nan("");
    float *col = T + lane;                   // this lane's observation in column 0
    // operand columns of this lane, li = l%16: 16 b + li in block b, or with TWO
    // li (X+Y), li or li + 8 (X+Z) and GX + li (Y+Z); lanes past the live
    // columns read a live one
    const int li = lane & 15;
    const float *src[NOP];
#pragma unroll
    for (int b = 0; b < NOP; ++b) {
        int c;
        if constexpr (TWO) c = b == 0 ? li : b == 1 ? (li < GX ? li : (li + 8 < NC ? li + 8 : li)) : GX + li;
        else c = 16 * b + li < NC ? 16 * b + li : NC - 1;
        src[b] = T + c * kGnCol + 16 * (lane >> 4);
    }

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
        // planet records with the lanes over the run's (planet, system) pairs
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
            d4 acc[NPAIR];
#pragma unroll
            for (int p = 0; p < NPAIR; ++p) acc[p] = d4{0.0, 0.0, 0.0, 0.0};
            bool bad_obs = false;
            for (int g = 0; g < n_groups; ++g) {
                if (n_groups > 1) load_group(g);
                // pass 1 (as the mixed adjoint): corrected velocities; sin E and
                // cos E - e kept per planet and chunk
                double model[NCH];
                float sE[NPL][NCH], cme[NPL][NCH];
#pragma unroll
                for (int c = 0; c < NCH; ++c) model[c] = gam;
#pragma nounroll
                for (int j = 0; j < NPL; ++j) {
                    const RecGrad &rr = rs[j];
                    double M64[NCH];
                    float M[NCH], E[NCH], sv[NCH], omc[NCH], sj[NCH], cj[NCH];
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
                        M64[c] = mean_anomaly64_exact(o[c].tt, rr.ph);
                        M[c] = (float)M64[c];
                    }
                    PolMixed::solve<NCH, false>(rr.k, uniform_int(rr.niter), uniform_int(rr.check) != 0, rr.tp, M, E,
                                                sv, omc, a.max_iter, kep_start_tab);
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
                // pass 2, one chunk at a time: the rows of sqrt(w) [J | 1 | r] into
                // the tile, then the tile's Gram matrix
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    const float var = o[c].s2 + jit2;
                    const bool use = o[c].in && o[c].ok && var > 0.0f;
                    if (o[c].in) bad_obs = bad_obs || !o[c].ok || !(var > 0.0f);
                    const float sw = use ? __builtin_amdgcn_rsqf(var) : 0.0f;   // sqrt(w)
                    const double r = model[c] - o[c].v;                          // residual in binary64
#pragma unroll
                    for (int j = 0; j < NPL; ++j) {
                        lds_reload_barrier();
                        const RecGrad &rr = rs[j];
                        float x[5];
                        grad_terms_ce(rr, sE[j][c], cme[j][c], (float)(o[c].tt * rr.ph.rP), x);
                        const float fK = (float)rr.fK;
                        float *cj = col + 5 * j * kGnCol;
                        cj[0 * kGnCol] = sw * ((float)rr.fP * x[0]);
                        cj[1 * kGnCol] = sw * x[1];
                        cj[2 * kGnCol] = sw * (fK * x[2]);
                        cj[3 * kGnCol] = -sw * (fK * x[3]);
                        cj[4 * kGnCol] = -sw * (fK * x[4]);
                    }
                    col[(NP - 1) * kGnCol] = sw;
                    col[NP * kGnCol] = use ? sw * (float)r : 0.0f;
                    wave_sync_lds();
                    f4 accf[NPAIR];
#pragma unroll
                    for (int p = 0; p < NPAIR; ++p) accf[p] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) {
                        f4 av[NOP];
#pragma unroll
                        for (int b = 0; b < NOP; ++b) av[b] = *reinterpret_cast<const f4 *>(src[b] + 4 * s4);
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            if constexpr (TWO) {
                                accf[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[0][u], av[1][u], accf[0], 0, 0, 0);
                                accf[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[2][u], av[2][u], accf[1], 0, 0, 0);
                            } else {
                                int p = 0;
#pragma unroll
                                for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
                                    for (int bj = bi; bj < NB; ++bj) {
                                        accf[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[bi][u], av[bj][u], accf[p],
                                                                                        0, 0, 0);
                                        ++p;
                                    }
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
            }
            const bool ok = !sbad && !__any(bad_obs);
            // lane l holds entry (4 (l/16) + q, l%16) of each product in acc[.][q]
            // (the binary32 16x16x4 product keeps four consecutive output rows per lane)
            if constexpr (TWO) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = 4 * (lane >> 4) + q;
                    // X+Y by X+Z: XX (upper triangle), YX (as XY), XZ and YZ
                    const int c = li < GX ? li : li + 8;
                    if (i < GX + 8 && li < GX + 8 && !(i < GX && c < GX && i > c))
                        gn_store(a, jtwr, jtwj, sys, NP, i < c ? i : c, i < c ? c : i, ok ? acc[0][q] : nan);
                    // Y+Z squared: YY and ZZ (upper triangles; YZ came from the first)
                    const int p2 = GX + i, c2 = GX + li;
                    if (p2 <= c2 && !(p2 < GX + 8 && c2 >= GX + 8))
                        gn_store(a, jtwr, jtwj, sys, NP, p2, c2, ok ? acc[1][q] : nan);
                }
            } else {
                int p = 0;
#pragma unroll
                for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
                    for (int bj = bi; bj < NB; ++bj) {
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            gn_store(a, jtwr, jtwj, sys, NP, 16 * bi + 4 * (lane >> 4) + q, 16 * bj + li,
                                     ok ? acc[p][q] : nan);
                        ++p;
                    }
                }
            }
        }
    }
}

template <int NPL, int NCH>
hipError_t launch_gn_obs_t(DenseArgs a, double *jtwr, double *jtwj, LaunchShape shape, hipStream_t st)
{
    const int block = shape.block > 0 ? shape.block : 256;
    const int wpb = block / 64;
    // systems per setup batch: tiles and records within 40 KiB per block (four
    // blocks of four wavefronts on a CU's 160 KiB), at most kMaxSB; the
    // block's sin/cos knots come on top
    int sb_cap = kMaxSB;
    while (sb_cap > 1 && (size_t)wpb * gn_obs_lds_per_wave<NPL>(sb_cap) > 40 * 1024) --sb_cap;
    auto lds_of = [&](int sbv) { return (size_t)wpb * gn_obs_lds_per_wave<NPL>(sbv) + kSc64Bytes; };
    void (*kern)(DenseArgs, double *, double *) = k_gn_obs<NPL, NCH>;
    int per_cu = shape.blocks_per_cu;
    if (per_cu <= 0) per_cu = cached_occupancy((const void *)kern, block, lds_of(sb_cap));
    const int64_t max_waves = (int64_t)device_cu_count() * per_cu * wpb;
    int64_t sb = (a.n_sys + max_waves - 1) / (max_waves > 0 ? max_waves : 1);
    sb = sb < 1 ? 1 : (sb > sb_cap ? sb_cap : sb);
    a.sb = (int)sb;
    const size_t lds = lds_of(a.sb);
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    // one block per wpb x sb systems, at most the resident count
    int64_t grid = (a.n_sys + (int64_t)wpb * sb - 1) / ((int64_t)wpb * sb);
    const int64_t cap = (int64_t)device_cu_count() * per_cu;
    if (grid > cap) grid = cap;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(block), lds, st, a, jtwr, jtwj);
    return hipGetLastError();
}

// Observation chunks per lane: one for n_obs <= 64, else two (at c4, 262,144 x 4
// x 256: one chunk 2.74 ms, two 2.50 ms, four 2.65 ms).
template <int NPL>
hipError_t launch_gn_obs_npl(DenseArgs a, double *jtwr, double *jtwj, LaunchShape shape, hipStream_t st)
{
    if (a.n_obs <= 64) return launch_gn_obs_t<NPL, 1>(a, jtwr, jtwj, shape, st);
    return launch_gn_obs_t<NPL, 2>(a, jtwr, jtwj, shape, st);
}

hipError_t launch_gn_mixed(DenseArgs a, double *jtwr, double *jtwj, LaunchShape shape, hipStream_t st)
{
    switch (a.n_pl) {
        case 1: return launch_gn_obs_npl<1>(a, jtwr, jtwj, shape, st);
        case 2: return launch_gn_obs_npl<2>(a, jtwr, jtwj, shape, st);
        case 3: return launch_gn_obs_npl<3>(a, jtwr, jtwj, shape, st);
        case 4: return launch_gn_obs_npl<4>(a, jtwr, jtwj, shape, st);
        case 5: return launch_gn_obs_npl<5>(a, jtwr, jtwj, shape, st);
        case 6: return launch_gn_obs_npl<6>(a, jtwr, jtwj, shape, st);
        case 7: return launch_gn_obs_npl<7>(a, jtwr, jtwj, shape, st);
        case 8: return launch_gn_obs_npl<8>(a, jtwr, jtwj, shape, st);
        default: return hipErrorInvalidValue;
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
hipError_t launch_gn64_t(DenseArgs a, double *jtwr, double *jtwj, LaunchShape shape, hipStream_t st)
{
    return launch_gn_k(k_gn64<NB>, gn64_lds_per_wave<NB>(), a, jtwr, jtwj, shape, st);
}

}  // namespace

hipError_t launch_gn(DenseArgs a, double *jtwr, double *jtwj, Prec prec, LaunchShape shape, hipStream_t st)
{
    if (a.n_sys <= 0) return hipSuccess;
    if (prec == Prec::Mixed) return launch_gn_mixed(a, jtwr, jtwj, shape, st);
    const int ncol = 5 * a.n_pl + 2;   // parameters, offset, residual
    if (ncol <= 16) return launch_gn64_t<1>(a, jtwr, jtwj, shape, st);
    if (ncol <= 32) return launch_gn64_t<2>(a, jtwr, jtwj, shape, st);
    if (ncol <= 48) return launch_gn64_t<3>(a, jtwr, jtwj, shape, st);
    return hipErrorInvalidValue;
}

}  // namespace kep
