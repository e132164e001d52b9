// Population MCMC by differential evolution (DE-MC, ter Braak 2006): the
// many-chain sampler that the batched chi-square is built for (Sec. 6 of the
// paper).  One generation is two fused half-step launches (propose, chi-square
// and accept for every chain of one half, k_demc_half) and, when the
// generation number lives in device memory for graph replay, a one-thread
// kernel that advances it.  The half-step kernel reuses the dense kernels'
// per-precision policies (kep_policy.h) for the chi-square.
//
// r1 != r2 index chains of the other half, which does not move while this
// half is updated.  Random numbers come from Philox-4x32-10 (Salmon et al.,
// SC'11) keyed by the seed, with counter (chain, draw, generation lo,
// generation hi | half << 31), so a proposal depends only on (seed, half,
// chain, generation) and the same generation can be replayed from a graph.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kep_internal.h"
#include "kep_philox.h"
#include "kep_policy.h"

namespace kep {

namespace {

// chi-square of a population from the dense kernel, NaN outside K >= 0
__global__ void __launch_bounds__(256) k_demc_support(const double *x, double *chi2, int64_t nh, int n_pl, int d)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * nh) return;
    const int64_t h = i / nh, k = i - h * nh;
    bool ok = true;
    for (int j = 0; j < n_pl; ++j) ok = ok && x[(h * d + n_pl + j) * nh + k] >= 0.0;
    if (!ok) chi2[i] = __builtin_nan("");
}

__global__ void k_demc_set_gen(uint64_t *gen, uint64_t value)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) gen[0] = value;
}

__global__ void k_demc_advance(uint64_t *gen, uint64_t inc)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) gen[0] = gen[0] + inc;
}

DenseArgs half_dense(const DemcArgs &a, const DenseArgs &base, const double *planes, const double *jitter,
                     double *out)
{
    DenseArgs b = base;
    const int64_t nh = a.nh;
    b.P = planes;
    b.K = planes + (int64_t)a.n_pl * nh;
    b.e = planes + (int64_t)2 * a.n_pl * nh;
    b.w = planes + (int64_t)3 * a.n_pl * nh;
    b.M0 = planes + (int64_t)4 * a.n_pl * nh;
    b.offset = planes + (int64_t)5 * a.n_pl * nh;
    b.jitter = jitter;
    b.n_sys = nh;
    b.n_pl = a.n_pl;
    b.out = out;
    b.grad = nullptr;
    b.dv = nullptr;
    return b;
}

}  // namespace

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
//   observations, exactly as the dense chi-square kernel does (in mixed
//   precision from the block's LDS copy of the Kepler starting-value table), and
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
    // mixed: the block's copy of the Kepler starting-value table after the wave slices
    const uint32_t *tab = nullptr;
    if constexpr (Pol::kMixed) {
        uint32_t *t = reinterpret_cast<uint32_t *>(smem + (size_t)wpb * demc_lds_per_wave(sb, npl, d, sizeof(Rec)));
        load_start_table(t);
        tab = t;
    }

    const int64_t nh = m.nh;
    const uint64_t g = m.gen_ptr ? *m.gen_ptr + m.gen : m.gen;
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
                for (int j = 0; j < npl; ++j) pol_add_planet<Pol, NCH>(recs[s * npl + j], o, mm, a, tab);
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
    const size_t table = Pol::kMixed ? sizeof(kep_start_tab) : 0;
    int sb_cap = kMaxSB;
    while (sb_cap > 1 && (size_t)wpb * demc_lds_per_wave(sb_cap, a.n_pl, m.d, rec) + table > 48 * 1024) sb_cap /= 2;
    const int nch_needed = (int)((a.n_obs + 63) / 64);
    void (*kern)(DenseArgs, DemcArgs, int);
    if (nch_needed <= 1) kern = k_demc_half<Pol, 1>;
    else if (nch_needed <= 2) kern = k_demc_half<Pol, 2>;
    else if (nch_needed <= 4) kern = k_demc_half<Pol, 4>;
    else kern = k_demc_half<Pol, 8>;
    int per_cu = shape.blocks_per_cu;
    if (per_cu <= 0) {
        const size_t lds = (size_t)wpb * demc_lds_per_wave(sb_cap, a.n_pl, m.d, rec) + table;
        per_cu = cached_occupancy((const void *)kern, block, lds);
    }
    const int64_t max_waves = (int64_t)device_cu_count() * per_cu * wpb;
    // ceil: every wave gets at most one batch when the cap allows it, so no wave
    // runs a second batch while the others idle
    const int64_t mw = max_waves > 0 ? max_waves : 1;
    int64_t sb = (m.nh + mw - 1) / mw;
    sb = sb < 1 ? 1 : (sb > sb_cap ? sb_cap : sb);
    a.sb = (int)sb;
    const size_t lds = (size_t)wpb * demc_lds_per_wave(a.sb, a.n_pl, m.d, rec) + table;
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

hipError_t launch_demc_chisq(DemcArgs a, DenseArgs base, Prec prec, LaunchShape shape, hipStream_t st)
{
    if (a.nh <= 0) return hipSuccess;
    for (int h = 0; h < 2; ++h) {
        const double *jit = a.jitter ? a.jitter + (int64_t)h * a.nh : nullptr;
        DenseArgs b = half_dense(a, base, a.x + (int64_t)h * a.d * a.nh, jit, a.chi2 + (int64_t)h * a.nh);
        hipError_t err = launch_dense(b, prec, false, shape, st);
        if (err != hipSuccess) return err;
    }
    const int64_t n = 2 * a.nh;
    hipLaunchKernelGGL(k_demc_support, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a.x, a.chi2, a.nh,
                       a.n_pl, a.d);
    return hipGetLastError();
}

hipError_t launch_demc_generation(DemcArgs a, DenseArgs base, Prec prec, LaunchShape shape, hipStream_t st)
{
    for (int h = 0; h < 2; ++h) {
        hipError_t err = launch_demc_half(a, base, prec, h, shape, st);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t launch_demc_advance(uint64_t *gen, uint64_t inc, hipStream_t st)
{
    hipLaunchKernelGGL(k_demc_advance, dim3(1), dim3(64), 0, st, gen, inc);
    return hipGetLastError();
}

hipError_t launch_demc_set_gen(uint64_t *gen, uint64_t value, hipStream_t st)
{
    hipLaunchKernelGGL(k_demc_set_gen, dim3(1), dim3(64), 0, st, gen, value);
    return hipGetLastError();
}

}  // namespace kep
