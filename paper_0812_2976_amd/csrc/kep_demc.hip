// Population MCMC by differential evolution (DE-MC, ter Braak 2006): the
// many-chain sampler that the batched chi-square is built for (Sec. 6 of the
// paper).  One generation updates the two halves of the population in turn:
//
//   propose (one thread per chain)   y_i = x_i + gam (x_r1 - x_r2) + eps z
//   chi-square of every proposal     the dense kernels, proposals as planes
//   accept  (one thread per chain)   2 ln u < chi2(x_i) - chi2(y_i)
//
// r1 != r2 index chains of the other half, which does not move while this
// half is updated.  Random numbers come from Philox-4x32-10 (Salmon et al.,
// SC'11) keyed by the seed, with counter (chain, draw, generation lo,
// generation hi | half << 31), so a proposal depends only on (seed, half,
// chain, generation) and the same generation can be replayed from a graph.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kep_internal.h"

namespace kep {

namespace {

constexpr double kTwoPiD = 6.283185307179586476925286766559;

struct U4 {
    uint32_t w0, w1, w2, w3;
};

// Philox-4x32-10: ten rounds of two 32x32->64-bit products with the counter
// words permuted and xored with the key; the key advances by the Weyl
// increments between rounds.
__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo_a = 0xD2511F53u * c0, hi_a = __umulhi(0xD2511F53u, c0);
        const uint32_t lo_b = 0xCD9E8D57u * c2, hi_b = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi_b ^ c1 ^ k0, n2 = hi_a ^ c3 ^ k1;
        c0 = n0;
        c1 = lo_b;
        c2 = n2;
        c3 = lo_a;
    }
    return U4{c0, c1, c2, c3};
}

// (0, 1]: 53 random bits n from the top of two words, (n + 1) 2^-53.
__device__ __forceinline__ double unit53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 1.0) * 0x1p-53;
}

__device__ __forceinline__ uint32_t below(uint32_t w, uint32_t m)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)m) >> 32);
}

__device__ __forceinline__ U4 draw(const DemcArgs &a, int h, uint32_t i, uint32_t j, uint64_t g)
{
    return philox(i, j, (uint32_t)g, (uint32_t)(g >> 32) | ((uint32_t)h << 31), a.key0, a.key1);
}

__device__ __forceinline__ uint64_t generation(const DemcArgs &a)
{
    return a.gen_ptr ? *a.gen_ptr : a.gen;
}

__global__ void __launch_bounds__(256) k_demc_propose(DemcArgs a, int h)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.nh) return;
    const uint64_t g = generation(a);
    const int64_t nh = a.nh;
    const double *xh = a.x + (int64_t)h * a.d * nh;
    const double *xo = a.x + (int64_t)(1 - h) * a.d * nh;
    double gam = a.gamma;
    if (a.jump_every > 0 && (g + 1) % (uint64_t)a.jump_every == 0) gam = 1.0;
    const U4 w = draw(a, h, (uint32_t)i, 0u, g);
    const uint32_t r1 = below(w.w0, (uint32_t)nh);
    uint32_t r2 = below(w.w1, (uint32_t)nh - 1u);
    if (r2 >= r1) r2 += 1u;
    for (int r = 0; r < a.d; r += 2) {
        const U4 q = draw(a, h, (uint32_t)i, (uint32_t)(1 + r / 2), g);
        const double u1 = unit53(q.w0, q.w1), u2 = unit53(q.w2, q.w3);
        const double rho = sqrt(-2.0 * log(u1));
        double s, c;
        sincos(kTwoPiD * u2, &s, &c);
        {
            // the proposal is rounded term by term, as written (no contraction)
#pragma clang fp contract(off)
            const double y0 = xh[(int64_t)r * nh + i] + gam * (xo[(int64_t)r * nh + r1] - xo[(int64_t)r * nh + r2]) +
                              a.eps[r] * (rho * c);
            a.y[(int64_t)r * nh + i] = y0;
            if (r + 1 < a.d) {
                const int64_t o = (int64_t)(r + 1) * nh;
                a.y[o + i] = xh[o + i] + gam * (xo[o + r1] - xo[o + r2]) + a.eps[r + 1] * (rho * s);
            }
        }
    }
}

__global__ void __launch_bounds__(256) k_demc_accept(DemcArgs a, int h)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.nh) return;
    const uint64_t g = generation(a);
    const int64_t nh = a.nh;
    const U4 w = draw(a, h, (uint32_t)i, 0u, g);
    const double u = unit53(w.w2, w.w3);
    bool support = true;
    for (int j = 0; j < a.n_pl; ++j) support = support && a.y[(int64_t)(a.n_pl + j) * nh + i] >= 0.0;
    const double c_new = a.c_new[i];
    double *chi = a.chi2 + (int64_t)h * nh + i;
    if (support && 2.0 * log(u) < *chi - c_new) {
        double *xh = a.x + (int64_t)h * a.d * nh;
        for (int r = 0; r < a.d; ++r) xh[(int64_t)r * nh + i] = a.y[(int64_t)r * nh + i];
        *chi = c_new;
        if (a.n_accept) a.n_accept[(int64_t)h * nh + i] += 1;
    }
}

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

__global__ void k_demc_advance(uint64_t *gen)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) gen[0] = gen[0] + 1;
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
    const unsigned grid = (unsigned)((a.nh + 255) / 256);
    for (int h = 0; h < 2; ++h) {
        hipLaunchKernelGGL(k_demc_propose, dim3(grid), dim3(256), 0, st, a, h);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
        const double *jit = a.jitter ? a.jitter + (int64_t)h * a.nh : nullptr;
        err = launch_dense(half_dense(a, base, a.y, jit, a.c_new), prec, false, shape, st);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k_demc_accept, dim3(grid), dim3(256), 0, st, a, h);
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    if (a.gen_ptr) {
        hipLaunchKernelGGL(k_demc_advance, dim3(1), dim3(64), 0, st, const_cast<uint64_t *>(a.gen_ptr));
        return hipGetLastError();
    }
    return hipSuccess;
}

hipError_t launch_demc_set_gen(uint64_t *gen, uint64_t value, hipStream_t st)
{
    hipLaunchKernelGGL(k_demc_set_gen, dim3(1), dim3(64), 0, st, gen, value);
    return hipGetLastError();
}

}  // namespace kep
