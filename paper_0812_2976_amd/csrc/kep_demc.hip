// Population MCMC by differential evolution (DE-MC, ter Braak 2006): the
// many-chain sampler that the batched chi-square is built for (Sec. 6 of the
// paper).  One generation is two fused half-step launches (propose, chi-square
// and accept for every chain of one half, k_demc_half) and, when the
// generation number lives in device memory for graph replay, a one-thread
// kernel that advances it.  This file holds the population chi-square and the
// generation counter; the half-step kernel sits with the dense kernels whose
// chi-square code it shares.
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
    for (int h = 0; h < 2; ++h) {
        hipError_t err = launch_demc_half(a, base, prec, h, shape, st);
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
