// Internal interface between the C ABI (kep_api.cpp) and the kernels
// (kep_kernels.hip).  Not installed; the public interface is include/kepler.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kep {

// Arguments of the dense kernels (observations shared by every system).
struct DenseArgs {
    const double *t, *v, *sigma;
    int64_t n_obs;
    double t0;
    const double *P, *K, *e, *w, *M0;
    const double *offset, *jitter;
    int64_t n_sys;
    int n_pl;
    int sb;            // systems per setup batch of one wavefront (1..kMaxSB)
    double *out;       // chi2 [n_sys] or model [n_sys][n_obs]
    double *grad;      // gradient [(5 n_pl + 1 (+1 for the likelihood))][n_sys] (gradient kernels only)
    float *dv;         // per-planet velocities or eccentric anomalies [n_pl][n_sys][n_obs]
    int fixed_iter;    // > 0: fixed Danby count; <= 0: eccentricity schedule
    int max_iter;      // cap of the convergence-tested loop
};

// Ragged (CSR) batch, one persistent launch.
struct RaggedArgs {
    const double *t, *v, *sigma;
    const int64_t *obs_off;
    double t0;
    const double *P, *K, *e, *w, *M0;
    const int64_t *pl_off;
    const double *offset, *jitter;
    const int32_t *order;     // systems by decreasing work
    int64_t n_sys;
    int64_t n_items;          // number of work items = ceil(n_sys / sb)
    int sb;                   // systems per work item
    int gmax;                 // largest observation group, in 64-lane chunks (2 or 4)
    unsigned int *queue;      // kQueueWords counters (kRaggedQueues work queues, blocks done); zero at
                              // launch, and the kernel leaves them zero
    double *out;
    int fixed_iter, max_iter;
    int64_t n_obs_total, n_pl_total;   // sizes of the CSR arrays (the allocation-free path checks against them)
};

// Work queues of the persistent ragged kernel: one counter per XCD (blocks go
// to the XCDs round-robin), each on its own 128-byte line, queue q handing out
// items q, q + kRaggedQueues, ...; a wave drains its own XCD's queue first,
// then the others.  The blocks-done counter follows the queues.
constexpr int kRaggedQueues = 8;
constexpr int kQueueStride = 32;                              // words between counters
constexpr int kQueueDone = kRaggedQueues * kQueueStride;      // index of the blocks-done counter
constexpr int kQueueWords = kQueueDone + 1;

// Astrometric batch (Thiele-Innes form): epochs t with measured offsets x
// (RA*cos Dec) and y (Dec), uncertainties sx, sy; planes P, e, M0, A, B, F, G
// [n_pl][n_sys]; offsets x0, y0 [n_sys] or null.
struct AstroArgs {
    const double *t, *x, *y, *sx, *sy;
    int64_t n_obs;
    double t0;
    const double *P, *e, *M0, *A, *B, *F, *G;
    const double *x0, *y0;
    int64_t n_sys;
    int n_pl;
    int sb;
    double *out;       // chi2 [n_sys] or positions [n_sys][2][n_obs]
    int fixed_iter, max_iter;
};

// Population sampler (DE-MC): two halves of n_half chains, each half laid out
// [d][nh] with rows P[n_pl], K[n_pl], e[n_pl], omega[n_pl], M0[n_pl], gamma.
struct DemcArgs {
    double *x;                // [2][d][nh]
    double *chi2;             // [2][nh]
    int64_t *n_accept;        // [2][nh] or null
    const double *jitter;     // [2][nh] or null
    double *y;                // proposals [d][nh] (caller's workspace)
    double *c_new;            // chi-square of the proposals [nh] (workspace)
    const double *eps;        // [d]
    int64_t nh;
    int n_pl, d;
    double gamma;             // resolved (> 0)
    int jump_every;
    uint32_t key0, key1;
    const uint64_t *gen_ptr;  // generation counter in device memory (graphs), or null
    uint64_t gen;             // the generation (gen_ptr null) or its offset from *gen_ptr
};

constexpr int kMaxSB = 32;
constexpr int kMaxPl = 8;

// Allocation-free ragged path: a static device array holds the queue counters
// (the first kStaticQueueBytes) and the int32 work order of at most
// kStaticMaxSys systems.
constexpr int64_t kStaticMaxSys = 1 << 21;
constexpr size_t kStaticQueueBytes = 2048;
static_assert(sizeof(unsigned int) * kQueueWords <= kStaticQueueBytes, "queue counters exceed their area");
constexpr size_t kStaticScratchBytes = kStaticQueueBytes + sizeof(int32_t) * (size_t)kStaticMaxSys;

enum class Prec { F64 = 0, Mixed = 1 };

struct LaunchShape {
    int block;         // threads per block (multiple of 64)
    int blocks_per_cu; // 0 = occupancy limit
};

// Launchers return hipSuccess or the launch error.  They do not synchronise.
hipError_t launch_kepler_solve(const double *M, const double *e, double *E, int64_t n, Prec prec,
                               int fixed_iter, int max_iter, LaunchShape shape, hipStream_t st);
hipError_t launch_dense(DenseArgs a, Prec prec, bool model, LaunchShape shape, hipStream_t st);
hipError_t launch_dense_grad(DenseArgs a, Prec prec, bool nll, LaunchShape shape, hipStream_t st);
// the mixed-precision adjoint (lanes over observations, binary64 correction of E and v)
hipError_t launch_grad_mixed(DenseArgs a, bool nll, LaunchShape shape, hipStream_t st);
hipError_t launch_planet_velocities(DenseArgs a, LaunchShape shape, hipStream_t st);
hipError_t launch_chisq_from_velocities(DenseArgs a, LaunchShape shape, hipStream_t st);
hipError_t launch_ragged(RaggedArgs a, LaunchShape shape, int grid, hipStream_t st);
int ragged_max_grid(LaunchShape shape, int sb, int gmax);
// The allocation-free variant: checks and orders the systems on the device
// (into the static scratch array), then runs the persistent kernel; a.order
// and a.queue are set here.  a.sb and a.gmax must be set.  No allocation.
hipError_t launch_ragged_static(RaggedArgs a, LaunchShape shape, hipStream_t st);
// Plain binary64 ragged chi-square (kep_ragged64.hip): one wavefront per system, grid-stride over the
// work order (a.order, or the systems in order when null); checks every system's offsets itself.
hipError_t launch_ragged64(RaggedArgs a, LaunchShape shape, hipStream_t st);
int ragged64_grid(LaunchShape shape, int64_t n_sys);   // the blocks launch_ragged64 launches
bool ragged_shape_fits(int block, int sb);   // LDS of the persistent kernel (slices + table) within 64 KiB
hipError_t launch_astro(AstroArgs a, Prec prec, bool model, LaunchShape shape, hipStream_t st);
// Gauss-Newton products: chi2 into a.out, J^T W r [np][n_sys], packed J^T W J
hipError_t launch_eccentric_anomalies(DenseArgs a, LaunchShape shape, hipStream_t st);
hipError_t launch_gn(DenseArgs a, double *jtwr, double *jtwj, Prec prec, LaunchShape shape, hipStream_t st);
// DE-MC: chi-square of the whole population (both halves; NaN where K < 0),
// one generation (both halves), the device generation counter's setter and
// increment.
hipError_t launch_demc_chisq(DemcArgs a, DenseArgs base, Prec prec, LaunchShape shape, hipStream_t st);
hipError_t launch_demc_generation(DemcArgs a, DenseArgs base, Prec prec, LaunchShape shape, hipStream_t st);
hipError_t launch_demc_set_gen(uint64_t *gen, uint64_t value, hipStream_t st);
hipError_t launch_demc_advance(uint64_t *gen, uint64_t inc, hipStream_t st);
// one fused half-step (propose, chi-square, accept) of half h
hipError_t launch_demc_half(DemcArgs m, DenseArgs base, Prec prec, int h, LaunchShape shape, hipStream_t st);
int device_cu_count();
// blocks of `kern` per CU at this block size and dynamic LDS (cached per device)
int cached_occupancy(const void *kern, int block, size_t lds);

}  // namespace kep
