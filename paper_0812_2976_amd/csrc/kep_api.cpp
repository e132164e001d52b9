// C ABI of the library (include/kepler.h): argument checking, launch shape,
// ragged plans (work ordering, autotuning, HIP graph) and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "kep_internal.h"
#include "kepler.h"

namespace {

thread_local std::string g_last_error;

kep_status fail(kep_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

kep_status launch_status(hipError_t err, const char *what)
{
    if (err == hipSuccess) return KEP_OK;
    return fail(KEP_ERR_LAUNCH, "%s: kernel launch failed: %s", what, hipGetErrorString(err));
}

struct Opts {
    int fixed_iter = 0;
    int max_iter = 10;
    kep::LaunchShape shape{0, 0};
};

kep_status parse_opts(const kep_options *o, const char *fn, Opts &out)
{
    out = Opts();
    if (!o) return KEP_OK;
    if (o->fixed_iter > 1000) return fail(KEP_ERR_ARG, "%s: fixed_iter = %d exceeds 1000", fn, o->fixed_iter);
    if (o->max_iter < 0 || o->max_iter > 1000)
        return fail(KEP_ERR_ARG, "%s: max_iter = %d outside [0, 1000]", fn, o->max_iter);
    if (o->block_threads < 0 || o->block_threads > 256 || o->block_threads % 64 != 0)
        return fail(KEP_ERR_ARG, "%s: block_threads = %d must be 0 or a multiple of 64 up to 256", fn,
                    o->block_threads);
    if (o->blocks_per_cu < 0 || o->blocks_per_cu > 64)
        return fail(KEP_ERR_ARG, "%s: blocks_per_cu = %d outside [0, 64]", fn, o->blocks_per_cu);
    out.fixed_iter = o->fixed_iter;
    if (o->max_iter > 0) out.max_iter = o->max_iter;
    out.shape.block = o->block_threads;
    out.shape.blocks_per_cu = o->blocks_per_cu;
    return KEP_OK;
}

kep_status check_prec(kep_prec p, const char *fn)
{
    if (p != KEP_FP64 && p != KEP_MIXED) return fail(KEP_ERR_ARG, "%s: unknown precision %d", fn, (int)p);
    return KEP_OK;
}

// The device count is read until a device is found, then remembered: the
// query costs as much as a small launch.
kep_status check_device(const char *fn)
{
    static std::atomic<bool> found{false};
    if (found.load(std::memory_order_relaxed)) return KEP_OK;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return fail(KEP_ERR_DEVICE, "%s: no HIP device", fn);
    found.store(true, std::memory_order_relaxed);
    return KEP_OK;
}

bool mul_overflows(int64_t a, int64_t b) { return a != 0 && b > INT64_MAX / a; }

kep_status check_dense(const kep_obs *obs, const kep_params *par, bool need_v, const char *fn)
{
    if (!obs || !par) return fail(KEP_ERR_ARG, "%s: obs and params must not be NULL", fn);
    if (obs->n_obs < 0) return fail(KEP_ERR_ARG, "%s: n_obs = %lld < 0", fn, (long long)obs->n_obs);
    if (par->n_sys < 0) return fail(KEP_ERR_ARG, "%s: n_sys = %lld < 0", fn, (long long)par->n_sys);
    if (par->n_pl < 1 || par->n_pl > KEP_MAX_PL)
        return fail(KEP_ERR_SHAPE, "%s: n_pl = %lld outside [1, %d]", fn, (long long)par->n_pl, KEP_MAX_PL);
    if (mul_overflows(par->n_sys, par->n_pl) || mul_overflows(par->n_sys, obs->n_obs) ||
        mul_overflows(par->n_sys, 5 * par->n_pl + 1))
        return fail(KEP_ERR_SHAPE, "%s: n_sys x n_pl or n_sys x n_obs overflows", fn);
    if (obs->n_obs > 0 && !obs->t) return fail(KEP_ERR_ARG, "%s: obs->t is NULL", fn);
    if (need_v && obs->n_obs > 0 && (!obs->v || !obs->sigma))
        return fail(KEP_ERR_ARG, "%s: obs->v and obs->sigma must not be NULL", fn);
    if (par->n_sys > 0 && (!par->P || !par->K || !par->e || !par->omega || !par->M0))
        return fail(KEP_ERR_ARG, "%s: a parameter plane (P, K, e, omega, M0) is NULL", fn);
    return KEP_OK;
}

kep::DenseArgs make_dense(const kep_obs *obs, const kep_params *par, const Opts &o, double *out, double *grad)
{
    kep::DenseArgs a;
    a.t = obs->t;
    a.v = obs->v;
    a.sigma = obs->sigma;
    a.n_obs = obs->n_obs;
    a.t0 = obs->t0;
    a.P = par->P;
    a.K = par->K;
    a.e = par->e;
    a.w = par->omega;
    a.M0 = par->M0;
    a.offset = par->offset;
    a.jitter = par->jitter;
    a.n_sys = par->n_sys;
    a.n_pl = (int)par->n_pl;
    a.sb = 1;
    a.out = out;
    a.grad = grad;
    a.dv = nullptr;
    a.fixed_iter = o.fixed_iter;
    a.max_iter = o.max_iter;
    return a;
}

kep::Prec to_prec(kep_prec p) { return p == KEP_MIXED ? kep::Prec::Mixed : kep::Prec::F64; }

}  // namespace

extern "C" {

const char *kep_last_error(void) { return g_last_error.c_str(); }

int kep_abi_version(void) { return KEP_ABI_VERSION; }

kep_status kepler_solve(const double *M, const double *e, double *E, int64_t n, kep_prec prec,
                        const kep_options *opts, void *stream)
{
    static const char *fn = "kepler_solve";
    if (n < 0) return fail(KEP_ERR_ARG, "%s: n = %lld < 0", fn, (long long)n);
    if (kep_status s = check_prec(prec, fn)) return s;
    Opts o;
    if (kep_status s = parse_opts(opts, fn, o)) return s;
    if (n == 0) return KEP_OK;
    if (!M || !e || !E) return fail(KEP_ERR_ARG, "%s: M, e and E must not be NULL", fn);
    if (E == M || E == e) return fail(KEP_ERR_ARG, "%s: E must not alias M or e", fn);
    if (kep_status s = check_device(fn)) return s;
    return launch_status(kep::launch_kepler_solve(M, e, E, n, to_prec(prec), o.fixed_iter, o.max_iter, o.shape,
                                                  (hipStream_t)stream),
                         fn);
}

kep_status rv_model(const kep_obs *obs, const kep_params *par, double *v_model, kep_prec prec,
                    const kep_options *opts, void *stream)
{
    static const char *fn = "rv_model";
    if (kep_status s = check_prec(prec, fn)) return s;
    if (kep_status s = check_dense(obs, par, false, fn)) return s;
    Opts o;
    if (kep_status s = parse_opts(opts, fn, o)) return s;
    if (par->n_sys == 0 || obs->n_obs == 0) return KEP_OK;
    if (!v_model) return fail(KEP_ERR_ARG, "%s: v_model is NULL", fn);
    if (kep_status s = check_device(fn)) return s;
    kep::DenseArgs a = make_dense(obs, par, o, v_model, nullptr);
    return launch_status(kep::launch_dense(a, to_prec(prec), true, o.shape, (hipStream_t)stream), fn);
}

kep_status rv_chisq(const kep_obs *obs, const kep_params *par, double *chi2, kep_prec prec,
                    const kep_options *opts, void *stream)
{
    static const char *fn = "rv_chisq";
    if (kep_status s = check_prec(prec, fn)) return s;
    if (kep_status s = check_dense(obs, par, true, fn)) return s;
    Opts o;
    if (kep_status s = parse_opts(opts, fn, o)) return s;
    if (par->n_sys == 0) return KEP_OK;
    if (!chi2) return fail(KEP_ERR_ARG, "%s: chi2 is NULL", fn);
    if (kep_status s = check_device(fn)) return s;
    kep::DenseArgs a = make_dense(obs, par, o, chi2, nullptr);
    return launch_status(kep::launch_dense(a, to_prec(prec), false, o.shape, (hipStream_t)stream), fn);
}

static kep_status dense_grad(const kep_obs *obs, const kep_params *par, double *out, double *grad, kep_prec prec,
                             const kep_options *opts, void *stream, bool nll, const char *fn)
{
    if (kep_status s = check_prec(prec, fn)) return s;
    if (kep_status s = check_dense(obs, par, true, fn)) return s;
    Opts o;
    if (kep_status s = parse_opts(opts, fn, o)) return s;
    if (par->n_sys == 0) return KEP_OK;
    if (!out || !grad) return fail(KEP_ERR_ARG, "%s: %s and grad must not be NULL", fn, nll ? "nll" : "chi2");
    if (kep_status s = check_device(fn)) return s;
    kep::DenseArgs a = make_dense(obs, par, o, out, grad);
    return launch_status(kep::launch_dense_grad(a, to_prec(prec), nll, o.shape, (hipStream_t)stream), fn);
}

kep_status rv_chisq_grad(const kep_obs *obs, const kep_params *par, double *chi2, double *grad, kep_prec prec,
                         const kep_options *opts, void *stream)
{
    return dense_grad(obs, par, chi2, grad, prec, opts, stream, false, "rv_chisq_grad");
}

kep_status rv_nll_grad(const kep_obs *obs, const kep_params *par, double *nll, double *grad, kep_prec prec,
                       const kep_options *opts, void *stream)
{
    return dense_grad(obs, par, nll, grad, prec, opts, stream, true, "rv_nll_grad");
}

kep_status rv_chisq_gn(const kep_obs *obs, const kep_params *par, double *chi2, double *jtwr, double *jtwj,
                       kep_prec prec, const kep_options *opts, void *stream)
{
    static const char *fn = "rv_chisq_gn";
    if (kep_status s = check_prec(prec, fn)) return s;
    if (kep_status s = check_dense(obs, par, true, fn)) return s;
    Opts o;
    if (kep_status s = parse_opts(opts, fn, o)) return s;
    if (o.shape.block != 0 && o.shape.block > 256) return fail(KEP_ERR_ARG, "%s: block_threads too large", fn);
    if (par->n_sys == 0) return KEP_OK;
    if (!chi2 || !jtwr || !jtwj) return fail(KEP_ERR_ARG, "%s: chi2, jtwr and jtwj must not be NULL", fn);
    if (kep_status s = check_device(fn)) return s;
    kep::DenseArgs a = make_dense(obs, par, o, chi2, nullptr);
    return launch_status(kep::launch_gn(a, jtwr, jtwj, to_prec(prec), o.shape, (hipStream_t)stream), fn);
}

static kep_status astro_common(const kep_astro_obs *obs, const kep_astro_params *par, double *out, kep_prec prec,
                               const kep_options *opts, void *stream, bool model, const char *fn)
{
    if (kep_status s = check_prec(prec, fn)) return s;
    if (!obs || !par) return fail(KEP_ERR_ARG, "%s: obs and params must not be NULL", fn);
    if (obs->n_obs < 0) return fail(KEP_ERR_ARG, "%s: n_obs = %lld < 0", fn, (long long)obs->n_obs);
    if (par->n_sys < 0) return fail(KEP_ERR_ARG, "%s: n_sys = %lld < 0", fn, (long long)par->n_sys);
    if (par->n_pl < 1 || par->n_pl > KEP_MAX_PL)
        return fail(KEP_ERR_SHAPE, "%s: n_pl = %lld outside [1, %d]", fn, (long long)par->n_pl, KEP_MAX_PL);
    if (mul_overflows(par->n_sys, par->n_pl) || mul_overflows(par->n_sys, 2 * obs->n_obs))
        return fail(KEP_ERR_SHAPE, "%s: n_sys x n_pl or n_sys x n_obs overflows", fn);
    if (obs->n_obs > 0 && !obs->t) return fail(KEP_ERR_ARG, "%s: obs->t is NULL", fn);
    if (!model && obs->n_obs > 0 && (!obs->x || !obs->y || !obs->sigma_x || !obs->sigma_y))
        return fail(KEP_ERR_ARG, "%s: obs->x, y, sigma_x and sigma_y must not be NULL", fn);
    if (par->n_sys > 0 && (!par->P || !par->e || !par->M0 || !par->A || !par->B || !par->F || !par->G))
        return fail(KEP_ERR_ARG, "%s: a parameter plane (P, e, M0, A, B, F, G) is NULL", fn);
    Opts o;
    if (kep_status s = parse_opts(opts, fn, o)) return s;
    if (par->n_sys == 0 || (model && obs->n_obs == 0)) return KEP_OK;
    if (!out) return fail(KEP_ERR_ARG, "%s: output is NULL", fn);
    if (kep_status s = check_device(fn)) return s;
    kep::AstroArgs a{};
    a.t = obs->t;
    a.x = obs->x;
    a.y = obs->y;
    a.sx = obs->sigma_x;
    a.sy = obs->sigma_y;
    a.n_obs = obs->n_obs;
    a.t0 = obs->t0;
    a.P = par->P;
    a.e = par->e;
    a.M0 = par->M0;
    a.A = par->A;
    a.B = par->B;
    a.F = par->F;
    a.G = par->G;
    a.x0 = par->x0;
    a.y0 = par->y0;
    a.n_sys = par->n_sys;
    a.n_pl = (int)par->n_pl;
    a.sb = 1;
    a.out = out;
    a.fixed_iter = o.fixed_iter;
    a.max_iter = o.max_iter;
    return launch_status(kep::launch_astro(a, to_prec(prec), model, o.shape, (hipStream_t)stream), fn);
}

kep_status astro_model(const kep_astro_obs *obs, const kep_astro_params *par, double *xy, kep_prec prec,
                       const kep_options *opts, void *stream)
{
    return astro_common(obs, par, xy, prec, opts, stream, true, "astro_model");
}

kep_status astro_chisq(const kep_astro_obs *obs, const kep_astro_params *par, double *chi2, kep_prec prec,
                       const kep_options *opts, void *stream)
{
    return astro_common(obs, par, chi2, prec, opts, stream, false, "astro_chisq");
}

kep_status rv_planet_velocities(const kep_obs *obs, const kep_params *par, float *dv, const kep_options *opts,
                                void *stream)
{
    static const char *fn = "rv_planet_velocities";
    if (kep_status s = check_dense(obs, par, false, fn)) return s;
    Opts o;
    if (kep_status s = parse_opts(opts, fn, o)) return s;
    if (par->n_sys == 0 || obs->n_obs == 0) return KEP_OK;
    if (!dv) return fail(KEP_ERR_ARG, "%s: dv is NULL", fn);
    if (mul_overflows(par->n_sys * par->n_pl, obs->n_obs)) return fail(KEP_ERR_SHAPE, "%s: n_pl x n_sys x n_obs overflows", fn);
    if (kep_status s = check_device(fn)) return s;
    kep::DenseArgs a = make_dense(obs, par, o, nullptr, nullptr);
    a.dv = dv;
    return launch_status(kep::launch_planet_velocities(a, o.shape, (hipStream_t)stream), fn);
}

kep_status rv_eccentric_anomalies(const kep_obs *obs, const kep_params *par, float *E, const kep_options *opts,
                                  void *stream)
{
    static const char *fn = "rv_eccentric_anomalies";
    if (kep_status s = check_dense(obs, par, false, fn)) return s;
    Opts o;
    if (kep_status s = parse_opts(opts, fn, o)) return s;
    if (par->n_sys == 0 || obs->n_obs == 0) return KEP_OK;
    if (!E) return fail(KEP_ERR_ARG, "%s: E is NULL", fn);
    if (mul_overflows(par->n_sys * par->n_pl, obs->n_obs)) return fail(KEP_ERR_SHAPE, "%s: n_pl x n_sys x n_obs overflows", fn);
    if (kep_status s = check_device(fn)) return s;
    kep::DenseArgs a = make_dense(obs, par, o, nullptr, nullptr);
    a.dv = E;
    return launch_status(kep::launch_eccentric_anomalies(a, o.shape, (hipStream_t)stream), fn);
}

kep_status rv_chisq_from_velocities(const kep_obs *obs, const kep_params *par, const float *dv, double *chi2,
                                    const kep_options *opts, void *stream)
{
    static const char *fn = "rv_chisq_from_velocities";
    if (!obs || !par) return fail(KEP_ERR_ARG, "%s: obs and params must not be NULL", fn);
    if (obs->n_obs < 0 || par->n_sys < 0) return fail(KEP_ERR_ARG, "%s: negative size", fn);
    if (par->n_pl < 1 || par->n_pl > KEP_MAX_PL)
        return fail(KEP_ERR_SHAPE, "%s: n_pl = %lld outside [1, %d]", fn, (long long)par->n_pl, KEP_MAX_PL);
    if (obs->n_obs > 1024)
        return fail(KEP_ERR_UNSUPPORTED, "%s: n_obs = %lld above 1024", fn, (long long)obs->n_obs);
    if (mul_overflows(par->n_sys * par->n_pl, obs->n_obs)) return fail(KEP_ERR_SHAPE, "%s: sizes overflow", fn);
    Opts o;
    if (kep_status s = parse_opts(opts, fn, o)) return s;
    if (par->n_sys == 0) return KEP_OK;
    if (obs->n_obs > 0 && (!obs->t || !obs->v || !obs->sigma || !dv))
        return fail(KEP_ERR_ARG, "%s: t, v, sigma and dv must not be NULL", fn);
    if (!chi2) return fail(KEP_ERR_ARG, "%s: chi2 is NULL", fn);
    if (kep_status s = check_device(fn)) return s;
    kep::DenseArgs a = make_dense(obs, par, o, chi2, nullptr);
    a.dv = const_cast<float *>(dv);
    return launch_status(kep::launch_chisq_from_velocities(a, o.shape, (hipStream_t)stream), fn);
}

}  // extern "C"

// ====================================================================== ragged
struct kep_plan {
    kep::RaggedArgs args;
    kep::LaunchShape shape;
    int grid = 0;
    int tuned = 0;
    double tuned_ms = 0.0;
    int64_t n_obs_total = 0, n_pl_total = 0, triples = 0;
    int32_t *d_order = nullptr;
    int64_t *d_obs_off = nullptr;     // the checked CSR offsets (the plan's own copies)
    int64_t *d_pl_off = nullptr;
    unsigned int *d_queue = nullptr;
    double *bound_out = nullptr;      // output pointer recorded in the graph
    bool fp64 = false;                // KEP_FP64: the binary64 kernel, launched directly (no tuning, no graph)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t kernel_node = nullptr;
};

namespace {

struct TuneEntry {
    std::string key;
    int block, sb, gmax;
    double ms;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;
bool g_tune_loaded = false;

std::string device_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    return std::string(prop.gcnArchName);
}

// Shape class of a ragged batch: log2 buckets of the system count and of the
// mean work per system.
std::string tune_key(int64_t n_sys, double mean_work)
{
    int b_sys = 0, b_work = 0;
    while ((1LL << (b_sys + 1)) <= n_sys) ++b_sys;
    while ((double)(1LL << (b_work + 1)) <= mean_work) ++b_work;
    char buf[160];
    snprintf(buf, sizeof buf, "%s/ragged_mixed/s%d/w%d", device_name().c_str(), b_sys, b_work);
    return buf;
}

// Optional persistence: KEP_TUNE_CACHE names a text file of "key block sb gmax ms" lines.
void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = getenv("KEP_TUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char key[200];
    int block, sb, gmax;
    double ms;
    while (fscanf(f, "%199s %d %d %d %lf", key, &block, &sb, &gmax, &ms) == 5) {
        const bool valid = (block == 64 || block == 128 || block == 192 || block == 256) && sb >= 1 &&
                           sb <= kep::kMaxSB && (gmax == 2 || gmax == 4);
        if (valid) g_tune.push_back({key, block, sb, gmax, ms});
    }
    fclose(f);
}

void tune_store_locked(const TuneEntry &e)
{
    for (auto &x : g_tune)
        if (x.key == e.key) { x = e; goto save; }
    g_tune.push_back(e);
save:
    const char *path = getenv("KEP_TUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "w");
    if (!f) return;
    for (auto &x : g_tune) fprintf(f, "%s %d %d %d %.6f\n", x.key.c_str(), x.block, x.sb, x.gmax, x.ms);
    fclose(f);
}

kep_status plan_capture(kep_plan *p, hipStream_t user)
{
    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
        return fail(KEP_ERR_DEVICE, "kep_plan_ragged: hipStreamCreate failed");
    hipError_t err = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (err == hipSuccess) err = kep::launch_ragged(p->args, p->shape, p->grid, cap);
    hipGraph_t g = nullptr;
    hipError_t err2 = hipStreamEndCapture(cap, &g);
    (void)hipStreamDestroy(cap);
    if (err != hipSuccess || err2 != hipSuccess || !g)
        return fail(KEP_ERR_LAUNCH, "kep_plan_ragged: graph capture failed: %s",
                    hipGetErrorString(err != hipSuccess ? err : err2));
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(KEP_ERR_LAUNCH, "kep_plan_ragged: graph instantiation failed");
    }
    // uploaded now: otherwise the first launches of the graph carry the upload
    (void)hipGraphUpload(ex, user);
    // the kernel node that runs the persistent kernel (the last node of the chain)
    size_t n = 0;
    (void)hipGraphGetNodes(g, nullptr, &n);
    std::vector<hipGraphNode_t> nodes(n);
    if (n) (void)hipGraphGetNodes(g, nodes.data(), &n);
    hipGraphNode_t kn = nullptr;
    for (auto nd : nodes) {
        hipGraphNodeType ty;
        if (hipGraphNodeGetType(nd, &ty) == hipSuccess && ty == hipGraphNodeTypeKernel) {
            hipKernelNodeParams kp;
            if (hipGraphKernelNodeGetParams(nd, &kp) == hipSuccess && kp.sharedMemBytes > 0) kn = nd;
        }
    }
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph = g;
    p->exec = ex;
    p->kernel_node = kn;
    p->bound_out = p->args.out;
    return KEP_OK;
}

double time_candidate(kep_plan *p, hipStream_t st, int reps)
{
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    // warm-up (the kernel leaves its queue counters at zero for the next launch)
    (void)kep::launch_ragged(p->args, p->shape, p->grid, st);
    (void)hipEventRecord(a, st);
    for (int r = 0; r < reps; ++r) (void)kep::launch_ragged(p->args, p->shape, p->grid, st);
    (void)hipEventRecord(b, st);
    (void)hipEventSynchronize(b);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (hipGetLastError() != hipSuccess) return 1e30;
    return (double)ms / reps;
}

void plan_free(kep_plan *p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->d_order) (void)hipFree(p->d_order);
    if (p->d_obs_off) (void)hipFree(p->d_obs_off);
    if (p->d_pl_off) (void)hipFree(p->d_pl_off);
    if (p->d_queue) (void)hipFree(p->d_queue);
    delete p;
}

}  // namespace

extern "C" {

kep_status kep_plan_ragged(const kep_obs_csr *obs, const kep_params_csr *par, kep_prec prec,
                           const kep_options *opts, void *stream, kep_plan **out)
{
    static const char *fn = "kep_plan_ragged";
    if (!out) return fail(KEP_ERR_ARG, "%s: out is NULL", fn);
    *out = nullptr;
    if (!obs || !par) return fail(KEP_ERR_ARG, "%s: obs and params must not be NULL", fn);
    if (kep_status s = check_prec(prec, fn)) return s;
    Opts o;
    if (kep_status s = parse_opts(opts, fn, o)) return s;
    const int64_t n_sys = par->n_sys;
    if (n_sys < 0 || n_sys > INT32_MAX) return fail(KEP_ERR_ARG, "%s: n_sys = %lld outside [0, 2^31)", fn, (long long)n_sys);
    if (obs->n_obs_total < 0 || par->n_pl_total < 0) return fail(KEP_ERR_ARG, "%s: negative totals", fn);
    if (!obs->obs_off || !par->pl_off) return fail(KEP_ERR_ARG, "%s: obs_off and pl_off must not be NULL", fn);
    if (obs->n_obs_total > 0 && (!obs->t || !obs->v || !obs->sigma))
        return fail(KEP_ERR_ARG, "%s: t, v, sigma must not be NULL", fn);
    if (par->n_pl_total > 0 && (!par->P || !par->K || !par->e || !par->omega || !par->M0))
        return fail(KEP_ERR_ARG, "%s: a parameter array is NULL", fn);
    if (kep_status s = check_device(fn)) return s;
    hipStream_t st = (hipStream_t)stream;

    std::vector<int64_t> ooff(n_sys + 1), poff(n_sys + 1);
    if (hipMemcpyAsync(ooff.data(), obs->obs_off, sizeof(int64_t) * (n_sys + 1), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(poff.data(), par->pl_off, sizeof(int64_t) * (n_sys + 1), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(KEP_ERR_DEVICE, "%s: cannot read the CSR offsets", fn);
    if (ooff[0] != 0 || poff[0] != 0) return fail(KEP_ERR_SHAPE, "%s: offsets must start at 0", fn);
    if (ooff[n_sys] != obs->n_obs_total || poff[n_sys] != par->n_pl_total)
        return fail(KEP_ERR_SHAPE, "%s: last offsets (%lld, %lld) differ from the totals (%lld, %lld)", fn,
                    (long long)ooff[n_sys], (long long)poff[n_sys], (long long)obs->n_obs_total,
                    (long long)par->n_pl_total);
    std::vector<int64_t> work(n_sys);
    int64_t triples = 0;
    for (int64_t i = 0; i < n_sys; ++i) {
        const int64_t no = ooff[i + 1] - ooff[i], np = poff[i + 1] - poff[i];
        if (no < 0) return fail(KEP_ERR_SHAPE, "%s: obs_off decreases at system %lld", fn, (long long)i);
        if (np < 1 || np > KEP_MAX_PL)
            return fail(KEP_ERR_SHAPE, "%s: system %lld has %lld planets, outside [1, %d]", fn, (long long)i,
                        (long long)np, KEP_MAX_PL);
        work[i] = np * std::max<int64_t>(no, 1);
        triples += np * no;
    }
    // work order: decreasing work (n_pl x n_obs), so the smallest items come
    // last; then, within each window of kOrderWindow systems, by planet count,
    // so that the systems of one work item mostly share a planet count (their
    // packed tails then run the same number of planet iterations) while
    // consecutive items still alternate between planet counts (a whole launch
    // phase of one-planet systems, whose per-observation loads weigh most,
    // measured 7% slower at c3)
    constexpr size_t kOrderWindow = 256;
    std::vector<int32_t> order(n_sys);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return work[a] > work[b]; });
    for (size_t w0 = 0; w0 < order.size(); w0 += kOrderWindow) {
        const auto e = order.begin() + (ptrdiff_t)std::min(order.size(), w0 + kOrderWindow);
        std::stable_sort(order.begin() + (ptrdiff_t)w0, e, [&](int32_t a, int32_t b) {
            return poff[a + 1] - poff[a] > poff[b + 1] - poff[b];
        });
    }

    kep_plan *p = new kep_plan();
    p->n_obs_total = obs->n_obs_total;
    p->n_pl_total = par->n_pl_total;
    p->triples = triples;
    if (n_sys > 0 && (hipMalloc(&p->d_order, sizeof(int32_t) * n_sys) != hipSuccess ||
                      hipMemcpy(p->d_order, order.data(), sizeof(int32_t) * n_sys, hipMemcpyHostToDevice) != hipSuccess)) {
        plan_free(p);
        return fail(KEP_ERR_DEVICE, "%s: cannot allocate the work order", fn);
    }
    // the kernel reads the offsets the plan checked, not the caller's arrays,
    // whose later contents could send it outside the observation arrays
    const size_t off_bytes = sizeof(int64_t) * (size_t)(n_sys + 1);
    if (hipMalloc(&p->d_obs_off, off_bytes) != hipSuccess || hipMalloc(&p->d_pl_off, off_bytes) != hipSuccess ||
        hipMemcpy(p->d_obs_off, ooff.data(), off_bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_pl_off, poff.data(), off_bytes, hipMemcpyHostToDevice) != hipSuccess) {
        plan_free(p);
        return fail(KEP_ERR_DEVICE, "%s: cannot copy the CSR offsets", fn);
    }
    // the queue and exit counters start at zero; every launch leaves them at zero
    if (hipMalloc(&p->d_queue, kep::kQueueWords * sizeof(unsigned int)) != hipSuccess ||
        hipMemset(p->d_queue, 0, kep::kQueueWords * sizeof(unsigned int)) != hipSuccess) {
        plan_free(p);
        return fail(KEP_ERR_DEVICE, "%s: cannot allocate the work queue", fn);
    }
    kep::RaggedArgs &a = p->args;
    a.t = obs->t;
    a.v = obs->v;
    a.sigma = obs->sigma;
    a.obs_off = p->d_obs_off;
    a.t0 = obs->t0;
    a.P = par->P;
    a.K = par->K;
    a.e = par->e;
    a.w = par->omega;
    a.M0 = par->M0;
    a.pl_off = p->d_pl_off;
    a.offset = par->offset;
    a.jitter = par->jitter;
    a.order = p->d_order;
    a.n_sys = n_sys;
    a.n_obs_total = obs->n_obs_total;
    a.n_pl_total = par->n_pl_total;
    a.queue = p->d_queue;
    a.out = nullptr;
    a.fixed_iter = o.fixed_iter;
    a.max_iter = o.max_iter;

    if (prec == KEP_FP64) {
        // the binary64 kernel: one wavefront per system over the work order
        // (decreasing work first balances the grid-stride), no tuning, no graph
        p->fp64 = true;
        p->shape.block = o.shape.block > 0 ? o.shape.block : 256;
        p->shape.blocks_per_cu = o.shape.blocks_per_cu;
        if (p->shape.block > 256) {
            plan_free(p);
            return fail(KEP_ERR_ARG, "%s: block_threads above 256 for KEP_FP64", fn);
        }
        a.sb = 1;
        a.gmax = 4;
        a.n_items = n_sys;
        p->grid = n_sys > 0 ? kep::ragged64_grid(p->shape, n_sys) : 0;
        *out = p;
        return KEP_OK;
    }

    auto configure = [&](int block, int sb, int gmax) {
        p->shape.block = block;
        p->shape.blocks_per_cu = o.shape.blocks_per_cu;
        a.sb = sb;
        a.gmax = gmax;
        a.n_items = (n_sys + sb - 1) / sb;
        const int wpb = block / 64;
        int64_t g = (a.n_items + wpb - 1) / wpb;
        const int cap = kep::ragged_max_grid(p->shape, sb, gmax);
        p->grid = (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
    };

    const double mean_work = n_sys > 0 ? (double)triples / (double)n_sys : 0.0;
    int best_block = o.shape.block > 0 ? o.shape.block : 256;
    int best_sb = 4, best_gmax = 4;
    if (o.shape.block == 0 && n_sys > 0) {
        const std::string key = tune_key(n_sys, mean_work);
        std::lock_guard<std::mutex> lock(g_tune_mu);
        tune_load_locked();
        bool found = false;
        for (auto &x : g_tune)
            if (x.key == key && (x.gmax == 2 || x.gmax == 4) && (x.block == 64 || x.block == 128 || x.block == 256) &&
                x.sb >= 1 && x.sb <= kep::kMaxSB && kep::ragged_shape_fits(x.block, x.sb)) {
                best_block = x.block;
                best_sb = x.sb;
                best_gmax = x.gmax;
                p->tuned_ms = x.ms;
                found = true;
            }
        if (!found && triples > 0) {
            // autotune: time every (block, systems per item) candidate on this batch
            double *scratch = nullptr;
            if (hipMalloc(&scratch, sizeof(double) * n_sys) != hipSuccess) {
                plan_free(p);
                return fail(KEP_ERR_DEVICE, "%s: cannot allocate tuning scratch", fn);
            }
            a.out = scratch;
            double best = 1e30;
            const int blocks[] = {64, 128, 256};
            const int sbs[] = {1, 2, 4, 8, 16, 32};
            const int gmaxs[] = {2, 4};
            // the shader clock ramps over the first launches: warm it up first,
            // so that the sweep's early candidates are not timed slower
            configure(256, 8, 4);
            (void)time_candidate(p, st, 12);
            struct Cand { int block, sb, gmax; double ms; };
            std::vector<Cand> cands;
            for (int gm : gmaxs)
                for (int b : blocks)
                    for (int sb : sbs) {
                        if (!kep::ragged_shape_fits(b, sb)) continue;
                        configure(b, sb, gm);
                        cands.push_back({b, sb, gm, time_candidate(p, st, 2)});
                    }
            // two launches per candidate separate shapes within a few percent only
            // roughly: the four fastest are timed again, in two interleaved rounds
            std::sort(cands.begin(), cands.end(), [](const Cand &x, const Cand &y) { return x.ms < y.ms; });
            const size_t top = std::min<size_t>(4, cands.size());
            std::vector<double> again(top, 0.0);
            for (int round = 0; round < 2; ++round)
                for (size_t k = 0; k < top; ++k) {
                    const size_t i = round == 0 ? k : top - 1 - k;
                    configure(cands[i].block, cands[i].sb, cands[i].gmax);
                    again[i] += time_candidate(p, st, 4);
                }
            for (size_t i = 0; i < top; ++i) {
                const double ms = again[i] / 2.0;
                if (ms < best) {
                    best = ms;
                    best_block = cands[i].block;
                    best_sb = cands[i].sb;
                    best_gmax = cands[i].gmax;
                }
            }
            (void)hipFree(scratch);
            a.out = nullptr;
            p->tuned_ms = best;
            tune_store_locked({key, best_block, best_sb, best_gmax, best});
        }
        p->tuned = 1;
    }
    configure(best_block, best_sb, best_gmax);
    *out = p;
    return KEP_OK;
}

static kep_status ragged_check(kep_plan *plan, double *chi2, const char *fn)
{
    if (!plan) return fail(KEP_ERR_ARG, "%s: plan is NULL", fn);
    if (plan->args.n_sys > 0 && !chi2) return fail(KEP_ERR_ARG, "%s: chi2 is NULL", fn);
    return KEP_OK;
}

kep_status rv_chisq_ragged(kep_plan *plan, double *chi2, void *stream)
{
    static const char *fn = "rv_chisq_ragged";
    if (kep_status s = ragged_check(plan, chi2, fn)) return s;
    if (plan->args.n_sys == 0) return KEP_OK;
    if (plan->fp64) {
        kep::RaggedArgs a = plan->args;
        a.out = chi2;
        return launch_status(kep::launch_ragged64(a, plan->shape, (hipStream_t)stream), fn);
    }
    if (!plan->exec || plan->bound_out != chi2) {
        // (re)record the graph for this output buffer
        plan->args.out = chi2;
        if (!plan->exec) {
            if (kep_status s = plan_capture(plan, (hipStream_t)stream)) return s;
        } else {
            bool updated = false;
            if (plan->kernel_node) {
                void *kargs[] = {&plan->args};
                hipKernelNodeParams kp;
                if (hipGraphKernelNodeGetParams(plan->kernel_node, &kp) == hipSuccess) {
                    kp.kernelParams = kargs;
                    updated = hipGraphExecKernelNodeSetParams(plan->exec, plan->kernel_node, &kp) == hipSuccess &&
                              hipGraphKernelNodeSetParams(plan->kernel_node, &kp) == hipSuccess;
                }
            }
            if (updated) plan->bound_out = chi2;
            else if (kep_status s = plan_capture(plan, (hipStream_t)stream)) return s;
        }
    }
    hipError_t err = hipGraphLaunch(plan->exec, (hipStream_t)stream);
    if (err != hipSuccess) return fail(KEP_ERR_LAUNCH, "%s: graph launch failed: %s", fn, hipGetErrorString(err));
    return KEP_OK;
}

kep_status rv_chisq_ragged_direct(kep_plan *plan, double *chi2, void *stream)
{
    static const char *fn = "rv_chisq_ragged_direct";
    if (kep_status s = ragged_check(plan, chi2, fn)) return s;
    if (plan->args.n_sys == 0) return KEP_OK;
    kep::RaggedArgs a = plan->args;
    a.out = chi2;
    hipStream_t st = (hipStream_t)stream;
    if (plan->fp64) return launch_status(kep::launch_ragged64(a, plan->shape, st), fn);
    hipError_t err = kep::launch_ragged(a, plan->shape, plan->grid, st);
    return launch_status(err, fn);
}

kep_status rv_chisq_ragged_static(const kep_obs_csr *obs, const kep_params_csr *par, double *chi2, kep_prec prec,
                                  const kep_options *opts, void *stream)
{
    static const char *fn = "rv_chisq_ragged_static";
    if (!obs || !par) return fail(KEP_ERR_ARG, "%s: obs and params must not be NULL", fn);
    if (kep_status s = check_prec(prec, fn)) return s;
    Opts o;
    if (kep_status s = parse_opts(opts, fn, o)) return s;
    const int64_t n_sys = par->n_sys;
    if (n_sys < 0) return fail(KEP_ERR_ARG, "%s: n_sys = %lld < 0", fn, (long long)n_sys);
    if (prec == KEP_MIXED && n_sys > kep::kStaticMaxSys)
        return fail(KEP_ERR_SHAPE, "%s: n_sys = %lld exceeds the %lld systems of the static work area (use a plan)",
                    fn, (long long)n_sys, (long long)kep::kStaticMaxSys);
    if (obs->n_obs_total < 0 || par->n_pl_total < 0) return fail(KEP_ERR_ARG, "%s: negative totals", fn);
    if (n_sys == 0) return KEP_OK;
    if (!chi2) return fail(KEP_ERR_ARG, "%s: chi2 is NULL", fn);
    if (!obs->obs_off || !par->pl_off) return fail(KEP_ERR_ARG, "%s: obs_off and pl_off must not be NULL", fn);
    if (obs->n_obs_total > 0 && (!obs->t || !obs->v || !obs->sigma))
        return fail(KEP_ERR_ARG, "%s: t, v, sigma must not be NULL", fn);
    if (par->n_pl_total > 0 && (!par->P || !par->K || !par->e || !par->omega || !par->M0))
        return fail(KEP_ERR_ARG, "%s: a parameter array is NULL", fn);
    if (kep_status s = check_device(fn)) return s;
    kep::RaggedArgs a{};
    a.t = obs->t;
    a.v = obs->v;
    a.sigma = obs->sigma;
    a.obs_off = obs->obs_off;
    a.t0 = obs->t0;
    a.P = par->P;
    a.K = par->K;
    a.e = par->e;
    a.w = par->omega;
    a.M0 = par->M0;
    a.pl_off = par->pl_off;
    a.offset = par->offset;
    a.jitter = par->jitter;
    a.n_sys = n_sys;
    a.n_obs_total = obs->n_obs_total;
    a.n_pl_total = par->n_pl_total;
    a.out = chi2;
    a.fixed_iter = o.fixed_iter;
    a.max_iter = o.max_iter;
    if (prec == KEP_FP64) {
        // the binary64 kernel needs no work area: one wavefront per system in
        // system order, each checking its own offsets against the totals
        a.order = nullptr;
        kep::LaunchShape shape64 = o.shape;
        if (shape64.block > 256) return fail(KEP_ERR_ARG, "%s: block_threads above 256 for KEP_FP64", fn);
        return launch_status(kep::launch_ragged64(a, shape64, (hipStream_t)stream), fn);
    }
    // the launch shape the autotuner picks for the c3-like batches it has seen:
    // 16 systems per work item, observation groups of up to four 64-lane chunks
    a.sb = 16;
    a.gmax = 4;
    kep::LaunchShape shape = o.shape;
    if (shape.block == 0) shape.block = 256;
    if (!kep::ragged_shape_fits(shape.block, a.sb)) return fail(KEP_ERR_ARG, "%s: block_threads too large", fn);
    return launch_status(kep::launch_ragged_static(a, shape, (hipStream_t)stream), fn);
}

kep_status kep_plan_get_info(const kep_plan *plan, kep_plan_info *info)
{
    if (!plan || !info) return fail(KEP_ERR_ARG, "kep_plan_get_info: NULL argument");
    info->n_sys = plan->args.n_sys;
    info->n_obs_total = plan->n_obs_total;
    info->n_pl_total = plan->n_pl_total;
    info->triples = plan->triples;
    info->block_threads = plan->shape.block;
    info->blocks = plan->grid;
    info->sys_per_batch = plan->args.sb;
    info->tuned = plan->tuned;
    info->tuned_ms = plan->tuned_ms;
    info->group_chunks = plan->args.gmax;
    info->reserved = 0;
    return KEP_OK;
}

void kep_plan_destroy(kep_plan *plan) { plan_free(plan); }

}  // extern "C"

// ------------------------------------------------------------------ DE-MC
struct kep_demc_plan {
    kep::DemcArgs args;
    kep::DenseArgs base;
    kep::Prec prec;
    kep::LaunchShape shape;
    uint64_t *d_gen = nullptr;
    hipGraph_t graph = nullptr, graph_many = nullptr;
    hipGraphExec_t exec = nullptr, exec_many = nullptr;   // one generation / kDemcGraphGens generations
};

// generations recorded in the plan's larger graph (one graph launch per this
// many generations; the remainder replays the one-generation graph)
constexpr int kDemcGraphGens = 8;

namespace {

kep_status check_demc(const kep_obs *obs, const kep_demc_state *st, const char *fn)
{
    if (!obs || !st) return fail(KEP_ERR_ARG, "%s: obs and state must not be NULL", fn);
    if (obs->n_obs < 0) return fail(KEP_ERR_ARG, "%s: n_obs = %lld < 0", fn, (long long)obs->n_obs);
    if (obs->n_obs > 0 && (!obs->t || !obs->v || !obs->sigma))
        return fail(KEP_ERR_ARG, "%s: obs->t, obs->v and obs->sigma must not be NULL", fn);
    if (st->n_pl < 1 || st->n_pl > KEP_MAX_PL)
        return fail(KEP_ERR_SHAPE, "%s: n_pl = %lld outside [1, %d]", fn, (long long)st->n_pl, KEP_MAX_PL);
    if (st->n_half < 2 || st->n_half > INT32_MAX)
        return fail(KEP_ERR_SHAPE, "%s: n_half = %lld outside [2, 2^31 - 1]", fn, (long long)st->n_half);
    if (mul_overflows(st->n_half, 2 * (5 * st->n_pl + 1)) || mul_overflows(st->n_half, obs->n_obs))
        return fail(KEP_ERR_SHAPE, "%s: population size overflows", fn);
    if (!st->x || !st->chi2) return fail(KEP_ERR_ARG, "%s: state x and chi2 must not be NULL", fn);
    return KEP_OK;
}

kep_status make_demc(const kep_obs *obs, const kep_demc_state *st, const kep_demc_options *d, double *work,
                     const Opts &o, const char *fn, kep::DemcArgs &a, kep::DenseArgs &base)
{
    const int dim = 5 * (int)st->n_pl + 1;
    a = kep::DemcArgs{};
    a.x = st->x;
    a.chi2 = st->chi2;
    a.n_accept = st->n_accept;
    a.jitter = st->jitter;
    a.nh = st->n_half;
    a.n_pl = (int)st->n_pl;
    a.d = dim;
    if (d) {
        if (!d->eps) return fail(KEP_ERR_ARG, "%s: options->eps must not be NULL", fn);
        if (!std::isfinite(d->gamma)) return fail(KEP_ERR_ARG, "%s: gamma is not finite", fn);
        if (d->jump_every < 0) return fail(KEP_ERR_ARG, "%s: jump_every = %d < 0", fn, d->jump_every);
        if (!work) return fail(KEP_ERR_ARG, "%s: work must not be NULL", fn);
        a.y = work;
        a.c_new = work + (int64_t)dim * st->n_half;
        a.eps = d->eps;
        a.gamma = d->gamma > 0.0 ? d->gamma : 2.38 / std::sqrt(2.0 * dim);
        a.jump_every = d->jump_every;
        a.key0 = (uint32_t)d->seed;
        a.key1 = (uint32_t)(d->seed >> 32);
    }
    base = kep::DenseArgs{};
    base.t = obs->t;
    base.v = obs->v;
    base.sigma = obs->sigma;
    base.n_obs = obs->n_obs;
    base.t0 = obs->t0;
    base.sb = 1;
    base.fixed_iter = o.fixed_iter;
    base.max_iter = o.max_iter;
    return KEP_OK;
}

void demc_plan_free(kep_demc_plan *p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->exec_many) (void)hipGraphExecDestroy(p->exec_many);
    if (p->graph_many) (void)hipGraphDestroy(p->graph_many);
    if (p->d_gen) (void)hipFree(p->d_gen);
    delete p;
}

}  // namespace

extern "C" {

kep_status demc_chisq(const kep_obs *obs, const kep_demc_state *st, kep_prec prec, const kep_options *opts,
                      void *stream)
{
    static const char *fn = "demc_chisq";
    if (kep_status s = check_prec(prec, fn)) return s;
    if (kep_status s = check_demc(obs, st, fn)) return s;
    Opts o;
    if (kep_status s = parse_opts(opts, fn, o)) return s;
    if (kep_status s = check_device(fn)) return s;
    kep::DemcArgs a;
    kep::DenseArgs base;
    if (kep_status s = make_demc(obs, st, nullptr, nullptr, o, fn, a, base)) return s;
    return launch_status(kep::launch_demc_chisq(a, base, to_prec(prec), o.shape, (hipStream_t)stream), fn);
}

kep_status demc_generations(const kep_obs *obs, const kep_demc_state *st, const kep_demc_options *dopt,
                            uint64_t gen0, int64_t n_gen, double *work, kep_prec prec, const kep_options *opts,
                            void *stream)
{
    static const char *fn = "demc_generations";
    if (kep_status s = check_prec(prec, fn)) return s;
    if (kep_status s = check_demc(obs, st, fn)) return s;
    if (!dopt) return fail(KEP_ERR_ARG, "%s: options must not be NULL", fn);
    if (n_gen < 0) return fail(KEP_ERR_ARG, "%s: n_gen = %lld < 0", fn, (long long)n_gen);
    Opts o;
    if (kep_status s = parse_opts(opts, fn, o)) return s;
    kep::DemcArgs a;
    kep::DenseArgs base;
    if (kep_status s = make_demc(obs, st, dopt, work, o, fn, a, base)) return s;
    if (n_gen == 0) return KEP_OK;
    if (kep_status s = check_device(fn)) return s;
    for (int64_t k = 0; k < n_gen; ++k) {
        a.gen = gen0 + (uint64_t)k;
        if (kep_status s = launch_status(kep::launch_demc_generation(a, base, to_prec(prec), o.shape,
                                                                     (hipStream_t)stream), fn))
            return s;
    }
    return KEP_OK;
}

kep_status kep_plan_demc(const kep_obs *obs, const kep_demc_state *st, const kep_demc_options *dopt, double *work,
                         kep_prec prec, const kep_options *opts, void *stream, kep_demc_plan **out)
{
    static const char *fn = "kep_plan_demc";
    (void)stream;
    if (!out) return fail(KEP_ERR_ARG, "%s: out must not be NULL", fn);
    *out = nullptr;
    if (kep_status s = check_prec(prec, fn)) return s;
    if (kep_status s = check_demc(obs, st, fn)) return s;
    if (!dopt) return fail(KEP_ERR_ARG, "%s: options must not be NULL", fn);
    Opts o;
    if (kep_status s = parse_opts(opts, fn, o)) return s;
    if (kep_status s = check_device(fn)) return s;
    kep_demc_plan *p = new kep_demc_plan();
    if (kep_status s = make_demc(obs, st, dopt, work, o, fn, p->args, p->base)) {
        delete p;
        return s;
    }
    p->prec = to_prec(prec);
    p->shape = o.shape;
    if (hipMalloc(&p->d_gen, sizeof(uint64_t)) != hipSuccess) {
        delete p;
        return fail(KEP_ERR_DEVICE, "%s: hipMalloc of the generation counter failed", fn);
    }
    p->args.gen_ptr = p->d_gen;
    for (int many = 0; many < 2; ++many) {
        hipStream_t cap = nullptr;
        if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
            demc_plan_free(p);
            return fail(KEP_ERR_DEVICE, "%s: hipStreamCreate failed", fn);
        }
        hipGraph_t &graph = many ? p->graph_many : p->graph;
        hipGraphExec_t &exec = many ? p->exec_many : p->exec;
        // generation k of the graph reads counter + k; one node advances the counter
        const int ng = many ? kDemcGraphGens : 1;
        hipError_t err = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        for (int k = 0; k < ng && err == hipSuccess; ++k) {
            kep::DemcArgs a = p->args;
            a.gen = (uint64_t)k;
            err = kep::launch_demc_generation(a, p->base, p->prec, p->shape, cap);
        }
        if (err == hipSuccess) err = kep::launch_demc_advance(p->d_gen, (uint64_t)ng, cap);
        hipError_t err2 = hipStreamEndCapture(cap, &graph);
        (void)hipStreamDestroy(cap);
        if (err != hipSuccess || err2 != hipSuccess || !graph) {
            demc_plan_free(p);
            return fail(KEP_ERR_LAUNCH, "%s: graph capture failed: %s", fn,
                        hipGetErrorString(err != hipSuccess ? err : err2));
        }
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            demc_plan_free(p);
            return fail(KEP_ERR_LAUNCH, "%s: graph instantiation failed", fn);
        }
        (void)hipGraphUpload(exec, (hipStream_t)stream);   // else the first launches carry the upload
    }
    *out = p;
    return KEP_OK;
}

kep_status demc_run(kep_demc_plan *plan, uint64_t gen0, int64_t n_gen, void *stream)
{
    static const char *fn = "demc_run";
    if (!plan) return fail(KEP_ERR_ARG, "%s: plan is NULL", fn);
    if (n_gen < 0) return fail(KEP_ERR_ARG, "%s: n_gen = %lld < 0", fn, (long long)n_gen);
    if (n_gen == 0) return KEP_OK;
    if (kep_status s = launch_status(kep::launch_demc_set_gen(plan->d_gen, gen0, (hipStream_t)stream), fn))
        return s;
    for (int64_t k = 0; k < n_gen;) {
        const bool many = n_gen - k >= kDemcGraphGens;
        hipError_t err = hipGraphLaunch(many ? plan->exec_many : plan->exec, (hipStream_t)stream);
        if (err != hipSuccess) return fail(KEP_ERR_LAUNCH, "%s: graph launch failed: %s", fn, hipGetErrorString(err));
        k += many ? kDemcGraphGens : 1;
    }
    return KEP_OK;
}

void kep_demc_plan_destroy(kep_demc_plan *plan) { demc_plan_free(plan); }

}  // extern "C"
