"""MI355X (gfx950) Keplerian radial-velocity chi-square — Python binding.

A thin ctypes layer over ``libkepler.so`` (C ABI in ``include/kepler.h``).
Every computation runs in the library's HIP kernels; this module only checks
and marshals torch tensors (device memory) and passes torch's current HIP
stream.  There is no CPU fallback: without the built library or a GPU every
call raises.

Functions keep the C names:
  kepler_solve(M, e)                       Kepler's equation (Eq. 1)
  rv_model(t, P, K, e, omega, M0, ...)     model velocities (Eq. 2, 3)
  rv_chisq(t, v, sigma, P, K, e, ...)      chi-square (Eq. 5)
  rv_chisq_grad(...)                       chi-square and its gradient
  rv_nll_grad(...)                         likelihood with jitter and its gradient
  rv_chisq_gn(...)                         Gauss-Newton products J^T W r, J^T W J (matrix cores)
  rv_planet_velocities / rv_chisq_from_velocities   the separate-function form
  rv_eccentric_anomalies(...)              Kepler's equation only, every (planet, system, time)
  RaggedPlan(...)                          CSR batches, persistent kernel + HIP graph
  DEMC(...)                                population sampler (DE-MC) on the batched chi-square
  astro_model / astro_chisq                astrometric Keplerian model (Thiele-Innes form)
  RVChiSq.apply(...)                       torch.autograd.Function over rv_chisq_grad
Parameter planes are float64 CUDA tensors shaped (n_pl, n_sys) (system index
fastest); observations are 1-D float64 CUDA tensors.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkepler.so")

KEP_FP64, KEP_MIXED = 0, 1
KEP_MAX_PL = 8
_PREC = {"fp64": KEP_FP64, "f64": KEP_FP64, "double": KEP_FP64, "mixed": KEP_MIXED}
_STATUS = {0: "KEP_OK", 1: "KEP_ERR_ARG", 2: "KEP_ERR_SHAPE", 3: "KEP_ERR_DEVICE", 4: "KEP_ERR_LAUNCH",
           5: "KEP_ERR_UNSUPPORTED"}

_D = ctypes.c_void_p


class KepObs(ctypes.Structure):
    _fields_ = [("t", _D), ("v", _D), ("sigma", _D), ("n_obs", ctypes.c_int64), ("t0", ctypes.c_double)]


class KepParams(ctypes.Structure):
    _fields_ = [("P", _D), ("K", _D), ("e", _D), ("omega", _D), ("M0", _D), ("offset", _D), ("jitter", _D),
                ("n_sys", ctypes.c_int64), ("n_pl", ctypes.c_int64)]


class KepOptions(ctypes.Structure):
    _fields_ = [("fixed_iter", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("block_threads", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32)]


class KepObsCSR(ctypes.Structure):
    _fields_ = [("t", _D), ("v", _D), ("sigma", _D), ("obs_off", _D), ("n_obs_total", ctypes.c_int64),
                ("t0", ctypes.c_double)]


class KepParamsCSR(ctypes.Structure):
    _fields_ = [("P", _D), ("K", _D), ("e", _D), ("omega", _D), ("M0", _D), ("pl_off", _D),
                ("offset", _D), ("jitter", _D), ("n_sys", ctypes.c_int64), ("n_pl_total", ctypes.c_int64)]


class KepPlanInfo(ctypes.Structure):
    _fields_ = [("n_sys", ctypes.c_int64), ("n_obs_total", ctypes.c_int64), ("n_pl_total", ctypes.c_int64),
                ("triples", ctypes.c_int64), ("block_threads", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("sys_per_batch", ctypes.c_int32), ("tuned", ctypes.c_int32), ("tuned_ms", ctypes.c_double),
                ("group_chunks", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class KepDemcState(ctypes.Structure):
    _fields_ = [("x", _D), ("chi2", _D), ("n_accept", _D), ("jitter", _D), ("n_half", ctypes.c_int64),
                ("n_pl", ctypes.c_int64)]


class KepDemcOptions(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("jump_every", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("eps", _D)]


class KepAstroObs(ctypes.Structure):
    _fields_ = [("t", _D), ("x", _D), ("y", _D), ("sigma_x", _D), ("sigma_y", _D), ("n_obs", ctypes.c_int64),
                ("t0", ctypes.c_double)]


class KepAstroParams(ctypes.Structure):
    _fields_ = [("P", _D), ("e", _D), ("M0", _D), ("A", _D), ("B", _D), ("F", _D), ("G", _D), ("x0", _D),
                ("y0", _D), ("n_sys", ctypes.c_int64), ("n_pl", ctypes.c_int64)]


class KeplerError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_LIB = None

EXPORTS = ("kepler_solve", "rv_model", "rv_chisq", "rv_chisq_grad", "rv_nll_grad", "rv_chisq_gn", "rv_planet_velocities",
           "rv_chisq_from_velocities", "rv_eccentric_anomalies", "kep_plan_ragged", "rv_chisq_ragged", "rv_chisq_ragged_direct",
           "rv_chisq_ragged_static", "kep_plan_get_info", "kep_plan_destroy", "demc_chisq", "demc_generations", "kep_plan_demc", "demc_run",
           "kep_demc_plan_destroy", "astro_model", "astro_chisq", "kep_last_error", "kep_abi_version")


def load_library(path: str = LIB_PATH):
    """Load libkepler.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_0812_2976_amd.build` "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    L.kepler_solve.argtypes = [_D, _D, _D, ctypes.c_int64, ctypes.c_int, P(KepOptions), _D]
    for name in ("rv_model", "rv_chisq"):
        getattr(L, name).argtypes = [P(KepObs), P(KepParams), _D, ctypes.c_int, P(KepOptions), _D]
    L.rv_chisq_grad.argtypes = [P(KepObs), P(KepParams), _D, _D, ctypes.c_int, P(KepOptions), _D]
    L.rv_nll_grad.argtypes = [P(KepObs), P(KepParams), _D, _D, ctypes.c_int, P(KepOptions), _D]
    L.rv_chisq_gn.argtypes = [P(KepObs), P(KepParams), _D, _D, _D, ctypes.c_int, P(KepOptions), _D]
    L.rv_planet_velocities.argtypes = [P(KepObs), P(KepParams), _D, P(KepOptions), _D]
    L.rv_chisq_from_velocities.argtypes = [P(KepObs), P(KepParams), _D, _D, P(KepOptions), _D]
    L.rv_eccentric_anomalies.argtypes = [P(KepObs), P(KepParams), _D, P(KepOptions), _D]
    L.kep_plan_ragged.argtypes = [P(KepObsCSR), P(KepParamsCSR), ctypes.c_int, P(KepOptions), _D, P(_D)]
    L.rv_chisq_ragged.argtypes = [_D, _D, _D]
    L.rv_chisq_ragged_direct.argtypes = [_D, _D, _D]
    L.rv_chisq_ragged_static.argtypes = [P(KepObsCSR), P(KepParamsCSR), _D, ctypes.c_int, P(KepOptions), _D]
    L.kep_plan_get_info.argtypes = [_D, P(KepPlanInfo)]
    L.kep_plan_destroy.argtypes = [_D]
    L.kep_plan_destroy.restype = None
    L.demc_chisq.argtypes = [P(KepObs), P(KepDemcState), ctypes.c_int, P(KepOptions), _D]
    L.demc_generations.argtypes = [P(KepObs), P(KepDemcState), P(KepDemcOptions), ctypes.c_uint64, ctypes.c_int64,
                                   _D, ctypes.c_int, P(KepOptions), _D]
    L.kep_plan_demc.argtypes = [P(KepObs), P(KepDemcState), P(KepDemcOptions), _D, ctypes.c_int, P(KepOptions), _D,
                                P(_D)]
    L.demc_run.argtypes = [_D, ctypes.c_uint64, ctypes.c_int64, _D]
    L.kep_demc_plan_destroy.argtypes = [_D]
    L.kep_demc_plan_destroy.restype = None
    for name in ("astro_model", "astro_chisq"):
        getattr(L, name).argtypes = [P(KepAstroObs), P(KepAstroParams), _D, ctypes.c_int, P(KepOptions), _D]
    L.kep_last_error.restype = ctypes.c_char_p
    L.kep_last_error.argtypes = []
    L.kep_abi_version.restype = ctypes.c_int
    for name in ("kepler_solve", "rv_model", "rv_chisq", "rv_chisq_grad", "rv_nll_grad", "rv_chisq_gn",
                 "rv_planet_velocities", "rv_chisq_from_velocities", "rv_eccentric_anomalies", "kep_plan_ragged",
                 "rv_chisq_ragged", "rv_chisq_ragged_direct", "rv_chisq_ragged_static",
                 "kep_plan_get_info", "demc_chisq", "demc_generations", "kep_plan_demc", "demc_run",
                 "astro_model", "astro_chisq"):
        getattr(L, name).restype = ctypes.c_int
    _LIB = L
    return L


def _check(status):
    if status != 0:
        raise KeplerError(status, load_library().kep_last_error().decode())


def _prec(prec):
    if isinstance(prec, int):
        return prec
    try:
        return _PREC[prec]
    except KeyError:
        raise ValueError(f"unknown precision {prec!r}; use 'fp64' or 'mixed'") from None


def _opts(opts):
    if opts is None:
        return None
    if isinstance(opts, KepOptions):
        return ctypes.byref(opts)
    o = KepOptions(int(opts.get("fixed_iter", 0)), int(opts.get("max_iter", 0)),
                   int(opts.get("block_threads", 0)), int(opts.get("blocks_per_cu", 0)))
    return ctypes.byref(o)


def _dev(x, name, ndim=None, dtype=torch.float64):
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if not x.is_cuda:
        raise ValueError(f"{name} must be on the GPU (got {x.device}); there is no CPU path")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {x.dtype})")
    if ndim is not None and x.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions (got shape {tuple(x.shape)})")
    return x.contiguous()


def _opt_dev(x, name, n):
    if x is None:
        return None
    x = _dev(x, name, 1)
    if x.numel() != n:
        raise ValueError(f"{name} must have n_sys = {n} elements")
    return x


def _out(x, name, shape, device, dtype=torch.float64):
    """A result tensor: allocated when None, else checked to be a contiguous GPU
    tensor of exactly `shape` (the kernels write through its pointer)."""
    shape = tuple(int(n) for n in shape)
    if x is None:
        return torch.empty(shape, dtype=dtype, device=device)
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if x.dtype != dtype or tuple(x.shape) != shape or not x.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape {shape} "
                         f"(got {x.dtype} {tuple(x.shape)})")
    if x.device != torch.device(device):
        raise ValueError(f"{name} must be on {device} (got {x.device})")
    return x


def _ptr(x):
    return None if x is None else x.data_ptr()


def _stream(device):
    return torch.cuda.current_stream(device).cuda_stream


def _planes(P, K, e, omega, M0):
    planes = [_dev(x, n, 2) for x, n in zip((P, K, e, omega, M0), ("P", "K", "e", "omega", "M0"))]
    shape = planes[0].shape
    for x in planes:
        if x.shape != shape:
            raise ValueError("P, K, e, omega, M0 must share the shape (n_pl, n_sys)")
    return planes


def kepler_solve(M, e, prec="mixed", out=None, opts=None):
    """E with E - e sin E = M, elementwise (Eq. 1)."""
    M = _dev(M, "M")
    e = _dev(e, "e")
    if M.shape != e.shape:
        raise ValueError("M and e must have the same shape")
    out = _out(out, "out", M.shape, M.device)
    L = load_library()
    _check(L.kepler_solve(M.data_ptr(), e.data_ptr(), out.data_ptr(), M.numel(), _prec(prec), _opts(opts),
                          _stream(M.device)))
    return out


def _obs_params(t, v, sigma, P, K, e, omega, M0, offset, jitter, t0):
    P, K, e, omega, M0 = _planes(P, K, e, omega, M0)
    n_pl, n_sys = P.shape
    t = _dev(t, "t", 1)
    v = None if v is None else _dev(v, "v", 1)
    sigma = None if sigma is None else _dev(sigma, "sigma", 1)
    for x, nm in ((v, "v"), (sigma, "sigma")):
        if x is not None and x.numel() != t.numel():
            raise ValueError(f"{nm} must have n_obs = {t.numel()} elements")
    offset = _opt_dev(offset, "offset", n_sys)
    jitter = _opt_dev(jitter, "jitter", n_sys)
    obs = KepObs(t.data_ptr(), _ptr(v), _ptr(sigma), t.numel(), float(t0))
    par = KepParams(P.data_ptr(), K.data_ptr(), e.data_ptr(), omega.data_ptr(), M0.data_ptr(), _ptr(offset),
                    _ptr(jitter), n_sys, n_pl)
    keep = (t, v, sigma, P, K, e, omega, M0, offset, jitter)
    return obs, par, keep, t.device


def rv_model(t, P, K, e, omega, M0, offset=None, t0=0.0, prec="mixed", out=None, opts=None):
    """Model velocities (n_sys, n_obs): sum over planets of the Keplerian velocity plus offset."""
    obs, par, keep, dev = _obs_params(t, None, None, P, K, e, omega, M0, offset, None, t0)
    out = _out(out, "out", (par.n_sys, obs.n_obs), dev)
    L = load_library()
    _check(L.rv_model(ctypes.byref(obs), ctypes.byref(par), out.data_ptr(), _prec(prec), _opts(opts), _stream(dev)))
    return out


def rv_chisq(t, v, sigma, P, K, e, omega, M0, offset=None, jitter=None, t0=0.0, prec="mixed", out=None, opts=None):
    """chi-square per system (Eq. 5), shape (n_sys,).

    P, K, e, omega, M0 are planes of shape (n_pl, n_sys). Parameters held
    system-major, (n_sys, n_pl), are passed as their transposed views (`P.T`); every
    entry point copies a non-contiguous argument into a contiguous plane first."""
    obs, par, keep, dev = _obs_params(t, v, sigma, P, K, e, omega, M0, offset, jitter, t0)
    out = _out(out, "out", (par.n_sys,), dev)
    L = load_library()
    _check(L.rv_chisq(ctypes.byref(obs), ctypes.byref(par), out.data_ptr(), _prec(prec), _opts(opts), _stream(dev)))
    return out


def rv_chisq_grad(t, v, sigma, P, K, e, omega, M0, offset=None, jitter=None, t0=0.0, prec="mixed",
                  out=None, grad=None, opts=None):
    """(chi2 (n_sys,), grad (5 n_pl + 1, n_sys)); rows P, K, e, omega, M0 per planet, then offset."""
    obs, par, keep, dev = _obs_params(t, v, sigma, P, K, e, omega, M0, offset, jitter, t0)
    out = _out(out, "out", (par.n_sys,), dev)
    grad = _out(grad, "grad", (5 * par.n_pl + 1, par.n_sys), dev)
    L = load_library()
    _check(L.rv_chisq_grad(ctypes.byref(obs), ctypes.byref(par), out.data_ptr(), grad.data_ptr(), _prec(prec),
                           _opts(opts), _stream(dev)))
    return out, grad


def rv_nll_grad(t, v, sigma, P, K, e, omega, M0, offset=None, jitter=None, t0=0.0, prec="mixed",
                out=None, grad=None, opts=None):
    """(nll (n_sys,), grad (5 n_pl + 2, n_sys)): nll = chi2 + sum_k ln(sigma_k^2 + s^2)
    (= -2 ln L without the n_obs ln 2 pi constant); rows P, K, e, omega, M0 per
    planet, then offset, then jitter."""
    obs, par, keep, dev = _obs_params(t, v, sigma, P, K, e, omega, M0, offset, jitter, t0)
    out = _out(out, "out", (par.n_sys,), dev)
    grad = _out(grad, "grad", (5 * par.n_pl + 2, par.n_sys), dev)
    L = load_library()
    _check(L.rv_nll_grad(ctypes.byref(obs), ctypes.byref(par), out.data_ptr(), grad.data_ptr(), _prec(prec),
                         _opts(opts), _stream(dev)))
    return out, grad


def rv_chisq_gn(t, v, sigma, P, K, e, omega, M0, offset=None, jitter=None, t0=0.0, prec="mixed", out=None,
                jtwr=None, jtwj=None, opts=None):
    """Gauss-Newton products: (chi2 (n_sys,), J^T W r (np, n_sys), J^T W J packed upper
    triangle (np (np + 1) / 2, n_sys)), np = 5 n_pl + 1, entry (a, b), a <= b, at row
    a np - a (a - 1) / 2 + (b - a)."""
    obs, par, keep, dev = _obs_params(t, v, sigma, P, K, e, omega, M0, offset, jitter, t0)
    npar = 5 * par.n_pl + 1
    out = _out(out, "out", (par.n_sys,), dev)
    jtwr = _out(jtwr, "jtwr", (npar, par.n_sys), dev)
    jtwj = _out(jtwj, "jtwj", (npar * (npar + 1) // 2, par.n_sys), dev)
    _check(load_library().rv_chisq_gn(ctypes.byref(obs), ctypes.byref(par), out.data_ptr(), jtwr.data_ptr(),
                                      jtwj.data_ptr(), _prec(prec), _opts(opts), _stream(dev)))
    return out, jtwr, jtwj


def rv_planet_velocities(t, P, K, e, omega, M0, t0=0.0, out=None, opts=None):
    """Every planet's velocity (n_pl, n_sys, n_obs) in binary32, mixed precision
    (first kernel of the paper's separate-function form)."""
    obs, par, keep, dev = _obs_params(t, None, None, P, K, e, omega, M0, None, None, t0)
    out = _out(out, "out", (par.n_pl, par.n_sys, obs.n_obs), dev, torch.float32)
    _check(load_library().rv_planet_velocities(ctypes.byref(obs), ctypes.byref(par), out.data_ptr(), _opts(opts),
                                               _stream(dev)))
    return out


def rv_eccentric_anomalies(t, P, K, e, omega, M0, t0=0.0, out=None, opts=None):
    """Every planet's eccentric anomaly (n_pl, n_sys, n_obs) in binary32, in [-pi, pi]
    (Kepler's equation only, mixed precision)."""
    obs, par, keep, dev = _obs_params(t, None, None, P, K, e, omega, M0, None, None, t0)
    out = _out(out, "out", (par.n_pl, par.n_sys, obs.n_obs), dev, torch.float32)
    _check(load_library().rv_eccentric_anomalies(ctypes.byref(obs), ctypes.byref(par), out.data_ptr(), _opts(opts),
                                                 _stream(dev)))
    return out


def rv_chisq_from_velocities(t, v, sigma, dv, offset=None, jitter=None, t0=0.0, out=None, opts=None):
    """chi-square per system from per-planet velocities dv (n_pl, n_sys, n_obs) binary32
    (second kernel of the separate-function form)."""
    dv = _dev(dv, "dv", 3, torch.float32)
    n_pl, n_sys, n_obs = dv.shape
    t, v, sigma = (_dev(x, n, 1) for x, n in ((t, "t"), (v, "v"), (sigma, "sigma")))
    if t.numel() != n_obs or v.numel() != n_obs or sigma.numel() != n_obs:
        raise ValueError("t, v, sigma must have n_obs elements")
    offset = _opt_dev(offset, "offset", n_sys)
    jitter = _opt_dev(jitter, "jitter", n_sys)
    obs = KepObs(t.data_ptr(), v.data_ptr(), sigma.data_ptr(), n_obs, float(t0))
    par = KepParams(None, None, None, None, None, _ptr(offset), _ptr(jitter), n_sys, n_pl)
    out = _out(out, "out", (n_sys,), dv.device)
    _check(load_library().rv_chisq_from_velocities(ctypes.byref(obs), ctypes.byref(par), dv.data_ptr(),
                                                   out.data_ptr(), _opts(opts), _stream(dv.device)))
    return out


def _astro(t, x, y, sigma_x, sigma_y, P, e, M0, A, B, F, G, x0, y0, t0):
    planes = [_dev(a, n, 2) for a, n in zip((P, e, M0, A, B, F, G), ("P", "e", "M0", "A", "B", "F", "G"))]
    shape = planes[0].shape
    if any(p.shape != shape for p in planes):
        raise ValueError("P, e, M0, A, B, F, G must share the shape (n_pl, n_sys)")
    n_pl, n_sys = shape
    t = _dev(t, "t", 1)
    obs_arrays = []
    for arr, nm in ((x, "x"), (y, "y"), (sigma_x, "sigma_x"), (sigma_y, "sigma_y")):
        arr = None if arr is None else _dev(arr, nm, 1)
        if arr is not None and arr.numel() != t.numel():
            raise ValueError(f"{nm} must have n_obs = {t.numel()} elements")
        obs_arrays.append(arr)
    x0 = _opt_dev(x0, "x0", n_sys)
    y0 = _opt_dev(y0, "y0", n_sys)
    obs = KepAstroObs(t.data_ptr(), *[_ptr(a) for a in obs_arrays], t.numel(), float(t0))
    par = KepAstroParams(*[p.data_ptr() for p in planes], _ptr(x0), _ptr(y0), n_sys, n_pl)
    return obs, par, (t, obs_arrays, planes, x0, y0), t.device


def astro_model(t, P, e, M0, A, B, F, G, x0=None, y0=None, t0=0.0, prec="mixed", out=None, opts=None):
    """Astrometric model offsets (n_sys, 2, n_obs): row 0 dRA* = B X + G Y (+ x0), row 1
    dDec = A X + F Y (+ y0), X = cos E - e, Y = sqrt(1 - e^2) sin E."""
    obs, par, keep, dev = _astro(t, None, None, None, None, P, e, M0, A, B, F, G, x0, y0, t0)
    out = _out(out, "out", (par.n_sys, 2, obs.n_obs), dev)
    _check(load_library().astro_model(ctypes.byref(obs), ctypes.byref(par), out.data_ptr(), _prec(prec),
                                      _opts(opts), _stream(dev)))
    return out


def astro_chisq(t, x, y, sigma_x, sigma_y, P, e, M0, A, B, F, G, x0=None, y0=None, t0=0.0, prec="mixed",
                out=None, opts=None):
    """chi-square per system of the astrometric model against offsets (x, y)."""
    obs, par, keep, dev = _astro(t, x, y, sigma_x, sigma_y, P, e, M0, A, B, F, G, x0, y0, t0)
    out = _out(out, "out", (par.n_sys,), dev)
    _check(load_library().astro_chisq(ctypes.byref(obs), ctypes.byref(par), out.data_ptr(), _prec(prec),
                                      _opts(opts), _stream(dev)))
    return out


class RaggedPlan:
    """Plan for a CSR batch (one persistent kernel replayed from a HIP graph).
    Holds references to the input tensors, whose addresses the plan keeps."""

    def __init__(self, t, v, sigma, obs_off, P, K, e, omega, M0, pl_off, offset=None, jitter=None, t0=0.0,
                 prec="mixed", opts=None):
        self.t, self.v, self.sigma = (_dev(x, n, 1) for x, n in ((t, "t"), (v, "v"), (sigma, "sigma")))
        self.obs_off = _dev(obs_off, "obs_off", 1, torch.int64)
        self.pl_off = _dev(pl_off, "pl_off", 1, torch.int64)
        self.P, self.K, self.e, self.omega, self.M0 = (_dev(x, n, 1) for x, n in
                                                      ((P, "P"), (K, "K"), (e, "e"), (omega, "omega"), (M0, "M0")))
        self.n_sys = self.obs_off.numel() - 1
        self.offset = _opt_dev(offset, "offset", self.n_sys)
        self.jitter = _opt_dev(jitter, "jitter", self.n_sys)
        self.device = self.t.device
        obs = KepObsCSR(self.t.data_ptr(), self.v.data_ptr(), self.sigma.data_ptr(), self.obs_off.data_ptr(),
                        self.t.numel(), float(t0))
        par = KepParamsCSR(self.P.data_ptr(), self.K.data_ptr(), self.e.data_ptr(), self.omega.data_ptr(),
                           self.M0.data_ptr(), self.pl_off.data_ptr(), _ptr(self.offset), _ptr(self.jitter),
                           self.n_sys, self.P.numel())
        L = load_library()
        h = ctypes.c_void_p()
        _check(L.kep_plan_ragged(ctypes.byref(obs), ctypes.byref(par), _prec(prec), _opts(opts),
                                 _stream(self.device), ctypes.byref(h)))
        self._h = h

    def __call__(self, out=None):
        """chi-square per system through the plan's HIP graph."""
        out = _out(out, "out", (self.n_sys,), self.device)
        _check(load_library().rv_chisq_ragged(self._h, out.data_ptr(), _stream(self.device)))
        return out

    def direct(self, out=None):
        """Same computation launched directly (no graph)."""
        out = _out(out, "out", (self.n_sys,), self.device)
        _check(load_library().rv_chisq_ragged_direct(self._h, out.data_ptr(), _stream(self.device)))
        return out

    def info(self):
        i = KepPlanInfo()
        _check(load_library().kep_plan_get_info(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in KepPlanInfo._fields_}

    def close(self):
        if getattr(self, "_h", None):
            torch.cuda.synchronize(self.device)        # no replay of the plan's graph may still be running
            load_library().kep_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rv_chisq_ragged_static(t, v, sigma, obs_off, P, K, e, omega, M0, pl_off, offset=None, jitter=None, t0=0.0,
                           prec="mixed", out=None, opts=None):
    """chi-square of a CSR batch in one call without a plan and without any
    device allocation by the library (the offsets are checked and the systems
    ordered on the device, in the library's static work area); n_sys <= 2^21.
    Calls that overlap in time on one GPU must not be made.  prec="fp64" runs
    the binary64 kernel, which uses no work area (no size limit, no sharing)."""
    t, v, sigma = (_dev(x, n, 1) for x, n in ((t, "t"), (v, "v"), (sigma, "sigma")))
    obs_off = _dev(obs_off, "obs_off", 1, torch.int64)
    pl_off = _dev(pl_off, "pl_off", 1, torch.int64)
    P, K, e, omega, M0 = (_dev(x, n, 1) for x, n in ((P, "P"), (K, "K"), (e, "e"), (omega, "omega"), (M0, "M0")))
    n_sys = obs_off.numel() - 1
    if pl_off.numel() != n_sys + 1:
        raise ValueError("obs_off and pl_off must have the same length")
    offset = _opt_dev(offset, "offset", n_sys)
    jitter = _opt_dev(jitter, "jitter", n_sys)
    dev = t.device
    out = _out(out, "out", (n_sys,), dev)
    obs = KepObsCSR(t.data_ptr(), v.data_ptr(), sigma.data_ptr(), obs_off.data_ptr(), t.numel(), float(t0))
    par = KepParamsCSR(P.data_ptr(), K.data_ptr(), e.data_ptr(), omega.data_ptr(), M0.data_ptr(), pl_off.data_ptr(),
                       _ptr(offset), _ptr(jitter), n_sys, P.numel())
    _check(load_library().rv_chisq_ragged_static(ctypes.byref(obs), ctypes.byref(par), out.data_ptr(), _prec(prec),
                                                 _opts(opts), _stream(dev)))
    return out


class DEMC:
    """Population sampler: differential-evolution MCMC (ter Braak 2006) over
    exp(-chi2/2), the many-chain application the batched chi-square serves
    (Sec. 6).  The population x is a float64 GPU tensor (2, 5 n_pl + 1, n_half):
    two halves, each a set of parameter planes P[n_pl], K, e, omega, M0, then
    the offset row.  x, chi2 (2, n_half) and n_accept (2, n_half) live on the
    GPU and are updated in place; generations are reproducible from
    (seed, generation) and identical whether launched directly
    (generations) or from the recorded HIP graph (run)."""

    def __init__(self, t, v, sigma, x, eps, seed, t0=0.0, jitter=None, gamma=0.0, jump_every=0, prec="mixed",
                 opts=None):
        self.t, self.v, self.sigma = (_dev(a, n, 1) for a, n in ((t, "t"), (v, "v"), (sigma, "sigma")))
        if not (self.t.numel() == self.v.numel() == self.sigma.numel()):
            raise ValueError("t, v, sigma must have the same length")
        self.x = _dev(x, "x", 3)
        two, d, nh = self.x.shape
        if two != 2 or d < 6 or (d - 1) % 5 != 0:
            raise ValueError("x must have shape (2, 5 n_pl + 1, n_half)")
        self.n_pl, self.n_half, self.d = (d - 1) // 5, nh, d
        self.device = self.x.device
        self.eps = _dev(eps, "eps", 1)
        if self.eps.numel() != d:
            raise ValueError(f"eps must have d = {d} elements")
        self.jitter = None if jitter is None else _dev(jitter, "jitter", 2)
        if self.jitter is not None and tuple(self.jitter.shape) != (2, nh):
            raise ValueError(f"jitter must have shape (2, {nh})")
        self.chi2 = torch.empty((2, nh), dtype=torch.float64, device=self.device)
        self.n_accept = torch.zeros((2, nh), dtype=torch.int64, device=self.device)
        self.work = torch.empty((d + 1) * nh, dtype=torch.float64, device=self.device)
        self.prec, self.opts = prec, opts
        self._obs = KepObs(self.t.data_ptr(), self.v.data_ptr(), self.sigma.data_ptr(), self.t.numel(), float(t0))
        self._state = KepDemcState(self.x.data_ptr(), self.chi2.data_ptr(), self.n_accept.data_ptr(),
                                   _ptr(self.jitter), nh, self.n_pl)
        self._dopt = KepDemcOptions(float(gamma), int(jump_every), 0, int(seed) & (2 ** 64 - 1),
                                    self.eps.data_ptr())
        self._plan = None
        self.chisq()

    def chisq(self):
        """(Re)compute chi2 of the current population (NaN where a K < 0)."""
        _check(load_library().demc_chisq(ctypes.byref(self._obs), ctypes.byref(self._state), _prec(self.prec),
                                         _opts(self.opts), _stream(self.device)))
        return self.chi2

    def generations(self, gen0, n_gen):
        """Generations gen0 .. gen0 + n_gen - 1, launched directly."""
        _check(load_library().demc_generations(ctypes.byref(self._obs), ctypes.byref(self._state),
                                               ctypes.byref(self._dopt), int(gen0), int(n_gen),
                                               self.work.data_ptr(), _prec(self.prec), _opts(self.opts),
                                               _stream(self.device)))

    def run(self, gen0, n_gen):
        """The same generations replayed from the recorded HIP graph."""
        L = load_library()
        if self._plan is None:
            h = ctypes.c_void_p()
            _check(L.kep_plan_demc(ctypes.byref(self._obs), ctypes.byref(self._state), ctypes.byref(self._dopt),
                                   self.work.data_ptr(), _prec(self.prec), _opts(self.opts), _stream(self.device),
                                   ctypes.byref(h)))
            self._plan = h
        _check(L.demc_run(self._plan, int(gen0), int(n_gen), _stream(self.device)))

    def close(self):
        if getattr(self, "_plan", None):
            torch.cuda.synchronize(self.device)
            load_library().kep_demc_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RVChiSq(torch.autograd.Function):
    """chi-square per system with a backward pass from the implicit-function
    adjoint kernel (rv_chisq_grad); the forward computes both in one launch.
    Differentiable inputs: P, K, e, omega, M0 (n_pl, n_sys) and offset (n_sys,)."""

    @staticmethod
    def forward(ctx, P, K, e, omega, M0, offset, t, v, sigma, jitter=None, t0=0.0, prec="mixed"):
        chi2, grad = rv_chisq_grad(t, v, sigma, P, K, e, omega, M0, offset, jitter, t0, prec)
        ctx.save_for_backward(grad)
        ctx.n_pl = P.shape[0]
        return chi2

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        n_pl = ctx.n_pl
        need = ctx.needs_input_grad
        gp = grad[:5 * n_pl].view(n_pl, 5, -1) * g[None, None, :]
        d = [gp[:, i, :] if need[i] else None for i in range(5)]
        doff = grad[5 * n_pl] * g if need[5] else None     # None also when offset was None
        return d[0], d[1], d[2], d[3], d[4], doff, None, None, None, None, None, None
