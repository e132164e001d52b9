"""CPU oracle for batched Keplerian radial-velocity chi-square — TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports, links or
calls it, and it shares no code with the GPU library.

The arithmetic lives in ``kepler_oracle.c`` (plain C, binary64 inputs, long
double internals); this module only marshals numpy arrays into it.  Functions
follow the paper (Ford 2008) section by section:

* ``kepler``        — root of Kepler's equation M = E - e sin E (Eq. 1, Sec. 4.3)
* ``mean_anomaly``  — Eq. 4 / Eq. 6 with the binary64 bracket of Sec. 5.1
* ``planet_rv``     — one planet's Keplerian velocity (Eq. 3, standard form)
* ``rv_model``      — planet sum plus offset (Eq. 2)
* ``chisq``         — Eq. 5 with per-system jitter
* ``chisq_grad``    — analytic gradient of Eq. 5 (partial derivatives, Sec. 6)
* ``nll_grad``      — likelihood with jitter (Eq. 5's weights) and its gradient
* ``chisq_ragged``  — Eq. 5 over CSR-packed systems of uneven size
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)


class _Dense(ctypes.Structure):
    _fields_ = [("t", _D), ("v", _D), ("sigma", _D), ("n_obs", ctypes.c_int64),
                ("t0", ctypes.c_double),
                ("P", _D), ("K", _D), ("e", _D), ("w", _D), ("M0", _D),
                ("offset", _D), ("jitter", _D),
                ("n_sys", ctypes.c_int64), ("n_pl", ctypes.c_int64)]


class _Ragged(ctypes.Structure):
    _fields_ = [("t", _D), ("v", _D), ("sigma", _D), ("obs_off", _I64),
                ("t0", ctypes.c_double),
                ("P", _D), ("K", _D), ("e", _D), ("w", _D), ("M0", _D),
                ("pl_off", _I64), ("offset", _D), ("jitter", _D),
                ("n_sys", ctypes.c_int64)]


class _Demc(ctypes.Structure):
    _fields_ = [("t", _D), ("v", _D), ("sigma", _D), ("n_obs", ctypes.c_int64), ("t0", ctypes.c_double),
                ("x", _D), ("chi2", _D), ("n_accept", _I64), ("jitter", _D),
                ("n_half", ctypes.c_int64), ("n_pl", ctypes.c_int64),
                ("gamma", ctypes.c_double), ("jump_every", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("eps", _D), ("margin", _D)]


class _Astro(ctypes.Structure):
    _fields_ = [("t", _D), ("x", _D), ("y", _D), ("sx", _D), ("sy", _D), ("n_obs", ctypes.c_int64),
                ("t0", ctypes.c_double), ("P", _D), ("e", _D), ("M0", _D), ("A", _D), ("B", _D), ("F", _D),
                ("G", _D), ("x0", _D), ("y0", _D), ("n_sys", ctypes.c_int64), ("n_pl", ctypes.c_int64)]


def lib():
    """Load (building first if nothing is built) the oracle shared library."""
    global _LIB
    if _LIB is None:
        path = os.environ.get("KEP_ORACLE_LIB")     # a deliberately broken copy (mutation tests)
        if path is None:
            path = _build.LIB
            if not os.path.exists(path):
                _build.build()
        L = ctypes.CDLL(path)
        L.oracle_kepler.restype = ctypes.c_double
        L.oracle_kepler.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_kepler_batch.restype = None
        L.oracle_kepler_batch.argtypes = [_D, _D, _D, ctypes.c_int64]
        L.oracle_mean_anomaly.restype = ctypes.c_double
        L.oracle_mean_anomaly.argtypes = [ctypes.c_double] * 4
        L.oracle_planet_rv.restype = ctypes.c_double
        L.oracle_planet_rv.argtypes = [ctypes.c_double] * 7
        for name in ("oracle_rv_model", "oracle_chisq"):
            f = getattr(L, name)
            f.restype = None
            f.argtypes = [ctypes.POINTER(_Dense), _D, ctypes.c_int64, ctypes.c_int64]
        L.oracle_chisq_grad.restype = None
        L.oracle_chisq_grad.argtypes = [ctypes.POINTER(_Dense), _D, _D, ctypes.c_int64, ctypes.c_int64]
        L.oracle_gn.restype = None
        L.oracle_gn.argtypes = [ctypes.POINTER(_Dense), _D, _D, _D, ctypes.c_int64, ctypes.c_int64]
        L.oracle_nll_grad.restype = None
        L.oracle_nll_grad.argtypes = [ctypes.POINTER(_Dense), _D, _D, ctypes.c_int64, ctypes.c_int64]
        L.oracle_chisq_grad_scales.restype = None
        L.oracle_chisq_grad_scales.argtypes = [ctypes.POINTER(_Dense), _D, _D, _D, _D, ctypes.c_int64, ctypes.c_int64]
        L.oracle_chisq_ragged.restype = None
        L.oracle_chisq_ragged.argtypes = [ctypes.POINTER(_Ragged), _D, ctypes.c_int64, ctypes.c_int64]
        _U32 = ctypes.POINTER(ctypes.c_uint32)
        L.oracle_philox4x32_10.restype = None
        L.oracle_philox4x32_10.argtypes = [_U32, _U32, _U32]
        for fn in ("oracle_astro_model", "oracle_astro_chisq"):
            getattr(L, fn).restype = None
            getattr(L, fn).argtypes = [ctypes.POINTER(_Astro), _D, ctypes.c_int64, ctypes.c_int64]
        L.oracle_demc_run.restype = None
        L.oracle_demc_run.argtypes = [ctypes.POINTER(_Demc), ctypes.c_uint64, ctypes.c_int64]
        _LIB = L
    return _LIB


def _f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_D)


def kepler(M, e):
    """E with E - e sin E = M for every pair (Eq. 1); NaN outside e in [0, 1)."""
    M, e = np.broadcast_arrays(_f64(M), _f64(e))
    M, e = _f64(M), _f64(e)
    out = np.empty_like(M)
    lib().oracle_kepler_batch(_ptr(M), _ptr(e), _ptr(out), M.size)
    return out


def mean_anomaly(t, t0, P, M0):
    """M in [0, 2 pi) for scalars (Eq. 4 with the binary64 bracket of Eq. 6)."""
    return lib().oracle_mean_anomaly(float(t), float(t0), float(P), float(M0))


def planet_rv(t, t0, P, K, e, w, M0):
    """Velocity of one planet at time t (scalars)."""
    return lib().oracle_planet_rv(float(t), float(t0), float(P), float(K), float(e), float(w), float(M0))


class Dense:
    """Dense batch: observations [n_obs] shared by all systems, parameter
    planes [n_pl, n_sys] (system index fastest), optional offset/jitter [n_sys]."""

    def __init__(self, t, v, sigma, P, K, e, w, M0, offset=None, jitter=None, t0=0.0):
        self.t, self.v, self.sigma = _f64(t), _f64(v), _f64(sigma)
        planes = [np.atleast_2d(_f64(x)) for x in (P, K, e, w, M0)]
        self.P, self.K, self.e, self.w, self.M0 = [_f64(x) for x in planes]
        self.n_pl, self.n_sys = self.P.shape
        self.offset = None if offset is None else _f64(offset)
        self.jitter = None if jitter is None else _f64(jitter)
        self.t0 = float(t0)
        self._s = _Dense(_ptr(self.t), _ptr(self.v), _ptr(self.sigma), self.t.size, self.t0,
                         _ptr(self.P), _ptr(self.K), _ptr(self.e), _ptr(self.w), _ptr(self.M0),
                         _ptr(self.offset), _ptr(self.jitter), self.n_sys, self.n_pl)

    def _range(self, i0, i1):
        i1 = self.n_sys if i1 is None else i1
        if not (0 <= i0 <= i1 <= self.n_sys):
            raise ValueError("bad system range")
        return i0, i1


def rv_model(d: Dense, i0=0, i1=None):
    """Model velocity [n_sys, n_obs] (Eq. 2 plus offset); rows outside [i0, i1) are NaN."""
    i0, i1 = d._range(i0, i1)
    out = np.full((d.n_sys, d.t.size), np.nan)
    lib().oracle_rv_model(ctypes.byref(d._s), _ptr(out), i0, i1)
    return out


def chisq(d: Dense, i0=0, i1=None, out=None):
    """chi-square per system (Eq. 5); entries outside [i0, i1) are left untouched."""
    i0, i1 = d._range(i0, i1)
    if out is None:
        out = np.full(d.n_sys, np.nan)
    lib().oracle_chisq(ctypes.byref(d._s), _ptr(out), i0, i1)
    return out


def chisq_grad(d: Dense, i0=0, i1=None):
    """(chi2 [n_sys], grad [5*n_pl+1, n_sys]); gradient rows are P,K,e,omega,M0 per planet, then offset."""
    i0, i1 = d._range(i0, i1)
    chi2 = np.full(d.n_sys, np.nan)
    grad = np.full((5 * d.n_pl + 1, d.n_sys), np.nan)
    lib().oracle_chisq_grad(ctypes.byref(d._s), _ptr(chi2), _ptr(grad), i0, i1)
    return chi2, grad


def nll_grad(d: Dense, i0=0, i1=None):
    """(-2 ln L [n_sys], grad [5*n_pl+2, n_sys]): Gaussian likelihood with jitter,
    -2 ln L = chi2 + sum_k ln(sigma_k^2 + s^2) (constant omitted); gradient rows
    as chisq_grad, then d/ds."""
    i0, i1 = d._range(i0, i1)
    nll = np.full(d.n_sys, np.nan)
    grad = np.full((5 * d.n_pl + 2, d.n_sys), np.nan)
    lib().oracle_nll_grad(ctypes.byref(d._s), _ptr(nll), _ptr(grad), i0, i1)
    return nll, grad


def gn(d: Dense, i0=0, i1=None):
    """Gauss-Newton products: (chi2 [n_sys], jtwr [np, n_sys], jtwj [np (np + 1) / 2, n_sys])
    with np = 5 n_pl + 1; jtwj packed upper triangle, (a, b), a <= b, at
    a np - a (a - 1) / 2 + (b - a)."""
    i0, i1 = d._range(i0, i1)
    np_ = 5 * d.n_pl + 1
    chi2 = np.full(d.n_sys, np.nan)
    jtwr = np.full((np_, d.n_sys), np.nan)
    jtwj = np.full((np_ * (np_ + 1) // 2, d.n_sys), np.nan)
    lib().oracle_gn(ctypes.byref(d._s), _ptr(chi2), _ptr(jtwr), _ptr(jtwj), i0, i1)
    return chi2, jtwr, jtwj


def unpack_sym(packed, n):
    """[n (n + 1) / 2, ...] packed upper triangle -> [n, n, ...] symmetric."""
    out = np.empty((n, n) + packed.shape[1:])
    idx = 0
    for a in range(n):
        for b in range(a, n):
            out[a, b] = out[b, a] = packed[idx]
            idx += 1
    return out


def chisq_grad_scales(d: Dense, i0=0, i1=None):
    """(chi2, grad, scale_r, scale_1): scale_r = sum_k |2 w r dv/dtheta|, scale_1 = sum_k 2 w |dv/dtheta|
    per gradient component; a residual error dr and a relative error eps per term change the gradient
    by at most dr * scale_1 + eps * scale_r."""
    i0, i1 = d._range(i0, i1)
    shp = (5 * d.n_pl + 1, d.n_sys)
    chi2 = np.full(d.n_sys, np.nan)
    grad, sr, s1 = np.full(shp, np.nan), np.full(shp, np.nan), np.full(shp, np.nan)
    lib().oracle_chisq_grad_scales(ctypes.byref(d._s), _ptr(chi2), _ptr(grad), _ptr(sr), _ptr(s1), i0, i1)
    return chi2, grad, sr, s1


class Ragged:
    """CSR batch: system i owns observations obs_off[i]:obs_off[i+1] and
    planets pl_off[i]:pl_off[i+1]."""

    def __init__(self, t, v, sigma, obs_off, P, K, e, w, M0, pl_off, offset=None, jitter=None, t0=0.0):
        self.t, self.v, self.sigma = _f64(t), _f64(v), _f64(sigma)
        self.obs_off = np.ascontiguousarray(obs_off, dtype=np.int64)
        self.pl_off = np.ascontiguousarray(pl_off, dtype=np.int64)
        self.P, self.K, self.e, self.w, self.M0 = [_f64(x) for x in (P, K, e, w, M0)]
        self.n_sys = self.obs_off.size - 1
        self.offset = None if offset is None else _f64(offset)
        self.jitter = None if jitter is None else _f64(jitter)
        self.t0 = float(t0)
        self._s = _Ragged(_ptr(self.t), _ptr(self.v), _ptr(self.sigma),
                          self.obs_off.ctypes.data_as(_I64), self.t0,
                          _ptr(self.P), _ptr(self.K), _ptr(self.e), _ptr(self.w), _ptr(self.M0),
                          self.pl_off.ctypes.data_as(_I64), _ptr(self.offset), _ptr(self.jitter),
                          self.n_sys)


def chisq_ragged(d: Ragged, i0=0, i1=None, out=None):
    """chi-square per CSR system (Eq. 5)."""
    i1 = d.n_sys if i1 is None else i1
    if out is None:
        out = np.full(d.n_sys, np.nan)
    lib().oracle_chisq_ragged(ctypes.byref(d._s), _ptr(out), i0, i1)
    return out


def philox4x32_10(ctr, key):
    """Philox-4x32-10 block (Salmon et al. 2011): four 32-bit words from a
    128-bit counter and a 64-bit key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    P32 = ctypes.POINTER(ctypes.c_uint32)
    lib().oracle_philox4x32_10(c.ctypes.data_as(P32), k.ctypes.data_as(P32), out.ctypes.data_as(P32))
    return out


def demc_init_chisq(t, v, sigma, x, n_pl, jitter=None, t0=0.0):
    """chi-square [2, n_half] of a population x [2, 5 n_pl + 1, n_half] (Eq. 5);
    NaN where a chain lies outside the prior support (K < 0 included)."""
    x = np.asarray(x, dtype=np.float64)
    nh = x.shape[2]
    out = np.empty((2, nh))
    for h in range(2):
        X = np.ascontiguousarray(x[h])
        planes = [X[a * n_pl:(a + 1) * n_pl] for a in range(5)]
        jit = None if jitter is None else np.asarray(jitter, dtype=np.float64)[h]
        out[h] = chisq(Dense(t, v, sigma, *planes, X[5 * n_pl], jit, t0))
        out[h][np.any(planes[1] < 0.0, axis=0)] = np.nan
    return out


def demc_run(t, v, sigma, x, chi2, n_pl, eps, seed, gen0, n_gen, jitter=None, t0=0.0, gamma=0.0,
             jump_every=0, n_accept=None, margin=False):
    """Run n_gen DE-MC generations (ter Braak 2006, split population; the
    sampler named in Sec. 6) on copies of x [2, 5 n_pl + 1, n_half] and
    chi2 [2, n_half]; returns (x, chi2, n_accept), plus, with margin=True,
    the last generation's decision margins (chi2(x) - chi2(y)) - 2 ln u
    [2, n_half] (a proposal is accepted iff its margin is > 0)."""
    t, v, sigma = _f64(t), _f64(v), _f64(sigma)
    x = np.array(x, dtype=np.float64, copy=True, order="C")
    chi2 = np.array(chi2, dtype=np.float64, copy=True, order="C")
    nh = x.shape[2]
    acc = np.zeros((2, nh), dtype=np.int64) if n_accept is None else np.array(n_accept, dtype=np.int64, copy=True)
    jit = None if jitter is None else np.ascontiguousarray(jitter, dtype=np.float64)
    eps = _f64(eps)
    mg = np.full((2, nh), np.nan) if margin else None
    s = _Demc(_ptr(t), _ptr(v), _ptr(sigma), t.size, float(t0), _ptr(x), _ptr(chi2), acc.ctypes.data_as(_I64),
              _ptr(jit), nh, n_pl, float(gamma), int(jump_every), 0, int(seed) & (2 ** 64 - 1), _ptr(eps), _ptr(mg))
    lib().oracle_demc_run(ctypes.byref(s), int(gen0), int(n_gen))
    return (x, chi2, acc, mg) if margin else (x, chi2, acc)


class Astro:
    """Astrometric batch (Thiele-Innes form): observation epochs t with measured
    offsets x (RA*cos Dec), y (Dec) and uncertainties sx, sy [n_obs]; planes
    P, e, M0, A, B, F, G [n_pl, n_sys]; optional offsets x0, y0 [n_sys]."""

    def __init__(self, t, x, y, sx, sy, P, e, M0, A, B, F, G, x0=None, y0=None, t0=0.0):
        self.t, self.x, self.y, self.sx, self.sy = (_f64(a) for a in (t, x, y, sx, sy))
        self.P, self.e, self.M0, self.A, self.B, self.F, self.G = (np.atleast_2d(_f64(a))
                                                                   for a in (P, e, M0, A, B, F, G))
        self.n_pl, self.n_sys = self.P.shape
        self.x0 = None if x0 is None else _f64(x0)
        self.y0 = None if y0 is None else _f64(y0)
        self.t0 = float(t0)
        self._s = _Astro(_ptr(self.t), _ptr(self.x), _ptr(self.y), _ptr(self.sx), _ptr(self.sy), self.t.size,
                         self.t0, _ptr(self.P), _ptr(self.e), _ptr(self.M0), _ptr(self.A), _ptr(self.B),
                         _ptr(self.F), _ptr(self.G), _ptr(self.x0), _ptr(self.y0), self.n_sys, self.n_pl)

    def _range(self, i0, i1):
        return int(i0), int(self.n_sys if i1 is None else i1)


def astro_model(d: Astro, i0=0, i1=None):
    """Model offsets [n_sys, 2, n_obs]: row 0 RA*cos Dec = B X + G Y, row 1 Dec = A X + F Y
    (X = cos E - e, Y = sqrt(1 - e^2) sin E), summed over planets, plus offsets."""
    i0, i1 = d._range(i0, i1)
    out = np.full((d.n_sys, 2, d.t.size), np.nan)
    lib().oracle_astro_model(ctypes.byref(d._s), _ptr(out), i0, i1)
    return out


def astro_chisq(d: Astro, i0=0, i1=None):
    """chi-square per system of the astrometric model against (x, y)."""
    i0, i1 = d._range(i0, i1)
    out = np.full(d.n_sys, np.nan)
    lib().oracle_astro_chisq(ctypes.byref(d._s), _ptr(out), i0, i1)
    return out
