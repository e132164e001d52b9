"""Seeded synthetic workloads shaped like the paper's benchmark (Sec. 5, Table 2).

This module only draws random numbers and packs arrays.  It holds none of the
method's arithmetic: wherever a workload needs model velocities (the noisy
"observed" velocities) or a mean anomaly (the periapsis stress set), the caller
passes the function that computes them — the CPU oracle in the tests, the GPU
library in the benchmark.

Draw order is fixed so that a seed reproduces the same bytes:
times (sorted), sigma, truth parameters, noise, model parameter planes
P, K, e, omega, M0 (planets sorted by P), then offsets and jitters.
System 0 of every dense batch is the truth system, so its chi-square is
distributed like chi-square with n_obs degrees of freedom.

Workloads (sizes n_sys x n_pl x n_obs):
  c0  1024 x 1 x 64        sigma = 3 m/s, plain FP64 case
  c1  65,536 x 4 x 256     sigma ~ U[1, 5] m/s
  c2  1,048,576 x 4 x 256  as c1 (mixed precision); stress set with e in [0.9, 0.99]
  c3  262,144 ragged       n_pl ~ U{1..7}, n_obs ~ round(logU[16, 1024]), CSR
  c4  262,144 x 4 x 256    e ~ U[0, 0.8], offsets ~ U[-10, 10] m/s (gradient)
Parameters: P log-uniform [1, 1000] d, K uniform [1, 100] m/s, e uniform
[0, 0.9], omega and M0 uniform [0, 2 pi); times uniform [2454000, 2457000] d.
"""
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

T_LO, T_HI = 2454000.0, 2457000.0
TWO_PI = 2.0 * np.pi

# (n_sys, n_pl, n_obs, e_max, sigma_mode, with_offset)
DENSE = {
    "c0": (1024, 1, 64, 0.9, "const3", False),
    "c1": (65536, 4, 256, 0.9, "uniform", False),
    "c2": (1048576, 4, 256, 0.9, "uniform", False),
    "c4": (262144, 4, 256, 0.8, "uniform", True),
}
SEEDS = {"c0": 1000, "c1": 1001, "c2": 1002, "c3": 1003, "c4": 1004, "stress": 1102,
         "kepler": 1200, "kepler_stress": 1201, "demc": 1300, "astro": 1400}


@dataclass
class DenseWorkload:
    name: str
    t: np.ndarray            # [n_obs] f64, sorted
    sigma: np.ndarray        # [n_obs] f64
    noise: np.ndarray        # [n_obs] f64, N(0, sigma^2)
    truth: dict              # planes of the truth system, each [n_pl]
    P: np.ndarray            # [n_pl, n_sys] f64, system index fastest
    K: np.ndarray
    e: np.ndarray
    w: np.ndarray
    M0: np.ndarray
    offset: Optional[np.ndarray] = None   # [n_sys] or None
    jitter: Optional[np.ndarray] = None   # [n_sys] or None
    t0: float = 0.0
    v: Optional[np.ndarray] = None        # [n_obs] set by with_observations()
    meta: dict = field(default_factory=dict)

    @property
    def n_sys(self):
        return self.P.shape[1]

    @property
    def n_pl(self):
        return self.P.shape[0]

    @property
    def n_obs(self):
        return self.t.size

    def params(self):
        return dict(P=self.P, K=self.K, e=self.e, w=self.w, M0=self.M0)


def _planet_params(rng, n_pl, n_sys, e_lo, e_hi):
    """P log-U[1, 1000] d, K U[1, 100] m/s, e U[e_lo, e_hi], omega, M0 U[0, 2pi);
    planets of each system sorted by period."""
    P = np.exp(rng.uniform(np.log(1.0), np.log(1000.0), size=(n_pl, n_sys)))
    K = rng.uniform(1.0, 100.0, size=(n_pl, n_sys))
    e = rng.uniform(e_lo, e_hi, size=(n_pl, n_sys))
    w = rng.uniform(0.0, TWO_PI, size=(n_pl, n_sys))
    M0 = rng.uniform(0.0, TWO_PI, size=(n_pl, n_sys))
    order = np.argsort(P, axis=0, kind="stable")
    P, K, e, w, M0 = (np.take_along_axis(x, order, axis=0) for x in (P, K, e, w, M0))
    return [np.ascontiguousarray(x) for x in (P, K, e, w, M0)]


def dense(name: str, n_sys: Optional[int] = None, seed: Optional[int] = None,
          e_range=None, t0: float = 0.0, jitter: bool = False, n_pl: Optional[int] = None) -> DenseWorkload:
    """Dense workload `name` (c0, c1, c2 or c4), optionally with fewer systems or
    another planet count (n_pl changes every draw after sigma).  The observed
    velocities are not filled in: call with_observations()."""
    n_sys0, n_pl0, n_obs, e_max, sig_mode, with_off = DENSE[name]
    n_pl = n_pl0 if n_pl is None else int(n_pl)
    n_sys = n_sys0 if n_sys is None else int(n_sys)
    rng = np.random.Generator(np.random.PCG64(SEEDS[name] if seed is None else seed))
    e_lo, e_hi = (0.0, e_max) if e_range is None else e_range
    t = np.sort(rng.uniform(T_LO, T_HI, size=n_obs))
    sigma = np.full(n_obs, 3.0) if sig_mode == "const3" else rng.uniform(1.0, 5.0, size=n_obs)
    tp = _planet_params(rng, n_pl, 1, e_lo, e_hi)
    truth = dict(zip(("P", "K", "e", "w", "M0"), (x[:, 0].copy() for x in tp)))
    noise = rng.normal(0.0, 1.0, size=n_obs) * sigma
    P, K, e, w, M0 = _planet_params(rng, n_pl, n_sys, e_lo, e_hi)
    for plane, key in zip((P, K, e, w, M0), ("P", "K", "e", "w", "M0")):
        if n_sys > 0:
            plane[:, 0] = truth[key]
    offset = rng.uniform(-10.0, 10.0, size=n_sys) if with_off else None
    if offset is not None and n_sys > 0:
        offset[0] = 0.0
    jit = rng.uniform(0.0, 3.0, size=n_sys) if jitter else None
    return DenseWorkload(name, t, sigma, noise, truth, P, K, e, w, M0, offset, jit, t0,
                         meta=dict(seed=SEEDS[name] if seed is None else seed))


def with_observations(wl: DenseWorkload, model_fn: Callable, noise_free: bool = False) -> DenseWorkload:
    """Set wl.v = model_fn(t, t0, truth) + noise.  model_fn(t [n_obs], t0,
    truth dict of [n_pl] arrays) -> [n_obs] returns the truth system's model
    velocities; it is supplied by the caller (oracle or GPU library)."""
    vm = np.asarray(model_fn(wl.t, wl.t0, wl.truth), dtype=np.float64)
    wl.v = vm if noise_free else vm + wl.noise
    return wl


def periapsis_stress(wl: DenseWorkload, phase_fn: Callable, seed: Optional[int] = None,
                     e_range=(0.9, 0.99)) -> DenseWorkload:
    """Move every planet of every system except the truth system close to
    periapsis at one of its observation times: e ~ U[e_range], and for each
    (system, planet) an index k* and an offset delta = +-10^U[-9, -1] rad are
    drawn; M0 is then set so that the mean anomaly at t[k*] equals delta.
    phase_fn(t, t0, P) -> fractional orbital phase in [0, 1) of time t for
    period P (vectorised); it is supplied by the caller."""
    rng = np.random.Generator(np.random.PCG64(SEEDS["stress"] if seed is None else seed))
    n_pl, n_sys = wl.P.shape
    e = rng.uniform(e_range[0], e_range[1], size=(n_pl, n_sys))
    kstar = rng.integers(0, wl.n_obs, size=(n_pl, n_sys))
    delta = np.power(10.0, rng.uniform(-9.0, -1.0, size=(n_pl, n_sys)))
    delta *= np.where(rng.uniform(size=(n_pl, n_sys)) < 0.5, -1.0, 1.0)
    frac = np.asarray(phase_fn(wl.t[kstar], wl.t0, wl.P), dtype=np.float64)
    M0 = np.mod(delta - TWO_PI * frac, TWO_PI)
    sl = slice(1, None)
    wl.e[:, sl] = e[:, sl]
    wl.M0[:, sl] = M0[:, sl]
    wl.meta["stress"] = dict(kstar=kstar, delta=delta)
    return wl


@dataclass
class RaggedWorkload:
    t: np.ndarray            # [n_obs_total]
    sigma: np.ndarray
    noise: np.ndarray
    obs_off: np.ndarray      # int64 [n_sys + 1]
    truth: dict
    P: np.ndarray            # [n_pl_total]
    K: np.ndarray
    e: np.ndarray
    w: np.ndarray
    M0: np.ndarray
    pl_off: np.ndarray       # int64 [n_sys + 1]
    offset: Optional[np.ndarray] = None
    jitter: Optional[np.ndarray] = None
    t0: float = 0.0
    v: Optional[np.ndarray] = None

    @property
    def n_sys(self):
        return self.obs_off.size - 1

    @property
    def n_obs(self):
        return np.diff(self.obs_off)

    @property
    def n_pl(self):
        return np.diff(self.pl_off)


def ragged(n_sys: int = 262144, seed: Optional[int] = None, n_pl_max: int = 7,
           n_obs_range=(16, 1024), uniform=None, e_max: float = 0.9, sizes=None) -> RaggedWorkload:
    """CSR ragged workload c3: n_pl ~ U{1..n_pl_max}, n_obs = round(exp U[ln lo, ln hi]),
    each system with its own sorted times and sigma ~ U[1, 5].  uniform=(n_pl, n_obs)
    makes every system the same size (for the ragged-equals-dense check);
    sizes=(n_pl array, n_obs array) gives every system's size explicitly."""
    rng = np.random.Generator(np.random.PCG64(SEEDS["c3"] if seed is None else seed))
    if sizes is not None:
        n_pl = np.asarray(sizes[0], dtype=np.int64)
        n_obs = np.asarray(sizes[1], dtype=np.int64)
        if n_pl.shape != (n_sys,) or n_obs.shape != (n_sys,):
            raise ValueError("sizes must hold n_sys planet counts and n_sys observation counts")
    elif uniform is None:
        n_pl = rng.integers(1, n_pl_max + 1, size=n_sys)
        lo, hi = n_obs_range
        n_obs = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=n_sys))).astype(np.int64)
    else:
        n_pl = np.full(n_sys, uniform[0], dtype=np.int64)
        n_obs = np.full(n_sys, uniform[1], dtype=np.int64)
    obs_off = np.zeros(n_sys + 1, dtype=np.int64)
    np.cumsum(n_obs, out=obs_off[1:])
    pl_off = np.zeros(n_sys + 1, dtype=np.int64)
    np.cumsum(n_pl, out=pl_off[1:])
    n_tot = int(obs_off[-1])
    # sorted times within each system: sort the key (system index + u) once
    u = rng.uniform(0.0, 1.0, size=n_tot)
    sys_of = np.repeat(np.arange(n_sys, dtype=np.float64), n_obs)
    u = np.sort(sys_of + u) - sys_of
    t = T_LO + (T_HI - T_LO) * u
    sigma = rng.uniform(1.0, 5.0, size=n_tot)
    tp = _planet_params(rng, 4, 1, 0.0, e_max)
    truth = dict(zip(("P", "K", "e", "w", "M0"), (x[:, 0].copy() for x in tp)))
    noise = rng.normal(0.0, 1.0, size=n_tot) * sigma
    n_pl_tot = int(pl_off[-1])
    P = np.exp(rng.uniform(np.log(1.0), np.log(1000.0), size=n_pl_tot))
    K = rng.uniform(1.0, 100.0, size=n_pl_tot)
    e = rng.uniform(0.0, e_max, size=n_pl_tot)
    w = rng.uniform(0.0, TWO_PI, size=n_pl_tot)
    M0 = rng.uniform(0.0, TWO_PI, size=n_pl_tot)
    # sort planets by period within each system
    sys_pl = np.repeat(np.arange(n_sys), n_pl)
    order = np.lexsort((P, sys_pl))
    P, K, e, w, M0 = (np.ascontiguousarray(x[order]) for x in (P, K, e, w, M0))
    return RaggedWorkload(t, sigma, noise, obs_off, truth, P, K, e, w, M0, pl_off)


def ragged_with_observations(wl: RaggedWorkload, model_fn: Callable) -> RaggedWorkload:
    """wl.v = model_fn(t_all, t0, truth) + noise, with every system observing
    the same truth system at its own times."""
    wl.v = np.asarray(model_fn(wl.t, wl.t0, wl.truth), dtype=np.float64) + wl.noise
    return wl


def kepler_pairs(n: int, seed: Optional[int] = None, stress: bool = False):
    """(M, e) pairs for the standalone Kepler solve.  Default: M ~ U[0, 2pi),
    e ~ U[0, 0.9].  stress: M = +-10^U[-9, 0] wrapped into [0, 2pi),
    e ~ U[0.9, 0.99]."""
    key = "kepler_stress" if stress else "kepler"
    rng = np.random.Generator(np.random.PCG64(SEEDS[key] if seed is None else seed))
    if not stress:
        M = rng.uniform(0.0, TWO_PI, size=n)
        e = rng.uniform(0.0, 0.9, size=n)
    else:
        mag = np.power(10.0, rng.uniform(-9.0, 0.0, size=n))
        sgn = np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
        M = np.mod(sgn * mag, TWO_PI)
        e = rng.uniform(0.9, 0.99, size=n)
    return M, e


def demc_population(truth: dict, n_half: int, seed: Optional[int] = None, rel_spread: float = 1e-4):
    """Initial population for the DE-MC sampler, [2, 5 n_pl + 1, n_half]: each
    half holds parameter planes P, K, e, omega, M0 (planet-major rows) and the
    offset row, scattered about a truth system by rel_spread (relative, at least
    0.05 absolute scale for e and the angles), e clipped to [0, 0.95], offset
    ~ N(0, 0.5 m/s).  Also returns the per-row proposal scale eps [d]
    (rel_spread / 10 of the same scales)."""
    rng = np.random.default_rng(SEEDS["demc"] if seed is None else seed)
    keys = ("P", "K", "e", "w", "M0")
    tr = {k: np.asarray(truth[k], dtype=np.float64).reshape(-1) for k in keys}
    n_pl = tr["P"].size
    x = np.empty((2, 5 * n_pl + 1, n_half))
    eps = []
    for a, k in enumerate(keys):
        scale = np.maximum(np.abs(tr[k]), 0.05)
        x[:, a * n_pl:(a + 1) * n_pl, :] = tr[k][:, None] + rel_spread * scale[:, None] * rng.normal(size=(2, n_pl, n_half))
        eps.append(0.1 * rel_spread * scale)
    x[:, 2 * n_pl:3 * n_pl, :] = np.clip(x[:, 2 * n_pl:3 * n_pl, :], 0.0, 0.95)
    x[:, 5 * n_pl, :] = rng.normal(scale=0.5, size=(2, n_half))
    return x, np.concatenate(eps + [np.array([0.1 * rel_spread])])


@dataclass
class AstroWorkload:
    """Astrometric batch: epochs t [n_obs] with offsets x (RA*cos Dec), y (Dec) and
    uncertainties sx, sy; planes P, e, M0, A, B, F, G [n_pl, n_sys]; offsets x0, y0."""
    t: np.ndarray
    sx: np.ndarray
    sy: np.ndarray
    P: np.ndarray
    e: np.ndarray
    M0: np.ndarray
    A: np.ndarray
    B: np.ndarray
    F: np.ndarray
    G: np.ndarray
    x0: np.ndarray
    y0: np.ndarray
    noise_x: np.ndarray
    noise_y: np.ndarray
    truth: dict
    t0: float = 0.0
    x: Optional[np.ndarray] = None
    y: Optional[np.ndarray] = None

    @property
    def n_sys(self):
        return self.P.shape[1]

    @property
    def n_pl(self):
        return self.P.shape[0]


def astro(n_sys: int = 1048576, n_pl: int = 2, n_obs: int = 128, seed: Optional[int] = None,
          e_range=(0.0, 0.9)) -> AstroWorkload:
    """Astrometric workload: n_obs epochs over five years (t ~ U[2457000, 2458826] d,
    sorted), sigma_x, sigma_y ~ U[0.02, 0.1] mas; per planet P log-uniform [10, 2000] d,
    e ~ U[e_range], M0 ~ U[0, 2 pi), Thiele-Innes constants a u with a log-uniform
    [1, 100] mas (a binary-star range: amplitudes up to 5000 times the noise) and
    u ~ U[-1, 1] for each of A, B, F, G; offsets ~ U[-1, 1] mas.  System 0 is the
    truth (zero offsets); its noise is drawn here, the observed offsets are formed
    by with_astro_observations."""
    rng = np.random.default_rng(SEEDS["astro"] if seed is None else seed)
    t = np.sort(rng.uniform(2457000.0, 2458826.0, n_obs))
    sx = rng.uniform(0.02, 0.1, n_obs)
    sy = rng.uniform(0.02, 0.1, n_obs)

    def planets(n):
        P = np.sort(np.exp(rng.uniform(np.log(10.0), np.log(2000.0), size=(n_pl, n))), axis=0)
        e = rng.uniform(e_range[0], e_range[1], size=(n_pl, n))
        M0 = rng.uniform(0.0, TWO_PI, size=(n_pl, n))
        a = np.exp(rng.uniform(0.0, np.log(100.0), size=(n_pl, n)))
        c = [a * rng.uniform(-1.0, 1.0, size=(n_pl, n)) for _ in range(4)]
        return [P, e, M0] + c

    truth = dict(zip(("P", "e", "M0", "A", "B", "F", "G"), planets(1)))
    noise_x = rng.normal(size=n_obs) * sx
    noise_y = rng.normal(size=n_obs) * sy
    planes = planets(n_sys)
    x0 = rng.uniform(-1.0, 1.0, n_sys)
    y0 = rng.uniform(-1.0, 1.0, n_sys)
    for k, arr in zip(("P", "e", "M0", "A", "B", "F", "G"), planes):
        arr[:, 0] = truth[k][:, 0]
    x0[0] = y0[0] = 0.0
    return AstroWorkload(t, sx, sy, *planes, x0, y0, noise_x, noise_y, truth)


def with_astro_observations(wl: AstroWorkload, model_fn: Callable, noise_free: bool = False) -> AstroWorkload:
    """Observed offsets = model of the truth system (model_fn(t, t0, truth) -> (2, n_obs))
    plus the drawn noise."""
    m = np.asarray(model_fn(wl.t, wl.t0, wl.truth))
    wl.x = m[0] + (0.0 if noise_free else wl.noise_x)
    wl.y = m[1] + (0.0 if noise_free else wl.noise_y)
    return wl
