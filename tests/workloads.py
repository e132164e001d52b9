"""Test-side workload helpers: seeded inputs (synth), observed velocities from the
oracle, and the oracle's reference values.  Shared by CPU and GPU tests."""
import numpy as np

import oracle
import synth

TWO_PI = 2.0 * np.pi


def oracle_truth_model(t, t0, truth):
    """Truth system's model velocities at times t, by the oracle."""
    cols = [np.asarray(truth[k], dtype=np.float64)[:, None] for k in ("P", "K", "e", "w", "M0")]
    d = oracle.Dense(t, np.zeros_like(t), np.ones_like(t), *cols, t0=t0)
    return oracle.rv_model(d)[0]


def oracle_phase(t, t0, P):
    """Fractional orbital phase frac((t - t0)/P) with the binary64 quotient (vectorised)."""
    q = (np.asarray(t, dtype=np.float64) - t0) / np.asarray(P, dtype=np.float64)
    return q - np.floor(q)


def dense(name, n_sys=None, n_obs=None, n_pl=None, seed=None, stress=False, jitter=False, t0=0.0, e_range=None):
    """Dense workload with observed velocities, optionally cut to n_obs / n_pl."""
    more = n_pl is not None and n_pl > synth.DENSE[name][1]
    wl = synth.dense(name, n_sys=n_sys, seed=seed, jitter=jitter, t0=t0, e_range=e_range,
                     n_pl=n_pl if more else None)
    if n_pl is not None and not more:
        wl.P, wl.K, wl.e, wl.w, wl.M0 = (np.ascontiguousarray(x[:n_pl]) for x in (wl.P, wl.K, wl.e, wl.w, wl.M0))
        wl.truth = {k: v[:n_pl] for k, v in wl.truth.items()}
    if n_obs is not None:
        rng = np.random.default_rng(0 if seed is None else seed)
        if n_obs <= wl.t.size:
            idx = np.sort(rng.choice(wl.t.size, size=n_obs, replace=False))
            wl.t, wl.sigma, wl.noise = wl.t[idx], wl.sigma[idx], wl.noise[idx]
        else:
            wl.t = np.sort(rng.uniform(synth.T_LO, synth.T_HI, n_obs))
            wl.sigma = rng.uniform(1, 5, n_obs)
            wl.noise = rng.normal(size=n_obs) * wl.sigma
    if stress:
        synth.periapsis_stress(wl, oracle_phase)
    synth.with_observations(wl, oracle_truth_model)
    return wl


def oracle_dense(wl):
    return oracle.Dense(wl.t, wl.v, wl.sigma, wl.P, wl.K, wl.e, wl.w, wl.M0, wl.offset, wl.jitter, wl.t0)


def rel_err_chi2(got, ref):
    """|chi2 - ref| / max(ref, 1)."""
    return np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)


def kepler_tol_mixed(M, e, E_ref):
    """Error bound of a binary32 Kepler solve (derivation in the design notes):
    the argument is reduced to [-pi, pi] in binary64 and rounded (u |Mr|), the
    converged iterate leaves |f| <= 8 u (|Mr| + |Er|) of evaluation error,
    divided by f' = 1 - e cos E, plus the rounding of E itself, the rounding of
    the last step (a few ulp of a step of at most 0.015 rad after the
    schedule's earlier steps) and the 1e-9 rad of the iteration schedule."""
    u = 2.0 ** -24
    k = np.rint(M / TWO_PI)
    Mr = M - k * TWO_PI
    Er = E_ref - k * TWO_PI
    fp = 1.0 - e * np.cos(E_ref)
    return 8 * u * (np.abs(Mr) + np.abs(Er)) / fp + 2 * u * np.abs(Er) + 4 * u * 0.015 + 1e-9 + 4e-16 * np.abs(E_ref)


def n_threads():
    import os
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def oracle_par(fn, d, n_sys):
    """Run an oracle batch function fn(d, i0, i1) over system chunks on host threads
    (the C oracle releases the GIL); fn returns arrays indexed by system in the
    last axis, which are merged."""
    from concurrent.futures import ThreadPoolExecutor
    nt = n_threads()
    bounds = np.linspace(0, n_sys, min(nt * 4, max(n_sys, 1)) + 1).astype(int)
    chunks = [(a, b) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    with ThreadPoolExecutor(nt) as ex:
        parts = list(ex.map(lambda ab: (ab, fn(d, ab[0], ab[1])), chunks))
    first = parts[0][1]
    multi = isinstance(first, tuple)
    outs = [np.array(x, copy=True) for x in (first if multi else (first,))]
    for (a, b), res in parts[1:]:
        res = res if multi else (res,)
        for o, r in zip(outs, res):
            o[..., a:b] = r[..., a:b]
    return tuple(outs) if multi else outs[0]


def to_gpu(wl, dev):
    """Torch views of a dense workload on the GPU (planes (n_pl, n_sys))."""
    import torch

    def g(x):
        return None if x is None else torch.from_numpy(np.ascontiguousarray(x)).to(dev)

    return dict(t=g(wl.t), v=g(wl.v), sigma=g(wl.sigma), P=g(wl.P), K=g(wl.K), e=g(wl.e), omega=g(wl.w),
                M0=g(wl.M0), offset=g(wl.offset), jitter=g(wl.jitter), t0=wl.t0)


# Velocity error allowed for the mixed path when a chi-square tolerance is derived
# from it (an order of magnitude below the stated 1e-3 m/s velocity tolerance).
DV_MIXED = 1e-4


def chi2_tol_mixed_ragged(rw, ref):
    """Per-system chi-square tolerance of the mixed path: the stated relative 1e-5
    (of max(chi2, 1)), or, where that is below what binary32 velocities allow
    (few observations, small residuals), the change a velocity error DV_MIXED
    can cause: 2 dv sum_k w_k |r_k| + dv^2 sum_k w_k."""
    import oracle as _o
    tol = 1e-5 * np.maximum(np.abs(ref), 1.0)
    for i in range(rw.n_sys):
        o0, o1 = rw.obs_off[i], rw.obs_off[i + 1]
        p0, p1 = rw.pl_off[i], rw.pl_off[i + 1]
        if o1 == o0 or not np.isfinite(ref[i]):
            continue
        off = None if rw.offset is None else rw.offset[i:i + 1]
        d = _o.Dense(rw.t[o0:o1], rw.v[o0:o1], rw.sigma[o0:o1], rw.P[p0:p1, None], rw.K[p0:p1, None],
                     rw.e[p0:p1, None], rw.w[p0:p1, None], rw.M0[p0:p1, None], off, None, rw.t0)
        r = _o.rv_model(d)[0] - rw.v[o0:o1]
        jit = 0.0 if rw.jitter is None else rw.jitter[i]
        w = 1.0 / (rw.sigma[o0:o1] ** 2 + jit ** 2)
        tol[i] = max(tol[i], 2 * DV_MIXED * np.sum(w * np.abs(r)) + DV_MIXED ** 2 * np.sum(w))
    return tol


def oracle_astro_truth(t, t0, truth):
    """Truth system's astrometric offsets (2, n_obs) by the oracle."""
    z = np.zeros_like(t)
    cols = [np.asarray(truth[k], dtype=np.float64).reshape(-1, 1) for k in ("P", "e", "M0", "A", "B", "F", "G")]
    return oracle.astro_model(oracle.Astro(t, z, z, z + 1, z + 1, *cols, t0=t0))[0]


def astro(n_sys, n_pl, n_obs, seed=None, e_range=(0.0, 0.9), noise_free=False):
    wl = synth.astro(n_sys=n_sys, n_pl=n_pl, n_obs=n_obs, seed=seed, e_range=e_range)
    return synth.with_astro_observations(wl, oracle_astro_truth, noise_free=noise_free)


def oracle_astro(wl):
    return oracle.Astro(wl.t, wl.x, wl.y, wl.sx, wl.sy, wl.P, wl.e, wl.M0, wl.A, wl.B, wl.F, wl.G, wl.x0, wl.y0,
                        wl.t0)


def astro_to_gpu(wl, dev):
    import torch

    def g(a):
        return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    return dict(t=g(wl.t), x=g(wl.x), y=g(wl.y), sigma_x=g(wl.sx), sigma_y=g(wl.sy), P=g(wl.P), e=g(wl.e),
                M0=g(wl.M0), A=g(wl.A), B=g(wl.B), F=g(wl.F), G=g(wl.G), x0=g(wl.x0), y0=g(wl.y0), t0=wl.t0)
