"""The allocation-free ragged entry point (rv_chisq_ragged_static, for callers
that cannot allocate device memory) against the plan-based entry point it
varies (kep_plan_ragged + rv_chisq_ragged) and against the oracle, called
through the C ABI.  Mixed-precision bar: chi2 within 1e-5 of max(chi2, 1).
Two calls in a row share the library's static work area, the second with a
smaller batch."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_0812_2976_amd as kp
import synth
from tests import workloads as W

pytestmark = pytest.mark.gpu


def _ragged(n_sys, seed, n_obs_range=(16, 1024)):
    rw = synth.ragged(n_sys=n_sys, seed=seed, n_obs_range=n_obs_range)
    synth.ragged_with_observations(rw, W.oracle_truth_model)
    rng = np.random.default_rng(seed)
    rw.offset = rng.uniform(-10, 10, rw.n_sys)
    rw.jitter = rng.uniform(0, 3, rw.n_sys)
    return rw


def _gpu(rw, dev):
    g = lambda x: None if x is None else torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    return {k: g(getattr(rw, k)) for k in ("t", "v", "sigma", "obs_off", "P", "K", "e", "w", "M0", "pl_off",
                                           "offset", "jitter")}


def _static_c_abi(g, n_sys, t0, dev):
    """rv_chisq_ragged_static called directly through ctypes (no binding logic)."""
    L = kp.load_library()
    out = torch.full((n_sys,), -1.0, dtype=torch.float64, device=dev)
    obs = kp.KepObsCSR(g["t"].data_ptr(), g["v"].data_ptr(), g["sigma"].data_ptr(), g["obs_off"].data_ptr(),
                       g["t"].numel(), float(t0))
    par = kp.KepParamsCSR(g["P"].data_ptr(), g["K"].data_ptr(), g["e"].data_ptr(), g["w"].data_ptr(),
                          g["M0"].data_ptr(), g["pl_off"].data_ptr(), g["offset"].data_ptr(), g["jitter"].data_ptr(),
                          n_sys, g["P"].numel())
    stream = torch.cuda.current_stream(dev).cuda_stream
    st = L.rv_chisq_ragged_static(ctypes.byref(obs), ctypes.byref(par), out.data_ptr(), kp.KEP_MIXED, None, stream)
    assert st == 0, L.kep_last_error().decode()
    return out


def _plan_chi2(g, rw, dev):
    plan = kp.RaggedPlan(g["t"], g["v"], g["sigma"], g["obs_off"], g["P"], g["K"], g["e"], g["w"], g["M0"],
                         g["pl_off"], g["offset"], g["jitter"], rw.t0, "mixed")
    out = plan().cpu().numpy()
    plan.close()
    return out


def _oracle(rw):
    d = oracle.Ragged(rw.t, rw.v, rw.sigma, rw.obs_off, rw.P, rw.K, rw.e, rw.w, rw.M0, rw.pl_off, rw.offset,
                      rw.jitter, rw.t0)
    return W.oracle_par(oracle.chisq_ragged, d, rw.n_sys)


def test_static_matches_plan_on_two_calls_in_a_row(dev):
    for n_sys, seed in ((3000, 21), (700, 22)):           # the second call is smaller
        rw = _ragged(n_sys, seed)
        g = _gpu(rw, dev)
        print(f"[no-alloc] rv_chisq_ragged_static n_sys={n_sys} seed={seed}", flush=True)
        got = _static_c_abi(g, rw.n_sys, rw.t0, dev).cpu().numpy()
        ref_plan = _plan_chi2(g, rw, dev)
        ref = _oracle(rw)
        e_plan = W.rel_err_chi2(got, ref_plan)
        e_orc = W.rel_err_chi2(got, ref)
        print(f"[no-alloc] n_sys={n_sys}: max rel vs plan {e_plan.max():.3e}, vs oracle {e_orc.max():.3e}",
              flush=True)
        assert np.all(np.isfinite(got))
        assert e_plan.max() <= 1e-5
        assert e_orc.max() <= 1e-5


def test_static_is_repeatable_and_matches_binding(dev):
    rw = _ragged(1200, 23)
    g = _gpu(rw, dev)
    a = _static_c_abi(g, rw.n_sys, rw.t0, dev).cpu().numpy()
    b = kp.rv_chisq_ragged_static(g["t"], g["v"], g["sigma"], g["obs_off"], g["P"], g["K"], g["e"], g["w"], g["M0"],
                                  g["pl_off"], g["offset"], g["jitter"], rw.t0).cpu().numpy()
    assert np.array_equal(a, b)       # the order is deterministic, so every call gives the same bits


def _valid(obs_off, pl_off, n_obs_total, n_pl_total):
    o0, o1, p0, p1 = obs_off[:-1], obs_off[1:], pl_off[:-1], pl_off[1:]
    return ((o0 >= 0) & (o0 <= o1) & (o1 <= n_obs_total) & (p0 >= 0) & (p0 < p1) & (p1 <= n_pl_total)
            & (p1 - p0 <= kp.KEP_MAX_PL))


def test_static_rejects_bad_offsets_per_system(dev):
    """Offsets outside the arrays, decreasing offsets or more than KEP_MAX_PL planets
    make those systems NaN (checked on the device); the others keep their chi-square."""
    rw = _ragged(500, 24, n_obs_range=(16, 300))
    g = _gpu(rw, dev)
    good = _static_c_abi(g, rw.n_sys, rw.t0, dev).cpu().numpy()
    n_obs_total, n_pl_total = int(rw.obs_off[-1]), int(rw.pl_off[-1])
    bad_obs = rw.obs_off.copy()
    bad_obs[101] = n_obs_total + 5               # system 100 ends, system 101 starts, past the array
    bad_obs[201] = bad_obs[200] - 1              # system 200 decreases (201 stays valid, longer)
    bad_pl = rw.pl_off.copy()
    bad_pl[-1] = n_pl_total + 2                  # the last system ends past the planet array
    valid = _valid(bad_obs, bad_pl, n_obs_total, n_pl_total)
    assert np.flatnonzero(~valid).tolist() == [100, 101, 200, rw.n_sys - 1]
    g2 = dict(g, obs_off=torch.from_numpy(bad_obs).to(dev), pl_off=torch.from_numpy(bad_pl).to(dev))
    got = _static_c_abi(g2, rw.n_sys, rw.t0, dev).cpu().numpy()
    assert np.all(np.isnan(got[~valid]))
    same = valid.copy()
    same[201] = False                            # valid, but with other observations than in `good`
    assert np.isfinite(got[201])
    assert np.all(W.rel_err_chi2(got[same], good[same]) <= 1e-5)
    # a system with nine planets (one more than KEP_MAX_PL), the rest unchanged
    n10 = int(rw.pl_off[11] - rw.pl_off[10])
    nine = rw.pl_off.copy()
    nine[11:] += 9 - n10
    planes = {k: np.concatenate([getattr(rw, k)[:rw.pl_off[10]], np.full(9, getattr(rw, k)[rw.pl_off[10]]),
                                 getattr(rw, k)[rw.pl_off[11]:]]) for k in ("P", "K", "e", "w", "M0")}
    g3 = dict(g, pl_off=torch.from_numpy(nine).to(dev),
              **{k: torch.from_numpy(np.ascontiguousarray(x)).to(dev) for k, x in planes.items()})
    got = _static_c_abi(g3, rw.n_sys, rw.t0, dev).cpu().numpy()
    assert np.isnan(got[10])
    others = np.arange(rw.n_sys) != 10
    assert np.all(W.rel_err_chi2(got[others], good[others]) <= 1e-5)


def test_static_size_limit_is_an_error(dev):
    L = kp.load_library()
    obs = kp.KepObsCSR(None, None, None, None, 0, 0.0)
    par = kp.KepParamsCSR(None, None, None, None, None, None, None, None, (1 << 21) + 1, 0)
    st = L.rv_chisq_ragged_static(ctypes.byref(obs), ctypes.byref(par), None, kp.KEP_MIXED, None, None)
    assert st == 2 and "static work area" in L.kep_last_error().decode()
    par = kp.KepParamsCSR(None, None, None, None, None, None, None, None, 0, 0)
    assert L.rv_chisq_ragged_static(ctypes.byref(obs), ctypes.byref(par), None, kp.KEP_MIXED, None, None) == 0
