"""GPU parity of the ragged (CSR) persistent kernel, its HIP-graph replay and its
autotuned launch shape, against the oracle.  Mixed precision: chi2 relative
error <= 1e-5 (relative to max(chi2, 1)).  The plain binary64 ragged path
(plans and the allocation-free call with KEP_FP64): relative 1e-12, as the
dense binary64 chi-square, and NaN exactly for the systems whose offsets are
inconsistent."""
import numpy as np
import pytest
import torch

import oracle
import paper_0812_2976_amd as kp
import synth
from tests import workloads as W

pytestmark = pytest.mark.gpu


def _ragged(n_sys, seed=None, n_obs_range=(16, 1024), uniform=None, offsets=False, jitter=False):
    rw = synth.ragged(n_sys=n_sys, seed=seed, n_obs_range=n_obs_range, uniform=uniform)
    synth.ragged_with_observations(rw, W.oracle_truth_model)
    rng = np.random.default_rng(7)
    if offsets:
        rw.offset = rng.uniform(-10, 10, rw.n_sys)
    if jitter:
        rw.jitter = rng.uniform(0, 3, rw.n_sys)
    return rw


def _plan(rw, dev, opts=None, prec="mixed"):
    g = lambda x: None if x is None else torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    return kp.RaggedPlan(g(rw.t), g(rw.v), g(rw.sigma), g(rw.obs_off), g(rw.P), g(rw.K), g(rw.e), g(rw.w),
                         g(rw.M0), g(rw.pl_off), g(rw.offset), g(rw.jitter), rw.t0, prec, opts)


def _static(rw, dev, prec, obs_off=None, pl_off=None):
    g = lambda x: None if x is None else torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    return kp.rv_chisq_ragged_static(g(rw.t), g(rw.v), g(rw.sigma), g(rw.obs_off if obs_off is None else obs_off),
                                     g(rw.P), g(rw.K), g(rw.e), g(rw.w), g(rw.M0),
                                     g(rw.pl_off if pl_off is None else pl_off), g(rw.offset), g(rw.jitter), rw.t0,
                                     prec=prec).cpu().numpy()


def _oracle(rw):
    d = oracle.Ragged(rw.t, rw.v, rw.sigma, rw.obs_off, rw.P, rw.K, rw.e, rw.w, rw.M0, rw.pl_off, rw.offset,
                      rw.jitter, rw.t0)
    return W.oracle_par(oracle.chisq_ragged, d, rw.n_sys)


@pytest.mark.parametrize("case", [
    dict(n_sys=3000),
    dict(n_sys=1500, n_obs_range=(1, 70), offsets=True, jitter=True),
    dict(n_sys=97, n_obs_range=(200, 1024)),
])
def test_ragged_matches_oracle(dev, case):
    rw = _ragged(case["n_sys"], n_obs_range=case.get("n_obs_range", (16, 1024)),
                 offsets=case.get("offsets", False), jitter=case.get("jitter", False))
    plan = _plan(rw, dev)
    chi2 = plan().cpu().numpy()
    ref = _oracle(rw)
    err = W.rel_err_chi2(chi2, ref)
    print(f"[ragged {case}] max rel {err.max():.3e}; systems within 1e-5: {np.mean(err <= 1e-5):.4f}; "
          f"info {plan.info()}", flush=True)
    if case.get("n_obs_range", (16, 1024))[0] >= 16:
        assert err.max() <= 1e-5                      # the stated tolerance on the paper-shaped batches
    else:
        # down to one observation per system: the bound a velocity error can cause
        assert np.all(np.abs(chi2 - ref) <= W.chi2_tol_mixed_ragged(rw, ref))


@pytest.mark.parametrize("case", [
    dict(n_sys=600),
    dict(n_sys=700, n_obs_range=(1, 70), offsets=True, jitter=True),
])
def test_ragged_fp64_matches_oracle(dev, case):
    """KEP_FP64 ragged: the plan's two calls and the allocation-free call give the
    same bits (one wavefront per system whatever the order) and match the oracle
    to 1e-12 relative."""
    rw = _ragged(case["n_sys"], seed=31, n_obs_range=case.get("n_obs_range", (16, 1024)),
                 offsets=case.get("offsets", False), jitter=case.get("jitter", False))
    print(f"[ragged fp64] {case}", flush=True)
    plan = _plan(rw, dev, prec="fp64")
    chi2 = plan().cpu().numpy()
    direct = plan.direct().cpu().numpy()
    info = plan.info()
    plan.close()
    static = _static(rw, dev, "fp64")
    ref = _oracle(rw)
    err = W.rel_err_chi2(chi2, ref)
    print(f"[ragged fp64 {case}] max rel {err.max():.3e}; info {info}", flush=True)
    assert np.all(np.isfinite(chi2))
    assert err.max() <= 1e-12
    assert np.array_equal(direct, chi2) and np.array_equal(static, chi2)
    assert info["tuned"] == 0 and info["blocks"] >= 1 and info["sys_per_batch"] == 1


def test_ragged_fp64_static_rejects_bad_offsets_per_system(dev):
    """The binary64 kernel checks each system's offsets itself: inconsistent ones
    (past the arrays, decreasing, too many planets) give NaN for exactly those
    systems, the others keep their chi-square."""
    rw = _ragged(300, seed=32, n_obs_range=(16, 300))
    good = _static(rw, dev, "fp64")
    n_obs_total, n_pl_total = int(rw.obs_off[-1]), int(rw.pl_off[-1])
    bad_obs = rw.obs_off.copy()
    bad_obs[101] = n_obs_total + 5               # system 100 ends, system 101 starts, past the array
    bad_obs[201] = bad_obs[200] - 1              # system 200 decreases (201 stays valid, longer)
    bad_pl = rw.pl_off.copy()
    bad_pl[51] = bad_pl[50] + kp.KEP_MAX_PL + 1  # system 50 with nine planets (51 then decreases)
    bad_pl[-1] = n_pl_total + 2                  # the last system ends past the planet array
    o0, o1, p0, p1 = bad_obs[:-1], bad_obs[1:], bad_pl[:-1], bad_pl[1:]
    valid = ((o0 >= 0) & (o0 <= o1) & (o1 <= n_obs_total) & (p0 >= 0) & (p0 < p1) & (p1 <= n_pl_total)
             & (p1 - p0 <= kp.KEP_MAX_PL))
    # system 51 starts after system 50's nine planets: it decreases or, if its old end
    # lies beyond that, stays valid with other planets
    assert {50, 100, 101, 200, rw.n_sys - 1} <= set(np.flatnonzero(~valid).tolist())
    assert set(np.flatnonzero(~valid).tolist()) <= {50, 51, 100, 101, 200, rw.n_sys - 1}
    got = _static(rw, dev, "fp64", obs_off=bad_obs, pl_off=bad_pl)
    assert np.all(np.isnan(got[~valid]))
    assert np.all(np.isfinite(got[valid]))
    same = valid.copy()
    same[[51, 201]] = False                      # valid or not, with other inputs than in `good`
    assert np.array_equal(got[same], good[same])


def test_ragged_graph_replay_equals_direct(dev):
    """Several graph replays, with eager work and synchronisation between them,
    each equal the direct launch bit for bit."""
    rw = _ragged(2000, seed=11)
    plan = _plan(rw, dev)
    direct = plan.direct().cpu().numpy()
    out = torch.empty(rw.n_sys, dtype=torch.float64, device=dev)
    for rep in range(4):
        out.fill_(-1.0)
        plan(out)
        torch.cuda.synchronize()
        x = torch.randn(1000, device=dev).sum()        # unrelated eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), direct), rep
    # a new output buffer re-targets the recorded graph
    other = plan(torch.empty(rw.n_sys, dtype=torch.float64, device=dev)).cpu().numpy()
    assert np.array_equal(other, direct)
    assert x.isfinite()


def test_ragged_uniform_equals_dense(dev):
    """A ragged batch whose systems all have the same size matches the dense kernel
    on the same systems (within the mixed tolerance; lane grouping may differ)."""
    n_sys, n_pl, n_obs = 300, 4, 256
    wl = W.dense("c1", n_sys=n_sys)
    rw = synth.ragged(n_sys=n_sys, uniform=(n_pl, n_obs))
    rw.t = np.tile(wl.t, n_sys)
    rw.v = np.tile(wl.v, n_sys)
    rw.sigma = np.tile(wl.sigma, n_sys)
    rw.P, rw.K, rw.e, rw.w, rw.M0 = (np.ascontiguousarray(x.T.ravel()) for x in (wl.P, wl.K, wl.e, wl.w, wl.M0))
    plan = _plan(rw, dev)
    ragged = plan().cpu().numpy()
    dense = kp.rv_chisq(**W.to_gpu(wl, dev), prec="mixed").cpu().numpy()
    assert W.rel_err_chi2(ragged, dense).max() <= 2e-5


def test_ragged_launch_shapes_and_fixed_options(dev):
    rw = _ragged(800, seed=3)
    ref = _oracle(rw)
    for block in (64, 128, 256):
        plan = _plan(rw, dev, opts=dict(block_threads=block))
        chi2 = plan().cpu().numpy()
        assert W.rel_err_chi2(chi2, ref).max() <= 1e-5, block


def test_ragged_domain_nan_and_edge_sizes(dev):
    rw = _ragged(60, seed=5, n_obs_range=(1, 300))
    rw.e[rw.pl_off[10]] = 1.0
    rw.P[rw.pl_off[20]] = -1.0
    rw.sigma[rw.obs_off[30]] = np.nan
    chi2 = _plan(rw, dev)().cpu().numpy()
    ref = _oracle(rw)
    bad = np.isnan(ref)
    assert set(np.nonzero(bad)[0]) == {10, 20, 30}
    assert np.array_equal(np.isnan(chi2), bad)
    assert W.rel_err_chi2(chi2[~bad], ref[~bad]).max() <= 1e-5


# observation counts around the 64-lane group boundaries, zero included: the
# kernel evaluates whole groups of 64 per system and packs the remainders of a
# work item's systems into one stream of lanes
_EDGE_NOBS = np.array([0, 1, 2, 31, 33, 40, 63, 64, 65, 127, 128, 129, 191, 192, 193, 255, 256, 257, 300, 1000])


def _edge_batch(n_sys, seed):
    rng = np.random.default_rng(seed)
    n_obs = _EDGE_NOBS[rng.integers(0, _EDGE_NOBS.size, n_sys)]
    n_pl = rng.integers(1, 9, n_sys)
    rw = synth.ragged(n_sys=n_sys, seed=seed, sizes=(n_pl, n_obs))
    synth.ragged_with_observations(rw, W.oracle_truth_model)
    rw.offset = rng.uniform(-10, 10, n_sys)
    # invalid data: a non-finite sigma in the partial last group of one system,
    # in a whole group of another, and a planet outside the domain in a system
    # that fits in one partial group
    sizes = np.diff(rw.obs_off)
    tail_sys = int(np.nonzero((sizes > 64) & (sizes % 64 != 0))[0][0])
    full_sys = int(np.nonzero(sizes >= 64)[0][-1])
    small_sys = int(np.nonzero((sizes > 0) & (sizes < 64))[0][1])
    rw.sigma = rw.sigma.copy()
    rw.sigma[rw.obs_off[tail_sys + 1] - 1] = np.nan
    rw.sigma[rw.obs_off[full_sys]] = np.inf
    rw.e = rw.e.copy()
    rw.e[rw.pl_off[small_sys + 1] - 1] = 1.5
    return rw, {tail_sys, full_sys, small_sys}


def _check_edge(chi2, rw, invalid):
    ref = _oracle(rw)
    bad = np.isnan(ref)
    assert set(np.nonzero(bad)[0]) == invalid
    assert np.array_equal(np.isnan(chi2), bad)
    empty = np.diff(rw.obs_off) == 0
    assert np.all(chi2[empty & ~bad] == 0.0)
    ok = ~bad
    return bool(np.all(np.abs(chi2[ok] - ref[ok]) <= W.chi2_tol_mixed_ragged(rw, ref)[ok]))


def test_ragged_packed_tails_edges(dev):
    """Observation counts on both sides of every group boundary (0 to 1000),
    one to eight planets, offsets and invalid systems whose bad value sits in a
    packed tail, a whole group or a one-group system: NaN exactly where the
    oracle has it, the oracle's value elsewhere."""
    rw, invalid = _edge_batch(700, seed=41)
    plan = _plan(rw, dev)
    assert _check_edge(plan().cpu().numpy(), rw, invalid)
    assert _check_edge(plan.direct().cpu().numpy(), rw, invalid)
    for block in (64, 256):
        assert _check_edge(_plan(rw, dev, opts=dict(block_threads=block))().cpu().numpy(), rw, invalid)


def test_ragged_fp64_edges(dev):
    """KEP_FP64 on the same edge batch: NaN exactly where the oracle has it, zero
    for systems without observations, within 1e-12 elsewhere; plans with 256-
    and 64-thread blocks and the allocation-free call give the same bits."""
    rw, invalid = _edge_batch(500, seed=43)
    ref = _oracle(rw)
    bad = np.isnan(ref)
    assert set(np.nonzero(bad)[0]) == invalid
    empty = np.diff(rw.obs_off) == 0
    assert np.any(empty & ~bad)
    runs = [_plan(rw, dev, prec="fp64")().cpu().numpy(),
            _plan(rw, dev, opts=dict(block_threads=64), prec="fp64")().cpu().numpy(),
            _static(rw, dev, "fp64")]
    for got in runs:
        assert np.array_equal(np.isnan(got), bad)
        assert np.all(got[empty & ~bad] == 0.0)
        assert W.rel_err_chi2(got[~bad], ref[~bad]).max() <= 1e-12
        assert np.array_equal(got[~bad], runs[0][~bad])


_SHAPES_SCRIPT = r"""
import json, sys
import numpy as np, torch
sys.path.insert(0, sys.argv[1])
from tests import test_gpu_ragged as T
res = []
for n in (300, 600, 1200):
    rw, invalid = T._edge_batch(n, seed=n)
    plan = T._plan(rw, torch.device("cuda", 0))
    ok = T._check_edge(plan().cpu().numpy(), rw, invalid)
    res.append(dict(ok=ok, info=plan.info()))
print(json.dumps(res))
"""


def test_ragged_forced_launch_shapes(dev, tmp_path):
    """Every work-item layout the autotuner can choose gives the oracle's values:
    a first process tunes three batches and stores their shapes in
    KEP_TUNE_CACHE; the file is rewritten to force one system per item (64
    threads, two groups in flight), 32 systems per item (four groups) and 16
    per item (256 threads), and a second process runs the batches with them."""
    import json
    import os
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, KEP_TUNE_CACHE=str(cache))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

    def run():
        r = subprocess.run([sys.executable, "-c", _SHAPES_SCRIPT, root], env=env, capture_output=True, text=True,
                           timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        return json.loads(r.stdout.strip().splitlines()[-1])

    first = run()
    assert all(x["ok"] for x in first), first
    lines = cache.read_text().splitlines()
    assert len(lines) == 3
    forced = [(64, 1, 2), (128, 32, 4), (256, 16, 2)]
    cache.write_text("".join(f"{ln.split()[0]} {b} {sb} {g} 1.0\n" for ln, (b, sb, g) in zip(lines, forced)))
    second = run()
    for x, (b, sb, g) in zip(second, forced):
        assert x["ok"], x
        assert (x["info"]["block_threads"], x["info"]["sys_per_batch"], x["info"]["group_chunks"]) == (b, sb, g)


def test_ragged_rejects_bad_offsets(dev):
    rw = _ragged(10, seed=2)
    rw.pl_off = rw.pl_off.copy()
    rw.pl_off[3] = rw.pl_off[2]          # a system with no planet
    with pytest.raises(kp.KeplerError):
        _plan(rw, dev)


def test_ragged_c3_full_size_sampled(dev):
    """The full 262,144-system ragged batch as the benchmark runs it; 64 systems
    spread over the batch are checked against the oracle.  Only the sampled
    systems observe the truth system (oracle model + noise); the others see
    noise alone, which changes their chi-square values but not the work."""
    rw = synth.ragged(n_sys=262144)
    idx = np.unique(np.linspace(0, rw.n_sys - 1, 64).astype(int))
    rw.v = rw.noise.copy()
    for i in idx:
        o0, o1 = rw.obs_off[i], rw.obs_off[i + 1]
        rw.v[o0:o1] += W.oracle_truth_model(rw.t[o0:o1], rw.t0, rw.truth)
    plan = _plan(rw, dev)
    chi2 = plan().cpu().numpy()
    assert np.all(np.isfinite(chi2))
    d = oracle.Ragged(rw.t, rw.v, rw.sigma, rw.obs_off, rw.P, rw.K, rw.e, rw.w, rw.M0, rw.pl_off, t0=rw.t0)
    ref = np.array([oracle.chisq_ragged(d, int(i), int(i) + 1)[i] for i in idx])
    err = W.rel_err_chi2(chi2[idx], ref)
    print(f"[ragged c3 full] max rel {err.max():.3e} info {plan.info()}", flush=True)
    assert err.max() <= 1e-5


_TUNE_SCRIPT = r"""
import json, sys
import numpy as np, torch
sys.path.insert(0, sys.argv[1])
import paper_0812_2976_amd as kp, synth
rw = synth.ragged(n_sys=4000, seed=21)
rw.v = rw.noise
g = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
plan = kp.RaggedPlan(g(rw.t), g(rw.v), g(rw.sigma), g(rw.obs_off), g(rw.P), g(rw.K), g(rw.e), g(rw.w), g(rw.M0),
                     g(rw.pl_off))
print(json.dumps(plan.info()))
"""


def test_autotune_table_persists(dev, tmp_path):
    """The tuned launch shape is written to KEP_TUNE_CACHE and read back by a
    second process, which then skips tuning and reuses it."""
    import json
    import os
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, KEP_TUNE_CACHE=str(cache))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    infos = []
    for _ in range(2):
        r = subprocess.run([sys.executable, "-c", _TUNE_SCRIPT, root], env=env, capture_output=True, text=True,
                           timeout=180)
        assert r.returncode == 0, r.stderr[-2000:]
        infos.append(json.loads(r.stdout.strip().splitlines()[-1]))
    lines = cache.read_text().split()
    assert len(lines) == 5 and "/ragged_mixed/" in lines[0]
    a, b = infos
    for k in ("block_threads", "sys_per_batch", "group_chunks"):
        assert a[k] == b[k]
    assert b["tuned_ms"] == pytest.approx(float(lines[4]), rel=1e-6)
    assert int(lines[1]) == a["block_threads"] and int(lines[2]) == a["sys_per_batch"] and int(lines[3]) == a["group_chunks"]


def test_ragged_plan_keeps_its_checked_offsets(dev):
    """The plan evaluates the offsets it checked: overwriting the caller's offset
    arrays afterwards (here with zeros, which would empty every system) changes
    nothing."""
    rw = _ragged(500, seed=9)
    plan = _plan(rw, dev)
    before = plan().cpu().numpy()
    plan.obs_off.zero_()
    plan.pl_off.zero_()
    torch.cuda.synchronize()
    after = plan().cpu().numpy()
    assert np.all(np.isfinite(before)) and np.array_equal(before, after)
