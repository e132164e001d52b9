"""Seeded generators: determinism and the distributions stated for each workload."""
import numpy as np

import synth


def _fake_model(t, t0, truth):
    return np.zeros_like(t)


def test_dense_is_deterministic_and_shaped():
    a = synth.with_observations(synth.dense("c1", n_sys=300), _fake_model)
    b = synth.with_observations(synth.dense("c1", n_sys=300), _fake_model)
    for x, y in zip((a.t, a.sigma, a.v, a.P, a.K, a.e, a.w, a.M0), (b.t, b.sigma, b.v, b.P, b.K, b.e, b.w, b.M0)):
        assert np.array_equal(x, y)
    assert a.P.shape == (4, 300) and a.t.shape == (256,)
    assert np.all(np.diff(a.t) >= 0) and a.t.min() >= 2454000 and a.t.max() <= 2457000
    assert np.all(np.diff(a.P, axis=0) >= 0)          # planets sorted by period
    assert a.P.min() >= 1 and a.P.max() <= 1000 and a.K.min() >= 1 and a.K.max() <= 100
    assert a.e.min() >= 0 and a.e.max() <= 0.9
    assert a.sigma.min() >= 1 and a.sigma.max() <= 5
    for k in ("P", "K", "e", "w", "M0"):              # system 0 is the truth
        assert np.array_equal(getattr(a, k)[:, 0], a.truth[k])


def test_dense_configs():
    c0 = synth.dense("c0")
    assert (c0.n_sys, c0.n_pl, c0.n_obs) == (1024, 1, 64) and np.all(c0.sigma == 3.0)
    c4 = synth.dense("c4", n_sys=1000)
    assert c4.e.max() <= 0.8 and c4.offset is not None and np.abs(c4.offset).max() <= 10


def test_log_uniform_period():
    a = synth.dense("c1", n_sys=20000)
    lp = np.log(a.P[:, 1:].ravel())
    # log P uniform on [0, ln 1000]: mean ln(1000)/2
    assert abs(lp.mean() - np.log(1000) / 2) < 0.05


def test_ragged_csr():
    r = synth.ragged(n_sys=5000)
    n_obs, n_pl = r.n_obs, r.n_pl
    assert n_obs.min() >= 16 and n_obs.max() <= 1024 and n_pl.min() >= 1 and n_pl.max() <= 7
    assert r.obs_off[-1] == r.t.size and r.pl_off[-1] == r.P.size
    # mean of round(logU[16, 1024]) is about (1024 - 16) / ln 64 = 242.4
    assert abs(n_obs.mean() - 242.4) < 10
    for i in range(0, 5000, 97):
        seg = r.t[r.obs_off[i]:r.obs_off[i + 1]]
        assert np.all(np.diff(seg) >= 0)
        ps = r.P[r.pl_off[i]:r.pl_off[i + 1]]
        assert np.all(np.diff(ps) >= 0)


def test_kepler_pairs():
    M, e = synth.kepler_pairs(10000)
    assert M.min() >= 0 and M.max() < 2 * np.pi and e.max() <= 0.9
    M, e = synth.kepler_pairs(10000, stress=True)
    assert e.min() >= 0.9 and e.max() <= 0.99
    near = np.minimum(M, 2 * np.pi - M)
    assert near.max() <= 1.0 + 1e-12
