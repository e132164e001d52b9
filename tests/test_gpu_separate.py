"""GPU parity of the separate-function form (per-planet velocities written to
device memory, then planet sums and chi-square) with the oracle, and with the
fused kernel.  Mixed precision: velocities within 1e-3 m/s, chi2 relative 1e-5."""
import numpy as np
import pytest
import torch

import oracle
import paper_0812_2976_amd as kp
from tests import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", [dict(n_sys=300, n_obs=256, n_pl=4), dict(n_sys=77, n_obs=100, n_pl=7),
                                  dict(n_sys=50, n_obs=1000, n_pl=2)])
def test_planet_velocities_match_oracle(dev, case):
    wl = W.dense("c1", n_sys=case["n_sys"], n_obs=case["n_obs"], n_pl=case["n_pl"])
    g = W.to_gpu(wl, dev)
    dv = kp.rv_planet_velocities(g["t"], g["P"], g["K"], g["e"], g["omega"], g["M0"]).cpu().numpy()
    assert dv.shape == (wl.n_pl, wl.n_sys, wl.n_obs) and dv.dtype == np.float32
    worst = 0.0
    for i in range(0, wl.n_sys, max(1, wl.n_sys // 25)):
        for j in range(wl.n_pl):
            ref = np.array([oracle.planet_rv(t, wl.t0, wl.P[j, i], wl.K[j, i], wl.e[j, i], wl.w[j, i], wl.M0[j, i])
                            for t in wl.t])
            worst = max(worst, np.max(np.abs(dv[j, i].astype(np.float64) - ref)))
    print(f"[planet velocities {case}] max |dv| {worst:.3e} m/s", flush=True)
    assert worst <= 1e-3


def test_separate_chisq_matches_oracle_and_fused(dev):
    wl = W.dense("c4", n_sys=1500, jitter=True)
    g = W.to_gpu(wl, dev)
    dv = kp.rv_planet_velocities(g["t"], g["P"], g["K"], g["e"], g["omega"], g["M0"])
    sep = kp.rv_chisq_from_velocities(g["t"], g["v"], g["sigma"], dv, g["offset"], g["jitter"]).cpu().numpy()
    ref = W.oracle_par(oracle.chisq, W.oracle_dense(wl), wl.n_sys)
    fused = kp.rv_chisq(**g, prec="mixed").cpu().numpy()
    print(f"[separate chi2] max rel vs oracle {W.rel_err_chi2(sep, ref).max():.3e}, "
          f"vs fused {W.rel_err_chi2(sep, fused).max():.3e}", flush=True)
    assert W.rel_err_chi2(sep, ref).max() <= 1e-5
    assert W.rel_err_chi2(sep, fused).max() <= 2e-5


def test_separate_domain_nan(dev):
    wl = W.dense("c1", n_sys=20, n_obs=40, n_pl=2)
    wl.e[1, 7] = 1.2
    g = W.to_gpu(wl, dev)
    dv = kp.rv_planet_velocities(g["t"], g["P"], g["K"], g["e"], g["omega"], g["M0"])
    assert torch.isnan(dv[:, 7]).all() and torch.isfinite(dv[:, 6]).all()
    chi2 = kp.rv_chisq_from_velocities(g["t"], g["v"], g["sigma"], dv).cpu().numpy()
    assert np.isnan(chi2[7]) and np.all(np.isfinite(np.delete(chi2, 7)))


def test_separate_rejects_long_series(dev):
    wl = W.dense("c1", n_sys=2, n_obs=1100, n_pl=1)
    g = W.to_gpu(wl, dev)
    dv = torch.zeros((1, 2, 1100), dtype=torch.float32, device=dev)
    with pytest.raises(kp.KeplerError, match="1024"):
        kp.rv_chisq_from_velocities(g["t"], g["v"], g["sigma"], dv)


# ------------------------------------------------------------------ Kepler's equation only
def _anomaly_ref(wl, i, j):
    """Oracle mean anomalies in [0, 2 pi) and their Kepler roots for planet j of system i."""
    M = np.array([oracle.mean_anomaly(t, wl.t0, wl.P[j, i], wl.M0[j, i]) for t in wl.t])
    e = np.full_like(M, wl.e[j, i])
    return M, e, oracle.kepler(M, e)


@pytest.mark.parametrize("case", [dict(n_sys=200, n_obs=256, n_pl=4), dict(n_sys=60, n_obs=100, n_pl=7),
                                  dict(n_sys=40, n_obs=1000, n_pl=2), dict(n_sys=33, n_obs=1, n_pl=1)])
def test_eccentric_anomalies_match_oracle(dev, case):
    """E for every (planet, system, observation) against the oracle's root for the
    oracle's binary64 mean anomaly, modulo 2 pi: within the binary32 Kepler bound
    plus 1e-8 rad / (1 - e cos E) for the two binary64 phases (each within a few
    ulp of q ~ 2.5e6 cycles, 4.4e-9 rad)."""
    wl = W.dense("c1", n_sys=case["n_sys"], n_obs=case["n_obs"], n_pl=case["n_pl"])
    g = W.to_gpu(wl, dev)
    E = kp.rv_eccentric_anomalies(g["t"], g["P"], g["K"], g["e"], g["omega"], g["M0"], t0=wl.t0).cpu().numpy()
    assert E.shape == (wl.n_pl, wl.n_sys, wl.n_obs) and E.dtype == np.float32
    assert np.all(np.abs(E) <= np.pi + 1e-6)                 # [-pi, pi] up to the rounding of E
    worst = 0.0
    for i in range(0, wl.n_sys, max(1, wl.n_sys // 20)):
        for j in range(wl.n_pl):
            M, e, ref = _anomaly_ref(wl, i, j)
            d = np.remainder(E[j, i].astype(np.float64) - ref + np.pi, 2 * np.pi) - np.pi
            tol = W.kepler_tol_mixed(M, e, ref) + 1e-8 / (1.0 - e * np.cos(ref))
            worst = max(worst, float(np.max(np.abs(d) / tol)))
            assert np.all(np.abs(d) <= tol), (i, j)
    print(f"[eccentric anomalies {case}] max |dE| / bound {worst:.3f}", flush=True)


def test_eccentric_anomalies_consistent_with_velocities(dev):
    """The velocities of the separate form follow from the written E by the
    closed form K [cos(w + f) + e cos w] (Eq. 3) evaluated in binary64."""
    wl = W.dense("c1", n_sys=100, n_obs=256, n_pl=3)
    g = W.to_gpu(wl, dev)
    E = kp.rv_eccentric_anomalies(g["t"], g["P"], g["K"], g["e"], g["omega"], g["M0"]).cpu().numpy()
    dv = kp.rv_planet_velocities(g["t"], g["P"], g["K"], g["e"], g["omega"], g["M0"]).cpu().numpy()
    E = E.astype(np.float64)
    e, K, w = wl.e[:, :, None], wl.K[:, :, None], wl.w[:, :, None]
    f = 2.0 * np.arctan2(np.sqrt(1.0 + e) * np.sin(E / 2), np.sqrt(1.0 - e) * np.cos(E / 2))
    v = K * (np.cos(w + f) + e * np.cos(w))
    assert np.max(np.abs(v - dv)) <= 1e-3


def test_eccentric_anomalies_domain_and_empty(dev):
    wl = W.dense("c1", n_sys=20, n_obs=40, n_pl=2)
    wl.e[1, 7] = 1.2
    wl.t = wl.t.copy()
    wl.t[5] = np.nan
    g = W.to_gpu(wl, dev)
    E = kp.rv_eccentric_anomalies(g["t"], g["P"], g["K"], g["e"], g["omega"], g["M0"])
    assert torch.isnan(E[:, 7]).all()
    assert torch.isnan(E[:, :, 5]).all()
    keep = torch.ones(40, dtype=torch.bool)
    keep[5] = False
    assert torch.isfinite(E[:, 6][:, keep]).all()
    empty = torch.empty(0, dtype=torch.float64, device=dev)
    assert kp.rv_eccentric_anomalies(empty, g["P"], g["K"], g["e"], g["omega"], g["M0"]).shape == (2, 20, 0)
