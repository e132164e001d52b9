"""Pins of the oracle's population sampler (DE-MC, ter Braak 2006; the many-chain
MCMC the paper targets, Sec. 6) and of its counter-based generator (no GPU).

* Philox-4x32-10 against the published known-answer vectors (tests/golden).
* The sampler's stationary distribution: on a high signal-to-noise one-planet
  problem with noise-free data the posterior of exp(-chi2/2) is Gaussian about
  the truth with covariance (J^T W J)^-1 (Laplace); J comes from central
  differences of the oracle's velocity model, independent of the sampler.
* The proposal structure on a flat target (no observations: chi2 = 0, every
  proposal inside the prior support is accepted): each move is gam times the
  difference of two distinct chains of the OTHER half, found by brute force.
* Prior support: chains never leave P > 0, K >= 0, 0 <= e < 1.
"""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [ln for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for ln in rows:
        ctr, key, out = ([int(w, 16) for w in part.split()] for part in ln.split("|"))
        assert list(oracle.philox4x32_10(ctr, key)) == out


def _one_planet_problem(n_obs=40, seed=7):
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(2455000.0, 2455200.0, n_obs))
    t0 = 2455100.0
    sigma = np.ones(n_obs)
    theta = np.array([12.3, 30.0, 0.2, 1.0, 2.0, 0.5])      # P, K, e, omega, M0, gamma

    def model(th):
        d = oracle.Dense(t, np.zeros(n_obs), sigma, [[th[0]]], [[th[1]]], [[th[2]]], [[th[3]]], [[th[4]]],
                         [th[5]], None, t0)
        return oracle.rv_model(d)[0]

    J = np.empty((n_obs, 6))
    for a in range(6):
        h = 1e-7 if a == 0 else 1e-6 * max(abs(theta[a]), 1.0)
        tp, tm = theta.copy(), theta.copy()
        tp[a] += h
        tm[a] -= h
        J[:, a] = (model(tp) - model(tm)) / (2 * h)
    C = np.linalg.inv(J.T @ J / 1.0 ** 2)
    return rng, t, t0, sigma, theta, model(theta), C


def test_demc_samples_the_laplace_posterior():
    rng, t, t0, sigma, theta, v, C = _one_planet_problem()
    sd = np.sqrt(np.diag(C))
    nh = 32
    x = rng.multivariate_normal(theta, C, size=(2, nh)).transpose(0, 2, 1).copy()
    chi = oracle.demc_init_chisq(t, v, sigma, x, 1, t0=t0)
    assert np.all(np.isfinite(chi))
    eps = 1e-3 * sd
    samples, acc, g = [], None, 0
    for k in range(220):
        x, chi, acc = oracle.demc_run(t, v, sigma, x, chi, 1, eps, seed=12345, gen0=g, n_gen=5, t0=t0,
                                      jump_every=10, n_accept=acc)
        g += 5
        if k >= 20:
            samples.append(x.transpose(0, 2, 1).reshape(-1, 6).copy())
    S = np.concatenate(samples)
    rate = acc.sum() / (2 * nh * g)
    ratio = np.var(S, axis=0) / np.diag(C)
    Cs = np.cov(S.T)
    R = Cs / np.sqrt(np.outer(np.diag(Cs), np.diag(Cs)))
    R0 = C / np.outer(sd, sd)
    print(f"acceptance {rate:.3f}; variance ratios {np.round(ratio, 3)}; max |dcorr| {np.max(np.abs(R - R0)):.3f}")
    assert 0.1 < rate < 0.6
    assert np.all((ratio > 0.85) & (ratio < 1.15))
    assert np.max(np.abs(R - R0)) < 0.06
    assert np.all(np.abs(S.mean(0) - theta) < 0.3 * sd)
    # the stored chi-square is the chi-square of the stored state
    assert np.allclose(oracle.demc_init_chisq(t, v, sigma, x, 1, t0=t0), chi, rtol=1e-14, atol=0)


def _flat_population(nh, n_pl, rng):
    d = 5 * n_pl + 1
    x = np.empty((2, d, nh))
    lo_hi = [(5.0, 6.0), (20.0, 30.0), (0.3, 0.4), (0.0, 6.0), (0.0, 6.0)]
    for a, (lo, hi) in enumerate(lo_hi):
        x[:, a * n_pl:(a + 1) * n_pl, :] = rng.uniform(lo, hi, size=(2, n_pl, nh))
    x[:, 5 * n_pl, :] = rng.uniform(-1.0, 1.0, size=(2, nh))
    return x


def _moves_are_other_half_differences(x_old_h, x_new_h, pool, gam):
    """Every chain's move equals gam (pool[a] - pool[b]) for some a != b."""
    nh = pool.shape[1]
    diffs = gam * (pool[:, :, None] - pool[:, None, :])          # [d, a, b]
    for i in range(nh):
        mv = x_new_h[:, i] - x_old_h[:, i]
        err = np.max(np.abs(diffs - mv[:, None, None]) / (np.abs(pool).max(axis=1)[:, None, None] + 1e-300), axis=0)
        np.fill_diagonal(err, np.inf)
        assert err.min() < 1e-13, (i, err.min())


@pytest.mark.parametrize("jump_every,gam", [(0, 0.5), (1, 1.0)])
def test_demc_flat_target_moves(jump_every, gam):
    rng = np.random.default_rng(11)
    nh, n_pl = 8, 2
    x0 = _flat_population(nh, n_pl, rng)
    none = np.empty(0)
    chi = np.zeros((2, nh))
    d = 5 * n_pl + 1
    x1, chi1, acc = oracle.demc_run(none, none, none, x0, chi, n_pl, np.zeros(d), seed=99, gen0=3, n_gen=1,
                                    gamma=0.5, jump_every=jump_every)
    assert np.all(acc == 1) and np.all(chi1 == 0.0)
    _moves_are_other_half_differences(x0[0], x1[0], x0[1], gam)     # half 0 from the old half 1
    _moves_are_other_half_differences(x0[1], x1[1], x1[0], gam)     # half 1 from the new half 0


def test_demc_stays_in_prior_support():
    """Flat target, population pressed against K = 0 and e = 0: proposals leave the
    support often and must all be rejected."""
    rng = np.random.default_rng(12)
    nh, n_pl = 16, 1
    x = _flat_population(nh, n_pl, rng)
    x[:, 1, :] = rng.uniform(0.0, 0.5, size=(2, nh))       # K
    x[:, 2, :] = rng.uniform(0.0, 0.02, size=(2, nh))      # e
    none = np.empty(0)
    x1, _, acc = oracle.demc_run(none, none, none, x, np.zeros((2, nh)), n_pl, np.full(6, 0.05), seed=5,
                                 gen0=0, n_gen=60)
    assert np.all(x1[:, 1, :] >= 0.0) and np.all(x1[:, 2, :] >= 0.0) and np.all(x1[:, 2, :] < 1.0)
    assert np.all(x1[:, 0, :] > 0.0)
    assert 0 < acc.sum() < 2 * nh * 60                      # some rejected, some accepted


def test_demc_margin_trace_matches_decisions():
    """The recorded margin (chi2(x) - chi2(y)) - 2 ln u is positive exactly for
    the chains that moved."""
    rng, t, t0, sigma, theta, v, C = _one_planet_problem()
    x = rng.multivariate_normal(theta, 4 * C, size=(2, 16)).transpose(0, 2, 1).copy()
    chi = oracle.demc_init_chisq(t, v, sigma, x, 1, t0=t0)
    x1, _, acc, mg = oracle.demc_run(t, v, sigma, x, chi, 1, 1e-3 * np.sqrt(np.diag(C)), seed=3, gen0=0, n_gen=1,
                                     t0=t0, margin=True)
    moved = np.any(x1 != x, axis=1)
    assert np.array_equal(moved, mg > 0) and np.array_equal(acc == 1, moved)
