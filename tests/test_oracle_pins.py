"""Pins of the CPU oracle against what the paper and mathematics fix (no GPU).

Each test names the passage it follows.  None of them re-types the oracle's
formula: they check closed forms, special cases, invariants, brute force and
an independent high-precision formula (tests/mp_reference.py).
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.special import jv

import oracle
import synth
from tests import mp_reference as mpr

TWO_PI = 2.0 * math.pi


# ---------------------------------------------------------------- Kepler, Eq. 1
def test_kepler_residual_at_roundoff():
    """Eq. 1: the residual E - e sin E - M, evaluated in 40 digits, is at binary64 roundoff."""
    rng = np.random.default_rng(1)
    M = rng.uniform(0.0, TWO_PI, 300)
    e = np.concatenate([rng.uniform(0.0, 0.99, 250), rng.uniform(0.99, 0.999999, 50)])
    E = oracle.kepler(M, e)
    for Mi, ei, Ei in zip(M, e, E):
        res = mp.mpf(Ei) - mp.mpf(ei) * mp.sin(mp.mpf(Ei)) - mp.mpf(Mi)
        # |g| <= 1 ulp of the larger operand plus the rounding of E times g'(E)
        scale = max(abs(Mi), abs(Ei), 1e-300)
        assert abs(res) <= 2.0 * np.spacing(scale) + 1e-300, (Mi, ei, Ei, res)


def test_kepler_matches_bisection_brute_force():
    """Eq. 1: 200-halving bisection in 40 digits on [M-e, M+e] gives the same root."""
    rng = np.random.default_rng(2)
    M = np.concatenate([rng.uniform(0, TWO_PI, 40), [1e-9, 1e-6, 3.14159, 6.2831]])
    e = np.concatenate([rng.uniform(0, 0.99, 40), [0.99, 0.95, 0.5, 0.9]])
    E = oracle.kepler(M, e)
    for Mi, ei, Ei in zip(M, e, E):
        Eb = mpr.kepler_bisect(Mi, ei)
        # root is well conditioned: |dE| <= |dM| / (1 - e cos E); binary64 rounding of E
        assert abs(mp.mpf(Ei) - Eb) <= 2.0 * np.spacing(max(abs(Ei), 1e-300)) + 4e-16 * abs(Mi) / (1 - ei), (Mi, ei)


def test_kepler_e_zero_is_identity():
    """Eq. 1 with e = 0: E = M exactly."""
    M = np.linspace(-10, 10, 101)
    assert np.array_equal(oracle.kepler(M, np.zeros_like(M)), M)


@pytest.mark.parametrize("e", [0.0, 0.1, 0.5, 0.9, 0.99, 0.999])
def test_kepler_fixed_points(e):
    """Eq. 1: M = 0 gives E = 0 and M = pi gives E = pi for every e (sin E = 0)."""
    assert oracle.kepler(0.0, e)[()] == 0.0
    assert abs(oracle.kepler(math.pi, e)[()] - math.pi) <= 4.5e-16


def test_kepler_symmetry():
    """Eq. 1 is odd about M = pi: E(2 pi - M) = 2 pi - E(M)."""
    rng = np.random.default_rng(3)
    M = rng.uniform(0, math.pi, 500)
    e = rng.uniform(0, 0.99, 500)
    E1 = oracle.kepler(M, e)
    E2 = oracle.kepler(TWO_PI - M, e)
    assert np.max(np.abs(E2 - (TWO_PI - E1))) < 2e-14


def test_kepler_bessel_series():
    """Eq. 1 classical series: E = M + sum_n (2/n) J_n(n e) sin(n M), convergent for e < 0.6627."""
    rng = np.random.default_rng(4)
    M = rng.uniform(0, TWO_PI, 200)
    e = rng.uniform(0, 0.6, 200)
    n = np.arange(1, 121)[:, None]
    series = M + np.sum(2.0 / n * jv(n, n * e) * np.sin(n * M), axis=0)
    assert np.max(np.abs(oracle.kepler(M, e) - series)) < 5e-14


def test_kepler_implicit_derivatives():
    """Implicit-function derivatives used by the adjoint: dE/dM = 1/(1 - e cos E),
    dE/de = sin E / (1 - e cos E) (central differences of the oracle)."""
    rng = np.random.default_rng(5)
    M = rng.uniform(0.2, 6.0, 50)
    e = rng.uniform(0.0, 0.9, 50)
    E = oracle.kepler(M, e)
    h = 1e-6
    dEdM = (oracle.kepler(M + h, e) - oracle.kepler(M - h, e)) / (2 * h)
    dEde = (oracle.kepler(M, e + h) - oracle.kepler(M, e - h)) / (2 * h)
    D = 1 - e * np.cos(E)
    assert np.max(np.abs(dEdM - 1 / D)) < 1e-7
    assert np.max(np.abs(dEde - np.sin(E) / D)) < 1e-7


def test_kepler_domain_nan():
    """Outside e in [0, 1) or for non-finite M the root is undefined: NaN."""
    out = oracle.kepler([1.0, 1.0, 1.0, np.nan, np.inf], [1.0, -0.1, np.nan, 0.5, 0.5])
    assert np.all(np.isnan(out))


# ------------------------------------------------------- mean anomaly, Eq. 4, 6
def test_phase_at_epoch_is_m0():
    """Eq. 4: at t = t0 the mean anomaly is M0 (the mean anomaly at the epoch)."""
    for M0 in (0.0, 0.3, 3.0, 6.2):
        assert oracle.mean_anomaly(2455000.0, 2455000.0, 7.3, M0) == pytest.approx(M0, abs=1e-15)


def test_phase_whole_orbits_return_to_m0():
    """Eq. 4 / Eq. 6: after a whole number of periods (exactly representable P and t),
    the bracket t/P - floor(t/P) is exactly 0 and M = M0."""
    for P, n in ((2.5, 982000), (0.75, 3272000), (1024.0, 2399)):
        t = P * n
        assert oracle.mean_anomaly(t, 0.0, P, 1.25) == pytest.approx(1.25, abs=1e-15)


def test_phase_half_orbit_and_sign_of_m0():
    """Eq. 4: half a period later M advances by pi; M0 enters with a plus sign
    (the reading of Eq. 4 over the -M0 printed in Eq. 6)."""
    P = 2.5
    t = P * 982000 + P / 2
    assert oracle.mean_anomaly(t, 0.0, P, 0.0) == pytest.approx(math.pi, abs=1e-12)
    a = oracle.mean_anomaly(2455123.4, 0.0, 17.0, 0.0)
    b = oracle.mean_anomaly(2455123.4, 0.0, 17.0, 0.25)
    assert (b - a) % TWO_PI == pytest.approx(0.25, abs=1e-12)


def test_phase_uses_binary64_bracket():
    """Sec. 5.1: the bracket is computed in double; the oracle's M is 2 pi times the
    fractional part of the binary64 quotient (checked in 40 digits)."""
    rng = np.random.default_rng(6)
    for _ in range(50):
        t = rng.uniform(2454000, 2457000)
        P = math.exp(rng.uniform(0, math.log(1000)))
        M0 = rng.uniform(0, TWO_PI)
        ref = mpr.mean_anomaly(t, 0.0, P, M0)
        assert abs(oracle.mean_anomaly(t, 0.0, P, M0) - ref) < 2e-15


# ------------------------------------------------------------- velocity, Eq. 3
def test_rv_circular_orbit_is_sinusoid():
    """Eq. 3 with e = 0: E = f = M, so v = K cos(omega + M), a pure sinusoid."""
    rng = np.random.default_rng(7)
    for _ in range(50):
        t, P, K = rng.uniform(2454000, 2457000), rng.uniform(1, 1000), rng.uniform(1, 100)
        w, M0 = rng.uniform(0, TWO_PI, 2)
        M = oracle.mean_anomaly(t, 0.0, P, M0)
        assert oracle.planet_rv(t, 0.0, P, K, 0.0, w, M0) == pytest.approx(K * math.cos(w + M), abs=1e-12)


def test_rv_periapsis_apoapsis_quadrature_closed_forms():
    """Eq. 3 at special points: periapsis (M=0, f=0) v = K(1+e)cos w; apoapsis (M=pi)
    v = -K(1-e)cos w; E = pi/2 (M = pi/2 - e) v = -K sqrt(1-e^2) sin w."""
    P, t = 2.5, 2.5 * 982000
    for e in (0.0, 0.3, 0.8, 0.97):
        for w in (0.1, 2.0, 4.0):
            K = 37.0
            assert oracle.planet_rv(t, 0.0, P, K, e, w, 0.0) == pytest.approx(K * (1 + e) * math.cos(w), abs=1e-12)
            assert oracle.planet_rv(t + P / 2, 0.0, P, K, e, w, 0.0) == pytest.approx(-K * (1 - e) * math.cos(w), abs=1e-10)
            vq = oracle.planet_rv(t, 0.0, P, K, e, w, math.pi / 2 - e)
            assert vq == pytest.approx(-K * math.sqrt(1 - e * e) * math.sin(w), abs=1e-11)


def test_rv_matches_eccentric_anomaly_form():
    """Eq. 3: the oracle's true-anomaly form equals the eccentric-anomaly form
    computed in 40 digits with a bisection root (independent code)."""
    rng = np.random.default_rng(8)
    for _ in range(60):
        t = rng.uniform(2454000, 2457000)
        P = math.exp(rng.uniform(0, math.log(1000)))
        K = rng.uniform(1, 100)
        e = rng.uniform(0, 0.99)
        w, M0 = rng.uniform(0, TWO_PI, 2)
        ref = mpr.planet_rv_eform(t, 0.0, P, K, e, w, M0)
        assert abs(oracle.planet_rv(t, 0.0, P, K, e, w, M0) - ref) < 1e-12 * K / (1 - e)


@pytest.mark.parametrize("e", [0.0, 0.2, 0.6, 0.9])
def test_rv_orbit_average_is_zero(e):
    """Eq. 3: the velocity averages to zero over one orbit in time (uniform mean
    anomaly).  A wrong e cos(omega) term would leave a mean of K e cos(omega)."""
    P, K, w = 4.0, 50.0, 1.1
    n = 4096
    t = P * 600000 + P * np.arange(n) / n     # exactly spaced in binary64
    v = np.array([oracle.planet_rv(ti, 0.0, P, K, e, w, 0.3) for ti in t])
    assert abs(v.mean()) < 1e-9 * K
    assert v.max() <= K * (1 + e * math.cos(w)) + 1e-9
    assert v.min() >= K * (e * math.cos(w) - 1) - 1e-9


# ----------------------------------------------------------------- chi2, Eq. 5
def _small_dense(n_sys=6, n_pl=3, n_obs=40, seed=11, jitter=False, offset=False):
    wl = synth.dense("c1", n_sys=n_sys, seed=seed, jitter=jitter)
    wl.P, wl.K, wl.e, wl.w, wl.M0 = (x[:n_pl] for x in (wl.P, wl.K, wl.e, wl.w, wl.M0))
    wl.truth = {k: v[:n_pl] for k, v in wl.truth.items()}
    wl.t, wl.sigma, wl.noise = wl.t[:n_obs], wl.sigma[:n_obs], wl.noise[:n_obs]
    if offset:
        wl.offset = np.random.default_rng(seed).uniform(-10, 10, n_sys)
    return wl


def _mp_model(t, t0, truth, K_scale=1.0):
    out = []
    for ti in t:
        s = mp.mpf(0)
        for j in range(len(truth["P"])):
            s += mpr.planet_rv_eform(ti, t0, truth["P"][j], truth["K"][j], truth["e"][j], truth["w"][j], truth["M0"][j])
        out.append(float(s))
    return np.array(out)


def _dense(wl):
    return oracle.Dense(wl.t, wl.v, wl.sigma, wl.P, wl.K, wl.e, wl.w, wl.M0, wl.offset, wl.jitter, wl.t0)


def test_chisq_noise_free_truth_is_zero():
    """Eq. 5: data generated noise-free (by the independent 40-digit model) from the
    true parameters give chi2 = 0 for the truth system, to rounding of the data."""
    wl = _small_dense(n_obs=24)
    synth.with_observations(wl, _mp_model, noise_free=True)
    chi2 = oracle.chisq(_dense(wl))
    # each residual is within the binary64 rounding of the data, |r| <= 1e-13 m/s
    assert chi2[0] < wl.n_obs * (1e-13) ** 2 * np.max(1 / wl.sigma ** 2)
    assert np.all(chi2[1:] > 1.0)


def test_chisq_constant_residual_and_sigma_scaling():
    """Eq. 5: data = model - c gives chi2 = c^2 sum_k w_k; sigma -> a sigma divides chi2 by a^2."""
    wl = _small_dense(n_obs=30)
    model = oracle.rv_model(oracle.Dense(wl.t, np.zeros_like(wl.t), wl.sigma, wl.P, wl.K, wl.e, wl.w, wl.M0))
    c = 2.5
    for i in range(wl.n_sys):
        d = oracle.Dense(wl.t, model[i] - c, wl.sigma, wl.P[:, i:i + 1], wl.K[:, i:i + 1], wl.e[:, i:i + 1],
                         wl.w[:, i:i + 1], wl.M0[:, i:i + 1])
        assert oracle.chisq(d)[0] == pytest.approx(c * c * np.sum(1 / wl.sigma ** 2), rel=1e-12)
    wl.v = model[0] + wl.noise
    a = 1.7
    base = oracle.chisq(_dense(wl))
    wl.sigma = wl.sigma * a
    assert np.allclose(oracle.chisq(_dense(wl)), base / a ** 2, rtol=1e-13)


def test_chisq_jitter_and_offset():
    """Eq. 5: jitter s adds in quadrature, w = 1/(sigma^2 + s^2); an offset gamma shifts
    the model, so shifting the data by gamma leaves chi2 unchanged."""
    wl = _small_dense(n_obs=30, jitter=True)
    synth.with_observations(wl, _mp_model)
    with_j = oracle.chisq(_dense(wl))
    for i in range(wl.n_sys):
        sig_eff = np.sqrt(wl.sigma ** 2 + wl.jitter[i] ** 2)
        d = oracle.Dense(wl.t, wl.v, sig_eff, wl.P[:, i:i + 1], wl.K[:, i:i + 1], wl.e[:, i:i + 1],
                         wl.w[:, i:i + 1], wl.M0[:, i:i + 1])
        assert oracle.chisq(d)[0] == pytest.approx(with_j[i], rel=1e-13)
    wl.jitter = None
    base = oracle.chisq(_dense(wl))
    g = np.linspace(-7, 9, wl.n_sys)
    wl.offset = g
    wl.v = None
    for i in range(wl.n_sys):
        d = oracle.Dense(wl.t, _mp_model(wl.t, 0.0, wl.truth) + wl.noise + g[i], wl.sigma,
                         wl.P, wl.K, wl.e, wl.w, wl.M0, g, None)
        assert oracle.chisq(d, i, i + 1)[i] == pytest.approx(base[i], rel=1e-11)


def test_chisq_domain_isolates_nan():
    """Domain (e in [0,1), P > 0, finite inputs, sigma >= 0 with sigma^2 + s^2 > 0):
    a bad system gets NaN and its neighbours are untouched."""
    wl = _small_dense(n_sys=8, n_obs=20)
    synth.with_observations(wl, _mp_model)
    base = oracle.chisq(_dense(wl))
    wl.e[1, 2] = 1.0
    wl.e[0, 3] = -0.1
    wl.P[2, 4] = 0.0
    wl.M0[0, 5] = np.nan
    out = oracle.chisq(_dense(wl))
    assert np.all(np.isnan(out[2:6]))
    assert np.array_equal(out[[0, 1, 6, 7]], base[[0, 1, 6, 7]])
    wl2 = _small_dense(n_sys=3, n_obs=20)
    synth.with_observations(wl2, _mp_model)
    wl2.sigma[3] = 0.0
    assert np.all(np.isnan(oracle.chisq(_dense(wl2))))
    wl2.jitter = np.array([0.0, 1.0, 2.0])
    out = oracle.chisq(_dense(wl2))
    assert np.isnan(out[0]) and np.all(np.isfinite(out[1:]))


# ------------------------------------------------------------ gradient (Sec. 6)
def test_grad_offset_and_amplitude_closed_forms():
    """Gradient of Eq. 5: d chi2/d gamma = 2 sum w r; chi2 is quadratic in the model,
    which is linear in K_j, so d chi2/d K_j = (2/K_j) sum w r v_j."""
    wl = _small_dense(n_sys=4, n_pl=2, n_obs=30, offset=True)
    synth.with_observations(wl, _mp_model)
    d = _dense(wl)
    chi2, grad = oracle.chisq_grad(d)
    model = oracle.rv_model(d)
    w = 1 / wl.sigma ** 2
    for i in range(wl.n_sys):
        r = model[i] - wl.v
        assert grad[-1, i] == pytest.approx(2 * np.sum(w * r), rel=1e-12, abs=1e-9)
        for j in range(wl.n_pl):
            vj = np.array([oracle.planet_rv(tk, 0.0, wl.P[j, i], wl.K[j, i], wl.e[j, i], wl.w[j, i], wl.M0[j, i])
                           for tk in wl.t])
            assert grad[5 * j + 1, i] == pytest.approx(2 / wl.K[j, i] * np.sum(w * r * vj), rel=1e-11)
        assert chi2[i] == pytest.approx(np.sum(w * r * r), rel=1e-13)


def test_grad_matches_central_differences():
    """Gradient of Eq. 5 against binary64 central differences of the oracle's chi2.
    The period step moves the latest phase by ~1e-6 rad (epoch at mid-baseline)."""
    wl = _small_dense(n_sys=5, n_pl=2, n_obs=30, offset=True)
    wl.t0 = 2455500.0
    synth.with_observations(wl, _mp_model)
    d = _dense(wl)
    _, grad = oracle.chisq_grad(d)
    span = np.max(np.abs(wl.t - wl.t0))
    names = ("P", "K", "e", "w", "M0")
    for i in range(wl.n_sys):
        for j in range(wl.n_pl):
            for a, nm in enumerate(names):
                x0 = getattr(wl, nm)[j, i]
                h = 1e-6 * x0 * x0 / (TWO_PI * span) if nm == "P" else 1e-6 * max(abs(x0), 1.0)
                vals = []
                for s in (+1, -1):
                    arr = getattr(wl, nm).copy()
                    arr[j, i] = x0 + s * h
                    kw = {k: getattr(wl, k) for k in names}
                    kw[nm] = arr
                    dd = oracle.Dense(wl.t, wl.v, wl.sigma, kw["P"], kw["K"], kw["e"], kw["w"], kw["M0"],
                                      wl.offset, None, wl.t0)
                    vals.append(oracle.chisq(dd, i, i + 1)[i])
                fd = (vals[0] - vals[1]) / (2 * h)
                g = grad[5 * j + a, i]
                assert abs(fd - g) <= 2e-5 * max(abs(g), 1.0), (i, j, nm, fd, g)


def test_grad_against_40_digit_derivative():
    """Gradient of Eq. 5 against a 40-digit central difference of an independent
    model (eccentric-anomaly form, exact phase), one system, one planet."""
    t = np.array([2454100.25, 2454630.5, 2455371.75, 2455990.0, 2456712.125])
    sigma = np.array([2.0, 3.0, 1.5, 4.0, 2.5])
    v = np.array([12.0, -31.0, 5.5, 40.0, -8.0])
    p = dict(P=37.25, K=42.0, e=0.61, w=2.3, M0=1.1)
    g_off = 1.5
    d = oracle.Dense(t, v, sigma, [[p["P"]]], [[p["K"]]], [[p["e"]]], [[p["w"]]], [[p["M0"]]], [g_off], None, 0.0)
    chi2, grad = oracle.chisq_grad(d)

    def chi2_mp(**kw):
        q = dict(p)
        q.update(kw)
        s = mp.mpf(0)
        for tk, sk, vk in zip(t, sigma, v):
            m = mpr.planet_rv_exact_phase(tk, 0.0, q["P"], q["K"], q["e"], q["w"], q["M0"]) + mp.mpf(q.get("g", g_off))
            s += (m - vk) ** 2 / mp.mpf(sk) ** 2
        return s

    assert abs(chi2[0] - float(chi2_mp())) < 1e-9 * float(chi2_mp())
    for a, nm in enumerate(("P", "K", "e", "w", "M0")):
        h = mp.mpf("1e-15")
        x0 = mp.mpf(p[nm])
        fd = (chi2_mp(**{nm: x0 + h}) - chi2_mp(**{nm: x0 - h})) / (2 * h)
        # the oracle's phase rounds q to binary64 (Sec. 5.1): relative 1e-9 allowance
        assert abs(grad[a, 0] - float(fd)) <= 1e-8 * abs(float(fd)) + 1e-9, (nm, grad[a, 0], float(fd))
    fd = (chi2_mp(g=mp.mpf(g_off) + mp.mpf("1e-15")) - chi2_mp(g=mp.mpf(g_off) - mp.mpf("1e-15"))) / mp.mpf("2e-15")
    assert abs(grad[5, 0] - float(fd)) <= 1e-10 * abs(float(fd))


def test_grad_zero_at_noise_free_truth():
    """At noise-free truth every residual is zero, so every gradient component is zero."""
    wl = _small_dense(n_sys=2, n_pl=2, n_obs=20)
    synth.with_observations(wl, _mp_model, noise_free=True)
    _, grad = oracle.chisq_grad(_dense(wl))
    assert np.max(np.abs(grad[:, 0])) < 1e-6


# ------------------------------------------- gradient error scales (Sec. 6)
# The scales S_r = sum_k |2 w_k r_k dv_k/dtheta| and S_1 = sum_k 2 w_k |dv_k/dtheta|
# turn a residual error and a relative error per term into a bound on the
# gradient's error; every mixed-precision gradient tolerance is built from them.
def _scales_case(jitter):
    wl = _small_dense(n_sys=4, n_pl=2, n_obs=30, offset=True, jitter=jitter)
    wl.t0 = 2455500.0
    synth.with_observations(wl, _mp_model)
    return wl


@pytest.mark.parametrize("jitter", [False, True])
def test_grad_scales_offset_and_amplitude_closed_forms(jitter):
    """Offset row: dv/dgamma = 1, so S_1 = 2 sum w and S_r = 2 sum w |r|.  K rows:
    the model is linear in K_j (Eq. 3), dv/dK_j = v_j / K_j, so S_1 = (2/K_j) sum w |v_j|
    and S_r = (2/K_j) sum w |r v_j|.  w = 1/(sigma^2 + s^2) (Eq. 5)."""
    wl = _scales_case(jitter)
    d = _dense(wl)
    _, _, s_r, s_1 = oracle.chisq_grad_scales(d)
    model = oracle.rv_model(d)
    for i in range(wl.n_sys):
        s = 0.0 if wl.jitter is None else wl.jitter[i]
        w = 1.0 / (wl.sigma ** 2 + s ** 2)
        r = model[i] - wl.v
        assert s_1[-1, i] == pytest.approx(2 * np.sum(w), rel=1e-13)
        assert s_r[-1, i] == pytest.approx(2 * np.sum(w * np.abs(r)), rel=1e-12)
        for j in range(wl.n_pl):
            vj = np.array([oracle.planet_rv(tk, wl.t0, wl.P[j, i], wl.K[j, i], wl.e[j, i], wl.w[j, i],
                                            wl.M0[j, i]) for tk in wl.t])
            K = wl.K[j, i]
            assert s_1[5 * j + 1, i] == pytest.approx(2 / K * np.sum(w * np.abs(vj)), rel=1e-12)
            assert s_r[5 * j + 1, i] == pytest.approx(2 / K * np.sum(w * np.abs(r * vj)), rel=1e-11)


def test_grad_scales_match_finite_difference_terms():
    """Every row of S_1 and S_r against the per-observation derivatives dv_k/dtheta
    taken by binary64 central differences of one planet's velocity (Eq. 3), with the
    residuals of the oracle's model: a wrong term, weight or row in the scales fails."""
    wl = _scales_case(False)
    d = _dense(wl)
    _, _, s_r, s_1 = oracle.chisq_grad_scales(d)
    model = oracle.rv_model(d)
    w = 1.0 / wl.sigma ** 2
    span = np.max(np.abs(wl.t - wl.t0))
    names = ("P", "K", "e", "w", "M0")
    for i in range(wl.n_sys):
        r = model[i] - wl.v
        for j in range(wl.n_pl):
            par = {nm: getattr(wl, nm)[j, i] for nm in names}
            for a, nm in enumerate(names):
                x0 = par[nm]
                h = 1e-6 * x0 * x0 / (TWO_PI * span) if nm == "P" else 1e-6 * max(abs(x0), 1.0)
                hi, lo = dict(par), dict(par)
                hi[nm], lo[nm] = x0 + h, x0 - h
                dv = np.array([(oracle.planet_rv(tk, wl.t0, hi["P"], hi["K"], hi["e"], hi["w"], hi["M0"]) -
                                oracle.planet_rv(tk, wl.t0, lo["P"], lo["K"], lo["e"], lo["w"], lo["M0"])) / (2 * h)
                               for tk in wl.t])
                assert s_1[5 * j + a, i] == pytest.approx(np.sum(2 * w * np.abs(dv)), rel=2e-6), (i, j, nm)
                assert s_r[5 * j + a, i] == pytest.approx(np.sum(np.abs(2 * w * r * dv)), rel=2e-6), (i, j, nm)


def test_grad_scales_bound_the_gradient():
    """|g| <= S_r componentwise (triangle inequality), with equality where every term
    has one sign: with a large offset every residual is positive, so the offset row
    has g = S_r exactly.  S_1 >= 0 and S_r <= max|r| S_1."""
    wl = _scales_case(True)
    d = _dense(wl)
    _, g, s_r, s_1 = oracle.chisq_grad_scales(d)
    assert np.all(np.abs(g) <= s_r * (1 + 1e-14))
    assert np.all(s_1 > 0)
    model = oracle.rv_model(d)
    rmax = np.max(np.abs(model - wl.v[None, :]), axis=1)
    assert np.all(s_r <= rmax[None, :] * s_1 * (1 + 1e-14))
    wl.offset = wl.offset + 1e4
    _, g, s_r, _ = oracle.chisq_grad_scales(_dense(wl))
    assert np.all(g[-1] > 0)
    assert np.allclose(g[-1], s_r[-1], rtol=1e-13, atol=0)


# ------------------------------------------------------------------ ragged CSR
def test_ragged_equals_per_system_dense():
    """CSR packing changes only the layout: each ragged system equals a dense
    single-system evaluation on its own observations."""
    rw = synth.ragged(n_sys=12, seed=5, n_obs_range=(3, 40))
    rw.v = rw.noise + 1.0
    rw.offset = np.linspace(-3, 3, rw.n_sys)
    out = oracle.chisq_ragged(oracle.Ragged(rw.t, rw.v, rw.sigma, rw.obs_off, rw.P, rw.K, rw.e, rw.w, rw.M0,
                                            rw.pl_off, rw.offset))
    for i in range(rw.n_sys):
        o0, o1 = rw.obs_off[i], rw.obs_off[i + 1]
        p0, p1 = rw.pl_off[i], rw.pl_off[i + 1]
        d = oracle.Dense(rw.t[o0:o1], rw.v[o0:o1], rw.sigma[o0:o1], rw.P[p0:p1, None], rw.K[p0:p1, None],
                         rw.e[p0:p1, None], rw.w[p0:p1, None], rw.M0[p0:p1, None], rw.offset[i:i + 1])
        assert oracle.chisq(d)[0] == out[i]


# ------------------------------------------------- likelihood with jitter (Eq. 5)
def test_nll_single_observation_closed_form_and_optimal_jitter():
    """One observation: -2 ln L = r^2/(sigma^2 + s^2) + ln(sigma^2 + s^2), whose
    derivative in s vanishes at s^2 = r^2 - sigma^2 (the maximum-likelihood jitter)."""
    t = np.array([2455123.25])
    p = dict(P=[[11.3]], K=[[40.0]], e=[[0.3]], w=[[1.0]], M0=[[2.0]])
    v_model = oracle.rv_model(oracle.Dense(t, [0.0], [1.0], *(p[k] for k in ("P", "K", "e", "w", "M0"))))[0, 0]
    v = np.array([v_model - 7.0])              # residual r = model - v = 7
    sigma = np.array([3.0])
    for s in (0.0, 2.0, 5.0):
        d = oracle.Dense(t, v, sigma, *(p[k] for k in ("P", "K", "e", "w", "M0")), jitter=[s])
        nll, grad = oracle.nll_grad(d)
        var = 9.0 + s * s
        assert nll[0] == pytest.approx(49.0 / var + math.log(var), rel=1e-12)
        assert grad[-1, 0] == pytest.approx(2 * s / var - 2 * s * 49.0 / var ** 2, abs=1e-12)
    s_opt = math.sqrt(49.0 - 9.0)
    d = oracle.Dense(t, v, sigma, *(p[k] for k in ("P", "K", "e", "w", "M0")), jitter=[s_opt])
    assert abs(oracle.nll_grad(d)[1][-1, 0]) < 1e-12


def test_nll_matches_chisq_plus_log_terms_and_fd_in_jitter():
    """-2 ln L - chi2 = sum ln(sigma^2 + s^2); the planet and offset rows equal the
    chi-square gradient; d/ds matches central differences."""
    wl = _small_dense(n_sys=5, n_pl=2, n_obs=30, jitter=True, offset=True)
    synth.with_observations(wl, _mp_model)
    d = _dense(wl)
    nll, grad = oracle.nll_grad(d)
    chi2, gchi = oracle.chisq_grad(d)
    for i in range(wl.n_sys):
        assert nll[i] - chi2[i] == pytest.approx(np.sum(np.log(wl.sigma ** 2 + wl.jitter[i] ** 2)), rel=1e-12)
    assert np.allclose(grad[:-1], gchi, rtol=1e-14, atol=0)
    h = 1e-6
    for i in range(wl.n_sys):
        vals = []
        for sgn in (1, -1):
            jit = wl.jitter.copy()
            jit[i] += sgn * h
            dd = oracle.Dense(wl.t, wl.v, wl.sigma, wl.P, wl.K, wl.e, wl.w, wl.M0, wl.offset, jit, wl.t0)
            vals.append(oracle.nll_grad(dd, i, i + 1)[0][i])
        assert (vals[0] - vals[1]) / (2 * h) == pytest.approx(grad[-1, i], rel=1e-6, abs=1e-6)


# ------------------------------------------------- Gauss-Newton products
def _gn_problem(seed=31, n_obs=60, noise=True):
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(2455000.0, 2455400.0, n_obs))
    sigma = rng.uniform(1.0, 3.0, n_obs)
    th = dict(P=[[9.7], [83.0]], K=[[25.0], [12.0]], e=[[0.25], [0.4]], w=[[1.1], [4.0]], M0=[[2.0], [0.7]])
    t0 = 2455200.0
    d0 = oracle.Dense(t, np.zeros(n_obs), sigma, *(np.array(th[k]) for k in ("P", "K", "e", "w", "M0")), [0.8],
                      None, t0)
    v = oracle.rv_model(d0)[0] + (rng.normal(size=n_obs) * sigma if noise else 0.0)
    return t, v, sigma, th, t0


def _flat(th, gam):
    return np.array([th[k][j][0] for j in range(2) for k in ("P", "K", "e", "w", "M0")] + [gam])


def _dense_from(t, v, sigma, theta, t0):
    planes = [np.array([[theta[5 * j + a]] for j in range(2)]) for a in range(5)]
    return oracle.Dense(t, v, sigma, *planes, [theta[-1]], None, t0)


def test_gn_products_match_finite_difference_jacobian():
    """J^T W J from central differences of the oracle's model (an independent route:
    numerical Jacobian and a numpy product) equals the analytic packed matrix;
    J^T W r is half the chi-square gradient."""
    t, v, sigma, th, t0 = _gn_problem()
    theta = _flat(th, 0.8)
    d = _dense_from(t, v, sigma, theta, t0)
    chi2, jtwr, jtwj = oracle.gn(d)
    n = theta.size
    J = np.empty((t.size, n))
    span = np.max(np.abs(t - t0))
    for a in range(n):
        h = 1e-6 * theta[a] ** 2 / (2 * np.pi * span) if a % 5 == 0 and a < n - 1 else 1e-6 * max(abs(theta[a]), 1.0)
        tp, tm = theta.copy(), theta.copy()
        tp[a] += h
        tm[a] -= h
        J[:, a] = (oracle.rv_model(_dense_from(t, v, sigma, tp, t0))[0] -
                   oracle.rv_model(_dense_from(t, v, sigma, tm, t0))[0]) / (2 * h)
    W = 1.0 / sigma ** 2
    ref = J.T @ (W[:, None] * J)
    scale = np.abs(J).T @ (W[:, None] * np.abs(J))
    got = oracle.unpack_sym(jtwj[:, 0], n)
    assert np.max(np.abs(got - ref) / scale) < 1e-6
    _, grad = oracle.chisq_grad(d)
    assert np.allclose(jtwr[:, 0], 0.5 * grad[:, 0], rtol=1e-13, atol=0)
    assert chi2[0] == pytest.approx(oracle.chisq(d)[0], rel=1e-15)
    ev = np.linalg.eigvalsh(got)
    assert ev.min() > -1e-12 * ev.max()


def test_gn_step_converges_quadratically_on_noise_free_data():
    """Noise-free data from theta*: a Gauss-Newton step theta - (J^T W J)^-1 J^T W r from a
    start 1e-4 (relative) away lands within the square of that distance (residuals
    vanish at the solution, so Gauss-Newton is Newton there)."""
    t, v, sigma, th, t0 = _gn_problem(noise=False)
    star = _flat(th, 0.8)
    rng = np.random.default_rng(5)
    scale = np.maximum(np.abs(star), 1.0)
    x0 = star + 1e-4 * scale * rng.normal(size=star.size) * np.where(np.arange(star.size) % 5 == 0, 1e-3, 1.0)
    _, jtwr, jtwj = oracle.gn(_dense_from(t, v, sigma, x0, t0))
    x1 = x0 - np.linalg.solve(oracle.unpack_sym(jtwj[:, 0], star.size), jtwr[:, 0])
    e0 = np.max(np.abs(x0 - star) / scale)
    e1 = np.max(np.abs(x1 - star) / scale)
    assert e1 < 100 * e0 ** 2 + 1e-12, (e0, e1)
