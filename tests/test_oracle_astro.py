"""Pins of the oracle's astrometric Keplerian model (Thiele-Innes form; the larger
dynamic-range application of the same phase and Kepler core, Sec. 5.1).  None
re-types the oracle: closed forms of the orbit geometry with an independent
40-digit Kepler root, the orbit average, the circular orbit, linearity and
chi-square identities."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from tests import mp_reference as mpr

TWO_PI = 2.0 * math.pi


def _one(t, P, e, M0, A, B, F, G, x0=None, y0=None, t0=0.0, x=None, y=None, sx=None, sy=None):
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    n = t.size
    z = np.zeros(n)
    return oracle.Astro(t, z if x is None else x, z if y is None else y, np.ones(n) if sx is None else sx,
                        np.ones(n) if sy is None else sy, [[P]], [[e]], [[M0]], [[A]], [[B]], [[F]], [[G]],
                        x0, y0, t0)


def test_face_on_orbit_is_the_keplerian_ellipse():
    """Face-on orbit (i = 0, omega = Omega = 0: A = G = a, B = F = 0): Dec = r cos f and
    RA = r sin f with r = a (1 - e cos E) and f the true anomaly, E from a 40-digit
    bisection of Eq. 1 (independent of the oracle's root finder)."""
    rng = np.random.default_rng(21)
    a = 37.5
    for _ in range(40):
        P, e, M0 = math.exp(rng.uniform(0, math.log(2000))), rng.uniform(0, 0.95), rng.uniform(0, TWO_PI)
        t = rng.uniform(2454000, 2457000)
        xy = oracle.astro_model(_one(t, P, e, M0, a, 0.0, 0.0, a))[0, :, 0]
        E = mpr.kepler_bisect(mpr.mean_anomaly(t, 0.0, P, M0), e)
        r = a * (1 - e * mp.cos(E))
        f = 2 * mp.atan2(mp.sqrt(1 + e) * mp.sin(E / 2), mp.sqrt(1 - e) * mp.cos(E / 2))
        assert xy[0] == pytest.approx(float(r * mp.sin(f)), abs=1e-11 * a / (1 - e))
        assert xy[1] == pytest.approx(float(r * mp.cos(f)), abs=1e-11 * a / (1 - e))


@pytest.mark.parametrize("e", [0.0, 0.3, 0.7, 0.95])
def test_orbit_average_is_minus_three_halves_e(e):
    """Time average over one orbit: <cos E - e> = -3e/2 (since <cos E> = -e/2 in mean
    anomaly) and <sqrt(1-e^2) sin E> = 0.  Uniform grid in t over one period."""
    P, a = 3.0, 10.0
    t = np.arange(8192) * (P / 8192)
    xy = oracle.astro_model(_one(t, P, e, 0.4, a, a, 0.0, 0.0))[0]    # Dec = a X, RA = a X
    assert np.mean(xy[1]) == pytest.approx(-1.5 * e * a, abs=1e-9 * a)
    xy = oracle.astro_model(_one(t, P, e, 0.4, 0.0, 0.0, a, a))[0]    # Dec = a Y, RA = a Y
    assert abs(np.mean(xy[1])) < 1e-9 * a


def test_circular_orbit_closed_form():
    """e = 0: X = cos M, Y = sin M, so RA = B cos M + G sin M, Dec = A cos M + F sin M."""
    rng = np.random.default_rng(22)
    for _ in range(30):
        P, M0 = rng.uniform(1, 500), rng.uniform(0, TWO_PI)
        A, B, F, G = rng.normal(size=4) * 20
        t = rng.uniform(2454000, 2457000)
        M = oracle.mean_anomaly(t, 0.0, P, M0)
        xy = oracle.astro_model(_one(t, P, 0.0, M0, A, B, F, G))[0, :, 0]
        assert xy[0] == pytest.approx(B * math.cos(M) + G * math.sin(M), abs=1e-12 * 80)
        assert xy[1] == pytest.approx(A * math.cos(M) + F * math.sin(M), abs=1e-12 * 80)


def test_linear_in_thiele_innes_constants():
    """For fixed (P, e, M0) the positions are linear in (A, B, F, G)."""
    rng = np.random.default_rng(23)
    t = np.sort(rng.uniform(2454000, 2457000, 50))
    z = np.zeros(50)
    P, e, M0 = np.array([[7.0], [300.0]]), np.array([[0.2], [0.6]]), np.array([[1.0], [4.0]])
    c1, c2 = rng.normal(size=(4, 2, 1)), rng.normal(size=(4, 2, 1))

    def model(c):
        return oracle.astro_model(oracle.Astro(t, z, z, z + 1, z + 1, P, e, M0, *c))[0]

    assert np.allclose(model(c1 + 2.5 * c2), model(c1) + 2.5 * model(c2), rtol=0, atol=1e-12)


def test_two_planets_sum_and_offsets():
    """Positions add over planets; offsets x0, y0 shift RA and Dec."""
    rng = np.random.default_rng(24)
    t = np.sort(rng.uniform(2454000, 2457000, 40))
    z = np.zeros(40)
    pl = [(5.5, 0.1, 0.3, 1.0, 2.0, -3.0, 0.5), (410.0, 0.5, 2.0, -7.0, 1.5, 2.5, 4.0)]
    singles = [oracle.astro_model(oracle.Astro(t, z, z, z + 1, z + 1, *[[[v]] for v in p]))[0] for p in pl]
    cols = [np.array([[p[k]] for p in pl]) for k in range(7)]
    both = oracle.astro_model(oracle.Astro(t, z, z, z + 1, z + 1, *cols, [0.25], [-1.5]))[0]
    assert np.allclose(both[0], singles[0][0] + singles[1][0] + 0.25, rtol=0, atol=1e-13)
    assert np.allclose(both[1], singles[0][1] + singles[1][1] - 1.5, rtol=0, atol=1e-13)


def test_chisq_identities():
    """Noise-free data give chi2 = 0; a constant offset c in RA adds c^2 sum 1/sx^2;
    scaling both uncertainties by s divides chi2 by s^2; sx <= 0 gives NaN."""
    rng = np.random.default_rng(25)
    t = np.sort(rng.uniform(2454000, 2457000, 30))
    par = (12.0, 0.4, 1.2, 5.0, -2.0, 3.0, 1.0)
    z = np.zeros(30)
    xy = oracle.astro_model(oracle.Astro(t, z, z, z + 1, z + 1, *[[[v]] for v in par]))[0]
    sx, sy = rng.uniform(0.05, 0.2, 30), rng.uniform(0.05, 0.2, 30)
    d = oracle.Astro(t, xy[0], xy[1], sx, sy, *[[[v]] for v in par])
    assert oracle.astro_chisq(d)[0] < 1e-20
    d = oracle.Astro(t, xy[0] - 0.3, xy[1], sx, sy, *[[[v]] for v in par])
    assert oracle.astro_chisq(d)[0] == pytest.approx(0.09 * np.sum(1 / sx ** 2), rel=1e-12)
    noisy_x, noisy_y = xy[0] + rng.normal(size=30) * sx, xy[1] + rng.normal(size=30) * sy
    c1 = oracle.astro_chisq(oracle.Astro(t, noisy_x, noisy_y, sx, sy, *[[[v]] for v in par]))[0]
    c2 = oracle.astro_chisq(oracle.Astro(t, noisy_x, noisy_y, 2 * sx, 2 * sy, *[[[v]] for v in par]))[0]
    assert c2 == pytest.approx(c1 / 4, rel=1e-12)
    bad = sx.copy()
    bad[3] = 0.0
    assert np.isnan(oracle.astro_chisq(oracle.Astro(t, noisy_x, noisy_y, bad, sy, *[[[v]] for v in par]))[0])
    badp = list(par)
    badp[1] = 1.0
    assert np.isnan(oracle.astro_chisq(oracle.Astro(t, noisy_x, noisy_y, sx, sy, *[[[v]] for v in badp]))[0])
