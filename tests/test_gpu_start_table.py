"""GPU parity at the edges of the Kepler starting-value table (Sec. 5.4's tabulated
guess, used by the mixed kernels for e <= 0.9, in bands of eccentricity).

Eccentricities on every row of every band, at 0, at the band edges, just inside and
just outside the table's range; observation times that put the mean anomaly exactly
on the M knots j pi / N of each band (N = 128 and 256), at 0, at +-pi and a hair
either side of them.  The eccentric anomalies must meet the same bound as elsewhere
(binary32 Kepler bound plus the two binary64 phases, modulo 2 pi) and the model
velocities the mixed velocity tolerance, 1e-3 m/s; in binary64 the velocities agree
to 1e-9 m/s.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_0812_2976_amd as kp
from tests import workloads as W
from tests.test_start_table import _read_header

pytestmark = pytest.mark.gpu


def _edge_case():
    emax, _, bands = _read_header()
    rows = sorted({bd["e0"] + i * (bd["e1"] - bd["e0"]) / bd["rows"] for bd in bands for i in range(bd["rows"] + 1)})
    es = ([0.0, 1e-12] + rows + [float(np.nextafter(bd["e0"], 0.0)) for bd in bands[1:]]
          + [emax * (1 - 1e-12), float(np.nextafter(emax, 1.0)), emax + 1e-9, 0.92, 0.95])
    n_sys = len(es)
    P = 10.0
    knots = np.unique(np.concatenate([np.arange(bd["knots"] + 1) * (math.pi / bd["knots"]) for bd in bands]))
    M = np.concatenate([knots, -knots[1:], [math.pi - 1e-7, -math.pi + 1e-7, 1e-7, -1e-7, 1e-3, -1e-3]])
    M = np.concatenate([M, np.random.default_rng(5).uniform(-math.pi, math.pi, 300)])
    t = np.sort(P * (M / (2 * math.pi)))                 # t0 = 0, M0 = 0: M(t) = 2 pi t / P
    shape = (1, n_sys)
    par = dict(P=np.full(shape, P), K=np.linspace(5.0, 400.0, n_sys).reshape(shape), e=np.array(es).reshape(shape),
               w=np.linspace(-3.0, 3.0, n_sys).reshape(shape), M0=np.zeros(shape))
    return t, par, n_sys


def _gpu(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def test_table_edges_eccentric_anomalies(dev):
    t, p, n_sys = _edge_case()
    E = kp.rv_eccentric_anomalies(_gpu(t, dev), *(_gpu(p[k], dev) for k in ("P", "K", "e", "w", "M0")),
                                  t0=0.0).cpu().numpy().astype(np.float64)
    worst = 0.0
    for i in range(n_sys):
        M = np.array([oracle.mean_anomaly(tk, 0.0, p["P"][0, i], 0.0) for tk in t])
        e = np.full_like(M, p["e"][0, i])
        ref = oracle.kepler(M, e)
        d = np.remainder(E[0, i] - ref + np.pi, 2 * np.pi) - np.pi
        tol = W.kepler_tol_mixed(M, e, ref) + 1e-8 / (1.0 - e * np.cos(ref))
        worst = max(worst, float(np.max(np.abs(d) / tol)))
        assert np.all(np.abs(d) <= tol), (i, p["e"][0, i], float(np.max(np.abs(d))))
    print(f"[table edges] max |dE| / bound {worst:.3f}", flush=True)


@pytest.mark.parametrize("prec,tol", [("mixed", 1e-3), ("fp64", 1e-9)])
def test_table_edges_velocities(dev, prec, tol):
    t, p, n_sys = _edge_case()
    g = [_gpu(p[k], dev) for k in ("P", "K", "e", "w", "M0")]
    vm = kp.rv_model(_gpu(t, dev), *g, t0=0.0, prec=prec).cpu().numpy()
    d = oracle.Dense(t, np.zeros_like(t), np.ones_like(t), p["P"], p["K"], p["e"], p["w"], p["M0"], None, None, 0.0)
    ref = oracle.rv_model(d)
    err = np.abs(vm - ref)
    print(f"[table edges {prec}] max |dv| {err.max():.3e} m/s", flush=True)
    assert err.max() <= tol
