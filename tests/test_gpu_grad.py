"""GPU parity of rv_chisq_grad (implicit-function adjoint) with the oracle's analytic
gradient and with central finite differences of the oracle's chi-square.

Tolerances (S_r = sum_k |2 w r dv/dtheta|, the oracle's error scale of each
component; the stated gradient tolerance is relative 1e-6, normalised by
max(|g|, S_r) because the gradient vanishes at a perfect fit):
  binary64 adjoint: componentwise |dg| <= 1e-6 (|g_ref| + 1e-6 S_r) against the
      oracle's analytic gradient, and against central differences within the
      differences' own error (relative 1e-5 of max(|g|, S_r)).
  mixed adjoint: |dg| <= 1e-6 max(|g_ref|, S_r) against the oracle's analytic
      gradient on every shape (the periapsis stress set and e up to 0.99
      included), and against binary64 central differences of the oracle's
      chi-square within 1e-6 max(|g|, S_r) plus the differences' own error
      (their distance from the analytic gradient, measured per component).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_0812_2976_amd as kp
from tests import workloads as W

pytestmark = pytest.mark.gpu


def _grad_ref(wl, n=None):
    d = W.oracle_dense(wl)
    n = wl.n_sys if n is None else n
    return W.oracle_par(oracle.chisq_grad_scales, d, n)


@pytest.mark.parametrize("case", [
    dict(n_sys=600, n_pl=4, n_obs=256),
    dict(n_sys=130, n_pl=1, n_obs=64),
    dict(n_sys=70, n_pl=7, n_obs=45, jitter=True),
    dict(n_sys=40, n_pl=8, n_obs=20),
])
def test_grad_fp64_matches_oracle(dev, case):
    wl = W.dense("c4", n_sys=case["n_sys"], n_pl=case["n_pl"], n_obs=case["n_obs"], jitter=case.get("jitter", False))
    g = W.to_gpu(wl, dev)
    chi2, grad = kp.rv_chisq_grad(**g, prec="fp64")
    chi2, grad = chi2.cpu().numpy(), grad.cpu().numpy()
    c_ref, g_ref, s_r, s_1 = _grad_ref(wl)
    assert W.rel_err_chi2(chi2, c_ref).max() <= 1e-12
    err = np.abs(grad - g_ref) / (np.abs(g_ref) + 1e-6 * s_r)
    print(f"[grad fp64 {case}] max normalised error {err.max():.3e}", flush=True)
    assert err.max() <= 1e-6


@pytest.mark.parametrize("case", [
    dict(n_sys=2048, n_pl=4, n_obs=256),
    dict(n_sys=300, n_pl=3, n_obs=100, jitter=True),
    dict(n_sys=100, n_pl=6, n_obs=300),
    dict(n_sys=256, n_pl=4, n_obs=256, stress=True),
    # lanes on both sides of the starting-value table's range within one wavefront
    dict(n_sys=640, n_pl=3, n_obs=120, e_range=(0.0, 0.99)),
])
def test_grad_mixed_matches_oracle(dev, case):
    wl = W.dense("c4", n_sys=case["n_sys"], n_pl=case["n_pl"], n_obs=case["n_obs"],
                 jitter=case.get("jitter", False), stress=case.get("stress", False), e_range=case.get("e_range"))
    g = W.to_gpu(wl, dev)
    chi2, grad = kp.rv_chisq_grad(**g, prec="mixed")
    chi2, grad = chi2.cpu().numpy(), grad.cpu().numpy()
    c_ref, g_ref, s_r, s_1 = _grad_ref(wl)
    assert W.rel_err_chi2(chi2, c_ref).max() <= 1e-5
    q13 = np.abs(grad - g_ref) / np.maximum(np.abs(g_ref), s_r)
    plain = np.abs(grad - g_ref) / np.maximum(np.abs(g_ref), 1e-300)
    print(f"[grad mixed {case}] max |dg|/max(|g|, S_r) {q13.max():.3e}; "
          f"median componentwise rel {np.median(plain):.2e}", flush=True)
    assert q13.max() <= 1e-6


def _central_differences(wl, i, j, nm, span):
    """binary64 central difference of the oracle's chi-square of system i in parameter
    nm of planet j; the period step moves the latest phase by ~1e-6 rad."""
    names = ("P", "K", "e", "w", "M0")
    x0 = getattr(wl, nm)[j, i]
    h = 1e-6 * x0 * x0 / (2 * np.pi * span) if nm == "P" else 1e-6 * max(abs(x0), 1.0)
    vals = []
    for s in (1, -1):
        arr = getattr(wl, nm).copy()
        arr[j, i] = x0 + s * h
        kw = {k: getattr(wl, k) for k in names}
        kw[nm] = arr
        d = oracle.Dense(wl.t, wl.v, wl.sigma, kw["P"], kw["K"], kw["e"], kw["w"], kw["M0"], wl.offset, None, wl.t0)
        vals.append(oracle.chisq(d, i, i + 1)[i])
    return (vals[0] - vals[1]) / (2 * h)


@pytest.mark.parametrize("case", [
    dict(n_sys=16, n_pl=4, n_obs=256),
    dict(n_sys=8, n_pl=3, n_obs=120, e_range=(0.0, 0.99)),
])
def test_grad_mixed_matches_central_differences(dev, case):
    """Mixed adjoint vs binary64 central differences of the oracle's chi-square, epoch
    mid-baseline (t0 = 2,455,500), steps as in the binary64 test.  Bound: 1e-6 of
    max(|g|, S_r) plus each difference's own error |fd - g_oracle|."""
    wl = W.dense("c4", n_sys=case["n_sys"], n_pl=case["n_pl"], n_obs=case["n_obs"], t0=2455500.0,
                 e_range=case.get("e_range"))
    g = W.to_gpu(wl, dev)
    _, grad = kp.rv_chisq_grad(**g, prec="mixed")
    grad = grad.cpu().numpy()
    _, g_ref, s_r, _ = _grad_ref(wl)
    span = np.max(np.abs(wl.t - wl.t0))
    worst = 0.0
    for i in range(wl.n_sys):
        for j in range(wl.n_pl):
            for a, nm in enumerate(("P", "K", "e", "w", "M0")):
                r = 5 * j + a
                fd = _central_differences(wl, i, j, nm, span)
                scale = max(abs(g_ref[r, i]), s_r[r, i])
                worst = max(worst, abs(grad[r, i] - fd) / scale)
                assert abs(grad[r, i] - fd) <= 1e-6 * scale + abs(fd - g_ref[r, i]), (i, j, nm, grad[r, i], fd)
    print(f"[grad mixed vs central differences {case}] max |g - fd|/max(|g|, S_r) {worst:.3e}", flush=True)


def test_grad_fp64_matches_central_differences(dev):
    """binary64 adjoint vs central differences of the oracle's chi-square; the epoch
    sits mid-baseline and the period step moves the latest phase by ~1e-6 rad."""
    wl = W.dense("c4", n_sys=6, n_pl=2, n_obs=60, t0=2455500.0)
    g = W.to_gpu(wl, dev)
    _, grad = kp.rv_chisq_grad(**g, prec="fp64")
    grad = grad.cpu().numpy()
    _, _, s_r, _ = _grad_ref(wl)
    span = np.max(np.abs(wl.t - wl.t0))
    names = ("P", "K", "e", "w", "M0")
    for i in range(wl.n_sys):
        for j in range(wl.n_pl):
            for a, nm in enumerate(names):
                x0 = getattr(wl, nm)[j, i]
                h = 1e-6 * x0 * x0 / (2 * np.pi * span) if nm == "P" else 1e-6 * max(abs(x0), 1.0)
                vals = []
                for s in (1, -1):
                    arr = getattr(wl, nm).copy()
                    arr[j, i] = x0 + s * h
                    kw = {k: getattr(wl, k) for k in names}
                    kw[nm] = arr
                    d = oracle.Dense(wl.t, wl.v, wl.sigma, kw["P"], kw["K"], kw["e"], kw["w"], kw["M0"],
                                     wl.offset, None, wl.t0)
                    vals.append(oracle.chisq(d, i, i + 1)[i])
                fd = (vals[0] - vals[1]) / (2 * h)
                gg = grad[5 * j + a, i]
                assert abs(fd - gg) <= 1e-5 * max(abs(gg), s_r[5 * j + a, i]), (i, j, nm, fd, gg)
    # offset: chi2 is quadratic in gamma, central differences are exact up to rounding
    for i in range(wl.n_sys):
        vals = []
        for s in (1, -1):
            off = wl.offset.copy()
            off[i] += s * 1e-3
            d = oracle.Dense(wl.t, wl.v, wl.sigma, wl.P, wl.K, wl.e, wl.w, wl.M0, off, None, wl.t0)
            vals.append(oracle.chisq(d, i, i + 1)[i])
        assert abs((vals[0] - vals[1]) / 2e-3 - grad[-1, i]) <= 1e-6 * max(abs(grad[-1, i]), s_r[-1, i])


def test_grad_chisq_equals_rv_chisq(dev):
    """The gradient kernel's chi-square equals the chi-square kernel within tolerance."""
    wl = W.dense("c4", n_sys=3000)
    g = W.to_gpu(wl, dev)
    c1, _ = kp.rv_chisq_grad(**g, prec="mixed")
    c2 = kp.rv_chisq(**g, prec="mixed")
    assert W.rel_err_chi2(c1.cpu().numpy(), c2.cpu().numpy()).max() <= 2e-5


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_autograd_function(dev, prec):
    """RVChiSq.backward returns grad_out * d chi2 / d theta (the same launch's gradient,
    so equal to rv_chisq_grad's bit for bit in either precision)."""
    wl = W.dense("c4", n_sys=50, n_pl=2, n_obs=40)
    g = W.to_gpu(wl, dev)
    leaves = [g[k].clone().requires_grad_(True) for k in ("P", "K", "e", "omega", "M0", "offset")]
    chi2 = kp.RVChiSq.apply(*leaves, g["t"], g["v"], g["sigma"], None, 0.0, prec)
    wts = torch.linspace(0.5, 2.0, wl.n_sys, dtype=torch.float64, device=dev)
    (chi2 * wts).sum().backward()
    _, grad = kp.rv_chisq_grad(**g, prec=prec)
    for j in range(2):
        for a in range(5):
            assert torch.equal(leaves[a].grad[j], grad[5 * j + a] * wts)
    assert torch.equal(leaves[5].grad, grad[-1] * wts)


def test_autograd_function_without_offset_and_frozen_inputs(dev):
    """offset=None and inputs that need no gradient get None from backward (no error)."""
    wl = W.dense("c4", n_sys=30, n_pl=2, n_obs=40)
    g = W.to_gpu(wl, dev)
    P = g["P"].clone().requires_grad_(True)
    K = g["K"].clone().requires_grad_(True)
    chi2 = kp.RVChiSq.apply(P, K, g["e"], g["omega"], g["M0"], None, g["t"], g["v"], g["sigma"], None, 0.0,
                            "mixed")
    chi2.sum().backward()
    _, grad = kp.rv_chisq_grad(g["t"], g["v"], g["sigma"], g["P"], g["K"], g["e"], g["omega"], g["M0"],
                               prec="mixed")
    assert torch.equal(P.grad, grad[0:10:5])
    assert torch.equal(K.grad, grad[1:10:5])


def test_grad_domain_nan(dev):
    wl = W.dense("c4", n_sys=20, n_pl=2, n_obs=30)
    wl.e[0, 4] = 1.5
    g = W.to_gpu(wl, dev)
    for prec in ("fp64", "mixed"):
        chi2, grad = kp.rv_chisq_grad(**g, prec=prec)
        chi2, grad = chi2.cpu().numpy(), grad.cpu().numpy()
        assert np.isnan(chi2[4]) and np.all(np.isnan(grad[:, 4]))
        assert np.all(np.isfinite(np.delete(grad, 4, axis=1)))
