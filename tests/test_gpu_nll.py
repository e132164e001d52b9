"""GPU parity of rv_nll_grad (Gaussian likelihood with jitter, Eq. 5's weights
1/(sigma^2 + s^2)) with the oracle's oracle_nll_grad.

Tolerances (u = 2^-24, n = n_obs, L = sum_k |ln(sigma_k^2 + s^2)|):
  binary64: nll within 1e-12 (chi2 + L); planet and offset rows as the binary64
      chi-square gradient; jitter row within 1e-10 of its scale
      2 s (sum w + sum w^2 r^2).
  mixed: nll within 1e-5 max(chi2, 1) + n 3u + 2u L (the chi-square bound plus a
      binary32 variance and logarithm per observation); planet and offset rows as
      the mixed chi-square gradient (|dg| <= 1e-6 max(|g|, S_r)); jitter row within
      2 s (4u sum w + 1e-5 sum w^2 r^2) (binary32 weights; the residuals carry the
      binary64 correction of the velocity).
"""
import numpy as np
import pytest

import oracle
import paper_0812_2976_amd as kp
from tests import workloads as W

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def _ref(wl):
    d = W.oracle_dense(wl)
    nll, grad = W.oracle_par(oracle.nll_grad, d, wl.n_sys)
    _, _, s_r, s_1 = W.oracle_par(oracle.chisq_grad_scales, d, wl.n_sys)
    # rv_model is [n_sys, n_obs]; oracle_par merges along the last axis
    r = W.oracle_par(lambda dd, i0, i1: oracle.rv_model(dd, i0, i1).T, d, wl.n_sys).T - wl.v[None, :]
    jit = np.zeros(wl.n_sys) if wl.jitter is None else wl.jitter
    w = 1.0 / (wl.sigma[None, :] ** 2 + jit[:, None] ** 2)
    logs = np.sum(np.abs(np.log(1.0 / w)), axis=1)
    chi2 = np.sum(w * r * r, axis=1)
    return dict(nll=nll, grad=grad, s_r=s_r, s_1=s_1, r=r, w=w, jit=jit, logs=logs, chi2=chi2)


@pytest.mark.parametrize("case", [
    dict(n_sys=300, n_pl=3, n_obs=100),
    dict(n_sys=130, n_pl=1, n_obs=64),
    dict(n_sys=40, n_pl=8, n_obs=20),
])
def test_nll_fp64_matches_oracle(dev, case):
    wl = W.dense("c4", n_sys=case["n_sys"], n_pl=case["n_pl"], n_obs=case["n_obs"], jitter=True)
    nll, grad = kp.rv_nll_grad(**W.to_gpu(wl, dev), prec="fp64")
    nll, grad = nll.cpu().numpy(), grad.cpu().numpy()
    ref = _ref(wl)
    assert grad.shape == (5 * wl.n_pl + 2, wl.n_sys)
    assert np.all(np.abs(nll - ref["nll"]) <= 1e-12 * (ref["chi2"] + ref["logs"]))
    err = np.abs(grad[:-1] - ref["grad"][:-1]) / (np.abs(ref["grad"][:-1]) + 1e-6 * ref["s_r"])
    assert err.max() <= 1e-6
    scale = 2 * ref["jit"] * np.sum(ref["w"] + ref["w"] ** 2 * ref["r"] ** 2, axis=1)
    assert np.all(np.abs(grad[-1] - ref["grad"][-1]) <= 1e-10 * scale + 1e-300)


@pytest.mark.parametrize("case", [
    dict(n_sys=2048, n_pl=4, n_obs=256),
    dict(n_sys=300, n_pl=3, n_obs=100),
    dict(n_sys=256, n_pl=4, n_obs=256, stress=True),
])
def test_nll_mixed_matches_oracle(dev, case):
    wl = W.dense("c4", n_sys=case["n_sys"], n_pl=case["n_pl"], n_obs=case["n_obs"], jitter=True,
                 stress=case.get("stress", False))
    nll, grad = kp.rv_nll_grad(**W.to_gpu(wl, dev), prec="mixed")
    nll, grad = nll.cpu().numpy(), grad.cpu().numpy()
    ref = _ref(wl)
    n = wl.t.size
    tol_nll = 1e-5 * np.maximum(ref["chi2"], 1.0) + n * 3 * U + 2 * U * ref["logs"]
    ratio = np.abs(nll - ref["nll"]) / tol_nll
    gratio = np.abs(grad[:-1] - ref["grad"][:-1]) / (1e-6 * np.maximum(np.abs(ref["grad"][:-1]), ref["s_r"]))
    w, r = ref["w"], ref["r"]
    tol_s = 2 * ref["jit"] * (4 * U * w.sum(1) + 1e-5 * np.sum(w * w * r * r, 1))
    sratio = np.abs(grad[-1] - ref["grad"][-1]) / np.maximum(tol_s, 1e-300)
    print(f"[nll mixed {case}] nll {ratio.max():.3e}  planet rows {gratio.max():.3e}  jitter row {sratio.max():.3e}",
          flush=True)
    assert ratio.max() <= 1.0 and gratio.max() <= 1.0 and sratio.max() <= 1.0


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_nll_rows_equal_chisq_grad_and_no_jitter(dev, prec):
    """Same launch shape and arithmetic: the planet and offset rows of rv_nll_grad are
    the rv_chisq_grad rows; without a jitter the last row is 0 and
    nll - chi2 = sum_k ln sigma_k^2."""
    wl = W.dense("c4", n_sys=500, n_pl=2, n_obs=80, jitter=True)
    g = W.to_gpu(wl, dev)
    nll, gn = kp.rv_nll_grad(**g, prec=prec)
    chi2, gc = kp.rv_chisq_grad(**g, prec=prec)
    assert np.array_equal(gn[:-1].cpu().numpy(), gc.cpu().numpy())
    lv = np.sum(np.log(wl.sigma[None, :] ** 2 + wl.jitter[:, None] ** 2), axis=1)
    tol = 1e-12 if prec == "fp64" else 2e-6
    assert np.allclose(nll.cpu().numpy() - chi2.cpu().numpy(), lv, rtol=0, atol=tol * np.max(np.abs(lv)))
    g["jitter"] = None
    nll0, g0 = kp.rv_nll_grad(**g, prec=prec)
    chi0, _ = kp.rv_chisq_grad(**g, prec=prec)
    assert np.all(g0[-1].cpu().numpy() == 0.0)
    d0 = nll0.cpu().numpy() - chi0.cpu().numpy()
    assert np.allclose(d0, np.sum(np.log(wl.sigma ** 2)), rtol=0, atol=tol * np.sum(np.abs(np.log(wl.sigma ** 2))))


def test_nll_jitter_gradient_finds_the_likelihood_maximum(dev):
    """The jitter row vanishes at the maximum-likelihood jitter: with a zero model
    (K = 0, no offset) and sigma = 0 every residual is -v and the optimum is
    s^2 = mean v^2; the binary64 kernel's derivative changes sign across it."""
    wl = W.dense("c4", n_sys=3, n_pl=1, n_obs=200, jitter=True)
    wl.sigma = np.zeros_like(wl.sigma)
    wl.K[:] = 0.0
    wl.offset[:] = 0.0
    s_opt = np.sqrt(np.mean(wl.v ** 2))
    wl.jitter = np.array([0.9 * s_opt, s_opt, 1.1 * s_opt])
    _, grad = kp.rv_nll_grad(**W.to_gpu(wl, dev), prec="fp64")
    gs = grad[-1].cpu().numpy()
    assert gs[0] < 0.0 < gs[2]
    assert abs(gs[1]) <= 1e-12 * np.sum(np.abs(gs))


def test_nll_domain_nan_and_bad_output(dev):
    wl = W.dense("c4", n_sys=20, n_pl=2, n_obs=30, jitter=True)
    wl.jitter[7] = -1.0
    g = W.to_gpu(wl, dev)
    for prec in ("fp64", "mixed"):
        nll, grad = kp.rv_nll_grad(**g, prec=prec)
        nll, grad = nll.cpu().numpy(), grad.cpu().numpy()
        assert np.isnan(nll[7]) and np.all(np.isnan(grad[:, 7]))
        assert np.all(np.isfinite(np.delete(grad, 7, axis=1)))
    import torch
    small = torch.empty((5 * 2 + 1, 20), dtype=torch.float64, device=dev)
    with pytest.raises(ValueError):
        kp.rv_nll_grad(**g, grad=small)
