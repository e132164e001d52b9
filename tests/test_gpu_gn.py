"""GPU parity of the Gauss-Newton products (rv_chisq_gn: chi2, J^T W r and packed
J^T W J on the matrix cores) with the oracle's oracle_gn.

Tolerances, with C = J^T W J from the oracle and entries normalised by the
Cauchy-Schwarz scale sqrt(C_aa C_bb) (the largest |C_ab| can be):
  binary64: 1e-9; mixed (binary32 derivative terms, as rv_chisq_grad): 1e-5.
J^T W r within the same normalised bounds against sqrt(C_aa chi2); chi2 as
rv_chisq (binary64 relative 1e-12, mixed 1e-5).  Sizes cover one, two and three
16-column blocks (n_pl = 1..2, 3..6, 7..8; in mixed precision the two-product
cover of 17 to 24 columns at n_pl = 3, 4 and all three block products at
n_pl = 5, 6) and observation counts that are not multiples of 64.
"""
import numpy as np
import pytest

import oracle
import paper_0812_2976_amd as kp
from tests import workloads as W

pytestmark = pytest.mark.gpu


def _check(wl, dev, prec, tol):
    g = W.to_gpu(wl, dev)
    chi2, jtwr, jtwj = (x.cpu().numpy() for x in kp.rv_chisq_gn(**g, prec=prec))
    c_ref, r_ref, j_ref = W.oracle_par(oracle.gn, W.oracle_dense(wl), wl.n_sys)
    npar = 5 * wl.n_pl + 1
    diag = np.array([j_ref[a * npar - a * (a - 1) // 2] for a in range(npar)])
    scale = np.empty_like(j_ref)
    idx = 0
    for a in range(npar):
        for b in range(a, npar):
            scale[idx] = np.sqrt(diag[a] * diag[b])
            idx += 1
    ej = np.abs(jtwj - j_ref) / scale
    er = np.abs(jtwr - r_ref) / np.sqrt(diag * np.maximum(c_ref, 1.0)[None, :])
    ec = W.rel_err_chi2(chi2, c_ref)
    return ej.max(), er.max(), ec.max()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("mixed", 1e-5)])
@pytest.mark.parametrize("case", [
    dict(n_sys=300, n_pl=4, n_obs=256),
    dict(n_sys=200, n_pl=1, n_obs=100),
    dict(n_sys=120, n_pl=3, n_obs=70, jitter=True),
    dict(n_sys=60, n_pl=8, n_obs=45),
    dict(n_sys=50, n_pl=7, n_obs=130),
    dict(n_sys=40, n_pl=5, n_obs=64),
    dict(n_sys=40, n_pl=6, n_obs=190),
])
def test_gn_matches_oracle(dev, prec, tol, case):
    wl = W.dense("c4", n_sys=case["n_sys"], n_pl=case["n_pl"], n_obs=case["n_obs"], jitter=case.get("jitter", False))
    ej, er, ec = _check(wl, dev, prec, tol)
    print(f"[gn {prec} {case}] J^T W J {ej:.3e}  J^T W r {er:.3e}  chi2 {ec:.3e}", flush=True)
    assert ej <= tol and er <= tol and ec <= (1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_gn_jtwr_is_half_the_gradient(dev, prec):
    """J^T W r is half the chi-square gradient.  Both mixed kernels correct the binary32
    root and form the velocity in binary64, and the Gauss-Newton kernel sums the
    binary32 products on the matrix cores: 2 J^T W r agrees with the gradient, and
    with the oracle's gradient, to the stated gradient tolerance (1e-6 of
    max(|g|, S_r))."""
    wl = W.dense("c4", n_sys=400, n_pl=2, n_obs=90)
    g = W.to_gpu(wl, dev)
    _, jtwr, _ = kp.rv_chisq_gn(**g, prec=prec)
    _, grad = kp.rv_chisq_grad(**g, prec=prec)
    jtwr, grad = jtwr.cpu().numpy(), grad.cpu().numpy()
    _, g_ref, s_r, _ = W.oracle_par(oracle.chisq_grad_scales, W.oracle_dense(wl), wl.n_sys)
    tol = 1e-12 if prec == "fp64" else 1e-6
    scale = np.maximum(np.abs(g_ref), s_r)
    err = np.max(np.abs(2 * jtwr - grad) / scale)
    err_ref = np.max(np.abs(2 * jtwr - g_ref) / scale)
    print(f"[gn vs grad {prec}] max |2 J^T W r - g| / max(|g|, S_r) = {err:.3e}; vs the oracle {err_ref:.3e}",
          flush=True)
    assert err <= tol and err_ref <= max(tol, 1e-12)


def test_gn_step_converges_on_noise_free_data(dev):
    """A Gauss-Newton step from the GPU's binary64 products, started 1e-4 (relative)
    from the truth of noise-free data, lands within the square of that distance."""
    wl = W.dense("c4", n_sys=8, n_pl=2, n_obs=120, t0=2455500.0)
    truth = {k: np.asarray(wl.truth[k], dtype=np.float64).reshape(-1) for k in ("P", "K", "e", "w", "M0")}
    wl.v = W.oracle_truth_model(wl.t, wl.t0, wl.truth)       # noise-free
    rng = np.random.default_rng(3)
    star = np.concatenate([[truth[k][j] for k in ("P", "K", "e", "w", "M0")] for j in range(2)] + [[0.0]])
    scale = np.maximum(np.abs(star), 1.0)
    rel = np.where(np.arange(star.size) % 5 == 0, 1e-7, 1e-4)
    X = star[:, None] + rel[:, None] * scale[:, None] * rng.normal(size=(star.size, wl.n_sys))
    for a, k in enumerate(("P", "K", "e", "w", "M0")):
        getattr(wl, k)[:] = X[[a, 5 + a], :]
    wl.offset = X[10].copy()
    _, jtwr, jtwj = (x.cpu().numpy() for x in kp.rv_chisq_gn(**W.to_gpu(wl, dev), prec="fp64"))
    for i in range(wl.n_sys):
        H = oracle.unpack_sym(jtwj[:, i], star.size)
        x1 = X[:, i] - np.linalg.solve(H, jtwr[:, i])
        e0 = np.max(np.abs(X[:, i] - star) / scale)
        e1 = np.max(np.abs(x1 - star) / scale)
        assert e1 < 100 * e0 ** 2 + 1e-12, (i, e0, e1)


def test_gn_edges(dev):
    wl = W.dense("c4", n_sys=30, n_pl=2, n_obs=40)
    wl.e[1, 4] = 1.2
    g = W.to_gpu(wl, dev)
    for prec in ("fp64", "mixed"):
        chi2, jtwr, jtwj = (x.cpu().numpy() for x in kp.rv_chisq_gn(**g, prec=prec))
        assert np.isnan(chi2[4]) and np.all(np.isnan(jtwr[:, 4])) and np.all(np.isnan(jtwj[:, 4]))
        assert np.all(np.isfinite(np.delete(jtwj, 4, axis=1)))
    import torch
    empty = torch.empty(0, dtype=torch.float64, device=dev)
    chi2, jtwr, jtwj = kp.rv_chisq_gn(empty, empty, empty, g["P"], g["K"], g["e"], g["omega"], g["M0"])
    ok = np.ones(30, bool)
    ok[4] = False
    assert np.all(chi2.cpu().numpy()[ok] == 0.0) and np.all(jtwj.cpu().numpy()[:, ok] == 0.0)
