"""Host-side checks of the C ABI (no GPU needed, no kernel launched): the library
loads, exports every function include/kepler.h declares, and rejects bad
arguments with a status and a message before touching the device."""
import ctypes
import os
import re

import pytest

import paper_0812_2976_amd as kp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kepler.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*([a-z_]+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(kp.LIB_PATH):
        pytest.fail("libkepler.so is not built (run __graft_entry__.build())")
    return kp.load_library()


def test_header_declares_the_boundary():
    fns = _declared_functions()
    for name in ("kepler_solve", "rv_model", "rv_chisq", "rv_chisq_grad", "rv_nll_grad", "kep_plan_ragged",
                 "rv_chisq_ragged",
                 "kep_plan_destroy", "kep_last_error"):
        assert name in fns


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert set(kp.EXPORTS) <= set(_declared_functions())
    assert lib.kep_abi_version() == 1


def _status(code, lib):
    return code, lib.kep_last_error().decode()


def test_kepler_solve_argument_errors(lib):
    code, msg = _status(lib.kepler_solve(None, None, None, -1, 0, None, None), lib)
    assert code == 1 and "n = -1" in msg
    code, msg = _status(lib.kepler_solve(None, None, None, 5, 7, None, None), lib)
    assert code == 1 and "precision" in msg
    code, msg = _status(lib.kepler_solve(None, None, None, 5, 1, None, None), lib)
    assert code == 1 and "NULL" in msg
    assert lib.kepler_solve(None, None, None, 0, 1, None, None) == 0          # empty: nothing to do
    bad = kp.KepOptions(0, 0, 100, 0)
    code, msg = _status(lib.kepler_solve(None, None, None, 0, 1, ctypes.byref(bad), None), lib)
    assert code == 1 and "block_threads" in msg


def test_dense_argument_errors(lib):
    obs = kp.KepObs(None, None, None, 10, 0.0)
    par = kp.KepParams(None, None, None, None, None, None, None, 5, 9)
    code, msg = _status(lib.rv_chisq(ctypes.byref(obs), ctypes.byref(par), None, 1, None, None), lib)
    assert code == 2 and "n_pl" in msg
    par.n_pl = 0
    assert lib.rv_chisq(ctypes.byref(obs), ctypes.byref(par), None, 1, None, None) == 2
    par.n_pl = 4
    code, msg = _status(lib.rv_chisq(ctypes.byref(obs), ctypes.byref(par), None, 1, None, None), lib)
    assert code == 1 and "obs->t" in msg
    obs.n_obs = -3
    assert lib.rv_model(ctypes.byref(obs), ctypes.byref(par), None, 0, None, None) == 1
    obs.n_obs = 0
    par.n_sys = 0
    assert lib.rv_chisq_grad(ctypes.byref(obs), ctypes.byref(par), None, None, 1, None, None) == 0
    assert lib.rv_nll_grad(ctypes.byref(obs), ctypes.byref(par), None, None, 1, None, None) == 0
    code, msg = _status(lib.rv_nll_grad(ctypes.byref(obs), ctypes.byref(par), None, None, 3, None, None), lib)
    assert code == 1 and "rv_nll_grad" in msg
    assert lib.rv_chisq(None, ctypes.byref(par), None, 1, None, None) == 1


def test_ragged_argument_errors(lib):
    out = ctypes.c_void_p()
    obs = kp.KepObsCSR(None, None, None, None, 0, 0.0)
    par = kp.KepParamsCSR(None, None, None, None, None, None, None, None, 4, 0)
    for prec in (0, 1):          # KEP_FP64 and KEP_MIXED both reach the argument checks
        code, msg = _status(lib.kep_plan_ragged(ctypes.byref(obs), ctypes.byref(par), prec, None, None,
                                                ctypes.byref(out)), lib)
        assert code == 1 and "pl_off" in msg
        code, msg = _status(lib.rv_chisq_ragged_static(ctypes.byref(obs), ctypes.byref(par), None, prec, None,
                                                       None), lib)
        assert code == 1 and "chi2" in msg
    code, msg = _status(lib.kep_plan_ragged(ctypes.byref(obs), ctypes.byref(par), 7, None, None, ctypes.byref(out)), lib)
    assert code == 1 and "prec" in msg
    assert lib.rv_chisq_ragged(None, None, None) == 1
    lib.kep_plan_destroy(None)


def test_python_binding_refuses_cpu_tensors():
    import torch
    x = torch.zeros(4, dtype=torch.float64)
    with pytest.raises(ValueError, match="GPU"):
        kp.kepler_solve(x, x)


def test_demc_argument_errors(lib):
    obs = kp.KepObs(None, None, None, 0, 0.0)
    st = kp.KepDemcState(None, None, None, None, 1, 2)
    code, msg = _status(lib.demc_chisq(ctypes.byref(obs), ctypes.byref(st), 1, None, None), lib)
    assert code == 2 and "n_half" in msg
    st.n_half, st.n_pl = 4, 9
    code, msg = _status(lib.demc_chisq(ctypes.byref(obs), ctypes.byref(st), 1, None, None), lib)
    assert code == 2 and "n_pl" in msg
    st.n_pl = 2
    code, msg = _status(lib.demc_chisq(ctypes.byref(obs), ctypes.byref(st), 1, None, None), lib)
    assert code == 1 and "x and chi2" in msg
    code, msg = _status(lib.demc_generations(ctypes.byref(obs), ctypes.byref(st), None, 0, 1, None, 1, None, None), lib)
    assert code == 1
    out = ctypes.c_void_p()
    assert lib.kep_plan_demc(ctypes.byref(obs), ctypes.byref(st), None, None, 1, None, None, None) == 1
    assert lib.demc_run(None, 0, 1, None) == 1
    lib.kep_demc_plan_destroy(None)
    del out
