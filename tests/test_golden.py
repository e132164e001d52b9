"""Regression pin of the oracle against its stored fixture (tests/golden)."""
import os

import numpy as np

from tests.golden import make_oracle_fixture as fx


def test_oracle_c0_fixture():
    ref = np.loadtxt(fx.OUT, comments="#")[:, 1]
    got = fx.compute()
    assert np.array_equal(got, ref)
    assert os.path.getsize(fx.OUT) < 4096
