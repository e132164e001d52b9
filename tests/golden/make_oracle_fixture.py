"""Write tests/golden/oracle_c0_first16.txt: the oracle's chi-square for the first
16 systems of the c0 workload (1024 x 1 x 64, sigma = 3 m/s, seed 1000), with
observed velocities = oracle model of the truth system + seeded noise.

Calls only oracle/ and synth/.  The file is a regression pin: a later change to
the oracle's arithmetic that moves these numbers must name, in its commit
message, the passage of the paper that justifies it.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_c0_first16.txt")


def truth_model(t, t0, truth):
    d = oracle.Dense(t, np.zeros_like(t), np.ones_like(t), *(np.asarray(truth[k])[:, None] for k in ("P", "K", "e", "w", "M0")), t0=t0)
    return oracle.rv_model(d)[0]


def compute():
    wl = synth.with_observations(synth.dense("c0"), truth_model)
    d = oracle.Dense(wl.t, wl.v, wl.sigma, wl.P, wl.K, wl.e, wl.w, wl.M0, t0=wl.t0)
    return oracle.chisq(d, 0, 16)[:16]


if __name__ == "__main__":
    chi2 = compute()
    with open(OUT, "w") as f:
        f.write("# chi-square (Eq. 5) of systems 0..15 of workload c0, written by make_oracle_fixture.py\n")
        for i, c in enumerate(chi2):
            f.write(f"{i} {float(c)!r}\n")
    print(OUT)
