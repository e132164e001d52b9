"""Host checks of the binary64 sine/cosine series that the mixed kernels use to
correct a binary32 Kepler root (kep_grad.h sincos_root64): the coefficients are
read from the header and the quadrant reduction and Horner sums replayed in
Python against math.sin / math.cos, so a wrong sign or factorial in the device
code fails here on the CPU."""
import math
import os
import re

import numpy as np
import pytest

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_0812_2976_amd", "csrc", "kep_grad.h")


def _coeffs(var, text):
    pat = var + r" = (?:fma\(" + var + r", y2, )?(-?1\.0 / [0-9.]+|-?0\.5)"
    return [eval(m.group(1)) for m in re.finditer(pat, text)]


def _series(full):
    src = open(HDR).read()
    body = src[src.index("__device__ __forceinline__ void sincos_root64"):]
    body = body[:body.index("\n}\n")]
    branch = body[body.index("if constexpr (FULL) {"):body.index("const double sy")]
    head = (branch[:branch.index("} else {")] if full
            else branch[branch.index("} else {"):branch.index("ps = fma(ps, y2, -1.0 / 39916800.0)")])
    ps = _coeffs("ps", head) + _coeffs("ps", body[body.index("ps = fma(ps, y2, -1.0 / 39916800.0)"):
                                                  body.index("const double sy")])
    pc = _coeffs("pc", head) + _coeffs("pc", body[body.index("const double sy"):body.index("const double cy")])
    return ps, pc


def _sincos(E, ps, pc):
    nf = float(np.rint(np.float32(E) * np.float32(0.636619772)))
    n = int(nf)
    y = (E - nf * 1.5707963267948965580) - nf * 6.123233995736766036e-17
    y2 = y * y
    a = ps[0]
    for c in ps[1:]:
        a = a * y2 + c
    b = pc[0]
    for c in pc[1:]:
        b = b * y2 + c
    sy, cy = y * y2 * a + y, y2 * b + 1.0
    q = n & 3
    s0, c0 = (cy, sy) if q & 1 else (sy, cy)
    return (-s0 if q & 2 else s0), (-c0 if q in (1, 2) else c0)


@pytest.mark.parametrize("full,bound_s,bound_c", [(False, 2.2e-14, 2.2e-14), (True, 3e-16, 3e-16)])
def test_root_sincos_series(full, bound_s, bound_c):
    ps, pc = _series(full)
    # degrees: sin to y^13 / y^17, cos to y^14 / y^18, with 1/n! magnitudes and alternating signs
    assert len(ps) == (8 if full else 6) and len(pc) == (9 if full else 7)
    for k, c in enumerate(reversed(ps)):
        assert c == pytest.approx((-1) ** (k + 1) / math.factorial(2 * k + 3), rel=1e-15)
    for k, c in enumerate(reversed(pc)):
        assert c == pytest.approx((-1) ** (k + 1) / math.factorial(2 * k + 2), rel=1e-15)
    rng = np.random.default_rng(11)
    E = np.concatenate([rng.uniform(-3.3, 3.3, 20000), np.linspace(-math.pi, math.pi, 4001),
                        [k * math.pi / 4 for k in range(-4, 5)]]).astype(np.float32).astype(np.float64)
    es = ec = 0.0
    for x in E:
        s, c = _sincos(float(x), ps, pc)
        es, ec = max(es, abs(s - math.sin(x))), max(ec, abs(c - math.cos(x)))
    assert es <= bound_s and ec <= bound_c, (es, ec)
