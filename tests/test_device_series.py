"""Host checks of the binary64 sine/cosine that the mixed kernels use to correct
a binary32 Kepler root (kep_grad.h): the quadrant-reduced series
(sincos_root64) and the knot form (sincos_root64_knots: knots n/64 filled with
the full series, short series of the exactly split remainder, rotation).  The
coefficients and constants are read from the header and the arithmetic is
replayed in Python against math.sin / math.cos, so a wrong sign, factorial or
scale in the device code fails here on the CPU."""
import math
import os
import re

import numpy as np
import pytest

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_0812_2976_amd", "csrc", "kep_grad.h")


def _coeffs(var, text):
    pat = var + r" = (?:fma\(" + var + r", y2, )?(-?1\.0 / [0-9.]+|-?0\.5)"
    return [eval(m.group(1)) for m in re.finditer(pat, text)]


def _series():
    src = open(HDR).read()
    body = src[src.index("__device__ __forceinline__ void sincos_root64(float E"):]
    body = body[:body.index("\n}\n")]
    return _coeffs("ps", body), _coeffs("pc", body)


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


def test_root_sincos_series():
    ps, pc = _series()
    # sin to y^17, cos to y^18, with 1/n! magnitudes and alternating signs
    assert len(ps) == 8 and len(pc) == 9
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
    assert es <= 3e-16 and ec <= 3e-16, (es, ec)


def _knot_form():
    src = open(HDR).read()
    half = int(re.search(r"constexpr int kSc64Half = (\d+);", src).group(1))
    body = src[src.index("__device__ __forceinline__ void sincos_root64_knots"):]
    body = body[:body.index("\n}\n")]
    lit = r"(-?[0-9.]+(?: / [0-9.]+)?)"
    scale = eval(re.search(r"rintf\(E \* " + lit + r"f\)", body).group(1))
    step = eval(re.search(r"fmaf\(fn, " + lit + r"f, E\)", body).group(1))
    s3, s5 = (eval(g) for g in re.search(r"const double sy = fma\(y \* y2, fma\(y2, " + lit + ", " + lit + r"\), y\)",
                                          body).groups()[::-1])
    c6, c4, c2 = (eval(g) for g in re.search(r"const double cy = fma\(y2, fma\(y2, fma\(y2, " + lit + ", " + lit +
                                             r"\), " + lit + r"\), 1\.0\)", body).groups())
    m = re.search(r"float clamp_root\(float E\) \{ return fabsf\(E\) > ([0-9.]+)f \? copysignf\(([0-9.]+)f, E\) : E; \}",
                  src)
    assert m.group(1) == m.group(2)
    clamp = float(m.group(1))
    return half, scale, step, (s3, s5), (c2, c4, c6), clamp


def test_root_sincos_knot_form():
    half, scale, step, (s3, s5), (c2, c4, c6), clamp = _knot_form()
    assert scale == 64.0 and step == -1.0 / 64.0 and clamp == half / 64.0 == 3.25
    assert (s3, s5) == (-1.0 / 6.0, 1.0 / 120.0) and (c2, c4, c6) == (-0.5, 1.0 / 24.0, -1.0 / 720.0)
    ps, pc = _series()
    knots = {n: _sincos(n / 64.0, ps, pc) for n in range(-half, half + 1)}
    for n in (-half, -100, -1, 0, 1, 37, half):
        assert abs(knots[n][0] - math.sin(n / 64.0)) <= 2.3e-16 and abs(knots[n][1] - math.cos(n / 64.0)) <= 2.3e-16
    rng = np.random.default_rng(12)
    E = np.concatenate([rng.uniform(-clamp, clamp, 20000), np.linspace(-clamp, clamp, 4001),
                        np.arange(-half, half + 1) / 64.0 + 1.0 / 128.0]).astype(np.float32)
    E = E[np.abs(E) <= clamp]
    es = ec = 0.0
    for x in E:
        fn = float(np.rint(np.float32(x) * np.float32(scale)))
        y = float(x) + fn * step                       # the device's fmaf
        assert float(np.float32(y)) == y and abs(y) <= 1.0 / 128.0 and abs(fn) <= half
        ks, kc = knots[int(fn)]
        y2 = y * y
        sy = y * y2 * (y2 * s5 + s3) + y
        cy = y2 * (y2 * (y2 * c6 + c4) + c2) + 1.0
        sv, cv = ks * cy + kc * sy, kc * cy - ks * sy
        es, ec = max(es, abs(sv - math.sin(float(x)))), max(ec, abs(cv - math.cos(float(x))))
    assert es <= 4.5e-16 and ec <= 4.5e-16, (es, ec)
