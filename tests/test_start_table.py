"""The starting-value table of the binary32 Kepler solve (kep_start_tab.h), checked
on the CPU against the oracle's roots (no GPU).

The header documents its contents: binary16 pairs (E(e_i, M_j), E(e_i+1, M_j) -
E(e_i, M_j)) on e_i = i emax / (NE - 1), M_j = j pi / 128.  The tests read the
header, check every entry against the oracle's root rounded to binary16, and check
the property the kernels rely on: the bilinear start lies within 4e-3 rad of the
root, and one Danby step (Sec. 4.3's quartic correction, float64) from there lands
within 1e-9 rad, over e <= emax and a dense grid of M including M -> 0 and |M| -> pi;
on the leading rows the header names, the second-order step alone does.
"""
import math
import os
import re

import numpy as np
import pytest

import oracle

HEADER = os.path.join(os.path.dirname(__file__), "..", "paper_0812_2976_amd", "csrc", "kep_start_tab.h")


def _read_header():
    text = open(HEADER).read()
    defs = dict(re.findall(r"#define (KEP_TAB_\w+) ([0-9.eE+-]+)f?", text))
    ne, nm, emax = int(defs["KEP_TAB_NE"]), int(defs["KEP_TAB_NM"]), float(defs["KEP_TAB_EMAX"])
    body = text[text.index("{") + 1:text.index("}")]
    words = np.array([int(w, 16) for w in re.findall(r"0x([0-9a-f]{8})u", body)], dtype=np.uint32)
    assert words.size == (ne - 1) * nm
    lo = (words & 0xFFFF).astype(np.uint16).view(np.float16).astype(np.float64)
    hi = (words >> 16).astype(np.uint16).view(np.float16).astype(np.float64)
    return ne, nm, emax, lo.reshape(ne - 1, nm), hi.reshape(ne - 1, nm), float(defs["KEP_TAB_MSCALE"])


def _start(tab, e, M):
    ne, nm, emax, T, D, mscale = tab
    fi = e * ((ne - 1) / emax)
    i = min(int(fi), ne - 2)
    we = fi - i
    fj = np.minimum(np.abs(M) * mscale, 128.0)
    j = fj.astype(int)
    wm = fj - j
    r0 = T[i, j] + we * D[i, j]
    r1 = T[i, j + 1] + we * D[i, j + 1]
    return np.copysign(r0 + wm * (r1 - r0), M)


def _danby(E, e, M):
    """One step of Danby's quartic iteration (Sec. 4.3) in float64."""
    f = E - e * np.sin(E) - M
    f1, f2, f3 = 1 - e * np.cos(E), e * np.sin(E), e * np.cos(E)
    d1 = -f / f1
    d2 = -f / (f1 + d1 * f2 / 2)
    d3 = -f / (f1 + d2 * f2 / 2 + d2 * d2 * f3 / 6)
    return E + d3


@pytest.fixture(scope="module")
def tab():
    return _read_header()


def test_entries_are_rounded_roots(tab):
    """Every first half is the oracle's root E(e_i, M_j) rounded to binary16; every
    second half the rounded difference to the next row."""
    ne, nm, emax, T, D, mscale = tab
    assert ne >= 3 and nm == 130 and 0.5 < emax < 1.0
    assert abs(mscale - 128 / math.pi) < 1e-5
    M = np.arange(nm) * (math.pi / 128)
    roots = np.array([oracle.kepler(M, np.full(nm, i * emax / (ne - 1))) for i in range(ne)])
    r16 = roots.astype(np.float16).astype(np.float64)
    assert np.array_equal(T, r16[:-1])
    assert np.array_equal(D, (r16[1:] - r16[:-1]).astype(np.float16).astype(np.float64))
    assert T[0, 0] == 0.0 and np.all(np.diff(T, axis=1) > 0)       # E(M) increases with M


def test_start_and_one_step(tab):
    ne, nm, emax, T, D, mscale = tab
    M = np.concatenate([np.linspace(-math.pi, math.pi, 8001),
                        np.outer([-1.0, 1.0], np.logspace(-9, 0, 400)).ravel(),
                        [math.pi - 1e-7, -math.pi + 1e-7]])
    far, err = 0.0, 0.0
    for e in np.concatenate([np.linspace(0.0, emax, 97), [emax * (1 - 1e-9)]]):
        R = oracle.kepler(M, np.full(M.size, e))
        E0 = _start(tab, e, M)
        far = max(far, float(np.max(np.abs(E0 - R))))
        err = max(err, float(np.max(np.abs(_danby(E0, e, M) - R))))
    print(f"start {far:.3e} rad, after one step {err:.3e} rad")
    assert far <= 4e-3
    assert err <= 1e-9


def _halley(E, e, M):
    """One step of the second-order member of Danby's family (Halley's correction,
    Sec. 4.3's d2 = -f / (f' + d1 f''/2) with d1 = -f / f'), float64."""
    f = E - e * np.sin(E) - M
    f1, f2 = 1 - e * np.cos(E), e * np.sin(E)
    d1 = -f / f1
    return E - f / (f1 + d1 * f2 / 2)


def test_halley_rows(tab):
    """On the leading KEP_TAB_HALLEY_ROWS rows the kernels take the second-order step
    instead of the quartic one: from the bilinear start it lands within 1e-9 rad of the
    oracle's root, and the start lies within 2e-3 rad (the range of the shortened
    rotation); the next row needs the quartic step (the band is as wide as it can be)."""
    ne, nm, emax, T, D, mscale = tab
    rows = int(re.search(r"#define KEP_TAB_HALLEY_ROWS (\d+)", open(HEADER).read()).group(1))
    assert 1 <= rows < ne - 1
    M = np.concatenate([np.linspace(-math.pi, math.pi, 8001),
                        np.outer([-1.0, 1.0], np.logspace(-9, 0, 400)).ravel(),
                        [math.pi - 1e-7, -math.pi + 1e-7]])
    h = emax / (ne - 1)

    def worst(lo, hi, n):
        far, err = 0.0, 0.0
        for e in np.linspace(lo, hi, n):
            R = oracle.kepler(M, np.full(M.size, e))
            E0 = _start(tab, e, M)
            far = max(far, float(np.max(np.abs(E0 - R))))
            err = max(err, float(np.max(np.abs(_halley(E0, e, M) - R))))
        return far, err

    far, err = worst(0.0, rows * h * (1 - 1e-12), 6 * rows + 1)
    print(f"Halley band e < {rows * h:.4f}: start {far:.3e} rad, after one step {err:.3e} rad")
    assert far <= 2e-3 and err <= 1e-9
    assert worst(rows * h, (rows + 1) * h * (1 - 1e-12), 13)[1] > 1e-9


def test_header_is_what_the_generator_writes(tmp_path):
    """kep_start_tab.h is exactly the output of gen_tables.py for the schedule's
    two-step bound (no hand edits; the generator's own scan asserts 1e-9)."""
    import importlib.util
    path = os.path.join(os.path.dirname(HEADER), "gen_tables.py")
    spec = importlib.util.spec_from_file_location("gen_tables", path)
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    out = tmp_path / "kep_start_tab.h"
    gen.write_start_table(_read_header()[2], out=str(out))
    assert out.read_text() == open(HEADER).read()
