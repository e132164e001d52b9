"""The starting-value table of the binary32 Kepler solve (kep_start_tab.h), checked
on the CPU against the oracle's roots (no GPU).

The header documents its contents: bands of eccentricity, each with rows
e_i = e0 + i (e1 - e0) / rows and knots M_j = j pi / knots, holding binary16 pairs
(E(e_i, M_j), E(e_i+1, M_j) - E(e_i, M_j)).  The tests read the header, check every
entry against the oracle's root rounded to binary16, and check the property the
kernels rely on: the bilinear start lies within 2e-3 rad of the root, and one step
from there lands within 1e-9 rad (float64) -- Halley's correction (the second-order
member of Sec. 4.3's family) in the bands marked for it, Danby's quartic correction
in the others -- over each band's e range and a dense grid of M including M -> 0 and
|M| -> pi.
"""
import math
import os
import re

import numpy as np
import pytest

import oracle

HEADER = os.path.join(os.path.dirname(__file__), "..", "paper_0812_2976_amd", "csrc", "kep_start_tab.h")
PI_F = float(np.float32(math.pi))


def _read_header():
    text = open(HEADER).read()
    scal = dict(re.findall(r"#define (KEP_TAB_\w+) ([0-9.eE+-]+)\s*$", text, re.M))
    arr = {k: [float(x) for x in v.split(",")] for k, v in re.findall(r"#define (KEP_TAB_\w+) \{([^}]*)\}", text)}
    body = text[text.index("= {") + 3:text.rindex("}")]
    words = np.array([int(w, 16) for w in re.findall(r"0x([0-9a-f]{8})u", body)], dtype=np.uint32)
    assert words.size == int(scal["KEP_TAB_WORDS"])
    lo = (words & 0xFFFF).astype(np.uint16).view(np.float16).astype(np.float64)
    hi = (words >> 16).astype(np.uint16).view(np.float16).astype(np.float64)
    bands = []
    for b in range(int(scal["KEP_TAB_NBANDS"])):
        rows, knots, off = (int(arr[k][b]) for k in ("KEP_TAB_BAND_ROWS", "KEP_TAB_BAND_KNOTS", "KEP_TAB_BAND_OFF"))
        n = rows * (knots + 2)
        bands.append(dict(e0=arr["KEP_TAB_BAND_E0"][b], e1=arr["KEP_TAB_BAND_E1"][b], rows=rows, knots=knots,
                          off=off, halley=int(arr["KEP_TAB_BAND_HALLEY"][b]) == 1,
                          T=lo[off:off + n].reshape(rows, knots + 2), D=hi[off:off + n].reshape(rows, knots + 2)))
    return float(scal["KEP_TAB_EMAX"]), int(scal["KEP_TAB_WORDS"]), bands


def _band_of(bands, e):
    """The kernels' band: the last one whose e0 <= e."""
    return [bd for bd in bands if e >= bd["e0"]][-1]


def _start(bd, e, M):
    """The kernels' starting value (bilinear in e and |M|, sign of M), in float64."""
    fi = (e - bd["e0"]) * (bd["rows"] / (bd["e1"] - bd["e0"]))
    i = min(int(fi), bd["rows"] - 1)
    we = fi - i
    fj = np.minimum(np.abs(M), PI_F) * (bd["knots"] / math.pi)
    j = fj.astype(int)
    wm = fj - j
    r0 = bd["T"][i, j] + we * bd["D"][i, j]
    r1 = bd["T"][i, j + 1] + we * bd["D"][i, j + 1]
    return np.copysign(r0 + wm * (r1 - r0), M)


def _danby(E, e, M):
    """One step of Danby's quartic iteration (Sec. 4.3) in float64."""
    f = E - e * np.sin(E) - M
    f1, f2, f3 = 1 - e * np.cos(E), e * np.sin(E), e * np.cos(E)
    d1 = -f / f1
    d2 = -f / (f1 + d1 * f2 / 2)
    d3 = -f / (f1 + d2 * f2 / 2 + d2 * d2 * f3 / 6)
    return E + d3


def _halley(E, e, M):
    """One step of the second-order member of Danby's family (Halley's correction,
    Sec. 4.3's d2 = -f / (f' + d1 f''/2) with d1 = -f / f'), float64."""
    f = E - e * np.sin(E) - M
    f1, f2 = 1 - e * np.cos(E), e * np.sin(E)
    d1 = -f / f1
    return E - f / (f1 + d1 * f2 / 2)


M_GRID = np.concatenate([np.linspace(-math.pi, math.pi, 8001),
                         np.outer([-1.0, 1.0], np.logspace(-9, 0, 400)).ravel(),
                         [math.pi - 1e-7, -math.pi + 1e-7]])


def _worst(bd, step, n):
    far, err = 0.0, 0.0
    for e in np.linspace(bd["e0"], bd["e1"] * (1 - 1e-12), n):
        R = oracle.kepler(M_GRID, np.full(M_GRID.size, e))
        E0 = _start(bd, e, M_GRID)
        far = max(far, float(np.max(np.abs(E0 - R))))
        err = max(err, float(np.max(np.abs(step(E0, e, M_GRID) - R))))
    return far, err


@pytest.fixture(scope="module")
def tab():
    return _read_header()


def test_bands_tile_the_range(tab):
    """The bands cover [0, KEP_TAB_EMAX] without gaps, their words are laid out one
    after the other, and every row has knots + 2 words (two knots beyond pi)."""
    emax, words, bands = tab
    assert 0.5 < emax < 1.0 and bands[0]["e0"] == 0.0 and bands[-1]["e1"] == emax
    off = 0
    for a, b in zip(bands, bands[1:]):
        assert a["e1"] == b["e0"]
    for bd in bands:
        assert bd["off"] == off and bd["rows"] >= 1 and bd["knots"] >= 128
        off += bd["rows"] * (bd["knots"] + 2)
    assert off == words


def test_entries_are_rounded_roots(tab):
    """Every first half is the oracle's root E(e_i, M_j) rounded to binary16; every
    second half the rounded difference to the next row (for a band's last row, the
    root at the band's upper edge on the same knots)."""
    _, _, bands = tab
    for bd in bands:
        M = np.arange(bd["knots"] + 2) * (math.pi / bd["knots"])
        es = [bd["e0"] + i * (bd["e1"] - bd["e0"]) / bd["rows"] for i in range(bd["rows"] + 1)]
        r16 = np.array([oracle.kepler(M, np.full(M.size, e)) for e in es]).astype(np.float16).astype(np.float64)
        assert np.array_equal(bd["T"], r16[:-1])
        assert np.array_equal(bd["D"], (r16[1:] - r16[:-1]).astype(np.float16).astype(np.float64))
        assert bd["T"][0, 0] == 0.0 and np.all(np.diff(bd["T"], axis=1) > 0)       # E(M) increases with M


def test_start_and_one_step(tab):
    """In every band the start lies within 2e-3 rad of the oracle's root and the band's
    step (Halley's or Danby's quartic) lands within 1e-9 rad; where the band takes
    Halley's step the start is within the 2e-3 rad that the two-term rotation of sin and
    cos after it assumes."""
    _, _, bands = tab
    for bd in bands:
        far, err = _worst(bd, _halley if bd["halley"] else _danby, 6 * bd["rows"] + 1)
        print(f"band [{bd['e0']}, {bd['e1']}] ({'Halley' if bd['halley'] else 'quartic'}): "
              f"start {far:.3e} rad, after one step {err:.3e} rad")
        assert far <= 2e-3 and err <= 1e-9


def test_quartic_band_needs_the_quartic_step(tab):
    """A band left on the quartic step is one where Halley's step would miss 1e-9 rad."""
    _, _, bands = tab
    quartic = [bd for bd in bands if not bd["halley"]]
    assert quartic
    for bd in quartic:
        assert _worst(bd, _halley, 4 * bd["rows"] + 1)[1] > 1e-9


def test_band_choice_at_the_edges(tab):
    """The kernels' band choice: a band's own lower edge belongs to it, and e just
    below it to the band before."""
    _, _, bands = tab
    for a, b in zip(bands, bands[1:]):
        assert _band_of(bands, b["e0"]) is b
        assert _band_of(bands, float(np.nextafter(b["e0"], 0.0))) is a


def test_header_is_what_the_generator_writes(tmp_path):
    """kep_start_tab.h is exactly the output of gen_tables.py (no hand edits; the
    generator's own scan asserts 1e-9 after each band's step)."""
    import importlib.util
    path = os.path.join(os.path.dirname(HEADER), "gen_tables.py")
    spec = importlib.util.spec_from_file_location("gen_tables", path)
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    out = tmp_path / "kep_start_tab.h"
    gen.write_start_table(out=str(out))
    assert out.read_text() == open(HEADER).read()
