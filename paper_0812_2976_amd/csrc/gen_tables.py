"""Derive the constant tables of the GPU kernels and write kep_tables.h.

1. Polynomials for the single-precision Kepler kernels, on |x| <= pi/2:
       x - sin x  = x^3 * p(x^2)        1 - cos x = x^2 * q(x^2)
   Both are relative-minimax fits (Lawson's iteratively reweighted least
   squares on a dense grid) of the exact functions evaluated in 30-digit
   arithmetic.  Written this way, E - sin E and 1 - cos E keep full relative
   precision near periapsis (E -> 0), where Kepler's function
   f(E) = (1-e) E + e (E - sin E) - M and its slope (1-e) + e (1 - cos E)
   would otherwise cancel catastrophically for e close to 1.
   A second pair, one degree higher, covers |x| <= 3.25 without folding the
   argument: the last step of the eccentricity schedule starts within
   0.015 rad of a root in [-pi, pi] (item 2's scan), so |E| <= 3.143 there.
   Its binary32 coefficients are rounded one at a time from the constant
   term up, the remaining ones refitted after each rounding.

2. Iteration schedules for Danby's quartic iteration started from the paper's
   guess E0 = M + 0.85 e sign(M) (Sec. 4.3) on a centred M in [-pi, pi]:
   for n = 2, 3, 4, 5 the largest eccentricity below which n iterations bring
   the worst error over M within the target (1e-9 rad for the single-precision
   kernels, 1e-15 rad for binary64).  The scan uses a dense grid of M (linear
   plus logarithmic near 0) and e in steps of 1/2000; the threshold is backed
   off by one step.  Above the last threshold the kernels fall back to a
   convergence test with an iteration cap.  There is no one-step band: a
   single step from the starting guess is large (up to 0.85 e), and its own
   binary32 rounding (a few ulp of the step) would exceed the target.

3. Starting values for the binary32 Kepler solve (the paper's interpolated initial
   guess, Sec. 5.4) for e <= 0.9, in three bands of eccentricity: E(e_i, M_j) on
   rows of e and knots M_j = j pi / N (N = 128 up to e = 0.7, 256 above, where the
   root bends more sharply near periapsis), stored as binary16 pairs (value,
   difference to the next eccentricity row) in kep_start_tab.h.  The scan checks that
   bilinear interpolation starts within a few 1e-3 rad of the root and that one step
   from there lands within 1e-9 rad (float64): the second-order step (Halley's
   correction) in the first two bands, Danby's quartic one in the last; the kernels
   that hold the table take that one step only.

Run:  python gen_tables.py         (rewrites kep_tables.h and kep_start_tab.h)
      python gen_tables.py start   (kep_start_tab.h only)
"""
import os

import mpmath as mp
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "kep_tables.h")
mp.mp.dps = 30


def _exact(fun, y):
    return np.array([float(fun(mp.sqrt(mp.mpf(v)))) for v in y])


def _p_exact(x):
    return (x - mp.sin(x)) / x ** 3 if x != 0 else mp.mpf(1) / 6


def _q_exact(x):
    return (1 - mp.cos(x)) / x ** 2 if x != 0 else mp.mpf(1) / 2


def fit_relative_minimax(target, grid, deg, iters=40):
    V = np.vander(grid, deg + 1, increasing=True)
    w = np.ones_like(grid)
    for _ in range(iters):
        W = np.sqrt(w) / target
        c, *_ = np.linalg.lstsq(V * W[:, None], target * W, rcond=None)
        err = np.abs(V @ c - target) / target
        w = w * err
        w /= w.sum()
    c32 = c.astype(np.float32)
    err32 = np.max(np.abs(V @ c32.astype(np.float64) - target) / target)
    return c32, err32


def fit_relative_minimax_f32(target, grid, deg, iters=40):
    """As fit_relative_minimax, with the coefficients rounded to binary32 one at
    a time from the constant term up and the others refitted to the residual."""
    V = np.vander(grid, deg + 1, increasing=True)
    fixed = []
    for k in range(deg + 1):
        resid = target - (V[:, :k] @ np.array(fixed) if k else 0.0)
        Vr = V[:, k:]
        w = np.ones_like(grid)
        for _ in range(iters):
            W = np.sqrt(w) / target
            c, *_ = np.linalg.lstsq(Vr * W[:, None], resid * W, rcond=None)
            err = np.abs(Vr @ c - resid) / target
            w = w * (err + 1e-30)
            w /= w.sum()
        fixed.append(float(np.float32(c[0])))
    c32 = np.array(fixed, dtype=np.float32)
    return c32, np.max(np.abs(V @ c32.astype(np.float64) - target) / target)


def last_step_reach(n_list=(2, 3, 4, 5), bands=None):
    """Largest |E| and distance to the root before the last step of the schedule."""
    M = np.concatenate([np.linspace(-np.pi, np.pi, 20001),
                        np.outer([-1.0, 1.0], np.logspace(-10, 0, 2001)).ravel()])
    far, reach = 0.0, 0.0
    for n, (lo, hi) in bands.items():
        for e in np.linspace(lo, hi, 60):
            E = M + 0.85 * e * np.sign(M)
            for _ in range(n - 1):
                E = _danby_step(E, e, M)
            R = E.copy()
            for _ in range(10):
                R = _danby_step(R, e, M)
            far = max(far, float(np.max(np.abs(E - R))))
            reach = max(reach, float(np.max(np.abs(E))))
    return far, reach


def danby_errors(e, M, n_max):
    """Worst |E_n - E*| over the M grid after n Danby steps (float64, n = 1..n_max)."""
    ld = np.longdouble
    Ml, el = M.astype(ld), ld(e)
    # reference root: Newton in extended precision from a converged Danby start
    E = M + 0.85 * e * np.sign(M)
    for _ in range(12):
        E = _danby_step(E, e, M)
    El = E.astype(ld)
    for _ in range(3):
        El = El - (El - el * np.sin(El) - Ml) / (1 - el * np.cos(El))
    E = M + 0.85 * e * np.sign(M)
    out = []
    for _ in range(n_max):
        E = _danby_step(E, e, M)
        out.append(float(np.max(np.abs(E.astype(ld) - El))))
    return out


def _danby_step(E, e, M):
    s, c = np.sin(E), np.cos(E)
    f = E - e * s - M
    f1, f2, f3 = 1 - e * c, e * s, e * c
    d1 = -f / f1
    d2 = -f / (f1 + 0.5 * d1 * f2)
    d3 = -f / (f1 + 0.5 * d2 * f2 + d2 * d2 * f3 / 6)
    return E + d3


def schedule(target, n_list=(2, 3, 4, 5), step=1.0 / 2000):
    M = np.concatenate([np.linspace(-np.pi, np.pi, 20001),
                        np.outer([-1.0, 1.0], np.logspace(-10, 0, 2001)).ravel()])
    thresholds = {}
    es = np.arange(0.0, 0.9995, step)
    errs = np.array([danby_errors(x, M, max(n_list)) for x in es])
    for n in n_list:
        ok = errs[:, n - 1] <= target
        bad = np.nonzero(~ok)[0]
        first_bad = bad[0] if bad.size else len(es)
        thresholds[n] = float(es[max(first_bad - 1, 0)])   # back off one step
    return thresholds


START_OUT = os.path.join(HERE, "kep_start_tab.h")
# Bands of the starting-value table: (e_lo, e_hi, rows, knots, last step).  Rows
# e_i = e_lo + i (e_hi - e_lo) / rows; knots M_j = j pi / knots, j = 0 .. knots + 1
# (two beyond pi: |M| may round past it).  The knots are denser where the root
# bends more sharply in M (near periapsis at high e); the last step is Halley's
# (second order) where the start is close enough for it, Danby's quartic above.
START_BANDS = ((0.0, 0.7, 14, 128, "halley"), (0.7, 0.85, 6, 256, "halley"), (0.85, 0.9, 2, 256, "quartic"))
STEP_TARGET = 1e-9


def _root64(e, M):
    """Root of Kepler's equation in float64 (Danby steps to convergence, then Newton)."""
    E = M + 0.85 * e * np.sign(np.sin(M))
    for _ in range(12):
        E = _danby_step(E, e, M)
    for _ in range(2):
        E = E - (E - e * np.sin(E) - M) / (1 - e * np.cos(E))
    return E


def _halley_step(E, e, M):
    """Second-order member of Danby's family (Halley's correction), float64."""
    s, c = np.sin(E), np.cos(E)
    f = E - e * s - M
    f1 = 1 - e * c
    return E - f * f1 / (f1 * f1 - 0.5 * f * e * s)


def band_table(e_lo, e_hi, rows, knots):
    """Rows of binary16 pairs (E(e_i, M_j), E(e_i+1, M_j) - E(e_i, M_j)) over M >= 0; the
    difference is taken between the rounded values.  Shape (rows, knots + 2, 2)."""
    M = np.arange(knots + 2) * (np.pi / knots)
    T = np.array([_root64(e_lo + i * (e_hi - e_lo) / rows, M) for i in range(rows + 1)]).astype(np.float16)
    pairs = np.empty((rows, knots + 2, 2), dtype=np.float16)
    pairs[:, :, 0] = T[:-1]
    pairs[:, :, 1] = (T[1:].astype(np.float64) - T[:-1]).astype(np.float16)
    return pairs


def band_lookup(pairs, band, e, M):
    """The kernels' starting value: bilinear in (e, |M|) from a band's binary16 pairs,
    sign of M (the interpolation itself in float64)."""
    e_lo, e_hi, rows, knots, _ = band
    fi = (np.float64(e) - e_lo) * (rows / (e_hi - e_lo))
    i = min(int(fi), rows - 1)
    we = fi - i
    fj = np.abs(M) * (knots / np.pi)
    j = fj.astype(int)
    wm = fj - j
    p = pairs.astype(np.float64)
    r0 = p[i, j, 0] + we * p[i, j, 1]
    r1 = p[i, j + 1, 0] + we * p[i, j + 1, 1]
    return np.copysign(r0 + wm * (r1 - r0), M)


def band_scan(pairs, band, n_per_row=16):
    """Worst distance of a band's start from the root, and worst error after its last
    step (float64), over the band's e range (both ends) and a dense M grid."""
    e_lo, e_hi, rows, _, step = band
    M = np.concatenate([np.linspace(-np.pi, np.pi, 20001),
                        np.outer([-1.0, 1.0], np.logspace(-10, 0, 2001)).ravel()])
    far, err = 0.0, 0.0
    for e in np.linspace(e_lo, e_hi, n_per_row * rows + 1):
        R = _root64(e, M)
        E0 = band_lookup(pairs, band, e, M)
        E1 = _halley_step(E0, e, M) if step == "halley" else _danby_step(E0, e, M)
        far = max(far, float(np.max(np.abs(E0 - R))))
        err = max(err, float(np.max(np.abs(E1 - R))))
    return far, err


def write_start_table(bands=START_BANDS, out=START_OUT):
    tables, scans, offs = [], [], []
    off = 0
    for b in bands:
        pairs = band_table(*b[:4])
        far, err = band_scan(pairs, b)
        assert err <= STEP_TARGET, (b, err)
        tables.append(pairs)
        scans.append((far, err))
        offs.append(off)
        off += pairs.shape[0] * pairs.shape[1]
    lines = [
        "// Generated by gen_tables.py -- do not edit by hand.",
        "#pragma once",
        "",
        "// Starting values for the binary32 Kepler solve at e <= KEP_TAB_EMAX, in bands of",
        "// eccentricity.  In band b, row i (e_i = e0 + i (e1 - e0) / rows) and knot",
        "// M_j = j pi / knots (j = 0 .. knots + 1), word KEP_TAB_BAND_OFF[b] + i (knots + 2) + j",
        "// holds the binary16 pair (E(e_i, M_j), E(e_i+1, M_j) - E(e_i, M_j)) (first value in",
        "// the low half).  Bilinear interpolation in (e, |M|) with the sign of M, then one",
        "// step: Halley's where KEP_TAB_BAND_HALLEY[b] is 1, Danby's quartic where it is 0.",
        "// float64 scan over each band's e range and M:",
    ]
    for b, (far, err) in zip(bands, scans):
        lines.append(f"//   e in [{b[0]}, {b[1]}], {b[2]} rows, {b[3]} knots: start within {far:.2e} rad, "
                     f"{b[4]} step within {err:.1e} rad")
    fmt = lambda xs: "{" + ", ".join(xs) + "}"
    lines += [
        f"#define KEP_TAB_EMAX {bands[-1][1]!r}",
        f"#define KEP_TAB_NBANDS {len(bands)}",
        f"#define KEP_TAB_BAND_E0 {fmt(repr(float(b[0])) for b in bands)}",
        f"#define KEP_TAB_BAND_E1 {fmt(repr(float(b[1])) for b in bands)}",
        f"#define KEP_TAB_BAND_ROWS {fmt(str(b[2]) for b in bands)}",
        f"#define KEP_TAB_BAND_KNOTS {fmt(str(b[3]) for b in bands)}",
        f"#define KEP_TAB_BAND_OFF {fmt(str(o) for o in offs)}",
        f"#define KEP_TAB_BAND_HALLEY {fmt('1' if b[4] == 'halley' else '0' for b in bands)}",
        f"#define KEP_TAB_WORDS {off}",
        "",
        "static __device__ const unsigned int kep_start_tab[KEP_TAB_WORDS] = {",
    ]
    flat = []
    for pairs in tables:
        bits = pairs.view(np.uint16).astype(np.uint32)
        flat += [f"0x{int(w):08x}u" for w in (bits[:, :, 0] | (bits[:, :, 1] << 16)).ravel()]
    for k in range(0, len(flat), 8):
        lines.append("    " + ", ".join(flat[k:k + 8]) + ",")
    lines.append("};")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    for b, (far, err) in zip(bands, scans):
        print(f"start table band {b}: far {far:.3e}, one step {err:.3e}")


def main():
    ymax = (np.pi / 2) ** 2 * 1.001
    grid = np.linspace(0.0, ymax, 3001)
    p, ep = fit_relative_minimax(_exact(_p_exact, grid), grid, 4)
    q, eq = fit_relative_minimax(_exact(_q_exact, grid), grid, 4)
    wmax = 3.25
    gridw = np.linspace(0.0, wmax * wmax, 3001)
    pw, epw = fit_relative_minimax_f32(_exact(_p_exact, gridw), gridw, 5)
    qw, eqw = fit_relative_minimax_f32(_exact(_q_exact, gridw), gridw, 5)
    pi_hi = np.float32(np.pi)
    pi_lo = np.float32(float(mp.pi - mp.mpf(float(pi_hi))))
    s32 = schedule(1e-9)
    s64 = schedule(1e-15)
    bands = {2: (0.0, s32[2]), 3: (s32[2], s32[3]), 4: (s32[3], s32[4]), 5: (s32[4], s32[5])}
    far, reach = last_step_reach(bands=bands)
    assert reach < wmax, (reach, wmax)
    lines = [
        "// Generated by gen_tables.py -- do not edit by hand.",
        "#pragma once",
        "",
        "// x - sin x = x^3 p(x^2), 1 - cos x = x^2 q(x^2) on |x| <= pi/2 (relative minimax,",
        f"// max relative error with float coefficients: p {ep:.2e}, q {eq:.2e}).",
    ]
    for name, c in (("KEP_P", p), ("KEP_Q", q)):
        for i, v in enumerate(c):
            lines.append(f"#define {name}{i} {float(v)!r}f")
    lines += [
        f"// The same on |x| <= {wmax} without folding (one degree higher; max relative error",
        f"// p {epw:.2e}, q {eqw:.2e}): the last step of the schedule starts at most {far:.3f} rad",
        f"// from the root, at |E| <= {reach:.4f}.",
    ]
    for name, c in (("KEP_PW", pw), ("KEP_QW", qw)):
        for i, v in enumerate(c):
            lines.append(f"#define {name}{i} {float(v)!r}f")
    lines += [
        f"#define KEP_PI_HI_F {float(pi_hi)!r}f",
        f"#define KEP_PI_LO_F {float(pi_lo)!r}f",
        "",
        "// Danby iterations from E0 = M + 0.85 e sign(M), M centred on [-pi, pi]:",
        "// n iterations are enough (worst error over M below the target) for e <= KEP_S*_E<n>.",
        "// Single precision target 1e-9 rad; binary64 target 1e-15 rad.",
    ]
    for tag, s in (("KEP_S32", s32), ("KEP_S64", s64)):
        for n, v in s.items():
            lines.append(f"#define {tag}_E{n} {v!r}")
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(open(OUT).read())
    write_start_table()


if __name__ == "__main__":
    import sys
    if sys.argv[1:] == ["start"]:
        write_start_table()
    else:
        main()
