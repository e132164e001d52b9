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
   guess, Sec. 5.4) on the two-step band e <= KEP_S32_E2: E(e_i, M_j) on 17
   eccentricities and 130 knots M_j = j pi / 128, stored as binary16 pairs (value,
   difference to the next eccentricity row) in kep_start_tab.h.  The scan checks that
   bilinear interpolation starts within a few 1e-3 rad of the root and that one Danby
   step from there lands within 1e-9 rad (float64), so the kernels that hold the table
   take the last step only.  A second scan finds the leading rows on which the
   second-order step (Halley's correction) alone already lands within 1e-9 rad
   (KEP_TAB_HALLEY_ROWS): there the kernels take that cheaper step instead.

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
START_NE = 17          # eccentricity rows e_i = i emax / 16
START_NM = 130         # knots M_j = j pi / 128, j = 0 .. 129 (two beyond pi: |M| may round past it)


def _root64(e, M):
    """Root of Kepler's equation in float64 (Danby steps to convergence, then Newton)."""
    E = M + 0.85 * e * np.sign(np.sin(M))
    for _ in range(12):
        E = _danby_step(E, e, M)
    for _ in range(2):
        E = E - (E - e * np.sin(E) - M) / (1 - e * np.cos(E))
    return E


def start_table(emax):
    """Rows i < NE - 1 of binary16 pairs (E(e_i, M_j), E(e_i+1, M_j) - E(e_i, M_j)), knots
    over M >= 0; the difference is taken between the rounded values."""
    M = np.arange(START_NM) * (np.pi / 128)
    T = np.array([_root64(i * emax / (START_NE - 1), M) for i in range(START_NE)]).astype(np.float16)
    pairs = np.empty((START_NE - 1, START_NM, 2), dtype=np.float16)
    pairs[:, :, 0] = T[:-1]
    pairs[:, :, 1] = (T[1:].astype(np.float64) - T[:-1]).astype(np.float16)
    return pairs


def start_lookup(pairs, emax, e, M):
    """The kernels' starting value: bilinear in (e, |M|) from the binary16 pairs, sign of M
    (the interpolation itself in float64)."""
    fi = np.float64(e) * ((START_NE - 1) / emax)
    i = min(int(fi), START_NE - 2)
    we = fi - i
    fj = np.abs(M) * (128 / np.pi)
    j = fj.astype(int)
    wm = fj - j
    p = pairs.astype(np.float64)
    r0 = p[i, j, 0] + we * p[i, j, 1]
    r1 = p[i, j + 1, 0] + we * p[i, j + 1, 1]
    return np.copysign(r0 + wm * (r1 - r0), M)


def start_scan(pairs, emax, n_e=400):
    """Worst distance of the table start from the root, and worst error after one
    Danby step from it (float64), over e in [0, emax] and a dense M grid."""
    M = np.concatenate([np.linspace(-np.pi, np.pi, 20001),
                        np.outer([-1.0, 1.0], np.logspace(-10, 0, 2001)).ravel()])
    far, err = 0.0, 0.0
    for e in np.linspace(0.0, emax, n_e):
        R = _root64(e, M)
        E0 = start_lookup(pairs, emax, e, M)
        far = max(far, float(np.max(np.abs(E0 - R))))
        err = max(err, float(np.max(np.abs(_danby_step(E0, e, M) - R))))
    return far, err


def _halley_step(E, e, M):
    """Second-order member of Danby's family (Halley's correction), float64."""
    s, c = np.sin(E), np.cos(E)
    f = E - e * s - M
    f1 = 1 - e * c
    return E - f * f1 / (f1 * f1 - 0.5 * f * e * s)


def halley_rows(pairs, emax, target=1e-9, n_e=60):
    """Number of leading table rows (e_i <= e <= e_i+1, endpoints included) on which
    one Halley step from the table start lands within `target` of the root (float64),
    and the worst start distance and step error over those rows."""
    M = np.concatenate([np.linspace(-np.pi, np.pi, 20001),
                        np.outer([-1.0, 1.0], np.logspace(-10, 0, 2001)).ravel()])
    rows, far, err = 0, 0.0, 0.0
    for i in range(START_NE - 1):
        row_far, row_err = 0.0, 0.0
        for e in np.linspace(i * emax / (START_NE - 1), (i + 1) * emax / (START_NE - 1), n_e):
            R = _root64(e, M)
            E0 = start_lookup(pairs, emax, e, M)
            row_far = max(row_far, float(np.max(np.abs(E0 - R))))
            row_err = max(row_err, float(np.max(np.abs(_halley_step(E0, e, M) - R))))
        if row_err > target:
            break
        rows, far, err = i + 1, max(far, row_far), max(err, row_err)
    return rows, far, err


def write_start_table(emax, out=START_OUT):
    pairs = start_table(emax)
    far, err = start_scan(pairs, emax)
    assert err <= 1e-9, err
    h_rows, h_far, h_err = halley_rows(pairs, emax)
    lines = [
        "// Generated by gen_tables.py -- do not edit by hand.",
        "#pragma once",
        "",
        "// Starting values for the binary32 Kepler solve at e <= KEP_TAB_EMAX.  With",
        f"// e_i = i KEP_TAB_EMAX / {START_NE - 1} and M_j = j pi / 128, word [i][j] holds the binary16",
        "// pair (E(e_i, M_j), E(e_i+1, M_j) - E(e_i, M_j)) (first value in the low half),",
        "// i < KEP_TAB_NE - 1, j < KEP_TAB_NM.  Bilinear interpolation in (e, |M|) with the sign",
        f"// of M starts at most {far:.2e} rad from the root; one Danby step from there lands",
        f"// within {err:.1e} rad (float64 scan over e and M).",
        f"#define KEP_TAB_NE {START_NE}",
        f"#define KEP_TAB_NM {START_NM}",
        f"#define KEP_TAB_EMAX {emax!r}",
        f"#define KEP_TAB_MSCALE {float(np.float32(128 / np.pi))!r}f",
        f"// On rows i < KEP_TAB_HALLEY_ROWS (e < {h_rows * emax / (START_NE - 1):.4f}) the start lies within {h_far:.2e} rad",
        f"// of the root and one Halley step (second order) from it lands within {h_err:.1e} rad.",
        f"#define KEP_TAB_HALLEY_ROWS {h_rows}",
        "",
        "static __device__ const unsigned int kep_start_tab[(KEP_TAB_NE - 1) * KEP_TAB_NM] = {",
    ]
    bits = pairs.view(np.uint16).astype(np.uint32)
    words = (bits[:, :, 0] | (bits[:, :, 1] << 16)).ravel()
    flat = [f"0x{int(w):08x}u" for w in words]
    for k in range(0, len(flat), 8):
        lines.append("    " + ", ".join(flat[k:k + 8]) + ",")
    lines.append("};")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"start table: far {far:.3e}, one step {err:.3e}; Halley rows {h_rows} (far {h_far:.3e}, "
          f"one step {h_err:.3e})")


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
    write_start_table(s32[2])


if __name__ == "__main__":
    import sys
    if sys.argv[1:] == ["start"]:
        write_start_table(0.8525)
    else:
        main()
