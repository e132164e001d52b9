"""Independent high-precision (mpmath) formulas used to pin the CPU oracle.

Nothing here calls the oracle or the GPU library.  The velocity is written in
the eccentric-anomaly form v = K b [b cos(w) cos E - sin(w) sin E] / (1 - e cos E)
with b = sqrt(1 - e^2), a different formula from the oracle's true-anomaly form
K [cos(w + f) + e cos w]; the two agree only if both are right.
"""
import mpmath as mp

mp.mp.dps = 40


def kepler_bisect(M, e, halvings=200):
    """Root of E - e sin E = M by plain bisection on [M - e, M + e] (Eq. 1)."""
    M = mp.mpf(M)
    e = mp.mpf(e)
    lo, hi = M - e, M + e
    for _ in range(halvings):
        mid = (lo + hi) / 2
        if mid - e * mp.sin(mid) - M > 0:
            hi = mid
        else:
            lo = mid
    return (lo + hi) / 2


def phase_frac(t, t0, P):
    """Fractional orbit phase with the binary64 quotient of the paper's mean-anomaly bracket."""
    q = (float(t) - float(t0)) / float(P)        # IEEE binary64, as prescribed
    return mp.mpf(q) - mp.floor(mp.mpf(q))


def mean_anomaly(t, t0, P, M0):
    M = 2 * mp.pi * phase_frac(t, t0, P) + mp.mpf(M0)
    return M - 2 * mp.pi * mp.floor(M / (2 * mp.pi))


def planet_rv_eform(t, t0, P, K, e, w, M0):
    M = mean_anomaly(t, t0, P, M0)
    E = kepler_bisect(M, e)
    e = mp.mpf(e)
    b = mp.sqrt((1 - e) * (1 + e))
    return mp.mpf(K) * b * (b * mp.cos(w) * mp.cos(E) - mp.sin(w) * mp.sin(E)) / (1 - e * mp.cos(E))


def planet_rv_exact_phase(t, t0, P, K, e, w, M0):
    """Same velocity with the phase computed exactly (no binary64 rounding of q):
    a smooth function of every parameter, used for high-precision derivatives."""
    q = (mp.mpf(t) - mp.mpf(t0)) / mp.mpf(P)
    M = 2 * mp.pi * q + mp.mpf(M0)
    E = kepler_bisect(M, e, halvings=160)
    e = mp.mpf(e)
    b = mp.sqrt((1 - e) * (1 + e))
    return mp.mpf(K) * b * (b * mp.cos(w) * mp.cos(E) - mp.sin(w) * mp.sin(E)) / (1 - e * mp.cos(E))
