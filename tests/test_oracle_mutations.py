"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (on the CPU,
in a temporary directory), builds it, and runs the pin suite against the
broken copy in a subprocess: the suite has to fail.
"""
import os
import subprocess
import sys

import pytest

from oracle import build as obuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "sign_of_e_cos_omega": ("+ (ld)e * cosl((ld)w));", "- (ld)e * cosl((ld)w));"),
    "minus_M0": ("ld M = TWO_PI_L * (ld)phi + (ld)M0;", "ld M = TWO_PI_L * (ld)phi - (ld)M0;"),
    "half_angle_dropped": ("sinl(0.5L * E), sqrtl(1.0L - e) * cosl(0.5L * E)", "sinl(E), sqrtl(1.0L - e) * cosl(E)"),
    "sqrt_swapped": ("sqrtl(1.0L + e) * sinl(0.5L * E), sqrtl(1.0L - e)", "sqrtl(1.0L - e) * sinl(0.5L * E), sqrtl(1.0L + e)"),
    "weight_sigma_not_squared": ("ld var = (ld)sigma * (ld)sigma + (ld)s * (ld)s;", "ld var = (ld)sigma + (ld)s * (ld)s;"),
    "jitter_dropped": ("ld var = (ld)sigma * (ld)sigma + (ld)s * (ld)s;", "ld var = (ld)sigma * (ld)sigma;"),
    "offset_dropped": ("if (d->offset) sum += (ld)d->offset[i];", ""),
    "dfde_factor": ("ld dfde = sinl(f) * (2.0L + e * cosl(f)) / one_m_e2;", "ld dfde = sinl(f) * (1.0L + e * cosl(f)) / one_m_e2;"),
    "dP_sign": ("ld dv_dP = dv_dM0 * (-TWO_PI_L * q / P);", "ld dv_dP = dv_dM0 * (TWO_PI_L * q / P);"),
    "dfdM_power": ("ld dfdM = ecf * ecf / (one_m_e2 * b);", "ld dfdM = ecf * ecf / one_m_e2;"),
    "kepler_wrong_sign": ("ld g = E - e * sinl(E) - M;\n        if (g == 0.0L) return E;", "ld g = E + e * sinl(E) - M;\n        if (g == 0.0L) return E;"),
    "phase_not_binary64": ("double q = dt / P;", "double q = (double)((float)dt / (float)P);"),
    "nll_log_term_dropped": ("sum_logvar -= logl(wk);", ""),
    "nll_jitter_grad_sign": ("(2.0L * s * (sum_w - sum_w2r2))", "(2.0L * s * (sum_w2r2 - sum_w))"),
    "gn_weight_dropped": ("JJ[a * np - a * (a - 1) / 2 + (b - a)] += wk * row[a] * row[b];",
                          "JJ[a * np - a * (a - 1) / 2 + (b - a)] += row[a] * row[b];"),
    "gn_jtwr_sign": ("Jr[a] += wk * row[a] * r;", "Jr[a] -= wk * row[a] * r;"),
    "gn_offset_column": ("row[np - 1] = 1.0L;", "row[np - 1] = 0.0L;"),
    # gradient error scales
    "scale_r_abs_dropped": ("sr[5 * j + a] += fabsl(c * dv[a]);", "sr[5 * j + a] += c * dv[a];"),
    "scale_1_factor_two_dropped": ("s1[5 * j + a] += 2.0L * wk * fabsl(dv[a]);", "s1[5 * j + a] += wk * fabsl(dv[a]);"),
    "scale_1_weight_dropped": ("s1[npar - 1] += 2.0L * wk;", "s1[npar - 1] += 2.0L;"),
    "scale_r_offset_abs_dropped": ("sr[npar - 1] += fabsl(c);", "sr[npar - 1] += c;"),
    "scale_row_mixup": ("s1[5 * j + a] += 2.0L * wk * fabsl(dv[a]);", "s1[5 * j + a] += 2.0L * wk * fabsl(dv[(a + 1) % 5]);"),
    # population sampler (pins in test_oracle_demc.py)
    "demc_acceptance_without_half": ("if (2.0 * log(u) < c_old - c_new)", "if (log(u) < c_old - c_new)", "demc"),
    "demc_own_half_differences": ("const double *xo = s->x + (int64_t)(1 - h) * d * nh;", "const double *xo = xh;",
                                  "demc"),
    "demc_pair_not_distinct": ("if (r2 >= r1) r2 += 1u;", "", "demc"),
    "demc_no_K_support": ("if (!(y[n + j] >= 0.0)) return NAN;", "if (0) return NAN;", "demc"),
    "philox_round_order": ("uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;", "uint32_t n0 = (uint32_t)(pa >> 32) ^ c1 ^ k0;",
                           "demc"),
    # astrometric model (pins in test_oracle_astro.py)
    "astro_Y_without_b": ("ld Y = sqrtl((1.0L - e) * (1.0L + e)) * sinl(E);", "ld Y = sinl(E);", "astro"),
    "astro_X_sign_of_e": ("ld X = cosl(E) - e;", "ld X = cosl(E) + e;", "astro"),
    "astro_ra_uses_A": ("sra += (ld)d->B[p] * X + (ld)d->G[p] * Y;", "sra += (ld)d->A[p] * X + (ld)d->G[p] * Y;",
                        "astro"),
    "astro_sigma_not_squared": ("acc += rx * rx / ((ld)sx * (ld)sx) + ry * ry / ((ld)sy * (ld)sy);",
                                "acc += rx * rx / (ld)sx + ry * ry / ((ld)sy * (ld)sy);", "astro"),
}
PIN_FILES = {None: "test_oracle_pins.py", "demc": "test_oracle_demc.py", "astro": "test_oracle_astro.py"}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new, *which = MUTANTS[name]
    pins = PIN_FILES[which[0] if which else None]
    src = open(obuild.SRC).read()
    assert src.count(old) >= 1, name
    mutated = tmp_path / "mutant.c"
    mutated.write_text(src.replace(old, new))
    lib = obuild.build(src=str(mutated), out=str(tmp_path / "libmutant.so"))
    env = dict(os.environ, KEP_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", pins)],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins did not catch mutant {name}:\n{r.stdout[-2000:]}"
