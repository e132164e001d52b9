"""Benchmark: batched Keplerian RV chi-square on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--rows ...]

One step is one chi-square evaluation of the whole batch through the fused
mixed-precision kernel (mean anomaly in binary64, Kepler solve, velocity,
planet sum and compensated chi-square in binary32, binary64 final sum) on the
workload of 1,048,576 systems x 4 planets x 256 observations, inputs resident
in device memory.  W untimed steps, then K timed steps bracketed by
torch.cuda.synchronize(), timed with HIP events on the launch stream.

Printed as ONE JSON line: the headline value (chi-square evaluations per
second), Kepler solves per second, the binary64 plain kernel on the
65,536 x 4 x 256 workload and the speed-up over it, the VALU roofline of the
fused kernel, the CPU oracle on a bounded sample, and one entry per other
path (gradient, ragged batch, standalone Kepler solve).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peak of the formulation's operation mix on MI355X (256 CUs x 4 SIMDs at
# 2.4 GHz).  Per SIMD and cycle the chip completes 32 binary32 lane operations
# (the published 157.3 TFLOP/s FP32 vector rate = 1024 SIMDs x 32 lanes x 2
# flops x 2.4 GHz), 16 binary64 ones (78.6 TFLOP/s) and 8 transcendental ones
# (hardware sine, cosine, reciprocal: a quarter of the binary32 rate).  A mix
# of n32 + n64 + ntr operations per triple needs n32/32 + n64/16 + ntr/8 SIMD
# cycles; its peak is the operation count over that time.
SIMDS, CLOCK_HZ = 256 * 4, 2.4e9
LANES_PER_CYCLE = {"f32": 32, "f64": 16, "trans": 8}


# Algorithmic VALU operations per (system, planet, observation) triple of the
# mixed-precision formulation (operation count of the method as written, each
# add/mul/fma/fract/convert/compare/select/reciprocal/sine/cosine counted once;
# in brackets the binary64 and transcendental ones, the rest binary32):
#   orbital phase in binary64: (t - t0)/P + phase offset as one fused
#     multiply-add 1, fraction 1, scale to [-pi, pi) 1, convert 1          4  [4 f64]
#   starting value at e <= 0.9 (the table of kep_start_tab.h): |M|
#     scaled 1, knot index and fraction 2, address 1, two interpolations
#     in e 2 (binary16 operands widened inside the multiply-add), one in
#     |M| 2, sign of M 1                                                     9  [one LDS read]
#   at e > 0.9 instead: the paper's starting guess 2, and each Danby
#     step before the last: scale, hardware sin and cos 3, f and its
#     three derivatives 5, three corrections with one reciprocal 11,
#     update 1                                                            20  [3 trans]
#   last step in the table's Halley bands (e < 0.85): Halley's
#     correction: sin, 1 - cos, E - sin E from the unfolded
#     polynomials on |E| <= 3.25 (square 1, two degree-5 polynomials 10,
#     cube, three products 4) 15, f and f' 3, f f''/2 2, denominator 1,
#     reciprocal 1, numerator 1, step and update 2                         25  [1 trans]
#   last step elsewhere: Danby's quartic correction: polynomials 15, f and
#     its three derivatives 5, three corrections with one reciprocal 11,
#     update and step 2                                                   33  [1 trans]
#   sin/1-cos carried to the final E: two-term rotation after the Halley
#     step 8, the full one 11; velocity 5 (D, numerator 2, reciprocal,
#     product); planet sum in binary64 (convert, add) 2                    [1 trans, 2 f64]
#   per observation: binary64 residual (two adds) and its binary32 copy 3,
#     weighted residual 1, binary64 accumulation of w r^2 (convert, fused
#     multiply-add) 2 -> 6 / n_pl                                                [5 f64]
# With e ~ U[0, e_max] the planets split into the three kinds by their share of
# [0, e_max]; beyond the table (0.9 < e <= 0.975 on the eccentricity schedule)
# a planet takes two steps before the last.
OPS_PHASE, OPS_TABLE, OPS_START, OPS_FAST = 4, 9, 2, 20
OPS_HALLEY, OPS_LAST, OPS_ROT_SMALL, OPS_ROT = 25, 33, 8, 11
OPS_VEL, OPS_SUM, OPS_OBS = 5, 2, 6
F64_PHASE, F64_SUM, F64_OBS = 4, 2, 5
TRANS_FAST, TRANS_LAST, TRANS_VEL = 3, 1, 1


def start_table_bands():
    """The starting-value table's bands from kep_start_tab.h: (e0, e1, Halley step)."""
    txt = open(os.path.join(ROOT, "paper_0812_2976_amd", "csrc", "kep_start_tab.h")).read()
    arr = {k: [float(x) for x in v.split(",")] for k, v in re.findall(r"#define (KEP_TAB_\w+) \{([^}]*)\}", txt)}
    return list(zip(arr["KEP_TAB_BAND_E0"], arr["KEP_TAB_BAND_E1"], (h == 1 for h in arr["KEP_TAB_BAND_HALLEY"])))


def mixed_ops_per_triple(n_pl, f_table, early, f_halley=0.0):
    """f_table: fraction of the planets started from the table (f_halley of them on
    the Halley rows); early: mean Danby steps before the last per triple."""
    return (OPS_PHASE + f_table * OPS_TABLE + (1.0 - f_table) * OPS_START + OPS_FAST * early
            + f_halley * (OPS_HALLEY + OPS_ROT_SMALL) + (1.0 - f_halley) * (OPS_LAST + OPS_ROT)
            + OPS_VEL + OPS_SUM + OPS_OBS / n_pl)


def mixed_op_classes(n_pl, f_table, early, f_halley=0.0):
    """The operations of mixed_ops_per_triple by class: binary64, transcendental, binary32."""
    f64 = F64_PHASE + F64_SUM + F64_OBS / n_pl
    trans = TRANS_FAST * early + TRANS_LAST + TRANS_VEL
    return {"f32": mixed_ops_per_triple(n_pl, f_table, early, f_halley) - f64 - trans, "f64": f64, "trans": trans}


def mix_peak_ops_per_s(classes):
    """Operations per second of a mix at the per-class lane rates (LANES_PER_CYCLE)."""
    cycles = sum(n / LANES_PER_CYCLE[c] for c, n in classes.items())
    return sum(classes.values()) / cycles * SIMDS * CLOCK_HZ


def table_fraction(e_max):
    """Fraction of e ~ U[0, e_max] inside the starting-value table's range."""
    return min(e_max, start_table_bands()[-1][1]) / e_max


def halley_fraction(e_max):
    """Fraction of e ~ U[0, e_max] in the table bands that take the Halley step."""
    return sum(max(0.0, min(e_max, e1) - e0) for e0, e1, h in start_table_bands() if h) / e_max


def early_steps(e_max, s3=0.975):
    """Mean Danby steps before the last per planet at e ~ U[0, e_max <= s3]: planets
    beyond the table's range follow the schedule, two early steps up to s3."""
    return 2.0 * max(0.0, min(e_max, s3) - start_table_bands()[-1][1]) / e_max


def op_fractions(e):
    """(f_table, early, f_halley) of mixed_ops_per_triple for the given planets'
    eccentricities: inside the table's bands one step (Halley's on its rows), beyond
    it the eccentricity schedule's steps before the last (2 to e = 0.975, 3 to 0.9955,
    4 to 0.999, 5 above)."""
    e = np.asarray(e, dtype=np.float64).ravel()
    bands = start_table_bands()
    in_tab = e <= bands[-1][1]
    halley = np.zeros(e.shape, dtype=bool)
    for e0, e1, h in bands:
        if h:
            halley |= (e >= e0) & (e < e1)
    steps = np.select([e <= 0.975, e <= 0.9955, e <= 0.999], [2.0, 3.0, 4.0], 5.0)
    early = np.where(in_tab, 0.0, steps)
    return float(in_tab.mean()), float(early.mean()), float((halley & in_tab).mean())


# The sources each timed kernel is compiled from (its counter summaries under
# profiles/ record their hash; a summary taken on other sources is not used).
DENSE_FILES = ("kep_kernels.hip", "kep_policy.h", "kep_device.h", "kep_tables.h", "kep_start_tab.h", "kep_grad.h")
ADJOINT_FILES = ("kep_adjoint.hip", "kep_grad.h", "kep_policy.h", "kep_device.h", "kep_tables.h", "kep_start_tab.h")


_CODE_TOKENS = re.compile(r'//[^\n]*|/\*.*?\*/|"(?:\\.|[^"\\])*"|\S+', re.S)


def code_tokens(text):
    """The source's tokens with comments dropped (string literals kept whole), so
    that an edit of comments or layout leaves the hash unchanged."""
    return [t for t in _CODE_TOKENS.findall(text) if not t.startswith(("//", "/*"))]


def kernel_source_hash(files=DENSE_FILES):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_0812_2976_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(" ".join(code_tokens(fh.read())).encode())
            h.update(b"\0")
    return h.hexdigest()[:16]


def recorded_traffic(name, files=DENSE_FILES):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{name}_traffic.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_h = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", txt)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_h or not m_b or m_h.group(1) != kernel_source_hash(files):
        return None
    return float(m_b.group(1))


# Algorithmic operations per (system, planet, observation) triple of the mixed
# adjoint (kep_adjoint.hip), counted as for the chi-square above; binary64 ones
# in the f64 class, hardware reciprocals in trans:
#   pass 1: orbital phase with the correctly rounded quotient (product, exact
#     remainder, correction, fraction, offset, fraction, scale) and the
#     conversion 8 f64; starting value 10; last step 25 on the Halley rows of
#     the table, 33 (Danby's quartic) above them (1 trans);
#   binary64 correction: the root moved onto [-3.25, 3.25] 3 f32-class;
#     sin/cos of the binary32 root from the nearest knot n/64 (scale,
#     rounding, conversion, remainder and address 5 f32-class; remainder to
#     binary64 1, square 1, sin y to y^5 3, cos y to y^6 3, rotation by the
#     knot 4: 12 f64), residual of Kepler's equation 2, D 1 + its binary32
#     reciprocal (1 trans), corrected step with the second-order term 5 f64
#     + 6 f32, sin/cos carried to the corrected root 6 f64 + 2 f32, velocity
#     8 f64 (1 trans), planet sum 1: 35 f64, 16 f32, 2 trans;
#   pass 2: 1/D (1 trans), cos f, sin f, sin(w+f), df/dM and the five terms
#     (two in their cancellation-free forms) 23, the quotient for dv/dP 2 f64,
#     five weighted accumulations 5: 28 f32, 2 f64, 1 trans;
#   per observation (/ n_pl): residual 2 f64, weight 2 f32 + 1 trans,
#     chi-square 1 f64, 2 w r and the offset row 2 f32;
#   per group of 64 NCH observations: the 5 n_pl + 1 lane sums reduced across
#     the wavefront (R - 1 exchanges, two selects and an add each, R the next
#     power of two), spread over the group's 64 NCH n_pl triples per lane.
ADJ_F64, ADJ_F32, ADJ_TRANS = 8 + 35 + 2, 10 + 16 + 28, 1 + 2 + 1
ADJ_OBS = {"f64": 3, "f32": 4, "trans": 1}


def adjoint_op_classes(n_pl, nch, f_halley=0.0):
    """f_halley: fraction of the planets whose last step is Halley's (the rest take
    Danby's quartic one; the adjoint's batches all lie within the table)."""
    r = 1
    while r < 5 * n_pl + 1:
        r *= 2
    red = 3.0 * (r - 1) / (nch * n_pl)
    last = f_halley * OPS_HALLEY + (1.0 - f_halley) * OPS_LAST
    return {"f32": ADJ_F32 + last + ADJ_OBS["f32"] / n_pl + red, "f64": ADJ_F64 + ADJ_OBS["f64"] / n_pl,
            "trans": ADJ_TRANS + ADJ_OBS["trans"] / n_pl}


def roofline_entry(kernel, classes, units, ms, traffic=None, unit_name="triple"):
    """The VALU roofline of a kernel: classes are operations per unit by class,
    units per launch, ms the mean launch time."""
    per_unit = sum(classes.values())
    achieved = per_unit * units / (ms * 1e-3) / 1e12
    peak = mix_peak_ops_per_s(classes) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": "TOP/s",
            "frac": round(achieved / peak, 4), "traffic": traffic, "kernel": kernel,
            f"ops_per_{unit_name}": round(per_unit, 2),
            f"ops_per_{unit_name}_by_class": {c: round(n, 3) for c, n in classes.items()},
            "units_per_launch": units, "launch_ms": round(ms, 4)}


def hbm_roofline(kernel, bytes_per_launch, ms, basis):
    """The HBM roofline of a streaming kernel: algorithmic bytes of one launch over its
    mean launch time, against the 8 TB/s of MI355X's HBM3E."""
    achieved = bytes_per_launch / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
            "frac": round(achieved / 8000.0, 4), "traffic": None, "kernel": kernel,
            "bytes_per_launch": int(bytes_per_launch), "bytes_basis": basis, "launch_ms": round(ms, 4)}


def cpu_threads():
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return max(1, min(cores, 16))


def time_oracle(fn, n, cores):
    """Wall seconds of fn(i0, i1) over [0, n) split across `cores` host threads."""
    from concurrent.futures import ThreadPoolExecutor
    bounds = np.linspace(0, n, cores * 4 + 1).astype(int)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        list(ex.map(lambda ab: fn(int(ab[0]), int(ab[1])), zip(bounds[:-1], bounds[1:])))
    return time.perf_counter() - t0


# Launches of the secondary rows: timed after a warm-up long enough for the
# shader clock to settle, and HIP graphs after more, since a graph's first
# replays (about 25 here) run slower than its later ones.
ROW_STEPS, ROW_WARMUP, GRAPH_WARMUP = 20, 10, 30


def timed(fn, steps, warmup, torch):
    """Mean milliseconds per call of fn over `steps` calls after `warmup` calls."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return a.elapsed_time(b) / steps, wall


def per_launch(fn, steps, torch):
    """Milliseconds of each of `steps` calls of fn, each bracketed by its own pair of events."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=25)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--rows", default="fp64,separate,grad,ragged,demc,astro,kepler",
                    help="extra paths to time (comma list or 'none')")
    ap.add_argument("--cpu-sample", type=int, default=16384, help="systems in the CPU oracle sample")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (to scale HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the systems are independent and the path has no cross-GPU "
              f"step; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_0812_2976_amd as kp
    import synth

    dev = torch.device("cuda", 0)
    kp.load_library()
    rows = [] if args.rows == "none" else args.rows.split(",")
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)      # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 1 GiB device copies")
        del src, dst

    def gpu(x):
        return None if x is None else torch.from_numpy(np.ascontiguousarray(x)).to(dev)

    def gpu_truth_model(t, t0, truth):
        cols = [gpu(np.asarray(truth[k], dtype=np.float64)[:, None]) for k in ("P", "K", "e", "w", "M0")]
        return kp.rv_model(gpu(t), *cols, t0=t0, prec="fp64").cpu().numpy()[0]

    # ------------------------------------------------------------ headline
    log("generating workload c2 (1,048,576 x 4 x 256)")
    wl = synth.with_observations(synth.dense("c2"), gpu_truth_model)
    g = dict(t=gpu(wl.t), v=gpu(wl.v), sigma=gpu(wl.sigma), P=gpu(wl.P), K=gpu(wl.K), e=gpu(wl.e),
             omega=gpu(wl.w), M0=gpu(wl.M0), t0=wl.t0)
    out = torch.empty(wl.n_sys, dtype=torch.float64, device=dev)
    step = lambda: kp.rv_chisq(**g, prec="mixed", out=out)
    ms, wall = timed(step, args.steps, args.warmup, torch)
    triples = wl.n_sys * wl.n_pl * wl.n_obs
    value = wl.n_sys / (ms * 1e-3)
    log(f"mixed rv_chisq c2: {ms:.3f} ms/launch, {value:.4e} chi2/s")
    each = per_launch(step, args.steps, torch)
    # the same launch followed by the copy of the chi-square vector into pinned host memory
    host = torch.empty(wl.n_sys, dtype=torch.float64, pin_memory=True)

    def step_d2h():
        step()
        host.copy_(out, non_blocking=True)

    ms_d2h, _ = timed(step_d2h, args.steps, args.warmup, torch)
    launch_stats = {"mean_ms": ms, "median_ms": float(np.median(each)), "min_ms": float(np.min(each)),
                    "max_ms": float(np.max(each)), "with_d2h_ms": ms_d2h,
                    "with_d2h_chi2_per_s": wl.n_sys / (ms_d2h * 1e-3)}
    chi2 = out.cpu().numpy()
    if not np.all(np.isfinite(chi2)):
        raise RuntimeError("non-finite chi-square in the benchmark batch")

    f_table, early, f_halley = table_fraction(0.9), early_steps(0.9), halley_fraction(0.9)
    ops = mixed_ops_per_triple(wl.n_pl, f_table, early, f_halley) * triples
    classes = mixed_op_classes(wl.n_pl, f_table, early, f_halley)
    achieved = ops / (ms * 1e-3) / 1e12
    peak = mix_peak_ops_per_s(classes) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": "TOP/s",
                "frac": round(achieved / peak, 4), "traffic": recorded_traffic("rv_chisq_mixed_c2"),
                "kernel": "k_dense<PolMixed,4,0>", "ops_per_triple": round(ops / triples, 2),
                "ops_per_triple_by_class": {c: round(n, 3) for c, n in classes.items()},
                "peak_basis": "per SIMD and cycle: 32 binary32, 16 binary64, 8 transcendental lane operations; "
                              "1024 SIMDs at 2.4 GHz",
                "launch_ms": round(ms, 4)}

    result = {
        "metric": "Kepler solves/s and chi2 evals/s (n_pl=4,n_obs=256) vs FP64 GPU, % VALU peak",
        "value": value, "unit": "chi2 evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "c2 mixed-precision chi2: n_sys=1048576, n_pl=4, n_obs=256, e~U[0,0.9]",
                   "n_sys": wl.n_sys, "n_pl": wl.n_pl, "n_obs": wl.n_obs, "precision": "mixed"},
        "kepler_solves_per_s": triples / (ms * 1e-3),
        "valu_peak_frac": round(achieved / peak, 4),
        "launch_stats": launch_stats,
        "roofline": roofline,
    }
    del g, out

    # ------------------------------------------------------------ FP64 plain kernel
    if "fp64" in rows:
        log("plain FP64 kernel on c1 (65,536 x 4 x 256, 30 fixed iterations)")
        w1 = synth.with_observations(synth.dense("c1"), gpu_truth_model)
        g1 = dict(t=gpu(w1.t), v=gpu(w1.v), sigma=gpu(w1.sigma), P=gpu(w1.P), K=gpu(w1.K), e=gpu(w1.e),
                  omega=gpu(w1.w), M0=gpu(w1.M0), t0=w1.t0)
        o1 = torch.empty(w1.n_sys, dtype=torch.float64, device=dev)
        ms64, _ = timed(lambda: kp.rv_chisq(**g1, prec="fp64", out=o1), 3, 1, torch)
        ms64e, _ = timed(lambda: kp.rv_chisq(**g1, prec="fp64", out=o1, opts=dict(fixed_iter=-1)), 5, 1, torch)
        msm1, _ = timed(lambda: kp.rv_chisq(**g1, prec="mixed", out=o1), ROW_STEPS, ROW_WARMUP, torch)
        r64 = w1.n_sys / (ms64 * 1e-3)
        result["fp64_gpu"] = {"workload": "c1 n_sys=65536 n_pl=4 n_obs=256", "chi2_per_s": r64,
                              "kepler_solves_per_s": r64 * 1024, "launch_ms": ms64,
                              "early_exit_chi2_per_s": w1.n_sys / (ms64e * 1e-3),
                              "mixed_same_workload_chi2_per_s": w1.n_sys / (msm1 * 1e-3)}
        # the headline speed-up compares the two kernels on the same batch (c1); the
        # split beside it separates the iteration count (30 fixed binary64 steps
        # against the early-exit binary64 variant) from the precision
        r64e = w1.n_sys / (ms64e * 1e-3)
        rmix1 = w1.n_sys / (msm1 * 1e-3)
        result["speedup_vs_fp64_gpu"] = rmix1 / r64
        result["speedup_split"] = {
            "mixed_vs_fp64_fixed30_same_workload": rmix1 / r64,
            "mixed_vs_fp64_early_exit_same_workload": rmix1 / r64e,
            "fp64_early_exit_vs_fp64_fixed30": r64e / r64,
            "c2_mixed_vs_c1_fp64_fixed30_per_system": value / r64,
            "workload": "c1 (65,536 x 4 x 256) for every same-workload ratio"}
        del g1, o1

    # ------------------------------------------------------------ separate-function form
    if "separate" in rows:
        log("separate-function form on c2 (per-planet velocities to HBM, then chi-square; Kepler's equation only)")
        g2 = dict(t=gpu(wl.t), v=gpu(wl.v), sigma=gpu(wl.sigma), P=gpu(wl.P), K=gpu(wl.K), e=gpu(wl.e),
                  omega=gpu(wl.w), M0=gpu(wl.M0))
        dv = torch.empty((wl.n_pl, wl.n_sys, wl.n_obs), dtype=torch.float32, device=dev)
        o2 = torch.empty(wl.n_sys, dtype=torch.float64, device=dev)
        msa, _ = timed(lambda: kp.rv_planet_velocities(g2["t"], g2["P"], g2["K"], g2["e"], g2["omega"], g2["M0"],
                                                       out=dv), ROW_STEPS, ROW_WARMUP, torch)
        msb, _ = timed(lambda: kp.rv_chisq_from_velocities(g2["t"], g2["v"], g2["sigma"], dv, out=o2), ROW_STEPS, ROW_WARMUP, torch)
        dv_bytes = dv.numel() * 4
        # Kepler's equation only: every eccentric anomaly written (into the same buffer)
        mse, _ = timed(lambda: kp.rv_eccentric_anomalies(g2["t"], g2["P"], g2["K"], g2["e"], g2["omega"], g2["M0"],
                                                         out=dv), ROW_STEPS, ROW_WARMUP, torch)
        result["separate_c2"] = {"chi2_per_s": wl.n_sys / ((msa + msb) * 1e-3), "velocities_ms": msa,
                                 "chisq_ms": msb, "intermediate_GB": dv_bytes / 1e9,
                                 "chisq_hbm_GBps": (dv_bytes + wl.n_sys * 8) / (msb * 1e-3) / 1e9,
                                 "time_vs_fused": (msa + msb) / ms,
                                 "roofline_chisq": hbm_roofline(
                                     "k_chisq_from_dv<4>", dv_bytes + wl.n_sys * 8, msb,
                                     "binary32 velocities read (n_pl x n_sys x n_obs x 4 B) + chi-square out 8 B per "
                                     "system"),
                                 "kepler_only": {"launch_ms": mse, "solves_per_s": dv.numel() / (mse * 1e-3),
                                                 "roofline": hbm_roofline(
                                                     "k_dense<PolMixed,4,3>", dv_bytes + wl.n_sys * wl.n_pl * 40, mse,
                                                     "binary32 E written (n_pl x n_sys x n_obs x 4 B) + parameters "
                                                     "40 B per planet read"),
                                                 "written_GB": dv_bytes / 1e9,
                                                 "hbm_write_GBps": dv_bytes / (mse * 1e-3) / 1e9,
                                                 "time_vs_fused_chisq": mse / ms}}
        del g2, dv, o2

    # ------------------------------------------------------------ gradient
    if "grad" in rows:
        log("gradient on c4 (262,144 x 4 x 256)")
        w4 = synth.with_observations(synth.dense("c4", jitter=True), gpu_truth_model)
        g4 = dict(t=gpu(w4.t), v=gpu(w4.v), sigma=gpu(w4.sigma), P=gpu(w4.P), K=gpu(w4.K), e=gpu(w4.e),
                  omega=gpu(w4.w), M0=gpu(w4.M0), offset=gpu(w4.offset), t0=w4.t0)
        o4 = torch.empty(w4.n_sys, dtype=torch.float64, device=dev)
        gr = torch.empty((5 * w4.n_pl + 1, w4.n_sys), dtype=torch.float64, device=dev)
        msg, _ = timed(lambda: kp.rv_chisq_grad(**g4, prec="mixed", out=o4, grad=gr), ROW_STEPS, ROW_WARMUP, torch)
        gn = torch.empty((5 * w4.n_pl + 2, w4.n_sys), dtype=torch.float64, device=dev)
        jit = gpu(w4.jitter)
        msn, _ = timed(lambda: kp.rv_nll_grad(**g4, jitter=jit, prec="mixed", out=o4, grad=gn), ROW_STEPS, ROW_WARMUP, torch)
        npar = 5 * w4.n_pl + 1
        jr = torch.empty((npar, w4.n_sys), dtype=torch.float64, device=dev)
        jj = torch.empty((npar * (npar + 1) // 2, w4.n_sys), dtype=torch.float64, device=dev)
        msgn, _ = timed(lambda: kp.rv_chisq_gn(**g4, prec="mixed", out=o4, jtwr=jr, jtwj=jj), ROW_STEPS, ROW_WARMUP, torch)
        msgn64, _ = timed(lambda: kp.rv_chisq_gn(**g4, prec="fp64", out=o4, jtwr=jr, jtwj=jj), 3, 1, torch)
        # Gram matrix of sqrt(w)[J | 1 | r]: (np + 1)(np + 2)/2 multiply-adds per (system, observation);
        # 16x16x4 products per four observations: two for 17 to 24 columns, else one per pair of blocks
        useful = w4.n_sys * w4.t.size * (npar + 1) * (npar + 2)
        nb = (npar + 1 + 15) // 16
        nprod = 2 if 16 < npar + 1 <= 24 else nb * (nb + 1) // 2
        issued = w4.n_sys * (w4.t.size // 4) * nprod * 2048
        tri4 = w4.n_sys * w4.n_pl * w4.t.size
        nch4 = 1 if w4.t.size <= 64 else (2 if (w4.n_pl > 4 or w4.t.size <= 128) else 4)
        result["gradient_c4"] = {"chi2_grad_per_s": w4.n_sys / (msg * 1e-3), "launch_ms": msg,
                                 "triples_per_s": tri4 / (msg * 1e-3),
                                 "roofline": roofline_entry(f"k_grad_obs<{w4.n_pl},{nch4}>",
                                                            adjoint_op_classes(w4.n_pl, nch4, halley_fraction(0.8)),
                                                            tri4, msg,
                                                            recorded_traffic("rv_chisq_grad_mixed_c4", ADJOINT_FILES)),
                                 "nll_grad_launch_ms": msn,
                                 "gauss_newton": {"launch_ms_mixed": msgn, "launch_ms_fp64": msgn64,
                                                  "systems_per_s_mixed": w4.n_sys / (msgn * 1e-3),
                                                  "gram_useful_tflops": useful / (msgn * 1e-3) / 1e12,
                                                  "mfma_issued_tflops": issued / (msgn * 1e-3) / 1e12,
                                                  "mfma_dtype_mixed": "f32 (binary64 sums per 64 observations)",
                                                  "mfma_f32_peak_tflops": 157.3,
                                                  "mfma_frac_mixed": issued / (msgn * 1e-3) / 157.3e12}}
        if not args.no_cpu:
            import oracle
            # the oracle's sample has its own observed velocities (the oracle's model of
            # the truth system + the same noise): no oracle input comes from the GPU path
            cols = [np.asarray(w4.truth[k])[:, None] for k in ("P", "K", "e", "w", "M0")]
            v4 = oracle.rv_model(oracle.Dense(w4.t, np.zeros_like(w4.t), w4.sigma, *cols, t0=w4.t0))[0] + w4.noise
            n4 = min(args.cpu_sample // 4, w4.n_sys)
            d4 = oracle.Dense(w4.t, v4, w4.sigma, *(np.ascontiguousarray(getattr(w4, a)[:, :n4])
                                                    for a in ("P", "K", "e", "w", "M0")),
                              w4.offset[:n4], None, w4.t0)
            cores = cpu_threads()
            oracle.lib()
            res = {}
            log(f"CPU oracle gradient on {n4} systems of c4 with {cores} threads")
            dt = time_oracle(lambda i0, i1: res.__setitem__(i0, oracle.chisq_grad_scales(d4, i0, i1)), n4, cores)
            result["gradient_c4"]["cpu_baseline"] = {
                "value": n4 / dt, "unit": "chi2+gradient evals/s", "cores": cores, "kind": "oracle",
                "sample": f"first {n4} systems of the same c4 batch ({n4 * 1024} triples), {dt:.2f} s wall"}
            # accuracy of the mixed adjoint on the first 256 of them, the GPU given the
            # oracle's observed velocities: |dg| / max(|g|, S_r) per component
            m4 = min(256, n4)
            part = {k: gpu(np.ascontiguousarray(getattr(w4, a)[:, :m4])) for k, a in
                    (("P", "P"), ("K", "K"), ("e", "e"), ("omega", "w"), ("M0", "M0"))}
            _, gg = kp.rv_chisq_grad(gpu(w4.t), gpu(v4), gpu(w4.sigma), **part, offset=gpu(w4.offset[:m4]),
                                     t0=w4.t0, prec="mixed")
            _, g_ref, s_r, _ = oracle.chisq_grad_scales(d4, 0, m4)
            q13 = np.abs(gg.cpu().numpy() - g_ref[:, :m4]) / np.maximum(np.abs(g_ref[:, :m4]), s_r[:, :m4])
            result["gradient_c4"]["accuracy_vs_oracle"] = {
                "grad_q13_max": float(q13.max()), "grad_q13_median": float(np.median(q13)),
                "sample": f"first {m4} systems of c4, |dg| / max(|g|, S_r), S_r = sum_k |2 w r dv/dtheta|"}
        del g4, o4, gr, gn, jit, jr, jj

    # ------------------------------------------------------------ ragged
    if "ragged" in rows:
        log("ragged c3 (262,144 CSR systems)")
        rw = synth.ragged_with_observations(synth.ragged(), gpu_truth_model)
        plan = kp.RaggedPlan(gpu(rw.t), gpu(rw.v), gpu(rw.sigma), gpu(rw.obs_off), gpu(rw.P), gpu(rw.K),
                             gpu(rw.e), gpu(rw.w), gpu(rw.M0), gpu(rw.pl_off), t0=rw.t0)
        o3 = torch.empty(rw.n_sys, dtype=torch.float64, device=dev)
        msr, _ = timed(lambda: plan(o3), ROW_STEPS, GRAPH_WARMUP, torch)
        msr_direct, _ = timed(lambda: plan.direct(o3), ROW_STEPS, ROW_WARMUP, torch)
        info = plan.info()
        plan64 = kp.RaggedPlan(gpu(rw.t), gpu(rw.v), gpu(rw.sigma), gpu(rw.obs_off), gpu(rw.P), gpu(rw.K),
                               gpu(rw.e), gpu(rw.w), gpu(rw.M0), gpu(rw.pl_off), t0=rw.t0, prec="fp64")
        msr64, _ = timed(lambda: plan64(o3), 3, 1, torch)
        plan64.close()
        # the formulation's operations summed over the batch: every triple as in the
        # dense count, the per-observation work once per observation of each system
        npl_i = np.diff(rw.pl_off)
        nobs_i = np.diff(rw.obs_off)
        core = {c: n - (F64_OBS if c == "f64" else (OPS_OBS - F64_OBS if c == "f32" else 0)) / 4
                for c, n in mixed_op_classes(4, table_fraction(0.9), early_steps(0.9), halley_fraction(0.9)).items()}
        tri3 = int(np.sum(npl_i * nobs_i))
        obs3 = int(np.sum(nobs_i))
        cls3 = {c: core[c] + (F64_OBS if c == "f64" else (OPS_OBS - F64_OBS if c == "f32" else 0)) * obs3 / tri3
                for c in core}
        # the row's rate and the kernel's roofline come from the direct launches (events around
        # back-to-back launches of the kernel itself); a graph replay adds 10-30 us of launch
        # overhead per call on this ROCm, reported beside them
        result["ragged_c3"] = {"chi2_per_s": rw.n_sys / (msr_direct * 1e-3), "launch_ms": msr_direct,
                               "launch_call": "rv_chisq_ragged_direct",
                               "graph_launch_ms": msr, "graph_chi2_per_s": rw.n_sys / (msr * 1e-3),
                               "fp64_launch_ms": msr64, "speedup_vs_fp64": msr64 / msr_direct,
                               "kepler_solves_per_s": info["triples"] / (msr_direct * 1e-3),
                               "triples": info["triples"],
                               "roofline": roofline_entry(f"k_ragged_mixed<{info['group_chunks']}>", cls3, tri3,
                                                          msr_direct, recorded_traffic("rv_chisq_ragged_c3")),
                               "hbm_GBps_algorithmic": (obs3 * 24 + int(rw.pl_off[-1]) * 40 + rw.n_sys * 24)
                                                       / (msr_direct * 1e-3) / 1e9,
                               "plan": {k: info[k] for k in ("block_threads", "blocks", "sys_per_batch", "group_chunks", "tuned")}}
        plan.close()
        del o3
        if not args.no_cpu:
            import oracle
            n3 = min(args.cpu_sample, rw.n_sys)
            o_end = int(rw.obs_off[n3])
            p_end = int(rw.pl_off[n3])
            # the sample's observed velocities from the oracle's model of the truth system
            cols = [np.asarray(rw.truth[k])[:, None] for k in ("P", "K", "e", "w", "M0")]
            t3 = rw.t[:o_end]
            v3 = oracle.rv_model(oracle.Dense(t3, np.zeros_like(t3), np.ones_like(t3), *cols, t0=rw.t0))[0] \
                + rw.noise[:o_end]
            d3 = oracle.Ragged(t3, v3, rw.sigma[:o_end], rw.obs_off[:n3 + 1], rw.P[:p_end], rw.K[:p_end],
                               rw.e[:p_end], rw.w[:p_end], rw.M0[:p_end], rw.pl_off[:n3 + 1], None, None, rw.t0)
            out3 = np.full(n3, np.nan)
            cores = cpu_threads()
            oracle.lib()
            log(f"CPU oracle ragged on {n3} systems of c3 with {cores} threads")
            dt = time_oracle(lambda i0, i1: oracle.chisq_ragged(d3, i0, i1, out=out3), n3, cores)
            tri_s = int(np.sum(npl_i[:n3] * nobs_i[:n3]))
            result["ragged_c3"]["cpu_baseline"] = {
                "value": n3 / dt, "unit": "chi2 evals/s", "cores": cores, "kind": "oracle",
                "triples_per_s": tri_s / dt,
                "sample": f"first {n3} systems of the same c3 batch ({tri_s} Kepler solves), {dt:.2f} s wall"}

    # ------------------------------------------------------------ DE-MC sampler
    if "demc" in rows:
        log("DE-MC sampler on c1 observations (n_obs=256, n_pl=4)")
        w1 = synth.with_observations(synth.dense("c1", n_sys=2), gpu_truth_model)
        demc = {}
        for nh in (2048, 32768):
            x0, eps = synth.demc_population(w1.truth, nh)
            s = kp.DEMC(gpu(w1.t), gpu(w1.v), gpu(w1.sigma), gpu(x0), gpu(eps), seed=1, t0=w1.t0,
                        jump_every=10, prec="mixed")
            gen, ng = [0], 16

            def graph_step():
                s.run(gen[0], ng)
                gen[0] += ng

            def direct_step():
                s.generations(gen[0], ng)
                gen[0] += ng

            ms_g, _ = timed(graph_step, 10, GRAPH_WARMUP // 2, torch)
            ms_d, _ = timed(direct_step, 10, GRAPH_WARMUP // 2, torch)
            # the chi-square launch of one half alone, for the share of a generation it takes
            half = {k: gpu(np.ascontiguousarray(x0[0, a * 4:(a + 1) * 4])) for a, k in
                    enumerate(("P", "K", "e", "omega", "M0"))}
            obs = dict(t=gpu(w1.t), v=gpu(w1.v), sigma=gpu(w1.sigma), t0=w1.t0)
            oh = torch.empty(nh, dtype=torch.float64, device=dev)
            ms_c, _ = timed(lambda: kp.rv_chisq(**obs, **half, prec="mixed", out=oh), ROW_STEPS, ROW_WARMUP, torch)
            acc = s.n_accept.sum().item() / (2 * nh * gen[0])
            best = min(ms_g, ms_d)
            tri_gen = 2 * nh * w1.n_pl * w1.t.size
            demc[f"chains_{2 * nh}"] = {
                "generations_per_s_graph": ng / (ms_g * 1e-3), "generations_per_s_direct": ng / (ms_d * 1e-3),
                "proposals_per_s": 2 * nh * ng / (best * 1e-3), "generation_ms": best / ng,
                "two_rv_chisq_calls_ms": 2 * ms_c, "acceptance": acc,
                # the chi-square part only (the dense formulation per triple); the
                # proposal draws and the acceptance are not counted
                "roofline": roofline_entry(f"k_demc_half<PolMixed,{(w1.t.size + 63) // 64}>",
                                           mixed_op_classes(w1.n_pl, *op_fractions(
                                               x0[:, 2 * w1.n_pl:3 * w1.n_pl, :])), tri_gen, best / ng)}
            s.close()
            del s, half, obs, oh
        result["demc_c1"] = demc

    # ------------------------------------------------------------ astrometry
    if "astro" in rows:
        log("astrometric model (1,048,576 x 2 x 128 epochs)")

        def gpu_astro_truth(t, t0, truth):
            cols = [gpu(np.asarray(truth[k], dtype=np.float64).reshape(-1, 1)) for k in
                    ("P", "e", "M0", "A", "B", "F", "G")]
            return kp.astro_model(gpu(t), *cols, t0=t0, prec="fp64").cpu().numpy()[0]

        wa = synth.with_astro_observations(synth.astro(), gpu_astro_truth)
        ga = dict(t=gpu(wa.t), x=gpu(wa.x), y=gpu(wa.y), sigma_x=gpu(wa.sx), sigma_y=gpu(wa.sy), P=gpu(wa.P),
                  e=gpu(wa.e), M0=gpu(wa.M0), A=gpu(wa.A), B=gpu(wa.B), F=gpu(wa.F), G=gpu(wa.G), x0=gpu(wa.x0),
                  y0=gpu(wa.y0), t0=wa.t0)
        oa = torch.empty(wa.n_sys, dtype=torch.float64, device=dev)
        msa, _ = timed(lambda: kp.astro_chisq(**ga, prec="mixed", out=oa), ROW_STEPS, ROW_WARMUP, torch)
        ms64, _ = timed(lambda: kp.astro_chisq(**ga, prec="fp64", out=oa), 3, 1, torch)
        ms64e, _ = timed(lambda: kp.astro_chisq(**ga, prec="fp64", out=oa, opts={"fixed_iter": -1}), 3, 1, torch)
        tri = wa.n_sys * wa.n_pl * wa.t.size
        result["astro"] = {"workload": "1,048,576 systems x 2 planets x 128 two-axis epochs, a ~ logU[1, 100] mas",
                           "chi2_per_s_mixed": wa.n_sys / (msa * 1e-3), "launch_ms_mixed": msa,
                           "kepler_solves_per_s_mixed": tri / (msa * 1e-3),
                           "launch_ms_fp64": ms64, "launch_ms_fp64_early_exit": ms64e,
                           "speedup_vs_fp64": ms64 / msa, "speedup_vs_fp64_early_exit": ms64e / msa}
        del ga, oa

    # ------------------------------------------------------------ Kepler only
    if "kepler" in rows:
        log("standalone Kepler solve (2^26 pairs)")
        M, e = synth.kepler_pairs(1 << 26)
        Mg, eg = gpu(M), gpu(e)
        Eg = torch.empty_like(Mg)
        msk, _ = timed(lambda: kp.kepler_solve(Mg, eg, prec="mixed", out=Eg), ROW_STEPS, ROW_WARMUP, torch)
        msk64, _ = timed(lambda: kp.kepler_solve(Mg, eg, prec="fp64", out=Eg), 3, 1, torch)
        n = M.size
        result["kepler_solve"] = {"n": n, "mixed_solves_per_s": n / (msk * 1e-3), "mixed_launch_ms": msk,
                                  "mixed_hbm_GBps": 24 * n / (msk * 1e-3) / 1e9,
                                  "roofline": hbm_roofline("k_kepler<true,4>", 24 * n, msk,
                                                           "M and e read, E written: 8 B each per pair"),
                                  "fp64_solves_per_s": n / (msk64 * 1e-3), "fp64_launch_ms": msk64}
        del Mg, eg, Eg

    # ------------------------------------------------------------ CPU oracle
    if not args.no_cpu:
        import oracle
        from concurrent.futures import ThreadPoolExecutor

        n = min(args.cpu_sample, wl.n_sys)
        # the oracle's sample has its own observed velocities (oracle model of the
        # truth system + the same noise): no oracle input comes from the GPU path
        cols = [np.asarray(wl.truth[k])[:, None] for k in ("P", "K", "e", "w", "M0")]
        v_cpu = oracle.rv_model(oracle.Dense(wl.t, np.zeros_like(wl.t), wl.sigma, *cols, t0=wl.t0))[0] + wl.noise
        try:
            cores = len(os.sched_getaffinity(0))
        except AttributeError:
            cores = os.cpu_count() or 1
        cores = max(1, min(cores, 16))
        d = oracle.Dense(wl.t, v_cpu, wl.sigma, wl.P[:, :n], wl.K[:, :n], wl.e[:, :n], wl.w[:, :n], wl.M0[:, :n],
                         None, None, wl.t0)
        oracle.lib()
        bounds = np.linspace(0, n, cores * 4 + 1).astype(int)
        out_c = np.full(n, np.nan)
        log(f"CPU oracle on {n} systems with {cores} threads")
        t0 = time.perf_counter()
        with ThreadPoolExecutor(cores) as ex:
            list(ex.map(lambda ab: oracle.chisq(d, int(ab[0]), int(ab[1]), out=out_c), zip(bounds[:-1], bounds[1:])))
        dt = time.perf_counter() - t0
        # one thread, as the paper's CPU baseline ran, on a sixteenth of the sample
        n1 = max(1, n // 16)
        out_1 = np.full(n1, np.nan)
        t1 = time.perf_counter()
        oracle.chisq(d, 0, n1, out=out_1)
        dt1 = time.perf_counter() - t1
        if not np.array_equal(out_1, out_c[:n1], equal_nan=True):
            raise RuntimeError("single-thread oracle run disagrees with the threaded run")
        result["cpu_baseline"] = {"value": n / dt, "unit": "chi2 evals/s", "cores": cores, "kind": "oracle",
                                  "sample": f"first {n} systems of the same c2 batch ({n * 1024} Kepler solves), "
                                            f"{dt:.2f} s wall",
                                  "single_thread": {"value": n1 / dt1, "sample": f"first {n1} systems, "
                                                                                  f"{dt1:.2f} s"},
                                  "host_cpu": host_cpu_model(), "host_cpus_online": os.cpu_count()}

        # Accuracy of the timed mixed-precision kernels against the oracle, outside
        # the timed region: chi2 of the same sample (the GPU given the oracle's
        # observed velocities), model velocities of its first 256 systems, and
        # standalone Kepler solves (uniform and periapsis-stress pairs).
        part = {k: gpu(np.ascontiguousarray(getattr(wl, a)[:, :n])) for k, a in
                (("P", "P"), ("K", "K"), ("e", "e"), ("omega", "w"), ("M0", "M0"))}
        chi_g = kp.rv_chisq(gpu(wl.t), gpu(v_cpu), gpu(wl.sigma), **part, t0=wl.t0, prec="mixed").cpu().numpy()
        m = min(256, n)
        vm_g = kp.rv_model(gpu(wl.t), *(p[:, :m].contiguous() for p in part.values()), t0=wl.t0,
                           prec="mixed").cpu().numpy()
        vm_o = oracle.rv_model(oracle.Dense(wl.t, v_cpu, wl.sigma, *(np.ascontiguousarray(getattr(wl, a)[:, :m])
                                                                    for a in ("P", "K", "e", "w", "M0")),
                                            None, None, wl.t0))
        acc = {"chi2_rel_max": float(np.max(np.abs(chi_g - out_c) / np.maximum(out_c, 1.0))),
               "v_abs_max_mps": float(np.max(np.abs(vm_g - vm_o))),
               "sample": f"chi2: first {n} systems of c2; velocities: first {m} systems x 256 epochs; "
                         f"Kepler: 2^18 pairs each"}
        for tag, stress in (("E_abs_max_rad", False), ("E_abs_max_rad_stress", True)):
            Ms, es = synth.kepler_pairs(1 << 18, stress=stress)
            E_g = kp.kepler_solve(gpu(Ms), gpu(es), prec="mixed").cpu().numpy()
            acc[tag] = float(np.max(np.abs(E_g - oracle.kepler(Ms, es))))
        result["accuracy_vs_oracle"] = acc
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
