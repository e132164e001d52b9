"""Host-side logic of the benchmark (no GPU): the one-GPU contract, the algorithmic
operation count used for the roofline, and the guard that only reports recorded
HBM traffic for the kernel sources it was measured on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_operation_count_of_the_mixed_formulation():
    """phase 4 + table start 9 for the planets inside the table's range (e <= 0.9),
    else the paper's start 2 and two early steps of 20; last step with its rotation:
    Halley's 25 + 8 in the table's Halley bands (e < 0.85), Danby's quartic 33 + 11
    elsewhere; velocity 5 + binary64 planet sum 2 + 6 per observation shared by 4
    planets."""
    bands = bench.start_table_bands()
    assert bands[0][0] == 0.0 and bands[-1][1] == 0.9 and [h for _, _, h in bands] == [True, True, False]
    f, early, h = bench.table_fraction(0.9), bench.early_steps(0.9), bench.halley_fraction(0.9)
    assert f == 1.0 and early == 0.0 and abs(h - 0.85 / 0.9) < 1e-12
    want = 4 + 9 + h * (25 + 8) + (1 - h) * (33 + 11) + 5 + 2 + 6 / 4
    assert abs(bench.mixed_ops_per_triple(4, f, early, h) - want) < 1e-12
    # beyond the table (e up to 0.975) the count is the schedule's
    assert abs(bench.table_fraction(0.975) - 0.9 / 0.975) < 1e-12
    assert abs(bench.early_steps(0.975) - 2 * 0.075 / 0.975) < 1e-12
    assert abs(bench.mixed_ops_per_triple(4, 0.0, 2.0) - (4 + 2 + 40 + 33 + 11 + 5 + 2 + 6 / 4)) < 1e-12


def test_mix_peak_of_the_formulation():
    """The classes add up to the operation count; a pure binary32 mix peaks at the
    FP32 vector rate (157.3 TFLOP/s / 2 flops per operation), a pure binary64 one at
    half of it, and the formulation's mix (binary32, 4 + 2 + 5/4 binary64 and 3 per
    early step + 2 transcendental operations per triple) at its operations over
    n32/32 + n64/16 + ntr/8 SIMD cycles."""
    f, early, h = bench.table_fraction(0.9), bench.early_steps(0.9), bench.halley_fraction(0.9)
    c = bench.mixed_op_classes(4, f, early, h)
    assert abs(sum(c.values()) - bench.mixed_ops_per_triple(4, f, early, h)) < 1e-12
    assert abs(c["f64"] - 7.25) < 1e-12 and abs(c["trans"] - (3 * early + 2)) < 1e-12
    assert abs(bench.mix_peak_ops_per_s({"f32": 1.0}) - 157.3e12 / 2) < 0.1e12
    assert abs(bench.mix_peak_ops_per_s({"f64": 1.0}) - 78.6e12 / 2) < 0.1e12
    cycles = c["f32"] / 32 + c["f64"] / 16 + c["trans"] / 8
    assert abs(bench.mix_peak_ops_per_s(c) - sum(c.values()) / cycles * 1024 * 2.4e9) < 1.0


def test_recorded_traffic_requires_a_matching_source_hash(tmp_path, monkeypatch):
    assert bench.recorded_traffic("no_such_profile") is None
    h = bench.kernel_source_hash()
    assert len(h) == 16
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "x_traffic.md").write_text(f"kernel_source_sha256: {h}\nhbm_bytes_per_launch: 1.5e+08\n")
    (prof / "y_traffic.md").write_text("kernel_source_sha256: 0000000000000000\nhbm_bytes_per_launch: 1.5e+08\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda files=bench.DENSE_FILES: h)
    assert bench.recorded_traffic("x") == 1.5e8
    assert bench.recorded_traffic("y") is None


def test_adjoint_op_count_and_roofline_entry():
    """The adjoint's count by class adds up, the cross-wavefront reduction shrinks with
    more observation chunks, and a roofline entry reports achieved / peak."""
    c4 = bench.adjoint_op_classes(4, 4)
    c1 = bench.adjoint_op_classes(4, 1)
    assert c1["f32"] > c4["f32"] and c1["f64"] == c4["f64"]
    assert abs(c4["f64"] - (bench.ADJ_F64 + 3 / 4)) < 1e-12
    # the Halley rows take 8 fewer binary32 operations in the last step
    assert abs(bench.adjoint_op_classes(4, 4, 1.0)["f32"] - (c4["f32"] - 8)) < 1e-12
    e = bench.roofline_entry("k", c4, 1000, 1.0)
    assert abs(e["achieved"] - sum(c4.values()) * 1000 / 1e-3 / 1e12) < 1e-3
    assert abs(e["frac"] - e["achieved"] / e["peak"]) < 1e-3 and e["bound"] == "alu"


def test_source_hash_ignores_comments_and_layout_only():
    code = 'int f(int x) {\n    return x + 1;   // one more\n}\n/* block */ const char *s = "a // b";\n'
    same = 'int f(int x)\n{ return x + 1;   // ONE MORE, reworded\n}\n/* other\n block */ const char *s = "a // b";\n'
    other = 'int f(int x) {\n    return x + 2;   // one more\n}\n/* block */ const char *s = "a // b";\n'
    lit = 'int f(int x) {\n    return x + 1;   // one more\n}\n/* block */ const char *s = "a // c";\n'
    assert bench.code_tokens(code) == bench.code_tokens(same)
    assert bench.code_tokens(code) != bench.code_tokens(other)
    assert bench.code_tokens(code) != bench.code_tokens(lit)


def test_op_fractions_match_the_uniform_closed_forms():
    import numpy as np
    for e_max in (0.8, 0.9, 0.975):
        e = np.random.default_rng(7).uniform(0.0, e_max, 400_000)
        f_tab, early, f_hal = bench.op_fractions(e)
        assert abs(f_tab - bench.table_fraction(e_max)) < 5e-3
        assert abs(early - bench.early_steps(e_max)) < 1e-2
        assert abs(f_hal - bench.halley_fraction(e_max)) < 5e-3


def test_hbm_roofline_entry():
    r = bench.hbm_roofline("k", 4.0e9, 1.0, "basis")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert abs(r["achieved"] - 4000.0) < 1e-6 and abs(r["frac"] - 0.5) < 1e-9
