"""Host logic of bench.py (CPU only): the algorithmic traffic model per kernel
and per step, the lookup of committed counter summaries, and the one-GPU
contract of the command line."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_model_below_1024():
    """Below 1024 the x pass writes five fields (U, V, W, F(kx v), F(kx w))
    and the inverse y pass forms the vorticity: 8C, 11C, 17C and 172C per
    fused step."""
    f = bench.fields_per_launch(512)
    assert bench.curl_in_y(512) and bench.curl_in_y(32)
    assert f["xinv_curl"] == 3 + 5
    assert f["yinv6"] == 5 + 6
    assert f["zcross"] == 6 + 3
    assert f["yfwd3"] == 3 + 3
    assert f["xstage"] == f["xrhs_rk4"] + 5
    assert bench.fields_per_step(512) == 4 * (11 + 9 + 6 + 17) == 172


def test_traffic_model_at_1024():
    f = bench.fields_per_launch(1024)
    assert not bench.curl_in_y(1024)
    assert (f["xinv_curl"], f["yinv6"], f["xstage"]) == (9, 12, 18)
    assert bench.fields_per_step(1024) == 180


def test_traffic_model_follows_the_plan():
    """A plan with the vorticity formed in the x pass moves the six-field
    figures at any N, and the five-field ones at 1024 when the y pass forms
    it."""
    assert bench.fields_per_step(512, cy=0) == 180
    assert bench.fields_per_step(1024, cy=1) == 172
    assert bench.fields_per_launch(128, cy=0)["yinv6"] == 12


def test_cpu_baseline_times_full_oracle_steps():
    """The CPU baseline times whole oracle RK4 steps and scales the larger
    size by the measured growth per doubling of N."""
    r = bench.cpu_baseline(32, sizes=((8, 1), (16, 1)))
    assert r["kind"] == "oracle_step" and r["unit"] == "ms/step"
    t8, t16 = r["measured_s_per_step"]["8"], r["measured_s_per_step"]["16"]
    assert abs(r["growth_per_doubling"] - t16 / t8) < 1e-12
    assert abs(r["value"] - t16 * (t16 / t8) * 1e3) < 1e-9 * r["value"]
    assert r["cores"] >= 1 and r["nproc"] >= 1


def test_rk4_state_traffic():
    """Regrouped RK4: the stages move 6, 12, 9 and 9 fields of state and read
    the 3 fields of N_hat each, 48C per step, 12C per stage on average."""
    assert 4 * bench.fields_per_launch(512)["xrhs_rk4"] == (6 + 12 + 9 + 9) + 4 * 3


def test_field_bytes():
    assert bench.field_bytes(512, "f64") == 512 * 512 * 257 * 16 == 1077936128
    assert bench.field_bytes(1024, "f32") == 1024 * 1024 * 513 * 8


def _summary(tmp_path, N, sha, kernels):
    d = tmp_path / "profiles"
    d.mkdir(exist_ok=True)
    rec = {"source_sha256": sha, "N": N,
           "kernels": {k: {"traffic_bytes_calibrated": v} for k, v in kernels.items()}}
    (d / f"traffic_tg{N}.json").write_text(json.dumps(rec))


def test_measured_traffic_lookup(tmp_path, monkeypatch):
    """Counter summaries are matched by kernel name and precision, averaged
    over the RK stages, and ignored when the kernel sources changed."""
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    sha = bench.kernel_source_hash()
    _summary(tmp_path, 512, sha, {
        "k_yinv_curl<double, 512, 8>": 11e9,
        "k_yline<double, 512, 8, -1, 3, 8>": 6e9,
        "k_zcross<double, 512, 4>": 9e9,
        "k_xstage<double, 512, 8, 0>": 15e9,
        "k_xstage<double, 512, 8, 1>": 21e9,
        "k_xstage<float, 512, 16, 0>": 7e9,
    })
    assert bench.measured_traffic(512, "f64", "yinv6") == 11e9
    assert bench.measured_traffic(512, "f64", "yfwd3") == 6e9
    assert bench.measured_traffic(512, "f64", "zcross") == 9e9
    assert bench.measured_traffic(512, "f64", "xstage") == (15e9 + 21e9) / 2
    assert bench.measured_traffic(512, "f32", "xstage") == 7e9
    assert bench.measured_traffic(512, "f32", "yinv6") is None
    # at 1024 the inverse y pass is the six-field k_yline<..., 1, 6>
    _summary(tmp_path, 1024, sha, {
        "k_yline<double, 1024, 8, 1, 6, 16>": 12e9,
        "k_yline<double, 1024, 8, -1, 3, 16>": 6e9,
    })
    assert bench.measured_traffic(1024, "f64", "yinv6") == 12e9
    assert bench.measured_traffic(1024, "f64", "yfwd3") == 6e9
    # a summary taken from other kernel sources is not used
    _summary(tmp_path, 512, "0" * 64, {"k_xstage<double, 512, 8, 0>": 15e9})
    assert bench.measured_traffic(512, "f64", "xstage") is None
    assert bench.measured_traffic(256, "f64", "xstage") is None


def test_source_hash_ignores_comments(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_1602_03638_amd" / "csrc"
    csrc.mkdir(parents=True)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (csrc / "k.hpp").write_text("int a = 1;\n")
    h = bench.kernel_source_hash()
    (csrc / "k.hpp").write_text("// a comment\nint a = 1;  // trailing\n\n")
    assert bench.kernel_source_hash() == h
    (csrc / "k.hpp").write_text("int a = 2;\n")
    assert bench.kernel_source_hash() != h


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_kernel_names_and_algorithmic_bytes():
    """Trace names reduce to the kernel instance; the algorithmic bytes of a
    stage kernel follow from its template arguments (fields C = N^2 (N/2+1)
    complex values)."""
    C = bench.field_bytes(512, "f64")
    name = bench.kernel_short_name("void dns::k_xstage<double, 512, 8, 1, true, false, false>(HIP_vector_type<double, 2u>*)")
    assert name == "k_xstage<double, 512, 8, 1, true, false, false>"
    assert bench.algorithmic_bytes(name) == (3 + 12 + 5) * C
    assert bench.algorithmic_bytes("k_xstage<double, 512, 8, 3, false, true, true>") == (3 + 9 + 6) * C
    assert bench.algorithmic_bytes("k_xrhs<double, 512, 8, 0, false, false>") == 9 * C
    assert bench.algorithmic_bytes("k_yinv_curl<double, 512, 8, false>") == 11 * C
    assert bench.algorithmic_bytes("k_yline<double, 512, 8, -1, 3, 8, false>") == 6 * C
    assert bench.algorithmic_bytes("k_zcross<double, 512, 4>") == 9 * C
    assert bench.algorithmic_bytes("k_xinv_curl<float, 1024, 8, false, true>") == 9 * bench.field_bytes(1024, "f32")
    assert bench.algorithmic_bytes("k_layout<double, 512, true>") is None


def _counter_csv(path, rows):
    hdr = ('"Correlation_Id","Dispatch_Id","Agent_Id","Queue_Id","Process_Id","Thread_Id","Grid_Size",'
           '"Kernel_Id","Kernel_Name","Workgroup_Size","LDS_Block_Size","Scratch_Size","VGPR_Count",'
           '"Accum_VGPR_Count","SGPR_Count","Counter_Name","Counter_Value","Start_Timestamp","End_Timestamp"')
    path.parent.mkdir(parents=True, exist_ok=True)
    lines = [hdr] + [f'{i},{i},"Agent 1",1,1,1,1,1,"{k}",256,0,0,8,0,32,"{c}",{v},0,1'
                     for i, (k, c, v) in enumerate(rows, 1)]
    path.write_text("\n".join(lines) + "\n")


def test_counter_summary_calibrates_and_keys_by_source(tmp_path):
    """Counter summaries scale FETCH_SIZE and WRITE_SIZE by the factors a copy
    of known size gives, average over dispatches, and carry the current
    kernel-source hash (never keyed by hand)."""
    k = "void dns::k_zcross<double, 512, 4>(HIP_vector_type<double, 2u>*, double, unsigned long)"
    _counter_csv(tmp_path / "f" / "h" / "run_counter_collection.csv",
                 [(k, "FETCH_SIZE", 3000000.0), (k, "FETCH_SIZE", 3000002.0)])
    _counter_csv(tmp_path / "w" / "h" / "run_counter_collection.csv", [(k, "WRITE_SIZE", 3100000.0)])
    _counter_csv(tmp_path / "cf" / "h" / "run_counter_collection.csv",
                 [("dns::k_copy_rows(x)", "FETCH_SIZE", 524288.0)])
    _counter_csv(tmp_path / "cw" / "h" / "run_counter_collection.csv",
                 [("dns::k_copy_rows(x)", "WRITE_SIZE", 1048576.0)])
    out_json, out_md = tmp_path / "t.json", tmp_path / "t.md"
    bench.summarize_counters(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"), str(tmp_path / "cw"),
                             1 << 30, 512, str(out_json), str(out_md), ["cmd a", "cmd b"], "title")
    rec = json.loads(out_json.read_text())
    assert rec["source_sha256"] == bench.kernel_source_hash()
    v = rec["kernels"]["k_zcross<double, 512, 4>"]
    assert abs(v["fetch_factor"] - 2.0) < 1e-12 and abs(v["write_factor"] - 1.0) < 1e-12
    assert abs(v["traffic_bytes_calibrated"] - (3000001.0 * 2 + 3100000.0) * 1024) < 1e-3
    assert v["dispatches"] == 2 and v["alg_bytes"] == 9 * bench.field_bytes(512, "f64")
    assert "cmd a" in out_md.read_text()


def test_trace_summary_table(tmp_path):
    d = tmp_path / "s" / "h"
    d.mkdir(parents=True)
    (d / "run_kernel_stats.csv").write_text(
        '"Name","Calls","TotalDurationNs","AverageNs","Percentage","MinNs","MaxNs","StdDev"\n'
        '"void dns::k_zcross<double, 512, 4>(double*)",4,7200000,1800000.0,50.0,1790000,1810000,0.0\n')
    out = tmp_path / "trace.md"
    bench.summarize_trace(str(tmp_path / "s"), str(out), "rocprofv3 ...", "title")
    text = out.read_text()
    assert "`k_zcross<double, 512, 4>` | 4 | 1800.0" in text
    assert f"{9 * bench.field_bytes(512, 'f64') / 1.8e-3 / 1e9:.0f}" in text


def test_long_run_summary(tmp_path):
    """The Taylor-Green long-run table: times, peaks, budget residuals, the
    relative differences of the FP32 and coarse runs, and the commands that
    reproduce the runs."""
    def run(N, dtype, scale, peak_at):
        steps, dt = 20000, 1e-3
        E = [0.125 * scale * (1.0 - 0.8 * n / steps) for n in range(steps + 1)]
        W = [0.375 + 10.0 * (1.0 - abs(n - peak_at) / steps) for n in range(steps + 1)]
        rec = {"N": N, "dtype": dtype, "nu": 1 / 1600, "dt": dt, "steps": steps, "ms_per_step": 1.5,
               "energy": E, "enstrophy": W, "max_rel_budget_residual": 2e-7}
        path = tmp_path / f"run_{N}_{dtype}.json"
        path.write_text(json.dumps(rec))
        return str(path)
    ref, f32, coarse = run(512, "f64", 1.0, 8976), run(512, "f32", 1.0 + 1e-5, 8976), run(256, "f64", 1.01, 8884)
    out = tmp_path / "long.md"
    assert bench.summarize_tg_long(str(out), ref, f32, coarse) == 0
    text = out.read_text()
    assert f"python -u bench.py --tg-long 512 f32 20000 --tg-long-out {f32}" in text
    assert f"python bench.py --summarize-tg-long {out} {ref} {f32} {coarse}" in text
    assert "| 512^3 FP64 | 1.500 | 0.025000000 | 10.37500 | 8.976 | 2.00e-07 |" in text
    assert "| 256^3 FP64 | 1.500 |" in text and "| 8.884 |" in text
    # t = 0 row: E, Omega, 2 nu Omega and the relative differences (1e-5 and 1e-2)
    row0 = [ln for ln in text.splitlines() if ln.startswith("| 0 |")][0]
    assert row0.startswith("| 0 | 0.125000 |") and "1.0e-05" in row0 and "1.0e-02" in row0
