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
