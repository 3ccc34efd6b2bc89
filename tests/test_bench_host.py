"""Host-side behaviour of bench.py (no GPU): the one-GPU contract and the
bookkeeping that turns committed rocprofv3 summaries into the JSON fields."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _run_bench(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, capture_output=True, text=True,
                          env=env, timeout=120)


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = _run_bench(["--gpus", str(n)])
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_world_size_above_one_is_refused():
    r = _run_bench([], {"WORLD_SIZE": "2"})
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _fake_profile(tmp_path, monkeypatch, kernel_hash):
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"kernel_hash": kernel_hash, "hbm_bytes_per_launch": 3_000_000_000,
           "hbm_read_bytes": 1_800_000_000, "hbm_write_bytes": 1_200_000_000}
    (prof / "k_march_c5_f64_pmc.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))


def test_stream_model_arithmetic(tmp_path, monkeypatch):
    h = bench.kernel_hash()  # hash of the real kernel sources (read before ROOT moves)
    _fake_profile(tmp_path, monkeypatch, h)
    monkeypatch.setattr(bench, "kernel_hash", lambda: h)
    probe = {"read": {"GBps": 6000.0}, "write": {"GBps": 4000.0}}
    m = bench.stream_model("k_march", "c5", "f64", probe, launch_ms=0.75)
    # 1.8 GB at 6 TB/s + 1.2 GB at 4 TB/s = 0.3 ms + 0.3 ms
    assert m["model_ms"] == pytest.approx(0.6)
    assert m["frac_of_model"] == pytest.approx(0.8)
    assert m["read_bytes"] == 1_800_000_000 and m["write_bytes"] == 1_200_000_000
    assert bench.traffic_from_profile("k_march", "c5", "f64") == 3_000_000_000


def test_stale_profile_is_ignored(tmp_path, monkeypatch):
    _fake_profile(tmp_path, monkeypatch, "0000000000000000")
    monkeypatch.setattr(bench, "kernel_hash", lambda: "ffffffffffffffff")
    probe = {"read": {"GBps": 6000.0}, "write": {"GBps": 4000.0}}
    assert bench.stream_model("k_march", "c5", "f64", probe, launch_ms=0.75) is None
    assert bench.traffic_from_profile("k_march", "c5", "f64") is None


def test_stream_model_needs_both_probes(tmp_path, monkeypatch):
    h = "abcdabcdabcdabcd"
    _fake_profile(tmp_path, monkeypatch, h)
    monkeypatch.setattr(bench, "kernel_hash", lambda: h)
    assert bench.stream_model("k_march", "c5", "f64", {"read": {"GBps": 6000.0}}, 0.75) is None
    assert bench.stream_model("k_march", "c5", "f64", None, 0.75) is None


def test_kernel_hash_covers_the_kernel_sources():
    """The hash that gates the profile-derived fields changes with any of the
    kernel headers (here: with their concatenated bytes)."""
    import hashlib
    h = hashlib.sha256()
    for s in bench.KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1712_06079_amd", "csrc", s), "rb") as fh:
            h.update(fh.read())
    assert bench.kernel_hash() == h.hexdigest()[:16]
    assert "lbm_march.hpp" in bench.KERNEL_SOURCES and "lbm_device.hpp" in bench.KERNEL_SOURCES


def test_oracle_config_timings_shape():
    """The oracle timings of the other configurations (tiny samples here):
    every entry present, positive rates, the thread count the oracle used."""
    out = bench.oracle_configs(c1_steps=4, c2_steps=1, c4_steps=2, every=1)
    assert out["kind"] == "oracle" and out["cores"] >= 1
    assert out["c1"]["steps"] == 4 and out["c1"]["mlups"] > 0
    assert out["c2"]["steps"] == 1 and out["c2"]["mlups"] > 0
    c4 = out["c4"]
    assert c4["steps"] == 2 and c4["checkpoint_every"] == 1
    assert c4["ms_forward_step"] > 0 and c4["ms_gradient_per_step"] > c4["ms_forward_step"]


def test_precision_diff_arithmetic():
    """The FP32-against-FP64 summary: largest relative density difference,
    relative mass difference, scalar differences (relative only when the FP64
    value is non-zero)."""
    import numpy as np
    rhos = {"f64": np.array([[1.0, 2.0], [4.0, 8.0]]), "f32": np.array([[1.0, 2.002], [4.0, 7.9]])}
    out = bench._precision_diff(rhos, {"mass": 15.0, "dp": 2.0, "z": 0.0}, {"mass": 14.902, "dp": 2.5, "z": 1e-9},
                                ("dp", "z"))
    assert out["rho_max_rel_diff"] == pytest.approx(0.1 / 8.0)
    assert out["mass_rel_diff"] == pytest.approx(0.098 / 15.0)
    assert out["dp_abs_diff"] == pytest.approx(0.5) and out["dp_rel_diff"] == pytest.approx(0.25)
    assert out["z_abs_diff"] == pytest.approx(1e-9) and out["z_rel_diff"] is None
