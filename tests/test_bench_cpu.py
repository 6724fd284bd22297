"""bench.py's host-side contract: the one-GPU rule, the byte accounting
behind the roofline, the timing spread and the traffic lookup."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "single" in r.stderr and "GPU" in r.stderr


def test_algorithmic_bytes_are_five_reads_and_one_write():
    """psi, h and the new psi are nx*ny*nz words; u1, u2, u3 carry one more
    face along their own axis: 48.2 B per FP64 cell on the benchmark grid."""
    nz, ny, nx = 64, 256, 512
    want = 8 * (3 * nx * ny * nz + (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1))
    assert bench.algorithmic_bytes((nz, ny, nx), 8) == want == 404094976
    assert bench.algorithmic_bytes((nz, ny, nx), 4) * 2 == want
    assert abs(want / (nx * ny * nz) - 48.2) < 0.05


def test_time_levels_add_three_face_arrays_and_keep_periodic_faces():
    import numpy as np
    shape = (16, 8, 4)
    nz, ny, nx = shape
    faces = (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)
    assert (bench.algorithmic_bytes(shape, 8, tvel=True) - bench.algorithmic_bytes(shape, 8)
            == 8 * faces)
    assert bench.tv_scale(0) == 1.0 and bench.tv_scale(bench.TV_LEVELS) == 1.0
    assert len({bench.tv_scale(k) for k in range(bench.TV_LEVELS)}) > 2
    u = np.random.default_rng(0).uniform(-0.4, 0.4, (3, 4, 9))
    u[..., -1] = u[..., 0]
    for k in range(bench.TV_LEVELS):
        v = u * bench.tv_scale(k)
        assert np.array_equal(v[..., -1], v[..., 0])


def test_chain_bytes_by_design():
    """iord 3 = head (5 in, psi out, 3 velocity faces, psi1) + last
    (iterate, h, psi1, psi^n and 3 velocity faces in, psi out)."""
    nz, ny, nx = 4, 5, 6
    n = nx * ny * nz
    faces = (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)
    head = (3 * n + faces) + faces + n
    last = 4 * n + faces + n
    assert bench.chain_bytes((nz, ny, nx), 8, 3) == 8 * (head + last)
    mid = 4 * n + faces + 3 * n + faces
    assert bench.chain_bytes((nz, ny, nx), 8, 5) == 8 * (head + 2 * mid + last)
    assert bench.chain_bytes((nz, ny, nx), 8, 3, nonos=False) < bench.chain_bytes((nz, ny, nx), 8, 3)


def test_timing_spread():
    assert bench.spread([0.2]) is None
    s = bench.spread([0.25, 0.25, 0.25])
    assert s["median_ms"] == 0.25 and s["ci95_half_ms"] == 0.0
    s = bench.spread([1.0, 2.0, 3.0, 4.0])
    assert s["median_ms"] == 2.5 and s["mean_ms"] == 2.5 and s["chunks_of_8_steps"] == 4
    # t(0.975, 3) = 3.1824..., sample std of 1..4 = 1.2910..., sqrt(4) = 2
    assert abs(s["ci95_half_ms"] - 3.182446 * 1.290994 / 2) < 1e-5


def test_traffic_needs_the_current_kernel_source(tmp_path, monkeypatch):
    import hashlib
    from paper_1507_01265_amd import build
    csrc = os.path.join(ROOT, "paper_1507_01265_amd", "csrc")
    flags = " ".join([*build.FLAGS, *dict(build.SOURCES)["mpdata_step.hip"]])
    assert "-amdgpu-use-amdgpu-trackers=1" in flags
    sha = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read()
                                  for f in ("mpdata_march.h", "mpdata_step.hip"))
                         + flags.encode()).hexdigest()
    good = tmp_path / "good.md"
    good.write_text(f"kernel_source_sha256: {sha}\ntraffic_bytes_per_launch: 12345\n")
    stale = tmp_path / "stale.md"
    stale.write_text("kernel_source_sha256: 0000\ntraffic_bytes_per_launch: 12345\n")
    monkeypatch.setattr(bench, "PROFILES", {"good": str(good), "stale": str(stale)})
    assert bench.measured_traffic("good") == 12345.0
    assert bench.measured_traffic("stale") is None
    assert bench.measured_traffic("missing") is None


def test_committed_profiles_match_the_kernel():
    """The committed counter summaries were taken with the current step
    kernel source, so the benchmark line reports measured traffic."""
    for w in ("rotation-fp64", "rotation-fp32", "streamfunction-fp32"):
        assert bench.measured_traffic(w) is not None, w


def _fake_profile(tmp_path, monkeypatch, **figs):
    p = tmp_path / "prof.md"
    p.write_text(f"kernel_source_sha256: {bench.kernel_source_sha()}\n" +
                 "".join(f"{k}: {v}\n" for k, v in figs.items()))
    monkeypatch.setattr(bench, "PROFILES", {"w": str(p)})


def test_roofline_names_the_roof_closer_to_saturation(tmp_path, monkeypatch):
    shape, word = (64, 256, 512), 8
    abytes = bench.algorithmic_bytes(shape, word)
    ms = 0.2                                       # 2.02 TB/s: 0.25 of the HBM roof
    # VALU busy 0.6 of 1024 SIMDs x 2.4 GHz over 0.2 ms
    quad = 0.6 * 1024 * 2.4e9 * 0.2e-3 / 4
    _fake_profile(tmp_path, monkeypatch, traffic_bytes_per_launch=5e8,
                  valu_insts_per_launch=5.6e7, valu_quad_cycles_per_launch=quad)
    roof, valu = bench.roofline("w", shape, word, ms)
    assert roof["bound"] == "alu" and abs(roof["frac"] - 0.6) < 1e-12
    assert abs(roof["hbm"]["frac"] - abytes / 0.2e-3 / 8e12) < 1e-12
    assert roof["traffic"] == 5e8
    assert abs(valu["lane_insts_per_cell_step"] - 5.6e7 * 64 / (512 * 256 * 64)) < 1e-9
    # a kernel whose VALU is idler than its HBM roof is reported against HBM
    _fake_profile(tmp_path, monkeypatch, valu_quad_cycles_per_launch=quad / 10)
    roof, valu = bench.roofline("w", shape, word, ms)
    assert roof["bound"] == "hbm" and valu["frac"] < roof["frac"]
    # no counters of the current source: HBM only
    monkeypatch.setattr(bench, "PROFILES", {})
    roof, valu = bench.roofline("w", shape, word, ms)
    assert roof["bound"] == "hbm" and valu is None and roof["traffic"] is None


def test_error_metrics():
    import numpy as np
    want = np.array([0.0, 1.0, 2.0, -4.0])
    got = want + np.array([0.0, 1e-6, 0.0, -2e-6])
    e = bench.errors(got, want, 3e-9, 7)
    assert abs(e["rel_linf"] / (2e-6 / 4) - 1) < 1e-9
    assert abs(e["rel_l2"] / (np.sqrt(5e-12) / np.sqrt(21)) - 1) < 1e-9
    assert e["mass_drift"] == 3e-9 and e["steps"] == 7


def test_error_steps_follow_the_configured_run():
    import argparse
    a = argparse.Namespace(error_steps=0, steps=20)
    assert bench.error_steps(a, "rotation") == 100  # the configured run, whatever --steps
    a.steps = 300
    assert bench.error_steps(a, "rotation") == 100
    assert bench.error_steps(a, "streamfunction") == 50
    a.error_steps = 3
    assert bench.error_steps(a, "streamfunction") == 3
