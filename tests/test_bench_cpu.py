"""Host logic of bench.py (no GPU): the one-GPU guard, the algorithmic work
model behind the roofline figures, the choice of bound, and the lookup of the
PMC-measured HBM traffic, which must go null when the measured kernels'
sources change."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

# plan_info fields of the headline workload (128^3, (128,64,128) nodes: 524 288
# half-set nodes, oversampled 256^3)
INFO64 = {"n": [128, 128, 128], "nf": [256, 256, 256], "width": 12, "n_half": 524288}
INFO32 = dict(INFO64, width=7)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_work_model_bytes_and_flops():
    N, f, cb, rb = 128, 256, 16, 8
    h = f // 2 + 1
    full, _ = bench.stage_work(INFO64, "fp64", half=False)
    # full complex: forward X takes the N-line plane set in, the whole
    # oversampled grid out; the last inverse pass reads the N^2 f input lines
    # and writes u, reading rho for the energy
    assert full["fwd_fft_x"] == N * f * f * cb + f ** 3 * cb
    assert full["inv_fft_z"] == N * N * f * cb + 2 * N ** 3 * rb
    assert full["interp"] == full["spread"] == f ** 3 * cb
    # about 56 N c_b + 2 N r_b with N the oversampled grid size over 8, 1.91 GB
    assert 1.85e9 < sum(full.values()) < 1.95e9
    by, fl = bench.stage_work(INFO64, "fp64")
    # Hermitian half: the last axis keeps h = f/2 + 1 of its f lines, except in
    # what spreading writes and the first inverse pass reads
    assert by["fwd_fft_x"] == N * f * h * cb + f * f * h * cb
    assert by["interp"] == f * f * h * cb and by["spread"] == f ** 3 * cb
    assert by["inv_fft_x"] == f ** 3 * cb + N * f * h * cb
    assert by["inv_fft_z"] == N * N * h * cb + 2 * N ** 3 * rb
    assert fl["interp"] == 5.0 * 524288 * 12 ** 3
    assert 1.2e9 < sum(by.values()) < 1.3e9
    by32, _ = bench.stage_work(INFO32, "mixed")
    assert by32["interp"] == f * f * h * 8


def test_roofline_picks_the_longer_bound():
    by, fl = bench.stage_work(INFO64, "fp64")
    r = bench.roofline("interp", 0.44, by, fl, "fp64")
    # 4.53 GFLOP at 78.6 TFLOP/s outlasts 268 MB at 8 TB/s
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(fl["interp"] / 0.44e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6)
    assert bench.roofline("spread", 0.44, by, fl, "fp64")["bound"] == "mfma"
    by32, fl32 = bench.stage_work(INFO32, "mixed")
    r32 = bench.roofline("interp", 0.07, by32, fl32, "mixed")
    assert r32["bound"] == "hbm" and r32["unit"] == "GB/s"
    assert r32["frac"] == pytest.approx(by32["interp"] / 0.07e-3 / 1e9 / 8000.0)
    # LDS reads of the interpolation: one grid value per tap
    assert bench.lds_bytes(INFO64, "fp64") == 524288 * 12 ** 3 * 16


def _recorded(stage, prec):
    vals = {}
    with open(os.path.join(ROOT, "profiles", "%s_%s_hbm_traffic.md" % (stage, prec))) as f:
        for line in f:
            for key in ("traffic_bytes_per_launch:", "sources_sha1:", "kernel_form:"):
                if line.strip().startswith(key):
                    vals[key] = line.split(":", 1)[1].strip()
    return int(vals["traffic_bytes_per_launch:"]), vals["sources_sha1:"], vals["kernel_form:"]


def test_measured_traffic_follows_the_sources(monkeypatch):
    """The summary's bytes are used while the kernels' sources hash to the value
    recorded with them and the plan runs the form of the kernel measured, and
    dropped (null) otherwise."""
    other = {"tiles": "staged", "staged": "tiles", "rings": "gather", "gather": "rings"}
    for stage in ("interp", "spread"):
        for prec in ("fp64", "mixed"):
            want, sha, form = _recorded(stage, prec)
            assert want > 0 and form in other
            monkeypatch.setattr(bench, "sources_sha1", lambda st, sha=sha: sha)
            assert bench.measured_traffic(stage, prec) == want
            assert bench.measured_traffic(stage, prec, form) == want
            assert bench.measured_traffic(stage, prec, other[form]) is None
            monkeypatch.setattr(bench, "sources_sha1", lambda st: "0" * 40)
            assert bench.measured_traffic(stage, prec) is None
    assert bench.measured_traffic("fwd_fft_x", "fp64") is None
    assert bench.kernel_form("interp", {"interp_chunk": 0, "spread_chunk": -4096}) == "tiles"
    assert bench.kernel_form("spread", {"interp_chunk": 0, "spread_chunk": -4096}) == "rings"
    assert bench.kernel_form("spread", {"interp_chunk": 512, "spread_chunk": 4096}) == "gather"
