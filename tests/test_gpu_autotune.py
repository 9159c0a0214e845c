"""Autotuned work-item sizes: the plan times the candidates on the device,
keeps the fastest, writes the JSON cache, and a second plan of the same shape
reads it back; results agree with a plan at the default sizes."""
import json
import os

import numpy as np
import pytest

import workloads as wl
from gpu_util import make_plan, rel_l2, say

pytestmark = pytest.mark.gpu
import torch  # noqa: E402


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_autotune_and_cache(prec, tmp_path, monkeypatch):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("JGB_AUTOTUNE_CACHE", str(cache))
    p, rho = wl.dipole3d_128(wl.FP64 if prec == "fp64" else wl.MIXED)
    say("autotune", prec)
    tuned = make_plan(p, autotune=True)
    ic, sc = tuned.info["interp_chunk"], tuned.info["spread_chunk"]
    say("   chose interp %d spread %d" % (ic, sc))
    # 0: the interpolation by tiles on the matrix cores was faster; a negative
    # spread chunk: the spreading by rings was
    assert ic in (0, 256, 512, 1024, 2048) and sc in (256, 512, 1024, 2048, 4096, 8192, -512, -1024, -2048, -4096, -8192, -16384)
    data = json.loads(cache.read_text())
    assert len(data) == 1
    entry = next(iter(data.values()))
    assert entry["interp_chunk"] == (ic if ic else -1) and entry["spread_chunk"] == sc
    again = make_plan(p, autotune=True)
    assert (again.info["interp_chunk"], again.info["spread_chunk"]) == (ic, sc)
    plain = make_plan(p)
    dt = torch.float64 if prec == "fp64" else torch.float32
    rt = torch.tensor(rho, dtype=dt, device="cuda")
    ua, Ea = tuned.potential(rt)
    ub, Eb = plain.potential(rt)
    e = rel_l2(ua.cpu().numpy(), ub.cpu().numpy())
    say("   tuned vs default relL2 %.2e" % e)
    assert e < (1e-13 if prec == "fp64" else 1e-6)
    for pl in (tuned, again, plain):
        pl.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_untuned_chunks_fill_the_device(prec):
    """I2's small node set (Algorithm 2 on the 128^3 headline grid): the
    untuned plan halves the default chunks until a launch has two work items
    per CU, and its result still meets the plan's tolerance against the
    density's semi-closed dipole potential; the 1 048 576-node pattern set
    keeps the defaults."""
    p, rho = wl.dipole3d_128(wl.FP64 if prec == "fp64" else wl.MIXED, nodes="split")
    plan = make_plan(p, split=True)
    ic, sc = plan.info["interp_chunk"], plan.info["spread_chunk"]
    say("split plan, untuned chunks: interp %d spread %d" % (ic, sc))
    assert ic < 512 or sc < 4096
    big = make_plan(wl.dipole3d_128(wl.FP64 if prec == "fp64" else wl.MIXED)[0])
    assert (big.info["interp_chunk"], big.info["spread_chunk"]) == (512, 4096)
    dt = torch.float64 if prec == "fp64" else torch.float32
    u, E = plan.potential(torch.tensor(rho, dtype=dt, device="cuda"))
    from oracle import closed_forms as cf
    x = wl.grid_axes(p.n, p.box)
    idx = np.array([[64, 64, 64], [0, 0, 0], [40, 80, 70], [100, 30, 64]])
    pts = np.stack([x[i][idx[:, i]] for i in range(3)], axis=1)
    ref = cf.dipole3d_gaussian_potential(pts, (1.0, 1.5, 0.7), p.axis)
    ug = u.cpu().numpy()
    err = np.max(np.abs(ug[tuple(idx.T)] - ref)) / np.max(np.abs(ug))
    say("   max err / max|u| %.2e" % err)
    assert err < p.eps
    plan.close()
    big.close()
