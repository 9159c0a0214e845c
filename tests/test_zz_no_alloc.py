"""jgb_potential_noalloc, the entry point for callers that cannot allocate:
called through the C ABI, it must give jgb_potential's u and E (bitwise: the
same kernels in the same order) on two calls in a row, the second on a smaller
problem, so that the shared scratch array holds the first call's leftovers;
a plan too large for the array is refused; the plan's own path is unchanged
afterwards."""
import ctypes

import numpy as np
import pytest

import workloads as wl
from gpu_util import MODES, make_plan, rel_l2, say

pytestmark = pytest.mark.gpu
import torch  # noqa: E402


def _problem(n, prec, kernel=wl.DIPOLE_3D, split=False):
    rng = np.random.default_rng(n)
    axis = tuple(wl.unit_vector(rng))
    L = 0.25 * n
    p = wl.Problem("noalloc_%d" % n, 3, (n, n, n), (L, L, L), kernel, n, n // 2, n, axis=axis,
                   eps=1e-10 if prec == "fp64" else 1e-5, precision=wl.FP64 if prec == "fp64" else wl.MIXED)
    rho = wl.anisotropic_gaussian(p.n, p.box, (1.0, 1.4, 0.8), center=(0.2, -0.3, 0.1))
    return p, rho


def _noalloc(plan, rho, u, E):
    from paper_1311_4120_amd import _lib
    return _lib.lib.jgb_potential_noalloc(plan._h, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                          ctypes.c_void_p(E.data_ptr()))


@pytest.mark.parametrize("mode", ["staged", "tiles+rings"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_equals_potential(prec, mode):
    from paper_1311_4120_amd import _lib
    dt = torch.float64 if prec == "fp64" else torch.float32
    for n in (48, 24):   # the second call is smaller: the array holds the first call's values
        p, rho = _problem(n, prec)
        say("noalloc", prec, n, mode)
        plan = make_plan(p, **MODES[mode])
        rt = torch.tensor(rho, dtype=dt, device="cuda")
        u_ref, E_ref = plan.potential(rt)
        u = torch.full_like(rt, float("nan"))
        E = torch.full((), float("nan"), dtype=torch.float64, device="cuda")
        assert _noalloc(plan, rt, u, E) == _lib.JGB_OK, _lib.lib.jgb_last_error()
        torch.cuda.synchronize()
        say("   max |u - u_ref| = %.3e, E %.17g vs %.17g" % ((u - u_ref).abs().max().item(), E.item(), E_ref.item()))
        assert torch.equal(u, u_ref) and E.item() == E_ref.item()
        # the plan's own path still gives the same result afterwards
        u2, E2 = plan.potential(rt)
        assert torch.equal(u2, u_ref) and E2.item() == E_ref.item()
        plan.close()


def test_noalloc_split_and_poisson():
    from paper_1311_4120_amd import _lib
    import paper_1311_4120_amd as jgb
    # Algorithm 2 (its grid G first receives the unmixed spectrum) and a kernel
    # with a node at k = 0 (its origin partials also live in the array)
    p, rho = _problem(32, "fp64", kernel=wl.COULOMB_3D)
    plan = make_plan(p, split=True)
    rt = torch.tensor(rho, dtype=torch.float64, device="cuda")
    u_ref, E_ref = plan.potential(rt)
    u = torch.empty_like(rt)
    E = torch.empty((), dtype=torch.float64, device="cuda")
    assert _noalloc(plan, rt, u, E) == _lib.JGB_OK
    torch.cuda.synchronize()
    assert torch.equal(u, u_ref) and E.item() == E_ref.item()
    plan.close()
    n = 64
    x = wl.grid_axes((n, n), (16.0, 16.0))
    r2 = x[0][:, None] ** 2 + x[1][None, :] ** 2
    r = torch.tensor(np.exp(-r2), dtype=torch.float64, device="cuda")
    plan = jgb.Plan((n, n), (16.0, 16.0), "poisson2d", (32, 64), eps=1e-10)
    u_ref, E_ref = plan.potential(r)
    u = torch.empty_like(r)
    E = torch.empty((), dtype=torch.float64, device="cuda")
    assert _noalloc(plan, r, u, E) == _lib.JGB_OK
    torch.cuda.synchronize()
    assert torch.equal(u, u_ref) and E.item() == E_ref.item()
    plan.close()


def test_noalloc_refuses_plans_beyond_the_array():
    from paper_1311_4120_amd import _lib
    p, rho = _problem(128, "fp64")
    plan = make_plan(p)
    assert plan.info["workspace_bytes"] > _lib.NOALLOC_SCRATCH_BYTES
    rt = torch.tensor(rho, dtype=torch.float64, device="cuda")
    u = torch.zeros_like(rt)
    E = torch.zeros((), dtype=torch.float64, device="cuda")
    assert _noalloc(plan, rt, u, E) == _lib.JGB_ERR_UNSUPPORTED
    assert b"exceeds" in _lib.lib.jgb_last_error()
    torch.cuda.synchronize()
    assert float(u.abs().max()) == 0.0   # nothing was enqueued
    u_ref, _ = plan.potential(rt)
    assert torch.isfinite(u_ref).all()
    plan.close()
