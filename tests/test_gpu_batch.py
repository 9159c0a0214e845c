"""Batched evaluation: many independent densities of uneven sizes in one HIP
graph launch (jgb_batch_*).  Every member's result must equal its own plan's
eager evaluation bitwise (same kernels, same order), every replay of the graph
must follow the current contents of the bound densities, and members must
match the oracle."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import load_sampled, rel_l2, sampled_errors, say

pytestmark = pytest.mark.gpu
import torch  # noqa: E402


def _members():
    rng = np.random.default_rng(41)
    out = []
    specs = [((16, 16, 16), 8.0, "coulomb3d", "fp64"), ((24, 20, 16), 10.0, "dipole3d", "fp64"),
             ((32, 32), 12.0, "coulomb2d", "fp64"), ((20, 20, 20), 9.0, "coulomb3d", "mixed"),
             ((16, 24, 20), 9.0, "dipole3d", "mixed"), ((40, 36), 14.0, "coulomb2d", "mixed")]
    for n, L, kern, prec in specs:
        d = len(n)
        box = tuple([L] * d)
        mix = wl.random_mixture(rng, 3, d, -L / 8, L / 8, 0.8, 1.2)
        kernel = {"coulomb3d": wl.COULOMB_3D, "coulomb2d": wl.COULOMB_2D, "dipole3d": wl.DIPOLE_3D}[kern]
        axis = tuple(wl.unit_vector(rng))
        nodes = (12, 8, 16) if d == 3 else (20, 1, 32)
        p = wl.Problem("m", d, n, box, kernel, *nodes, axis=axis if kern == "dipole3d" else (0, 0, 1),
                       eps=1e-10 if prec == "fp64" else 1e-5, precision=wl.FP64 if prec == "fp64" else wl.MIXED)
        kw = dict(n=n, box=box, kernel=kern, nodes=nodes if d == 3 else (nodes[0], nodes[2]), eps=p.eps,
                  precision=prec, axis=p.axis)
        out.append((p, kw, mix.evaluate(n, box)))
    return out


def _dt(kw):
    return torch.float64 if kw["precision"] == "fp64" else torch.float32


def test_batch_equals_eager_and_oracle():
    import paper_1311_4120_amd as jgb
    mem = _members()
    say("batch of", len(mem))
    b = jgb.Batch([kw for _, kw, _ in mem], nstreams=1)
    rhos = [torch.tensor(r, dtype=_dt(kw), device="cuda") for _, kw, r in mem]
    u, E = b.bind(rhos)
    # one stream: one launch per pipeline site over the members that have it
    # (members of different kinds and precisions share few sites)
    say("   %d launches per run" % b.launches())
    assert 0 < b.launches() <= 6 * 12
    b.run()
    torch.cuda.synchronize()
    for i, (p, kw, r) in enumerate(mem):
        ue, Ee = b.plans[i].potential(rhos[i])
        torch.cuda.synchronize()
        assert torch.equal(u[i], ue), i
        assert E[i].item() == Ee.item(), i
        rin = r if kw["precision"] == "fp64" else r.astype(np.float32).astype(np.float64)
        res = oracle.evaluate(p, rin)
        e = rel_l2(u[i].cpu().numpy(), res.u)
        say("   member %d %s %s relL2 %.2e" % (i, kw["kernel"], kw["precision"], e))
        assert e < p.eps
    b.close()


@pytest.mark.parametrize("nstreams", [1, 2])
def test_graph_replays_follow_inputs(nstreams):
    import paper_1311_4120_amd as jgb
    mem = _members()[:4]
    b = jgb.Batch([kw for _, kw, _ in mem], nstreams=nstreams)
    rhos = [torch.tensor(r, dtype=_dt(kw), device="cuda") for _, kw, r in mem]
    u, E = b.bind(rhos)
    gen = torch.Generator(device="cpu").manual_seed(3)
    for rep in range(3):
        say("replay", rep)
        # eager work between replays: rewrite the densities in place
        for r in rhos:
            r.copy_(torch.rand(r.shape, generator=gen, dtype=torch.float64).to(r.dtype).cuda())
        torch.cuda.synchronize()
        b.run()
        torch.cuda.synchronize()
        for i in range(len(mem)):
            ue, Ee = b.plans[i].potential(rhos[i])
            torch.cuda.synchronize()
            assert torch.equal(u[i], ue), (rep, i)
            assert E[i].item() == Ee.item(), (rep, i)
    b.close()


@pytest.mark.parametrize("nstreams,autotune", [(1, False), (4, False), (1, True)])
def test_batched_coulomb_workload(nstreams, autotune):
    """64 seeded densities, N in {64, 96, 128, 160}, mixed precision, one graph:
    one launch per pipeline site over all members (one stream) or the members'
    pipelines on four streams; with autotuned members, the tap-kernel forms the
    tuner picks per member (the interpolation by tiles among them, whose
    forward transform stores only each line's read range, here on 128- to
    320-point lines)."""
    import paper_1311_4120_amd as jgb
    members = wl.batched_coulomb()
    kws, rhos = [], []
    for p, mix in members:
        kws.append(dict(n=p.n, box=p.box, kernel="coulomb3d", nodes=(p.n_r, p.n_theta, p.n_phi), eps=p.eps,
                        precision="mixed", autotune=autotune))
    say("batched_coulomb: planning 64 members", "(autotuned)" if autotune else "")
    b = jgb.Batch(kws, nstreams=nstreams)
    if autotune:
        tiles = sum(pl.info["interp_chunk"] == 0 for pl in b.plans)
        say("   %d members interpolate by tiles" % tiles)
        assert tiles > 0
    for p, mix in members:
        rhos.append(torch.tensor(mix.evaluate(p.n, p.box), dtype=torch.float32, device="cuda"))
    u, E = b.bind(rhos)
    say("   %d launches per run" % b.launches())
    if nstreams == 1:  # about ten launches instead of 64 pipelines of about ten kernels
        assert b.launches() <= 16
    else:
        assert b.launches() >= 64 * 8
    b.run()
    torch.cuda.synchronize()
    say("   run ok; checking members against their eager results and the closed forms")
    for i in (0, 17, 63):
        ue, Ee = b.plans[i].potential(rhos[i])
        torch.cuda.synchronize()
        assert torch.equal(u[i], ue)
    # energies against the Gaussian-mixture closed form (a physics check: the
    # grid, box and node counts of this workload resolve it to ~1e-5)
    worst = 0.0
    for i, (p, mix) in enumerate(members):
        Ec = oracle.closed_forms.mixture_energy(mix, 3)
        worst = max(worst, abs(E[i].item() / Ec - 1))
    say("   worst energy deviation from the closed form %.2e" % worst)
    assert worst < 1e-3
    # the smallest member against the whole-grid oracle
    i = min(range(64), key=lambda k: members[k][0].npoints)
    p, mix = members[i]
    res = oracle.evaluate(p, rhos[i].double().cpu().numpy())
    e = rel_l2(u[i].cpu().numpy(), res.u)
    say("   member %d (%s) relL2 vs oracle %.2e" % (i, p.n, e))
    assert e < 1e-5
    # one member of each grid size (64^3 .. 160^3) against the oracle's sampled
    # values (4096 sub-lattice points, three axis lines, 512 random points) and
    # its Fourier-side energy
    for i in (7, 3, 0, 1):
        ref = load_sampled("batched_coulomb_%d" % i)
        assert tuple(ref["n"]) == members[i][0].n
        e, emax, ns = sampled_errors(u[i].cpu().numpy().astype(np.float64), ref)
        eE = abs(E[i].item() / float(ref["energy"]) - 1)
        say("   member %d (%s): %d sampled points relL2 %.2e max/|u|max %.2e  E %.2e" % (i, members[i][0].n, ns, e,
                                                                                      emax, eE))
        assert e < 1e-5 and emax < 1e-5 and eE < 1e-5
    b.close()
