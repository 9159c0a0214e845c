"""Throughput of the free-space dipole convolution on one MI355X.

Workload: 3D dipole-dipole kernel U^ = -1 + 3 (n.k)^2/|k|^2 on a 128^3 grid over
[-12,12)^3, rho = |psi|^2 for the anisotropic Gaussian psi with axes
(1, 1.5, 0.7), seeded dipole axis, Fourier nodes (128, 64, 128) with the theta
Gauss-Legendre rule (M = 1 048 576).  One step = one potential evaluation: u on
the whole grid plus the energy E, i.e. Algorithm 1 (type-2 NUFFT, weight x
symbol, type-1 NUFFT) and the trapezoid energy sum, inputs resident in HBM.

Runs the path in float64 at eps = 1e-10 (the headline value) and in mixed
precision at eps = 1e-5, prints one JSON line.  Per-kernel durations come from
HIP events recorded on the plan's stream inside the timed loop.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
# LDS: 128 bytes per clock per CU, 256 CUs at 2.4 GHz
LDS_PEAK_TBS = 128 * 256 * 2.4e9 / 1e12
METRIC = "potential evals/s + ns/grid-pt at 128³: FP64 ε=1e-10 vs mixed FP32 ε=1e-5"


def stage_work(info, prec, energy=True, half=True):
    """Algorithmic HBM bytes and flops of one launch of each stage.

    FFT passes: input + output of the pass.  For a real density (Algorithm 1)
    the spectrum is kept on the Hermitian half h = f/2 + 1 of the lines along
    the last axis (half=True): every pass but the inverse's first moves h/f of
    the full-complex bytes, and that first pass is counted as reading all of G
    (each line and its mirror; the kernel itself loads only the part of each
    line that node footprints reach, so its rate against this count overstates
    the HBM rate it achieves).  Tap kernels: one pass over the oversampled grid
    (interpolation reads the stored spectrum, spreading writes G) and 5 flops
    per tap (complex x real multiply-add + the weight product) over the w^3
    taps of every node the launch processes (the half set; the other half is
    its mirror image)."""
    n = info["n"]
    nf = info["nf"]
    N = n[0]
    f = nf[0]
    h = f // 2 + 1 if half else f
    rb = 8 if prec == "fp64" else 4
    cb = 2 * rb
    w = info["width"]
    Mh = info["n_half"]
    N3, F3 = N ** 3, f ** 3
    by = {
        "fwd_fft_z": N3 * rb + N * N * h * cb,
        "fwd_fft_y": N * N * h * cb + N * f * h * cb,
        "fwd_fft_x": N * f * h * cb + f * f * h * cb,
        "inv_fft_x": F3 * cb + N * f * h * cb,
        "inv_fft_y": N * f * h * cb + N * N * h * cb,
        "inv_fft_z": N * N * h * cb + N3 * rb + (N3 * rb if energy else 0),
        "interp": f * f * h * cb,
        "spread": F3 * cb,
    }
    fl = {"interp": 5.0 * Mh * w ** 3, "spread": 5.0 * Mh * w ** 3}
    return by, fl


def lds_bytes(info, prec):
    """LDS bytes the interpolation reads per launch: one grid value per tap."""
    cb = 16 if prec == "fp64" else 8
    return info["n_half"] * info["width"] ** 3 * cb


# Kernel sources whose measured HBM traffic a stage's roofline may quote: the
# summary in profiles/ is used only while these files are unchanged.
STAGE_SOURCES = {
    "interp": ["paper_1311_4120_amd/csrc/interp.hip"],
    "spread": ["paper_1311_4120_amd/csrc/spread.hip", "paper_1311_4120_amd/csrc/ring.hip"],
}
TRAFFIC_SOURCES_COMMON = ["paper_1311_4120_amd/csrc/plan.hip", "paper_1311_4120_amd/csrc/common.h",
                          "paper_1311_4120_amd/csrc/nodes.hip", "paper_1311_4120_amd/csrc/lists.h"]


def sources_sha1(stage):
    import hashlib
    h = hashlib.sha1()
    for rel in STAGE_SOURCES.get(stage, []) + TRAFFIC_SOURCES_COMMON:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def kernel_form(stage, tuned):
    """The form of the stage's kernel the plan chose: the interpolation by
    tiles or staged, the spreading by rings or the three-axis gather."""
    if stage == "interp":
        return "tiles" if tuned["interp_chunk"] == 0 else "staged"
    if stage == "spread":
        return "rings" if tuned["spread_chunk"] < 0 else "gather"
    return None


def measured_traffic(stage, prec, form=None):
    """HBM bytes per launch of the stage's kernel from the committed PMC
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's counters), or
    None when there is none, the kernel sources changed since, or the summary
    measured another form of the kernel than `form`."""
    if stage not in STAGE_SOURCES:
        return None
    path = os.path.join(ROOT, "profiles", "%s_%s_hbm_traffic.md" % (stage, prec))
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            for key in ("traffic_bytes_per_launch:", "sources_sha1:", "kernel_form:"):
                if line.strip().startswith(key):
                    vals[key] = line.split(":", 1)[1].strip()
    if vals.get("sources_sha1:") != sources_sha1(stage) or "traffic_bytes_per_launch:" not in vals:
        return None
    if form is not None and vals.get("kernel_form:") != form:
        return None
    return int(vals["traffic_bytes_per_launch:"])


def copy_calibration(mib=256, reps=5):
    """A plain device copy of a known size, for scaling the PMC byte counters."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4, "reps": reps}))


def roofline(stage, ms, by, fl, prec):
    """The stage's roofline: whichever bound (HBM bytes, or flops at the
    compute peak of its unit) takes longer, and the achieved fraction of it."""
    t = ms * 1e-3
    t_mem = by[stage] / (HBM_PEAK_GBS * 1e9)
    peak = FP64_PEAK_TFLOPS if prec == "fp64" else FP32_PEAK_TFLOPS
    t_cmp = fl[stage] / (peak * 1e12) if stage in fl else 0.0
    if t_cmp > t_mem:
        ach = fl[stage] / t / 1e12
        return {"kernel": stage, "bound": "mfma" if stage == "spread" else "alu", "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak, "traffic": None, "flops_per_launch": fl[stage],
                "bytes_per_launch": by[stage]}
    ach = by[stage] / t / 1e9
    out = {"kernel": stage, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": ach / HBM_PEAK_GBS, "traffic": None, "bytes_per_launch": by[stage]}
    if stage in fl:
        out["flops_per_launch"] = fl[stage]
    return out


def run_gpu(prec, steps, warmup, nodes="pattern", eps=None, gaussian=False):
    import torch

    import paper_1311_4120_amd as jgb
    import workloads as wl

    p, rho = wl.dipole3d_128(wl.FP64 if prec == "fp64" else wl.MIXED, nodes=nodes)
    dt = torch.float64 if prec == "fp64" else torch.float32
    t0 = time.time()
    if eps is not None:
        p.eps = eps
    plan = jgb.Plan(p.n, p.box, "dipole3d", (p.n_r, p.n_theta, p.n_phi), eps=p.eps, precision=prec,
                    lam=p.lam, axis=p.axis, theta_rule="theta" if p.theta_rule == wl.THETA_GL else "costheta",
                    autotune=True, split=(nodes == "split"), gaussian_kernel=gaussian)
    torch.cuda.synchronize()
    plan_s = time.time() - t0
    rt = torch.tensor(rho, dtype=dt, device="cuda")
    u = torch.empty_like(rt)
    E = torch.empty((), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        plan.potential(rt, out=u)
    torch.cuda.synchronize()
    # the timed steps carry no instrumentation
    t0 = time.perf_counter()
    for _ in range(steps):
        u, E = plan.potential(rt, out=u)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-step durations (HIP events around each call on the plan's stream), in
    # a separate run: median and the p10-p90 range
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in evs:
        a.record(plan.stream)
        plan.potential(rt, out=u)
        b.record(plan.stream)
    torch.cuda.synchronize()
    per = np.array([a.elapsed_time(b) for a, b in evs])
    step_pct = {"p10": float(np.percentile(per, 10)), "median": float(np.median(per)),
                "p90": float(np.percentile(per, 90))}
    # per-stage durations from HIP events on the plan's stream, in a separate
    # run of the same steps
    plan.timing_begin(steps)
    for _ in range(steps):
        u, E = plan.potential(rt, out=u)
    torch.cuda.synchronize()
    stages, ncalls = plan.timing_end()
    energy = float(E.item())
    info = plan.info
    plan.close()
    return {"wall_s": wall, "ms_per_step": 1e3 * wall / steps, "step_ms": step_pct, "stages_ms": stages, "calls": ncalls,
            "plan_s": plan_s, "energy": energy, "info": info, "eps": p.eps,
            "tuned": {"interp_chunk": info["interp_chunk"], "spread_chunk": info["spread_chunk"]}}


def run_batched(steps, warmup, nstreams=1):
    """64 seeded Gaussian-mixture densities, N in {64, 96, 128, 160}, mixed
    precision, evaluated by one HIP graph launch per step: with one stream the
    graph holds one kernel launch per pipeline site over all members; with
    more, every member's own pipeline on nstreams concurrent branches."""
    import torch

    import paper_1311_4120_amd as jgb
    import workloads as wl

    members = wl.batched_coulomb()
    kws = [dict(n=p.n, box=p.box, kernel="coulomb3d", nodes=(p.n_r, p.n_theta, p.n_phi), eps=p.eps,
                precision="mixed", autotune=True) for p, _ in members]
    # members of one grid size share a tuning: cache it for the run
    os.environ.setdefault("JGB_AUTOTUNE_CACHE", os.path.join("/tmp", "jgb_autotune_bench_%d.json" % os.getpid()))
    t0 = time.time()
    b = jgb.Batch(kws, nstreams=nstreams)
    rhos = [torch.tensor(mix.evaluate(p.n, p.box), dtype=torch.float32, device="cuda") for p, mix in members]
    b.bind(rhos)
    torch.cuda.synchronize()
    plan_s = time.time() - t0
    launches = b.launches()
    for _ in range(warmup):
        b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.run()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    npts = sum(p.npoints for p, _ in members)
    nodes = sum(p.nnodes for p, _ in members)
    b.close()
    return {"workload": "batched_coulomb", "members": len(members), "grid_points": npts, "nodes": nodes,
            "ms_per_launch": 1e3 * wall / steps, "evals_per_s": len(members) * steps / wall,
            "grid_points_per_s": npts * steps / wall, "launches": steps, "plan_and_capture_s": plan_s,
            "precision": "mixed", "eps": 1e-5, "nstreams": nstreams, "kernel_launches_per_step": launches,
            "ns_per_point": 1e9 * wall / steps / npts,
            "graph": ("one hipGraph launch per step: one kernel launch per pipeline site over all members"
                      if nstreams == 1 else
                      "one hipGraph launch per step: the members' pipelines on %d branches" % nstreams)}


def run_resolved(steps, warmup):
    """The accuracy-matched node sets of the 128^3 dipole workload: (256,128,256)
    cos(theta) nodes in float64, (192,96,192) in mixed precision."""
    out = {"workload": "dipole3d_128, accuracy-matched nodes"}
    for prec, nodes in (("fp64", [256, 128, 256]), ("mixed", [192, 96, 192])):
        r = run_gpu(prec, steps, warmup, nodes="resolved")
        out[prec] = {"nodes": nodes, "n_nodes": r["info"]["n_nodes"], "eps": r["eps"], "ms_per_step": r["ms_per_step"],
                     "evals_per_s": 1e3 / r["ms_per_step"], "ns_per_point": r["ms_per_step"] * 1e6 / 128 ** 3,
                     "stages_ms": {k: v for k, v in r["stages_ms"].items() if v > 0}}
    return out


def run_algorithm2(steps, warmup, resolved=None, precs=("fp64", "mixed")):
    """The same 128^3 dipole evaluation by Algorithm 2 (the partition-of-unity
    split of Section 3.3) at the default window and I2 cut-off, with I2's node
    sets matched to the accuracy of the resolved Algorithm 1 sets."""
    out = {"workload": "dipole3d_128 by Algorithm 2, accuracy-matched I2 nodes"}
    for prec, nodes in (("fp64", [28, 20, 40]), ("mixed", [20, 16, 32])):
        if prec not in precs:
            continue
        r = run_gpu(prec, steps, warmup, nodes="split")
        d = {"nodes": nodes, "n_nodes": r["info"]["n_nodes"], "kmax_I2": r["info"]["kmax"],
             "window_a": r["info"]["window"][0], "eps": r["eps"], "ms_per_step": r["ms_per_step"],
             "evals_per_s": 1e3 / r["ms_per_step"], "ns_per_point": r["ms_per_step"] * 1e6 / 128 ** 3,
             "energy": r["energy"], "stages_ms": {k: v for k, v in r["stages_ms"].items() if v > 0}}
        if resolved and prec in resolved:
            d["speedup_vs_algorithm1_resolved"] = resolved[prec]["ms_per_step"] / r["ms_per_step"]
        out[prec] = d
    return out


def run_gpe(steps, warmup):
    """Real-time Strang steps of a dipolar condensate on the 128^3 grid of the
    dipole workload: psi with axes (1, 1.5, 0.7) normalised, trap (1, 1, 2),
    beta = 100, lambda = 30 (dipole axis of the workload), dt = 1e-3, the
    potential by Algorithm 2 with the accuracy-matched I2 nodes.  One step =
    two local phase kernels, a periodic FFT pair with the kinetic multiplier,
    and one potential evaluation, replayed from one HIP graph."""
    import torch

    import paper_1311_4120_amd as jgb
    import workloads as wl

    out = {"workload": "dipolar GPE on dipole3d_128's grid, real time, potential by Algorithm 2",
           "dt": 1e-3, "beta": 100.0, "lambda": 30.0, "trap": [1.0, 1.0, 2.0]}
    for prec in ("fp64", "mixed"):
        p, rho = wl.dipole3d_128(wl.FP64 if prec == "fp64" else wl.MIXED, nodes="split")
        cdt = torch.complex128 if prec == "fp64" else torch.complex64
        H = float(np.prod([b / m for b, m in zip(p.box, p.n)]))
        psi0 = np.sqrt(rho)
        psi0 = psi0 / np.sqrt(H * np.sum(psi0 ** 2))
        drv = jgb.GPE(p.n, p.box, "dipole3d", (p.n_r, p.n_theta, p.n_phi), dt=1e-3, beta=100.0,
                      trap=(1.0, 1.0, 2.0), eps=p.eps, precision=prec, lam=30.0, axis=p.axis,
                      theta_rule="costheta", split=True, autotune=True)
        psi = torch.tensor(psi0, dtype=cdt, device="cuda")
        drv.step(psi, warmup)
        torch.cuda.synchronize()
        _, e0 = drv.energy(psi)
        t0 = time.perf_counter()
        drv.step(psi, steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        _, e1 = drv.energy(psi)
        drv.close()
        out[prec] = {"nodes": [p.n_r, p.n_theta, p.n_phi], "eps": p.eps, "ms_per_step": 1e3 * wall / steps,
                     "steps_per_s": steps / wall, "potential_evals_per_step": 1,
                     "norm_drift": abs(e1["norm"] - e0["norm"]), "energy_drift_rel": abs(e1["total"] / e0["total"] - 1),
                     "energy": e1["total"], "mu": e1["mu"]}
    return out


def run_grad256(steps, warmup):
    """Differentiable dipolar energy on 256^3 (psi = 6 wave packets, complex64,
    mixed precision, nodes (256,128,256)): one step = E(|psi|^2) forward and
    dE/dpsi* backward through the autograd function."""
    import torch

    import paper_1311_4120_amd as jgb
    import workloads as wl

    p, packets = wl.dipole_grad_256()
    plan = jgb.Plan(p.n, p.box, "dipole3d", (p.n_r, p.n_theta, p.n_phi), eps=p.eps, precision="mixed",
                    lam=p.lam, axis=p.axis, theta_rule="costheta", autotune=True)
    psi = torch.tensor(packets.evaluate(p.n, p.box), dtype=torch.complex64, device="cuda", requires_grad=True)

    def step():
        psi.grad = None
        E = jgb.DipolarEnergy.apply(psi, plan)
        E.backward()
        return E

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        E = step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.close()
    return {"workload": "dipole_grad_256", "grid": [256, 256, 256], "nodes": [256, 128, 256], "precision": "mixed",
            "eps": p.eps, "ms_per_step": 1e3 * wall / steps, "steps_per_s": steps / wall,
            "step": "E(|psi|^2) forward + dE/dpsi* backward", "energy": float(E.item())}


def fft_comparison(res):
    """The six pruned passes of one evaluation against rocFFT (torch.fft on ROCm)
    doing the unpruned forward and inverse 3D transforms of the same 256^3
    oversampled grid."""
    import torch

    out = {}
    passes = ["fwd_fft_z", "fwd_fft_y", "fwd_fft_x", "inv_fft_x", "inv_fft_y", "inv_fft_z"]
    for prec, dt in (("fp64", torch.complex128), ("mixed", torch.complex64)):
        if prec not in res:
            continue
        x = torch.randn((256, 256, 256), dtype=dt, device="cuda")
        for _ in range(3):
            y = torch.fft.ifftn(torch.fft.fftn(x))
        torch.cuda.synchronize()
        n = 20
        t0 = time.perf_counter()
        for _ in range(n):
            y = torch.fft.ifftn(torch.fft.fftn(x))
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / n
        del x, y
        ours = sum(res[prec]["stages_ms"].get(k, 0.0) for k in passes)
        out[prec] = {"rocfft_fwd_plus_inv_ms": ms, "pruned_passes_ms": ours, "speedup": ms / ours if ours else None}
    return out


def cpu_baseline(sample_nodes=32768):
    """The oracle (direct O(N M) sums) on a bounded sample of the same workload:
    the type-2 sum at every 32nd node and the type-1 sum from those nodes to the
    whole grid, extrapolated linearly in the node count to a full evaluation."""
    from threadpoolctl import threadpool_info, threadpool_limits

    import oracle
    import workloads as wl

    p, rho = wl.dipole3d_128()
    k, W = oracle.fourier_nodes(p)
    stride = max(1, len(k) // sample_nodes)
    idx = np.arange(0, len(k), stride)[:sample_nodes]
    kb, Wb = k[idx], W[idx]
    t0 = time.perf_counter()
    rh = oracle.rho_hat(rho, p.box, kb)
    c = oracle.coefficients(p.kernel, kb, Wb, p.axis)
    oracle.sum_to_grid(c * rh, kb, p.n, p.box)
    t = time.perf_counter() - t0
    full = t * len(k) / len(idx)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    # the same sums on one BLAS thread, at an 8 times smaller sample
    idx1 = idx[::8]
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        rh1 = oracle.rho_hat(rho, p.box, k[idx1])
        c1 = oracle.coefficients(p.kernel, k[idx1], W[idx1], p.axis)
        oracle.sum_to_grid(c1 * rh1, k[idx1], p.n, p.box)
        t1 = time.perf_counter() - t1
    full1 = t1 * len(k) / len(idx1)
    # the two small workloads, one whole oracle evaluation each (u both ways and E)
    small = {}
    p1, rho1 = wl.coulomb3d_32()
    p2, rho2, _ = wl.coulomb2d_256()
    for name, (pp, rr) in (("coulomb3d_32", (p1, rho1)), ("coulomb2d_256", (p2, rho2))):
        ts = time.perf_counter()
        oracle.evaluate(pp, rr)
        ts = time.perf_counter() - ts
        small[name] = {"s_per_eval": ts, "evals_per_s": 1.0 / ts}
    cpu_model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": 1.0 / full, "unit": "evals/s", "cores": int(threads), "kind": "oracle",
            "cpu_model": cpu_model, "host_cpus_available": len(os.sched_getaffinity(0)),
            "sample": "type-2 sum at %d of %d nodes (every %d-th) + type-1 sum from them to all 128^3 points, "
                      "%.1f s, extrapolated x%.1f to one full evaluation (%.0f s); O(N M) direct sums"
                      % (len(idx), len(k), stride, t, len(k) / len(idx), full),
            "one_thread": {"value": 1.0 / full1, "unit": "evals/s", "cores": 1,
                           "sample": "the same sums at %d nodes, %.1f s, extrapolated x%.0f (%.0f s)"
                                     % (len(idx1), t1, len(k) / len(idx1), full1)},
            "full_small": small,
            "context": "the paper's Algorithm 2 timings on its Xeon workstation: about 7.3 us per grid point "
                       "at 2 097 152 points (another machine and code; context only)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["fp64", "mixed"], default=None)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--algorithm2-only", action="store_true",
                    help="only time the 128^3 dipole by Algorithm 2 and print its object")
    ap.add_argument("--gpe-only", action="store_true", help="only time the GPE driver and print its object")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (PMC byte-counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the path runs on a single MI355X; "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.gpe_only:
        print(json.dumps(run_gpe(args.steps, args.warmup)))
        return
    if args.algorithm2_only:
        print(json.dumps(run_algorithm2(args.steps, args.warmup,
                                        precs=("fp64", "mixed") if args.only is None else (args.only,))))
        return

    res = {}
    for prec in (["fp64", "mixed"] if args.only is None else [args.only]):
        print("[bench] %s: plan + %d warmup + %d timed steps" % (prec, args.warmup, args.steps), file=sys.stderr,
              flush=True)
        res[prec] = run_gpu(prec, args.steps, args.warmup)
        print("[bench] %s: %.4f ms/step" % (prec, res[prec]["ms_per_step"]), file=sys.stderr, flush=True)

    head = "fp64" if "fp64" in res else "mixed"
    r = res[head]
    npts = 128 ** 3
    by, fl = stage_work(r["info"], head)
    st = r["stages_ms"]
    dom = max((k for k in st if st[k] > 0), key=lambda k: st[k])
    roof = roofline(dom, st[dom], by, fl, head)
    roof["form"] = kernel_form(dom, r["tuned"])
    roof["traffic"] = measured_traffic(dom, head, roof["form"])
    stages = {}
    for k, v in st.items():
        if v <= 0:
            continue
        d = {"ms": v, "GB/s": by.get(k, 0) / (v * 1e-3) / 1e9 if k in by else None}
        if k in fl:
            d["TFLOP/s"] = fl[k] / (v * 1e-3) / 1e12
        if k in by:
            # the fraction of the stage's own bounding roofline: HBM for the FFT
            # passes; for the tap kernels the longest of HBM, arithmetic and
            # (interpolation) LDS reads
            rf = roofline(k, v, by, fl, head)
            d["bound"], d["frac"] = rf["bound"], rf["frac"]
            if k == "interp" and kernel_form(k, r["tuned"]) == "staged":
                t_lds = lds_bytes(r["info"], head) / (LDS_PEAK_TBS * 1e12)
                if t_lds / (v * 1e-3) > d["frac"]:
                    d["bound"], d["frac"] = "lds", t_lds / (v * 1e-3)
        stages[k] = d
    total_bytes = sum(by.values())
    # the full-complex model of the scope (no Hermitian halving), for comparison
    full_bytes = sum(stage_work(r["info"], head, half=False)[0].values())
    out = {
        "metric": METRIC,
        "value": 1e3 / r["ms_per_step"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "dipole3d_128", "kernel": "dipole3d", "grid": [128, 128, 128],
                   "box": [-12, 12], "nodes": [128, 64, 128], "theta_rule": "theta_gl",
                   "n_nodes": r["info"]["n_nodes"], "eps": r["eps"], "width": r["info"]["width"],
                   "oversampled_grid": r["info"]["nf"]},
        "ns_per_point": r["ms_per_step"] * 1e6 / npts,
        "step_ms": r["step_ms"],
        "energy": r["energy"],
        "plan_s": r["plan_s"],
        "autotuned": r["tuned"],
        "model_hbm_bytes_per_step": total_bytes,
        "model_hbm_frac": total_bytes / (r["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "model_hbm_bytes_full_complex": full_bytes,
        "model_hbm_frac_full_complex": full_bytes / (r["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "stages": stages,
        "roofline": roof,
    }
    if "mixed" in res and head == "fp64":
        m = res["mixed"]
        out["mixed"] = {"value": 1e3 / m["ms_per_step"], "unit": "evals/s", "ms_per_step": m["ms_per_step"],
                        "step_ms": m["step_ms"],
                        "ns_per_point": m["ms_per_step"] * 1e6 / npts, "eps": m["eps"],
                        "width": m["info"]["width"], "energy": m["energy"],
                        "speedup_vs_fp64": r["ms_per_step"] / m["ms_per_step"],
                        "stages_ms": {k: v for k, v in m["stages_ms"].items() if v > 0}}
    if "mixed" in res and head == "fp64":
        # both precisions at the same stated accuracy: float64 at eps = 1e-5
        print("[bench] fp64 at eps 1e-5 (the mixed path's accuracy)", file=sys.stderr, flush=True)
        f5 = run_gpu("fp64", args.steps, args.warmup, eps=1e-5)
        m = res["mixed"]
        out["equal_accuracy_1e-5"] = {
            "eps": 1e-5, "fp64": {"value": 1e3 / f5["ms_per_step"], "ms_per_step": f5["ms_per_step"],
                                  "width": f5["info"]["width"]},
            "mixed": {"value": 1e3 / m["ms_per_step"], "ms_per_step": m["ms_per_step"], "width": m["info"]["width"]},
            "mixed_speedup": f5["ms_per_step"] / m["ms_per_step"]}
        # the paper's Gaussian spreading kernel (12 points per axis, about six
        # digits) against the exponential of a semicircle at the same eps
        print("[bench] the paper's Gaussian kernel at eps 1e-6", file=sys.stderr, flush=True)
        ga = {}
        for prec in ("fp64", "mixed"):
            e6 = 1e-6 if prec == "fp64" else 1e-5
            g = run_gpu(prec, args.steps, args.warmup, eps=e6, gaussian=True)
            es = run_gpu(prec, args.steps, args.warmup, eps=e6)
            ga[prec] = {"eps": e6, "gaussian": {"ms_per_step": g["ms_per_step"], "width": g["info"]["width"]},
                        "semicircle": {"ms_per_step": es["ms_per_step"], "width": es["info"]["width"]},
                        "gaussian_cost": g["ms_per_step"] / es["ms_per_step"]}
        out["gaussian_kernel"] = ga
    if not args.no_batched and args.only is None:
        print("[bench] batched_coulomb: 64 densities, one graph launch per step", file=sys.stderr, flush=True)
        out["batched"] = run_batched(max(3, args.steps // 10), 2)
        out["batched_streams"] = run_batched(max(3, args.steps // 10), 2, nstreams=4)
        print("[bench] dipole3d_128 with accuracy-matched node sets", file=sys.stderr, flush=True)
        out["resolved"] = run_resolved(max(3, args.steps // 5), 2)
        print("[bench] dipole3d_128 by Algorithm 2", file=sys.stderr, flush=True)
        out["algorithm2"] = run_algorithm2(max(3, args.steps // 2), 3, out["resolved"])
        print("[bench] dipolar GPE, real-time steps", file=sys.stderr, flush=True)
        out["gpe"] = run_gpe(max(10, args.steps), 3)
        print("[bench] dipole_grad_256: forward + backward", file=sys.stderr, flush=True)
        out["grad_256"] = run_grad256(max(3, args.steps // 10), 2)
        print("[bench] FFT passes against rocFFT", file=sys.stderr, flush=True)
        out["fft_vs_rocfft"] = fft_comparison(res)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle on a bounded sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
