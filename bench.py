"""Benchmark: hierarchical multicontinuum cell solves on one MI355X.

One step = the whole hot path on one batch: every constrained cell problem
(mch_solve_cells), the effective tensors (mch_effective_coeffs) and their
adjoint gradient with respect to log kappa (mch_effective_coeffs_backward)
for the loss sum_p ||A_eff(p) - A_target(p)||_F^2. Inputs are seeded
synthetic media already resident in HBM. Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from paper_2503_01276_amd import workloads as W  # noqa: E402

FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector
HBM_PEAK_GBS = 8000.0
# floor of the element-wise gradient check, relative to the field's largest entry
GRAD_FLOOR = 1e-3
# Algorithmic FP64 flops of one projected-PCG iteration per free node of a 2D
# cell, as the hot-path accounting states them: the matrix-free Q1 stencil
# apply 36, the PCG vector operations 11, the constraint projection 16.
FLOPS_PER_NODE_ITER = 63
# 3D, same accounting: the fine operator row has 21 points (self, 12 face
# diagonals, 8 body diagonals; edge neighbours do not couple) -> 42, a Galerkin
# level row 27 -> 54; the other terms as in 2D (20).
FLOPS_PER_NODE_ITER_3D_FINE = 62
FLOPS_PER_NODE_ITER_3D_GAL = 74

# HBM traffic per launch of the dominant kernel, from two rocprofv3 --pmc runs of
# this script (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch), each scaled by what
# the same counter reads for a plain device copy of known size (--copy-probe).
# An entry holds only while the kernel sources hash to the recorded value.
# Sources of the kernels whose counters are recorded below, per dimension.
KERNEL_SOURCES = {
    2: ("paper_2503_01276_amd/csrc/solve2d_kernel.h", "paper_2503_01276_amd/csrc/solve2d_inst.hip",
        "paper_2503_01276_amd/csrc/kernels2d.h", "paper_2503_01276_amd/csrc/device_common.h"),
    3: ("paper_2503_01276_amd/csrc/cells3d.hip", "paper_2503_01276_amd/csrc/device_common.h"),
}
# HBM bytes per launch of a workload's dominant kernel: FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch, averaged over the kernel's dispatches) from two
# rocprofv3 --pmc runs, each scaled by the ratio of a plain copy's known size
# to what the same counter reads for it. An entry holds only while the kernel
# sources hash to the recorded value; otherwise traffic is reported as null.
_SHA_2D = "20e92547a39d54f9f1b450021a59c07bb7c978199c29dd0e41896f18c75ee764"
_SHA_3D = "3a5c6d28d2e609d6d0cd1faaff50a32235d5b19661ca27678dca3f6d5c42be57"
_COPY_SCALE = {"fetch": 1048576.0 / 524304.79, "write": 1048576.0 / 1048576.0}  # 1 GiB copy
TRAFFIC = {
    # level-2 (32^2 Galerkin) forward solve: two launches per step (756 and 396
    # workgroups), counters averaged over both
    ("c2", "solve_L2"): {"sha256": _SHA_2D, "fetch_kib": 9080.5, "write_kib": 4916.1,
                         "fetch_scale": _COPY_SCALE["fetch"], "write_scale": _COPY_SCALE["write"]},
    ("c2", "adjsolve_L2"): {"sha256": _SHA_2D, "fetch_kib": 12170.0, "write_kib": 9830.1,
                            "fetch_scale": _COPY_SCALE["fetch"], "write_scale": _COPY_SCALE["write"]},
    # level-1 (64^2, band coarse correction) forward chunks (252 and 132
    # workgroups) averaged, and the single adjoint launch (384)
    ("c2", "solve_L1"): {"sha256": _SHA_2D, "fetch_kib": 1751.3, "write_kib": 10136.0,
                         "fetch_scale": _COPY_SCALE["fetch"], "write_scale": _COPY_SCALE["write"]},
    ("c2", "adjsolve_L1"): {"sha256": _SHA_2D, "fetch_kib": 8855.5, "write_kib": 18228.1,
                            "fetch_scale": _COPY_SCALE["fetch"], "write_scale": _COPY_SCALE["write"]},
    # 2048^2 batch, level 1 (64^2 cells, two sub-bands): forward and adjoint
    # launches share kernel and grid; the counters are the mean over both
    ("c5", "solve_L1"): {"sha256": _SHA_2D, "fetch_kib": 283922.0, "write_kib": 9298468.2,
                         "fetch_scale": _COPY_SCALE["fetch"], "write_scale": _COPY_SCALE["write"]},
    # 3D fine level: forward and adjoint launches share kernel and grid; the
    # counters are the mean over both, so either may be the dominant launch
    ("c3", "solve_L1"): {"sha256": _SHA_3D, "fetch_kib": 76635078.4, "write_kib": 81523225.1,
                         "fetch_scale": _COPY_SCALE["fetch"], "write_scale": _COPY_SCALE["write"]},
}
TRAFFIC[("c3", "adjsolve_L1")] = TRAFFIC[("c3", "solve_L1")]
TRAFFIC[("c5", "adjsolve_L1")] = TRAFFIC[("c5", "solve_L1")]


def kernel_sources_sha256(dim: int) -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES[dim]:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, kernel: str):
    t = TRAFFIC.get((workload, kernel))
    if t is None or t["sha256"] != kernel_sources_sha256(W.PRESETS[workload].dim):
        return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0


def copy_probe(mib: int, reps: int = 3):
    """A plain device-to-device copy of a known size, for scaling the traffic counters."""
    import torch

    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "reps": reps}))


DESCR = {
    "c2": "hierarchical L=3 eta=2, 2D 512^2 fine grid, 32x32 macropoints, 64^2-element cells "
          "(levels 64^2/32^2/16^2), N=2, contrast 1e4",
    "c2ml": "hierarchical L=3 eta=2 with multilinear inheritance from T_(n-1), 2D 512^2 fine grid, "
            "32x32 macropoints, 64^2-element cells (levels 64^2/32^2/16^2), N=2, contrast 1e4",
    "c2flat": "flat L=1, 2D 512^2 fine grid, 32x32 macropoints, 64^2-element cells, N=2, contrast 1e4",
    "c1": "flat L=1, 2D 128^2 fine grid, 8x8 macropoints, 32^2-element cells, N=2, contrast 1e4",
    "c5": "hierarchical L=4 eta=2, 2D 2048^2 fine grid, 256x256 macropoints, 64^2-element cells "
          "(levels 64^2/32^2/16^2/8^2), N=3 with inclusions, contrast 1e8",
    "c5ml": "hierarchical L=4 eta=2 with multilinear inheritance from T_(n-1), 2D 2048^2 fine grid, "
            "256x256 macropoints, 64^2-element cells (levels 64^2/32^2/16^2/8^2), N=3 with inclusions, contrast 1e8",
    "c3": "hierarchical L=2 eta=2, 3D 128^3 fine grid, 8^3 macropoints, 32^3-element cells "
          "(levels 32^3/16^3), N=2, contrast 1e4",
    "c3flat": "flat L=1, 3D 128^3 fine grid, 8^3 macropoints, 32^3-element cells, N=2, contrast 1e4",
    "c6": "hierarchical L=3 eta=2, 2D 512^2 fine grid, 16x16 macropoints, 128^2-element cells "
          "(levels 128^2/64^2/32^2, 4x4 constraint sub-blocks), N=2, contrast 1e4",
    "c7": "hierarchical L=3 eta=2, 2D 512^2 fine grid, 16x16 macropoints, block-aligned cells of 3x3 coarse "
          "blocks (96^2 elements; levels 96^2/48^2/24^2; constraint regions = the blocks), N=2, contrast 1e4",
}


def cpu_baseline(name: str, workers: int):
    """Time the oracle (as it stands) on the host cores; runs before any GPU use."""
    import oracle

    cfg = W.PRESETS[name]
    k, l = W.medium(name)
    if cfg.n_points > 4096 or cfg.dim == 3:
        # bounded sample: every cell of two level-1 groups, forward only
        lev = oracle.hierarchy.levels(cfg.n_macro, cfg.dim, cfg.levels, cfg.eta)
        par = oracle.hierarchy.parents(cfg.n_macro, cfg.dim, cfg.levels, cfg.eta)
        l1 = np.flatnonzero(lev == 1)
        groups = [int(l1[0])] if cfg.dim == 3 else [int(l1[0]), int(l1[len(l1) // 2])]
        pts = sorted(set(groups) | set(int(p) for p in np.flatnonzero(np.isin(par, groups))))
        t0 = time.perf_counter()
        oracle.forward(cfg, k, l, points=pts, workers=workers)
        t1 = time.perf_counter()
        solves = len(pts) * cfg.n_rhs
        return {"value": solves / (t1 - t0), "unit": "cell-solves/s", "cores": workers, "kind": "oracle",
                "sample": f"{len(pts)} cells of {len(groups)} whole level-1 group(s) of {name} ({solves} solves), "
                          f"SciPy SuperLU forward only, {t1 - t0:.2f} s, one process per core"}, None
    kt, _ = W.medium(name, channel_factor=W.target_factor(4))
    T = oracle.stack_A(oracle.forward(cfg, kt, l, workers=workers), cfg)
    t0 = time.perf_counter()
    fwd = oracle.forward(cfg, k, l, workers=workers)
    A = oracle.stack_A(fwd, cfg)
    t1 = time.perf_counter()
    gA = {p: 2.0 * (A[p] - T[p]) for p in range(cfg.n_points)}
    g = oracle.backward(cfg, k, l, fwd, gA, workers=workers)
    t2 = time.perf_counter()
    solves = cfg.n_points * cfg.n_rhs
    return {
        "value": solves / (t2 - t0),
        "unit": "cell-solves/s",
        "cores": workers,
        "kind": "oracle",
        "sample": f"full {name} workload ({solves} solves): SciPy SuperLU forward {t1 - t0:.2f} s + "
                  f"adjoint {t2 - t1:.2f} s, one process per core",
    }, {"A": A, "g": g, "T": T}


class Runner:
    instances = []

    def __init__(self, name: str, target=None):
        """target: A_target [P, M, M] of the loss (host array), or None to form it
        with the GPU path on the target medium (outside the timed region)."""
        import torch

        from paper_2503_01276_amd import mch

        Runner.instances.append(self)
        self.torch = torch
        self.stream = torch.cuda.Stream()  # non-default stream: launch sequences are captured as hipGraphs
        self.cfg = W.PRESETS[name]
        self.plan = mch.Plan(self.cfg)
        dev = torch.device("cuda:0")
        k, l = W.medium(name)
        kt, _ = W.medium(name, channel_factor=W.target_factor(4))
        self.k = torch.from_numpy(k.reshape(-1).copy()).to(dev)
        self.l = torch.from_numpy(l.reshape(-1).copy()).to(dev)
        P, M = self.plan.P, self.plan.M
        self.A = torch.empty(P * M * M, dtype=torch.float64, device=dev)
        self.gA = torch.empty_like(self.A)
        self.g = torch.empty_like(self.k)
        if target is not None:
            # the oracle's target tensors (an input of the loss)
            self.T = torch.from_numpy(np.ascontiguousarray(target).reshape(-1)).to(dev)
        else:
            # target tensors: same path on the perturbed medium (outside timing)
            kt_d = torch.from_numpy(kt.reshape(-1).copy()).to(dev)
            self.plan.solve_cells(kt_d, self.l)
            self.T = torch.empty_like(self.A)
            self.plan.effective_coeffs(kt_d, self.T)
        torch.cuda.synchronize()

    def step(self, ev=None):
        """One pass of the hot path; ev = four events recorded between the phases (or None)."""
        if ev:
            ev[0].record()
        self.plan.solve_cells(self.k, self.l)
        if ev:
            ev[1].record()
        self.plan.effective_coeffs(self.k, self.A)
        if ev:
            ev[2].record()
        self.torch.sub(self.A, self.T, out=self.gA)
        self.gA.mul_(2.0)
        self.plan.effective_coeffs_backward(self.k, self.gA, self.g)
        if ev:
            ev[3].record()

    def time_steps(self, steps: int, warmup: int, profile: bool):
        torch = self.torch
        with torch.cuda.stream(self.stream):
            return self._time_steps(steps, warmup, profile)

    def _time_steps(self, steps: int, warmup: int, profile: bool):
        torch = self.torch
        self.plan.profile(profile)
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        self.plan.profile(profile)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        # per-phase events on the launch stream (the library forks and joins its level
        # streams inside each call, so these bracket each call's whole span)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)] if profile else None
        # step boundaries (the median step time of the replayed graphs is reported too)
        sevs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)] if not profile else None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        for i in range(steps):
            if sevs:
                sevs[i].record()
            self.step(evs[i] if evs else None)
        if sevs:
            sevs[steps].record()
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1) / steps
        phases = None
        if evs:
            ph = np.array([[e[j].elapsed_time(e[j + 1]) for j in range(3)] for e in evs])
            phases = {"solve_ms": float(ph[:, 0].mean()), "eff_ms": float(ph[:, 1].mean()),
                      "grad_ms_incl_loss": float(ph[:, 2].mean()),
                      "solve_ms_median": float(np.median(ph[:, 0])), "eff_ms_median": float(np.median(ph[:, 1])),
                      "grad_ms_incl_loss_median": float(np.median(ph[:, 2]))}
        if sevs:
            phases = {"ms_per_step_median": float(np.median([sevs[i].elapsed_time(sevs[i + 1])
                                                              for i in range(steps)]))}
        recs = self.plan.profile_records() if profile else []
        self.plan.profile(False)
        return ms, wall, recs, phases


def macro_measure(runner, reps: int = 3):
    """Time the macroscopic system (block loads + assembly + CG) on the runner's
    last forward and tensors; returns the timings and the block averages."""
    torch = runner.torch
    cfg, plan = runner.cfg, runner.plan
    N, nm, dev = cfg.n_cont, cfg.n_macro, runner.k.device
    lab = runner.l.cpu().numpy().reshape((cfg.n_fine,) * cfg.dim)
    f = torch.from_numpy(W.source_from_labels(lab).reshape(-1).copy()).to(dev)
    b = torch.empty(plan.P * N, dtype=torch.float64, device=dev)
    U = torch.empty((nm + 1) ** cfg.dim * N, dtype=torch.float64, device=dev)
    Ub = torch.empty(plan.P * N, dtype=torch.float64, device=dev)
    with torch.cuda.stream(runner.stream):
        plan.macro_load(f, b)
        plan.macro_solve(runner.A, b, U, Ub, rtol=1e-12, max_iter=50000)  # allocates the scratch
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.macro_load(f, b)
            plan.macro_solve(runner.A, b, U, Ub, rtol=1e-12, max_iter=50000)
        e1.record()
        torch.cuda.synchronize()
    it, rs = plan.macro_diagnostics()
    return {"ms": e0.elapsed_time(e1) / reps, "cg_iterations": it, "relative_residual": rs,
            "unknowns": (nm - 1) ** cfg.dim * N}, Ub.cpu().numpy().reshape(-1, N)


def kernel_table(recs, steps):
    tab = {}
    for name, ms in recs:
        t = tab.setdefault(name, [0.0, 0])
        t[0] += ms
        t[1] += 1
    return {k: {"avg_ms": v[0] / v[1], "launches_per_step": v[1] / steps} for k, v in tab.items()}


def free_nodes(cfg, NC: int) -> int:
    """Free nodes of a level cell NC elements wide (Dirichlet: interior; Neumann: all)."""
    return (NC + 1 if cfg.bc else NC - 1) ** cfg.dim


def solve_flops(runner, level_idx: int, iters: np.ndarray, levels: np.ndarray, adjoint: bool = False):
    cfg = runner.cfg
    r = cfg.eta ** level_idx
    NC = cfg.n_cell // r
    nfree = free_nodes(cfg, NC)
    m = runner.plan.m
    its = iters[levels == level_idx + 1].astype(np.float64)
    per_node = FLOPS_PER_NODE_ITER if cfg.dim == 2 else (FLOPS_PER_NODE_ITER_3D_FINE if r == 1 else FLOPS_PER_NODE_ITER_3D_GAL)
    return float(its.sum()) * (per_node * nfree + 2 * m * m + 2 * m)


# Algorithmic bytes of one iteration per free node of the 3D fine-level solve,
# whose Krylov vectors live in HBM: the stencil sweep reads p, r and D^-1 and
# writes K p; the update sweep reads K p, D^-1, x, r, p and writes x, r, p
# (12 FP64 values); the element window adds kappa h/12 and a label byte per
# element (one element per node) in the stencil sweep and the label byte again
# in the update sweep. Neighbour values of p are counted once (they are reused
# from registers); the re-projection sweep every 16 iterations is left out.
BYTES_PER_NODE_ITER_3D = 12 * 8 + 10


# The generic 2D solve kernel keeps its Krylov vectors in device memory too:
# the same 12 FP64 vector values per free node and iteration; on the fine
# level kappa (8 B) and a label byte in each of the two sweeps, on a Galerkin
# level the node's 9 stencil weights (72 B) and its 4 N binary32 constraint
# weights in each sweep.
def bytes_per_node_iter_2d_generic(galerkin: bool, n_cont: int) -> int:
    return 12 * 8 + ((9 * 8 + 2 * 16 * n_cont) if galerkin else (8 + 2))


def solve_bytes(runner, level_idx: int, iters: np.ndarray, levels: np.ndarray):
    cfg = runner.cfg
    NC = cfg.n_cell // cfg.eta ** level_idx
    nfree = free_nodes(cfg, NC)
    its = iters[levels == level_idx + 1].astype(np.float64)
    per = BYTES_PER_NODE_ITER_3D if cfg.dim == 3 else bytes_per_node_iter_2d_generic(level_idx > 0, cfg.n_cont)
    return float(its.sum()) * per * nfree


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(DESCR))
    ap.add_argument("--flat", default=None, help="flat workload for the speedup (default: c2flat for c2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tuned", action="store_true",
                    help="use the library's default kernel knobs instead of the stored tuned ones")
    ap.add_argument("--cpu-workers", type=int, default=None)
    ap.add_argument("--copy-probe", type=int, default=None, metavar="MIB",
                    help="only run a plain copy of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the path shards by independent groups of macropoints, but only one GPU is driven here)",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return

    cpu, oracle_ref = None, None
    if not args.no_cpu_baseline:
        # one process per core of the CPU share this process may use (a GPU
        # host gives one GPU's jobs 16 cores, whatever the machine has)
        avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        workers = args.cpu_workers or min(16, avail)
        cpu, oracle_ref = cpu_baseline(args.workload, workers)
        cpu["host_cpus"] = os.cpu_count()
        cpu["affinity_cpus"] = avail
        print(f"[bench] cpu baseline: {cpu['value']:.1f} solves/s on {workers} cores", file=sys.stderr, flush=True)

    tuned = {}
    if not args.no_tuned:
        from paper_2503_01276_amd import autotune

        for w in {args.workload, args.flat or {"c2": "c2flat", "c2ml": "c2flat", "c3": "c3flat"}.get(args.workload)}:
            if w and w != "none" and autotune.load(w):
                tuned[w] = autotune.load(w)
    if args.workload in tuned:
        from paper_2503_01276_amd import autotune

        autotune.apply(tuned[args.workload])
    run = Runner(args.workload, target=None if oracle_ref is None else oracle_ref["T"])
    try:
        out = measure(args, run, cpu, oracle_ref, tuned)
    finally:
        # release every plan before the interpreter (and torch) shut down
        for r in Runner.instances:
            r.plan.close()
    print(json.dumps(out))


def _knobs(table):
    if not table:
        return None
    return {"rows_per_thread": {k: v["best"] for k, v in table.get("rows", {}).items()},
            "band_correction": {k: v["best"] for k, v in table.get("prec", {}).items()},
            "level1_split": table.get("split", {}).get("best")}


def measure(args, run, cpu, oracle_ref, tuned):
    cfg, plan = run.cfg, run.plan
    ms, wall, recs, phases = run.time_steps(args.steps, args.warmup, profile=True)
    print(f"[bench] {args.workload}: {ms:.3f} ms/step (eager, per-kernel events)", file=sys.stderr, flush=True)
    ms_graph, _, _, gph = run.time_steps(args.steps, 1, profile=False)
    print(f"[bench] {args.workload}: {ms_graph:.3f} ms/step (hipGraph replay)", file=sys.stderr, flush=True)
    ktab = kernel_table(recs, args.steps)
    iters, _ = plan.diagnostics()
    aiters, _ = plan.diagnostics(adjoint=True)
    lev, _ = plan.hierarchy()
    lev_pm = np.repeat(lev[:, None], plan.M, axis=1)
    # dominant kernel (the solve launches, whose roofline the flop and byte
    # models describe; the auxiliary kernels' event times include the time they
    # share the GPU with concurrent solves) and its algorithmic work per launch
    solve_kernels = [k for k in ktab if k.startswith(("solve_L", "adjsolve_L"))]
    dom = max(solve_kernels or ktab, key=lambda k: ktab[k]["avg_ms"] * ktab[k]["launches_per_step"])
    roof = None
    if dom.startswith(("solve_L", "adjsolve_L")):
        li = int(dom.split("_L")[1]) - 1
        # a level may run as several launches (chunks); per launch = per step / launches
        nl = ktab[dom]["launches_per_step"]
        its = aiters if dom.startswith("adj") else iters
        if (cfg.dim == 3 and li == 0) or (cfg.dim == 2 and plan.rows_per_thread[li] == 0):
            # the 3D fine level and the generic 2D kernel stream their Krylov
            # vectors through device memory: HBM roofline
            nbytes = solve_bytes(run, li, its, lev_pm) / nl
            achieved = nbytes / (ktab[dom]["avg_ms"] * 1e-3) / 1e9
            roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                    "traffic": measured_traffic(args.workload, dom), "bytes_per_launch": nbytes,
                    "launches_per_step": nl}
        else:
            flops = solve_flops(run, li, its, lev_pm) / nl
            achieved = flops / (ktab[dom]["avg_ms"] * 1e-3) / 1e12
            roof = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                    "traffic": measured_traffic(args.workload, dom), "flops_per_launch": flops,
                    "launches_per_step": nl}
    if roof is not None and roof.get("traffic"):
        # measured HBM bytes per launch over the launch's live average duration
        roof["traffic_gbs"] = roof["traffic"] / (ktab[dom]["avg_ms"] * 1e-3) / 1e9
    solves = plan.P * plan.M
    fwd_ms = phases["solve_ms"]

    def free_dof(n):  # free nodes of a level-(n+1) cell
        return free_nodes(cfg, cfg.n_cell // cfg.eta ** n)
    detail = {
        **phases,
        "eff_tensor_time_ms": phases["solve_ms"] + phases["eff_ms"],
        "solves_per_s_forward_only": solves / (fwd_ms * 1e-3),
        "iterations": {f"L{n}": [int(iters[lev == n].min()), float(np.median(iters[lev == n])),
                                 int(iters[lev == n].max())] for n in range(1, cfg.levels + 1)},
        "adjoint_iterations": {f"L{n}": [int(aiters[lev == n].min()), float(np.median(aiters[lev == n])),
                                         int(aiters[lev == n].max())] for n in range(1, cfg.levels + 1)},
        "kernels": ktab,
        "wall_s": wall,
        "ms_per_step_graph_replay": ms_graph,
        "ms_per_step_graph_replay_median": gph["ms_per_step_median"],
        # degrees of freedom of all solves, hierarchical / flat (Sec. 3.4 models
        # this as L eta^((1-L) d))
        "dof_model": {"paper_model": cfg.levels * float(cfg.eta) ** ((1 - cfg.levels) * cfg.dim),
                      "dof_ratio": sum(int((lev == n + 1).sum()) * free_dof(n) for n in range(cfg.levels)) /
                                   (plan.P * free_dof(0))},
    }
    if oracle_ref is not None:
        # the timed run's own outputs (same inputs every step) against the
        # oracle's on the full workload: per-point relative Frobenius error of
        # A_eff (worst point) and relative 2-norm error of dLoss/dlog kappa
        P, M = plan.P, plan.M
        Ag = run.A.cpu().numpy().reshape(P, M, M)
        gg = run.g.cpu().numpy()
        Ar = oracle_ref["A"]
        eA = float(max(np.linalg.norm(Ag[p] - Ar[p]) / np.linalg.norm(Ar[p]) for p in range(P)))
        gr = np.asarray(oracle_ref["g"]).reshape(-1)  # x1 fastest, as the device field
        eg = float(np.linalg.norm(gg - gr) / np.linalg.norm(gr))
        # element-wise: |dg_e| / max(|g_e|, GRAD_FLOOR max|g|), and per continuum
        dg = np.abs(gg - gr)
        ee = float((dg / np.maximum(np.abs(gr), GRAD_FLOOR * np.abs(gr).max())).max())
        labs = run.l.cpu().numpy()
        ej = {str(j): float(np.linalg.norm((gg - gr)[labs == j]) / np.linalg.norm(gr[labs == j]))
              for j in np.unique(labs)}
        detail["rel_err_vs_oracle"] = {"A_eff_worst_point": eA, "grad_log_kappa": eg,
                                       "grad_log_kappa_worst_element": ee, "grad_floor": GRAD_FLOOR,
                                       "grad_log_kappa_per_continuum": ej}
        print(f"[bench] relative error against the oracle: A_eff {eA:.2e} (worst point), gradient {eg:.2e} "
              f"(worst element {ee:.2e} at floor {GRAD_FLOOR:g}; per continuum {ej})", file=sys.stderr, flush=True)
    flat = args.flat or {"c2": "c2flat", "c2ml": "c2flat", "c3": "c3flat"}.get(args.workload)
    if flat == "none":
        flat = None
    if flat:
        if flat in tuned:
            from paper_2503_01276_amd import autotune

            autotune.apply(tuned[flat])
        frun = Runner(flat)
        fms, _, _, fph = frun.time_steps(max(3, args.steps // 4), 1, profile=True)
        detail["flat"] = {"workload": flat, "ms_per_step": fms, **fph,
                          "speedup_step": fms / ms, "speedup_solve": fph["solve_ms"] / fwd_ms,
                          "speedup_eff_tensor_time": (fph["solve_ms"] + fph["eff_ms"]) /
                                                     (phases["solve_ms"] + phases["eff_ms"])}
        if frun.cfg.levels == 1 and frun.cfg.n_cell == cfg.n_cell:
            # forward work weighted by the measured iterations, hierarchical / flat
            fits, _ = frun.plan.diagnostics()
            work_flat = float(fits.astype(np.float64).sum()) * free_dof(0)
            work_h = sum(float(iters[lev == n + 1].astype(np.float64).sum()) * free_dof(n) for n in range(cfg.levels))
            detail["dof_model"]["work_ratio_iterations"] = work_h / work_flat
            detail["dof_model"]["time_ratio_solve"] = fwd_ms / fph["solve_ms"]
        print(f"[bench] {flat}: {fms:.3f} ms/step", file=sys.stderr, flush=True)
        if frun.cfg.dim == cfg.dim and frun.cfg.n_macro == cfg.n_macro:
            # the macroscopic system from both sets of tensors, and the paper's
            # Type-3 error (hierarchical against flat block averages, per continuum)
            mh, ubh = macro_measure(run)
            mf, ubf = macro_measure(frun)
            e3 = np.sqrt(((ubf - ubh) ** 2).sum(axis=0) / (ubf ** 2).sum(axis=0))
            detail["macro"] = {"hierarchical": mh, "flat": mf, "type3_error": e3.tolist()}
            print(f"[bench] macroscopic system: {mh['ms']:.3f} ms, {mh['cg_iterations']} CG iterations; "
                  f"Type-3 error {e3}", file=sys.stderr, flush=True)
    if "macro" not in detail and cfg.n_macro >= 2:
        # no flat run on the same blocks: the macroscopic system from the
        # hierarchical tensors alone
        mh, _ = macro_measure(run, reps=1)
        detail["macro"] = {"hierarchical": mh}
        print(f"[bench] macroscopic system: {mh['ms']:.3f} ms, {mh['cg_iterations']} CG iterations",
              file=sys.stderr, flush=True)
    detail["tuned_knobs"] = {w: _knobs(t) for w, t in tuned.items()} or None
    detail["band_subbands_per_level"] = list(plan.band_subbands)
    out = {
        "metric": "cell-solves/sec & eff-tensor+grad time, hier L=3 vs flat, 1 GPU, rel err <=1e-8",
        "value": solves / (ms * 1e-3),
        "unit": "cell-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": DESCR[args.workload], "preset": args.workload, "macropoints": plan.P,
                   "rhs_per_macropoint": plan.M, "solves_per_step": solves, "levels": cfg.levels,
                   "eta": cfg.eta, "n_fine": cfg.n_fine, "n_cell": cfg.n_cell, "rtol": cfg.rtol},
        "roofline": roof,
        "cpu_baseline": cpu,
        "detail": detail,
    }
    return out


if __name__ == "__main__":
    main()
