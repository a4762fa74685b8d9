"""Size-class autotuner for the 2D cell solves: node rows per thread.

Each level of a plan solves cells of one width NC with the 2D solve kernel,
whose shape is the number of node rows a thread owns (the workgroup then has
NC^2 / rows threads). The library takes the shape from a static table and
from the environment override MCH_RPT_<NC>, read when a plan is created. This
tuner times, per cell width of a configuration, every shape the library
instantiates. It builds a plan with the override set, checks that the plan
took that shape, and times that width's solve launches with the library's own
kernel events (median over repetitions). `apply` sets the fastest shapes for
the plans created afterwards.

    python -m paper_2503_01276_amd.autotune --workload c2

Needs a GPU; PyTorch provides the device buffers.
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np

from . import mch
from . import workloads as W

CANDIDATES = (1, 2, 4, 8, 16)


def _env_name(nc: int) -> str:
    return f"MCH_RPT_{nc}"


def tune(cfg, kappa, label, reps: int = 3, candidates=CANDIDATES) -> dict:
    """{NC: {"best": rows, "ms": {rows: median ms of that width's solve launches per forward}}}."""
    import torch

    if cfg.dim != 2:
        raise ValueError("the size-class shapes are those of the 2D solve kernel")
    dev = torch.device("cuda:0")
    kd = torch.from_numpy(np.ascontiguousarray(kappa).reshape(-1).copy()).to(dev)
    ld = torch.from_numpy(np.ascontiguousarray(label).reshape(-1).copy()).to(dev)
    widths = sorted({cfg.n_cell // cfg.eta ** l for l in range(cfg.levels)}, reverse=True)
    saved = {nc: os.environ.get(_env_name(nc)) for nc in widths}
    out = {}
    try:
        for nc in widths:
            times = {}
            for rows in candidates:
                os.environ[_env_name(nc)] = str(rows)
                try:
                    plan = mch.Plan(cfg)
                except mch.MchError:
                    continue  # no kernel instantiated for this shape
                try:
                    levels = [l for l in range(cfg.levels) if cfg.n_cell // cfg.eta ** l == nc]
                    if any(plan.rows_per_thread[l] != rows for l in levels):
                        continue  # the library fell back to another valid shape
                    names = {f"solve_L{l + 1}" for l in levels if plan.level_counts[l] > 0}
                    plan.solve_cells(kd, ld)  # warm-up
                    torch.cuda.synchronize()
                    per = []
                    for _ in range(reps):
                        plan.profile(True)
                        plan.solve_cells(kd, ld)
                        torch.cuda.synchronize()
                        per.append(sum(ms for name, ms in plan.profile_records() if name in names))
                        plan.profile(False)
                    times[rows] = float(np.median(per))
                finally:
                    plan.close()
            if not times:
                raise RuntimeError(f"no instantiated shape for cell width {nc}")
            best = min(times, key=times.get)
            out[nc] = {"best": best, "ms": times}
            # later widths are timed with this width at its best shape
            os.environ[_env_name(nc)] = str(best)
    finally:
        for nc, v in saved.items():
            if v is None:
                os.environ.pop(_env_name(nc), None)
            else:
                os.environ[_env_name(nc)] = v
    return out


def apply(table: dict) -> None:
    """Use the tuned shapes for every plan created from now on in this process."""
    for nc, entry in table.items():
        os.environ[_env_name(int(nc))] = str(int(entry["best"]))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", default="c2", choices=sorted(W.PRESETS))
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    cfg = W.PRESETS[args.workload]
    kappa, label = W.medium(args.workload)
    table = tune(cfg, kappa, label, reps=args.reps)
    print(json.dumps({str(k): v for k, v in table.items()}))


if __name__ == "__main__":
    main()
