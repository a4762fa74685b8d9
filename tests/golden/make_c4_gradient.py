"""Write the oracle's adjoint-workload gradient on a seeded sample of elements.

Workload: the hierarchical L=3 preset on the 512^2 grid (channel medium,
seed 2); loss sum_p ||A_eff(p) - A_target(p)||_F^2 with A_target from the same
medium whose channel value carries the lognormal(0, 0.3) factor of seed 4.
Output: c4_gradient_sample.txt with dLoss/dlog(kappa) at 4096 elements drawn
without replacement by numpy default_rng(444), plus the 20 finite-difference
elements (10 channel + 10 matrix, default_rng(44)). Calls only the oracle.

Usage: python tests/golden/make_c4_gradient.py [workers]
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2503_01276_amd import workloads as W  # noqa: E402


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    cfg = W.PRESETS["c2"]
    k, l = W.medium("c2")
    kt, _ = W.medium("c2", channel_factor=W.target_factor(4))
    T = oracle.stack_A(oracle.forward(cfg, kt, l, workers=workers), cfg)
    fwd = oracle.forward(cfg, k, l, workers=workers)
    A = oracle.stack_A(fwd, cfg)
    gA = {p: 2.0 * (A[p] - T[p]) for p in range(cfg.n_points)}
    g = oracle.backward(cfg, k, l, fwd, gA, workers=workers).reshape(-1)
    idx = np.sort(np.random.default_rng(444).choice(g.size, 4096, replace=False))
    fd = W.fd_elements(l, seed=44, n_each=10)
    sel = np.unique(np.concatenate([idx, fd]))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_gradient_sample.txt")
    with open(out, "w") as fh:
        fh.write("# Oracle dLoss/dlog(kappa) for the adjoint workload on the hierarchical L=3 preset\n")
        fh.write("# (512^2 grid, 32x32 macropoints, 64^2 cells; loss sum_p ||A_eff - A_target||_F^2),\n")
        fh.write("# written by tests/golden/make_c4_gradient.py from the oracle only.\n")
        fh.write(f"# loss {float(np.sum((A - T) ** 2)):.17e} grad_norm {float(np.linalg.norm(g)):.17e}\n")
        for e in sel:
            fh.write(f"{int(e)} {g[e]:.17e}\n")
    print(out, len(sel))


if __name__ == "__main__":
    main()
