"""Helpers for the GPU tests: run the HIP path through the C ABI and compare with the oracle."""
from __future__ import annotations

import sys

import numpy as np


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_forward(cfg, kappa, label, cells=None):
    """Run mch_solve_cells + mch_effective_coeffs; return (plan, A[P,M,M], Phi dict, iters, resid, tensors)."""
    import torch

    from paper_2503_01276_amd import mch

    plan = mch.Plan(cfg)
    dev = torch.device("cuda:0")
    k = torch.from_numpy(np.ascontiguousarray(kappa).reshape(-1)).to(dev)
    lab = torch.from_numpy(np.ascontiguousarray(label).reshape(-1)).to(dev)
    plan.solve_cells(k, lab)
    A = torch.empty(plan.P * plan.M * plan.M, dtype=torch.float64, device=dev)
    plan.effective_coeffs(k, A)
    torch.cuda.synchronize()
    it, rs = plan.diagnostics()
    Phi = {}
    if cells is not None and len(cells):
        nn = (cfg.n_cell + 1) ** cfg.dim
        out = torch.empty(len(cells) * plan.M * nn, dtype=torch.float64, device=dev)
        plan.local_solutions(np.asarray(cells), out)
        torch.cuda.synchronize()
        o = out.cpu().numpy().reshape(len(cells), plan.M, nn)
        for i, p in enumerate(cells):
            Phi[int(p)] = o[i].T  # [nn, M] like the oracle
    return plan, A.cpu().numpy().reshape(plan.P, plan.M, plan.M), Phi, it, rs, (k, lab)


def phi_rel_err(gpu: np.ndarray, ref: np.ndarray) -> float:
    """max over right-hand sides of ||gpu - ref||_2 / ||ref||_2 over the cell's nodes."""
    num = np.linalg.norm(gpu - ref, axis=0)
    den = np.maximum(np.linalg.norm(ref, axis=0), 1e-300)
    return float((num / den).max())


def A_rel_err(gpu: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """per macropoint ||gpu - ref||_F / ||ref||_F."""
    num = np.linalg.norm((gpu - ref).reshape(len(ref), -1), axis=1)
    den = np.linalg.norm(ref.reshape(len(ref), -1), axis=1)
    return num / den
