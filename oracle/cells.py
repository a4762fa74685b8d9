"""Oracle, part 3: one constrained cell problem, solved by an assembled sparse direct method.

TEST INFRASTRUCTURE ONLY.

For a macropoint of level n (paper Sec. 3.3, Eqs. phi_avar_corrector and
phi_grad_corrector; level 1 is Eqs. phi_avar / phi_grad with I = 0):

    [ K_n   B_n^T ] [ xi   ]   [ -P_n^T K_h I ]
    [ B_n   0     ] [ beta ] = [  g - B_h I   ],    Phi = I + P_n xi,

with K_n = P_n^T K_h P_n and B_n = B_h P_n (V_n is a subspace of V_h, so the
Galerkin restriction is the exact form of the problem posed in V_n), K_h the
fine stiffness with kappa of this cell, B_h the fine constraint rows, g the
constraint right-hand sides, and I the inherited fine solution (the type-2
right-hand side uses phi^m_{i,t}; the paper's printed phi_{i,t} there is a typo).

Boundary conditions on the cell: homogeneous Dirichlet (bc = 0, the
configured workloads) or natural Neumann conditions (bc = 1, every node free;
K_n is then singular on constants, and the KKT matrix stays regular because
the constraint rows do not vanish on constants).

The KKT matrix is factored with SciPy's SuperLU and every solve takes one step
of iterative refinement. The effective tensor (Eq. Bs_defi, with R_p = K_p so
|K_p|/|R_p| = 1) is A_{ab} = Phi_a^T K_h^{K_p} Phi_b, the K_p-restricted
stiffness Gram matrix of the M local solutions.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem


@dataclasses.dataclass
class CellSystem:
    """Everything the oracle assembles for one cell on one level."""

    Kf: sp.csr_matrix      # fine stiffness on free nodes
    Bf: np.ndarray         # fine constraint rows on free nodes [m, n_free]
    g: np.ndarray          # [m, M]
    P: sp.csr_matrix       # free fine <- free coarse
    Kn: sp.csr_matrix
    Bn: np.ndarray
    lu: object
    free: np.ndarray
    n_nodes: int
    Kkp: sp.csr_matrix     # K_p-restricted fine stiffness over all nodes
    kc: np.ndarray
    lc: np.ndarray


def cell_origin(cfg, p: int):
    """Lower corner (fine elements, per axis x1 first) of macropoint p's cell."""
    nm = cfg.n_macro
    j = [(p // nm ** k) % nm for k in range(cfg.dim)]
    return [cfg.H_el * jj + cfg.H_el // 2 - cfg.n_cell // 2 for jj in j]


def assemble_cell(cfg, kappa, label, p: int, level: int) -> CellSystem:
    dim, nc, h = cfg.dim, cfg.n_cell, cfg.h
    org = cell_origin(cfg, p)
    kc = fem.window(kappa, org, nc)
    lc = fem.window(label, org, nc)
    K = fem.assemble_stiffness(kc, h)
    B, g, _ = fem.constraints(lc, cfg.n_sub, cfg.n_cont, cfg.H_el, h)
    free = fem.free_nodes(nc, dim, cfg.bc)
    Kf = K[free][:, free].tocsr()
    Bf = B[:, free]
    r = cfg.eta ** (level - 1)
    Pfull = fem.prolongation(nc, r, dim)
    cfree = fem.free_nodes(nc // r, dim, cfg.bc)
    P = Pfull[free][:, cfree].tocsr()
    Kn = (P.T @ Kf @ P).tocsr()
    Bn = np.asarray(Bf @ P)  # dense [m, n_coarse_free]
    kkt = sp.bmat([[Kn, sp.csr_matrix(Bn).T], [sp.csr_matrix(Bn), None]], format="csc")
    lu = spla.splu(kkt)
    kpm = fem.kp_element_mask(nc, cfg.H_el, dim)
    Kkp = fem.assemble_stiffness(kc, h, elem_mask=kpm)
    return CellSystem(Kf=Kf, Bf=Bf, g=g, P=P, Kn=Kn, Bn=Bn, lu=lu, free=free,
                      n_nodes=(nc + 1) ** dim, Kkp=Kkp, kc=kc, lc=lc)


def kkt_solve(cs: CellSystem, rhs_top: np.ndarray, rhs_bot: np.ndarray):
    """Solve the KKT system for many right-hand sides with one refinement step."""
    n = cs.Kn.shape[0]
    kkt = sp.bmat([[cs.Kn, sp.csr_matrix(cs.Bn).T], [sp.csr_matrix(cs.Bn), None]], format="csr")
    rhs = np.concatenate([rhs_top, rhs_bot], axis=0)
    sol = cs.lu.solve(rhs)
    res = rhs - kkt @ sol
    sol = sol + cs.lu.solve(res)
    return sol[:n], sol[n:]


def solve_cell(cs: CellSystem, I_full: np.ndarray | None, M: int):
    """Return (Phi [n_nodes, M] over all cell nodes, xi [n_coarse_free, M], beta [m, M])."""
    nf = len(cs.free)
    if I_full is None:
        If = np.zeros((nf, M))
    else:
        If = I_full[cs.free]
    top = -(cs.P.T @ (cs.Kf @ If))
    bot = cs.g - cs.Bf @ If
    xi, beta = kkt_solve(cs, top, bot)
    Phi = np.zeros((cs.n_nodes, M), dtype=np.result_type(xi, If))
    Phi[cs.free] = If + cs.P @ xi
    return Phi, xi, beta


def effective_tensor(cs: CellSystem, Phi: np.ndarray) -> np.ndarray:
    return Phi.T @ (cs.Kkp @ Phi)
