"""Oracle, part 5: the upscaled multicontinuum system (Sec. 2, Eq. macro_eq; the last step of Algorithm 1).

TEST INFRASTRUCTURE ONLY.

The macroscopic unknowns U_i (one per continuum) satisfy, in weak form
(Sec. 2, the identity above Eq. macro_eq, summed over the coarse blocks K_p),

    sum_p [ B_ji U_i V_j + B^m_ji d_m U_i V_j + Bbar^n_ji U_i d_n V_j
            + B^mn_ji d_m U_i d_n V_j ] = sum_p b_j V_j,

with the coefficients of Eq. Bs_defi, i.e. the blocks of A_eff(p): for
w = (U_0 .. U_{N-1}, d_1 U_0 .. d_d U_0, d_1 U_1, ...) in the right-hand-side
order of the cell problems (alpha = i for phi_i, N + i d + m for phi_i^m),
the integrand is w_V^T A_eff(p) w_U. Readings where the paper leaves the
discretisation open:

* U is continuous, bilinear (Q1) on the coarse blocks, with nodes at the
  block corners of the macrogrid on [0, 1]^d, and U = 0 on the boundary of the
  domain;
* A_eff(p) / |K_p| is taken as a constant density on K_p and integrated
  exactly against the Q1 functions (the paper evaluates U and its gradient at
  the block centre, which for Q1 blocks would leave checkerboard modes
  unconstrained);
* b_j(p) = int_{K_p} f phi_j (R_p = K_p), likewise spread as a constant
  density over K_p, so each corner of the block receives b_j(p) / 2^d;
* the result reported per block is the block average of U_i (the mean of its
  corner values), the quantity of Eq. U_MH_defi.

The discrete operator is symmetric positive semi-definite (a sum of Gram
forms) and is solved by a sparse direct solve.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem


def q1_tables(dim: int, Hc: float) -> np.ndarray:
    """T[s, t, a, b] = int_K D_s N_a D_t N_b on a block of side Hc.

    s, t = 0 is the value, s = 1 + m the derivative along axis m; corners in
    tensor order (axis 1 fastest).
    """
    vv = Hc * np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])
    vd = np.array([[-0.5, 0.5], [-0.5, 0.5]])  # int N_a N_b'
    dv = vd.T                                     # int N_a' N_b
    dd = np.array([[1.0, -1.0], [-1.0, 1.0]]) / Hc
    tab = {(False, False): vv, (False, True): vd, (True, False): dv, (True, True): dd}
    K = 2 ** dim
    T = np.zeros((1 + dim, 1 + dim, K, K))
    for s in range(1 + dim):
        for t in range(1 + dim):
            M = np.ones((1, 1))
            for ax in range(dim):  # the Kronecker product puts the last factor fastest
                M = np.kron(tab[(s == 1 + ax, t == 1 + ax)], M)
            T[s, t] = M
    return T


def element_matrix(A_p: np.ndarray, N: int, dim: int, Hc: float, T: np.ndarray | None = None) -> np.ndarray:
    """E[(a, j), (b, i)] (index a N + j) of one block from its effective tensor."""
    if T is None:
        T = q1_tables(dim, Hc)
    K = 2 ** dim
    vol = Hc ** dim
    E = np.zeros((K * N, K * N))

    def comps(j):
        return [(j, 0)] + [(N + j * dim + m, 1 + m) for m in range(dim)]

    for j in range(N):
        for i in range(N):
            blk = np.zeros((K, K))
            for al, s in comps(j):
                for be, t in comps(i):
                    blk += A_p[al, be] * T[s, t]
            E[j::N, i::N] = blk / vol
    return E


def block_corners(n_macro: int, dim: int) -> np.ndarray:
    """Macro node indices of the corners of every block: [P, 2^dim]."""
    off = fem.corner_offsets(dim)
    j = np.stack([(np.arange(n_macro ** dim) // n_macro ** k) % n_macro for k in range(dim)], axis=1)
    out = np.zeros((n_macro ** dim, 2 ** dim), np.int64)
    for c in range(2 ** dim):
        idx = np.zeros(n_macro ** dim, np.int64)
        stride = 1
        for k in range(dim):
            idx += (j[:, k] + off[c, k]) * stride
            stride *= n_macro + 1
        out[:, c] = idx
    return out


def interior_nodes(n_macro: int, dim: int) -> np.ndarray:
    n1 = n_macro + 1
    k = np.stack([(np.arange(n1 ** dim) // n1 ** a) % n1 for a in range(dim)], axis=1)
    return np.flatnonzero(np.all((k >= 1) & (k <= n_macro - 1), axis=1))


def assemble(A: np.ndarray, b: np.ndarray, n_macro: int, N: int, dim: int):
    """Global matrix and load on the interior nodes (unknown = interior index * N + j)."""
    Hc = 1.0 / n_macro
    T = q1_tables(dim, Hc)
    corners = block_corners(n_macro, dim)
    n_nodes = (n_macro + 1) ** dim
    rows, cols, vals = [], [], []
    F = np.zeros(n_nodes * N)
    K = 2 ** dim
    for p in range(n_macro ** dim):
        E = element_matrix(A[p], N, dim, Hc, T)
        dof = (corners[p][:, None] * N + np.arange(N)[None, :]).reshape(-1)  # a-major, j fastest
        rows.append(np.repeat(dof, K * N))
        cols.append(np.tile(dof, K * N))
        vals.append(E.reshape(-1))
        for a in range(K):
            F[corners[p][a] * N + np.arange(N)] += b[p] / K
    Kg = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(n_nodes * N, n_nodes * N))
    keep = (interior_nodes(n_macro, dim)[:, None] * N + np.arange(N)[None, :]).reshape(-1)
    return Kg[keep][:, keep].tocsc(), F[keep], keep


def solve(A: np.ndarray, b: np.ndarray, n_macro: int, N: int, dim: int):
    """Nodal U [(n_macro+1)^dim, N] (zero on the boundary) and block averages [P, N]."""
    Kg, F, keep = assemble(A, b, n_macro, N, dim)
    u = spla.spsolve(Kg, F)
    U = np.zeros(((n_macro + 1) ** dim) * N)
    U[keep] = u
    U = U.reshape(-1, N)
    Ub = U[block_corners(n_macro, dim)].mean(axis=1)
    return U, Ub


def block_load(cfg, f: np.ndarray, Phi: dict) -> np.ndarray:
    """b[p, j] = int_{K_p} f phi_j, f piecewise constant per fine element.

    Exact for bilinear phi_j on each fine element: |e| times the mean of its
    corner values. Phi[p] are the cell's local solutions [n_nodes, M].
    """
    from . import cells

    dim, N, nc, H = cfg.dim, cfg.n_cont, cfg.n_cell, cfg.H_el
    nodes = fem.element_nodes(nc, dim)
    kpm = fem.kp_element_mask(nc, H, dim)
    b = np.zeros((cfg.n_points, N))
    for p in range(cfg.n_points):
        fe = fem.window(f, cells.cell_origin(cfg, p), nc).reshape(-1)
        mean_phi = Phi[p][nodes[kpm]][:, :, :N].mean(axis=1)  # [elements of K_p, N]
        b[p] = (cfg.h ** dim) * (fe[kpm][:, None] * mean_phi).sum(axis=0)
    return b


def type3_error(Ua: np.ndarray, Ub: np.ndarray) -> np.ndarray:
    """Per continuum sqrt(sum |Ua - Ub|^2 / sum |Ua|^2) over the blocks (the paper's e_2)."""
    return np.sqrt(((Ua - Ub) ** 2).sum(axis=0) / (Ua ** 2).sum(axis=0))
