"""Oracle, part 1: Q1 finite elements on one oversampled cell (plain, assembled).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import this package.

Everything here is written from the definitions in the paper, Sec. 2
(Eqs. phi_avar, phi_grad) and Sec. 3.2 (nested spaces V_n):

* K_ref: the Q1 element stiffness matrix, built as the Kronecker sum of the 1D
  stiffness [[1,-1],[-1,1]]/h and mass h*[[1/3,1/6],[1/6,1/3]] matrices;
* K_h = sum_e kappa_e K_ref on the cell's fine elements (kappa piecewise
  constant per fine element, Sec. 4);
* constraint rows: the average of v over R_q intersected with continuum j,
  i.e. int_{R_q} psi_j v / int_{R_q} psi_j, integrated exactly (a Q1 function
  integrates to |e| times the mean of its nodal values on an element);
* right-hand sides g: delta_ij (type 1) and delta_ij (xbar_{m,qj} - c_mj)
  (type 2), where c_mj is the continuum-j centroid in K_p;
* P_n: tensor-product linear interpolation from mesh h*eta^(n-1) to h.

Layout: local element (a1, a2[, a3]) and node (b1, b2[, b3]) with x1 fastest;
node index b1 + (nc+1)*(b2 + (nc+1)*b3); local element corner c has offsets
(c & 1, (c >> 1) & 1, (c >> 2) & 1). Local coordinates are centred at the
macropoint (the cell centre).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def k1_m1(h: float):
    k1 = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    m1 = h * np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])
    return k1, m1


def kref(dim: int, h: float) -> np.ndarray:
    """Q1 element stiffness for -div(grad) on a cube of side h, tensor corner order."""
    k1, m1 = k1_m1(h)
    if dim == 2:
        # factor order (x2, x1): corner index c = c1 + 2*c2
        return np.kron(m1, k1) + np.kron(k1, m1)
    return (np.kron(np.kron(m1, m1), k1) + np.kron(np.kron(m1, k1), m1)
            + np.kron(np.kron(k1, m1), m1))


def corner_offsets(dim: int) -> np.ndarray:
    c = np.arange(2 ** dim)
    return np.stack([(c >> k) & 1 for k in range(dim)], axis=1)  # [corner, axis]


def element_nodes(nc: int, dim: int) -> np.ndarray:
    """Node indices of every local element: [n_elem, 2^dim], elements x1-fastest."""
    nn = nc + 1
    grids = np.meshgrid(*([np.arange(nc)] * dim), indexing="ij")  # axis order (x_d .. x1)
    a = [g.reshape(-1) for g in reversed(grids)]  # a[0] = a1 (fastest)
    off = corner_offsets(dim)
    nodes = np.zeros((nc ** dim, 2 ** dim), np.int64)
    for c in range(2 ** dim):
        idx = np.zeros(nc ** dim, np.int64)
        stride = 1
        for k in range(dim):
            idx += (a[k] + off[c, k]) * stride
            stride *= nn
        nodes[:, c] = idx
    return nodes


def element_coords(nc: int, dim: int) -> np.ndarray:
    """Integer element coordinates [n_elem, dim] (a1, a2[, a3])."""
    grids = np.meshgrid(*([np.arange(nc)] * dim), indexing="ij")
    return np.stack([g.reshape(-1) for g in reversed(grids)], axis=1)


def free_nodes(nc: int, dim: int, bc: int = 0) -> np.ndarray:
    """Free nodes: the interior ones for homogeneous Dirichlet data on the cell
    boundary (bc = 0), every node for natural (Neumann) conditions (bc = 1)."""
    nn = nc + 1
    if bc == 1:
        return np.arange(nn ** dim)
    grids = np.meshgrid(*([np.arange(nn)] * dim), indexing="ij")
    b = [g.reshape(-1) for g in reversed(grids)]
    mask = np.ones(nn ** dim, bool)
    for k in range(dim):
        mask &= (b[k] > 0) & (b[k] < nc)
    return np.flatnonzero(mask)


def assemble_stiffness(kc: np.ndarray, h: float, elem_mask: np.ndarray | None = None) -> sp.csr_matrix:
    """K = sum_e kappa_e K_ref over the cell's elements (optionally a subset)."""
    dim = kc.ndim
    nc = kc.shape[0]
    nodes = element_nodes(nc, dim)
    kv = kc.reshape(-1)
    if elem_mask is not None:
        nodes = nodes[elem_mask]
        kv = kv[elem_mask]
    kr = kref(dim, h)
    nloc = 2 ** dim
    rows = np.repeat(nodes, nloc, axis=1).reshape(-1)
    cols = np.tile(nodes, (1, nloc)).reshape(-1)
    vals = (kv[:, None, None] * kr[None, :, :]).reshape(-1)
    n = (nc + 1) ** dim
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def kp_element_mask(nc: int, H_el: int, dim: int) -> np.ndarray:
    """Elements of the coarse block K_p (the central H_el^d block of the cell)."""
    lo = (nc - H_el) // 2
    ac = element_coords(nc, dim)
    return np.all((ac >= lo) & (ac < lo + H_el), axis=1)


def constraints(lc: np.ndarray, n_sub: int, n_cont: int, H_el: int, h: float):
    """Constraint rows B (dense, over all cell nodes) and right-hand sides g.

    Rows are ordered (q, j) with q = qx + s*qy (+ s^2*qz); rows whose region
    R_q holds no element of continuum j are dropped. Returns
    (B [m, n_nodes], g [m, M], row_ids [m] = q*N + j).
    M = N + N*d right-hand sides: alpha = i (type 1), alpha = N + i*d + m (type 2).
    """
    dim = lc.ndim
    nc = lc.shape[0]
    sb = nc // n_sub
    nodes = element_nodes(nc, dim)
    ac = element_coords(nc, dim)
    lab = lc.reshape(-1)
    ycen = (ac + 0.5 - nc / 2.0) * h  # element centroids, local coordinates
    qc = ac // sb
    q = np.zeros(len(lab), np.int64)
    stride = 1
    for k in range(dim):
        q += qc[:, k] * stride
        stride *= n_sub
    kp = kp_element_mask(nc, H_el, dim)
    # continuum centroids in K_p (zero when the continuum is absent from K_p)
    cmj = np.zeros((dim, n_cont))
    for j in range(n_cont):
        sel = kp & (lab == j)
        if sel.any():
            cmj[:, j] = ycen[sel].mean(axis=0)
    M = n_cont * (1 + dim)
    nn = (nc + 1) ** dim
    B_rows, g_rows, ids = [], [], []
    for qq in range(n_sub ** dim):
        for j in range(n_cont):
            sel = (q == qq) & (lab == j)
            cnt = int(sel.sum())
            if cnt == 0:
                continue
            row = np.zeros(nn)
            np.add.at(row, nodes[sel].reshape(-1), 1.0 / (2 ** dim * cnt))
            g = np.zeros(M)
            g[j] = 1.0
            xbar = ycen[sel].mean(axis=0)
            for m in range(dim):
                g[n_cont + j * dim + m] = xbar[m] - cmj[m, j]
            B_rows.append(row)
            g_rows.append(g)
            ids.append(qq * n_cont + j)
    return np.array(B_rows), np.array(g_rows), np.array(ids)


def prolongation_1d(nc: int, r: int) -> np.ndarray:
    """Linear interpolation from nodes of spacing r (in fine elements) to spacing 1."""
    nco = nc // r
    b = np.arange(nc + 1)[:, None]
    c = np.arange(nco + 1)[None, :]
    return np.maximum(0.0, 1.0 - np.abs(b - r * c) / r)


def prolongation(nc: int, r: int, dim: int) -> sp.csr_matrix:
    p1 = sp.csr_matrix(prolongation_1d(nc, r))
    out = p1
    for _ in range(dim - 1):
        out = sp.kron(p1, out, format="csr")  # slower axes on the left
    return out.tocsr()


def window(field: np.ndarray, origin, nc: int) -> np.ndarray:
    """Cell window of a global element field with periodic wrap; origin per axis (x1 first)."""
    dim = field.ndim
    n = field.shape[0]
    idx = [((origin[k] + np.arange(nc)) % n) for k in range(dim)]
    return field[np.ix_(*reversed(idx))]


def window_flat_indices(n: int, origin, nc: int, dim: int) -> np.ndarray:
    """Global flat element index of every local element (x1 fastest)."""
    ac = element_coords(nc, dim)
    g = np.zeros(len(ac), np.int64)
    stride = 1
    for k in range(dim):
        g += ((origin[k] + ac[:, k]) % n) * stride
        stride *= n
    return g
