"""Pins for the oracle's finite-element pieces (no GPU).

Each check compares against something the mathematics fixes independently of
the oracle's own formulas: textbook element matrices, exact integrals of
polynomials, direct coarse assembly, and the partition-of-unity identity of
the Neumann cell problem.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import cells, fem
from paper_2503_01276_amd import workloads as W


def test_kref_2d_textbook():
    # Textbook bilinear stiffness on a square, counter-clockwise corner order,
    # independent of h in 2D.
    ccw = np.array([[4, -1, -2, -1], [-1, 4, -1, -2], [-2, -1, 4, -1], [-1, -2, -1, 4]]) / 6.0
    perm = [0, 1, 3, 2]  # ccw corner -> tensor corner (c1 + 2 c2)
    for h in (1.0, 0.125, 1 / 512):
        k = fem.kref(2, h)
        assert np.allclose(k[np.ix_(perm, perm)], ccw, atol=1e-15, rtol=0)


def test_kref_3d_textbook():
    # Trilinear stiffness on a cube of side h: diagonal h/3, edge neighbours 0,
    # face diagonals -h/12, body diagonal -h/12.
    h = 0.25
    k = fem.kref(3, h)
    off = fem.corner_offsets(3)
    for a in range(8):
        for b in range(8):
            dist = int(np.abs(off[a] - off[b]).sum())
            want = {0: h / 3, 1: 0.0, 2: -h / 12, 3: -h / 12}[dist]
            assert abs(k[a, b] - want) < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_kref_energy_of_linear(dim):
    # For v linear, v^T K_ref v = |e| |grad v|^2 exactly; constants have zero energy.
    h = 0.5
    off = fem.corner_offsets(dim) * h
    k = fem.kref(dim, h)
    rng = np.random.default_rng(0)
    for _ in range(5):
        a = rng.standard_normal(dim)
        v = off @ a + rng.standard_normal()
        assert np.isclose(v @ k @ v, h ** dim * (a @ a), rtol=1e-13)
    assert np.allclose(k.sum(axis=1), 0, atol=1e-15)


def _mass_ref(dim, h):
    m1 = h * np.array([[1 / 3, 1 / 6], [1 / 6, 1 / 3]])
    out = m1
    for _ in range(dim - 1):
        out = np.kron(m1, out)
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_q1_basis_integral(dim):
    # int_e N_a = |e| / 2^d for every Q1 corner function (mass-matrix row sums).
    h = 0.3
    assert np.allclose(_mass_ref(dim, h).sum(axis=1), h ** dim / 2 ** dim, rtol=1e-14)


def _random_cell(dim, nc, n_cont, seed):
    rng = np.random.default_rng(seed)
    lc = rng.integers(0, n_cont, size=(nc,) * dim).astype(np.uint8)
    kc = np.exp(rng.standard_normal((nc,) * dim))
    return kc, lc


@pytest.mark.parametrize("dim,nc,s", [(2, 8, 2), (2, 12, 3), (3, 4, 2)])
def test_constraint_rows_exact_averages(dim, nc, s):
    # Row (q, j) applied to a nodal interpolant of a (multi)linear function is
    # its exact average over R_q intersected with continuum j: 1 for the
    # constant, the region centroid for x_m.  This pins the row weights, the
    # normalisation and the type-2 right-hand side.
    h = 1.0 / 16
    kc, lc = _random_cell(dim, nc, 2, 1)
    H_el = nc // 2
    B, g, ids = fem.constraints(lc, s, 2, H_el, h)
    nn = nc + 1
    grids = np.meshgrid(*([np.arange(nn)] * dim), indexing="ij")
    b = [gg.reshape(-1) for gg in reversed(grids)]
    assert np.allclose(B @ np.ones(nn ** dim), 1.0, atol=1e-14)
    ac = fem.element_coords(nc, dim)
    for m in range(dim):
        xm = (b[m] - nc / 2) * h
        avg = B @ xm
        # brute force: centroid of the region's elements
        for r, rid in enumerate(ids):
            q, j = divmod(int(rid), 2)
            qc = [(q // s ** k) % s for k in range(dim)]
            sel = np.all(ac // (nc // s) == qc, axis=1) & (lc.reshape(-1) == j)
            want = ((ac[sel, m] + 0.5) - nc / 2).mean() * h
            assert abs(avg[r] - want) < 1e-14
            # type-2 rhs equals delta_ij (xbar - c_mj)
            for i in range(2):
                val = g[r, 2 + i * dim + m]
                if i != j:
                    assert val == 0.0
    # type-1 rhs
    for r, rid in enumerate(ids):
        j = int(rid) % 2
        assert g[r, j] == 1.0 and g[r, 1 - j] == 0.0


def test_cmj_is_kp_centroid():
    # int_{K_p} (x_m - c_mj) psi_j = 0 (paper Eq. phi_grad): the region average
    # of (x_m - c_mj) over K_p and continuum j vanishes.
    nc, H_el, h, dim = 16, 8, 1 / 64, 2
    kc, lc = _random_cell(dim, nc, 2, 3)
    B, g, ids = fem.constraints(lc, 2, 2, H_el, h)
    ac = fem.element_coords(nc, dim)
    kp = fem.kp_element_mask(nc, H_el, dim)
    for j in range(2):
        sel = kp & (lc.reshape(-1) == j)
        y = (ac[sel] + 0.5 - nc / 2) * h
        # reconstruct c_mj from any row of continuum j: c = xbar - g
        r = [k for k, rid in enumerate(ids) if rid % 2 == j][0]
        q = int(ids[r]) // 2
        qc = [(q // 2 ** k) % 2 for k in range(dim)]
        selq = np.all(ac // (nc // 2) == qc, axis=1) & (lc.reshape(-1) == j)
        xbar = ((ac[selq] + 0.5 - nc / 2) * h).mean(axis=0)
        c = xbar - g[r, 2 + j * dim: 2 + j * dim + dim]
        assert np.allclose((y - c).sum(axis=0), 0, atol=1e-13)


@pytest.mark.parametrize("dim,nc,r", [(2, 16, 2), (2, 16, 4), (2, 24, 8), (3, 8, 2)])
def test_galerkin_equals_direct_coarse_assembly(dim, nc, r):
    # With constant kappa, P^T K_h P is the Q1 stiffness assembled directly on
    # the coarse mesh of size r*h (exact because V_n is a subspace of V_h).
    h = 1 / 32
    K_h = fem.assemble_stiffness(np.full((nc,) * dim, 2.5), h)
    P = fem.prolongation(nc, r, dim)
    Kn = (P.T @ K_h @ P).toarray()
    K_c = fem.assemble_stiffness(np.full((nc // r,) * dim, 2.5), h * r).toarray()
    assert np.allclose(Kn, K_c, atol=1e-12 * np.abs(K_c).max())


def test_prolongation_reproduces_linears():
    nc, r, dim = 16, 4, 2
    P = fem.prolongation(nc, r, dim)
    nco = nc // r
    cg = np.meshgrid(np.arange(nco + 1), np.arange(nco + 1), indexing="ij")
    fg = np.meshgrid(np.arange(nc + 1), np.arange(nc + 1), indexing="ij")
    for coef in [(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.3, -2.0, 1.5)]:
        vc = coef[0] * cg[1].reshape(-1) * r + coef[1] * cg[0].reshape(-1) * r + coef[2]
        vf = coef[0] * fg[1].reshape(-1) + coef[1] * fg[0].reshape(-1) + coef[2]
        assert np.allclose(P @ vc, vf, atol=1e-13)


@pytest.mark.parametrize("dim,nc,s,n_cont", [(2, 16, 2, 2), (2, 12, 3, 3), (3, 8, 2, 2)])
def test_neumann_partition_of_unity(dim, nc, s, n_cont):
    # Neumann variant of the type-1 cell problem: the constant 1 satisfies the
    # sum over i of the type-1 constraints and has zero energy, so
    # sum_i phi_i == 1 exactly, and sum_i A_ji = 0 (Eq. Bs_defi).  A wrong row
    # weight, a dropped row or a wrong right-hand side breaks this identity.
    h = 1 / 32
    kc, lc = _random_cell(dim, nc, n_cont, 5)
    kc = kc * 1e3 ** (lc == 1)
    K = fem.assemble_stiffness(kc, h)
    B, g, _ = fem.constraints(lc, s, n_cont, nc // 2, h)
    kkt = sp.bmat([[K, sp.csr_matrix(B).T], [sp.csr_matrix(B), None]]).toarray()
    n = K.shape[0]
    phis = []
    for i in range(n_cont):
        rhs = np.concatenate([np.zeros(n), g[:, i]])
        phis.append(np.linalg.solve(kkt, rhs)[:n])
    tot = np.sum(phis, axis=0)
    assert np.allclose(tot, 1.0, atol=1e-9)
    kpm = fem.kp_element_mask(nc, nc // 2, dim)
    Kkp = fem.assemble_stiffness(kc, h, elem_mask=kpm)
    Phi = np.stack(phis, axis=1)
    A = Phi.T @ (Kkp @ Phi)
    assert np.allclose(A.sum(axis=1), 0, atol=1e-9 * np.abs(A).max())


def test_window_periodic_wrap():
    n = 8
    f = np.arange(n * n, dtype=float).reshape(n, n)
    w = fem.window(f, [-2, 6], 4)
    want = f[np.ix_([6, 7, 0, 1], [6, 7, 0, 1])]
    assert np.array_equal(w, want)
    idx = fem.window_flat_indices(n, [-2, 6], 4, 2)
    assert np.array_equal(f.reshape(-1)[idx].reshape(4, 4), want)


def test_cell_origin_centres_cell_on_macropoint():
    cfg = W.PRESETS["c2"]
    for p in [0, 5, 33, 1023]:
        org = cells.cell_origin(cfg, p)
        j = [p % cfg.n_macro, p // cfg.n_macro]
        for k in range(2):
            centre = org[k] + cfg.n_cell / 2
            assert centre == cfg.H_el * (j[k] + 0.5)
