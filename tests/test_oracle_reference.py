"""Pins for the global fine-grid reference of the Type 1 / Type 2 errors (no GPU)."""
import numpy as np

from oracle import reference


def test_fine_poisson_second_order():
    # -Lap u = 2 pi^2 sin(pi x) sin(pi y), kappa = 1: the nodal error falls at
    # least at second order (on uniform grids Q1 is superconvergent at nodes
    # for this separable solution, so the measured ratio is about 16)
    errs = []
    for n in (32, 64):
        x = (np.arange(n) + 0.5) / n
        f = 2 * np.pi ** 2 * np.outer(np.sin(np.pi * x), np.sin(np.pi * x))
        u = reference.fine_solution(np.ones((n, n)), f)
        xn = np.arange(n + 1) / n
        exact = np.outer(np.sin(np.pi * xn), np.sin(np.pi * xn)).reshape(-1)
        errs.append(np.abs(u - exact).max())
    assert errs[1] < 1e-6
    assert errs[0] / errs[1] > 3.5, errs


def test_continuum_block_averages_of_a_linear_field():
    # u = x1 + 2 x2 is exactly Q1; element means are centroid values, so the
    # continuum average over K_p is the mean of the centroids of its elements
    n, nm = 16, 4
    xn = np.arange(n + 1) / n
    u = (xn[None, :] + 2 * xn[:, None]).reshape(-1)
    lab = np.zeros((n, n), np.uint8)
    lab[3, :] = 1
    lab[9:11, :] = 1
    U = reference.continuum_block_averages(u, lab, nm, 2)
    H = n // nm
    xc = (np.arange(n) + 0.5) / n
    cent = xc[None, :] + 2 * xc[:, None]
    for p in range(nm * nm):
        j1, j2 = p % nm, p // nm
        blk = (slice(H * j2, H * (j2 + 1)), slice(H * j1, H * (j1 + 1)))
        for i in range(2):
            m = lab[blk] == i
            ref = cent[blk][m].mean() if m.any() else np.nan
            assert (np.isnan(ref) and np.isnan(U[p, i])) or abs(U[p, i] - ref) < 1e-14


def test_e2_ignores_undefined_blocks():
    Uref = np.array([[1.0, np.nan], [2.0, 3.0]])
    U = np.array([[1.1, 7.0], [2.0, 3.3]])
    e = reference.e2(Uref, U)
    assert np.allclose(e, [0.1 / np.sqrt(5.0), 0.1])
