"""Pins of the oracle's multigrid hierarchy, V-cycle and PCG (no GPU)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, mg, pcg


def _setup(nel, seed=0, lo=1e-2):
    g = fem.Grid(nel)
    K0 = fem.element_stiffness(g.dim)
    x = np.random.default_rng(seed).uniform(lo, 1.0, g.m)
    return g, K0, x


def test_prolongation_stencil_2d():
    c = fem.Grid((4, 2))
    P = mg.prolongation_slots(c).toarray()
    nxf = 9
    I, J = 2, 1                                     # an interior coarse node
    col = P[:, 2 * (J * 5 + I)]                     # x-component column
    W = np.zeros((5, 9))
    for j in range(5):
        for i in range(9):
            W[j, i] = col[2 * (j * nxf + i)]
    expect = np.zeros((5, 9))
    expect[1:4, 3:6] = [[0.25, 0.5, 0.25], [0.5, 1.0, 0.5], [0.25, 0.5, 0.25]]
    np.testing.assert_array_equal(W, expect)
    assert col.sum() == 4.0
    assert np.all(col[1::2] == 0)                   # components do not mix


def test_prolongation_column_sums_3d():
    c = fem.Grid((2, 2, 2))
    P = mg.prolongation_slots(c).toarray()
    q = (1 * 3 + 1) * 3 + 1                         # interior coarse node (1,1,1)
    assert P[:, 3 * q + 2].sum() == 8.0             # 1 + 6/2 + 12/4 + 8/8


@pytest.mark.parametrize("nel", [(8, 4), (4, 4, 2)])
def test_galerkin_equals_rediscretisation(nel):
    # x constant on each coarse element: P' K_h(x) P = K_2h(x_c) on nested spaces.
    fine = fem.Grid(nel)
    coarse = fine.coarsen()
    rng = np.random.default_rng(4)
    xc = rng.uniform(0.1, 1.0, coarse.m)
    # fine element (i,j,k) lies in coarse element (i//2, j//2, k//2)
    ijk = np.stack(np.unravel_index(np.arange(fine.m), fine.nel[::-1]), 1)[:, ::-1]
    cidx = np.ravel_multi_index(tuple((ijk // 2)[:, ::-1].T), coarse.nel[::-1])
    xf = xc[cidx]
    K0f = fem.element_stiffness(fine.dim, h=1.0)
    K0c = fem.element_stiffness(fine.dim, h=2.0)
    P = mg.prolongation_free(fine, coarse)
    Ag = (P.T @ fem.stiffness_free(fine, xf, K0f) @ P).toarray()
    Ac = fem.stiffness_free(coarse, xc, K0c).toarray()
    np.testing.assert_allclose(Ag, Ac, rtol=0, atol=1e-13 * np.abs(Ac).max())


def test_vcycle_symmetric_positive_definite():
    g, K0, x = _setup((8, 4))
    H = mg.kstiffness_hierarchy(g, x, K0, 3)
    M = mg.vcycle_matrix(H)
    assert np.abs(M - M.T).max() < 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


def test_vcycle_contracts():
    g, K0, x = _setup((8, 4), lo=0.5)
    H = mg.kstiffness_hierarchy(g, x, K0, 3)
    M = mg.vcycle_matrix(H)
    E = np.eye(M.shape[0]) - M @ H.A[-1].toarray()
    assert np.abs(np.linalg.eigvals(E)).max() < 1.0


def test_one_level_is_the_direct_solve():
    g, K0, x = _setup((8, 4))
    H = mg.kstiffness_hierarchy(g, x, K0, 1)
    b = np.random.default_rng(7).standard_normal(H.A[-1].shape[0])
    np.testing.assert_allclose(H.A[-1] @ mg.vcycle(H, b), b, rtol=0, atol=1e-12)
    res = pcg.mg_pcg(H, b, rtol=1e-10)
    assert res.iters == 1 and res.converged


def test_pcg_exact_preconditioner_one_step():
    g, K0, x = _setup((6, 4))
    A = fem.stiffness_free(g, x, K0)
    lu = spla.splu(A.tocsc())
    b = np.random.default_rng(8).standard_normal(A.shape[0])
    res = pcg.pcg(lambda v: A @ v, b, lu.solve, rtol=1e-12)
    assert res.iters == 1
    np.testing.assert_allclose(res.z, lu.solve(b), rtol=1e-10)


def test_pcg_identity_preconditioner_textbook_cg():
    # With M = I the recurrence is plain CG: exact within n steps on an SPD matrix.
    g, K0, x = _setup((3, 2), lo=0.5)
    A = fem.stiffness_free(g, x, K0).toarray()
    b = np.random.default_rng(9).standard_normal(A.shape[0])
    res = pcg.pcg(lambda v: A @ v, b, lambda r: r.copy(), rtol=1e-13, maxit=200)
    np.testing.assert_allclose(res.z, np.linalg.solve(A, b), rtol=1e-9)
    assert res.converged


def test_flexible_ratio_equals_standard_with_fixed_preconditioner():
    # With one fixed symmetric preconditioner, r~'y = 0 (conjugacy of successive
    # residuals in the M inner product), so the Polak-Ribiere ratio reproduces the
    # iterates of Algorithm PCG up to rounding.  (With a preconditioner that varies
    # between steps the two differ; that case has no closed form: parity unpinned.)
    g, K0, x = _setup((32, 16))
    A = fem.stiffness_free(g, x, K0)
    H = mg.Hierarchy(g, A, 3)
    b = np.random.default_rng(10).standard_normal(A.shape[0])
    std = pcg.mg_pcg(H, b, rtol=1e-10)
    flex = pcg.mg_pcg(H, b, rtol=1e-10, flexible=True)
    assert std.converged and flex.converged and std.iters == flex.iters
    np.testing.assert_allclose(flex.z, std.z, rtol=1e-8)
    # the correction term it subtracts is at rounding level here
    np.testing.assert_allclose(flex.history, std.history, rtol=1e-6)


@pytest.mark.parametrize("nel,levels", [((32, 16), 4), ((8, 4, 4), 3)])
def test_mg_pcg_matches_direct_within_bound(nel, levels):
    g, K0, x = _setup(nel, lo=1e-3)
    A = fem.stiffness_free(g, x, K0)
    H = mg.Hierarchy(g, A, levels)
    f = fem.to_free(g, fem.load_vector(g, [((g.nel[0],) + tuple(v // 2 for v in g.nel[1:]), 1, -1.0)]))
    res = pcg.mg_pcg(H, f, rtol=1e-8)
    assert res.converged and res.true_relres <= 1e-8
    ustar = spla.spsolve(A.tocsc(), f)
    e = res.z - ustar
    errK = np.sqrt(e @ (A @ e)) / np.sqrt(ustar @ (A @ ustar))
    ev = np.linalg.eigvalsh(A.toarray()) if A.shape[0] < 3000 else None
    kappa = ev[-1] / ev[0]
    assert errK <= np.sqrt(kappa) * res.true_relres


def test_iterations_mesh_independent():
    # Constant density: MG-PCG counts stay flat under refinement (Sec. 7 observation).
    its = []
    for nel, L in [((16, 8), 2), ((32, 16), 3), ((64, 32), 4), ((128, 64), 5)]:
        g = fem.Grid(nel)
        K0 = fem.element_stiffness(2)
        H = mg.kstiffness_hierarchy(g, np.full(g.m, 0.5), K0, L)
        f = fem.to_free(g, fem.load_vector(g, [((nel[0], nel[1] // 2), 1, -1.0)]))
        its.append(pcg.mg_pcg(H, f, rtol=1e-8).iters)
    assert max(its) - min(its) <= 3, its


def test_pcg_breakdown_on_indefinite():
    A = np.diag([1.0, -1.0, 2.0])
    b = np.array([1.0, 1.0, 1.0])
    res = pcg.pcg(lambda v: A @ v, b, lambda r: r.copy(), rtol=1e-12)
    assert not res.converged and res.status == "breakdown"


def test_pcg_maxit_reported():
    g, K0, x = _setup((16, 8), lo=1e-3)
    A = fem.stiffness_free(g, x, K0)
    b = np.ones(A.shape[0])
    res = pcg.pcg(lambda v: A @ v, b, lambda r: r.copy(), rtol=1e-12, maxit=3)
    assert res.status == "maxit" and res.iters == 3 and not res.converged
