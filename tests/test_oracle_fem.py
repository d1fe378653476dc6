"""Pins of the oracle's discretisation against closed forms, invariants and the
paper's printed DOF counts (no GPU)."""
import os

import numpy as np
import pytest

from oracle import fem

HERE = os.path.dirname(os.path.abspath(__file__))
NU = 0.3


def _c2d(E=1.0, nu=NU):
    c = E / (1 - nu * nu)
    return c, c * nu, c * (1 - nu) / 2           # C11, C12, C33


def test_k0_2d_row0_closed_form():
    # Row 0 (node 0, x-DOF) integrated by hand over the unit square with
    # N0=(1-xi)(1-eta), N1=xi(1-eta), N2=xi*eta, N3=(1-xi)eta.
    C11, C12, C33 = _c2d()
    expect = [(C11 + C33) / 3, (C12 + C33) / 4, -C11 / 3 + C33 / 6, (C12 - C33) / 4,
              -(C11 + C33) / 6, -(C12 + C33) / 4, C11 / 6 - C33 / 3, (C33 - C12) / 4]
    K0 = fem.element_stiffness(2, 1.0, NU)
    np.testing.assert_allclose(K0[0], expect, rtol=0, atol=1e-15)
    assert abs(K0[0, 0] - 0.4945054945054945) < 1e-15          # (3-nu)/6 / (1-nu^2)
    assert abs(K0[0, 1] - 0.17857142857142858) < 1e-15         # (1+nu)/8 / (1-nu^2)


def test_k0_2d_size_independent_and_symmetric():
    K1 = fem.element_stiffness(2, 1.0, NU, h=1.0)
    K3 = fem.element_stiffness(2, 1.0, NU, h=3.0)
    np.testing.assert_allclose(K1, K3, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(K1, K1.T, rtol=0, atol=1e-15)


def test_k0_3d_closed_form_entries():
    E, nu = 1.0, NU
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    K0 = fem.element_stiffness(3, E, nu)
    # int (dN0/dx)^2 = 1/9 etc. on the unit cube; int dN0/dx dN0/dy = 1/12
    assert abs(K0[0, 0] - (lam + 2 * mu + 2 * mu) / 9) < 1e-15
    assert abs(K0[0, 0] - 0.23504273504273504) < 1e-14
    assert abs(K0[0, 1] - (lam + mu) / 12) < 1e-15
    assert abs(K0[1, 1] - K0[0, 0]) < 1e-15
    np.testing.assert_allclose(K0, K0.T, rtol=0, atol=1e-15)
    np.testing.assert_allclose(fem.element_stiffness(3, E, nu, h=2.0), 2.0 * K0, rtol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_k0_rigid_body_null_space(dim):
    K0 = fem.element_stiffness(dim, 1.0, NU)
    X = fem._local_corner_coords(dim)
    modes = []
    for c in range(dim):                         # translations
        v = np.zeros((len(X), dim))
        v[:, c] = 1
        modes.append(v.ravel())
    for a in range(dim):                         # infinitesimal rotations
        for b in range(a + 1, dim):
            v = np.zeros((len(X), dim))
            v[:, a] = -X[:, b]
            v[:, b] = X[:, a]
            modes.append(v.ravel())
    for v in modes:
        assert np.linalg.norm(K0 @ v) < 1e-14
    ev = np.linalg.eigvalsh(K0)
    assert np.sum(ev > 1e-12) == dim * 2 ** dim - len(modes)    # rank 5 (2D), 18 (3D)
    assert ev.min() > -1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_patch_test_affine_energy(dim):
    # u(X) = G X is affine; the element energy u'K0u must equal |e| eps'C eps exactly.
    rng = np.random.default_rng(5)
    G = rng.standard_normal((dim, dim))
    X = fem._local_corner_coords(dim)
    u = (X @ G.T).ravel()
    eps = 0.5 * (G + G.T)
    if dim == 2:
        ev = np.array([eps[0, 0], eps[1, 1], 2 * eps[0, 1]])
    else:
        ev = np.array([eps[0, 0], eps[1, 1], eps[2, 2], 2 * eps[0, 1], 2 * eps[1, 2], 2 * eps[0, 2]])
    C = fem.elasticity_matrix(dim, 1.0, NU)
    K0 = fem.element_stiffness(dim, 1.0, NU)
    assert abs(u @ K0 @ u - ev @ C @ ev) < 1e-13


def test_dof_counts_match_paper_tables():
    rows = []
    with open(os.path.join(HERE, "golden", "dof_counts.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                nx, ny, var, plus, _ = line.split()
                rows.append((int(nx), int(ny), int(var), int(plus)))
    assert len(rows) == 16
    for nx, ny, var, plus in rows:
        g = fem.Grid((nx, ny))
        nfree = int(np.count_nonzero(~g.clamped_mask()))
        assert nfree + plus == var, (nx, ny)
        assert len(g.free_to_slot()) == nfree


def test_indexing_brute_force_small():
    g = fem.Grid((3, 2))
    nodes = g.element_nodes()
    # element (i=2, j=1) is e = 1*3 + 2 = 5; its nodes (2,1),(3,1),(3,2),(2,2)
    assert list(nodes[5]) == [1 * 4 + 2, 1 * 4 + 3, 2 * 4 + 3, 2 * 4 + 2]
    g3 = fem.Grid((2, 2, 2))
    n3 = g3.element_nodes()
    e = (1 * 2 + 0) * 2 + 1                      # (i=1, j=0, k=1)
    node = lambda i, j, k: (k * 3 + j) * 3 + i
    assert list(n3[e]) == [node(1, 0, 1), node(2, 0, 1), node(2, 1, 1), node(1, 1, 1),
                           node(1, 0, 2), node(2, 0, 2), node(2, 1, 2), node(1, 1, 2)]
    mask = g.clamped_mask()
    coords = g.node_coords()
    for q in range(g.nnodes):
        assert mask[2 * q] == mask[2 * q + 1] == (coords[q, 0] == 0)


def test_assembly_vs_pointwise_loop():
    # Element loop with explicit coordinates, written independently of element_dofs.
    nx, ny = 3, 2
    g = fem.Grid((nx, ny))
    K0 = fem.element_stiffness(2)
    rng = np.random.default_rng(0)
    x = rng.uniform(0.1, 1.0, g.m)
    ref = np.zeros((g.nslots, g.nslots))
    for j in range(ny):
        for i in range(nx):
            corners = [(i, j), (i + 1, j), (i + 1, j + 1), (i, j + 1)]
            sl = []
            for (a, b) in corners:
                q = b * (nx + 1) + a
                sl += [2 * q, 2 * q + 1]
            ref[np.ix_(sl, sl)] += x[j * nx + i] * K0
    A = fem.stiffness_slots(g, x, K0).toarray()
    np.testing.assert_allclose(A, ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("nel", [(8, 4), (4, 2, 2)])
def test_k_symmetric_positive_definite(nel):
    g = fem.Grid(nel)
    K0 = fem.element_stiffness(g.dim)
    x = np.random.default_rng(1).uniform(1e-3, 1.0, g.m)
    K = fem.stiffness_free(g, x, K0).toarray()
    np.testing.assert_allclose(K, K.T, rtol=0, atol=1e-15)
    assert np.linalg.eigvalsh(K).min() > 0
    full = fem.stiffness_slots(g, x, K0).toarray()
    # unclamped operator keeps the rigid translations in its null space
    for c in range(g.dim):
        t = np.zeros(g.nslots)
        t[c::g.dim] = 1.0
        assert np.linalg.norm(full @ t) < 1e-12


@pytest.mark.parametrize("nel", [(6, 4), (2, 2, 2)])
def test_uniform_strain_energy(nel):
    # u = (eps_xx X, 0[, 0]) on the whole grid: u'K(x)u = sum_e x_e eps'C eps |e|.
    g = fem.Grid(nel)
    K0 = fem.element_stiffness(g.dim)
    x = np.random.default_rng(2).uniform(0.1, 1.0, g.m)
    u = np.zeros(g.nslots)
    u[0::g.dim] = 0.01 * g.node_coords()[:, 0]
    C = fem.elasticity_matrix(g.dim)
    e = np.zeros(C.shape[0])
    e[0] = 0.01
    K = fem.stiffness_slots(g, x, K0)
    assert abs(u @ (K @ u) - x.sum() * (e @ C @ e)) < 1e-15


def test_compliance_identity_and_dense_solve():
    g = fem.Grid((8, 4))
    K0 = fem.element_stiffness(2)
    x = np.random.default_rng(3).uniform(0.01, 1.0, g.m)
    f = fem.load_vector(g, [((8, 2), 1, -1.0)])
    K = fem.stiffness_free(g, x, K0)
    ff = fem.to_free(g, f)
    u = np.linalg.solve(K.toarray(), ff)
    L = np.linalg.cholesky(K.toarray())
    u2 = np.linalg.solve(L.T, np.linalg.solve(L, ff))
    np.testing.assert_allclose(u, u2, rtol=1e-12)
    assert abs(ff @ u - u @ (K @ u)) < 1e-12 * abs(ff @ u)


@pytest.mark.parametrize("nel", [(7, 3), (3, 2, 2)])
def test_matrix_free_apply_equals_assembled(nel):
    g = fem.Grid(nel)
    K0 = fem.element_stiffness(g.dim)
    rng = np.random.default_rng(11)
    x = rng.uniform(0.1, 1.0, g.m)
    v = rng.standard_normal(g.nslots)
    A = fem.stiffness_slots(g, x, K0)
    np.testing.assert_allclose(fem.apply_slots(g, x, K0, v), A @ v, rtol=0, atol=1e-13 * np.abs(A @ v).max())
    Af = fem.stiffness_free(g, x, K0)
    yf = fem.apply_free_masked(g, x, K0, v)
    np.testing.assert_allclose(fem.to_free(g, yf), Af @ fem.to_free(g, v), rtol=0, atol=1e-13 * np.abs(yf).max())
    assert np.all(yf[g.clamped_mask()] == 0)
