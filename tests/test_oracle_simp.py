"""Pins of the oracle's SIMP model with a density filter (Sec. 9), no GPU."""
import numpy as np
import pytest

from oracle import fem, simp


def test_filter_matrix_by_hand():
    # 3 x 2 elements, rmin = 2, Manhattan: weight 2 on the element, 1 on each edge
    # neighbour.  Column sums of W^: corners 2 + 1 + 1 = 4, the two middle elements
    # 2 + 1 + 1 + 1 = 5; W_ji = W^_ji / s_i.
    W = simp.filter_matrix(fem.Grid((3, 2)), 2.0).toarray()
    s = [4, 5, 4, 4, 5, 4]
    What = np.array([[2, 1, 0, 1, 0, 0],
                     [1, 2, 1, 0, 1, 0],
                     [0, 1, 2, 0, 0, 1],
                     [1, 0, 0, 2, 1, 0],
                     [0, 1, 0, 1, 2, 1],
                     [0, 0, 1, 0, 1, 2]], dtype=float)
    np.testing.assert_array_equal(W, What / np.array(s, dtype=float)[None, :])


def test_filter_properties():
    g = fem.Grid((7, 5))
    W = simp.filter_matrix(g, 2.0)
    np.testing.assert_allclose(np.asarray(W.sum(axis=0)).ravel(), 1.0, rtol=1e-15)   # sum x~ = sum x
    assert np.array_equal(simp.filter_matrix(g, 1.0).toarray(), np.eye(g.m))          # rmin = 1: no filter
    # interior element of a constant field: (W x)_j = 6 x / 6
    x = np.full(g.m, 0.7)
    xt = W @ x
    assert abs(xt[2 * 7 + 3] - 0.7) < 1e-15
    # 3D: an interior element has six face neighbours, s = 2 + 6
    W3 = simp.filter_matrix(fem.Grid((3, 3, 3)), 2.0).toarray()
    assert abs(W3[13, 13] - 2.0 / 8.0) < 1e-15 and abs(W3[12, 13] - 1.0 / 8.0) < 1e-15


def _cantilever(nel):
    g = fem.Grid(nel)
    K0 = fem.element_stiffness(g.dim)
    f = fem.load_vector(g, [((nel[0], nel[1] // 2), 1, -1.0)])
    return g, K0, f


def test_simp_gradient_central_differences():
    g, K0, f = _cantilever((6, 4))
    x = np.random.default_rng(4).uniform(0.3, 1.0, g.m)
    W = simp.filter_matrix(g, 2.0)
    c, u, grad, xt = simp.compliance_and_gradient(g, K0, f, x, 2.0, 3.0, W)
    h = 1e-6
    for e in (0, 5, 11, 23):
        xp, xm = x.copy(), x.copy()
        xp[e] += h
        xm[e] -= h
        fd = (simp.compliance_and_gradient(g, K0, f, xp, 2.0, 3.0, W)[0] -
              simp.compliance_and_gradient(g, K0, f, xm, 2.0, 3.0, W)[0]) / (2 * h)
        assert abs(fd - grad[e]) <= 1e-6 * np.abs(grad).max(), (e, fd, grad[e])


def test_simp_reduces_to_the_plain_model():
    # p = 1 and no filter (rmin = 1): K^ = K(x) and the gradient is -u_e'K0u_e
    g, K0, f = _cantilever((6, 4))
    x = np.random.default_rng(5).uniform(0.3, 1.0, g.m)
    c, u, grad, xt = simp.compliance_and_gradient(g, K0, f, x, 1.0, 1.0)
    K = fem.stiffness_free(g, x, K0)
    ff = fem.to_free(g, f)
    np.testing.assert_allclose(u, np.linalg.solve(K.toarray(), ff), rtol=1e-10)
    # Euler: c(t x) = c(x)/t for the linear model, so sum x_e dc/dx_e = -c
    assert abs(float(x @ grad) + c) <= 1e-10 * c


# ---- interior-point method on the SIMP model (Sec. 9) --------------------------
from oracle import ip  # noqa: E402


def _simp_problem(nel=(6, 4), rmin=2.0, p=3.0, xbar=3.0):
    g, K0, f = _cantilever(nel)
    return simp.SimpProblem(g, K0, f, 0.4 * g.m, xbar, rmin=rmin, p=p)


def _simp_state(prob, seed=0):
    rng = np.random.default_rng(seed)
    m, n = prob.grid.m, len(prob.free)
    return ip.IPState(rng.standard_normal(n), 0.7, rng.uniform(0.3, 1.5, m), rng.uniform(0.5, 2, m),
                      rng.uniform(0.5, 2, m), 0.3, 0.2)


def test_simp_bhat_is_the_derivative_of_the_equilibrium_operator():
    # b^_i = d(K^(x) u)/dx_i, by central differences of the assembled K^ (no formula shared)
    prob = _simp_problem()
    st = _simp_state(prob, 1)
    B = prob.Bmat(st).toarray()
    h = 1e-6
    for i in (0, 7, 13, 23):
        xp, xm = st.x.copy(), st.x.copy()
        xp[i] += h
        xm[i] -= h
        fd = (prob.K(xp) @ st.u - prob.K(xm) @ st.u) / (2 * h)
        assert np.abs(B[:, i] - fd).max() <= 1e-6 * np.abs(fd).max(), i


def test_simp_energy_term_is_the_derivative_of_the_energy():
    # (W'(C E))_i = d(u'K^(x)u)/dx_i at fixed u
    prob = _simp_problem()
    st = _simp_state(prob, 2)
    t = prob.energy_term(st)
    h = 1e-6
    for i in (2, 11, 19):
        xp, xm = st.x.copy(), st.x.copy()
        xp[i] += h
        xm[i] -= h
        fd = (st.u @ (prob.K(xp) @ st.u) - st.u @ (prob.K(xm) @ st.u)) / (2 * h)
        assert abs(t[i] - fd) <= 1e-6 * abs(fd), i


def test_simp_with_p1_and_no_filter_is_the_convex_problem():
    # p = 1, rmin = 1 (W = I): K^ = K(x), B^ = B(u), and the lumped preconditioner
    # matrix equals Z, so Newton system, direction and preconditioner reduce exactly
    g, K0, f = _cantilever((6, 4))
    ps = simp.SimpProblem(g, K0, f, 0.4 * g.m, 3.0, rmin=1.0, p=1.0)
    pc = ip.Problem(g, K0, f, 0.4 * g.m, 3.0)
    st = _simp_state(ps, 3)
    Zs, rs, parts = ps.z_system(st)
    Zc, rc, _ = pc.z_system(st)
    assert np.abs((Zs - Zc).toarray()).max() <= 1e-13 * np.abs(Zc.toarray()).max()
    np.testing.assert_allclose(rs, rc, rtol=1e-13, atol=1e-13 * np.abs(rc).max())
    Zp = ps.z_preconditioner(st, parts)
    assert np.abs((Zp - Zc).toarray()).max() <= 1e-12 * np.abs(Zc.toarray()).max()


def test_simp_newton_step_solves_the_full_block_system():
    # the eliminated system Z with B^ against a dense solve of the Newton system
    # J d = -F with B^ in place of B (Sec. 9), and the lumped preconditioner SPD
    prob = _simp_problem((4, 4))
    st = _simp_state(prob, 4)
    J = prob.jacobian_dense(st)
    d_full = np.linalg.solve(J, -prob.F_vector(st))
    Z, rhs, parts = prob.z_system(st)
    sol = np.linalg.solve(Z.toarray(), rhs)
    dx, dphi, dpsi = prob.recover(st, sol[:-1], sol[-1], parts)
    d_z = np.concatenate([sol[:-1], [sol[-1]], dx, dphi, dpsi])
    np.testing.assert_allclose(d_z, d_full, rtol=1e-9, atol=1e-9 * np.abs(d_full).max())
    # the F3 block of J is minus B^' in u, as the derivative of F3 requires
    n = len(prob.free)
    Ju = J[n + 1:n + 1 + prob.grid.m, :n]
    np.testing.assert_allclose(Ju, -prob.Bmat(st).toarray().T, atol=1e-14)
    Zp = prob.z_preconditioner(st, parts).toarray()
    assert np.abs(Zp - Zp.T).max() <= 1e-12 * np.abs(Zp).max()
    assert np.linalg.eigvalsh(Zp).min() > 0


def test_simp_interior_point_run_converges():
    # Example 4 settings (xbar = 3, rmin = 2, p = 3) on a small grid, direct solves
    prob = _simp_problem((16, 8), xbar=3.0)
    st, log = ip.run(prob, ip.IPParams(stop="kkt", kkt_tol=1e-6, solver="direct", max_newton=200))
    assert log.status == "converged"
    x = st.x
    assert x.min() > 0 and x.max() < 3.0 and abs(x.sum() - prob.V) <= 1e-6 * prob.V
    # at the solution the filtered KKT3 holds up to the barrier terms
    F1, F2, F3, F4, F5 = prob.residuals(st)
    assert np.linalg.norm(F1) <= 1e-2 * np.linalg.norm(prob.f)
