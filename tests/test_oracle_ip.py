"""Pins of the oracle's interior-point method and sensitivities (no GPU)."""
import os

import numpy as np
import pytest
import scipy.optimize as so

from oracle import fem, ip, sens

HERE = os.path.dirname(os.path.abspath(__file__))


def _problem(nel=(8, 4), vfrac=0.5, xbar=1.0):
    g = fem.Grid(nel)
    K0 = fem.element_stiffness(g.dim)
    f = fem.load_vector(g, [((nel[0],) + tuple(v // 2 for v in nel[1:]), 1, -1.0)])
    return ip.Problem(g, K0, f, vfrac * g.m, xbar)


def _perturbed_state(prob, seed=0):
    rng = np.random.default_rng(seed)
    m, n = prob.grid.m, len(prob.free)
    x = rng.uniform(0.2, 0.8, m)
    return ip.IPState(rng.standard_normal(n) * 10, 0.7, x, rng.uniform(0.5, 2, m),
                      rng.uniform(0.5, 2, m), 0.3, 0.2)


def test_jacobian_matches_central_differences():
    prob = _problem((4, 2))
    st = _perturbed_state(prob)
    J = prob.jacobian_dense(st)
    z0 = np.concatenate([st.u, [st.lam], st.x, st.phi, st.psi])
    n, m = len(prob.free), prob.grid.m

    def F(z):
        s = ip.IPState(z[:n], z[n], z[n + 1:n + 1 + m], z[n + 1 + m:n + 1 + 2 * m],
                       z[n + 1 + 2 * m:], st.s, st.r)
        return prob.F_vector(s)

    h = 1e-6
    Jfd = np.zeros_like(J)
    for k in range(len(z0)):
        e = np.zeros_like(z0)
        e[k] = h
        Jfd[:, k] = (F(z0 + e) - F(z0 - e)) / (2 * h)
    assert np.abs(J - Jfd).max() < 1e-6 * max(1.0, np.abs(J).max())


def test_z_route_equals_full_newton_solve():
    prob = _problem((8, 4))
    st = _perturbed_state(prob, 1)
    J = prob.jacobian_dense(st)
    d_full = np.linalg.solve(J, -prob.F_vector(st))
    Z, rhs, parts = prob.z_system(st)
    sol = np.linalg.solve(Z.toarray(), rhs)
    du, dlam = sol[:-1], sol[-1]
    dx, dphi, dpsi = prob.recover(st, du, dlam, parts)
    d_z = np.concatenate([du, [dlam], dx, dphi, dpsi])
    np.testing.assert_allclose(d_z, d_full, rtol=1e-9, atol=1e-9 * np.abs(d_full).max())
    Zd = Z.toarray()
    np.testing.assert_allclose(Zd, Zd.T, atol=1e-12 * np.abs(Zd).max())
    assert np.linalg.eigvalsh(Zd).min() > 0


def test_barrier_reduction_counts_table7():
    rows = []
    with open(os.path.join(HERE, "golden", "barrier_counts.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                t, k = line.split()
                rows.append((float(t), int(k)))
    prob = _problem((8, 4), xbar=1.0)
    for tau, expect in rows[:1]:
        params = ip.IPParams(stop="barrier", tau_ip=tau, solver="direct")
        st, log = ip.run(prob, params)
        assert log.status == "converged"
        assert log.barrier_updates == expect
    for tau, expect in rows:
        k, s = 0, 1.0
        while s > tau:
            s *= 0.2
            k += 1
        assert k == expect


@pytest.fixture(scope="module")
def ip_solution():
    prob = _problem((8, 4))
    params = ip.IPParams(stop="kkt", kkt_tol=1e-6, solver="mg", levels=3)
    st, log = ip.run(prob, params)
    return prob, st, log


def test_ip_terminal_conditions(ip_solution):
    prob, st, log = ip_solution
    assert log.status == "converged"
    assert np.all(st.x > 0) and np.all(st.x < prob.xbar)
    assert np.all(st.phi > 0) and np.all(st.psi > 0)
    assert abs(st.x.sum() - prob.V) <= 1e-8 * prob.V
    F1, F2, F3, F4, F5 = prob.residuals(st)
    assert np.linalg.norm(F1) <= 1e-2 * np.linalg.norm(prob.f)
    assert log.gap[-1] <= 1e-6 and log.nwt[-1] <= 0.1
    # complementarity: phi_i x_i and psi_i (xbar - x_i) sit near the final barrier value
    assert np.all(st.phi * st.x < 10 * st.s / 0.2) and np.all(st.psi * (prob.xbar - st.x) < 10 * st.r / 0.2)
    assert np.all(np.isfinite(log.alpha)) and min(log.alpha) > 0


def test_ip_volume_kept_along_path():
    prob = _problem((8, 4))
    params = ip.IPParams(stop="kkt", kkt_tol=1e-6, solver="mg", levels=3, pcg_rtol=1e-10)
    vols = []
    ip.run(prob, params, callback=lambda st, log: vols.append(st.x.sum()))
    assert max(abs(v - prob.V) for v in vols) <= 1e-7 * prob.V


def test_ip_matches_independent_convex_solve(ip_solution):
    # Compliance f'K(x)^-1 f minimised over {sum x = V, 0 <= x <= xbar} by an unrelated
    # trust-region solver with the exact gradient -u_e'K0u_e.
    prob, st, log = ip_solution
    g, K0 = prob.grid, prob.K0

    def obj(x):
        c, grad, _ = sens.compliance_gradient(g, x, K0, prob.f_slots)
        return c, grad

    cons = so.LinearConstraint(np.ones((1, g.m)), prob.V, prob.V)
    res = so.minimize(obj, np.full(g.m, prob.V / g.m), jac=True, method="trust-constr",
                      constraints=[cons], bounds=so.Bounds(1e-9, prob.xbar),
                      options={"maxiter": 3000, "gtol": 1e-10, "xtol": 1e-14})
    c_ip = float(prob.f @ st.u)
    c_ref = obj(res.x)[0]
    assert abs(c_ip - c_ref) <= 1e-4 * c_ref
    assert c_ip <= c_ref * (1 + 1e-4)


def test_self_adjoint_and_euler_identity():
    g = fem.Grid((8, 4))
    K0 = fem.element_stiffness(2)
    x = np.random.default_rng(3).uniform(0.01, 1.0, g.m)
    f = fem.load_vector(g, [((8, 2), 1, -1.0)])
    gv = np.random.default_rng(33).standard_normal(g.nslots)
    # J = f'u: adjoint equals u
    J, grad, u, lam = sens.linear_objective_gradient(g, x, K0, f, np.zeros(g.nslots))
    np.testing.assert_allclose(lam, u, rtol=0, atol=1e-14 * np.abs(u).max())
    # Euler: J(t x) = J(x)/t  =>  sum x_e dJ/dx_e = -J
    J, grad, u, lam = sens.linear_objective_gradient(g, x, K0, f, gv)
    assert abs(x @ grad + J) <= 1e-10 * abs(J)


def test_gradient_central_differences():
    g = fem.Grid((8, 4))
    K0 = fem.element_stiffness(2)
    x = np.random.default_rng(3).uniform(0.01, 1.0, g.m)
    f = fem.load_vector(g, [((8, 2), 1, -1.0)])
    gv = np.random.default_rng(33).standard_normal(g.nslots)
    J, grad, _, _ = sens.linear_objective_gradient(g, x, K0, f, gv)
    for e in (0, 5, 17, 31):
        h = 1e-5 * x[e]
        xp, xm = x.copy(), x.copy()
        xp[e] += h
        xm[e] -= h
        Jp = sens.linear_objective_gradient(g, xp, K0, f, gv)[0]
        Jm = sens.linear_objective_gradient(g, xm, K0, f, gv)[0]
        fd = (Jp - Jm) / (2 * h)
        assert abs(fd - grad[e]) <= 1e-6 * np.abs(grad).max(), e


def test_z_vcycle_needs_and_gets_damping_safeguard():
    # Late interior-point iterate: plain omega = 0.6 Jacobi diverges on Z (the V-cycle is
    # indefinite); the safeguarded weights restore a symmetric positive definite V-cycle.
    from oracle import mg
    prob = _problem((32, 16))
    params = ip.IPParams(stop="barrier", tau_ip=1e-5, solver="direct")
    st, log = ip.run(prob, params)
    Z, rhs, parts = prob.z_system(st)
    rho = mg.jacobi_radius(Z, Z.diagonal(), mg.power_start(prob.grid, True), steps=200)
    assert 0.6 * rho > 2.0
    H = mg.Hierarchy(prob.grid, Z, 3, augmented=True, safeguard=True)
    assert max(w * r for w, r in zip(H.omega[1:], H.rho[1:])) <= mg.SAFE_PRODUCT + 1e-12
    M = mg.vcycle_matrix(H)
    assert np.abs(M - M.T).max() < 1e-10 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0
    H0 = mg.Hierarchy(prob.grid, Z, 3, augmented=True, safeguard=False)
    assert np.linalg.eigvalsh(0.5 * (mg.vcycle_matrix(H0) + mg.vcycle_matrix(H0).T)).min() < 0


@pytest.mark.slow
def test_ip_64x32_mg_matches_direct():
    # The 64x32 cantilever run: MG-PCG (1e-8) and exact solves follow the same path.
    prob = _problem((64, 32))
    out = {}
    for solver in ("mg", "direct"):
        params = ip.IPParams(stop="kkt", kkt_tol=1e-6, solver=solver, levels=4)
        st, log = ip.run(prob, params)
        assert log.status == "converged"
        out[solver] = (log.newton, log.barrier_updates, float(prob.f @ st.u))
    assert abs(out["mg"][0] - out["direct"][0]) <= 1
    assert out["mg"][1] == out["direct"][1]
    assert abs(out["mg"][2] - out["direct"][2]) <= 1e-6 * out["direct"][2]


def test_matrix_free_measures_equal_assembled():
    # The element-by-element residual (for grids too large to assemble) equals
    # the assembled one.
    from paper_1606_06201_amd import inputs
    nel = (6, 4, 4)
    g = fem.Grid(nel)
    K0 = fem.element_stiffness(3)
    prob = ip.Problem(g, K0, fem.load_vector(g, inputs.point_load(nel)), 0.3 * g.m, 1.0)
    rng = np.random.default_rng(4)
    st = ip.IPState(rng.standard_normal(len(prob.f)), 0.4, rng.uniform(0.1, 0.9, g.m),
                     rng.uniform(0.5, 2, g.m), rng.uniform(0.5, 2, g.m), 0.1, 0.1)
    a, b = prob.measures(st), prob.measures(st, matrix_free=True)
    np.testing.assert_allclose(a, b, rtol=1e-13)
