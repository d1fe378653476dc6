"""Pins of the oracle's Optimality Conditions methods (Sec. 4, Sec. 6.2), no GPU."""
import numpy as np
import pytest

from oracle import fem, ip, oc


def test_bisection_closed_form_unclamped():
    # no bound active: sum t / lambda = V gives lambda = sum t / V = 10 / 5 = 2
    t = np.array([1.0, 2.0, 3.0, 4.0])
    x, lam, steps = oc.bisect(t, 5.0, 100.0)
    assert abs(lam - 2.0) <= 2e-11
    assert abs(x.sum() - 5.0) <= 1e-10
    # 1e4 / 2^n <= 1e-11 first at n = 50 (2^49 < 1e15 < 2^50)
    assert steps == 50


def test_bisection_closed_form_clamped():
    # x_0 = min(10 / lambda, 2) = 2 at the solution, the others 1 / lambda: 2 + 2 / lambda = 3
    t = np.array([10.0, 1.0, 1.0])
    x, lam, _ = oc.bisect(t, 3.0, 2.0)
    assert abs(lam - 2.0) <= 2e-11
    np.testing.assert_allclose(x, [2.0, 0.5, 0.5], rtol=1e-10)


def test_bisection_bracket_rule():
    # the lower end rises while the sum is above V: a multiplier above the upper
    # bracket end cannot be reached, the trials stop at lam_hi
    t = np.array([1e6, 1e6])
    x, lam, _ = oc.bisect(t, 1.0, 1e9, lam_hi=1e4)
    assert 1e4 - lam <= 2e-11 and x.sum() > 1.0


def _problem(nel=(8, 4)):
    g = fem.Grid(nel)
    K0 = fem.element_stiffness(2)
    f = fem.load_vector(g, [((nel[0], nel[1] // 2), 1, -1.0)])
    return ip.Problem(g, K0, f, 0.5 * g.m, 1.0)


@pytest.fixture(scope="module")
def ip_optimum():
    prob = _problem()
    st, log = ip.run(prob, ip.IPParams(stop="kkt", kkt_tol=1e-9, solver="direct"))
    assert log.status == "converged"
    return prob, float(prob.f @ st.u)


@pytest.mark.parametrize("variant", ["oc", "doc", "aoc"])
def test_oc_variants_reach_the_convex_optimum(ip_optimum, variant):
    # the problem is convex: every OC fixed point with x > 0 satisfies the optimality
    # conditions (KKT3 without active bounds), so all three methods approach the
    # optimal compliance of the interior-point method (itself pinned against an
    # independent convex solver)
    prob, c_opt = ip_optimum
    x0 = np.full(prob.grid.m, prob.V / prob.grid.m)
    x, u, log = oc.run(prob, x0, variant=variant, tau_oc=1e-9, solver="direct", max_outer=20000)
    assert log.status == "converged"
    c = float(prob.f @ u)
    assert abs(c - c_opt) <= 1e-5 * c_opt, (c, c_opt)
    assert abs(x.sum() - prob.V) <= 1e-9 * prob.V
    assert x.min() >= 0.0 and x.max() <= prob.xbar
    # feasible descent: the compliance never rises by more than the solve tolerance
    assert all(b <= a * (1 + 1e-9) for a, b in zip(log.compliance, log.compliance[1:]))


def test_oc_update_is_the_optimality_condition():
    # at a fixed point every element strictly inside the bounds has E_i = lambda
    prob = _problem((4, 2))
    x0 = np.full(prob.grid.m, prob.V / prob.grid.m)
    x, u, log = oc.run(prob, x0, variant="aoc", tau_oc=1e-13, solver="direct", max_outer=50000)
    E = prob.energies(u)
    inner = (x > 1e-3) & (x < prob.xbar - 1e-3)
    assert inner.sum() >= 2
    assert np.ptp(E[inner]) <= 1e-4 * E[inner].mean()
