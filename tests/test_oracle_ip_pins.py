"""Hand-computed pins of the oracle's step length (Sec. 3.3) and of its
Newton-test / duality-gap measures (Sec. 3.4), no GPU.

Every expected value below is worked out by hand from the formulas of the
paper, on inputs small enough to do so; none is produced by the function under
test.  Each case is chosen so that a plausible slip changes the result: the
fraction 0.9 applied after the minimum with 1, the wrong sign set of d_x for
either bound, the bound measured from the wrong side, the rule left off phi or
psi, F3 used where G3 belongs, or a flipped sign inside G3 or the gap."""
import numpy as np
import pytest

from oracle import fem, ip


def _st(x, phi=(1.0, 1.0), psi=(1.0, 1.0)):
    return ip.IPState(None, 0.0, np.array(x, float), np.array(phi, float), np.array(psi, float), 0.0, 0.0)


Z2 = np.zeros(2)

# (state, d_x, d_phi, d_psi, expected alpha with the rule on all blocks, expected
# alpha with the rule on x only); xbar = 1, fraction 0.9.
STEP_CASES = {
    # lower bound binds: 0.9 * 0.5 / 1 = 0.45 (the upper ratio 0.9 * 0.5 / 0.1 = 4.5)
    "lower": (_st([0.5, 0.5]), [-1.0, 0.1], Z2, Z2, 0.45, 0.45),
    # upper bound binds: 0.9 * min(0.8 / 0.1, 0.1 / 0.5) = 0.18; no d_x < 0 (alpha_l = inf)
    "upper": (_st([0.2, 0.9]), [0.1, 0.5], Z2, Z2, 0.18, 0.18),
    # both ratios 0.9 * 0.5 / 0.1 = 4.5 > 1: the full step
    "one": (_st([0.5, 0.5]), [-0.1, 0.1], Z2, Z2, 1.0, 1.0),
    # phi binds: 0.9 * min(1 / 4) = 0.225 (positive d_phi and d_psi never bind)
    "phi": (_st([0.5, 0.5], phi=[1.0, 2.0]), [-0.1, 0.1], [-4.0, 1.0], [0.5, 0.5], 0.225, 1.0),
    # psi binds: 0.9 * min(3 / 1, 1 / 10) = 0.09
    "psi": (_st([0.5, 0.5], psi=[3.0, 1.0]), [-0.1, 0.1], Z2, [-1.0, -10.0], 0.09, 1.0),
    # d = 0: every set is empty
    "empty": (_st([0.5, 0.5]), Z2, Z2, Z2, 1.0, 1.0),
    # lower and upper ratios of the same size on different elements: 0.9 * min(0.3/0.6, 0.3/0.5)
    "mixed": (_st([0.3, 0.7]), [-0.6, 0.5], Z2, Z2, 0.45, 0.45),
}


@pytest.mark.parametrize("name", sorted(STEP_CASES))
def test_step_length_hand_cases(name):
    st, dx, dphi, dpsi, a_all, a_x = STEP_CASES[name]
    dx, dphi, dpsi = (np.array(v, float) for v in (dx, dphi, dpsi))
    assert ip.step_length(st, dx, dphi, dpsi, 1.0, 0.9, True) == pytest.approx(a_all, rel=1e-15)
    assert ip.step_length(st, dx, dphi, dpsi, 1.0, 0.9, False) == pytest.approx(a_x, rel=1e-15)
    # the defaults are the paper's fraction 0.9 with the rule on every block
    assert ip.step_length(st, dx, dphi, dpsi, 1.0) == pytest.approx(a_all, rel=1e-15)


def test_paper_constants_are_the_defaults():
    # Sec. 3.2 (sigma = 0.2), Sec. 3.3 (fraction 0.9), Sec. 3.4 (tau_NWT = 0.1),
    # Sec. 8.1 (at most 1000 PCG iterations per system)
    p = ip.IPParams()
    assert (p.sigma, p.frac, p.tau_nwt, p.pcg_maxit) == (0.2, 0.9, 0.1, 1000)


def test_step_length_fraction_and_bound():
    # xbar = 2: the upper distance is 2 - x; fraction 0.5 halves the ratio
    st = _st([0.5, 1.5])
    a = ip.step_length(st, np.array([0.2, 1.0]), Z2, Z2, 2.0, 0.5, True)
    assert a == pytest.approx(0.5 * min(1.5 / 0.2, 0.5 / 1.0), rel=1e-15)


def test_measures_closed_form():
    """2 x 1 grid, u = unit y-displacement of the corner node (2, 0), which lies in
    element 1 only.  With the square-element K0 every diagonal entry is
    E (3 - nu) / (6 (1 - nu^2)), so element 1 has energy u_e'K0u_e = Ekk and
    element 0 none.  f = K(x) u + g with g = 0.3 on the x-DOF of node (1, 1), so
    F1 = -g and f'u = x_1 Ekk.  With F3 + F4/x - F5/(xbar - x) the phi and psi
    terms cancel: G3_e = -Ekk_e / 2 - lambda - s / x_e + r / (xbar - x_e)."""
    nu = 0.3
    Ekk = (3.0 - nu) / (6.0 * (1.0 - nu * nu))
    g = fem.Grid((2, 1))
    K0 = fem.element_stiffness(2, 1.0, nu)
    assert np.allclose(np.diag(K0), Ekk, rtol=1e-14)
    # slots by hand: node (i, j) -> 3 j + i, slot 2 node + c; element 1 has the nodes
    # (1,0), (2,0), (2,1), (1,1) = 1, 2, 5, 4 in local order
    e1_slots = [2, 3, 4, 5, 10, 11, 8, 9]
    x = np.array([0.5, 0.25])
    f = np.zeros(g.nslots)
    f[e1_slots] = x[1] * K0[:, 3]             # K(x) u: column of local DOF 3 (node (2,0), y)
    f[8] += 0.3                               # g on node (1, 1), x component
    free = [2, 3, 4, 5, 8, 9, 10, 11]         # slots of nodes with i >= 1
    assert list(g.free_to_slot()) == free
    u = np.zeros(len(free))
    u[free.index(5)] = 1.0
    V, xbar, lam, s, r = 0.6, 1.0, 0.1, 0.04, 0.06
    phi, psi = np.array([2.0, 1.0]), np.array([3.0, 0.5])
    prob = ip.Problem(g, K0, f, V, xbar)
    st = ip.IPState(u, lam, x, phi, psi, s, r)

    G3 = np.array([-lam - s / 0.5 + r / 0.5, -Ekk / 2 - lam - s / 0.25 + r / 0.75])
    nwt = 0.3 / np.linalg.norm(f) + np.hypot(*G3) / (np.sqrt(4.0 + 1.0) + np.sqrt(9.0 + 0.25))
    gap = (2.0 * 0.5 + 1.0 * 0.25 + 3.0 * 0.5 + 0.5 * 0.75) / (0.25 * Ekk)
    for mf in (False, True):
        n, gp, F2 = prob.measures(st, matrix_free=mf)
        assert n == pytest.approx(nwt, rel=1e-13)
        assert gp == pytest.approx(gap, rel=1e-13)
        assert F2 == pytest.approx(0.75 - V, rel=1e-13)
    F1, F2, F3, F4, F5 = prob.residuals(st)
    assert np.allclose(F1, -0.3 * (np.array(free) == 8), atol=1e-15)
    np.testing.assert_allclose(F3, [-lam - 2.0 + 3.0, -Ekk / 2 - lam - 1.0 + 0.5], rtol=1e-14)
    np.testing.assert_allclose(F4, [2.0 * 0.5 - s, 1.0 * 0.25 - s], rtol=1e-14)
    np.testing.assert_allclose(F5, [3.0 * 0.5 - r, 0.5 * 0.75 - r], rtol=1e-14)


def test_newton_solve_acceptance_rule():
    # Sec. 6 stopping rule: a solve stopped by the iteration limit is an inexact
    # direction only within accept_rtol; a breakdown never is
    p = ip.IPParams(accept_rtol=1e-2)
    assert ip.accept_solve("ok", 0.0, p) is False
    assert ip.accept_solve("maxit", 1e-3, p) is True
    assert ip.accept_solve("maxit", 1e-2, p) is True
    with pytest.raises(ip.NewtonSolveError):
        ip.accept_solve("maxit", 2e-2, p)
    with pytest.raises(ip.NewtonSolveError):
        ip.accept_solve("breakdown", 1e-9, p)
