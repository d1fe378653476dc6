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
