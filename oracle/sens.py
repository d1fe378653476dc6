"""Element sensitivities and the adjoint gradient (oracle; test infrastructure only).

For K(x) u = f with K(x) = sum_e x_e K_e (Sec. 1, problem (1)) and an objective
J(u), the adjoint lambda solves K lambda = dJ/du (K is symmetric) and
dJ/dx_e = -lambda_e' K_e u_e.  For the paper's compliance objective (1/2) f'u
the adjoint is u/2, giving the term -(1/2) u' K_i u of the KKT condition
(KKT3) in Sec. 2.
"""
import numpy as np
import scipy.sparse.linalg as spla

from . import fem


def element_products(grid, K0, w_slots, u_slots):
    """(w_e' K0 u_e) for every element e (local gathers of two slot vectors)."""
    we = fem.element_values(grid, w_slots)
    ue = fem.element_values(grid, u_slots)
    return np.einsum("ei,ij,ej->e", we, K0, ue)


def direct_solve(grid, x, K0, rhs_slots):
    """Exact reference solve K(x) u = rhs on the free DOFs (sparse LU of the SPD
    matrix in symmetric mode, no pivoting); returns a slot vector."""
    K = fem.stiffness_free(grid, x, K0).tocsc()
    lu = spla.splu(K, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                   options={"SymmetricMode": True})
    return fem.to_slots(grid, lu.solve(fem.to_free(grid, rhs_slots)))


def linear_objective_gradient(grid, x, K0, f_slots, g_slots, solve=None):
    """J = g'u + f'u with K(x) u = f.  Returns (J, dJ/dx, u, lambda) where
    K lambda = g + f and dJ/dx_e = -lambda_e' K0 u_e."""
    solve = solve or (lambda rhs: direct_solve(grid, x, K0, rhs))
    u = solve(f_slots)
    lam = solve(np.asarray(g_slots) + np.asarray(f_slots))
    J = float(np.dot(g_slots, u) + np.dot(f_slots, u))
    grad = -element_products(grid, K0, lam, u)
    return J, grad, u, lam


def compliance_gradient(grid, x, K0, f_slots, solve=None):
    """c = f'u; dc/dx_e = -u_e' K0 u_e (self-adjoint: lambda = u)."""
    solve = solve or (lambda rhs: direct_solve(grid, x, K0, rhs))
    u = solve(f_slots)
    return float(np.dot(f_slots, u)), -element_products(grid, K0, u, u), u
