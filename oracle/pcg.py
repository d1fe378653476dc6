"""Preconditioned conjugate gradients (oracle; test infrastructure only).

Paper, Sec. 5.2 (Algorithm PCG) with one V-cycle as the preconditioner.  The
paper's sign convention is kept: the residual is r = A z - b, the first search
direction p = -y with y the preconditioned residual.

Readings:
  * search-direction update: the paper lists p := -y + beta p before y := y~;
    the only reading consistent with its beta (the Fletcher-Reeves ratio
    r~'y~ / r'y) and with the cited textbook method is p := -y~ + beta p;
  * stopping test: the printed criterion "||rho|| ||b|| <= tol" (eq. (cgstop),
    Sec. 6.1) is read as the relative residual ||rho||_2 / ||b||_2 <= tol,
    tested after each residual update; on success the true residual
    ||A z - b|| / ||b|| is recomputed and, if it fails the test, the iteration
    restarts from r := A z - b (the restart costs no counted iteration);
  * at most maxit iterations per system (1000, Sec. 8.1).
"""
import numpy as np


class PCGResult:
    def __init__(self, z, iters, relres, true_relres, converged, restarts, history, status):
        self.z = z
        self.iters = iters
        self.relres = relres
        self.true_relres = true_relres
        self.converged = converged
        self.restarts = restarts
        self.history = history
        self.status = status


def pcg(apply_A, b, precond, rtol=1e-8, maxit=1000, z0=None, flexible=False):
    """flexible=True replaces the ratio r~'y~ / r'y by the Polak-Ribiere form
    r~'(y~ - y) / r'y (inexact / flexible PCG, an option beyond the paper's
    Algorithm PCG for a preconditioner that varies slightly between applications,
    such as a V-cycle evaluated in reduced precision).  In exact arithmetic with a
    fixed symmetric preconditioner both forms coincide (pinned); the varying case
    has no closed form to pin against (parity unpinned)."""
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    z = np.zeros_like(b) if z0 is None else np.array(z0, dtype=np.float64)
    if bnorm == 0.0:
        return PCGResult(np.zeros_like(b), 0, 0.0, 0.0, True, 0, [], "ok")
    r = apply_A(z) - b
    history = [float(np.linalg.norm(r)) / bnorm]
    iters, restarts = 0, 0
    if history[-1] <= rtol:
        return PCGResult(z, 0, history[-1], history[-1], True, 0, history, "ok")
    y = precond(r)
    p = -y
    rho = float(r @ y)
    if not rho > 0.0:
        return PCGResult(z, 0, history[-1], history[-1], False, 0, history, "breakdown")
    while iters < maxit:
        q = apply_A(p)
        pq = float(p @ q)
        if not pq > 0.0:
            rel = float(np.linalg.norm(apply_A(z) - b)) / bnorm
            return PCGResult(z, iters, history[-1], rel, False, restarts, history, "breakdown")
        alpha = rho / pq
        z = z + alpha * p
        r = r + alpha * q
        iters += 1
        rel = float(np.linalg.norm(r)) / bnorm
        history.append(rel)
        if rel <= rtol:
            rt = apply_A(z) - b
            true_rel = float(np.linalg.norm(rt)) / bnorm
            if true_rel <= rtol:
                return PCGResult(z, iters, rel, true_rel, True, restarts, history, "ok")
            restarts += 1
            r = rt
            y = precond(r)
            p = -y
            rho = float(r @ y)
            continue
        y_new = precond(r)
        rho_new = float(r @ y_new)
        if not rho_new > 0.0:
            true_rel = float(np.linalg.norm(apply_A(z) - b)) / bnorm
            return PCGResult(z, iters, rel, true_rel, False, restarts, history, "breakdown")
        beta = (rho_new - float(r @ y)) / rho if flexible else rho_new / rho
        y = y_new
        p = -y + beta * p
        rho = rho_new
    true_rel = float(np.linalg.norm(apply_A(z) - b)) / bnorm
    return PCGResult(z, iters, history[-1], true_rel, False, restarts, history, "maxit")


def mg_pcg(H, b, rtol=1e-8, maxit=1000, z0=None, nu1=2, nu2=2, flexible=False, A=None):
    """PCG on the finest operator of hierarchy H (or on the matrix A, when given)
    with one V-cycle of H per step (the damping weights live in the hierarchy)."""
    from . import mg
    A = H.A[-1] if A is None else A
    return pcg(lambda v: A @ v, b, lambda r: mg.vcycle(H, r, nu1, nu2), rtol, maxit, z0, flexible)
