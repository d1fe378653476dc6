"""Optimality Conditions methods (oracle; test infrastructure only).

Paper, Sec. 4 (Algorithms OC, DOC and AOC) and Sec. 6.2 (multigrid CG inside OC:
the stopping rule of the outer loop and the adaptive tolerance of the solves).

One update of the densities, for the element energies E_i = u_i'K_i u_i (K_i the
unit element matrix, K(x) = sum_i x_i K_i):
    x_i_new(lambda) = min(x_i * E_i**q / lambda, xbar),
with q = 1 (OC) or the damping exponent q (DOC, typically 1/2), and lambda fixed by
the bisection of Algorithm OC: start from [0, 1e4] and, while the bracket is wider
than tau_lambda = 1e-11, take its midpoint, compute x_new there and keep the half in
which sum x_new = V is crossed (lower end raised when sum x_new > V, upper end
lowered otherwise).  Reading: the listing assigns x = x_new inside the bisection
loop; taken literally every trial would compound the previous one, so x_new is
formed from the fixed current x at every trial and x takes the value of the last
trial when the bracket is narrow enough.
AOC (Algorithm AOC): x1 = OC(x), x2 = OC(x1), x = (x1 + x2)/2, where OC(y) means
one solve at y followed by the update above.

Outer loop (Sec. 6.2): stop when |f'u_k - f'u_{k-1}| <= tau_OC = 1e-5 (eq.
(OCstop)); the relative tolerance of the solves starts at 1e-4 and is multiplied by
0.1 whenever the compliance increases.  feval counts the linear systems solved.
"""
import numpy as np

from . import mg, pcg as pcg_mod

LAMBDA_HI = 1e4
TAU_LAMBDA = 1e-11


def bisect(t, V, xbar, lam_hi=LAMBDA_HI, tau=TAU_LAMBDA):
    """Bisection for lambda with x_new = min(t / lambda, xbar), t = x * E**q.
    Returns (x_new, lambda, number of trials)."""
    lo, hi = 0.0, float(lam_hi)
    lam, xn, steps = None, None, 0
    while hi - lo > tau:
        lam = (hi + lo) / 2.0
        xn = np.minimum(t / lam, xbar)
        steps += 1
        if xn.sum() > V:
            lo = lam
        else:
            hi = lam
    return xn, lam, steps


def update(prob, x, u, q=1.0, lam_hi=LAMBDA_HI, tau=TAU_LAMBDA):
    """One density update of OC (q = 1) or DOC (q < 1) at the displacement u of x."""
    E = prob.energies(u)
    return bisect(x * E ** q, prob.V, prob.xbar, lam_hi, tau)


class OCLog:
    def __init__(self):
        self.outer = 0
        self.feval = 0
        self.pcg_iters = []
        self.compliance = []
        self.cg_tol = []
        self.lam = []
        self.status = "running"


def solve(prob, x, rtol, levels, maxit=1000, solver="mg"):
    """u = K(x)^-1 f: the oracle's MG-PCG (or a sparse direct solve)."""
    K = prob.K(x)
    if solver == "direct":
        import scipy.sparse.linalg as spla
        return spla.spsolve(K.tocsc(), prob.f), 0
    H = mg.Hierarchy(prob.grid, K, levels)
    res = pcg_mod.mg_pcg(H, prob.f, rtol, maxit)
    return res.z, res.iters


def run(prob, x0, variant="oc", q=0.5, tau_oc=1e-5, cg_tol=1e-4, levels=4, max_outer=10000,
        solver="mg", lam_hi=LAMBDA_HI, tau_lam=TAU_LAMBDA):
    """Algorithm OC / DOC / AOC with the stopping rule and tolerance rule of Sec. 6.2.
    Returns (x, u, log)."""
    log = OCLog()
    qq = q if variant == "doc" else 1.0
    x = np.array(x0, dtype=np.float64)
    tol = float(cg_tol)

    def solve_at(y):
        u, it = solve(prob, y, tol, levels, solver=solver)
        log.feval += 1
        log.pcg_iters.append(it)
        return u

    u = solve_at(x)
    c_prev = float(prob.f @ u)
    log.compliance.append(c_prev)
    while log.outer < max_outer:
        if variant == "aoc":
            x1, _, _ = update(prob, x, u, 1.0, lam_hi, tau_lam)
            u1 = solve_at(x1)
            x2, lam, _ = update(prob, x1, u1, 1.0, lam_hi, tau_lam)
            x = 0.5 * (x1 + x2)
        else:
            x, lam, _ = update(prob, x, u, qq, lam_hi, tau_lam)
        u = solve_at(x)
        c = float(prob.f @ u)
        log.outer += 1
        log.compliance.append(c)
        log.lam.append(lam)
        log.cg_tol.append(tol)
        if c > c_prev:
            tol *= 0.1
        if abs(c - c_prev) <= tau_oc:
            log.status = "converged"
            return x, u, log
        c_prev = c
    log.status = "max_outer"
    return x, u, log
