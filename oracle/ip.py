"""Primal-dual interior-point method (oracle; test infrastructure only).

Paper, Sec. 2 (KKT conditions, Newton system, elimination, augmented system Z)
and Sec. 3 (algorithm, barrier update, step length, stopping rules).

Unknowns z = (u, lambda, x, phi, psi) with barrier parameters s, r.  With
F = -Res (eqs. (KKT1), (KKT2), (KKT3), (KKT4p), (KKT5p)):
  F1 = K(x) u - f,  F2 = sum x - V,  F3_e = -1/2 u_e'K_e u_e - lambda - phi_e + psi_e,
  F4 = phi o x - s,  F5 = psi o (xbar - x) - r.
Each Newton step solves J d = -F, J the Jacobian of F, through the augmented
system Z of eq. (nwtr2Z): with D = phi/x + psi/(xbar-x),
G3 = F3 + F4/x - F5/(xbar-x) (= -Res~(3)) and B = (K_1 u, ..., K_m u),
  Z = [[K + B D^-1 B', B D^-1 e], [e' D^-1 B', e' D^-1 e]],
  Z [d_u; d_lambda] = [-F1 + B D^-1 G3; -F2 + e' D^-1 G3],
  d_x = D^-1 (B' d_u + e d_lambda - G3),
  d_phi = (-F4 - phi o d_x)/x,  d_psi = (-F5 + psi o d_x)/(xbar - x).
Readings (the paper's printed signs are not mutually consistent): the block
system is derived from J d = -F as above; the elimination formulas (phipsi)
use d_x where d_t is printed and the sign of the psi term follows from the
fifth block row; the d_x recovery (nwtr2Za) uses d_u, d_lambda where the
residuals are printed.  The dense full-system solve in the tests checks all
of this mechanically.

Newton-system solves (Sec. 6, stopping rule): a solve that reaches pcg_rtol
gives the direction; one stopped by the iteration limit is taken as an inexact
direction only if its true relative residual is within accept_rtol (1e-2, the
paper's own inexact stopping rule, eq. (cgstop)); a breakdown, or a larger
residual, ends the run with status "solve_failed".

Step length (Sec. 3.3): fraction 0.9 of the distance to the bounds 0 < x < xbar,
alpha <= 1; by default the same rule keeps phi, psi > 0 (the text asks for
strict feasibility of all of (KKT6); flag `step_all_blocks`).
Newton stop (Sec. 3.4): ||F1||/||f|| + ||G3||/(||phi|| + ||psi||) <= tau_NWT
  -> s, r <- sigma s, sigma r (Sec. 3.2, sigma = 0.2).
Overall stop: either the paper's rule max(s, r) <= tau_IP (eq. (crit:ip)),
checked after each barrier update, or a scaled KKT residual after the Remark
in Sec. 3.4.  The Remark adds to the Newton-test quantity the complementarity
cosines phi'x/(||phi|| ||x||) and psi'(xbar-x)/(||phi|| ||x||).  Two readings:
(i) the Newton-test part never falls much below tau_NWT in this inexact
path-following scheme (one or two Newton steps per barrier value), so the
tolerance is applied to the complementarity part at iterates that pass the
Newton test; (ii) the cosines are invariant under scaling phi, psi and do not
tend to zero when one bound is inactive at the solution, so complementarity is
measured as the duality gap relative to the compliance,
  gap = (phi'x + psi'(xbar - x)) / f'u.
Stop when ||F1||/||f|| + ||G3||/(||phi|| + ||psi||) <= tau_NWT and gap <= tol.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem, mg, pcg as pcg_mod


class IPParams:
    def __init__(self, sigma=0.2, tau_nwt=0.1, pcg_rtol=1e-8, pcg_maxit=1000,
                 frac=0.9, stop="kkt", kkt_tol=1e-6, tau_ip=1e-8, max_newton=300,
                 step_all_blocks=True, solver="mg", levels=4, omega=0.6, nu1=2, nu2=2,
                 accept_rtol=1e-2, cg_tol_factor=1.0):
        self.__dict__.update(locals())
        del self.__dict__["self"]


class IPState:
    def __init__(self, u, lam, x, phi, psi, s, r):
        self.u, self.lam, self.x, self.phi, self.psi = u, lam, x, phi, psi
        self.s, self.r = s, r

    def copy(self):
        return IPState(self.u.copy(), float(self.lam), self.x.copy(), self.phi.copy(),
                       self.psi.copy(), float(self.s), float(self.r))


class Problem:
    """Minimum compliance, problem (1), on a structured grid (free-DOF vectors)."""

    def __init__(self, grid, K0, f_slots, V, xbar):
        self.grid, self.K0 = grid, K0
        self.f_slots = np.asarray(f_slots, dtype=np.float64)
        self.f = fem.to_free(grid, self.f_slots)
        self.V, self.xbar = float(V), float(xbar)
        self.free = grid.free_to_slot()
        self.edofs = grid.element_dofs()
        # position of each element slot in the free vector (-1 if clamped)
        pos = -np.ones(grid.nslots, dtype=np.int64)
        pos[self.free] = np.arange(len(self.free))
        self.epos = pos[self.edofs]

    def K(self, x):
        return fem.stiffness_free(self.grid, x, self.K0)

    def elem(self, v_free):
        ve = np.zeros(self.epos.shape)
        mask = self.epos >= 0
        ve[mask] = v_free[self.epos[mask]]
        return ve

    def B(self, u):
        """B(u) = (K_1 u, ..., K_m u) as a sparse n_free x m matrix."""
        g = self.elem(u) @ self.K0           # rows g_e = K0 u_e (K0 symmetric)
        m, nd = g.shape
        mask = self.epos >= 0
        rows = self.epos[mask]
        cols = np.repeat(np.arange(m), nd).reshape(m, nd)[mask]
        return sp.csr_matrix((g[mask], (rows, cols)), shape=(len(self.free), m))

    def energies(self, u):
        ue = self.elem(u)
        return np.einsum("ei,ij,ej->e", ue, self.K0, ue)

    def Bmat(self, st):
        """The matrix B of the Newton system at st (B(u) for problem (1))."""
        return self.B(st.u)

    def energy_term(self, st):
        """u' [dK/dx_i] u per design variable, the energy part of F3 (KKT3)."""
        return self.energies(st.u)

    def z_preconditioner(self, st, parts):
        """Matrix whose multigrid hierarchy preconditions Z (None: Z itself)."""
        return None

    def residuals(self, st, matrix_free=False):
        """F1..F5 (Sec. 2).  matrix_free: K(x) u element by element instead of the
        assembled matrix (same sum; for grids too large to assemble)."""
        if matrix_free:
            Ku = fem.apply_free_masked(self.grid, st.x, self.K0, fem.to_slots(self.grid, st.u))
            F1 = fem.to_free(self.grid, Ku) - self.f
        else:
            F1 = self.K(st.x) @ st.u - self.f
        F2 = float(st.x.sum() - self.V)
        F3 = -0.5 * self.energy_term(st) - st.lam - st.phi + st.psi
        F4 = st.phi * st.x - st.s
        F5 = st.psi * (self.xbar - st.x) - st.r
        return F1, F2, F3, F4, F5

    def measures(self, st, matrix_free=False):
        F1, F2, F3, F4, F5 = self.residuals(st, matrix_free)
        xt = self.xbar - st.x
        G3 = F3 + F4 / st.x - F5 / xt
        nphi, npsi = np.linalg.norm(st.phi), np.linalg.norm(st.psi)
        nwt = np.linalg.norm(F1) / np.linalg.norm(self.f) + np.linalg.norm(G3) / (nphi + npsi)
        gap = (st.phi @ st.x + st.psi @ xt) / float(self.f @ st.u)
        return float(nwt), float(gap), F2

    # --- Newton system -------------------------------------------------------
    def z_system(self, st):
        """Assembled augmented matrix Z (eq. (nwtr2Z)) and its right-hand side."""
        F1, F2, F3, F4, F5 = self.residuals(st)
        xt = self.xbar - st.x
        D = st.phi / st.x + st.psi / xt
        G3 = F3 + F4 / st.x - F5 / xt
        B = self.Bmat(st)
        Dinv = sp.diags(1.0 / D)
        Zuu = self.K(st.x) + B @ Dinv @ B.T
        bvec = B @ (1.0 / D)
        c = float(np.sum(1.0 / D))
        Z = sp.bmat([[Zuu, sp.csr_matrix(bvec[:, None])],
                     [sp.csr_matrix(bvec[None, :]), sp.csr_matrix([[c]])]]).tocsr()
        rhs = np.concatenate([-F1 + B @ (G3 / D), [-F2 + np.sum(G3 / D)]])
        return Z, rhs, (F1, F2, F3, F4, F5, D, G3, B)

    def recover(self, st, du, dlam, parts):
        F1, F2, F3, F4, F5, D, G3, B = parts
        dx = (B.T @ du + dlam - G3) / D
        dphi = (-F4 - st.phi * dx) / st.x
        dpsi = (-F5 + st.psi * dx) / (self.xbar - st.x)
        return dx, dphi, dpsi

    def jacobian_dense(self, st):
        """Dense Jacobian of F with respect to (u, lambda, x, phi, psi)."""
        n, m = len(self.free), self.grid.m
        K = self.K(st.x).toarray()
        B = self.Bmat(st).toarray()
        N = n + 1 + 3 * m
        J = np.zeros((N, N))
        iu, il, ix, ip, iq = 0, n, n + 1, n + 1 + m, n + 1 + 2 * m
        J[iu:il, iu:il] = K
        J[iu:il, ix:ip] = B
        J[il, ix:ip] = 1.0
        J[ix:ip, iu:il] = -B.T
        J[ix:ip, il] = -1.0
        J[ix:ip, ip:iq] = -np.eye(m)
        J[ix:ip, iq:] = np.eye(m)
        J[ip:iq, ix:ip] = np.diag(st.phi)
        J[ip:iq, ip:iq] = np.diag(st.x)
        J[iq:, ix:ip] = -np.diag(st.psi)
        J[iq:, iq:] = np.diag(self.xbar - st.x)
        return J

    def F_vector(self, st):
        F1, F2, F3, F4, F5 = self.residuals(st)
        return np.concatenate([F1, [F2], F3, F4, F5])


def step_length(st, dx, dphi, dpsi, xbar, frac=0.9, all_blocks=True):
    """alpha = min(alpha_l, alpha_u, 1) with the fraction-to-boundary rule."""
    def ratio(val, d, neg):
        sel = d < 0 if neg else d > 0
        if not np.any(sel):
            return np.inf
        return float(np.min((val[sel] if neg else val[sel]) / np.abs(d[sel])))
    a = min(frac * ratio(st.x, dx, True), frac * ratio(xbar - st.x, dx, False), 1.0)
    if all_blocks:
        a = min(a, frac * ratio(st.phi, dphi, True), frac * ratio(st.psi, dpsi, True))
    return a


class NewtonSolveError(RuntimeError):
    """A Newton system whose PCG solve broke down, or stopped at the iteration
    limit with a true relative residual above the acceptance bound."""


class IPLog:
    def __init__(self):
        self.newton = 0
        self.short_solves = 0      # Newton solves accepted short of pcg_rtol
        self.barrier_updates = 0
        self.pcg_iters = []
        self.alpha = []
        self.nwt = []
        self.gap = []
        self.s = []
        self.status = "running"


def solve_linear(Z, rhs, params, grid, augmented, x0=None, Zprec=None):
    """MG-PCG (or a sparse direct solve); returns (solution, iterations, status,
    true relative residual), status "ok", "maxit" or "breakdown".  Zprec: the
    multigrid hierarchy is built from this matrix instead of Z (PCG still on Z)."""
    if params.solver == "direct":
        return spla.spsolve(Z.tocsc(), rhs), 0, "ok", 0.0
    H = mg.Hierarchy(grid, Z if Zprec is None else Zprec, params.levels, augmented=augmented, omega=params.omega)
    A = None if Zprec is None else Z
    res = pcg_mod.mg_pcg(H, rhs, params.pcg_rtol, params.pcg_maxit, None,
                         params.nu1, params.nu2, A=A)
    iters = res.iters
    if res.status == "breakdown":
        # the V-cycle was not positive definite (the estimate of rho came out too
        # low): damping estimated again, more steps and a smaller product, and the
        # solve continued from its last iterate
        H.damping(mg.RETRY_POWER_FACTOR * mg.POWER_STEPS_Z, mg.SAFE_PRODUCT_RETRY)
        res = pcg_mod.mg_pcg(H, rhs, params.pcg_rtol, params.pcg_maxit, res.z, params.nu1, params.nu2, A=A)
        iters += res.iters
    return res.z, iters, res.status, res.true_relres


def initial_state(prob, params):
    m = prob.grid.m
    x = np.full(m, prob.V / m)
    u, it, status, _ = solve_linear(prob.K(x), prob.f, params, prob.grid, False)
    if status != "ok":
        raise NewtonSolveError(f"initial equilibrium solve: {status}")
    st = IPState(u, 1.0, x, np.ones(m), np.ones(m), 1.0, 1.0)
    return st, it


def accept_solve(status, true_relres, params):
    """Acceptance of a Newton-system solve as the search direction (Sec. 6, stopping
    rule): a solve that reached pcg_rtol; or one stopped by the iteration limit whose
    true relative residual is within accept_rtol, an inexact Newton direction (the
    paper stops every Newton solve at a relative residual of 1e-2, eq. (cgstop)).
    A breakdown of the recurrence is never accepted.  Returns True for a solve
    accepted short of pcg_rtol."""
    if status == "ok":
        return False
    if status == "maxit" and true_relres <= params.accept_rtol:
        return True
    raise NewtonSolveError(f"Newton system solve: {status}, true relative residual {true_relres:.3e}")


def newton_step(prob, st, params, log=None):
    Z, rhs, parts = prob.z_system(st)
    Zp = prob.z_preconditioner(st, parts) if params.solver == "mg" else None
    sol, iters, status, true_rel = solve_linear(Z, rhs, params, prob.grid, True, Zprec=Zp)
    short = accept_solve(status, true_rel, params)
    if log is not None:
        log.short_solves += int(short)
    du, dlam = sol[:-1], float(sol[-1])
    dx, dphi, dpsi = prob.recover(st, du, dlam, parts)
    alpha = step_length(st, dx, dphi, dpsi, prob.xbar, params.frac, params.step_all_blocks)
    new = IPState(st.u + alpha * du, st.lam + alpha * dlam, st.x + alpha * dx,
                  st.phi + alpha * dphi, st.psi + alpha * dpsi, st.s, st.r)
    return new, alpha, iters


def run(prob, params, state=None, log=None, callback=None):
    """Interior-point loop of Sec. 3.1; returns (state, log).  With
    params.cg_tol_factor < 1 the PCG tolerance is multiplied by it after every
    barrier update (the "CG tol decreasing" variant of Sec. 8.1, factor 0.5)."""
    import copy
    params = copy.copy(params)
    log = log or IPLog()
    if state is None:
        state, it = initial_state(prob, params)
        log.pcg_iters.append(it)
    st = state
    while log.newton < params.max_newton:
        try:
            st, alpha, iters = newton_step(prob, st, params, log)
        except NewtonSolveError:
            log.status = "solve_failed"
            return st, log
        log.newton += 1
        log.pcg_iters.append(iters)
        log.alpha.append(alpha)
        nwt, gap, _ = prob.measures(st)
        log.nwt.append(nwt)
        log.gap.append(gap)
        log.s.append(st.s)
        if callback:
            callback(st, log)
        if not (np.isfinite(nwt) and np.isfinite(gap) and alpha > 0):
            log.status = "failed"
            return st, log
        if params.stop == "kkt" and nwt <= params.tau_nwt and gap <= params.kkt_tol:
            log.status = "converged"
            return st, log
        if nwt <= params.tau_nwt:
            st.s *= params.sigma
            st.r *= params.sigma
            log.barrier_updates += 1
            if params.cg_tol_factor != 1.0:       # "CG tol decreasing" (Sec. 8.1)
                params.pcg_rtol *= params.cg_tol_factor
            if params.stop == "barrier" and max(st.s, st.r) <= params.tau_ip:
                log.status = "converged"
                return st, log
    log.status = "max_newton"
    return st, log
