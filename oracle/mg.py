"""Geometric multigrid V-cycle (oracle; test infrastructure only).

Paper, Sec. 5.1 (Algorithm MG, correction scheme) with the transfer operators of
Sec. 7: the prolongation is the nine-point bilinear interpolation stencil
[1/4 1/2 1/4; 1/2 1 1/2; 1/4 1/2 1/4] applied to each displacement component
(the 3D analogue is its trilinear tensor product), the restriction is its
transpose, and the coarse operators are the Galerkin products
A_{k-1} = I_k^{k-1} A_k I_{k-1}^k.  For the augmented system Z the single extra
unknown lambda is transferred by the identity (Sec. 7).

Readings where the paper is silent (shared with the GPU path):
  * smoother: damped Jacobi with weight omega (0.6), nu1 pre- and nu2
    post-sweeps (2 + 2), a fixed number of sweeps (the tolerance argument of
    the smoother is not used), so one V-cycle is a fixed linear operator;
  * coarsest level: exact solve by a dense Cholesky factorisation;
  * the algorithm's "if k = 0" branch is read as the coarsest level k = 1,
    which is where the paper defines A_1;
  * clamped nodes stay clamped on every level (the clamped edge x = 0 is a
    grid line of every level, so the coarse spaces are nested subspaces);
  * damping safeguard: damped Jacobi diverges (and the V-cycle stops being
    positive definite) once omega * rho(D^-1 A) >= 2.  That happens for
    omega = 0.6 on 3D elasticity (rho about 3.3-3.8) and on the augmented
    system Z late in the interior-point run (its rank-one element terms push
    rho near 4).  Every non-coarsest level therefore uses
    omega_k = min(omega, SAFE_PRODUCT / rho_k), rho_k the Rayleigh-quotient
    estimate of the largest eigenvalue of D_k^-1 A_k after POWER_STEPS power
    iterations (POWER_STEPS_Z for the augmented system) from the vector
    (-1)^(i+j+k) (1 + c) on DOF component c of node (i, j, k) (and 1 on lambda).
    For 2D K(x), rho stays near 2.2-2.6, so omega = 0.6 is kept there.  The top
    of the spectrum of D^-1 Z late in a 3D interior-point run is a cluster of
    element-local modes of the rank-one terms, which power iteration approaches
    slowly from below: 12 steps gave rho = 6.2 where the value is about 7.9, so
    omega * rho > 2 and PCG broke down; 30 steps stay within SAFE_PRODUCT / 2.
"""
import numpy as np
import scipy.sparse as sp
import scipy.linalg as sla

from . import fem


def interp_1d(nc):
    """(2*nc+1, nc+1) linear interpolation between a 1D node row and its
    refinement: fine node 2I <- coarse I (weight 1), fine 2I+-1 <- 1/2."""
    nf = 2 * nc
    rows, cols, vals = [], [], []
    for I in range(nc + 1):
        rows.append(2 * I)
        cols.append(I)
        vals.append(1.0)
        for off in (-1, 1):
            r = 2 * I + off
            if 0 <= r <= nf:
                rows.append(r)
                cols.append(I)
                vals.append(0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf + 1, nc + 1))


def prolongation_slots(coarse):
    """Prolongation I_{k-1}^k over all DOF slots, fine grid = coarse refined.
    Nodes are x-fastest, so the node operator is kron(z, kron(y, x));
    each of the dim components is interpolated independently."""
    mats = [interp_1d(n) for n in coarse.nel]
    Pn = mats[0]
    for M in mats[1:]:
        Pn = sp.kron(M, Pn)
    return sp.kron(Pn, sp.identity(coarse.dim)).tocsr()


def prolongation_free(fine, coarse):
    P = prolongation_slots(coarse)
    return P[fine.free_to_slot()][:, coarse.free_to_slot()].tocsr()


SAFE_PRODUCT = 1.6
POWER_STEPS = 12
POWER_STEPS_Z = 30
# after a breakdown of a solve: four times the power steps and the product 1.2
RETRY_POWER_FACTOR = 4
SAFE_PRODUCT_RETRY = 1.2


def power_start(grid, augmented):
    """Deterministic start vector for the spectral-radius estimate."""
    coords = grid.node_coords()
    sign = np.where(coords.sum(axis=1) % 2 == 0, 1.0, -1.0)
    v = (sign[:, None] * (1.0 + np.arange(grid.dim))[None, :]).ravel()
    v = v[grid.free_to_slot()]
    return np.concatenate([v, [1.0]]) if augmented else v


def jacobi_radius(A, d, v0, steps=POWER_STEPS):
    """Rayleigh quotient v'Av / v'Dv after `steps` power iterations on D^-1 A."""
    v = v0 / np.linalg.norm(v0)
    for _ in range(steps):
        w = (A @ v) / d
        v = w / np.linalg.norm(w)
    return float(v @ (A @ v)) / float(v @ (d * v))


class Hierarchy:
    """Level data for levels 1 (coarsest) .. L (finest) for one SPD operator.

    A_fine is the operator on the free DOFs of the finest grid (for Z: the
    (n+1)x(n+1) augmented matrix with lambda last)."""

    def __init__(self, fine_grid, A_fine, levels, augmented=False, omega=0.6, safeguard=True):
        if levels < 1:
            raise ValueError("levels >= 1")
        self.augmented = augmented
        grids = [fine_grid]
        for _ in range(levels - 1):
            grids.append(grids[-1].coarsen())
        grids = grids[::-1]                     # index 0 = coarsest (level 1)
        self.grids = grids
        self.L = levels
        self.P = [None]                         # P[k]: level k -> level k+1 (0-based)
        for k in range(levels - 1):
            P = prolongation_free(grids[k + 1], grids[k])
            if augmented:                       # identity transfer for lambda
                P = sp.block_diag([P, sp.identity(1)]).tocsr()
            self.P.append(P)
        A = [None] * levels
        A[-1] = sp.csr_matrix(A_fine)
        for k in range(levels - 1, 0, -1):      # Galerkin products
            Pk = self.P[k]
            A[k - 1] = (Pk.T @ A[k] @ Pk).tocsr()
        self.A = A
        self.diag = [a.diagonal().copy() for a in A]
        self.chol = sla.cho_factor(A[0].toarray(), lower=True)
        self.omega = [omega] * levels
        self.rho = [None] * levels
        self.omega0 = omega
        if safeguard:
            self.damping(POWER_STEPS_Z if augmented else POWER_STEPS, SAFE_PRODUCT)

    def damping(self, steps, product):
        """omega_k = min(omega, product / rho_k) on every non-coarsest level, rho_k
        estimated with `steps` power iterations."""
        for k in range(1, self.L):
            self.rho[k] = jacobi_radius(self.A[k], self.diag[k], power_start(self.grids[k], self.augmented),
                                        steps)
            self.omega[k] = min(self.omega0, product / self.rho[k])


def jacobi(A, d, b, z, omega, sweeps):
    """z <- z + omega D^-1 (b - A z), repeated `sweeps` times."""
    for _ in range(sweeps):
        z = z + omega * (b - A @ z) / d
    return z


def mgm(H, k, b, nu1=2, nu2=2):
    """One V-cycle from the zero initial guess on level k (0-based, 0 = coarsest),
    right-hand side b.  Returns the correction z (Algorithm MG)."""
    if k == 0:
        return sla.cho_solve(H.chol, b)
    A, d, w = H.A[k], H.diag[k], H.omega[k]
    z = np.zeros_like(b)
    z = jacobi(A, d, b, z, w, nu1)                       # pre-smoothing
    rc = H.P[k].T @ (b - A @ z)                          # restricted residual
    v = mgm(H, k - 1, rc, nu1, nu2)                      # coarse-grid correction
    z = z + H.P[k] @ v                                   # solution update
    z = jacobi(A, d, b, z, w, nu2)                       # post-smoothing
    return z


def vcycle(H, b, nu1=2, nu2=2):
    return mgm(H, H.L - 1, np.asarray(b, dtype=np.float64), nu1, nu2)


def vcycle_matrix(H, nu1=2, nu2=2):
    """Dense matrix of the V-cycle operator (tiny grids only)."""
    n = H.A[-1].shape[0]
    return np.stack([vcycle(H, e, nu1, nu2) for e in np.eye(n)], axis=1)


def kstiffness_hierarchy(grid, x, K0, levels, omega=0.6):
    return Hierarchy(grid, fem.stiffness_free(grid, x, K0), levels, omega=omega)
