"""SIMP model with a density filter (oracle; test infrastructure only).

Paper, Sec. 9: the equilibrium K(x) u = f is replaced by K^(x~) u = f with
K^(x~) = sum_i x~_i^p K_i and the filtered densities x~ = W x, where
  W^_ij = max(0, rmin - dist(i, j)),  W_:i = W^_:i / sum_j W^_ij,
dist the distance of the element centres (Manhattan in Example 4, rmin = 2), so
every column of W sums to one (sum x~ = sum x).  For the compliance c = f'u the
derivative follows from K^ du/dx_i = -(dK^/dx_i) u:
  dc/dx_i = -u' [p sum_j W_ji x~_j^(p-1) K_j] u = -sum_j W_ji p x~_j^(p-1) E_j,
E_j = u_j'K0u_j; this is the bracket of the paper's modified condition (KKT3).

Interior-point method on the SIMP model (Sec. 9): the method of Sec. 2-3 with
K(x) replaced by K^(x~) and the matrix B(u) of the Newton system (eq. (nwtr), and
so Z of eq. (nwtr2)) replaced by
  B^(u) = (b_1, ..., b_m),  b_i = p sum_j W_ji x~_j^(p-1) K_j u = B(u) C W e_i,
C = diag(p x~^(p-1)), B(u) = (K_1 u, ..., K_m u) with the unit element matrices;
F3_i = -1/2 (W'(C E))_i - lambda - phi_i + psi_i.  Reading: the paper keeps the
Newton system of the convex problem with B^ in place of B (it calls the method
"vanilla"), so the term of d(B^'u)/dx (second derivatives of K^) is not part of
the Newton matrix; the Newton matrix here is exactly that system.
Preconditioner (reading: the paper does not say how its multigrid treats the
filtered rank-one terms, whose vectors b_i span the elements of a filter patch):
the hierarchy is built from the element-local SPD matrix
  Z~ = [[K^, 0], [0, 0]] + sum_j [h_j; g_j][h_j; g_j]',
  h_j = sqrt(w~_j) K_j u,  w~_j = c_j^2 (W2 w)_j,  (W2)_ji = W_ji^2,  w = D^-1,
  g_j = beta_j / sqrt(w~_j),  beta_j = c_j (W w)_j,
that is the rank-one terms w_i b_i b_i' with the couplings between different
elements of a patch dropped, and the border sum_j beta_j K_j u = B^ D^-1 e exact;
PCG runs on the exact Z.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem, ip


def filter_matrix(grid, rmin, metric="manhattan"):
    """W as a sparse m x m matrix (element order of fem.Grid), built from the
    definition by comparing every pair of element centres within the radius."""
    nel = grid.nel
    coords = np.stack(np.meshgrid(*[np.arange(n) for n in nel[::-1]], indexing="ij")[::-1], axis=-1)
    coords = coords.reshape(-1, grid.dim)             # element e -> (i, j[, k]), x fastest
    R = int(np.ceil(rmin))
    rows, cols, vals = [], [], []
    m = grid.m
    for e in range(m):
        c = coords[e]
        lo = np.maximum(c - R, 0)
        hi = np.minimum(c + R, np.array(nel) - 1)
        rng = [np.arange(lo[d], hi[d] + 1) for d in range(grid.dim)]
        nb = np.stack(np.meshgrid(*rng, indexing="ij"), axis=-1).reshape(-1, grid.dim)
        diff = np.abs(nb - c)
        dist = diff.sum(axis=1) if metric == "manhattan" else np.sqrt((diff ** 2).sum(axis=1))
        w = np.maximum(0.0, rmin - dist)
        keep = w > 0
        idx = np.zeros(int(keep.sum()), dtype=np.int64)
        for d in range(grid.dim - 1, -1, -1):          # element index of each neighbour
            idx = idx * nel[d] + nb[keep][:, d]
        rows.append(np.full(len(idx), e))
        cols.append(idx)
        vals.append(w[keep])
    What = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(m, m))
    colsum = np.asarray(What.sum(axis=0)).ravel()
    return (What @ sp.diags(1.0 / colsum)).tocsr()


def compliance_and_gradient(grid, K0, f_slots, x, rmin, p, W=None):
    """(c, u_free, grad, x~) of the SIMP model at x by a sparse direct solve."""
    W = filter_matrix(grid, rmin) if W is None else W
    xt = W @ x
    K = fem.stiffness_free(grid, xt ** p, K0)
    f = fem.to_free(grid, f_slots)
    u = spla.spsolve(K.tocsc(), f)
    ue = fem.to_slots(grid, u)[grid.element_dofs()]
    E = np.einsum("ei,ij,ej->e", ue, K0, ue)
    grad = -(W.T @ (p * xt ** (p - 1) * E))
    return float(f @ u), u, grad, xt


class SimpProblem(ip.Problem):
    """Problem (1) with the SIMP model and density filter of Sec. 9 for the
    interior-point method (readings in the module header)."""

    def __init__(self, grid, K0, f_slots, V, xbar, rmin=2.0, p=3.0, W=None):
        super().__init__(grid, K0, f_slots, V, xbar)
        self.rmin, self.p = float(rmin), float(p)
        self.W = filter_matrix(grid, rmin) if W is None else W

    def xt(self, x):
        return self.W @ x

    def cfac(self, x):
        """c = p x~^(p-1), the derivative of x~^p."""
        return self.p * self.xt(x) ** (self.p - 1.0)

    def K(self, x):
        return fem.stiffness_free(self.grid, self.xt(x) ** self.p, self.K0)

    def Bmat(self, st):
        return self.B(st.u) @ sp.diags(self.cfac(st.x)) @ self.W

    def energy_term(self, st):
        return self.W.T @ (self.cfac(st.x) * self.energies(st.u))

    def z_preconditioner(self, st, parts):
        F1, F2, F3, F4, F5, D, G3, B = parts
        w = 1.0 / D
        cf = self.cfac(st.x)
        wt = cf ** 2 * (self.W.multiply(self.W) @ w)
        beta = cf * (self.W @ w)
        Bu = self.B(st.u)
        Zuu = self.K(st.x) + Bu @ sp.diags(wt) @ Bu.T
        bvec = Bu @ beta
        corner = float(np.sum(beta ** 2 / wt))
        return sp.bmat([[Zuu, sp.csr_matrix(bvec[:, None])],
                        [sp.csr_matrix(bvec[None, :]), sp.csr_matrix([[corner]])]]).tocsr()
