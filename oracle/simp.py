"""SIMP model with a density filter (oracle; test infrastructure only).

Paper, Sec. 9: the equilibrium K(x) u = f is replaced by K^(x~) u = f with
K^(x~) = sum_i x~_i^p K_i and the filtered densities x~ = W x, where
  W^_ij = max(0, rmin - dist(i, j)),  W_:i = W^_:i / sum_j W^_ij,
dist the distance of the element centres (Manhattan in Example 4, rmin = 2), so
every column of W sums to one (sum x~ = sum x).  For the compliance c = f'u the
derivative follows from K^ du/dx_i = -(dK^/dx_i) u:
  dc/dx_i = -u' [p sum_j W_ji x~_j^(p-1) K_j] u = -sum_j W_ji p x~_j^(p-1) E_j,
E_j = u_j'K0u_j; this is the bracket of the paper's modified condition (KKT3).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem


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
