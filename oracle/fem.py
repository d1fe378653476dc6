"""Structured Q1 finite-element discretisation (oracle; test infrastructure only).

Paper: the design variable x is one value per element, the displacement u uses
bilinear basis functions on square elements (Sec. 7, discretisation paragraph);
the stiffness is K(x) = sum_i x_i K_i with K_i symmetric positive semidefinite
(Sec. 1, problem (1)); Young's modulus 1 and Poisson ratio 0.3 (Sec. 7).  The
3D trilinear hexahedral element follows the same construction one dimension up.

Indexing (the paper is silent on numbering; this is the layout both paths use):
  element (i,j[,k])  ->  e = (k*ny + j)*nx + i                 (x fastest)
  node    (i,j[,k])  ->  q = (k*(ny+1) + j)*(nx+1) + i
  DOF slot           ->  dim*q + c,  c = 0 (x), 1 (y), 2 (z)
  local element node order: counter-clockwise on the face k,
  (i,j) (i+1,j) (i+1,j+1) (i,j+1), then the same on face k+1 (3D).
  Clamped DOFs: every DOF of a node with i == 0 (left edge / x=0 face).
  Free DOFs: the remaining slots in increasing slot order.
"""
import numpy as np
import scipy.sparse as sp


class Grid:
    """A structured grid of nx*ny (2D) or nx*ny*nz (3D) unit elements."""

    def __init__(self, nel, h=1.0):
        nel = tuple(int(v) for v in nel)
        if len(nel) not in (2, 3) or min(nel) < 1:
            raise ValueError("grid needs 2 or 3 positive element counts")
        self.dim = len(nel)
        self.nel = nel
        self.h = float(h)
        self.nnode_axis = tuple(v + 1 for v in nel)
        self.m = int(np.prod(nel))
        self.nnodes = int(np.prod(self.nnode_axis))
        self.nslots = self.dim * self.nnodes

    # --- integer maps -----------------------------------------------------
    def node_index(self, i, j, k=0):
        nx1, ny1 = self.nnode_axis[0], self.nnode_axis[1]
        return (np.asarray(k) * ny1 + np.asarray(j)) * nx1 + np.asarray(i)

    def node_coords(self):
        """(nnodes, dim) integer coordinates of every node, node order."""
        axes = [np.arange(v) for v in self.nnode_axis]
        mesh = np.meshgrid(*axes[::-1], indexing="ij")  # slowest axis first
        cols = [mg.ravel() for mg in mesh[::-1]]
        return np.stack(cols, axis=1)

    def clamped_mask(self):
        """Boolean mask over slots: True where the DOF is clamped (node i == 0)."""
        i_of_node = self.node_coords()[:, 0]
        return np.repeat(i_of_node == 0, self.dim)

    def free_to_slot(self):
        return np.flatnonzero(~self.clamped_mask()).astype(np.int64)

    def element_nodes(self):
        """(m, 2**dim) node indices of every element in local order."""
        nx, ny = self.nel[0], self.nel[1]
        nz = self.nel[2] if self.dim == 3 else 1
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        i, j, k = i.ravel(), j.ravel(), k.ravel()
        face = [(0, 0), (1, 0), (1, 1), (0, 1)]
        cols = []
        for dk in ((0,) if self.dim == 2 else (0, 1)):
            for di, dj in face:
                cols.append(self.node_index(i + di, j + dj, k + dk))
        return np.stack(cols, axis=1).astype(np.int64)

    def element_dofs(self):
        """(m, dim*2**dim) slot indices of every element, node-major."""
        nodes = self.element_nodes()
        d = self.dim
        return (nodes[:, :, None] * d + np.arange(d)[None, None, :]).reshape(len(nodes), -1)

    def coarsen(self):
        if any(v % 2 for v in self.nel):
            raise ValueError("cannot coarsen an odd grid")
        return Grid(tuple(v // 2 for v in self.nel), h=2.0 * self.h)


# --- element stiffness ------------------------------------------------------

def elasticity_matrix(dim, E=1.0, nu=0.3):
    """Isotropic constitutive matrix: plane stress in 2D, Lame form in 3D.
    Engineering shear strains (gamma = 2 eps)."""
    if dim == 2:
        c = E / (1.0 - nu * nu)
        return c * np.array([[1.0, nu, 0.0], [nu, 1.0, 0.0], [0.0, 0.0, (1.0 - nu) / 2.0]])
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[np.arange(3), np.arange(3)] += 2.0 * mu
    C[3, 3] = C[4, 4] = C[5, 5] = mu
    return C


def _local_corner_coords(dim):
    face = [(0, 0), (1, 0), (1, 1), (0, 1)]
    if dim == 2:
        return np.array(face, dtype=float)
    return np.array([(a, b, c) for c in (0, 1) for a, b in face], dtype=float)


def shape_gradients(dim, xi):
    """Gradients (2**dim, dim) of the Q1 shape functions on the unit reference
    cell [0,1]^dim at point xi; N_a = prod_d (c_ad xi_d + (1-c_ad)(1-xi_d))."""
    corners = _local_corner_coords(dim)
    grads = np.zeros((len(corners), dim))
    for a, c in enumerate(corners):
        f = [xi[d] if c[d] else 1.0 - xi[d] for d in range(dim)]
        df = [1.0 if c[d] else -1.0 for d in range(dim)]
        for d in range(dim):
            g = df[d]
            for e in range(dim):
                if e != d:
                    g *= f[e]
            grads[a, d] = g
    return grads


def strain_displacement(dim, grads):
    """B matrix (n_strain, dim*2**dim) from shape-function gradients."""
    nn = grads.shape[0]
    if dim == 2:
        B = np.zeros((3, 2 * nn))
        for a in range(nn):
            gx, gy = grads[a]
            B[0, 2 * a] = gx
            B[1, 2 * a + 1] = gy
            B[2, 2 * a] = gy
            B[2, 2 * a + 1] = gx
        return B
    B = np.zeros((6, 3 * nn))
    for a in range(nn):
        gx, gy, gz = grads[a]
        B[0, 3 * a] = gx
        B[1, 3 * a + 1] = gy
        B[2, 3 * a + 2] = gz
        B[3, 3 * a] = gy
        B[3, 3 * a + 1] = gx
        B[4, 3 * a + 1] = gz
        B[4, 3 * a + 2] = gy
        B[5, 3 * a] = gz
        B[5, 3 * a + 2] = gx
    return B


def element_stiffness(dim, E=1.0, nu=0.3, h=1.0):
    """K0 = integral over the element of B^T C B, 2-point Gauss-Legendre rule per
    axis (exact for Q1 on a square / cube).  Element of side h, thickness 1 in 2D."""
    C = elasticity_matrix(dim, E, nu)
    g = 0.5 / np.sqrt(3.0)
    pts = (0.5 - g, 0.5 + g)
    w1 = 0.5
    nd = dim * 2 ** dim
    K = np.zeros((nd, nd))
    for idx in np.ndindex(*(2,) * dim):
        xi = [pts[t] for t in idx]
        grads = shape_gradients(dim, xi) / h        # d/dx = (1/h) d/dxi
        B = strain_displacement(dim, grads)
        K += (w1 ** dim) * (h ** dim) * (B.T @ C @ B)
    return K


# --- assembly -----------------------------------------------------------------

def assemble_slots(grid, elem_mats):
    """Sum element matrices (m, nd, nd) into a CSR matrix over all DOF slots."""
    dofs = grid.element_dofs()
    nd = dofs.shape[1]
    rows = np.repeat(dofs, nd, axis=1).ravel()
    cols = np.tile(dofs, (1, nd)).ravel()
    vals = np.asarray(elem_mats).reshape(len(dofs), -1).ravel()
    A = sp.coo_matrix((vals, (rows, cols)), shape=(grid.nslots, grid.nslots)).tocsr()
    A.sum_duplicates()
    return A


def stiffness_slots(grid, x, K0):
    """K(x) = sum_e x_e K_e over all DOF slots (clamped ones included)."""
    x = np.asarray(x, dtype=np.float64)
    if x.shape != (grid.m,):
        raise ValueError("x must have one value per element")
    return assemble_slots(grid, x[:, None, None] * K0[None, :, :])


def restrict_free(grid, A):
    free = grid.free_to_slot()
    return A[free][:, free].tocsr()


def stiffness_free(grid, x, K0):
    """K(x) restricted to the free DOFs: the equilibrium matrix of problem (1)."""
    return restrict_free(grid, stiffness_slots(grid, x, K0))


def to_free(grid, v_slots):
    return np.asarray(v_slots)[..., grid.free_to_slot()]


def to_slots(grid, v_free):
    out = np.zeros(grid.nslots)
    out[grid.free_to_slot()] = v_free
    return out


def element_values(grid, v_slots):
    """(m, nd) element-local gather of a slot vector (v_e in the paper's notation)."""
    return np.asarray(v_slots)[grid.element_dofs()]


def load_vector(grid, loads):
    """Slot vector from a list of point loads (node coords tuple, component, value)."""
    f = np.zeros(grid.nslots)
    for coords, comp, val in loads:
        q = int(grid.node_index(*coords))
        f[grid.dim * q + comp] += val
    return f


def apply_slots(grid, x, K0, v_slots):
    """y = K(x) v = sum_e x_e K_e v over all slots, element by element (the
    definition of K(x), problem (1)), without forming the matrix.  Used to
    certify residuals of large solves."""
    edofs = grid.element_dofs()
    ve = np.asarray(v_slots, dtype=np.float64)[edofs]
    ye = (ve @ K0) * np.asarray(x, dtype=np.float64)[:, None]   # K0 symmetric
    return np.bincount(edofs.ravel(), weights=ye.ravel(), minlength=grid.nslots)


def apply_free_masked(grid, x, K0, v_slots):
    """K(x) restricted to the free DOFs, as a slot vector: clamped inputs are
    treated as zero and clamped outputs are zero."""
    mask = grid.clamped_mask()
    v = np.where(mask, 0.0, np.asarray(v_slots, dtype=np.float64))
    y = apply_slots(grid, x, K0, v)
    y[mask] = 0.0
    return y
