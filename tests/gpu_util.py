"""Helpers shared by the GPU tests (conversion between torch device tensors and
numpy, oracle-side references)."""
import numpy as np
import torch

from oracle import fem

DEV = "cuda:0"


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def N(t):
    return t.detach().cpu().numpy()


def relerr(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def tip_load(nel):
    """Unit downward point load at the right-edge mid node (2D) or split over a
    4x4 node patch on the x = max face (3D)."""
    from paper_1606_06201_amd import inputs
    return inputs.point_load(nel)


def grid_and_k0(nel):
    g = fem.Grid(nel)
    return g, fem.element_stiffness(g.dim)
