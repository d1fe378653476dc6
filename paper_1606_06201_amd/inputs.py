"""Seeded synthetic inputs (densities, loads, objective vectors) and the
workload table.  This module holds none of the method's arithmetic: it only
draws random numbers and names grid coordinates, so the GPU library and the
CPU oracle can both be fed identical arrays.

Workloads (cantilevers of Sec. 7, Example 2 shapes, and a 3D analogue):
  ip64x32        64x32 elements, IP run from x = V/m, V = 0.5 m, xbar = 1, 4 levels
  grf1024x512    1024x512, Gaussian random field -> logistic in [1e-3, 1], 7 levels
  thr2048x1024   2048x1024, band-connected random field thresholded to {1e-6, 1},
                 about 40 % solid, 6 levels (coarsest 64x32, chosen by measurement)
  uni512x256     512x256, x ~ U[0.01, 1], objective g ~ N(0, 1), 6 levels
  ip128x64x64    128x64x64 hexahedra, IP run from x = 0.3, V = 0.3 m, 5 levels
Loads: a unit downward (-y) point load at the right-edge mid node in 2D; in 3D
a unit load split over a 4x4 node patch on the x = max face.
"""
import numpy as np


def gaussian_random_field(shape, corr_len, seed):
    """White N(0,1) noise on an element grid (C order, x fastest), convolved
    periodically with exp(-d^2 / (2 corr_len^2)) via FFT, standardised."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(shape)
    kern = np.ones(shape)
    for ax, n in enumerate(shape):
        d = np.minimum(np.arange(n), n - np.arange(n)).astype(np.float64)
        g = np.exp(-d * d / (2.0 * corr_len * corr_len))
        sh = [1] * len(shape)
        sh[ax] = n
        kern = kern * g.reshape(sh)
    field = np.real(np.fft.ifftn(np.fft.fftn(noise) * np.fft.fftn(kern)))
    field -= field.mean()
    field /= field.std()
    return field


def _grid_shape(nel):
    return tuple(int(v) for v in nel[::-1])       # (nz,) ny, nx: x fastest


def density_logistic(nel, seed=1, lo=1e-3, gain=4.0, corr_len=16.0):
    g = gaussian_random_field(_grid_shape(nel), corr_len, seed).ravel()
    return lo + (1.0 - lo) / (1.0 + np.exp(-gain * g))


def density_threshold(nel, seed=2, solid=0.4, lo=1e-6, corr_len=16.0, band=0.125):
    """Two-phase densities {lo, 1} (2D): the solid set is grown from a band of
    rows along the cantilever axis (|y - ny/2| < band*ny/2, which carries the tip
    load to the clamped edge) by the elements with the largest values of a
    Gaussian random field, keeping only solid connected (across element edges) to
    the band, with the largest field threshold whose connected solid fraction is
    <= `solid`.  A plain threshold at 40 % leaves the loaded part floating on the
    void phase (the solid does not percolate at this correlation length), which
    makes K(x) nearly singular; the connected recipe keeps contrast 1e6 and void
    regions without floating islands."""
    import scipy.ndimage as ndi
    nx, ny = int(nel[0]), int(nel[1])
    g = gaussian_random_field((ny, nx), corr_len, seed)
    yc = np.arange(ny)[:, None] + 0.5
    inband = np.broadcast_to(np.abs(yc - ny / 2.0) < band * ny / 2.0, (ny, nx))
    m = nx * ny
    rank = np.empty(m, dtype=np.int64)
    rank[np.argsort(-g.ravel(), kind="stable")] = np.arange(m)
    rank = rank.reshape(ny, nx)
    target = int(round(solid * m))

    def connected(k):
        lab, _ = ndi.label(inband | (rank < k))
        keep = np.unique(lab[inband])
        return np.isin(lab, keep[keep > 0])

    lo_k, hi_k = 0, m
    while lo_k < hi_k:                       # largest k with |S(k)| <= target
        mid = (lo_k + hi_k + 1) // 2
        if connected(mid).sum() <= target:
            lo_k = mid
        else:
            hi_k = mid - 1
    return np.where(connected(lo_k).ravel(), 1.0, lo)


def density_uniform(nel, seed=3, lo=0.01, hi=1.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, int(np.prod(nel)))


def normal_slots(nslots, seed=33):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(int(nslots))


def sample_elements(m, count=32, seed=333):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(int(m), size=int(count), replace=False))


def point_load(nel):
    """[(node coords, component, value)]: unit downward load (component 1 = y)."""
    if len(nel) == 2:
        nx, ny = nel
        return [((nx, ny // 2), 1, -1.0)]
    nx, ny, nz = nel
    out = []
    for k in range(nz // 2 - 2, nz // 2 + 2):
        for j in range(ny // 2 - 2, ny // 2 + 2):
            out.append(((nx, j, k), 1, -1.0 / 16.0))
    return out


# The paper's own examples (Sec. 7): coarsest mesh 2x2 (Example 1, square) or 4x2
# (Example 2, slender), left edge clamped, vertical load (-1/2, -1, -1/2) on the
# right-edge middle node and its two neighbours on that edge, upper bound xbar = 2.
# Problem "ab k" is the a x b coarsest mesh refined k - 1 times (k levels), which
# reproduces the variable counts of Tables 1 and 3 (e.g. 423: 16 x 8 elements,
# 288 free DOFs).  The volume is not stated in the paper; V = m (the start point
# x = V/m = 1 is the middle of [0, xbar]).
PAPER_COARSEST = {1: (2, 2), 2: (4, 2)}


def paper_problem(example, k):
    """(nel, levels, loads, V, xbar) of problem "<coarsest>k" of Example 1 or 2."""
    cx, cy = PAPER_COARSEST[int(example)]
    s = 2 ** (int(k) - 1)
    nx, ny = cx * s, cy * s
    loads = [((nx, ny // 2 - 1), 1, -0.5), ((nx, ny // 2), 1, -1.0), ((nx, ny // 2 + 1), 1, -0.5)]
    return (nx, ny), int(k), loads, float(nx * ny), 2.0


WORKLOADS = {
    "ip64x32": dict(nel=(64, 32), levels=4, kind="ip", vfrac=0.5, xbar=1.0),
    "grf1024x512": dict(nel=(1024, 512), levels=7, kind="solve", density="logistic", seed=1),
    "thr2048x1024": dict(nel=(2048, 1024), levels=6, kind="solve", density="threshold", seed=2),
    "uni512x256": dict(nel=(512, 256), levels=6, kind="adjoint", density="uniform", seed=3),
    "ip128x64x64": dict(nel=(128, 64, 64), levels=5, kind="ip", vfrac=0.3, xbar=1.0),
}


def density_for(name, nel=None):
    w = WORKLOADS[name]
    nel = nel or w["nel"]
    kind = w.get("density")
    if kind == "logistic":
        return density_logistic(nel, w["seed"])
    if kind == "threshold":
        return density_threshold(nel, w["seed"])
    if kind == "uniform":
        return density_uniform(nel, w["seed"])
    return np.full(int(np.prod(nel)), w["vfrac"])
