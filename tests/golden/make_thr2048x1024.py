"""Writes tests/golden/thr2048x1024.txt: the oracle's own FP64 solution of
K(x) u = f on the 2048x1024 two-phase workload (contrast 1e6, 6 multigrid
levels), solved by the oracle's MG-PCG aiming at a relative residual of 1e-9 so
that the GPU solutions (1e-8) can be compared with it.  At this contrast the FP64
recurrence does not reach 1e-9: the run stops at its 2000-step limit with a true
relative residual of 4.1e-9, which is what the stored file records.

Calls only oracle/ and the seeded input generators (no GPU, no library code).
Stored: the iteration count and both residuals, the compliance f'u, ||u||_2,
max |u|, and u at 4096 free DOFs drawn by a seeded generator (plus the loaded
DOF).  Run from the repository root:

    python tests/golden/make_thr2048x1024.py      # about an hour on one core, 4 GB
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import fem, mg, pcg  # noqa: E402
from paper_1606_06201_amd import inputs  # noqa: E402

NEL, LEVELS, RTOL, SAMPLES, SEED = (2048, 1024), 6, 1e-9, 4096, 2048


def main(out=os.path.join(HERE, "thr2048x1024.txt")):
    t0 = time.perf_counter()
    g = fem.Grid(NEL)
    K0 = fem.element_stiffness(2)
    x = inputs.density_for("thr2048x1024")
    f = fem.to_free(g, fem.load_vector(g, inputs.point_load(NEL)))
    H = mg.kstiffness_hierarchy(g, x, K0, LEVELS)
    res = pcg.mg_pcg(H, f, rtol=RTOL, maxit=2000)
    u = res.z
    free = g.free_to_slot()
    rng = np.random.default_rng(SEED)
    pick = np.unique(np.concatenate([rng.choice(len(free), SAMPLES, replace=False), [int(np.argmin(f))]]))
    with open(out, "w") as fh:
        fh.write("# Oracle FP64 MG-PCG solution of K(x) u = f, 2048x1024 two-phase densities\n")
        fh.write("# (band-connected random field thresholded to {1e-6, 1}, seed 2), unit tip load,\n")
        fh.write(f"# 6 levels, damped Jacobi 2+2, tolerance {RTOL:g}; written by make_thr2048x1024.py\n")
        fh.write(f"status {res.status}\niters {res.iters}\nrelres {res.relres:.17e}\n")
        fh.write(f"true_relres {res.true_relres:.17e}\n")
        fh.write(f"compliance {float(f @ u):.17e}\nnorm2 {float(np.linalg.norm(u)):.17e}\n")
        fh.write(f"maxabs {float(np.abs(u).max()):.17e}\n")
        fh.write("# slot value (u at free DOFs drawn with default_rng(2048), and the loaded DOF)\n")
        for k in pick:
            fh.write(f"{int(free[k])} {u[k]:.17e}\n")
    print(f"wrote {out}: {res.iters} iterations, true relres {res.true_relres:.2e}, "
          f"{time.perf_counter() - t0:.0f} s")


def load(path=os.path.join(HERE, "thr2048x1024.txt")):
    """(scalars dict, slots array, values array) of the stored golden."""
    sc, slots, vals = {}, [], []
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            a, b = line.split()
            if a.isdigit():
                slots.append(int(a))
                vals.append(float(b))
            else:
                sc[a] = b if a == "status" else float(b)
    return sc, np.array(slots, dtype=np.int64), np.array(vals)


if __name__ == "__main__":
    main()
