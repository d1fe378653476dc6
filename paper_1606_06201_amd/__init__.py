"""MI355X-native multigrid-preconditioned CG for the primal-dual interior-point
method of minimum-compliance topology optimisation (Kocvara & Mohammed).

    from paper_1606_06201_amd import Solver, solve_K
"""
from .solver import Solver, IPMGError, OP_K, OP_Z  # noqa: F401
from .autograd import solve_K  # noqa: F401
from . import inputs  # noqa: F401
