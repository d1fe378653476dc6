"""The paper's own inexact interior-point settings on its own examples, GPU against
the oracle (Sec. 3, Sec. 6.1 eq. (cgstop), Sec. 7 Examples 1-2, Sec. 8.1 Table 7):
Newton systems solved to the relative residual 1e-2, xbar = 2, the (-1/2, -1, -1/2)
load, the stop rule max(s, r) <= tau_IP, multigrid down to the coarsest mesh of the
example.  The paper's own feval / CG counts (Tables 3 and 7) depend on its smoother,
which it does not name: they are context, not pins; GPU and oracle run the same
algorithm and are compared with each other."""
import numpy as np
import pytest

from oracle import fem, ip as oip
from tests.gpu_util import T, N

pytestmark = pytest.mark.gpu


def _prob(example, k):
    from paper_1606_06201_amd import inputs
    nel, levels, loads, V, xbar = inputs.paper_problem(example, k)
    g = fem.Grid(nel)
    f = fem.load_vector(g, loads)
    return oip.Problem(g, fem.element_stiffness(2), f, V, xbar), nel, levels


def _run_gpu(prob, nel, levels, fp32, cg_tol_factor=1.0, tau_ip=1e-8):
    from paper_1606_06201_amd import Solver
    s = Solver(nel, levels, fp32=fp32)
    params = s.ip_params_paper(prob.V, prob.xbar, tau_ip=tau_ip)
    gst, log = s.ip_run(T(prob.f_slots), params, cg_tol_factor=cg_tol_factor)
    return gst, log


@pytest.mark.parametrize("fp32", [False, True])
def test_paper_preset_425(fp32):
    # problem 425: Example 2, 64 x 32 elements, 5 levels (coarsest 4 x 2)
    prob, nel, levels = _prob(2, 5)
    po = oip.IPParams(stop="barrier", tau_ip=1e-8, pcg_rtol=1e-2, solver="mg", levels=levels)
    st_o, log_o = oip.run(prob, po)
    gst, log = _run_gpu(prob, nel, levels, fp32)
    cg, cg_o = int(sum(log["pcg_iters"])), int(sum(log_o.pcg_iters))
    print(f"425 fp32={fp32}: GPU feval {1 + log['newton']} CG {cg}; oracle feval {1 + log_o.newton} CG {cg_o}; "
          f"per system GPU {log['pcg_iters']} oracle {log_o.pcg_iters}", flush=True)
    assert log["status"] == log_o.status == "converged"
    assert log["barrier_updates"] == log_o.barrier_updates == 12       # 0.2^12 <= 1e-8 < 0.2^11
    assert log["short_solves"] == 0 and log_o.short_solves == 0
    assert abs(log["newton"] - log_o.newton) <= 1
    assert abs(cg - cg_o) <= max(3, 0.03 * cg_o)
    c, c_o = float(prob.f_slots @ N(gst["u"])), float(prob.f @ st_o.u)
    assert abs(c - c_o) <= 1e-6 * c_o, (c, c_o)
    x = N(gst["x"])
    assert x.min() > 0 and x.max() < prob.xbar
    assert abs(x.sum() - prob.V) <= 1e-2 * prob.V


@pytest.mark.parametrize("factor", [1.0, 0.5])
def test_table7_cg_tolerance_variants_226(factor):
    # problem 226: Example 1, 64 x 64 elements, 6 levels; "CG tol fixed" (factor 1)
    # and "CG tol decreasing" (tolerance halved after every barrier update)
    prob, nel, levels = _prob(1, 6)
    po = oip.IPParams(stop="barrier", tau_ip=1e-8, pcg_rtol=1e-2, solver="mg", levels=levels,
                      cg_tol_factor=factor)
    st_o, log_o = oip.run(prob, po)
    gst, log = _run_gpu(prob, nel, levels, False, cg_tol_factor=factor)
    cg, cg_o = int(sum(log["pcg_iters"])), int(sum(log_o.pcg_iters))
    xmin, xmin_o = float(N(gst["x"]).min()), float(st_o.x.min())
    print(f"226 factor {factor}: GPU NWT {log['newton']} CG {cg} xmin {xmin:.2e}; "
          f"oracle NWT {log_o.newton} CG {cg_o} xmin {xmin_o:.2e}", flush=True)
    assert log["status"] == log_o.status == "converged"
    assert log["barrier_updates"] == log_o.barrier_updates == 12
    assert abs(log["newton"] - log_o.newton) <= 1
    assert abs(cg - cg_o) <= max(5, 0.03 * cg_o)
    assert abs(xmin - xmin_o) <= 1e-3 * xmin_o
