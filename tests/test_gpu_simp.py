"""SIMP model with a density filter on the GPU (Sec. 9) against the oracle: the
filter W and its transpose, and the compliance and its gradient
-W'(p x~^(p-1) o u_e'K0u_e) of the penalised, filtered stiffness."""
import numpy as np
import pytest

from oracle import fem, simp
from tests.gpu_util import T, N, relerr

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nel,rmin", [((64, 32), 2.0), ((64, 32), 2.5), ((37, 11), 3.0), ((64, 32), 1.0),
                                      ((8, 6, 4), 2.0)])
def test_filter_matches_oracle(nel, rmin):
    from paper_1606_06201_amd import Solver
    g = fem.Grid(nel)
    W = simp.filter_matrix(g, rmin)
    v = np.random.default_rng(12).uniform(0.0, 1.0, g.m)
    s = Solver(nel, 1, fp32=False)
    assert relerr(N(s.filter(T(v), rmin)), W @ v) < 1e-14
    assert relerr(N(s.filter(T(v), rmin, transpose=True)), W.T @ v) < 1e-14
    if rmin == 1.0:
        assert np.array_equal(N(s.filter(T(v), rmin)), v)


@pytest.mark.parametrize("fp32", [False, True])
def test_simp_compliance_and_gradient_match_oracle(fp32):
    # Example 4 settings (Sec. 9.1: rmin = 2, Manhattan) with p = 3 at seeded densities
    from paper_1606_06201_amd import Solver, inputs
    nel, levels = (64, 32), 4
    g = fem.Grid(nel)
    K0 = fem.element_stiffness(2)
    f = fem.load_vector(g, inputs.point_load(nel))
    x = np.random.default_rng(13).uniform(0.2, 1.0, g.m)
    c_o, u_o, grad_o, xt_o = simp.compliance_and_gradient(g, K0, f, x, 2.0, 3.0)
    s = Solver(nel, levels, fp32=fp32)
    u, grad, info = s.simp_compliance(T(x), T(f), rmin=2.0, p=3.0, rtol=1e-10)
    print(f"SIMP 64x32 fp32={fp32}: {info['iters']} PCG iterations, compliance {info['bu']:.10g} "
          f"(oracle {c_o:.10g})", flush=True)
    assert info["rc"] == 0 and info["true_relres"] <= 1e-10
    assert abs(info["bu"] - c_o) <= 1e-9 * c_o
    assert relerr(fem.to_free(g, N(u)), u_o) < 1e-8
    assert relerr(N(grad), grad_o) < 1e-8
    # the filter keeps the volume: the gradient's Euler sum is -p c for x~ = W x linear in x
    assert abs(float(x @ N(grad)) + 3.0 * c_o) <= 1e-8 * c_o


# ---- interior-point method on the SIMP model (Sec. 9) --------------------------
def _simp_ip_problem(nel, xbar=3.0, vfrac=0.4, loads=None):
    from oracle import simp as osimp
    from paper_1606_06201_amd import inputs
    g = fem.Grid(nel)
    f = fem.load_vector(g, inputs.point_load(nel) if loads is None else loads)
    return osimp.SimpProblem(g, fem.element_stiffness(2), f, vfrac * g.m, xbar, rmin=2.0, p=3.0)


def _gpu_state_np(st):
    return {k: (N(v) if hasattr(v, "detach") else v) for k, v in st.items()}


def test_simp_ip_steps_match_oracle_newton_steps():
    # Newton steps on the GPU (PCG on the exact matrix-free Z^ to 1e-11) against the
    # oracle's steps with direct solves of its assembled Z^, from the same start
    from oracle import ip as oip
    from paper_1606_06201_amd import Solver
    nel, levels = (32, 16), 3
    prob = _simp_ip_problem(nel)
    po = oip.IPParams(solver="direct")
    st_o, _ = oip.initial_state(prob, po)
    s = Solver(nel, levels, fp32=False)
    params = s.ip_params(prob.V, prob.xbar, pcg_rtol=1e-11, pcg_maxit=4000)
    st, init = s.ip_init(T(prob.f_slots), params, simp=(2.0, 3.0))
    g = prob.grid
    assert relerr(fem.to_free(g, N(st["u"])), st_o.u) < 1e-9
    for k in range(6):
        inf = s.ip_step(T(prob.f_slots), params, st, simp=(2.0, 3.0))
        st_o, alpha_o, _ = oip.newton_step(prob, st_o, po)
        nwt_o, gap_o, _ = prob.measures(st_o)
        if nwt_o <= po.tau_nwt:
            st_o.s *= po.sigma
            st_o.r *= po.sigma
        print(f"step {k + 1}: PCG {inf['pcg_iters']}, alpha GPU {inf['alpha']:.10f} oracle {alpha_o:.10f}, "
              f"nwt {inf['nwt']:.6f} / {nwt_o:.6f}", flush=True)
        assert inf["rc"] == 0 and inf["pcg_status"] == 0
        assert abs(inf["alpha"] - alpha_o) <= 1e-7
        assert abs(inf["nwt"] - nwt_o) <= 1e-6 * max(1.0, nwt_o)
        assert relerr(N(st["x"]), st_o.x) < 1e-7
        assert relerr(fem.to_free(g, N(st["u"])), st_o.u) < 1e-7
        assert abs(st["lam"] - st_o.lam) <= 1e-7 * max(1.0, abs(st_o.lam))
        assert st["s"] == pytest.approx(st_o.s, rel=1e-12)


@pytest.mark.parametrize("fp32", [False, True])
def test_simp_newton_solve_iterations_match_oracle(fp32):
    # the first Newton system: PCG on Z^ preconditioned by the V-cycle of the
    # element-local matrix, GPU against the oracle's same algorithm (tolerance 1e-8)
    from oracle import ip as oip
    from paper_1606_06201_amd import Solver
    nel, levels = (64, 32), 4
    prob = _simp_ip_problem(nel)
    po = oip.IPParams(solver="mg", levels=levels, pcg_rtol=1e-8)
    st_o, _ = oip.initial_state(prob, oip.IPParams(solver="direct"))
    Z, rhs, parts = prob.z_system(st_o)
    Zp = prob.z_preconditioner(st_o, parts)
    _, it_o, status_o, _ = oip.solve_linear(Z, rhs, po, prob.grid, True, Zprec=Zp)
    s = Solver(nel, levels, fp32=fp32)
    params = s.ip_params(prob.V, prob.xbar, pcg_rtol=1e-8)
    st, _ = s.ip_init(T(prob.f_slots), params, simp=(2.0, 3.0))
    inf = s.ip_step(T(prob.f_slots), params, st, simp=(2.0, 3.0))
    print(f"first SIMP Newton system fp32={fp32}: PCG GPU {inf['pcg_iters']} oracle {it_o}", flush=True)
    assert status_o == "ok" and inf["pcg_status"] == 0 and inf["pcg_true_relres"] <= 1e-8
    assert abs(inf["pcg_iters"] - it_o) <= (2 if fp32 else 1)


def test_simp_ip_run_example4_settings_matches_oracle():
    # Example 4 (Sec. 9.1): Example 2's problem 425 (64 x 32, 5 levels) with xbar = 3,
    # rmin = 2 (Manhattan), p = 3, the paper's inexact Newton solves (1e-2) with the
    # tolerance halved after every barrier update (Sec. 8.1 "CG tol decreasing"),
    # stop at max(s, r) <= 1e-8.  Non-convex: runs whose solves differ in rounding
    # may end in neighbouring local minima (the paper reports the same for its two
    # solvers), so counts are compared loosely and the compliance to 1e-2.
    from oracle import ip as oip
    from paper_1606_06201_amd import Solver, inputs
    nel, levels, loads, V, _ = inputs.paper_problem(2, 5)
    prob = _simp_ip_problem(nel, xbar=3.0, loads=loads)
    prob.V = V
    po = oip.IPParams(stop="barrier", tau_ip=1e-8, solver="mg", levels=levels, pcg_rtol=1e-2, max_newton=300,
                      cg_tol_factor=0.5)
    st_o, log_o = oip.run(prob, po)
    s = Solver(nel, levels, fp32=False)
    params = s.ip_params_paper(V, 3.0)
    params.max_newton = 300
    gst, log = s.ip_run(T(prob.f_slots), params, cg_tol_factor=0.5, simp=(2.0, 3.0))
    c, c_o = float(prob.f_slots @ N(gst["u"])), float(prob.f @ st_o.u)
    print(f"SIMP 425: GPU {log['status']} NWT {log['newton']} CG {sum(log['pcg_iters'])} compliance {c:.6f}; "
          f"oracle {log_o.status} NWT {log_o.newton} CG {sum(log_o.pcg_iters)} compliance {c_o:.6f}", flush=True)
    assert log["status"] == log_o.status == "converged"
    assert log["barrier_updates"] == log_o.barrier_updates == 12
    assert abs(c - c_o) <= 1e-2 * c_o
    x = N(gst["x"])
    assert x.min() > 0 and x.max() < 3.0 and abs(x.sum() - V) <= 1e-2 * V
