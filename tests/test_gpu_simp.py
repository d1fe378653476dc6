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
