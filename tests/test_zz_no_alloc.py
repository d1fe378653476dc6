"""The allocation-free PCG entry point (ipmg_pcg_noalloc) against ipmg_pcg, through
the C ABI: two calls in a row on one GPU, the second on a smaller grid, each equal
bit for bit to the allocating entry point on the same data (same kernels, same
deterministic reduction order); a grid beyond the static scratch is rejected."""
import numpy as np
import pytest

from tests.gpu_util import DEV, N, T

pytestmark = pytest.mark.gpu


def _solver(nel, levels, fp32):
    from paper_1606_06201_amd import Solver, inputs
    s = Solver(nel, levels, fp32=fp32, device=DEV)
    s.set_density(T(inputs.density_logistic(nel, seed=5)))
    f = s.load_vector(inputs.point_load(nel))
    return s, f


@pytest.mark.parametrize("fp32", [True, False])
def test_noalloc_pcg_equals_pcg(fp32):
    from paper_1606_06201_amd import _lib as L
    sizes = [((128, 64), 5), ((64, 32), 4)]       # second call on a smaller grid
    for nel, levels in sizes:
        print(f"noalloc pcg fp32={fp32} nel={nel} levels={levels}", flush=True)
        s, f = _solver(nel, levels, fp32)
        assert 0 < s.pcg_noalloc_bytes() <= L.C.c_uint(64 << 20).value
        u_ref, inf_ref = s.pcg(f, rtol=1e-8)              # builds the hierarchy
        u, inf = s.pcg_noalloc(f, rtol=1e-8)
        assert inf["status"] == 0 and inf["iters"] == inf_ref["iters"] > 0
        assert inf["true_relres"] <= 1e-8
        assert np.array_equal(N(u), N(u_ref))
        # a warm start and an iteration limit, against the same call of ipmg_pcg
        u0 = 0.5 * u_ref
        u_ref2, i2 = s.pcg(f, u0=u0, rtol=1e-12, maxit=3, check=False)
        u2, j2 = s.pcg_noalloc(f, u0=u0, rtol=1e-12, maxit=3, check=False)
        assert i2["rc"] == j2["rc"] == L.E_NOT_CONVERGED and i2["iters"] == j2["iters"] == 3
        assert np.array_equal(N(u2), N(u_ref2))
        s.close()


def test_noalloc_pcg_rejections():
    from paper_1606_06201_amd import Solver, _lib as L
    from paper_1606_06201_amd.solver import IPMGError
    s, f = _solver((64, 32), 4, True)
    with pytest.raises(IPMGError) as e:          # hierarchy not built yet: no setup here
        s.pcg_noalloc(f)
    assert e.value.code == L.E_STATE
    s.close()
    big = Solver((2048, 1024), 6, fp32=True, device=DEV)   # 4.2M slots: beyond 64 MiB
    assert big.pcg_noalloc_bytes() > (64 << 20)
    big.set_density(T(np.ones(big.m)))
    big.mg_setup()
    with pytest.raises(IPMGError) as e:
        big.pcg_noalloc(T(np.zeros(big.n_slots)))
    assert e.value.code == L.E_INVALID
    big.close()
