"""GPU parity tests: the HIP library (through its C ABI) against the FP64 oracle
on seeded inputs.  Sizes span several 64-wide tiles plus ragged tails."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, mg, pcg as opcg, sens
from tests.gpu_util import T, N, relerr, grid_and_k0, tip_load

pytestmark = pytest.mark.gpu


def _solver(nel, levels, fp32=False, **kw):
    from paper_1606_06201_amd import Solver
    return Solver(nel, levels, fp32=fp32, **kw)


@pytest.mark.parametrize("dim", [2, 3])
def test_element_matrix_matches_oracle(dim):
    nel = (4, 2) if dim == 2 else (2, 2, 2)
    s = _solver(nel, 1)
    K0 = s.element_matrix()
    np.testing.assert_allclose(K0, fem.element_stiffness(dim), rtol=0, atol=2e-16 * 8)


@pytest.mark.parametrize("nel,levels", [((16, 8), 4), ((8, 4, 4), 3), ((130, 66), 2)])
def test_dof_maps_bit_exact(nel, levels):
    s = _solver(nel, levels)
    g = fem.Grid(nel)
    for lev in range(levels - 1, -1, -1):
        n_slots, n_free, m = s.sizes(lev)
        assert (n_slots, n_free, m) == (g.nslots, len(g.free_to_slot()), g.m)
        assert np.array_equal(s.dof_map(lev), g.free_to_slot())
        assert s.slot_of(lev, g.nel[0], 1, 0 if g.dim == 2 else 1, 1) == \
            g.dim * int(g.node_index(g.nel[0], 1, 0 if g.dim == 2 else 1)) + 1
        if lev > 0:
            g = g.coarsen()


@pytest.mark.parametrize("nel", [(5, 3), (130, 67), (7, 3, 2), (9, 5, 4)])
def test_apply_K_matches_oracle(nel):
    g, K0 = grid_and_k0(nel)
    rng = np.random.default_rng(21)
    x = rng.uniform(1e-3, 1.0, g.m)
    v = rng.standard_normal(g.nslots)            # clamped entries are ignored by contract
    s = _solver(nel, 1)
    s.set_density(T(x))
    y = N(s.apply_K(T(v)))
    ref = fem.apply_free_masked(g, x, K0, v)
    assert relerr(y, ref) < 1e-13
    assert np.all(y[g.clamped_mask()] == 0.0)


def _kproblem(nel, seed=5, lo=1e-2):
    g, K0 = grid_and_k0(nel)
    x = np.random.default_rng(seed).uniform(lo, 1.0, g.m)
    return g, K0, x


@pytest.mark.parametrize("nel,levels,fp32,tol", [((32, 16), 3, False, 1e-11), ((8, 4, 4), 2, False, 1e-11),
                                                  ((32, 16), 4, True, 2e-4), ((8, 8, 4), 3, True, 2e-4),
                                                  ((128, 64), 4, False, 1e-11), ((128, 64), 5, True, 2e-4),
                                                  ((96, 48), 4, False, 1e-11)])
def test_vcycle_matches_oracle(nel, levels, fp32, tol):
    # (128, 64) and (96, 48): the fused passes of the stored 2D levels run on several
    # tiles per level with ragged last tiles.
    g, K0, x = _kproblem(nel)
    H = mg.kstiffness_hierarchy(g, x, K0, levels)
    r = np.random.default_rng(6).standard_normal(g.nslots)
    r[g.clamped_mask()] = 0
    s = _solver(nel, levels, fp32=fp32)
    s.set_density(T(x))
    s.mg_setup()
    for k in range(1, levels):
        w, rho = s.level_damping(k)
        assert abs(rho - H.rho[k]) <= (1e-10 if not fp32 else 1e-5) * H.rho[k]
        assert abs(w - H.omega[k]) <= 1e-5 * H.omega[k]
    z = N(s.vcycle(T(r)))
    zref = mg.vcycle(H, fem.to_free(g, r))
    assert relerr(fem.to_free(g, z), zref) < tol
    assert np.all(z[g.clamped_mask()] == 0)
    # determinism: bitwise identical on a second call
    z2 = N(s.vcycle(T(r)))
    assert np.array_equal(z, z2)


@pytest.mark.parametrize("nel,levels", [((40, 18), 1), ((80, 36), 2), ((8, 4, 4), 1)])
def test_dense_coarse_solve_many_tiles(nel, levels):
    # The coarsest-level factorization, explicit inverse and apply run on 64 x 64
    # tiles: sizes of 1520 (2D) and 600 (3D) unknowns span many tiles and end in a
    # padded one.
    g, K0, x = _kproblem(nel)
    s = _solver(nel, levels)
    s.set_density(T(x))
    s.mg_setup()
    r = np.random.default_rng(8).standard_normal(g.nslots)
    r[g.clamped_mask()] = 0
    z = fem.to_free(g, N(s.vcycle(T(r))))
    if levels == 1:     # one level: the V-cycle is the exact solve
        K = fem.stiffness_free(g, x, K0)
        ref = spla.spsolve(K.tocsc(), fem.to_free(g, r))
        assert relerr(z, ref) < 1e-9
    else:
        H = mg.kstiffness_hierarchy(g, x, K0, levels)
        assert relerr(z, mg.vcycle(H, fem.to_free(g, r))) < 1e-10


@pytest.mark.parametrize("nel,levels,fp32,flexible", [((64, 32), 4, False, False), ((64, 32), 4, True, False),
                                                      ((16, 8, 8), 3, False, False), ((16, 8, 8), 3, True, False),
                                                      ((64, 32), 4, False, True), ((64, 32), 4, True, True),
                                                      ((16, 8, 8), 3, True, True)])
def test_pcg_matches_direct_solve(nel, levels, fp32, flexible):
    g, K0, x = _kproblem(nel, lo=1e-3)
    f = fem.load_vector(g, tip_load(nel))
    s = _solver(nel, levels, fp32=fp32, flexible=flexible)
    s.set_density(T(x))
    u, info = s.pcg(T(f), rtol=1e-8)
    u = N(u)
    assert info["true_relres"] <= 1e-8 and info["status"] == 0
    K = fem.stiffness_free(g, x, K0)
    ustar = spla.spsolve(K.tocsc(), fem.to_free(g, f))
    uf = fem.to_free(g, u)
    # oracle-side true residual of the GPU solution
    rres = np.linalg.norm(fem.to_free(g, f) - K @ uf) / np.linalg.norm(fem.to_free(g, f))
    assert rres <= 1.01e-8
    c_gpu, c_ref = float(f @ u), float(fem.to_free(g, f) @ ustar)
    assert abs(c_gpu - c_ref) <= 1e-6 * abs(c_ref)
    # same iteration count as the oracle's FP64 MG-PCG (mixed precision within a few)
    H = mg.kstiffness_hierarchy(g, x, K0, levels)
    ref = opcg.mg_pcg(H, fem.to_free(g, f), rtol=1e-8, flexible=flexible)
    assert abs(info["iters"] - ref.iters) <= (0 if not fp32 else 2), (info["iters"], ref.iters)


def test_pcg_contrast_1e6_threshold_density():
    from paper_1606_06201_amd import inputs
    nel, levels = (128, 64), 5
    g, K0 = grid_and_k0(nel)
    x = inputs.density_threshold(nel, seed=2)
    f = fem.load_vector(g, tip_load(nel))
    K = fem.stiffness_free(g, x, K0)
    ustar = spla.spsolve(K.tocsc(), fem.to_free(g, f))
    c_ref = float(fem.to_free(g, f) @ ustar)
    for fp32 in (False, True):
        s = _solver(nel, levels, fp32=fp32)
        s.set_density(T(x))
        u, info = s.pcg(T(f), rtol=1e-8)
        assert info["true_relres"] <= 1e-8
        assert abs(float(f @ N(u)) - c_ref) <= 1e-6 * c_ref


def test_pcg_edge_cases():
    nel = (16, 8)
    g, K0, x = _kproblem(nel)
    s = _solver(nel, 3)
    s.set_density(T(x))
    # zero right-hand side -> zero solution, no iterations
    u, info = s.pcg(T(np.zeros(g.nslots)))
    assert info["iters"] == 0 and np.all(N(u) == 0)
    # initial guess equal to the solution -> no iterations
    f = fem.load_vector(g, tip_load(nel))
    u, _ = s.pcg(T(f), rtol=1e-10)
    u2, info2 = s.pcg(T(f), u0=u, rtol=1e-8)
    assert info2["iters"] == 0
    # maxit reached -> status reported, iterate returned
    u3, info3 = s.pcg(T(f), rtol=1e-14, maxit=2, check=False)
    assert info3["iters"] == 2 and info3["rc"] != 0
    # one level: the V-cycle is the exact coarse solve -> one iteration
    s1 = _solver((8, 4), 1)
    x1 = np.random.default_rng(1).uniform(0.1, 1, 32)
    s1.set_density(T(x1))
    u4, info4 = s1.pcg(T(fem.load_vector(fem.Grid((8, 4)), tip_load((8, 4)))), rtol=1e-10)
    assert info4["iters"] == 1


@pytest.mark.parametrize("env", ["IPMG_NO_FOLD_SOLUTION", "IPMG_NO_FOLD_RN2"])
@pytest.mark.parametrize("fp32", [False, True])
def test_pcg_folded_steps_are_exact(env, fp32, monkeypatch):
    # With the register-blocked passes a PCG step's z += alpha p is done by the next
    # step's direction kernel (the last step's by a flush after the loop: converged,
    # stopped at maxit, or zero steps), and its ||r||^2 finalize by the first pass of
    # the V-cycle.  Same arithmetic in the same order: the iterates and counts equal
    # those of the separate kernels bit for bit.
    nel, levels = (96, 48), 4
    g, K0, x = _kproblem(nel)
    f = fem.load_vector(g, tip_load(nel))
    monkeypatch.setenv("IPMG_TILED_MIN_NODES", "0")
    out = {}
    for off in ("0", "1"):
        monkeypatch.setenv(env, off)
        s = _solver(nel, levels, fp32=fp32)
        s.set_density(T(x))
        u, info = s.pcg(T(f), rtol=1e-9)
        u2, info2 = s.pcg(T(f), rtol=1e-12, maxit=3, check=False)
        u3, info3 = s.pcg(T(f), u0=u, rtol=1e-3)
        assert info["true_relres"] <= 1e-9
        out[off] = (N(u), info["iters"], N(u2), info2["iters"], N(u3), info3["iters"])
    monkeypatch.delenv(env)
    a, b = out["0"], out["1"]
    assert a[1] == b[1] and a[3] == b[3] == 3 and a[5] == b[5] == 0
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2]) and np.array_equal(a[4], b[4])


@pytest.mark.parametrize("nj32,nj64,nj_dir", [("1", "1", "1"), ("2", "4", "2"), ("8", "8", "3")])
@pytest.mark.parametrize("fp32", [False, True])
def test_register_block_widths_match_oracle(nj32, nj64, nj_dir, fp32, monkeypatch):
    # Nodes per thread of the register-blocked level passes (FP32 / FP64) and of the
    # PCG direction kernel, on every level (several tiles and ragged tails at each
    # width): V-cycle and PCG as the oracle's.
    nel, levels = (96, 48), 4
    g, K0, x = _kproblem(nel)
    H = mg.kstiffness_hierarchy(g, x, K0, levels)
    r = np.random.default_rng(6).standard_normal(g.nslots)
    r[g.clamped_mask()] = 0
    for k, v in (("IPMG_TILED_MIN_NODES", "0"), ("IPMG_NJ32", nj32), ("IPMG_NJ64", nj64), ("IPMG_NJ_DIR", nj_dir)):
        monkeypatch.setenv(k, v)
    s = _solver(nel, levels, fp32=fp32)
    for k in ("IPMG_TILED_MIN_NODES", "IPMG_NJ32", "IPMG_NJ64", "IPMG_NJ_DIR"):
        monkeypatch.delenv(k)
    s.set_density(T(x))
    s.mg_setup()
    z = N(s.vcycle(T(r)))
    assert relerr(fem.to_free(g, z), mg.vcycle(H, fem.to_free(g, r))) < (2e-4 if fp32 else 1e-11)
    f = fem.load_vector(g, tip_load(nel))
    u, info = s.pcg(T(f), rtol=1e-8)
    assert info["true_relres"] <= 1e-8
    ref = opcg.mg_pcg(H, fem.to_free(g, f), rtol=1e-8)
    assert abs(info["iters"] - ref.iters) <= (2 if fp32 else 1), (info["iters"], ref.iters)


def test_invalid_arguments_raise():
    import torch
    from paper_1606_06201_amd import IPMGError, Solver
    with pytest.raises(IPMGError):
        Solver((10, 6), 3)                          # 6 not divisible by 4
    s = _solver((8, 4), 2)
    with pytest.raises(IPMGError):
        s.set_density(T(-np.ones(32)))              # x <= 0
    with pytest.raises(TypeError):
        s.set_density(torch.ones(32, dtype=torch.float32, device="cuda:0"))
    with pytest.raises(ValueError):
        s.set_density(T(np.ones(31)))
    with pytest.raises(IPMGError):
        s.pcg(T(np.ones(s.n_slots)))                # before any density -> state error


def test_element_sensitivities_match_oracle():
    nel = (33 * 2, 17 * 2)
    g, K0, x = _kproblem(nel)
    rng = np.random.default_rng(9)
    w, u = rng.standard_normal(g.nslots), rng.standard_normal(g.nslots)
    s = _solver(nel, 1)
    gs = N(s.element_sens(T(w), T(u), -0.5))
    wm, um = w.copy(), u.copy()
    wm[g.clamped_mask()] = 0
    um[g.clamped_mask()] = 0
    ref = -0.5 * sens.element_products(g, K0, wm, um)
    assert relerr(gs, ref) < 1e-13


@pytest.mark.parametrize("nel,levels", [((256, 128), 4), ((96, 48), 3), ((72, 40), 3)])
def test_first_coarse_level_matrix_cores_match_vector_units(nel, levels, monkeypatch):
    # The first coarse level's fused passes with the element products on the matrix
    # cores against the same passes on the vector units (FP32 V-cycle).  Each
    # 32x32x2 step rounds like two chained FMAs in the order of the vector code, so
    # the results agree to FP32 rounding (bit for bit on MI355X); the bound allows
    # a reordering.  The grids give one or several tiles per direction with ragged
    # last tiles; every element block of a tile ends in a partly filled group of 32.
    g, K0, x = _kproblem(nel, seed=9)
    r = np.random.default_rng(10).standard_normal(g.nslots)
    r[g.clamped_mask()] = 0
    z = {}
    for v in ("0", "1"):
        monkeypatch.setenv("IPMG_NO_MFMA", v)
        s = _solver(nel, levels, fp32=True)
        s.set_density(T(x))
        s.mg_setup()
        z[v] = N(s.vcycle(T(r)))
    monkeypatch.delenv("IPMG_NO_MFMA")
    print(f"{nel}: matrix cores vs vector units bitwise equal: {np.array_equal(z['0'], z['1'])}", flush=True)
    assert relerr(z["0"], z["1"]) < 1e-6


@pytest.mark.parametrize("nel,levels", [((256, 128), 4), ((248, 124), 3), ((124, 60), 3), ((60, 30), 2), ((8, 4), 2)])
@pytest.mark.parametrize("fp32", [True, False])
def test_finest_level_lane_shared_tiles_match_per_thread_tiles(nel, levels, fp32, monkeypatch):
    # The finest level's register-blocked passes on lane-shared tiles (each lane
    # forms one column of the neighbourhood and takes the other two from its
    # neighbouring lanes; 62 output columns per tile) against the per-thread tiles.
    # Column counts 257, 249, 125, 61 and 9 leave 9, 1, 1, 61 and 9 columns in the
    # last tile.  Tiles are forced on every level size.
    #  - Prolongation as a pass of its own: every finest-level pass forms the same
    #    values in the same order, so the V-cycles agree bit for bit.
    #  - FP64, prolongation folded into the first post-sweep: the lane-shared pass
    #    sums z2 + P zc as the prolongation pass does, bit for bit.  (The per-thread
    #    folded pass differs from it by rounding.)
    #  - Default paths: equal to rounding, the same PCG iteration count.
    monkeypatch.setenv("IPMG_TILED_MIN_NODES", "0")
    g, K0, x = _kproblem(nel, seed=12)
    r = np.random.default_rng(13).standard_normal(g.nslots)
    r[g.clamped_mask()] = 0
    f = fem.load_vector(g, tip_load(nel))
    z, its = {}, {}
    for ls in ("0", "1"):
        for fold in ("0", "1"):
            monkeypatch.setenv("IPMG_NO_LANE_SHARE", ls)
            monkeypatch.setenv("IPMG_NO_FOLD_PROLONG", fold)
            s = _solver(nel, levels, fp32=fp32)
            s.set_density(T(x))
            s.mg_setup()
            z[ls, fold] = N(s.vcycle(T(r)))
            _, info = s.pcg(T(f), rtol=1e-8)
            assert info["true_relres"] <= 1e-8
            its[ls, fold] = info["iters"]
    for k in ("IPMG_NO_LANE_SHARE", "IPMG_NO_FOLD_PROLONG", "IPMG_TILED_MIN_NODES"):
        monkeypatch.delenv(k)
    assert np.array_equal(z["0", "1"], z["1", "1"])
    assert its["0", "1"] == its["1", "1"]
    if not fp32:
        assert np.array_equal(z["0", "0"], z["1", "1"])
    assert relerr(z["0", "0"], z["1", "0"]) < (1e-6 if fp32 else 1e-14)
    assert abs(its["0", "0"] - its["1", "0"]) <= 1


@pytest.mark.parametrize("nel,levels", [((256, 128), 4), ((248, 124), 3), ((124, 60), 3), ((60, 30), 2), ((8, 4), 2)])
@pytest.mark.parametrize("fp32", [True, False])
def test_finest_level_sweeps_and_residual_in_one_pass_match_separate_passes(nel, levels, fp32, monkeypatch):
    # The two pre-smoothing sweeps from zero and the residual of their result in one
    # lane-shared pass (60 output columns per tile; column counts 257, 249, 125, 61
    # and 9 leave 17, 9, 5, 1 and 9 columns in the last tile) against the two
    # separate passes: z2 and the residual are formed by the same formulas in the same
    # order, so in FP64 the V-cycles agree bit for bit; in FP32 the compiler fuses a
    # multiply and an add differently in the two kernels, so they agree to a few ulps.
    # PCG takes the same iterations (FP64) or within one (FP32).
    monkeypatch.setenv("IPMG_TILED_MIN_NODES", "0")
    g, K0, x = _kproblem(nel, seed=14)
    r = np.random.default_rng(15).standard_normal(g.nslots)
    r[g.clamped_mask()] = 0
    f = fem.load_vector(g, tip_load(nel))
    z, its = {}, {}
    for v in ("0", "1"):
        monkeypatch.setenv("IPMG_NO_JACOBI2_RESID", v)
        s = _solver(nel, levels, fp32=fp32)
        s.set_density(T(x))
        s.mg_setup()
        z[v] = N(s.vcycle(T(r)))
        _, info = s.pcg(T(f), rtol=1e-8)
        assert info["true_relres"] <= 1e-8
        its[v] = info["iters"]
    monkeypatch.delenv("IPMG_NO_JACOBI2_RESID")
    monkeypatch.delenv("IPMG_TILED_MIN_NODES")
    if fp32:
        assert relerr(z["0"], z["1"]) < 1e-6
        assert abs(its["0"] - its["1"]) <= 1
    else:
        assert np.array_equal(z["0"], z["1"])
        assert its["0"] == its["1"]


@pytest.mark.parametrize("nel,levels", [((256, 128), 4), ((248, 124), 3), ((124, 60), 3), ((60, 30), 2), ((8, 4), 2)])
@pytest.mark.parametrize("fp32", [True, False])
def test_finest_level_prolongation_and_post_sweeps_in_one_pass_match_separate_passes(nel, levels, fp32,
                                                                                      monkeypatch):
    # z2 + P zc and both post-smoothing sweeps in one lane-shared pass against the
    # folded-prolongation sweep and the last sweep as separate passes.  Same formulas
    # and order: the FP64 V-cycles agree bit for bit, the FP32 ones to a few ulps.  In
    # PCG the last sweep's partial sums for the ratio are grouped by the new tiles, so
    # the iterates agree to rounding and the iteration counts within one.
    monkeypatch.setenv("IPMG_TILED_MIN_NODES", "0")
    g, K0, x = _kproblem(nel, seed=16)
    r = np.random.default_rng(17).standard_normal(g.nslots)
    r[g.clamped_mask()] = 0
    f = fem.load_vector(g, tip_load(nel))
    z, its, u = {}, {}, {}
    for v in ("0", "1"):
        monkeypatch.setenv("IPMG_NO_PJACOBI2", v)
        s = _solver(nel, levels, fp32=fp32)
        s.set_density(T(x))
        s.mg_setup()
        z[v] = N(s.vcycle(T(r)))
        uu, info = s.pcg(T(f), rtol=1e-8)
        assert info["true_relres"] <= 1e-8
        its[v], u[v] = info["iters"], N(uu)
    monkeypatch.delenv("IPMG_NO_PJACOBI2")
    monkeypatch.delenv("IPMG_TILED_MIN_NODES")
    if fp32:
        assert relerr(z["0"], z["1"]) < 1e-6
    else:
        assert np.array_equal(z["0"], z["1"])
    assert abs(its["0"] - its["1"]) <= 1
    assert relerr(u["0"], u["1"]) < 1e-7


@pytest.mark.parametrize("env,val", [("IPMG_STORED_COARSE", "1"), ("IPMG_NO_LANE_SHARE", "1"),
                                     ("IPMG_NO_JACOBI2_RESID", "1"), ("IPMG_NO_PJACOBI2", "1"),
                                     ("IPMG_TILED_MIN_NODES", "0"), ("IPMG_UNTILED", "1"), ("IPMG_UNFUSED", "1"),
                                     ("IPMG_UNSTAGED", "1"), ("IPMG_STAGED_MAX_NODES", "1048576"),
                                     ("IPMG_NO_FOLD_PROLONG", "1"), ("IPMG_NO_FOLD_RESTRICT", "1"),
                                     ("IPMG_NO_MFMA", "1")])
@pytest.mark.parametrize("nel,levels,fp32,tol", [((32, 16), 4, False, 1e-11), ((32, 16), 4, True, 2e-4),
                                                  ((8, 4, 4), 3, False, 1e-11), ((128, 64), 4, False, 1e-11),
                                                  ((128, 64), 4, True, 2e-4)])
def test_vcycle_alternative_paths_match_oracle(env, val, nel, levels, fp32, tol, monkeypatch):
    # Opt-in execution paths (stored first coarse level; register-blocked 2D tiles on
    # every level; one node per thread everywhere; separate passes instead of the
    # fused coarse ones; fused passes reading global memory, or staged, on every
    # coarse level; prolongation and restriction as passes of their own; the first
    # coarse level's element products on the vector units instead of the matrix
    # cores) must give the same V-cycle as the default path and the oracle.
    g, K0, x = _kproblem(nel)
    H = mg.kstiffness_hierarchy(g, x, K0, levels)
    r = np.random.default_rng(6).standard_normal(g.nslots)
    r[g.clamped_mask()] = 0
    monkeypatch.setenv(env, val)
    s = _solver(nel, levels, fp32=fp32)
    monkeypatch.delenv(env)
    s.set_density(T(x))
    s.mg_setup()
    z = N(s.vcycle(T(r)))
    assert relerr(fem.to_free(g, z), mg.vcycle(H, fem.to_free(g, r))) < tol
    f = fem.load_vector(g, tip_load(nel))
    u, info = s.pcg(T(f), rtol=1e-8)
    assert info["true_relres"] <= 1e-8


@pytest.mark.parametrize("env,val", [("IPMG_ELEM_APPLY3_MIN", "0"), ("IPMG_NO_ELEM_APPLY3", "1"),
                                     ("IPMG_NO_ELEM_FINE3", "1")])
@pytest.mark.parametrize("nel,levels,fp32,tol", [((16, 8, 8), 3, False, 1e-11), ((16, 8, 8), 3, True, 2e-4),
                                                  ((12, 8, 4), 3, False, 1e-11)])
def test_vcycle_3d_element_products_match_oracle(env, val, nel, levels, fp32, tol, monkeypatch):
    # 3D stored coarse levels: element products y_e = E_e v_e formed by a pass of
    # their own and gathered three per element by the node passes (forced on every
    # stored level), or the node passes' own gathers of E_e and v_e; both against
    # the oracle's V-cycle (a ragged 12 x 8 x 4 grid included).
    g, K0, x = _kproblem(nel)
    H = mg.kstiffness_hierarchy(g, x, K0, levels)
    r = np.random.default_rng(8).standard_normal(g.nslots)
    r[g.clamped_mask()] = 0
    monkeypatch.setenv(env, val)
    s = _solver(nel, levels, fp32=fp32)
    monkeypatch.delenv(env)
    s.set_density(T(x))
    s.mg_setup()
    for k in range(1, levels):
        w, rho = s.level_damping(k)
        assert abs(rho - H.rho[k]) <= (1e-9 if not fp32 else 1e-4) * H.rho[k]
    z = N(s.vcycle(T(r)))
    assert relerr(fem.to_free(g, z), mg.vcycle(H, fem.to_free(g, r))) < tol
