"""GPU parity of the LOD step (C ABI, HIP kernels) against the FP64 oracle.

Bar: FP64 storage/arithmetic within 1e-12 normwise relative error per
substrate (max|d| / max|ref|); FP32 storage with FP64 arithmetic within 1e-5.
Cases span several tiles and ragged tails for every kernel kind and plan,
degenerate line lengths (1, 2, 3), non-cubic grids, duplicate and
overlapping source/Dirichlet entries, and the workloads at full size
(sampled or through properties that hold at any size).
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import gpu_run, make_grid, oracle_lists, oracle_run, rel_err, small_problem, upload

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
F32_TOL = 1e-5


def _plan(kind, axis, n, S, m=8, lpw=16, rows=1):
    if kind == 0:
        return (0, 0, 0, 0)
    K = math.ceil(n / m)
    if kind in (1, 3):
        spw = 64 // lpw
        K = math.ceil(K / spw) * spw
        return (kind, m, K * lpw // 64, lpw)
    return (2, m, math.ceil(rows * K * S / 64), rows)


def test_gaussian_64cube_matches_oracle():
    p = workloads.config(1)
    ref = oracle_run(p)
    got = gpu_run(p)
    emax, e2 = rel_err(got, ref)
    print(f"gaussian 64^3x1 f64: e_max={emax:.3e} e_2={e2:.3e}")
    assert emax <= F64_TOL
    # mass decays exactly by (1+beta)^-3 per step (no sources, no Dirichlet)
    beta = p.dt * p.lam[0] / 3.0
    ref_mass = np.sum(p.u0) * (1.0 + beta) ** (-3 * p.nsteps)
    assert abs(np.sum(got) - ref_mass) <= 1e-12 * ref_mass


def test_cells_recipe_scaled_matches_oracle():
    p = workloads.config(2, n=48, nsub=3, n_sources=3000, nsteps=5)
    ref = oracle_run(p)
    got = gpu_run(p)
    emax, e2 = rel_err(got, ref)
    print(f"cells 48^3x3 f64: e_max={emax:.3e} e_2={e2:.3e}")
    assert emax <= F64_TOL
    assert np.all(got.reshape(-1, p.S)[p.dr.voxel, 0] == 38.0)


NONCUBIC = (37, 29, 41)


@pytest.mark.parametrize("m", [4, 8, 16, 32])
@pytest.mark.parametrize("lpw", [16, 32, 64])
def test_strided_kernel_plans(m, lpw):
    nx, ny, nz = NONCUBIC
    S = 3
    p = small_problem(NONCUBIC, S, seed=200 + m + lpw, nsrc=300, ndir=40, nsteps=2)
    plans = {1: _plan(1, 1, ny, S, m=m, lpw=lpw), 2: _plan(1, 2, nz, S, m=m, lpw=lpw),
             0: _plan(0, 0, nx, S)}
    ref = oracle_run(p)
    got = gpu_run(p, plans=plans)
    emax, _ = rel_err(got, ref)
    assert emax <= F64_TOL, (m, lpw, emax)


@pytest.mark.parametrize("m", [4, 8, 16, 32])
@pytest.mark.parametrize("rows", [1, 2, 3])
def test_xtile_kernel_plans(m, rows):
    nx, ny, nz = NONCUBIC
    S = 3
    p = small_problem(NONCUBIC, S, seed=300 + m + rows, nsrc=300, ndir=40, nsteps=2)
    plans = {0: _plan(2, 0, nx, S, m=m, rows=rows)}
    ref = oracle_run(p)
    got = gpu_run(p, plans=plans)
    emax, _ = rel_err(got, ref)
    assert emax <= F64_TOL, (m, rows, emax)


@pytest.mark.parametrize("m", [8, 16])
@pytest.mark.parametrize("rows", [1, 2, 3])
@pytest.mark.parametrize("dtype,tol", [("f64", F64_TOL), ("f32", F32_TOL)])
def test_xpipe_kernel_plans(m, rows, dtype, tol):
    # the pipelined row-tile kernel needs rows of whole 16-byte chunks: an x
    # extent of 48 voxels and 4 substrates; 128 x 101 rows give more row
    # tiles than the persistent grid holds (256 CUs x at most 12 blocks), so
    # blocks loop, and 3 rows per tile leave a one-row last tile
    shape = (48, 128, 101)
    S = 4
    p = small_problem(shape, S, seed=330 + m + rows, nsrc=300, ndir=40, nsteps=2)
    K = math.ceil(shape[0] / m)
    plans = {0: (4, m, math.ceil(rows * K * S / 64), rows)}
    ref = oracle_run(p)
    got = gpu_run(p, dtype=dtype, plans=plans)
    emax, _ = rel_err(got, ref)
    assert emax <= tol, (m, rows, emax)


@pytest.mark.parametrize("m", [4, 8, 16, 32])
@pytest.mark.parametrize("lpw", [16, 32, 64])
def test_xrows_kernel_plans(m, lpw):
    nx, ny, nz = NONCUBIC
    S = 3
    p = small_problem(NONCUBIC, S, seed=350 + m + lpw, nsrc=300, ndir=40, nsteps=2)
    plans = {0: _plan(3, 0, nx, S, m=m, lpw=lpw)}
    ref = oracle_run(p)
    got = gpu_run(p, plans=plans)
    emax, _ = rel_err(got, ref)
    assert emax <= F64_TOL, (m, lpw, emax)


@pytest.mark.parametrize("sched,w", [(1, 1), (1, 3), (1, 5), (1, 16), (1, 37), (2, 1), (2, 4), (2, 7), (2, 41)])
@pytest.mark.parametrize("dtype,tol", [("f64", F64_TOL), ("f32", F32_TOL)])
def test_fused_slab_schedule(sched, w, dtype, tol):
    # two sweeps back to back on slabs, Dirichlet entries spread over the slabs
    p = small_problem(NONCUBIC, 3, seed=380 + w, nsrc=300, ndir=60, nsteps=3)
    ref = oracle_run(p)
    got = gpu_run(p, dtype=dtype, schedule=(sched, w))
    emax, _ = rel_err(got, ref)
    assert emax <= tol, (w, emax)
    assert np.all(got.reshape(-1, 3)[p.dr.voxel] == p.dr.value.astype(got.dtype))


def test_fused_and_plain_schedules_agree_bitwise():
    p = small_problem((40, 33, 27), 4, seed=390, nsrc=200, ndir=30, nsteps=3)
    a = gpu_run(p, schedule=(0, 0))
    b = gpu_run(p, schedule=(1, 6))
    c = gpu_run(p, schedule=(2, 5))
    assert np.array_equal(a, b)
    assert np.array_equal(a, c)


@pytest.mark.parametrize("shape", [(1000, 20, 24), (24, 1000, 20), (20, 24, 1000)])
@pytest.mark.parametrize("dtype,tol", [("f64", F64_TOL), ("f32", F32_TOL)])
def test_compressed_coefficient_rows(shape, dtype, tol):
    # 1000-long lines with 8 substrates: the full LDS coefficient table of
    # the strided kernel would take more than 48 KB, so the sweep along the
    # long axis builds its coefficient rows from the exact compressed table
    # (head, interior constant, last slot); D up to 1e5 keeps the head short
    S = 8
    p = small_problem(shape, S, seed=450 + shape.index(1000), nsrc=500, ndir=60, nsteps=2)
    ref = oracle_run(p)
    got = gpu_run(p, dtype=dtype)
    emax, _ = rel_err(got, ref)
    assert emax <= tol, (shape, dtype, emax)


def test_x_rows_with_the_global_coefficient_table():
    # 2000-voxel rows x 8 substrates with r = 1e5: the constants do not settle
    # within 512 slots (no compressed form) and the full table exceeds the
    # LDS, so the x rows read their constants from the global table
    S = 8
    p = small_problem((2000, 3, 2), S, seed=470, nsrc=40, ndir=8, nsteps=2)
    p.D = np.full(S, 1e9)
    # bar: each of the 6 solves (2 steps x 3 axes) may amplify the rounding
    # difference between the reciprocal-multiply and the oracle's division by
    # cond(A) <= 1 + 4r (r = 1e5 on x); the other axes are far better
    # conditioned, so 6 (1 + 4r) 2^-53 bounds the whole run
    r = p.dt * p.D[0] / p.h[0] ** 2
    tol = 6 * (1 + 4 * r) * 2.0 ** -53
    ref = oracle_run(p)
    got = gpu_run(p)
    emax, _ = rel_err(got, ref)
    print(f"r = {r:.3g}: e_max = {emax:.3e} (bar {tol:.2e})")
    assert emax <= tol, emax


def test_line_kernel_all_axes():
    p = small_problem(NONCUBIC, 2, seed=400, nsrc=100, ndir=10, nsteps=2)
    plans = {a: (0, 0, 0, 0) for a in range(3)}
    ref = oracle_run(p)
    got = gpu_run(p, plans=plans)
    assert rel_err(got, ref)[0] <= F64_TOL


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 5, 7), (2, 1, 3), (3, 4, 1), (5, 2, 2), (1, 1, 9),
                                   (9, 1, 1), (2, 3, 64), (130, 3, 2)])
@pytest.mark.parametrize("S", [1, 5])
def test_degenerate_and_tiny_shapes(shape, S):
    p = small_problem(shape, S, seed=sum(shape) * 7 + S, nsrc=3, ndir=2, nsteps=3)
    ref = oracle_run(p)
    got = gpu_run(p)
    assert rel_err(got, ref)[0] <= F64_TOL


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("dtype,tol", [("f64", F64_TOL), ("f32", F32_TOL)])
def test_single_sweep(axis, dtype, tol):
    import torch
    p = small_problem((33, 20, 27), 4, seed=500 + axis)
    ref = np.array(p.field(), copy=True)
    oracle.sweep(ref, p.h, p.D, p.lam, p.dt, axis)
    g = make_grid(p, dtype)
    u = upload(p, g)
    g.sweep(u, axis)
    torch.cuda.synchronize()
    got = g.read_field(u)
    assert rel_err(got, ref)[0] <= tol


@pytest.mark.parametrize("case", [1, 2])
def test_fp32_storage_fp64_arithmetic(case):
    if case == 1:
        p = workloads.config(1)
    else:
        p = workloads.config(2, n=40, nsub=4, n_sources=2000, nsteps=10)
    ref = oracle_run(p)
    got = gpu_run(p, dtype="f32")
    emax, e2 = rel_err(got, ref)
    print(f"f32 storage case {case}: e_max={emax:.3e} e_2={e2:.3e}")
    assert emax <= F32_TOL


def _oracle_fp32_storage(p, nsteps):
    """The oracle's stages in the step's order, each result rounded to FP32:
    what FP32 storage with FP64 arithmetic stores after every stage."""
    def rnd(u):
        u[...] = u.astype(np.float32)
    src, dr = oracle_lists(p)
    u = np.array(p.field(), dtype=np.float64, copy=True)
    rnd(u)
    for _ in range(nsteps):
        if src is not None:
            oracle.source(u, src, p.dt)
            rnd(u)
        for axis in (None, 0, 1, 2):
            if axis is not None:
                oracle.sweep(u, p.h, p.D, p.lam, p.dt, axis)
                rnd(u)
            if dr is not None:
                oracle.dirichlet(u, dr)
                rnd(u)
    return u


def test_fp32_storage_matches_the_oracle_rounded_per_stage():
    # Every stored value is the FP32 rounding of an FP64 result.  GPU and
    # oracle differ in FP64 by a few units of 2^-53 (reciprocals, FMA), which
    # moves a stored value by one FP32 ulp only when it straddles a rounding
    # boundary; every stage is non-expansive (||A^-1|| <= 1/(1+beta), |1/Q| <= 1,
    # Dirichlet exact), so after k stores the gap is at most k ulps:
    # e_max <= k * 2^-23.
    nsteps = 5
    p = small_problem((40, 30, 20), 3, seed=810, nsrc=300, ndir=40, nsteps=nsteps)
    ref = _oracle_fp32_storage(p, nsteps)
    got = gpu_run(p, dtype="f32").astype(np.float64)
    stores = nsteps * 8
    emax, _ = rel_err(got, ref)
    exact = float(np.mean(got == ref))
    print(f"f32 storage vs per-stage-rounded oracle, {nsteps} steps: e_max={emax:.3e}, bit-exact {exact:.6f}")
    assert emax <= stores * 2.0 ** -23
    assert exact >= 0.99


def test_fp32_fast_arithmetic_within_the_fp32_bar():
    # FP32 arithmetic with coefficients rounded to FP32 drifts with r and the
    # step count.  The cells recipe at 40^3 x 4 has r <= 0.53; 20 steps stay
    # within the FP32 form's 1e-5
    p = workloads.config(2, n=40, nsub=4, n_sources=2000, nsteps=20)
    ref = oracle_run(p)
    got = gpu_run(p, dtype="f32fast")
    emax, e2 = rel_err(got, ref)
    print(f"f32fast 40^3x4 (r <= 0.53), 20 steps: e_max={emax:.3e} e_2={e2:.3e}")
    assert emax <= 1e-5


def test_fp32_fast_arithmetic_at_r10_is_held_to_the_looser_bar():
    # At r = 10 the rounded constants and FP32 recurrences accumulate to about
    # 1.4e-5 after 20 steps (the coefficients' relative rounding 6e-8 grows
    # with the conditioning, up to 1 + 2r = 21), above the FP32 bar: this
    # case alone is held to 1e-4, and its error is reported
    p = workloads.config(2, n=40, nsub=2, n_sources=2000, nsteps=20)
    p.D = np.array([1.0e5, 1.0e5])        # r = dt D / h^2 = 10
    ref = oracle_run(p)
    got = gpu_run(p, dtype="f32fast")
    emax, e2 = rel_err(got, ref)
    print(f"f32fast 40^3x2 at r = 10, 20 steps: e_max={emax:.3e} e_2={e2:.3e}")
    assert emax <= 1e-4


def test_repeat_runs_are_bitwise_identical():
    p = small_problem((50, 41, 33), 3, seed=600, nsrc=200, ndir=20, nsteps=4)
    a = gpu_run(p)
    b = gpu_run(p)
    assert np.array_equal(a, b)


def test_duplicate_sources_and_dirichlet_entries():
    p = small_problem((12, 10, 9), 2, seed=700, nsteps=3)
    vox = np.array([5, 77, 5, 300, 77])
    rng = np.random.default_rng(1)
    sec = rng.uniform(0, 10, (5, 2))
    upt = rng.uniform(0, 10, (5, 2))
    sat = np.ones((5, 2))
    p.src = workloads.SourceList(vox, sec, sat, upt)
    dvox = np.array([3, 3, 500, 42])
    val = rng.uniform(0, 5, (4, 2))
    act = np.array([[1, 1], [1, 0], [0, 1], [1, 1]], dtype=np.uint8)
    p.dr = workloads.DirichletList(dvox, val, act)
    ref = oracle_run(p)
    got = gpu_run(p)
    assert rel_err(got, ref)[0] <= F64_TOL
    flat = got.reshape(-1, 2)
    assert flat[3, 0] == val[1, 0] and flat[3, 1] == val[0, 1]


def test_cells_full_workload_100_steps():
    # the 256^3 x 8 workload exactly: 1e5 sources, 64 Dirichlet voxels, 100 steps
    p = workloads.config(2)
    assert p.nsteps == 100
    ref = oracle_run(p)
    got = gpu_run(p)
    emax, e2 = rel_err(got, ref)
    print(f"cells 256^3x8 f64 100 steps: e_max={emax:.3e} e_2={e2:.3e}")
    assert emax <= F64_TOL
    # every active Dirichlet entry holds its value exactly after the last step
    flat = got.reshape(-1, p.S)
    act = p.dr.active.astype(bool)
    assert np.array_equal(flat[p.dr.voxel[act[:, 0]], 0], p.dr.value[act[:, 0], 0])


@pytest.mark.parametrize("dtype,tol", [("f64", F64_TOL), ("f32", F32_TOL)])
def test_autotuned_plans_are_valid_and_keep_parity(dtype, tol):
    import torch
    p = small_problem((150, 70, 90), 3, seed=820, nsrc=200, ndir=20, nsteps=4)
    g = make_grid(p, dtype)
    scratch = torch.empty(p.shape, dtype=g.torch_dtype, device="cuda")
    g.fill_uniform(scratch, 3, 0)
    plans, ms = g.autotune(scratch, reps=2)
    assert all(t > 0 for t in ms)
    for axis, plan in enumerate(plans):
        g.set_plan(axis, *plan)                  # read back, accepted as is
    u = upload(p, g)
    g.step(u, p.nsteps)
    torch.cuda.synchronize()
    got = g.read_field(u)
    g.close()
    emax, _ = rel_err(got, oracle_run(p))
    print(f"autotuned {dtype} plans {plans} ({['%.3f' % t for t in ms]} ms): e_max {emax:.3e}")
    assert emax <= tol
