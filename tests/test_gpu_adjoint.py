"""GPU adjoint form: transposed sweeps in reverse axis order behind
torch.autograd, checked against the oracle's adjoint, finite differences and
closed-form eigenmode gradients; checkpointing must not change the result.

Bars.  One LOD step's gradient (FP64) within 1e-12 of the oracle's.  Over N
steps the gradient passes through 3N forward and 3N transposed sweeps whose
rounding (reciprocal multiply on the GPU, division in the oracle) is
amplified by at most the factors' conditioning, about 1 + 2r (21 at r = 10),
per sweep: 6N * 21 * 2^-53 ~ 7e-13 at N = 50, so the multi-step bar is
1e-11.  Central differences (h = 1e-6 relative, FP64 forward) within 1e-4.
FP32 storage: dL/du0 and dL/dlambda within 1e-5 of the FP64 oracle; dL/dD
sums y^T (L_N x), a difference of neighbouring stored values, which
amplifies the 2^-24 storage rounding by the smoothness of the field, so it
is held to the finite-difference bar 1e-4.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import make_grid, oracle_lists, rel_err, small_problem, upload

pytestmark = pytest.mark.gpu


def _gpu_grad(p, target, nsteps, dtype="f64", K=10, D=None, lam=None):
    import torch
    import paper_2602_05017_amd as bf
    from paper_2602_05017_amd.autograd import simulate
    g = make_grid(p, dtype)
    u0 = upload(p, g).requires_grad_(True)
    Dt = torch.tensor(p.D if D is None else D, dtype=torch.float64, requires_grad=True)
    Lt = torch.tensor(p.lam if lam is None else lam, dtype=torch.float64, requires_grad=True)
    uN = simulate(g, u0, Dt, Lt, p.dt, nsteps, checkpoint_every=K)
    tt = torch.from_numpy(target).to(device="cuda", dtype=uN.dtype)
    loss = ((uN.double() - tt.double()) ** 2).sum()
    loss.backward()
    out = (float(loss), u0.grad.double().cpu().numpy(), Dt.grad.numpy().copy(), Lt.grad.numpy().copy())
    g.close()
    return out


def _loss_gpu(p, target, nsteps, D, lam):
    import torch
    g = make_grid(p, "f64")
    g.set_params(D, lam, p.dt)
    u = upload(p, g)
    g.step(u, nsteps)
    torch.cuda.synchronize()
    uN = g.read_field(u)
    g.close()
    return float(np.sum((uN - target) ** 2))


# Without sources and Dirichlet entries the recomputed x sweep reads the
# state itself, out of place; the x kernel follows the default plan: row
# lines (3 substrates), LDS row tiles (2 substrates, 96 voxels) and pipelined
# row tiles (2 substrates, 400 voxels).  Axes of one voxel (no neighbours:
# L_N x = 0 there) and 300 substrates (more than the 256 threads of the line
# sums' blocks: each thread then adds whole substrates) close the list.
@pytest.mark.parametrize("shape,S,nsrc,ndir", [((21, 17, 13), 3, 80, 12), ((21, 17, 13), 3, 80, 0),
                                               ((21, 17, 13), 3, 0, 12), ((21, 17, 13), 3, 0, 0),
                                               ((96, 9, 7), 2, 0, 0), ((400, 5, 4), 2, 0, 0),
                                               ((1, 5, 7), 2, 3, 2), ((9, 1, 1), 3, 0, 0),
                                               ((6, 5, 4), 300, 20, 3)])
def test_adjoint_step_matches_oracle(shape, S, nsrc, ndir):
    import torch
    p = small_problem(shape, S, seed=800, nsrc=nsrc, ndir=ndir)
    rng = np.random.default_rng(3)
    gin = rng.random(p.shape) - 0.5
    g = make_grid(p)
    u = upload(p, g)
    gg = torch.from_numpy(gin.copy()).cuda()
    gD, gL = g.step_adjoint(u, gg)
    torch.cuda.synchronize()
    got = gg.cpu().numpy()
    assert np.array_equal(g.read_field(u), p.u0)      # the state is only read
    g.close()
    src, dr = oracle_lists(p)
    ref = gin.copy()
    rD = np.zeros(p.S)
    rL = np.zeros(p.S)
    oracle.adjoint_step(np.array(p.u0), ref, rD, rL, p.h, p.D, p.lam, p.dt, src, dr)
    assert rel_err(got, ref)[0] <= 1e-12
    assert np.max(np.abs(gD - rD) / np.abs(rD)) <= 1e-12
    assert np.max(np.abs(gL - rL) / np.abs(rL)) <= 1e-12


def test_adjoint_step_fp32_arithmetic_matches_oracle():
    # FP32 storage and arithmetic, constants rounded to FP32: the oracle's
    # FP64 adjoint of the FP32-rounded state and gradient, within the FP32
    # form's 1e-5 (dL/dD, a sum of neighbour differences, within 1e-4);
    # measured 2.4e-7, 5.4e-6 (dL/dD) and 4.9e-7 (dL/dlambda)
    import torch
    p = small_problem((21, 17, 13), 3, seed=801, nsrc=40, ndir=6)
    rng = np.random.default_rng(4)
    gin = (rng.random(p.shape) - 0.5).astype(np.float32)
    g = make_grid(p, "f32fast")
    u = upload(p, g)
    gg = torch.from_numpy(gin.copy()).cuda()
    gD, gL = g.step_adjoint(u, gg)
    torch.cuda.synchronize()
    got = gg.double().cpu().numpy()
    g.close()
    src, dr = oracle_lists(p)
    ref = gin.astype(np.float64)
    rD = np.zeros(p.S)
    rL = np.zeros(p.S)
    oracle.adjoint_step(p.u0.astype(np.float32).astype(np.float64), ref, rD, rL, p.h, p.D, p.lam, p.dt, src, dr)
    e = rel_err(got, ref)[0]
    eD = np.max(np.abs(gD - rD) / np.abs(rD))
    eL = np.max(np.abs(gL - rL) / np.abs(rL))
    print(f"f32fast adjoint step: grad e_max {e:.2e}, dD {eD:.2e}, dlambda {eL:.2e}")
    assert e <= 1e-5 and eL <= 1e-5 and eD <= 1e-4


@pytest.mark.parametrize("K", [1, 3, 10])
def test_autograd_matches_oracle_gradient(K):
    p = small_problem((24, 19, 22), 2, seed=810, nsrc=60, ndir=10, nsteps=7)
    target = np.random.default_rng(4).random(p.shape)
    L, g0, gD, gL = _gpu_grad(p, target, 7, K=K)
    src, dr = oracle_lists(p)
    rL_, ruN, rg0, rgD, rgL = oracle.run_with_gradient(p.u0, target, p.h, p.D, p.lam, p.dt, 7, src, dr)
    assert abs(L - rL_) <= 1e-12 * rL_
    assert rel_err(g0, rg0)[0] <= 1e-11
    assert np.max(np.abs(gD - rgD) / np.abs(rgD)) <= 1e-11
    assert np.max(np.abs(gL - rgL) / np.abs(rgL)) <= 1e-11


def test_checkpointing_is_bitwise_neutral():
    p = small_problem((20, 18, 16), 2, seed=820, nsrc=40, ndir=6, nsteps=9)
    target = np.random.default_rng(5).random(p.shape)
    a = _gpu_grad(p, target, 9, K=1)
    b = _gpu_grad(p, target, 9, K=4)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


def test_central_differences_on_gpu():
    p = small_problem((18, 15, 20), 2, seed=830, nsrc=50, ndir=8, nsteps=5)
    target = np.random.default_rng(6).random(p.shape)
    L, g0, gD, gL = _gpu_grad(p, target, 5)
    for s in range(p.S):
        for which, grad in (("D", gD), ("L", gL)):
            base = p.D if which == "D" else p.lam
            eps = 1e-6 * base[s]
            plus, minus = base.copy(), base.copy()
            plus[s] += eps
            minus[s] -= eps
            if which == "D":
                fd = (_loss_gpu(p, target, 5, plus, p.lam) - _loss_gpu(p, target, 5, minus, p.lam)) / (2 * eps)
            else:
                fd = (_loss_gpu(p, target, 5, p.D, plus) - _loss_gpu(p, target, 5, p.D, minus)) / (2 * eps)
            assert abs(grad[s] - fd) <= 1e-4 * abs(fd), (which, s, grad[s], fd)


def test_eigenmode_closed_form_on_gpu():
    nx, ny, nz = 20, 14, 24
    ks = (3, 2, 5)
    p = small_problem((nx, ny, nz), 1, seed=840, h=(10.0, 14.0, 9.0), dt=0.03, nsteps=5)
    p.D = np.array([3e2])
    p.lam = np.array([0.4])
    cx = np.cos(np.pi * ks[0] * (np.arange(nx) + 0.5) / nx)
    cy = np.cos(np.pi * ks[1] * (np.arange(ny) + 0.5) / ny)
    cz = np.cos(np.pi * ks[2] * (np.arange(nz) + 0.5) / nz)
    p.u0 = np.ascontiguousarray((cz[:, None, None] * cy[None, :, None] * cx[None, None, :])[..., None])
    N = 5
    L, g0, gD, gL = _gpu_grad(p, np.zeros(p.shape), N)
    beta = p.dt * p.lam[0] / 3.0
    mus, s2s = [], []
    for n, k, a in ((nx, ks[0], 0), (ny, ks[1], 1), (nz, ks[2], 2)):
        s2 = 4.0 * np.sin(np.pi * k / (2.0 * n)) ** 2
        mus.append(1.0 + beta + p.dt * p.D[0] / p.h[a] ** 2 * s2)
        s2s.append(s2)
    Lref = np.sum(p.u0 ** 2) * np.prod([m ** (-2 * N) for m in mus])
    gD_ref = sum(-2 * N * Lref * s2s[a] / mus[a] * p.dt / p.h[a] ** 2 for a in range(3))
    gL_ref = -2 * N * Lref * sum(1.0 / m for m in mus) * p.dt / 3.0
    assert abs(L - Lref) <= 1e-12 * Lref
    assert abs(gD[0] - gD_ref) <= 1e-12 * abs(gD_ref)
    assert abs(gL[0] - gL_ref) <= 1e-12 * abs(gL_ref)


_C4_REF = {}


def _c4_reference(p, target):
    if "ref" not in _C4_REF:
        src, dr = oracle_lists(p)
        _C4_REF["ref"] = oracle.run_with_gradient(p.u0, target, p.h, p.D, p.lam, p.dt, p.nsteps, src, dr,
                                                  checkpoint_every=10)
    return _C4_REF["ref"]


@pytest.mark.parametrize("dtype,tol,tolD", [("f64", 1e-11, 1e-11), ("f32", 1e-5, 1e-4)])
def test_differentiation_workload_128cube(dtype, tol, tolD):
    # 128^3 x 2, 50 steps, checkpoints every 10, loss = sum (u_N - target)^2;
    # the variant with 1e3 source voxels and 16 Dirichlet voxels covers the
    # transposed source and Dirichlet stages
    p = workloads.config(4, n_sources=1000)
    p.dr = workloads.dirichlet_variant(p, 16)
    target = workloads.target_field(p)
    L, g0, gD, gL = _gpu_grad(p, target, p.nsteps, dtype=dtype, K=10)
    rL_, ruN, rg0, rgD, rgL = _c4_reference(p, target)
    e0 = rel_err(g0, rg0)
    eD = np.max(np.abs(gD - rgD) / np.abs(rgD))
    eL = np.max(np.abs(gL - rgL) / np.abs(rgL))
    print(f"128^3x2 {dtype} 50 steps: loss rel {abs(L - rL_) / rL_:.2e}, grad u0 e_max {e0[0]:.2e} "
          f"e_2 {e0[1]:.2e}, grad D {eD:.2e}, grad lambda {eL:.2e}")
    assert abs(L - rL_) <= tol * rL_
    assert e0[0] <= tol and eL <= tol and eD <= tolD


def test_backward_uses_its_own_forward_params_after_another_forward_on_the_grid():
    # one grid, two forward passes with different D before the first pass's
    # backward: the backward must re-install the first pass's D, lambda and
    # dt (the second pass left the grid with its own), so its gradient equals
    # the oracle's for the first pass's parameters
    import torch
    from paper_2602_05017_amd.autograd import simulate
    p = small_problem((19, 16, 14), 2, seed=850, nsrc=40, ndir=6, nsteps=4)
    target = np.random.default_rng(8).random(p.shape)
    g = make_grid(p, "f64")
    tt = torch.from_numpy(target).cuda()
    u0 = upload(p, g).requires_grad_(True)
    D1 = torch.tensor(p.D, dtype=torch.float64, requires_grad=True)
    L1 = torch.tensor(p.lam, dtype=torch.float64, requires_grad=True)
    loss1 = ((simulate(g, u0, D1, L1, p.dt, 4, checkpoint_every=2) - tt) ** 2).sum()
    D2 = torch.tensor(p.D * 3.0, dtype=torch.float64, requires_grad=True)
    L2 = torch.tensor(p.lam * 0.5, dtype=torch.float64, requires_grad=True)
    u0b = upload(p, g).requires_grad_(True)
    loss2 = ((simulate(g, u0b, D2, L2, p.dt * 2.0, 4, checkpoint_every=2) - tt) ** 2).sum()
    loss1.backward()
    src, dr = oracle_lists(p)
    rL_, _, rg0, rgD, rgL = oracle.run_with_gradient(p.u0, target, p.h, p.D, p.lam, p.dt, 4, src, dr)
    assert abs(float(loss1) - rL_) <= 1e-12 * rL_
    assert rel_err(u0.grad.cpu().numpy(), rg0)[0] <= 1e-11
    assert np.max(np.abs(D1.grad.numpy() - rgD) / np.abs(rgD)) <= 1e-11
    assert np.max(np.abs(L1.grad.numpy() - rgL) / np.abs(rgL)) <= 1e-11
    # and the second pass's backward, run after the first's, gets its own
    loss2.backward()
    rL2, _, rg02, rgD2, rgL2 = oracle.run_with_gradient(p.u0, target, p.h, p.D * 3.0, p.lam * 0.5, p.dt * 2.0, 4,
                                                        src, dr)
    assert abs(float(loss2) - rL2) <= 1e-12 * rL2
    assert rel_err(u0b.grad.cpu().numpy(), rg02)[0] <= 1e-11
    assert np.max(np.abs(D2.grad.numpy() - rgD2) / np.abs(rgD2)) <= 1e-11
    assert np.max(np.abs(L2.grad.numpy() - rgL2) / np.abs(rgL2)) <= 1e-11
    g.close()


@pytest.mark.parametrize("nz", [64, 500, 512, 513, 600])
@pytest.mark.parametrize("dtype", ["f64", "f32", "f32fast"])
@pytest.mark.parametrize("nx", [5, 8])
def test_reverse_step_z_pass_fused_and_two_kernel(nx, nz, dtype):
    # z lines of up to 512 voxels run the z recomputation and the z
    # transposed sweep as one kernel (k_adj_z_fused: the z output formed and
    # consumed in registers); longer lines run the two kernels with the
    # workspace between them.  The fused kernel fetches the gradient tile
    # straight into LDS (last template argument true) where the z-planes'
    # rows are 16-byte aligned and the lines fill whole 16-byte chunks: nx =
    # 8 (48 values per plane) in every storage form, nx = 5 (30) in FP64
    # only.  Every form against the oracle's adjoint of the state and
    # gradient the GPU holds: the gradient at the storage form's bar, dL/dD
    # and dL/dlambda within their normwise bars; the kernel names the
    # profiler records show which form ran
    import torch
    from torch.profiler import ProfilerActivity, profile
    from gpu_helpers import oracle_adjoint, param_grad_bars
    p = small_problem((nx, 3, nz), 2, seed=810 + nz + nx, nsrc=30, ndir=8)
    p.dtype = dtype
    rng = np.random.default_rng(nz)
    gin = (rng.random(p.shape) - 0.5).astype(np.float64 if dtype == "f64" else np.float32)
    g = make_grid(p, dtype)
    u = upload(p, g)
    gg = torch.from_numpy(gin.copy()).cuda()
    torch.cuda.synchronize()
    with profile(activities=[ProfilerActivity.CUDA]) as prof:
        gD, gL = g.step_adjoint(u, gg)
        torch.cuda.synchronize()
    names = {e.name for e in prof.events()}
    state = g.read_field(u)
    g.close()
    fused = [n for n in names if "k_adj_z_fused" in n]
    assert bool(fused) == (nz <= 512), sorted(names)
    inner = nx * 3 * 2
    dma = nz <= 512 and inner % (2 if dtype == "f64" else 4) == 0
    assert any("1, true>" in n for n in fused) == dma and any("1, false>" in n for n in fused) == (
        nz <= 512 and not dma), fused
    rg, rD, rL = oracle_adjoint(p, state, gin)
    barD, barL = param_grad_bars(p, state, gin)
    e = rel_err(gg.double().cpu().numpy(), rg)[0]
    assert e <= {"f64": 1e-12, "f32": 1e-5, "f32fast": 1e-5}[dtype], (nz, dtype, e)
    assert np.all(np.abs(gD - rD) <= barD) and np.all(np.abs(gL - rL) <= barL), (nz, dtype)


@pytest.mark.parametrize("ny", [1, 17, 100, 512, 513])
@pytest.mark.parametrize("dtype", ["f64", "f32", "f32fast"])
@pytest.mark.parametrize("nx", [5, 8])
def test_reverse_step_y_sweep_with_the_x_tile_in_lds(nx, ny, dtype):
    # the transposed y sweep of the reverse step forms its parameter sums
    # from the recomputed x, which k_adj_tr_tile fetches into LDS while it
    # solves (y lines of up to 512 voxels, rows of whole 16-byte chunks: nx =
    # 8 gives 16 values per row in every storage form, nx = 5 gives 10, FP64
    # only); elsewhere the strided kernel reads x after its solve.  Both
    # against the oracle's adjoint: the gradient at the storage form's bar,
    # dL/dD and dL/dlambda within their normwise bars
    import torch
    from torch.profiler import ProfilerActivity, profile
    from gpu_helpers import oracle_adjoint, param_grad_bars
    p = small_problem((nx, ny, 6), 2, seed=830 + ny + nx, nsrc=30, ndir=8)
    p.dtype = dtype
    rng = np.random.default_rng(ny + 7 * nx)
    gin = (rng.random(p.shape) - 0.5).astype(np.float64 if dtype == "f64" else np.float32)
    g = make_grid(p, dtype)
    u = upload(p, g)
    gg = torch.from_numpy(gin.copy()).cuda()
    torch.cuda.synchronize()
    with profile(activities=[ProfilerActivity.CUDA]) as prof:
        gD, gL = g.step_adjoint(u, gg)
        torch.cuda.synchronize()
    names = {e.name for e in prof.events()}
    state = g.read_field(u)
    g.close()
    tile = ny <= 512 and (nx * 2) % (2 if dtype == "f64" else 4) == 0
    # k_adj_tr_tile<T, C, M, COEF, XROWS>: the y lines' form ends in "false>"
    assert any("k_adj_tr_tile" in n and n.split("(")[0].rstrip().endswith("false>") for n in names) == tile, \
        sorted(names)
    rg, rD, rL = oracle_adjoint(p, state, gin)
    barD, barL = param_grad_bars(p, state, gin)
    e = rel_err(gg.double().cpu().numpy(), rg)[0]
    assert e <= {"f64": 1e-12, "f32": 1e-5, "f32fast": 1e-5}[dtype], (nx, ny, dtype, e)
    assert np.all(np.abs(gD - rD) <= barD) and np.all(np.abs(gL - rL) <= barL), (nx, ny, dtype)


@pytest.mark.parametrize("nx", [17, 100, 300, 512, 513])
@pytest.mark.parametrize("dtype", ["f64", "f32", "f32fast"])
@pytest.mark.parametrize("S", [2, 4])
def test_reverse_step_x_sweep_with_the_x_tile_in_lds(S, nx, dtype):
    # the transposed x sweep through x rows (plan kind 3) forms its sums with
    # the recomputed x fetched into LDS (k_adj_tr_tile) where a 16-byte chunk
    # holds whole substrates of one row: S = 4 in every storage form, S = 2 in
    # FP64; other x plans (row tiles) keep their own kernels.  Against the
    # oracle's adjoint at the usual bars
    import torch
    from torch.profiler import ProfilerActivity, profile
    from gpu_helpers import oracle_adjoint, param_grad_bars
    p = small_problem((nx, 3, 4), S, seed=850 + nx + S, nsrc=30, ndir=8)
    p.dtype = dtype
    rng = np.random.default_rng(nx + 5 * S)
    gin = (rng.random(p.shape) - 0.5).astype(np.float64 if dtype == "f64" else np.float32)
    g = make_grid(p, dtype)
    kind = g.get_plan(0)[0]
    u = upload(p, g)
    gg = torch.from_numpy(gin.copy()).cuda()
    torch.cuda.synchronize()
    with profile(activities=[ProfilerActivity.CUDA]) as prof:
        gD, gL = g.step_adjoint(u, gg)
        torch.cuda.synchronize()
    names = {e.name for e in prof.events()}
    state = g.read_field(u)
    g.close()
    per_chunk = 2 if dtype == "f64" else 4
    tile = kind == 3 and nx <= 512 and S % per_chunk == 0
    assert any("k_adj_tr_tile" in n and n.split("(")[0].rstrip().endswith("true>") for n in names) == tile, \
        (kind, sorted(names))
    rg, rD, rL = oracle_adjoint(p, state, gin)
    barD, barL = param_grad_bars(p, state, gin)
    e = rel_err(gg.double().cpu().numpy(), rg)[0]
    assert e <= {"f64": 1e-12, "f32": 1e-5, "f32fast": 1e-5}[dtype], (S, nx, dtype, e)
    assert np.all(np.abs(gD - rD) <= barD) and np.all(np.abs(gL - rL) <= barL), (S, nx, dtype)
