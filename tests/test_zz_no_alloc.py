"""The allocation-free reverse step (bfvm_step_adjoint_noalloc), called
through the C ABI, against the allocating one (bfvm_step_adjoint) on the
same state and gradient: calls in a row on one GPU share the scratch array,
each later call with a smaller grid, and a grid beyond the array's limit is
refused before any device work."""
import ctypes

import numpy as np
import pytest

import workloads
from gpu_helpers import make_grid, oracle_adjoint, rel_err, small_problem, upload

pytestmark = pytest.mark.gpu


def _both(p, dtype, seed):
    import torch
    import paper_2602_05017_amd as bf
    L = bf.lib()
    g = make_grid(p, dtype)
    u = upload(p, g)
    rng = np.random.default_rng(seed)
    gin = torch.from_numpy(rng.random(p.shape) - 0.5).to(device="cuda", dtype=g.torch_dtype)
    ga, gb = gin.clone(), gin.clone()
    Da, La, Db, Lb = (np.zeros(p.S) for _ in range(4))
    torch.cuda.synchronize()
    h = g.handle
    p_u = ctypes.c_void_p(u.data_ptr())
    assert L.bfvm_step_adjoint(h, p_u, ctypes.c_void_p(ga.data_ptr()), bf._ptr(Da), bf._ptr(La)) == 0
    assert L.bfvm_step_adjoint_noalloc(h, p_u, ctypes.c_void_p(gb.data_ptr()), bf._ptr(Db), bf._ptr(Lb)) == 0, \
        bf.last_error()
    torch.cuda.synchronize()
    state = g.read_field(u)
    g.close()
    return state, gin.double().cpu().numpy(), ga.double().cpu().numpy(), gb.double().cpu().numpy(), Da, La, Db, Lb


def test_noalloc_reverse_step_matches_the_allocating_one():
    # 1: the largest grid the array holds (128^3 x 2 FP64: 96 MiB of sweep
    # outputs), no sources or Dirichlet entries; 2: smaller, with sources and
    # Dirichlet entries (the copying path); 3: smaller still, FP32 storage
    p1 = workloads.config(4, nsteps=1)
    p2 = small_problem((61, 47, 39), 3, seed=870, nsrc=200, ndir=25, nsteps=1)
    p3 = small_problem((33, 21, 18), 2, seed=871, nsrc=40, ndir=5, nsteps=1)
    for k, (p, dtype) in enumerate(((p1, "f64"), (p2, "f64"), (p3, "f32"))):
        state, gin, ga, gb, Da, La, Db, Lb = _both(p, dtype, 30 + k)
        tol = 1e-12 if dtype == "f64" else 1e-5
        exact = np.array_equal(ga, gb) and np.array_equal(Da, Db) and np.array_equal(La, Lb)
        print(f"call {k + 1}: {p.nx}x{p.ny}x{p.nz}x{p.S} {dtype}: bit-identical {exact}, "
              f"grad e_max {rel_err(gb, ga)[0]:.2e}")
        assert rel_err(gb, ga)[0] <= tol
        assert np.all(np.abs(Db - Da) <= tol * np.abs(Da)) and np.all(np.abs(Lb - La) <= tol * np.abs(La))
        if k == 1:
            # and the oracle's reverse step agrees with both (FP64)
            rg, rD, rL = oracle_adjoint(p, state, gin)
            assert rel_err(gb, rg)[0] <= 1e-12


def test_noalloc_refuses_a_grid_beyond_its_array():
    import torch
    import paper_2602_05017_amd as bf
    L = bf.lib()
    g = bf.Grid(256, 256, 128, 2)            # 3 x 128 MiB of sweep outputs
    g.set_params(np.array([1e3, 1e4]), np.array([0.1, 0.2]), 0.01)
    u = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
    gr = torch.ones(g.shape, dtype=torch.float64, device="cuda")
    D = np.zeros(2)
    lam = np.zeros(2)
    st = L.bfvm_step_adjoint_noalloc(g.handle, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(gr.data_ptr()),
                                     bf._ptr(D), bf._ptr(lam))
    assert st == -1 and "too large" in bf.last_error()
    torch.cuda.synchronize()
    assert bool(torch.all(gr == 1.0)) and not D.any() and not lam.any()
    g.close()
