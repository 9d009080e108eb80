"""Fields allocated by the library with their placement chosen by timing
(bfvm_field_alloc): shape, type and lifetime of the returned tensor, the
per-candidate times, and that a step on such a field matches the oracle."""
import gc

import numpy as np
import pytest

from gpu_helpers import make_grid, oracle_run, rel_err, small_problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype,candidates", [("f64", 3), ("f32", 2), ("f64", 1)])
def test_placed_field_steps_like_any_field(dtype, candidates):
    import torch
    p = small_problem((70, 45, 33), 3, seed=900, nsrc=150, ndir=12, nsteps=4)
    g = make_grid(p, dtype)
    u, ms = g.alloc_field(candidates)
    assert tuple(u.shape) == p.shape and u.dtype == g.torch_dtype and u.is_cuda and u.is_contiguous()
    assert len(ms) == candidates
    timed = [m for m in ms if m >= 0]
    assert (len(timed) == candidates and all(m > 0 for m in timed)) if candidates > 1 else ms == [-1.0]
    assert u.data_ptr() % 256 == 0
    u.copy_(torch.from_numpy(p.u0))
    g.step(u, p.nsteps)
    torch.cuda.synchronize()
    got = g.read_field(u)
    ref = oracle_run(p)
    assert rel_err(got, ref)[0] <= (1e-12 if dtype == "f64" else 1e-5)
    g.close()


def test_placed_field_is_released_with_its_tensor():
    import torch
    import paper_2602_05017_amd as bf
    g = bf.Grid(512, 512, 512, 1)
    g.set_params(np.array([1e3]), np.array([0.1]), 0.01)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    u, _ = g.alloc_field(2)
    view = u[3:5]                              # a view keeps the allocation alive
    del u
    gc.collect()
    assert torch.cuda.mem_get_info()[0] <= free0 - (1 << 30) + (64 << 20)
    view.fill_(1.0)
    torch.cuda.synchronize()
    del view
    gc.collect()
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] >= free0 - (64 << 20)
    g.close()


def test_field_alloc_rejects_bad_arguments():
    import paper_2602_05017_amd as bf
    g = bf.Grid(10, 10, 10, 1)
    with pytest.raises(bf.BfvmError) as ei:
        g.alloc_field(2)                      # before set_params
    assert ei.value.code == "ESTATE"
    g.set_params(np.array([1e3]), np.array([0.1]), 0.01)
    for bad in (0, 17):
        with pytest.raises(bf.BfvmError) as ei:
            g.alloc_field(bad)
        assert ei.value.code == "EINVAL"
    g.close()
