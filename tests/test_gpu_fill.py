"""Device-side field set-up against the seeded input generator of the test
harness (workloads/), which implements the same published counter-based
generator independently (numpy / C).

Bars.  Uniform values in [0, 1) are integer work plus an exact scaling:
bit-exact, in FP64 and after rounding to FP32.  With other bounds the device
may fuse lo + (hi - lo) * U into one FMA: within one rounding (2^-52
relative).  The Gaussian profile goes through exp, whose last bit may differ
between the device and the host library: within 4 ulp of the value.
"""
import numpy as np
import pytest

import workloads
from gpu_helpers import make_grid, small_problem

pytestmark = pytest.mark.gpu


def _grid(shape, S, dtype):
    p = small_problem(shape, S, seed=1, nsteps=1)
    return p, make_grid(p, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("seed,stream", [(1003, 0), (7, 3), (2**63 + 5, 255)])
def test_uniform_fill_is_bit_exact(dtype, seed, stream):
    import torch
    shape, S = (37, 29, 41), 3
    p, g = _grid(shape, S, dtype)
    u = torch.empty(p.shape, dtype=g.torch_dtype, device="cuda")
    g.fill_uniform(u, seed, stream)
    got = g.read_field(u)
    g.close()
    ref = workloads.uniform(seed, stream, int(np.prod(p.shape))).reshape(p.shape)
    if dtype == "f32":
        ref = ref.astype(np.float32)
    assert np.array_equal(got, ref)
    assert got.min() >= 0.0 and got.max() < 1.0


def test_uniform_fill_bounds():
    import torch
    p, g = _grid((20, 9, 11), 2, "f64")
    u = torch.empty(p.shape, dtype=torch.float64, device="cuda")
    g.fill_uniform(u, 42, 1, lo=-3.0, hi=5.0)
    got = g.read_field(u)
    g.close()
    U = workloads.uniform(42, 1, int(np.prod(p.shape))).reshape(p.shape)
    ref = -3.0 + 8.0 * U
    assert np.max(np.abs(got - ref)) <= 2.0 ** -52 * 8.0
    assert got.min() >= -3.0 and got.max() < 5.0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gaussian_fill_matches_the_64cube_recipe(dtype):
    import torch
    p = workloads.config(1)                    # 64^3 x 1: sigma 8 at the centre, 0.01 * U noise, stream 0
    g = make_grid(p, dtype)
    u = torch.empty(p.shape, dtype=g.torch_dtype, device="cuda")
    g.fill_gaussian(u, (p.nx / 2.0, p.ny / 2.0, p.nz / 2.0), 8.0, peak=1.0, noise=0.01, seed=p.seed, stream=0)
    got = g.read_field(u).astype(np.float64)
    g.close()
    ref = p.u0
    if dtype == "f32":
        ref = ref.astype(np.float32).astype(np.float64)
        tol = 4 * 2.0 ** -24
    else:
        tol = 4 * 2.0 ** -52
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)) <= tol


def test_uniform_fill_full_size_sampled():
    # the 1000^3 x 4 field of the benchmark, written on the device, against
    # the host generator on 8 sampled runs of 10^6 consecutive elements
    import torch
    p = workloads.config(3, with_field=False)
    g = make_grid(p, "f64")
    u = torch.empty(p.shape, dtype=torch.float64, device="cuda")
    g.fill_uniform(u, p.seed, 0)
    torch.cuda.synchronize()
    flat = u.view(-1)
    n = flat.numel()
    rng = np.random.default_rng(3)
    starts = [0, n - 10**6] + list(rng.integers(0, n - 10**6, 6))
    for st in starts:
        got = flat[int(st):int(st) + 10**6].cpu().numpy()
        ref = workloads.uniform(p.seed, 0, 10**6, start=int(st))
        assert np.array_equal(got, ref), st
    g.close()
    del u, flat
    torch.cuda.empty_cache()


def test_fill_rejects_bad_arguments():
    import torch
    import paper_2602_05017_amd as bf
    p, g = _grid((8, 8, 8), 1, "f64")
    u = torch.empty(p.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(bf.BfvmError):
        g.fill_uniform(u, 1, 0, lo=1.0, hi=0.0)
    with pytest.raises(bf.BfvmError):
        g.fill_gaussian(u, (4, 4, 4), 0.0)
    with pytest.raises(bf.BfvmError):
        g.fill_gaussian(u, (4, float("nan"), 4), 1.0)
    g.close()


def test_device_bytes_accounts_for_the_library_allocations():
    import torch
    p = small_problem((40, 30, 20), 3, seed=11, nsrc=100, ndir=10, nsteps=1)
    g = make_grid(p, "f64")
    n_tab = sum(n * p.S * (8 + 4) + p.S * (8 + 4) for n in (p.nx, p.ny, p.nz))   # invd64, invd32, r64, r32
    b0 = g.device_bytes()
    assert b0 >= n_tab
    u = torch.from_numpy(p.u0).cuda()
    gg = torch.zeros_like(u)
    g.step_adjoint(u, gg)                       # allocates the three-field workspace
    b1 = g.device_bytes()
    assert b1 - b0 >= 3 * p.V * p.S * 8
    g.close()
