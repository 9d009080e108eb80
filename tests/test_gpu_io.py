"""Field files: bfvm_save_npy / bfvm_load_npy against NumPy's own .npy reader
and writer.  Both directions move bytes only, so the bar is bit-exact."""
import numpy as np
import pytest

from gpu_helpers import make_grid, small_problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape,S", [((37, 29, 41), 3),        # one 32 MB chunk, partly filled
                                     ((256, 256, 100), 4)])    # 7 chunks (FP64) with a ragged tail
def test_save_then_numpy_load_is_bit_exact(tmp_path, dtype, shape, S):
    import torch
    p = small_problem(shape, S, seed=3, nsteps=1)
    g = make_grid(p, dtype)
    u = torch.empty(p.shape, dtype=g.torch_dtype, device="cuda")
    g.fill_uniform(u, 77, 2)
    g.step(u, 1)                               # enqueued work the save must follow
    path = tmp_path / "field.npy"
    g.save_npy(u, path)
    got = np.load(path)
    ref = g.read_field(u)
    g.close()
    assert got.shape == p.shape and got.dtype == ref.dtype
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_numpy_save_then_load_is_bit_exact(tmp_path, dtype):
    import torch
    p = small_problem((200, 130, 90), 3, seed=4, nsteps=1)   # 56 MB in FP64: two chunks
    g = make_grid(p, dtype)
    rng = np.random.default_rng(12)
    host = rng.standard_normal(p.shape).astype(np.float64 if dtype == "f64" else np.float32)
    path = tmp_path / "in.npy"
    np.save(path, host)
    u = torch.zeros(p.shape, dtype=g.torch_dtype, device="cuda")
    g.load_npy(u, path)
    got = g.read_field(u)
    g.close()
    assert np.array_equal(got, host)


def test_load_accepts_format_2_and_three_dimensional_single_substrate_files(tmp_path):
    import torch
    p = small_problem((20, 30, 40), 1, seed=5, nsteps=1)
    g = make_grid(p, "f64")
    host = np.random.default_rng(1).random((p.nz, p.ny, p.nx))
    path = tmp_path / "v2.npy"
    with open(path, "wb") as f:
        np.lib.format.write_array(f, host, version=(2, 0))
    u = torch.zeros(p.shape, dtype=torch.float64, device="cuda")
    g.load_npy(u, path)
    assert np.array_equal(g.read_field(u)[..., 0], host)
    g.close()


def test_io_errors_raise(tmp_path):
    import torch
    import paper_2602_05017_amd as bf
    p = small_problem((8, 8, 8), 2, seed=6, nsteps=1)
    g = make_grid(p, "f64")
    u = torch.zeros(p.shape, dtype=torch.float64, device="cuda")
    np.save(tmp_path / "wrong.npy", np.zeros((8, 8, 8, 2), np.float32))
    with pytest.raises(bf.BfvmError):
        g.load_npy(u, tmp_path / "wrong.npy")
    with pytest.raises(bf.BfvmError):
        g.save_npy(u, tmp_path / "missing_dir" / "x.npy")
    # the grid keeps working after the failed calls
    g.save_npy(u, tmp_path / "ok.npy")
    assert np.array_equal(np.load(tmp_path / "ok.npy"), g.read_field(u))
    g.close()
