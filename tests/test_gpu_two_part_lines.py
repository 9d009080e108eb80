"""Plan kind 5: lines longer than one block's K = 64 w / lpw segments of M
cover (K*M < n <= 2*K*M), taken in two parts by one block, the first part
kept in LDS between its passes: y and z lines in the kind-1 layout, x with
every (row, substrate) one line as in kind 3.

Against the FP64 oracle at each storage form's bar, on ragged line lengths
and tiles (heads of one segment up to K segments, tails up to K*M), with
sources and Dirichlet entries; and against the kind-1 (kind-3 on x) plan of
twice the segments, whose carry scans the two-part form repeats step by step (idle
segments pass every carry through unchanged), within 16 units of rounding
of the storage form: the two kernels compute the same expressions, but the
compiler fuses multiplies and adds differently in them (measured: 1-ulp
differences in about 1% of the FP64 elements, none on some shapes).
"""
import numpy as np
import pytest

from gpu_helpers import make_grid, oracle_adjoint, oracle_run, param_grad_bars, rel_err, small_problem, upload

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f32fast": 1e-5}
EPS = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "f32fast": 2.0 ** -24}

# (m, lpw, w, n): K = 64 w / lpw segments per part
CASES = [
    (4, 16, 1, 17),      # K = 4: a head of one segment
    (4, 16, 1, 29),
    (8, 16, 2, 100),     # K = 8
    (8, 32, 4, 128),     # n = 2 K M: head and tail of K full segments
    (16, 16, 4, 300),    # K = 16
    (16, 32, 8, 509),
    (32, 16, 8, 1500),   # K = 32: the long-line plan of the Table 1 cubes
    (32, 16, 8, 2000),
]


def _shape(axis, n):
    other = (7, 5) if n <= 512 else (3, 2)
    return {0: (n, other[0], other[1]), 1: (other[0], n, other[1]), 2: (other[0], other[1], n)}[axis]


def _run(p, dtype, axis, plan, nsteps):
    import torch
    g = make_grid(p, dtype, plans={axis: plan})
    assert tuple(g.get_plan(axis)) == plan
    u = upload(p, g)
    g.step(u, nsteps)
    torch.cuda.synchronize()
    g.close()
    return u


@pytest.mark.parametrize("m,lpw,w,n", CASES)
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("dtype", ["f64", "f32", "f32fast"])
def test_two_part_lines_match_oracle_and_the_one_part_plan(m, lpw, w, n, axis, dtype):
    import torch
    S = 3 if n <= 512 else 2
    shape = _shape(axis, n)
    p = small_problem(shape, S, seed=700 + n + axis, nsrc=60, ndir=12, nsteps=2)
    p.dtype = dtype
    two = _run(p, dtype, axis, (5, m, w, lpw), 2)
    one = _run(p, dtype, axis, (3 if axis == 0 else 1, m, 2 * w, lpw), 2)
    a = two.double().cpu().numpy()
    d = rel_err(a, one.double().cpu().numpy())[0]
    assert d <= 16 * EPS[dtype], (m, lpw, w, n, axis, dtype, d)
    emax, _ = rel_err(a, oracle_run(p, 2))
    assert emax <= TOL[dtype], (m, lpw, w, n, axis, dtype, emax)


def test_two_part_plans_are_checked():
    import paper_2602_05017_amd as bf
    p = small_problem((40, 100, 30), 2, seed=731, nsteps=1)
    g = make_grid(p)
    for axis, plan in ((0, (5, 8, 2, 16)),      # K*M = 64 >= 40 on x: one part covers the line
                       (1, (5, 8, 4, 16)),      # K*M = 128 >= 100: one part covers the line
                       (1, (5, 4, 2, 16)),      # 2*K*M = 64 < 100
                       (1, (5, 8, 16, 16)),     # more than 512 threads
                       (1, (5, 8, 2, 8))):      # lpw
        with pytest.raises(bf.BfvmError) as ei:
            g.set_plan(axis, *plan)
        assert ei.value.code == "EINVAL", (axis, plan)
    g.set_plan(1, 5, 8, 2, 16)
    assert tuple(g.get_plan(1)) == (5, 8, 2, 16)
    g.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_reverse_step_with_two_part_plans(dtype):
    # the transposed sweeps of a kind-5 axis run as a kind-1 plan (as few
    # segments as cover the line): the reverse step still matches the
    # oracle's adjoint
    import torch
    p = small_problem((9, 100, 70), 2, seed=741, nsrc=40, ndir=10, nsteps=1)
    p.dtype = dtype
    g = make_grid(p, dtype, plans={1: (5, 8, 2, 16), 2: (5, 8, 2, 16)})
    u = upload(p, g)
    rng = np.random.default_rng(41)
    gin = (rng.random(p.shape) - 0.5).astype(np.float64 if dtype == "f64" else np.float32)
    gr = torch.from_numpy(gin.copy()).to("cuda")
    gD, gL = g.step_adjoint(u, gr)
    torch.cuda.synchronize()
    state = g.read_field(u)
    rg, rD, rL = oracle_adjoint(p, state, gin)
    barD, barL = param_grad_bars(p, state, gin)
    g.close()
    assert rel_err(gr.double().cpu().numpy(), rg)[0] <= TOL[dtype]
    assert np.all(np.abs(gD - rD) <= barD) and np.all(np.abs(gL - rL) <= barL)


@pytest.mark.parametrize("dtype", ["f64", "f32", "f32fast"])
def test_two_part_plan_runs_its_own_kernel(dtype):
    # the forward sweep of a kind-5 axis launches the two-part kernel (not
    # the kind-1 plan it falls back to), its transposed sweep the kind-1
    # kernel (the reverse step's forward recomputation runs the two-part
    # kernel again); kernel names as the profiler records them.  Rows of 21
    # values are not whole 16-byte chunks, so the reverse step's y sweep is
    # not the LDS-tile form (k_adj_tr_tile)
    import torch
    from torch.profiler import ProfilerActivity, profile
    p = small_problem((7, 100, 5), 3, seed=751, nsrc=10, nsteps=1)
    p.dtype = dtype
    g = make_grid(p, dtype, plans={1: (5, 8, 2, 16)})
    u = upload(p, g)
    gr = torch.zeros_like(u)
    torch.cuda.synchronize()
    with profile(activities=[ProfilerActivity.CUDA]) as prof:
        g.sweep(u, 1)
        torch.cuda.synchronize()
    fwd = {e.name for e in prof.events()}
    with profile(activities=[ProfilerActivity.CUDA]) as prof:
        g.step_adjoint(u, gr)
        torch.cuda.synchronize()
    rev = {e.name for e in prof.events()}
    g.close()
    def strided_args(n):   # template arguments of a kind-1 kernel name
        return [a.strip() for a in n.split("k_sweep_seg_strided<", 1)[1].split(">", 1)[0].split(",")]

    assert any("k_sweep_seg_halves" in n for n in fwd), sorted(fwd)
    assert not any("k_sweep_seg_strided" in n and strided_args(n)[6] == "1" for n in fwd), sorted(fwd)
    # k_sweep_seg_strided<T, C, M, TR, COEF, XROWS, AX, RED>: the y axis transposed
    assert any("k_sweep_seg_strided" in n and strided_args(n)[3] == "true" and strided_args(n)[6] == "1"
               for n in rev), sorted(rev)
