"""One x-slab's share of the distributed x sweep (Sec. 3.2): the domain split
along x into slabs, the forward elimination run slab after slab with each
slab's last x-plane of eliminated values handed to the next, the backward
substitution run back with each slab's first x-plane of solution values
handed to the previous, the lines taken in blocks.

The slabs are separate arrays, as on separate processes; the hand-offs are
the carry arrays.  Chained over the slabs and blocks, the two kernels must
give the oracle's x sweep of the whole field (FP64 within 1e-12, FP32
storage within 1e-5) and agree with the library's whole-line x sweep within
a few units of rounding (the carries enter at other places in the
recurrence's evaluation order).
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import make_grid, rel_err, small_problem, upload

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f32fast": 1e-5}
EPS = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "f32fast": 2.0 ** -24}


def _slabbed_x_sweep(g, u, xb, lb):
    """The x sweep of field u (not modified) through slabs x in [xb[r], xb[r+1])
    and blocks of lines [lb[b], lb[b+1]): forward slab 0..P-1, backward P-1..0
    per block.  Returns the reassembled field."""
    import torch
    P = len(xb) - 1
    slabs = [u[:, :, xb[r]:xb[r + 1], :].clone(memory_format=torch.contiguous_format) for r in range(P)]
    cdt = torch.float32 if g.dtype == "f32fast" else torch.float64
    for b in range(len(lb) - 1):
        l0, l1 = lb[b], lb[b + 1]
        carry = None
        for r in range(P):
            out = torch.empty(l1 - l0, dtype=cdt, device="cuda")
            g.xslab_forward(slabs[r], xb[r], xb[r + 1], l0, l1, carry, out)
            carry = out
        carry = None
        for r in reversed(range(P)):
            out = torch.empty(l1 - l0, dtype=cdt, device="cuda")
            g.xslab_backward(slabs[r], xb[r], xb[r + 1], l0, l1, carry, out)
            carry = out
    torch.cuda.synchronize()
    return torch.cat(slabs, dim=2)


CASES = [
    ((50, 7, 5), 3, [0, 13, 31, 50], [0, 40, 70, 105]),       # three slabs, three uneven blocks
    ((50, 7, 5), 3, [0, 50], [0, 105]),                       # one slab: no carries
    ((61, 6, 4), 2, [0, 1, 2, 60, 61], [0, 48]),              # slabs of one voxel at both ends
    ((300, 5, 3), 2, [0, 70, 170, 300], [0, 7, 30]),          # M = 16 / 32 tiles, ragged blocks
    ((1500, 3, 2), 2, [0, 600, 1500], [0, 12]),               # slabs up to 900 voxels
]


@pytest.mark.parametrize("shape,S,xb,lb", CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32", "f32fast"])
def test_slabbed_x_sweep_matches_the_oracle_and_the_whole_line_sweep(shape, S, xb, lb, dtype):
    import torch
    p = small_problem(shape, S, seed=900 + shape[0], nsteps=1)
    p.dtype = dtype
    g = make_grid(p, dtype)
    u = upload(p, g)
    got = _slabbed_x_sweep(g, u, xb, lb)
    whole = u.clone()
    g.sweep(whole, 0)
    torch.cuda.synchronize()
    g.close()
    ref = np.array(p.field(), dtype=np.float64, copy=True)
    if dtype != "f64":
        ref = ref.astype(np.float32).astype(np.float64)
    oracle.sweep(ref, p.h, p.D, p.lam, p.dt, 0)
    a = got.double().cpu().numpy()
    e = rel_err(a, ref)[0]
    d = rel_err(a, whole.double().cpu().numpy())[0]
    print(f"{shape}x{S} {dtype} slabs {xb} blocks {lb}: vs oracle {e:.2e}, vs whole-line sweep {d:.2e}")
    assert e <= TOL[dtype], (shape, dtype, e)
    assert d <= 64 * EPS[dtype], (shape, dtype, d)


def test_slab_calls_check_their_arguments():
    import torch
    import paper_2602_05017_amd as bf
    p = small_problem((40, 4, 3), 2, seed=931, nsteps=1)
    g = make_grid(p)
    nl = 4 * 3 * 2
    slab = torch.zeros((3, 4, 10, 2), dtype=torch.float64, device="cuda")
    c = torch.zeros(nl + 1, dtype=torch.float64, device="cuda")
    for call, args in (
            (g.xslab_forward, (slab, 10, 20, 0, nl, None, c)),    # x0 > 0 needs carry_in
            (g.xslab_forward, (slab, 0, 10, 0, nl, c, c)),        # x0 == 0 takes none
            (g.xslab_backward, (slab, 10, 20, 0, nl, None, c)),   # x1 < nx needs carry_in
            (g.xslab_forward, (slab, 10, 20, 0, nl + 1, c, c)),   # l1 beyond the lines
            (g.xslab_forward, (slab, 10, 20, 5, 5, c, c))):       # empty block
        with pytest.raises((bf.BfvmError, ValueError)) as ei:
            call(*args)
        if isinstance(ei.value, bf.BfvmError):
            assert ei.value.code == "EINVAL"
    big = small_problem((2100, 2, 2), 1, seed=932, nsteps=1)
    gb = make_grid(big)
    s2 = torch.zeros((2, 2, 2100, 1), dtype=torch.float64, device="cuda")
    c2 = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(bf.BfvmError) as ei:
        gb.xslab_forward(s2, 0, 2100, 0, 4, None, c2)    # longer than 2048
    assert ei.value.code == "EINVAL"
    gb.close()
    g.close()


def test_chained_schedule_on_slab_streams_matches_the_oracle():
    # the schedule the processes would run (paper_2602_05017_amd.slabs):
    # one stream per slab, an event per (slab, block) hand-off, so slab r
    # works on block b while slab r + 1 works on block b - 1.  Same result,
    # bit for bit, as the shares run one after another on one stream, and
    # the oracle's x sweep of the whole field
    import torch
    from paper_2602_05017_amd.slabs import chained_x_sweep
    p = small_problem((80, 9, 6), 2, seed=941, nsteps=1)
    g = make_grid(p)
    u = upload(p, g)
    xb = [0, 17, 40, 41, 80]
    nl = 9 * 6 * 2
    lb = [0, 5, 33, 34, 70, nl]
    cut = lambda: [u[:, :, xb[r]:xb[r + 1], :].clone(memory_format=torch.contiguous_format) for r in range(4)]
    par = cut()
    streams = [torch.cuda.Stream() for _ in range(4)]
    chained_x_sweep(g, par, xb, lb, streams)
    seq = cut()
    chained_x_sweep(g, seq, xb, lb)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(par, seq))
    ref = np.array(p.field(), dtype=np.float64, copy=True)
    oracle.sweep(ref, p.h, p.D, p.lam, p.dt, 0)
    e = rel_err(torch.cat(par, dim=2).cpu().numpy(), ref)[0]
    assert e <= 1e-12, e
    g.close()
