"""Batched multi-domain form: uneven domains (each axis 24..192 voxels, 1..8
substrates, FP32/FP64 storage mixed) stepped together, one graph replay per
step.  Every batched result a test asserts is compared with the FP64 oracle
at its storage type's bar: forward fields, and the reverse step's gradient
field, dL/dD and dL/dlambda against the oracle's adjoint step on the same
state and gradient.  Some tests compare with the domain's own single-grid
GPU run as well (same bar; the batch reads the Thomas constants from its
LDS copy of the tables, which changes only the operation order); graph
replays must equal eager launches exactly.

Adjoint bars against the oracle's FP64 adjoint of the state and gradient the
GPU holds (FP32 values widened): the gradient field within 1e-12 (FP64
storage) or 1e-5 (FP32 storage) normwise per substrate; dL/dD and
dL/dlambda, sums of terms of both signs, within the normwise bars of
gpu_helpers.param_grad_bars (the stored values' rounding carried through
Cauchy-Schwarz, ||L_N||_2 <= 4 and 2-norm-contractive solves).

Modes.  "grouped" (one launch per stage over all domains) is the library's
default.  "persistent" (one launch per step, blocks waiting on per-stage
counters) hung on gfx950 twice and is switched off in the library (its mode
switch returns EOFF); its cases stay here, skipped, until the cause of the
hang is shown.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import (make_grid, one_substrate, oracle_adjoint, oracle_lists, oracle_run, param_grad_bars, rel_err,
                         rel_vec, small_problem, upload)

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f32fast": 1e-4}
ADJ_TOL = {"f64": 1e-12, "f32": 1e-5, "f32fast": 1e-5}    # gradient field


def _check_adjoint_vs_oracle(p, state, gin, got, gD, gL):
    """Batched reverse step of domain p against the oracle's: the gradient
    field normwise per substrate, dL/dD and dL/dlambda against their
    normwise bars; returns (field e_max, |dD error| / bar, |dlambda error| / bar)."""
    rg, rD, rL = oracle_adjoint(p, state, gin)
    barD, barL = param_grad_bars(p, state, gin)
    e = rel_err(got, rg)[0]
    qD = float(np.max(np.abs(np.asarray(gD) - rD) / barD))
    qL = float(np.max(np.abs(np.asarray(gL) - rL) / barL))
    assert e <= ADJ_TOL[p.dtype] and qD <= 1.0 and qL <= 1.0, (p.name, p.dtype, e, qD, qL, rel_vec(gD, rD))
    return e, qD, qL


_PERSISTENT_OFF = ("persistent single-launch mode switched off: its cross-block dependency waits "
                   "did not complete on gfx950 (hung twice); not run until the cause is shown")
MODES = ["grouped", pytest.param("persistent", marks=pytest.mark.skip(reason=_PERSISTENT_OFF))]


def _domains(n, lo=24, hi=64, nsteps=3, seed=1005):
    return workloads.batch_config(n_domains=n, lo=lo, hi=hi, nsteps=nsteps, seed=seed)


def _setup(probs):
    grids = [make_grid(p, p.dtype) for p in probs]
    fields = [upload(p, g) for p, g in zip(probs, grids)]
    return grids, fields


@pytest.mark.parametrize("mode", MODES)
def test_batch_matches_oracle_per_domain_and_graph_equals_eager(mode):
    import torch
    import paper_2602_05017_amd as bf
    probs = _domains(12, nsteps=3)
    # add Dirichlet entries to a few domains so every stage type is exercised
    for k in (1, 4, 7):
        probs[k].dr = workloads.dirichlet_variant(probs[k], 9)
    grids, fields = _setup(probs)
    b = bf.Batch(grids, fields, mode=mode)
    b.step(3, graph=True)
    got = [g.read_field(f) for g, f in zip(grids, fields)]
    for p, out in zip(probs, got):
        u = np.array(p.u0, copy=True)
        src, dr = oracle_lists(p)
        oracle.step(u, p.h, p.D, p.lam, p.dt, src, dr, 3)
        assert rel_err(out, u)[0] <= TOL[p.dtype], p.name
    # replay vs eager: same launches, same results, every replay checked
    grids2, fields2 = _setup(probs)
    b2 = bf.Batch(grids2, fields2, mode=mode)
    b2.step(3, graph=False)
    for rep in range(3):
        b.step(1, graph=True)
        b2.step(1, graph=False)
        torch.cuda.synchronize()
        for f1, f2 in zip(fields, fields2):
            assert torch.equal(f1, f2), rep
        # eager work and a sync between replays
        _ = [f.sum().item() for f in fields[:2]]
    b.close()
    b2.close()


@pytest.mark.parametrize("mode", MODES)
def test_batch_equals_single_grid_steps(mode):
    import torch
    import paper_2602_05017_amd as bf
    probs = _domains(8, lo=24, hi=192, nsteps=4, seed=1006)
    grids, fields = _setup(probs)
    b = bf.Batch(grids, fields, mode=mode)
    info = b.info()
    assert info["items"] > 0 and info["launches"] >= 3
    b.step(4)
    batched = [g.read_field(f) for g, f in zip(grids, fields)]
    b.close()
    for p, out in zip(probs, batched):
        single = make_grid(p, p.dtype)
        u = upload(p, single)
        single.step(u, 4)
        torch.cuda.synchronize()
        ref = single.read_field(u)
        single.close()
        assert rel_err(out, ref)[0] <= TOL[p.dtype], p.name


def test_batch_hand_set_plans_match_oracle():
    # every (M, lines per tile) shape the autotuner may choose, fixed by hand
    # on both storage types, against the oracle: M = 16 tiles are held to
    # 128 VGPRs (a few spilled) and reached otherwise only by tuning
    import paper_2602_05017_amd as bf
    probs = _domains(6, lo=24, hi=120, nsteps=2, seed=1012)
    probs[3].dr = workloads.dirichlet_variant(probs[3], 5)
    grids, fields = _setup(probs)
    b = bf.Batch(grids, fields)
    shapes = [(16, 16), (16, 32), (16, 64), (8, 16), (8, 32), (8, 64), (4, 16), (4, 32), (4, 64)]
    set_any = {"f64": 0, "f32": 0}
    for d, p in enumerate(probs):
        for a, n in enumerate((p.nx, p.ny, p.nz)):
            fits = [(m, l) for m, l in shapes if (512 // l) * m >= n]
            m, l = fits[(3 * d + a) % len(fits)]
            b.set_plan(d, a, m, l)
            assert b.plan(d, a) == (m, l)
            set_any[p.dtype] += m == 16
    assert set_any["f64"] and set_any["f32"]
    b.step(2)
    for p, g, f in zip(probs, grids, fields):
        u = np.array(p.u0, copy=True)
        src, dr = oracle_lists(p)
        oracle.step(u, p.h, p.D, p.lam, p.dt, src, dr, 2)
        assert rel_err(g.read_field(f), u)[0] <= TOL[p.dtype], p.name
    b.close()


def test_batch_with_fp32_arithmetic_domains():
    # three storage types, so three launch chains (batch stream and two side
    # streams); FP32-arithmetic domains against the oracle at their bar, and
    # their reverse step against the single-grid one
    import torch
    import paper_2602_05017_amd as bf
    probs = _domains(6, lo=24, hi=80, nsteps=2, seed=1013)
    for k in (1, 4):
        probs[k].dtype = "f32fast"
    assert {p.dtype for p in probs} == {"f64", "f32", "f32fast"}
    grids, fields = _setup(probs)
    b = bf.Batch(grids, fields)
    b.step(2)
    for p, g, f in zip(probs, grids, fields):
        u = np.array(p.u0, copy=True)
        src, dr = oracle_lists(p)
        oracle.step(u, p.h, p.D, p.lam, p.dt, src, dr, 2)
        assert rel_err(g.read_field(f), u)[0] <= TOL[p.dtype], p.name
    rng = np.random.default_rng(13)
    grads = [torch.from_numpy(rng.random(p.shape) - 0.5).to(device="cuda", dtype=g.torch_dtype)
             for p, g in zip(probs, grids)]
    gin = [x.clone() for x in grads]
    b.set_grads(grads)
    subset = [1, 2, 4]
    gD, gL = b.step_adjoint(subset)
    off = 0
    for i in subset:
        p, g = probs[i], grids[i]
        got = grads[i].double().cpu().numpy()
        e = _check_adjoint_vs_oracle(p, g.read_field(fields[i]), gin[i].double().cpu().numpy(), got,
                                     gD[off:off + p.S], gL[off:off + p.S])
        print(f"{p.name} {p.dtype} batched reverse step vs oracle: grad {e[0]:.2e}, dD at {e[1]:.2f} "
              f"and dlambda at {e[2]:.2f} of their bars")
        ref_g = gin[i].clone()
        rD, rL = g.step_adjoint(fields[i], ref_g)
        tol = TOL[p.dtype]
        assert rel_err(got, ref_g.double().cpu().numpy())[0] <= tol, p.name
        assert np.max(np.abs(gL[off:off + p.S] - rL) / np.abs(rL)) <= max(tol, 1e-11), p.name
        off += p.S
    b.close()


@pytest.mark.parametrize("mode", MODES)
def test_autotuner_picks_valid_plans_and_keeps_results(tmp_path, mode):
    import torch
    import paper_2602_05017_amd as bf
    probs = _domains(10, lo=24, hi=192, nsteps=2, seed=1007)
    grids, fields = _setup(probs)
    b = bf.Batch(grids, fields, mode=mode)
    cache = str(tmp_path / "tune.json")
    ms = b.autotune(cache)
    assert ms > 0
    for d, p in enumerate(probs):
        for a, n in enumerate((p.nx, p.ny, p.nz)):
            m, lpw = b.plan(d, a)
            assert m in (4, 8, 12, 16) and lpw in (16, 32, 64) and (512 // lpw) * m >= n
    # autotuning ran steps on the fields: reload them, then step and compare
    for p, g, f in zip(probs, grids, fields):
        f.copy_(upload(p, g))
    torch.cuda.synchronize()
    b.step(2)
    for p, g, f in zip(probs, grids, fields):
        u = np.array(p.u0, copy=True)
        src, dr = oracle_lists(p)
        oracle.step(u, p.h, p.D, p.lam, p.dt, src, dr, 2)
        assert rel_err(g.read_field(f), u)[0] <= TOL[p.dtype], p.name
    # a second batch with the same classes reuses the cache
    ms2 = b.autotune(cache)
    assert ms2 > 0
    b.close()


@pytest.mark.parametrize("mode", MODES)
def test_batch_adjoint_subset_matches_oracle_adjoint(mode):
    import torch
    import paper_2602_05017_amd as bf
    probs = _domains(9, lo=24, hi=64, nsteps=1, seed=1008)
    # subset domains: 2 with Dirichlet entries (every copy kept), 0 and 8 with
    # sources only (inner copies dropped), 5 with neither (no copy: the x
    # sweep reads the state itself)
    probs[2].dr = workloads.dirichlet_variant(probs[2], 7)
    probs[5].src = None
    assert all(probs[i].src is not None for i in (0, 2, 8)) and probs[5].dr is None
    grids, fields = _setup(probs)
    state = [f.clone() for f in fields]
    rng = np.random.default_rng(9)
    grads = [torch.from_numpy(rng.random(p.shape) - 0.5).to(device="cuda", dtype=g.torch_dtype)
             for p, g in zip(probs, grids)]
    gin = [x.clone() for x in grads]
    b = bf.Batch(grids, fields, mode=mode)
    before = b.plan(1, 1)
    # M = 16 axes in the subset: their transposed sweeps run as M = 8 tiles of
    # half the lines (64 -> 32, 32 -> 16, 16 -> 16)
    for dom, axis, plan in ((0, 1, (16, 64)), (2, 2, (16, 32)), (5, 0, (16, 16)), (8, 1, (16, 64))):
        b.set_plan(dom, axis, *plan)
        assert b.plan(dom, axis) == plan
    b.set_grads(grads)
    subset = [0, 2, 5, 8]
    gD, gL = b.step_adjoint(subset)
    torch.cuda.synchronize()
    assert all(torch.equal(f, f0) for f, f0 in zip(fields, state))   # states are only read
    off = 0
    for i in subset:
        p, g = probs[i], grids[i]
        S = p.S
        got = grads[i].double().cpu().numpy()
        # the oracle's reverse step on the state and gradient the GPU holds
        e = _check_adjoint_vs_oracle(p, g.read_field(fields[i]), gin[i].double().cpu().numpy(), got,
                                     gD[off:off + S], gL[off:off + S])
        print(f"{p.name} {p.dtype} {p.nx}x{p.ny}x{p.nz}x{S} batched reverse step vs oracle: grad {e[0]:.2e}, "
              f"dD at {e[1]:.2f} and dlambda at {e[2]:.2f} of their bars")
        # and the single-grid reverse step (the other kernel family) agrees
        ref_g = gin[i].clone()
        rD, rL = g.step_adjoint(fields[i], ref_g)
        tol = TOL[p.dtype]
        assert rel_err(got, ref_g.double().cpu().numpy())[0] <= tol
        assert np.max(np.abs(gD[off:off + S] - rD) / np.abs(rD)) <= max(tol, 1e-11)
        assert np.max(np.abs(gL[off:off + S] - rL) / np.abs(rL)) <= max(tol, 1e-11)
        off += S
    # domains outside the subset keep their gradients
    for i in set(range(9)) - set(subset):
        assert torch.equal(grads[i], gin[i])
    # a second call on the same subset replays the captured graph
    gD2, gL2 = b.step_adjoint(subset)
    assert np.all(np.isfinite(gD2)) and np.all(np.isfinite(gL2))
    # plans that do not fit are refused, and the domain keeps its plan
    for dom, axis, m, lpw, code in ((1, 1, 4, 64, "EINVAL"),     # 8 segments x 4 < 63
                                    (1, 1, 5, 16, "EINVAL"), (1, 1, 8, 128, "EINVAL"),
                                    (1, 3, 8, 16, "ERANGE"), (9, 0, 8, 16, "ERANGE")):
        with pytest.raises(bf.BfvmError) as ei:
            b.set_plan(dom, axis, m, lpw)
        assert ei.value.code == code
    assert b.plan(1, 1) == before
    b.close()


def test_persistent_mode_is_refused():
    import paper_2602_05017_amd as bf
    probs = _domains(2, nsteps=1, seed=1009)
    grids, fields = _setup(probs)
    with pytest.raises(bf.BfvmError) as ei:
        bf.Batch(grids, fields, mode="persistent")
    assert ei.value.code == "EOFF"


def test_full_batch_workload_autotuned_100_steps():
    # the benchmark's batch: 96 domains, autotuned plans, 100 graph replays,
    # then the reverse step of domains 0..31 on the final state, as the
    # benchmark runs them.  Against the oracle (one substrate per domain:
    # substrates do not couple): the largest domain of each storage type,
    # the largest domain of each (storage type, axis) whose autotuned tile
    # holds 16 elements per thread, and the two smallest of each storage
    # type after 100 steps; every reverse step of the subset.  Every domain
    # is also compared with its own single-grid GPU run.
    import torch
    import paper_2602_05017_amd as bf
    probs = workloads.batch_config()
    assert len(probs) == 96 and probs[0].nsteps == 100
    grids, fields = _setup(probs)
    b = bf.Batch(grids, fields)
    b.autotune(None)
    plans = [[b.plan(d, a) for a in range(3)] for d in range(96)]
    for p, g, f in zip(probs, grids, fields):
        f.copy_(upload(p, g))
    torch.cuda.synchronize()
    b.step(100)
    got = [g.read_field(f) for g, f in zip(grids, fields)]
    # reverse step of the 32-domain subset on the final state
    subset = list(range(32))
    rng = np.random.default_rng(1005)
    gin = [(rng.random(probs[i].shape) - 0.5).astype(np.float64 if probs[i].dtype == "f64" else np.float32)
           for i in subset]
    grads = [torch.from_numpy(gin[i]).to("cuda") if i < 32 else None for i in range(96)]
    b.set_grads(grads)
    gD, gL = b.step_adjoint(subset)
    gout = [grads[i].double().cpu().numpy() for i in subset]
    b.close()

    size = {i: probs[i].V * probs[i].S for i in range(96)}
    pick = {}
    for dt in ("f64", "f32"):
        of = sorted((i for i in range(96) if probs[i].dtype == dt), key=lambda i: size[i])
        pick[of[-1]] = f"largest {dt}"
        for i in of[:2]:
            pick.setdefault(i, f"smallest {dt}")
        for a in range(3):
            m16 = [i for i in of if plans[i][a][0] == 16]
            if m16:
                pick.setdefault(m16[-1], f"largest {dt} with M=16 on axis {a}")
    n16 = sum(plans[i][a][0] == 16 for i in range(96) for a in range(3))
    print(f"autotuned: {n16} of 288 domain axes at M=16")
    for i, why in sorted(pick.items()):
        p = probs[i]
        s = int(np.argmax(p.D))
        q = one_substrate(p, s)
        u = np.array(q.u0, copy=True)
        src, dr = oracle_lists(q)
        oracle.step(u, q.h, q.D, q.lam, q.dt, src, dr, 100)
        e = rel_err(got[i][..., s:s + 1], u)[0]
        print(f"{p.name} ({why}) {p.dtype} {p.nx}x{p.ny}x{p.nz}x{p.S} plans {plans[i]}, substrate {s}, "
              f"100 steps vs oracle: e_max {e:.3e}")
        assert e <= TOL[p.dtype], (p.name, e)
    off = 0
    worst = {}
    for k, i in enumerate(subset):
        p = probs[i]
        s = k % p.S                     # sampled substrate
        q = one_substrate(p, s)
        st = got[i][..., s:s + 1]
        e = _check_adjoint_vs_oracle(q, st, gin[k][..., s:s + 1], gout[k][..., s:s + 1],
                                     gD[off + s:off + s + 1], gL[off + s:off + s + 1])
        worst[p.dtype] = np.maximum(worst.get(p.dtype, np.zeros(3)), e)
        off += p.S
    print(f"32-domain batched reverse step vs oracle (one substrate each), worst (grad e_max, dD / bar, "
          f"dlambda / bar): {worst}")
    worst = {}
    for p, out in zip(probs, got):
        single = make_grid(p, p.dtype)
        u = upload(p, single)
        single.step(u, 100)
        torch.cuda.synchronize()
        ref = single.read_field(u)
        single.close()
        e = rel_err(out, ref)[0]
        worst[p.dtype] = max(worst.get(p.dtype, 0.0), e)
        assert e <= TOL[p.dtype], (p.name, e)
    print(f"96 domains vs single-grid runs, 100 steps: worst e_max {worst}")


def test_batch_with_members_beyond_the_grouped_limits():
    # members the grouped kernels cannot take (a 300-voxel x line; a z axis of
    # 40 voxels x 64 substrates = 2560 table entries; a 270-voxel y line with
    # FP32 arithmetic) run their own grid's kernels inside the batch's graph,
    # beside grouped members: every domain follows the oracle, the graph
    # equals eager launches, a member beyond the limits equals its own grid's
    # bfvm_step exactly (the same kernels), and the reverse step of a subset
    # mixing both kinds matches the oracle's adjoint
    import torch
    import paper_2602_05017_amd as bf
    small = _domains(3, lo=24, hi=48, nsteps=3, seed=1021)
    big = []
    for k, (shape, S, dtype, ndir) in enumerate((((300, 20, 16), 2, "f64", 9), ((24, 20, 40), 64, "f32", 0),
                                                  ((16, 270, 12), 3, "f32fast", 0))):
        q = small_problem(shape, S, 1030 + k, nsrc=30, ndir=ndir, nsteps=3)
        q.dtype = dtype
        big.append(q)
    probs = [small[0], big[0], small[1], big[1], big[2], small[2]]
    large = {1, 3, 4}
    grids, fields = _setup(probs)
    start = [f.clone() for f in fields]
    b = bf.Batch(grids, fields)
    for i in large:
        with pytest.raises(bf.BfvmError) as ei:
            b.plan(i, 0)
        assert ei.value.code == "ESTATE"
    b.step(3)
    torch.cuda.synchronize()
    for i, (p, g, f) in enumerate(zip(probs, grids, fields)):
        e = rel_err(g.read_field(f), oracle_run(p, 3))[0]
        print(f"{p.name} {p.dtype} {p.nx}x{p.ny}x{p.nz}x{p.S} {'own kernels' if i in large else 'grouped'}: "
              f"3 steps vs oracle e_max {e:.2e}")
        assert e <= TOL[p.dtype], (i, p.dtype, e)
    eager = [x.clone() for x in start]
    b2 = bf.Batch(grids, eager)
    b2.step(3, graph=False)
    torch.cuda.synchronize()
    assert all(torch.equal(x, f) for x, f in zip(eager, fields))
    b2.close()
    for i in large:
        own = start[i].clone()
        grids[i].step(own, 3)
        torch.cuda.synchronize()
        assert torch.equal(own, fields[i]), i
    # a grid beyond the limits may hold one member only
    with pytest.raises(bf.BfvmError) as ei:
        bf.Batch([grids[1], grids[1]], [fields[1], start[1]])
    assert ei.value.code == "EINVAL"
    # reverse step of a subset with grouped and own-kernel members
    rng = np.random.default_rng(21)
    gin = [(rng.random(p.shape) - 0.5).astype(np.float64 if p.dtype == "f64" else np.float32) for p in probs]
    grads = [torch.from_numpy(x.copy()).to("cuda") for x in gin]
    b.set_grads(grads)
    subset = [3, 0, 1, 4, 5]
    gD, gL = b.step_adjoint(subset)
    torch.cuda.synchronize()
    off = 0
    for i in subset:
        p = probs[i]
        e = _check_adjoint_vs_oracle(p, grids[i].read_field(fields[i]), gin[i], grads[i].double().cpu().numpy(),
                                     gD[off:off + p.S], gL[off:off + p.S])
        print(f"{p.name} {p.dtype} reverse step vs oracle: grad {e[0]:.2e}, dD at {e[1]:.2f} and dlambda at "
              f"{e[2]:.2f} of their bars")
        off += p.S
    assert torch.equal(grads[2], torch.from_numpy(gin[2]).to("cuda"))   # outside the subset
    # new gradient buffers (the graph is captured again for the members
    # whose launches carry their pointers): the same sums from the same
    # gradients, and the previous buffers are left alone
    kept = [g.clone() for g in grads]
    fresh = [torch.from_numpy(x.copy()).to("cuda") for x in gin]
    b.set_grads(fresh)
    gD2, gL2 = b.step_adjoint(subset)
    assert np.array_equal(gD2, gD) and np.array_equal(gL2, gL)
    assert all(torch.equal(x, y) for x, y in zip(grads, kept))
    assert all(torch.equal(fresh[i], grads[i]) for i in subset)
    # new field buffers for the forward graph likewise
    before = [f.clone() for f in fields]
    moved = [f.clone() for f in fields]
    b.set_fields(moved)
    b.step(1)
    torch.cuda.synchronize()
    assert all(torch.equal(f, f0) for f, f0 in zip(fields, before))
    for i in large:
        own = before[i].clone()
        grids[i].step(own, 1)
        torch.cuda.synchronize()
        assert torch.equal(own, moved[i]), i
    b.close()


def test_batch_follows_member_grid_changes():
    # params, sources and Dirichlet lists of member grids change after the
    # batch was created (their device tables and lists are reallocated, with
    # new lengths): the batch re-reads the grids and re-captures its graphs,
    # so each domain follows the oracle run with the same change
    import torch
    import paper_2602_05017_amd as bf
    probs = _domains(4, lo=24, hi=48, nsteps=2, seed=1014)
    probs[2].dr = workloads.dirichlet_variant(probs[2], 6)
    grids, fields = _setup(probs)
    b = bf.Batch(grids, fields)
    b.step(2)
    ref = []
    for p in probs:
        u = np.array(p.u0, copy=True)
        src, dr = oracle_lists(p)
        oracle.step(u, p.h, p.D, p.lam, p.dt, src, dr, 2)
        ref.append(u)
    # domain 1: new D, lambda and dt; domain 2: a longer source list and no
    # Dirichlet entries; domain 3: Dirichlet entries added
    p1, p2, p3 = probs[1], probs[2], probs[3]
    p1.D, p1.lam, p1.dt = p1.D * 2.5, p1.lam * 0.3, p1.dt * 1.5
    grids[1].set_params(p1.D, p1.lam, p1.dt)
    p2.src = workloads.make_sources(p2.seed + 7, p2.V, p2.S, 3 * len(p2.src))
    grids[2].set_sources(p2.src.voxel, p2.src.secretion, p2.src.saturation, p2.src.uptake)
    p2.dr = None
    grids[2].set_dirichlet(np.zeros(0, dtype=np.int64), np.zeros(0), np.zeros(0, dtype=np.uint8))
    p3.dr = workloads.dirichlet_variant(p3, 5)
    grids[3].set_dirichlet(p3.dr.voxel, p3.dr.value, p3.dr.active)
    b.step(2)
    for k, (p, g, f) in enumerate(zip(probs, grids, fields)):
        src, dr = oracle_lists(p)
        oracle.step(ref[k], p.h, p.D, p.lam, p.dt, src, dr, 2)
        e = rel_err(g.read_field(f), ref[k])[0]
        assert e <= TOL[p.dtype], (k, p.dtype, e)
    # the reverse step of the changed domains uses the new tables too
    rng = np.random.default_rng(14)
    gin = [(rng.random(p.shape) - 0.5).astype(np.float64 if p.dtype == "f64" else np.float32) for p in probs]
    grads = [torch.from_numpy(x.copy()).to("cuda") for x in gin]
    b.set_grads(grads)
    gD, gL = b.step_adjoint([1, 2, 3])
    off = 0
    for i in (1, 2, 3):
        p = probs[i]
        _check_adjoint_vs_oracle(p, grids[i].read_field(fields[i]), gin[i], grads[i].double().cpu().numpy(),
                                 gD[off:off + p.S], gL[off:off + p.S])
        off += p.S
    b.close()
