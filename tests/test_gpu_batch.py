"""Batched multi-domain form: uneven domains (each axis 24..192 voxels, 1..8
substrates, FP32/FP64 storage mixed) stepped together, one graph replay per
step.  Every domain is compared with the FP64 oracle at its storage type's
bar and with its own single-grid GPU run within the same bar (the batch
reads the Thomas constants from the global tables instead of LDS, which
can change the rounding of individual products only through operation
order, so equality is not required); graph replays must equal eager
launches exactly.

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
from gpu_helpers import make_grid, oracle_lists, rel_err, upload

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f32fast": 1e-4}

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
        ref_g = gin[i].clone()
        rD, rL = g.step_adjoint(fields[i], ref_g)
        tol = TOL[p.dtype]
        assert rel_err(grads[i].double().cpu().numpy(), ref_g.double().cpu().numpy())[0] <= tol, p.name
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
            assert m in (4, 8, 16) and lpw in (16, 32, 64) and (512 // lpw) * m >= n
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
def test_batch_adjoint_subset_matches_single_grid_adjoint(mode):
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
        ref_g = gin[i].clone()
        rD, rL = g.step_adjoint(fields[i], ref_g)
        tol = TOL[p.dtype]
        assert rel_err(grads[i].double().cpu().numpy(), ref_g.double().cpu().numpy())[0] <= tol
        S = p.S
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
    # the benchmark's batch: 96 domains, autotuned plans, 100 graph replays;
    # every domain against its own single-grid GPU run, and the two smallest
    # domains of each storage type against the oracle
    import torch
    import paper_2602_05017_amd as bf
    probs = workloads.batch_config()
    assert len(probs) == 96 and probs[0].nsteps == 100
    grids, fields = _setup(probs)
    b = bf.Batch(grids, fields)
    b.autotune(None)
    for p, g, f in zip(probs, grids, fields):
        f.copy_(upload(p, g))
    torch.cuda.synchronize()
    b.step(100)
    got = [g.read_field(f) for g, f in zip(grids, fields)]
    b.close()
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
    by_size = sorted(range(96), key=lambda k: probs[k].V * probs[k].S)
    sample = [i for i in by_size if probs[i].dtype == "f64"][:2] + [i for i in by_size if probs[i].dtype == "f32"][:2]
    for i in sample:
        p = probs[i]
        u = np.array(p.u0, copy=True)
        src, dr = oracle_lists(p)
        oracle.step(u, p.h, p.D, p.lam, p.dt, src, dr, 100)
        e = rel_err(got[i], u)[0]
        print(f"{p.name} {p.dtype} {p.nx}x{p.ny}x{p.nz}x{p.S} vs oracle, 100 steps: e_max {e:.3e}")
        assert e <= TOL[p.dtype]


def test_batch_rejects_tables_too_large_for_lds():
    import paper_2602_05017_amd as bf
    g = bf.Grid(256, 24, 24, 9, (10.0, 10.0, 10.0), dtype="f64")   # 256 x 9 > 2048 on x
    g.set_params(np.full(9, 1e3), np.full(9, 0.1), 0.01)
    import torch
    u = torch.zeros((24, 24, 256, 9), dtype=torch.float64, device="cuda")
    with pytest.raises(bf.BfvmError) as ei:
        bf.Batch([g], [u])
    assert ei.value.code == "EINVAL"
    g.close()
