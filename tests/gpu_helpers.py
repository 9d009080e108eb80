"""Helpers shared by the GPU parity tests: run a workload through the C ABI
(paper_2602_05017_amd) and through the oracle on the same seeded inputs."""
import numpy as np

import oracle
import workloads


def rel_err(got, ref):
    """Per-substrate normwise errors: max|d|/max|ref| and ||d||_2/||ref||_2 (worst substrate)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    S = ref.shape[-1]
    g = got.reshape(-1, S)
    r = ref.reshape(-1, S)
    d = g - r
    emax = np.max(np.abs(d), axis=0) / np.maximum(np.max(np.abs(r), axis=0), 1e-300)
    e2 = np.sqrt(np.sum(d * d, axis=0)) / np.maximum(np.sqrt(np.sum(r * r, axis=0)), 1e-300)
    return float(np.max(emax)), float(np.max(e2))


def oracle_lists(p):
    src = dr = None
    if p.src is not None and len(p.src):
        src = oracle.Sources(p.src.voxel, p.src.secretion, p.src.saturation, p.src.uptake)
    if p.dr is not None and len(p.dr):
        dr = oracle.Dirichlet(p.dr.voxel, p.dr.value, p.dr.active)
    return src, dr


def oracle_run(p, nsteps=None):
    u = np.array(p.field(), dtype=np.float64, copy=True)
    src, dr = oracle_lists(p)
    oracle.step(u, p.h, p.D, p.lam, p.dt, src, dr, p.nsteps if nsteps is None else nsteps)
    return u


def make_grid(p, dtype="f64", plans=None, schedule=None):
    import paper_2602_05017_amd as bf
    g = bf.Grid(p.nx, p.ny, p.nz, p.S, tuple(p.h), dtype=dtype)
    if schedule is not None:
        g.set_schedule(*schedule)
    g.set_params(p.D, p.lam, p.dt)
    if p.src is not None and len(p.src):
        g.set_sources(p.src.voxel, p.src.secretion, p.src.saturation, p.src.uptake)
    if p.dr is not None and len(p.dr):
        g.set_dirichlet(p.dr.voxel, p.dr.value, p.dr.active)
    if plans:
        for axis, plan in plans.items():
            g.set_plan(axis, *plan)
    return g


def upload(p, g):
    import torch
    return torch.from_numpy(np.ascontiguousarray(p.field())).to(device="cuda", dtype=g.torch_dtype)


def gpu_run(p, dtype="f64", nsteps=None, plans=None, schedule=None):
    import torch
    g = make_grid(p, dtype, plans, schedule)
    u = upload(p, g)
    g.step(u, p.nsteps if nsteps is None else nsteps)
    torch.cuda.synchronize()
    out = g.read_field(u)
    g.close()
    return out


def small_problem(shape, S, seed, nsrc=0, ndir=0, D_range=(2.0, 5.0), dt=0.01, h=(10.0, 10.0, 10.0),
                  nsteps=3):
    """A seeded problem of any shape: D log-uniform, lambda U(0.01, 1), uniform field."""
    nx, ny, nz = shape
    D, L = workloads.random_coefficients(seed, S, D_range, (0.01, 1.0))
    p = workloads.Problem(f"small{shape}x{S}", nx, ny, nz, S, np.array(h, dtype=np.float64), D, L, dt,
                          nsteps, seed)
    if nsrc:
        p.src = workloads.make_sources(seed, p.V, S, min(nsrc, p.V))
    if ndir:
        p.dr = workloads.dirichlet_variant(p, min(ndir, p.V))
    p.field()
    return p
