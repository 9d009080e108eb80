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


def one_substrate(p, s):
    """Substrate s of problem p as a problem of its own (substrates do not
    couple: sources, Dirichlet entries and sweeps act per substrate)."""
    q = workloads.Problem(f"{p.name}[s={s}]", p.nx, p.ny, p.nz, 1, p.h, p.D[s:s + 1].copy(), p.lam[s:s + 1].copy(),
                          p.dt, p.nsteps, p.seed, dtype=p.dtype)
    if p.src is not None and len(p.src):
        q.src = workloads.SourceList(p.src.voxel, p.src.secretion[:, s:s + 1], p.src.saturation[:, s:s + 1],
                                     p.src.uptake[:, s:s + 1])
    if p.dr is not None and len(p.dr):
        keep = p.dr.active[:, s] != 0
        if keep.any():
            q.dr = workloads.DirichletList(p.dr.voxel[keep], p.dr.value[keep, s:s + 1],
                                           p.dr.active[keep, s:s + 1])
    q.u0 = np.ascontiguousarray(p.field()[..., s:s + 1])
    return q


def oracle_adjoint(p, state, gin):
    """The oracle's reverse of one step of p started from `state` (host,
    converted to FP64) applied to the gradient `gin`: (grad, dL/dD, dL/dlambda)."""
    src, dr = oracle_lists(p)
    g = np.array(gin, dtype=np.float64, copy=True)
    gD = np.zeros(p.S)
    gL = np.zeros(p.S)
    oracle.adjoint_step(np.ascontiguousarray(state, dtype=np.float64), g, gD, gL, p.h, p.D, p.lam, p.dt, src, dr)
    return g, gD, gL


def rel_vec(got, ref):
    """max_s |got_s - ref_s| / |ref_s|."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)))


# Rounding units of the reverse step's stored values, per storage form, and
# how many roundings reach one term of the parameter-gradient sums (below).
_EPS = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "f32fast": 2.0 ** -24}


def param_grad_bars(p, state, gin):
    """Normwise bars for one reverse step's dL/dD and dL/dlambda per substrate.

    dL/dD_s = -sum_a dt/h_a^2 sum_i y_i (L_N x)_i and dL/dlambda_s =
    -(dt/3) sum_a sum_i y_i x_i are sums of terms of both signs (the columns
    of L_N sum to zero), so their relative error is not bounded; the
    absolute one is.  If every stored y and x value carries a relative error
    of at most k*eps, each sum moves by at most k*eps * sum_i |y_i| |(L_N
    x)_i| (plus the same with x), and by Cauchy-Schwarz with ||L_N||_2 <= 4
    this is <= 2 * 4 k eps ||y||_2 ||x||_2.  Every solve and the masks are
    contractions in the 2-norm (A symmetric with eigenvalues >= 1 + beta), so
    ||y||_2 <= ||g||_2, and ||x||_2 is at most the largest 2-norm of the
    forward stage outputs (computed here with the oracle's stages).
    k: FP64 storage 64 (about log2 of the terms for the tree sums plus the
    roundings of one term); FP32 storage 16 (three stored sweep outputs and
    three stored transposed outputs of 2^-24 each); FP32 arithmetic 16 (1 +
    2 r), the rounded constants amplified by the conditioning."""
    S = p.S
    u = np.array(state, dtype=np.float64, copy=True)
    src, dr = oracle_lists(p)
    xn = np.sqrt(np.sum(u.reshape(-1, S) ** 2, axis=0))
    if src is not None:
        oracle.source(u, src, p.dt)
    for axis in (None, 0, 1, 2):
        if axis is not None:
            oracle.sweep(u, p.h, p.D, p.lam, p.dt, axis)
        if dr is not None:
            oracle.dirichlet(u, dr)
        xn = np.maximum(xn, np.sqrt(np.sum(u.reshape(-1, S) ** 2, axis=0)))
    gn = np.sqrt(np.sum(np.asarray(gin, dtype=np.float64).reshape(-1, S) ** 2, axis=0))
    r_max = float(np.max(p.dt * np.asarray(p.D)[None, :] / np.asarray(p.h)[:, None] ** 2))
    k = {"f64": 64.0, "f32": 16.0, "f32fast": 16.0 * (1.0 + 2.0 * r_max)}[p.dtype]
    base = k * _EPS[p.dtype] * gn * xn
    barD = 2.0 * 4.0 * base * sum(p.dt / h ** 2 for h in p.h)
    barL = 2.0 * base * p.dt
    return barD, barL
