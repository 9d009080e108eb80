"""Closed forms and invariants that pin the FP64 oracle at any size (CPU only).

K3 DCT-II eigenmodes, K4 mass decay (1+beta)^-3 per step, K5 constant field,
K6 axis permutations, K7 D = 0 / lambda = 0, K8 source-only relaxation,
K9 linearity, K10 positivity and maximum principle, K11 Dirichlet values.
The facts used: the zero-flux matrix of App. A is (1+beta) I + r L_N with L_N
the Neumann Laplacian, whose eigenvectors are cos(pi k (i + 1/2) / n) with
eigenvalues 4 sin^2(pi k / 2n), and whose rows and columns sum to 0.
"""
import itertools

import numpy as np
import pytest

import oracle
import workloads


def eigenmode(nx, ny, nz, kx, ky, kz):
    cx = np.cos(np.pi * kx * (np.arange(nx) + 0.5) / nx)
    cy = np.cos(np.pi * ky * (np.arange(ny) + 0.5) / ny)
    cz = np.cos(np.pi * kz * (np.arange(nz) + 0.5) / nz)
    return cz[:, None, None] * cy[None, :, None] * cx[None, None, :]


def mu(n, k, r, beta):
    return 1.0 + beta + 4.0 * r * np.sin(np.pi * k / (2.0 * n)) ** 2


@pytest.mark.parametrize("shape,ks", [
    ((64, 64, 64), (3, 1, 5)),          # 64^3 Gaussian workload's grid
    ((1000, 8, 6), (37, 1, 1)),         # a 1000-long x-line
    ((8, 1000, 6), (1, 999, 0)),        # a 1000-long y-line, highest mode
    ((6, 8, 1000), (0, 1, 500)),        # a 1000-long z-line
    ((1, 5, 3), (0, 2, 1)),             # single-voxel axis
])
def test_eigenmode_decay(shape, ks):
    nx, ny, nz = shape
    kx, ky, kz = ks
    S = 2
    h = np.array([20.0, 10.0, 15.0])
    D = np.array([2.0e3, 3.0e2])
    L = np.array([0.1, 0.7])
    dt = 0.01
    m = 3
    base = eigenmode(nx, ny, nz, kx, ky, kz)
    u = np.ascontiguousarray(np.repeat(base[..., None], S, axis=3))
    oracle.step(u, h, D, L, dt, nsteps=m)
    for s in range(S):
        beta = dt * L[s] / 3.0
        fac = 1.0
        for n, k, a in ((nx, kx, 0), (ny, ky, 1), (nz, kz, 2)):
            fac *= mu(n, k, dt * D[s] / h[a] ** 2, beta) ** (-m)
        ref = base * fac
        # rounding enters at the size of the initial field and A^-1 is a
        # contraction, so the error is bounded relative to max |u0|; the
        # decay factors are kept moderate so that this still pins mu to ~1e-8
        err = np.max(np.abs(u[..., s] - ref)) / np.max(np.abs(base))
        assert err <= 1e-12, (s, err)
        assert fac > 1e-4


@pytest.mark.parametrize("shape", [(64, 64, 64), (17, 9, 30)])
def test_mass_decays_by_one_plus_beta_cubed(shape):
    nx, ny, nz = shape
    S = 3
    rng = np.random.default_rng(11)
    u0 = rng.random((nz, ny, nx, S))
    h = np.array([10.0, 10.0, 10.0])
    D = np.array([1e2, 1e4, 1e5])
    L = np.array([0.0, 0.3, 1.0])
    dt = 0.01
    m = 5
    u = oracle.step(u0.copy(), h, D, L, dt, nsteps=m)
    for s in range(S):
        beta = dt * L[s] / 3.0
        ref = np.sum(u0[..., s]) * (1.0 + beta) ** (-3 * m)
        assert abs(np.sum(u[..., s]) - ref) <= 1e-12 * abs(ref)


def test_constant_field_stays_uniform():
    S = 2
    u = np.full((12, 7, 9, S), 2.5)
    D = np.array([5e4, 10.0])
    L = np.array([0.2, 0.05])
    dt = 0.02
    m = 4
    oracle.step(u, np.array([10.0, 7.0, 13.0]), D, L, dt, nsteps=m)
    for s in range(S):
        ref = 2.5 * (1.0 + dt * L[s] / 3.0) ** (-3 * m)
        # r reaches 20 here; Thomas rounding grows like (1 + 2r) eps
        assert np.max(np.abs(u[..., s] - ref)) <= 1e-13 * ref


def test_axis_permutation_symmetry_on_cubes():
    rng = np.random.default_rng(5)
    n, S = 9, 2
    u0 = rng.random((n, n, n, S))
    h = np.array([10.0] * 3)
    D = np.array([3e3, 9e4])
    L = np.array([0.1, 0.5])
    dt = 0.01
    # sources permute with the voxels; no Dirichlet (it does not commute with the sweeps)
    vz, vy, vx = rng.integers(0, n, (3, 6))
    sec = rng.uniform(0, 10, (6, S))
    upt = rng.uniform(0, 10, (6, S))
    sat = np.ones((6, S))
    base_src = oracle.Sources((vz * n + vy) * n + vx, sec, sat, upt)
    ref = oracle.step(u0.copy(), h, D, L, dt, base_src, nsteps=2)
    for perm in itertools.permutations(range(3)):
        # perm acts on the spatial axes of the [z, y, x] array
        up = np.array(np.transpose(u0, perm + (3,)), order="C", copy=True)
        coords = np.stack([vz, vy, vx])
        pc = coords[list(perm)]
        src = oracle.Sources((pc[0] * n + pc[1]) * n + pc[2], sec, sat, upt)
        got = oracle.step(up, h, D, L, dt, src, nsteps=2)
        want = np.transpose(ref, perm + (3,))
        assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want)), perm


def test_no_diffusion_is_pure_decay_and_no_decay_conserves_mass():
    rng = np.random.default_rng(6)
    u0 = rng.random((6, 5, 7, 2))
    h = np.array([10.0, 10.0, 10.0])
    dt = 0.05
    L = np.array([0.4, 0.9])
    u = oracle.step(u0.copy(), h, np.zeros(2), L, dt, nsteps=3)
    ref = u0 / ((1.0 + dt * L / 3.0) ** 9)[None, None, None, :]
    assert np.max(np.abs(u - ref)) <= 1e-15
    u = oracle.step(u0.copy(), h, np.array([1e4, 1e5]), np.zeros(2), dt, nsteps=3)
    assert np.allclose(u.sum(axis=(0, 1, 2)), u0.sum(axis=(0, 1, 2)), rtol=1e-13, atol=0)


def test_source_only_relaxes_to_equilibrium():
    rng = np.random.default_rng(7)
    u0 = rng.random((4, 4, 4, 2))
    vox = np.array([3, 17, 40])
    sec = rng.uniform(0, 10, (3, 2))
    upt = rng.uniform(0, 10, (3, 2))
    sat = np.ones((3, 2))
    dt = 0.01
    m = 6
    src = oracle.Sources(vox, sec, sat, upt)
    u = oracle.step(u0.copy(), np.array([10.0] * 3), np.zeros(2), np.zeros(2), dt, src, nsteps=m)
    flat0 = u0.reshape(64, 2)
    flat = u.reshape(64, 2)
    Q = 1.0 + dt * (sec + upt)
    ueq = sec * sat / (sec + upt)
    ref = ueq + (flat0[vox] - ueq) * Q ** (-m)
    assert np.max(np.abs(flat[vox] - ref)) <= 1e-14
    others = np.setdiff1d(np.arange(64), vox)
    assert np.array_equal(flat[others], flat0[others])


def test_linearity_without_sources():
    rng = np.random.default_rng(8)
    a, b = rng.random((2, 5, 6, 7, 3))
    h = np.array([10.0, 12.0, 8.0])
    D = np.array([1e3, 1e4, 1e5])
    L = np.array([0.1, 0.2, 0.3])
    dt = 0.01
    alpha, gamma = 1.7, -0.3
    lhs = oracle.step(alpha * a + gamma * b, h, D, L, dt, nsteps=2)
    rhs = alpha * oracle.step(a.copy(), h, D, L, dt, nsteps=2) + gamma * oracle.step(b.copy(), h, D, L, dt, nsteps=2)
    assert np.max(np.abs(lhs - rhs)) <= 1e-13 * np.max(np.abs(lhs))


def test_positivity_and_maximum_principle():
    rng = np.random.default_rng(9)
    u0 = rng.random((10, 11, 12, 2)) ** 8      # spiky, non-negative
    h = np.array([10.0] * 3)
    D = np.array([1e5, 1e3])
    L = np.array([0.3, 1.0])
    dt = 0.1
    m = 4
    u = oracle.step(u0.copy(), h, D, L, dt, nsteps=m)
    assert np.all(u >= 0.0)
    for s in range(2):
        bound = np.max(u0[..., s]) * (1.0 + dt * L[s] / 3.0) ** (-3 * m)
        assert np.max(u[..., s]) <= bound * (1 + 1e-15)
        assert np.min(u[..., s]) >= np.min(u0[..., s]) * (1.0 + dt * L[s] / 3.0) ** (-3 * m) * (1 - 1e-15)


def test_dirichlet_values_hold_exactly_after_each_step():
    p = workloads.config(2, n=24, nsub=3, n_sources=200, nsteps=1)
    u = p.field().copy()
    src = oracle.Sources(p.src.voxel, p.src.secretion, p.src.saturation, p.src.uptake)
    dr = oracle.Dirichlet(p.dr.voxel, p.dr.value, p.dr.active)
    for _ in range(3):
        oracle.step(u, p.h, p.D, p.lam, p.dt, src, dr, 1)
        flat = u.reshape(-1, p.S)
        assert np.all(flat[p.dr.voxel, 0] == 38.0)


def test_gaussian_workload_mass_matches_closed_form():
    # the 64^3 Gaussian workload has no sources or Dirichlet nodes: K4 applies exactly
    p = workloads.config(1)
    u = p.field().copy()
    oracle.step(u, p.h, p.D, p.lam, p.dt, nsteps=p.nsteps)
    beta = p.dt * p.lam[0] / 3.0
    ref = np.sum(p.u0) * (1.0 + beta) ** (-3 * p.nsteps)
    assert abs(np.sum(u) - ref) <= 1e-12 * ref
