"""Pins of the FP64 oracle against brute force and hand-derived values (CPU only).

K1: every stage of the step against dense Kronecker solves on tiny grids.
K2: Thomas factors against an LU factorisation of the matrix (App. A).
Golden: hand-derived factors and solves (tests/golden/thomas_small.txt).
"""
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "thomas_small.txt")


def _random_case(rng, shape_zyx, S, nsrc=0, ndir=0, dup=False):
    nz, ny, nx = shape_zyx
    V = nx * ny * nz
    u = rng.random((nz, ny, nx, S))
    h = rng.uniform(5.0, 20.0, 3)
    D = 10.0 ** rng.uniform(1.0, 4.5, S)
    L = rng.uniform(0.0, 1.0, S)
    dt = rng.uniform(0.01, 0.1)
    src = dr = None
    if nsrc:
        vox = rng.integers(0, V, nsrc)
        if dup and nsrc > 1:
            vox[-1] = vox[0]
        src = oracle.Sources(vox, rng.uniform(0, 10, (nsrc, S)), rng.uniform(0, 2, (nsrc, S)),
                             rng.uniform(0, 10, (nsrc, S)))
    if ndir:
        vox = rng.integers(0, V, ndir)
        if dup and ndir > 1:
            vox[-1] = vox[0]
        act = (rng.random((ndir, S)) < 0.7).astype(np.uint8)
        dr = oracle.Dirichlet(vox, rng.uniform(0, 50, (ndir, S)), act)
    return u, h, D, L, dt, src, dr


SHAPES = [(1, 1, 1), (1, 1, 5), (2, 3, 1), (3, 5, 4), (5, 2, 8), (8, 3, 2), (4, 4, 4), (2, 8, 5)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("S", [1, 3])
def test_step_matches_dense_plain(shape, S):
    rng = np.random.default_rng(hash((shape, S)) % (1 << 32))
    u, h, D, L, dt, _, _ = _random_case(rng, shape, S)
    got = oracle.step(u.copy(), h, D, L, dt, nsteps=2)
    ref = dense.step_dense(u, h, D, L, dt, nsteps=2)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("shape", SHAPES[2:])
@pytest.mark.parametrize("dup", [False, True])
def test_step_matches_dense_with_sources_and_dirichlet(shape, dup):
    rng = np.random.default_rng(7 + hash(shape) % 1000 + dup)
    V = int(np.prod(shape))
    u, h, D, L, dt, src, dr = _random_case(rng, shape, 3, nsrc=min(5, V), ndir=min(4, V), dup=dup)
    got = oracle.step(u.copy(), h, D, L, dt, src, dr, nsteps=3)
    ref = dense.step_dense(u, h, D, L, dt, src, dr, nsteps=3)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_single_sweep_is_the_axis_operator(axis):
    # each sweep alone must equal the dense solve with its own axis' operator
    rng = np.random.default_rng(100 + axis)
    shape = (3, 5, 4)
    u, h, D, L, dt, _, _ = _random_case(rng, shape, 2)
    got = oracle.sweep(u.copy(), h, D, L, dt, axis)
    V = int(np.prod(shape))
    for s in range(2):
        A = dense.sweep_operator(shape, axis, dt * D[s] / h[axis] ** 2, dt * L[s] / 3.0)
        ref = np.linalg.solve(A, u[..., s].reshape(V)).reshape(shape)
        assert np.max(np.abs(got[..., s] - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_source_and_dirichlet_stages_alone():
    rng = np.random.default_rng(3)
    u = rng.random((2, 3, 4, 2))
    src = oracle.Sources([5, 1, 5], rng.uniform(0, 10, (3, 2)), np.ones((3, 2)), rng.uniform(0, 10, (3, 2)))
    dt = 0.05
    got = oracle.source(u.copy(), src, dt)
    P, Q = dense.source_affine(24, 2, dt, src)
    ref = ((u.reshape(24, 2) + P) / Q).reshape(u.shape)
    assert np.max(np.abs(got - ref)) <= 1e-15
    dr = oracle.Dirichlet([2, 2, 7], [[1.0, 2.0], [3.0, 4.0], [5.0, 6.0]],
                          np.array([[1, 1], [1, 0], [0, 1]], dtype=np.uint8))
    got = oracle.dirichlet(u.copy(), dr).reshape(24, 2)
    assert got[2, 0] == 3.0 and got[2, 1] == 2.0 and got[7, 1] == 6.0
    assert got[7, 0] == u.reshape(24, 2)[7, 0]


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 257])
@pytest.mark.parametrize("r,beta", [(0.01, 1e-4), (2.5, 3.3e-4), (10.0, 0.3), (100.0, 0.0)])
def test_factors_are_lu_of_matrix(n, r, beta):
    A = dense.fv_matrix(n, r, beta)
    P, Lw, U = scipy.linalg.lu(A)
    assert np.array_equal(P, np.eye(n))             # diagonally dominant: no pivoting
    denom, cprime = oracle.factor(n, r, beta)
    # denom_i = b_i - r |c'_{i-1}| cancels up to a factor ~ (1 + 2r) / denom_i
    tol = 4e-16 * (1.0 + 2.0 * r + beta)
    assert np.max(np.abs(denom - np.diag(U)) / np.diag(U)) <= tol
    if n > 1:
        sup = np.diag(U, 1) / np.diag(U)[:-1]
        assert np.max(np.abs(cprime[:-1] - sup)) <= tol
    # stability facts used by the GPU path's division-free form
    assert np.all(denom >= 1.0 + beta - 1e-15)
    assert np.all(np.abs(cprime) < 1.0)


def _golden_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            head, denom, cp, d, x = [p.strip() for p in line.split("|")]
            name, n, r, beta = head.split()
            rows.append((name, int(n), float(r), float(beta),
                         [float(v) for v in denom.split()], [float(v) for v in cp.split()],
                         [float(v) for v in d.split()], [float(v) for v in x.split()]))
    return rows


@pytest.mark.parametrize("row", _golden_rows(), ids=lambda r: r[0])
def test_hand_derived_factors_and_solve(row):
    name, n, r, beta, denom_ref, cp_ref, d, x_ref = row
    denom, cprime = oracle.factor(n, r, beta)
    assert np.allclose(denom, denom_ref, rtol=1e-15, atol=0)
    assert np.allclose(cprime[: n - 1], cp_ref, rtol=1e-15, atol=0)
    # a single x-line: field [1, 1, n, 1], hx chosen so that r = dt D / hx^2
    u = np.array(d, dtype=np.float64).reshape(1, 1, n, 1)
    dt = 1.0
    oracle.sweep(u, np.array([1.0, 1.0, 1.0]), np.array([r]), np.array([3.0 * beta]), dt, 0)
    assert np.allclose(u.reshape(-1), x_ref, rtol=1e-15, atol=1e-16)
