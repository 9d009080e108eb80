"""Pins of the oracle's adjoint step (CPU only).

K12 (i) dot-product test of the linear part of one step, (ii) central finite
differences for D, lambda and the initial field, (iii) closed-form gradients
of an eigenmode, (iv) dense transposes on tiny grids.  Loss: L = sum (u_N - t)^2.
"""
import numpy as np
import pytest

import oracle
from oracle import dense


def _setup(rng, shape=(4, 5, 6), S=2, with_lists=True):
    nz, ny, nx = shape
    V = nx * ny * nz
    u0 = rng.random((nz, ny, nx, S))
    h = np.array([10.0, 8.0, 12.0])
    D = np.array([2e3, 4e4])[:S]
    L = np.array([0.3, 0.8])[:S]
    dt = 0.02
    src = dr = None
    if with_lists:
        src = oracle.Sources(rng.integers(0, V, 5), rng.uniform(0, 10, (5, S)), np.ones((5, S)),
                             rng.uniform(0, 10, (5, S)))
        dr = oracle.Dirichlet(rng.integers(0, V, 3), rng.uniform(0, 5, (3, S)),
                              (rng.random((3, S)) < 0.6).astype(np.uint8))
    return u0, h, D, L, dt, src, dr


def test_dot_product_of_linear_part():
    rng = np.random.default_rng(21)
    u0, h, D, L, dt, src, dr = _setup(rng)
    # linear part: zero saturation (P = 0) and zero Dirichlet values
    lin_src = oracle.Sources(src.voxel, src.secretion, np.zeros_like(src.saturation), src.uptake)
    lin_dr = oracle.Dirichlet(dr.voxel, np.zeros_like(dr.value), dr.active)
    v = rng.random(u0.shape) - 0.5
    w = rng.random(u0.shape) - 0.5
    Mv = oracle.step(v.copy(), h, D, L, dt, lin_src, lin_dr, 1)
    MTw = oracle.adjoint_step(u0, w.copy(), np.zeros(2), np.zeros(2), h, D, L, dt, lin_src, lin_dr)
    lhs = float(np.sum(Mv * w))
    rhs = float(np.sum(v * MTw))
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1e-300) * 10


def test_dense_transpose_of_several_steps():
    rng = np.random.default_rng(22)
    shape = (3, 4, 5)
    u0, h, D, L, dt, src, dr = _setup(rng, shape)
    N = 3
    t = rng.random(u0.shape)
    Lval, uN, g0, gD, gL = oracle.run_with_gradient(u0, t, h, D, L, dt, N, src, dr)
    V = int(np.prod(shape))
    P, Q = dense.source_affine(V, 2, dt, src)
    mask, _ = dense.dirichlet_table(V, 2, dr)
    for s in range(2):
        M = dense.step_matrix(shape, h, D[s], L[s], dt, mask[:, s], Q[:, s])
        MN = np.linalg.matrix_power(M, N)
        ref = 2.0 * MN.T @ (uN[..., s] - t[..., s]).reshape(V)
        got = g0[..., s].reshape(V)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def _loss(u0, t, h, D, L, dt, N, src, dr):
    u = oracle.step(u0.copy(), h, D, L, dt, src, dr, N)
    return float(np.sum((u - t) ** 2))


def test_central_differences():
    rng = np.random.default_rng(23)
    u0, h, D, L, dt, src, dr = _setup(rng)
    N = 4
    t = rng.random(u0.shape)
    Lval, uN, g0, gD, gL = oracle.run_with_gradient(u0, t, h, D, L, dt, N, src, dr)
    assert abs(Lval - _loss(u0, t, h, D, L, dt, N, src, dr)) <= 1e-14 * Lval
    for s in range(2):
        for which, grad in (("D", gD), ("L", gL)):
            base = D if which == "D" else L
            eps = 1e-6 * base[s]
            plus, minus = base.copy(), base.copy()
            plus[s] += eps
            minus[s] -= eps
            if which == "D":
                fd = (_loss(u0, t, h, plus, L, dt, N, src, dr) - _loss(u0, t, h, minus, L, dt, N, src, dr)) / (2 * eps)
            else:
                fd = (_loss(u0, t, h, D, plus, dt, N, src, dr) - _loss(u0, t, h, D, minus, dt, N, src, dr)) / (2 * eps)
            assert abs(grad[s] - fd) <= 1e-6 * abs(fd) + 1e-12, (which, s, grad[s], fd)
    direc = rng.random(u0.shape) - 0.5
    eps = 1e-6
    fd = (_loss(u0 + eps * direc, t, h, D, L, dt, N, src, dr)
          - _loss(u0 - eps * direc, t, h, D, L, dt, N, src, dr)) / (2 * eps)
    assert abs(np.sum(g0 * direc) - fd) <= 1e-6 * abs(fd)


def test_eigenmode_closed_form_gradients():
    nx, ny, nz = 10, 7, 12
    kx, ky, kz = 3, 2, 5
    cx = np.cos(np.pi * kx * (np.arange(nx) + 0.5) / nx)
    cy = np.cos(np.pi * ky * (np.arange(ny) + 0.5) / ny)
    cz = np.cos(np.pi * kz * (np.arange(nz) + 0.5) / nz)
    u0 = (cz[:, None, None] * cy[None, :, None] * cx[None, None, :])[..., None].copy()
    h = np.array([10.0, 14.0, 9.0])
    # moderate decay, so that rounding noise in the other modes stays far below the mode
    D = np.array([3e2])
    Lam = np.array([0.4])
    dt = 0.03
    N = 5
    Lval, uN, g0, gD, gL = oracle.run_with_gradient(u0, np.zeros_like(u0), h, D, Lam, dt, N)
    beta = dt * Lam[0] / 3.0
    mus, sins, rs = [], [], []
    for n, k, a in ((nx, kx, 0), (ny, ky, 1), (nz, kz, 2)):
        r = dt * D[0] / h[a] ** 2
        s2 = 4.0 * np.sin(np.pi * k / (2.0 * n)) ** 2
        mus.append(1.0 + beta + r * s2)
        sins.append(s2)
    Lref = np.sum(u0 ** 2) * np.prod([m ** (-2 * N) for m in mus])
    assert abs(Lval - Lref) <= 1e-12 * Lref
    dL_dr = [-2 * N * Lref * sins[a] / mus[a] for a in range(3)]
    dL_dbeta = -2 * N * Lref * sum(1.0 / m for m in mus)
    gD_ref = sum(dL_dr[a] * dt / h[a] ** 2 for a in range(3))
    gL_ref = dL_dbeta * dt / 3.0
    assert abs(gD[0] - gD_ref) <= 1e-12 * abs(gD_ref)
    assert abs(gL[0] - gL_ref) <= 1e-12 * abs(gL_ref)
    g_ref = 2.0 * uN * np.prod([m ** (-N) for m in mus])
    assert np.max(np.abs(g0 - g_ref)) <= 1e-12 * np.max(np.abs(g_ref))


@pytest.mark.parametrize("K", [1, 2, 3, 10])
def test_checkpointing_does_not_change_gradients(K):
    rng = np.random.default_rng(24)
    u0, h, D, L, dt, src, dr = _setup(rng)
    t = rng.random(u0.shape)
    ref = oracle.run_with_gradient(u0, t, h, D, L, dt, 7, src, dr, checkpoint_every=1)
    got = oracle.run_with_gradient(u0, t, h, D, L, dt, 7, src, dr, checkpoint_every=K)
    for a, b in zip(ref[2:], got[2:]):
        assert np.array_equal(a, b)
