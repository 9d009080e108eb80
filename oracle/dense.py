"""Brute-force dense checker for the LOD step on tiny grids (test infrastructure).

TEST INFRASTRUCTURE ONLY, used to pin the C oracle.  Nothing here is shared
with ``bfvm_oracle.c``: the matrices are assembled from the finite-volume flux
form instead of the diagonal formulas, and every sweep is a dense solve
(LAPACK gesv through ``numpy.linalg.solve``) of the whole field.

For one substrate with line length n, the zero-flux finite-volume matrix is
    A = (1 + beta) I + r G^T G,
where G is the (n-1) x n forward-difference matrix (one row per interior face)
and r = dt D / h^2, beta = dt lambda / 3 (Sec. 2 LOD splitting, App. A).  On
the field flattened as (z, y, x) with x fastest the three sweeps are the
Kronecker operators I (x) I (x) A_x, I (x) A_y (x) I and A_z (x) I (x) I.
"""
from __future__ import annotations

import numpy as np


def fv_matrix(n: int, r: float, beta: float) -> np.ndarray:
    """(1+beta) I + r G^T G with G the face-difference operator (zero flux at the ends)."""
    G = np.zeros((max(n - 1, 0), n))
    for f in range(n - 1):
        G[f, f] = -1.0
        G[f, f + 1] = 1.0
    return (1.0 + beta) * np.eye(n) + r * (G.T @ G)


def sweep_operator(shape_zyx, axis: int, r: float, beta: float) -> np.ndarray:
    """Dense V x V matrix of one sweep for one substrate; axis 0=x, 1=y, 2=z."""
    nz, ny, nx = shape_zyx
    Iz, Iy, Ix = np.eye(nz), np.eye(ny), np.eye(nx)
    if axis == 0:
        return np.kron(Iz, np.kron(Iy, fv_matrix(nx, r, beta)))
    if axis == 1:
        return np.kron(Iz, np.kron(fv_matrix(ny, r, beta), Ix))
    return np.kron(fv_matrix(nz, r, beta), np.kron(Iy, Ix))


def source_affine(V, S, dt, src):
    """Per (voxel, substrate): u -> (u + P) / Q with duplicates merged additively."""
    P = np.zeros((V, S))
    Qs = np.zeros((V, S))
    if src is not None:
        for k in range(len(src.voxel)):
            v = int(src.voxel[k])
            P[v] += src.secretion[k] * src.saturation[k]
            Qs[v] += src.secretion[k] + src.uptake[k]
    return dt * P, 1.0 + dt * Qs


def dirichlet_table(V, S, dr):
    """Mask and values after applying the list in order (last active entry wins)."""
    mask = np.zeros((V, S), dtype=bool)
    val = np.zeros((V, S))
    if dr is not None:
        for k in range(len(dr.voxel)):
            v = int(dr.voxel[k])
            for s in range(S):
                if dr.active[k, s]:
                    mask[v, s] = True
                    val[v, s] = dr.value[k, s]
    return mask, val


def step_dense(u, h, D, lam, dt, src=None, dr=None, nsteps=1):
    """Brute-force LOD steps on u [nz, ny, nx, S]; returns a new array."""
    nz, ny, nx, S = u.shape
    V = nx * ny * nz
    P, Q = source_affine(V, S, dt, src)
    mask, val = dirichlet_table(V, S, dr)
    w = np.array(u, dtype=np.float64).reshape(V, S).copy()
    ops = []
    for s in range(S):
        beta = dt * lam[s] / 3.0
        ops.append([sweep_operator((nz, ny, nx), a, dt * D[s] / h[a] ** 2, beta) for a in range(3)])
    for _ in range(nsteps):
        w = (w + P) / Q
        for a in range(3):
            w = np.where(mask, val, w)
            for s in range(S):
                w[:, s] = np.linalg.solve(ops[s][a], w[:, s])
        w = np.where(mask, val, w)
    return w.reshape(nz, ny, nx, S)


def step_matrix(shape_zyx, h, D_s, lam_s, dt, mask_s=None, Q_s=None):
    """Linear part M of one step for one substrate (Dirichlet values set to 0):
    u_next = M u + (affine terms).  Used for dense adjoint checks."""
    nz, ny, nx = shape_zyx
    V = nx * ny * nz
    beta = dt * lam_s / 3.0
    Mk = np.diag(1.0 / Q_s) if Q_s is not None else np.eye(V)
    keep = np.diag((~mask_s).astype(float)) if mask_s is not None else np.eye(V)
    for a in range(3):
        A = sweep_operator(shape_zyx, a, dt * D_s / h[a] ** 2, beta)
        Mk = np.linalg.solve(A, keep @ Mk)
    return keep @ Mk
