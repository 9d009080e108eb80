"""Plain FP64 CPU oracle of the BioFVM-B diffusion-decay step (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The GPU library and its Python
binding never import, link or call anything in this package.

The arithmetic lives in ``bfvm_oracle.c`` (plain C, IEEE double, divisions as
divisions, ``-ffp-contract=off``); this module compiles it with gcc and
marshals numpy arrays through ctypes.  ``dense.py`` is an independent
brute-force checker (explicit Kronecker operators + LAPACK solves) used to pin
the C oracle on tiny grids.

Paper anchors: LOD step and 7-stage structure (Sec. 2), Thomas algorithm and
operation count (Sec. 2.1, Eqs. 1-3), precomputed coefficients (App. A),
production/uptake by cells (Sec. 5.3).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bfvm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_f64p = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double


def build(cc: str = "gcc") -> str:
    """Compile liboracle.so (plain -O2, OpenMP across independent lines, no FMA contraction)."""
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = [cc, "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
           "-shared", "-fPIC", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("BFVM_ORACLE_LIB")  # a planted-mistake build, used by the mutation test
    if not path:
        path = _LIB
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
    lib = ctypes.CDLL(path)
    lib.oracle_factor.argtypes = [_i64, _dbl, _dbl, _f64p, _f64p]
    lib.oracle_factor.restype = None
    lib.oracle_sweep.argtypes = [_f64p, _i64, _i64, _i64, _i32, _f64p, _f64p, _f64p, _dbl, _i32]
    lib.oracle_source.argtypes = [_f64p, _i32, _i64, _i64p, _f64p, _f64p, _f64p, _dbl]
    lib.oracle_dirichlet.argtypes = [_f64p, _i32, _i64, _i64p, _f64p, _u8p]
    lib.oracle_step.argtypes = [_f64p, _i64, _i64, _i64, _i32, _f64p, _f64p, _f64p, _dbl,
                                _i64, _i64p, _f64p, _f64p, _f64p,
                                _i64, _i64p, _f64p, _u8p, _i64]
    lib.oracle_adjoint_step.argtypes = [_f64p, _f64p, _f64p, _f64p,
                                        _i64, _i64, _i64, _i32, _f64p, _f64p, _f64p, _dbl,
                                        _i64, _i64p, _f64p, _f64p, _f64p,
                                        _i64, _i64p, _f64p, _u8p]
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    for name in ("oracle_sweep", "oracle_source", "oracle_dirichlet", "oracle_step",
                 "oracle_adjoint_step"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def threads() -> int:
    """OpenMP threads the oracle's sweeps run on."""
    return int(_load().oracle_threads())


def set_threads(n: int) -> None:
    """Run the following oracle calls on n OpenMP threads."""
    _load().oracle_set_threads(int(n))


def _p(a, t=_f64p):
    return a.ctypes.data_as(t) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(st, what):
    if st != 0:
        raise RuntimeError(f"oracle {what} failed with status {st}")


def factor(n: int, r: float, beta: float):
    """Thomas factors (denom, c') of the n x n matrix with parameters r, beta (App. A)."""
    lib = _load()
    denom = np.empty(n)
    cprime = np.empty(n)
    lib.oracle_factor(n, r, beta, _p(denom), _p(cprime))
    return denom, cprime


def _grid(u):
    if u.ndim != 4:
        raise ValueError("field must be [nz, ny, nx, S]")
    if u.dtype != np.float64 or not u.flags.c_contiguous:
        raise ValueError("field must be a C-contiguous float64 array")
    nz, ny, nx, S = u.shape
    return nx, ny, nz, S


class Sources:
    """Bulk source/sink list: voxel[count] (flat (z*ny+y)*nx+x), rates [count, S]."""

    def __init__(self, voxel, secretion, saturation, uptake):
        self.voxel = np.ascontiguousarray(voxel, dtype=np.int64)
        self.secretion = _f64(secretion)
        self.saturation = _f64(saturation)
        self.uptake = _f64(uptake)

    def __len__(self):
        return int(self.voxel.shape[0])


class Dirichlet:
    """Dirichlet list: voxel[count], value [count, S], active [count, S] (uint8)."""

    def __init__(self, voxel, value, active):
        self.voxel = np.ascontiguousarray(voxel, dtype=np.int64)
        self.value = _f64(value)
        self.active = np.ascontiguousarray(active, dtype=np.uint8)

    def __len__(self):
        return int(self.voxel.shape[0])


def _src_args(src):
    if src is None or len(src) == 0:
        return (0, None, None, None, None)
    return (len(src), _p(src.voxel, _i64p), _p(src.secretion), _p(src.saturation), _p(src.uptake))


def _dir_args(dr):
    if dr is None or len(dr) == 0:
        return (0, None, None, None)
    return (len(dr), _p(dr.voxel, _i64p), _p(dr.value), _p(dr.active, _u8p))


def sweep(u, h, D, lam, dt, axis):
    """One sweep along axis (0=x, 1=y, 2=z), in place on u [nz, ny, nx, S]."""
    lib = _load()
    nx, ny, nz, S = _grid(u)
    h, D, lam = _f64(h), _f64(D), _f64(lam)
    _check(lib.oracle_sweep(_p(u), nx, ny, nz, S, _p(h), _p(D), _p(lam), dt, axis), "sweep")
    return u


def source(u, src, dt):
    lib = _load()
    nx, ny, nz, S = _grid(u)
    n, v, se, sa, up = _src_args(src)
    _check(lib.oracle_source(_p(u), S, n, v, se, sa, up, dt), "source")
    return u


def dirichlet(u, dr):
    lib = _load()
    nx, ny, nz, S = _grid(u)
    n, v, val, act = _dir_args(dr)
    _check(lib.oracle_dirichlet(_p(u), S, n, v, val, act), "dirichlet")
    return u


def step(u, h, D, lam, dt, src=None, dr=None, nsteps=1):
    """nsteps LOD steps (Src, Dir, X, Dir, Y, Dir, Z, Dir), in place on u."""
    lib = _load()
    nx, ny, nz, S = _grid(u)
    h, D, lam = _f64(h), _f64(D), _f64(lam)
    st = lib.oracle_step(_p(u), nx, ny, nz, S, _p(h), _p(D), _p(lam), dt,
                         *_src_args(src), *_dir_args(dr), nsteps)
    _check(st, "step")
    return u


def adjoint_step(u_in, g, gD, gL, h, D, lam, dt, src=None, dr=None):
    """Reverse of one step started from u_in: g <- (dstep/du)^T g (in place);
    gD, gL [S] are incremented by the step's contribution to dL/dD, dL/dlambda."""
    lib = _load()
    nx, ny, nz, S = _grid(u_in)
    _grid(g)
    h, D, lam = _f64(h), _f64(D), _f64(lam)
    st = lib.oracle_adjoint_step(_p(u_in), _p(g), _p(gD), _p(gL), nx, ny, nz, S,
                                 _p(h), _p(D), _p(lam), dt, *_src_args(src), *_dir_args(dr))
    _check(st, "adjoint_step")
    return g


def run_with_gradient(u0, target, h, D, lam, dt, nsteps, src=None, dr=None, checkpoint_every=None):
    """Forward nsteps from u0, loss L = sum (u_N - target)^2, and the reverse
    sweep.  Returns (L, u_N, dL/du0, dL/dD, dL/dlambda).  With checkpoint_every
    = K only every K-th state is kept and the rest recomputed."""
    S = u0.shape[-1]
    K = checkpoint_every or 1
    u = np.array(u0, dtype=np.float64, copy=True)
    ckpt = {}
    for t in range(nsteps):
        if t % K == 0:
            ckpt[t] = u.copy()
        step(u, h, D, lam, dt, src, dr, 1)
    uN = u.copy()
    diff = uN - target
    L = float(np.sum(diff * diff))
    g = 2.0 * diff
    gD = np.zeros(S)
    gL = np.zeros(S)
    for seg0 in sorted(ckpt.keys(), reverse=True):
        seg1 = min(seg0 + K, nsteps)
        states = [ckpt[seg0].copy()]
        for t in range(seg0, seg1 - 1):
            w = states[-1].copy()
            step(w, h, D, lam, dt, src, dr, 1)
            states.append(w)
        for t in range(seg1 - 1, seg0 - 1, -1):
            adjoint_step(states[t - seg0], g, gD, gL, h, D, lam, dt, src, dr)
    return L, uN, g, gD, gL
