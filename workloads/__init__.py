"""Seeded synthetic inputs for the diffusion-decay workloads.

This module only generates inputs (fields, coefficients, source and Dirichlet
lists, targets, batch shapes).  It holds none of the method's arithmetic and
is the one piece shared by the oracle side and the GPU side of the tests and
of the benchmark.

Random numbers: counter-based SplitMix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), keyed as
    key(seed, stream, i) = mix(mix(seed ^ (stream << 56)) ^ i)
and turned into a double in [0, 1) as (key >> 11) * 2^-53.  Streams:
0 field, 1 coefficients, 2 source voxels, 3 Dirichlet, 4 target, 5 FD
direction, 6 batch shapes, 7 secretion rates, 8 uptake rates.

Workload shapes follow the paper's benchmark cubes (Table 1: cubic domains at
10 um resolution, 1-8 substrates; the 8% liver case is 1000^3 x 4) and its
end-to-end run (Sec. 5.3: Gaussian initial profile, source and sink cells).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import List, Optional

import numpy as np

MASK64 = (1 << 64) - 1
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

_HERE = os.path.dirname(os.path.abspath(__file__))
_CSRC = os.path.join(_HERE, "splitmix.c")
_CLIB = os.path.join(_HERE, "libsplitmix.so")
_clib = None


def mix64_int(x: int) -> int:
    """SplitMix64 output function on a Python int (reference for the vector forms)."""
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def _mix64(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = z + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> int:
    return mix64_int((seed ^ (stream << 56)) & MASK64)


def keys(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    k0 = np.uint64(stream_key(seed, stream))
    idx = np.arange(start, start + count, dtype=np.uint64)
    return _mix64(idx ^ k0)


def uniform(seed: int, stream: int, count: int, start: int = 0) -> np.ndarray:
    """count doubles in [0, 1) for indices start..start+count-1."""
    k = keys(seed, stream, start, count)
    return (k >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def build(cc: str = "gcc") -> str:
    tmp = _CLIB + ".tmp%d" % os.getpid()
    subprocess.run([cc, "-O2", "-fopenmp", "-std=c99", "-shared", "-fPIC", "-o", tmp, _CSRC],
                   check=True)
    os.replace(tmp, _CLIB)
    return _CLIB


def _c():
    global _clib
    if _clib is None:
        if not os.path.exists(_CLIB) or os.path.getmtime(_CLIB) < os.path.getmtime(_CSRC):
            build()
        lib = ctypes.CDLL(_CLIB)
        lib.splitmix_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                         ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_void_p]
        lib.splitmix_uniform.restype = None
        _clib = lib
    return _clib


def uniform_fill(out: np.ndarray, seed: int, stream: int, lo: float = 0.0, hi: float = 1.0,
                 start: int = 0) -> np.ndarray:
    """Fill a C-contiguous float64 array with lo + (hi-lo)*U[0,1) (multi-threaded C)."""
    assert out.dtype == np.float64 and out.flags.c_contiguous
    _c().splitmix_uniform(stream_key(seed, stream), 0, start, out.size, lo, hi,
                          out.ctypes.data_as(ctypes.c_void_p))
    return out


# ----------------------------------------------------------------- inputs


@dataclasses.dataclass
class SourceList:
    voxel: np.ndarray        # int64 [count], flat (z*ny + y)*nx + x
    secretion: np.ndarray    # float64 [count, S]
    saturation: np.ndarray   # float64 [count, S]
    uptake: np.ndarray       # float64 [count, S]

    def __len__(self):
        return int(self.voxel.shape[0])


@dataclasses.dataclass
class DirichletList:
    voxel: np.ndarray        # int64 [count]
    value: np.ndarray        # float64 [count, S]
    active: np.ndarray       # uint8 [count, S]

    def __len__(self):
        return int(self.voxel.shape[0])


@dataclasses.dataclass
class Problem:
    name: str
    nx: int
    ny: int
    nz: int
    S: int
    h: np.ndarray            # (hx, hy, hz) um
    D: np.ndarray            # [S] um^2/min
    lam: np.ndarray          # [S] 1/min
    dt: float                # min
    nsteps: int
    seed: int
    src: Optional[SourceList] = None
    dr: Optional[DirichletList] = None
    u0: Optional[np.ndarray] = None   # [nz, ny, nx, S] float64 (None: generate lazily)
    u0_kind: str = "uniform"          # "uniform" or "gaussian"
    dtype: str = "f64"
    gauss_sigma: float = 8.0          # Gaussian profile: sigma (voxels) and noise amplitude
    gauss_noise: float = 0.01

    @property
    def V(self):
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx, self.S)

    def field(self) -> np.ndarray:
        if self.u0 is None:
            self.u0 = make_field(self)
        return self.u0


def distinct_voxels(seed: int, stream: int, V: int, count: int) -> np.ndarray:
    """count distinct voxels: key mod V in index order, later repeats skipped."""
    if count > V:
        raise ValueError("more distinct voxels requested than the grid has")
    out = np.empty(0, dtype=np.int64)
    start = 0
    while out.size < count:
        n = max(2 * (count - out.size), 1024)
        cand = (keys(seed, stream, start, n) % np.uint64(V)).astype(np.int64)
        start += n
        allc = np.concatenate([out, cand])
        _, first = np.unique(allc, return_index=True)
        first.sort()
        out = allc[first]
    return out[:count]


def make_sources(seed: int, V: int, S: int, count: int) -> SourceList:
    """Secretion ~ U[0,10], saturation density 1.0, uptake ~ U[0,10] per (voxel, substrate)."""
    vox = distinct_voxels(seed, 2, V, count)
    sec = 10.0 * uniform(seed, 7, count * S).reshape(count, S)
    upt = 10.0 * uniform(seed, 8, count * S).reshape(count, S)
    sat = np.ones((count, S))
    return SourceList(vox, sec, sat, upt)


def make_field(p: Problem) -> np.ndarray:
    nz, ny, nx, S = p.shape
    if p.u0_kind == "gaussian":
        # Gaussian blob (sigma 8 voxels unless set), peak 1 at the centre
        # (voxel-centre coordinates i + 1/2), plus noise * U[0,1) (0.01 unless set)
        sig = p.gauss_sigma
        cz, cy, cx = nz / 2.0, ny / 2.0, nx / 2.0
        z = (np.arange(nz) + 0.5 - cz)[:, None, None]
        y = (np.arange(ny) + 0.5 - cy)[None, :, None]
        x = (np.arange(nx) + 0.5 - cx)[None, None, :]
        g = np.exp(-(x * x + y * y + z * z) / (2.0 * sig * sig))
        u = np.repeat(g[..., None], S, axis=3)
        if p.gauss_noise:
            u += p.gauss_noise * uniform(p.seed, 0, u.size).reshape(u.shape)
        return np.ascontiguousarray(u)
    u = np.empty(p.shape, dtype=np.float64)
    if u.size > (1 << 22):
        uniform_fill(u, p.seed, 0)
    else:
        u[...] = uniform(p.seed, 0, u.size).reshape(p.shape)
    return u


def random_coefficients(seed: int, S: int, log10_D=(2.0, 5.0), lam=(0.01, 1.0)):
    """D_s log-uniform on [10^a, 10^b], lambda_s uniform on [lo, hi] (stream 1)."""
    w = uniform(seed, 1, 2 * S)
    D = 10.0 ** (log10_D[0] + (log10_D[1] - log10_D[0]) * w[:S])
    L = lam[0] + (lam[1] - lam[0]) * w[S:]
    return D, L


def config(k: int, *, n: Optional[int] = None, nsub: Optional[int] = None,
           n_sources: Optional[int] = None, nsteps: Optional[int] = None,
           with_field: bool = True) -> Problem:
    """Workload k (1..4) at full size, or scaled down by overriding n (cube side),
    nsub, n_sources or nsteps while keeping the same recipe."""
    seed = 1000 + k
    if k == 1:
        side = n or 64
        S = nsub or 1
        p = Problem("gaussian-64^3x1-f64", side, side, side, S, np.array([20.0] * 3),
                    np.full(S, 1.0e5), np.full(S, 0.1), 0.01, nsteps or 10, seed,
                    u0_kind="gaussian")
    elif k == 2:
        side = n or 256
        S = nsub or 8
        D, L = random_coefficients(seed, S, (2.0, 5.0), (0.01, 1.0))
        p = Problem("cells-256^3x8-f64", side, side, side, S, np.array([10.0] * 3), D, L, 0.01,
                    nsteps or 100, seed)
        V = side ** 3
        p.src = make_sources(seed, V, S, min(n_sources if n_sources is not None else 100_000, V))
        # 8x8 block of Dirichlet voxels on the x = 0 face, centred, substrate 0 at 38.0
        c = side // 2
        lo = max(c - 4, 0)
        hi = min(lo + 8, side)
        ys = np.arange(lo, hi)
        zs = np.arange(lo, hi)
        zz, yy = np.meshgrid(zs, ys, indexing="ij")
        vox = ((zz * side + yy) * side + 0).reshape(-1).astype(np.int64)
        val = np.zeros((vox.size, S))
        act = np.zeros((vox.size, S), dtype=np.uint8)
        val[:, 0] = 38.0
        act[:, 0] = 1
        p.dr = DirichletList(vox, val, act)
    elif k == 3:
        side = n or 1000
        S = nsub or 4
        D, L = random_coefficients(seed, S, (3.0, 5.0), (0.01, 0.1))
        p = Problem("liver8pct-1000^3x4-f64", side, side, side, S, np.array([10.0] * 3), D, L,
                    0.01, nsteps or 20, seed)
        V = side ** 3
        p.src = make_sources(seed, V, S, min(n_sources if n_sources is not None else 1_000_000, V))
    elif k == 4:
        side = n or 128
        S = nsub or 2
        D, L = random_coefficients(seed, S, (2.0, 5.0), (0.01, 1.0))
        p = Problem("adjoint-128^3x2", side, side, side, S, np.array([10.0] * 3), D, L, 0.01,
                    nsteps or 50, seed)
        if n_sources:
            V = side ** 3
            p.src = make_sources(seed, V, S, min(n_sources, V))
    else:
        raise ValueError("config k must be 1..4 (batches: batch_config)")
    if with_field:
        p.field()
    return p


def endtoend_config(nsteps: int = 500, with_field: bool = True) -> Problem:
    """The paper's end-to-end run (Sec. 5.3): a 5 mm cube at 10 um (500^3), one
    substrate, a Gaussian initial profile, 500 bulk-source agents and 500
    uptake-sink agents in distinct seeded voxels, 500 steps of 0.01 min.
    Unstated values chosen here: D = 1e5 um^2/min, lambda = 0.1 /min (the
    64^3 case's), sigma = 62.5 voxels (1/8 of the side, as 8 of 64), no
    noise, sources secrete 10 /min towards saturation 1, sinks take up
    10 /min."""
    side, seed = 500, 1010
    p = Problem("endtoend-500^3x1", side, side, side, 1, np.array([10.0] * 3), np.array([1.0e5]),
                np.array([0.1]), 0.01, nsteps, seed, u0_kind="gaussian", gauss_sigma=side / 8.0, gauss_noise=0.0)
    vox = distinct_voxels(seed, 2, p.V, 1000)
    sec = np.zeros((1000, 1))
    upt = np.zeros((1000, 1))
    sec[:500, 0] = 10.0          # bulk sources
    upt[500:, 0] = 10.0          # uptake sinks
    p.src = SourceList(vox, sec, np.ones((1000, 1)), upt)
    if with_field:
        p.field()
    return p


# Table 1 cases beyond the 1000^3 x 4 cube, at 10 um: (side, substrates, storage)
LARGE_CASES = {
    "liver4": (500, 2, "f64"),      # "4% liver": 500^3 x 2, 2 GB in FP64 (the paper's one-node case)
    "liver12": (1500, 8, "f64"),    # "12.5% liver": 1500^3 x 8, 216 GB in FP64
    "liver16": (2000, 8, "f32"),    # "16.6% liver": 2000^3 x 8, 256 GB in FP32 (512 GB in FP64)
}


def large_config(name: str, n_sources: int = 1_000_000, nsteps: int = 5) -> Problem:
    """A Table 1 cube with the tumour-scale recipe (D log-uniform in [1e3, 1e5],
    lambda in [0.01, 0.1], dt = 0.01, distinct source voxels with the 256^3
    workload's rates).  No host field: the field is written on the device
    with the same seeded uniform stream (seed, stream 0)."""
    side, S, dtype = LARGE_CASES[name]
    seed = 1100 + side // 100
    D, L = random_coefficients(seed, S, (3.0, 5.0), (0.01, 0.1))
    p = Problem(f"{name}-{side}^3x{S}-{dtype}", side, side, side, S, np.array([10.0] * 3), D, L, 0.01,
                nsteps, seed, dtype=dtype)
    p.src = make_sources(seed, p.V, S, n_sources)
    return p


def target_field(p: Problem) -> np.ndarray:
    return uniform(p.seed, 4, int(np.prod(p.shape))).reshape(p.shape)


def direction_field(p: Problem) -> np.ndarray:
    return uniform(p.seed, 5, int(np.prod(p.shape))).reshape(p.shape) - 0.5


def dirichlet_variant(p: Problem, count: int = 16) -> DirichletList:
    """count seeded distinct Dirichlet voxels, all substrates active, values U[0,1) (stream 3)."""
    vox = distinct_voxels(p.seed, 3, p.V, count)
    val = uniform(p.seed, 3, count * p.S, start=1 << 40).reshape(count, p.S)
    act = np.ones((count, p.S), dtype=np.uint8)
    return DirichletList(vox, val, act)


def batch_config(n_domains: int = 96, lo: int = 24, hi: int = 192, max_sub: int = 8,
                 source_fraction: float = 0.01, nsteps: int = 100, seed: int = 1005,
                 with_field: bool = True) -> List[Problem]:
    """Uneven independent domains: each axis ~ U{lo..hi}, S ~ U{1..max_sub},
    dtype by a seeded coin, D/lambda as the 256^3 workload, dt ~ U[0.01, 0.1],
    source_fraction of the voxels as source/sink cells."""
    probs = []
    w = uniform(seed, 6, 6 * n_domains).reshape(n_domains, 6)
    for d in range(n_domains):
        nx, ny, nz = (lo + np.minimum((w[d, :3] * (hi - lo + 1)).astype(int), hi - lo))
        S = 1 + min(int(w[d, 3] * max_sub), max_sub - 1)
        dtype = "f32" if w[d, 4] < 0.5 else "f64"
        dt = 0.01 + 0.09 * w[d, 5]
        dseed = (seed << 16) + d + 1
        D, L = random_coefficients(dseed, S, (2.0, 5.0), (0.01, 1.0))
        p = Problem(f"domain{d}", int(nx), int(ny), int(nz), S, np.array([10.0] * 3), D, L, dt,
                    nsteps, dseed, dtype=dtype)
        nsrc = int(round(source_fraction * p.V))
        if nsrc > 0:
            p.src = make_sources(dseed, p.V, S, nsrc)
        if with_field:
            p.field()
        probs.append(p)
    return probs
