"""Python binding of the gfx950 diffusion-decay library (libbfvm.so).

Argument marshalling only: every stage of the LOD step (source/sink,
Dirichlet, x/y/z Thomas sweeps, their transposes) runs in the HIP kernels
behind the C ABI declared in ``include/bfvm.h``.  PyTorch provides device
memory (field tensors) and streams.  There is no CPU fallback: if the library
is not built, loading it raises.

Field tensors are contiguous CUDA tensors of shape [nz, ny, nx, S] with
dtype float64 (``"f64"``) or float32 (``"f32"``, ``"f32fast"``); element
((z*ny + y)*nx + x)*S + s, substrate innermost (Sec. 3.1 contiguous density
array).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbfvm.so")

F64, F32, F32_FAST = 0, 1, 2
DTYPES = {"f64": F64, "f32": F32, "f32fast": F32_FAST}
STATUS = {0: "OK", -1: "EINVAL", -2: "ERANGE", -3: "ESTATE", -4: "EDEVICE", -5: "ENOMEM", -6: "EOFF", -7: "EIO"}

# every entry point declared in include/bfvm.h
EXPORTS = [
    "bfvm_create", "bfvm_destroy", "bfvm_set_stream", "bfvm_set_params", "bfvm_set_sources",
    "bfvm_set_dirichlet", "bfvm_step", "bfvm_sweep", "bfvm_xslab_forward", "bfvm_xslab_backward",
    "bfvm_step_adjoint", "bfvm_step_adjoint_noalloc",
    "bfvm_read_field",
    "bfvm_save_npy", "bfvm_load_npy",
    "bfvm_fill_uniform", "bfvm_fill_gaussian", "bfvm_device_bytes",
    "bfvm_timing_enable", "bfvm_timing_read", "bfvm_timing_reset", "bfvm_timing_elements",
    "bfvm_set_schedule", "bfvm_get_schedule", "bfvm_get_plan", "bfvm_set_plan", "bfvm_autotune",
    "bfvm_field_alloc", "bfvm_field_free",
    "bfvm_batch_create", "bfvm_batch_destroy", "bfvm_batch_set_mode", "bfvm_batch_set_fields", "bfvm_batch_step",
    "bfvm_batch_step_eager", "bfvm_batch_step_adjoint", "bfvm_batch_autotune", "bfvm_batch_get_plan",
    "bfvm_batch_set_plan",
    "bfvm_batch_info",
    "bfvm_status_string", "bfvm_last_error", "bfvm_version",
]

_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double
_f64p = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)


class BfvmError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str):
        self.status = status
        self.code = STATUS.get(status, str(status))
        super().__init__(f"{what}: {self.code} ({detail})")


def lib():
    """Load libbfvm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                          f"python paper_2602_05017_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    L.bfvm_create.argtypes = [ctypes.POINTER(_vp), _i64, _i64, _i64, _i32, _dbl, _dbl, _dbl, _i32, _vp]
    L.bfvm_destroy.argtypes = [_vp]
    L.bfvm_set_stream.argtypes = [_vp, _vp]
    L.bfvm_set_params.argtypes = [_vp, _f64p, _f64p, _dbl]
    L.bfvm_set_sources.argtypes = [_vp, _i64, _i64p, _f64p, _f64p, _f64p]
    L.bfvm_set_dirichlet.argtypes = [_vp, _i64, _i64p, _f64p, _u8p]
    L.bfvm_step.argtypes = [_vp, _vp, _i64]
    L.bfvm_sweep.argtypes = [_vp, _vp, _i32]
    L.bfvm_xslab_forward.argtypes = [_vp, _vp, _i64, _i64, _i64, _i64, _vp, _vp]
    L.bfvm_xslab_backward.argtypes = [_vp, _vp, _i64, _i64, _i64, _i64, _vp, _vp]
    L.bfvm_step_adjoint.argtypes = [_vp, _vp, _vp, _f64p, _f64p]
    L.bfvm_step_adjoint_noalloc.argtypes = [_vp, _vp, _vp, _f64p, _f64p]
    L.bfvm_read_field.argtypes = [_vp, _vp, _vp]
    L.bfvm_save_npy.argtypes = [_vp, _vp, ctypes.c_char_p]
    L.bfvm_load_npy.argtypes = [_vp, _vp, ctypes.c_char_p]
    L.bfvm_timing_enable.argtypes = [_vp, _i32]
    L.bfvm_timing_read.argtypes = [_vp, _i32, _f64p, _i64p]
    L.bfvm_timing_reset.argtypes = [_vp]
    L.bfvm_timing_elements.argtypes = [_vp, _i32, _i64p]
    L.bfvm_set_schedule.argtypes = [_vp, _i32, _i64]
    L.bfvm_get_schedule.argtypes = [_vp, _i32p, _i64p]
    L.bfvm_get_plan.argtypes = [_vp, _i32, _i32p, _i32p, _i32p, _i32p]
    L.bfvm_set_plan.argtypes = [_vp, _i32, _i32, _i32, _i32, _i32]
    L.bfvm_autotune.argtypes = [_vp, _vp, _i32, ctypes.POINTER(ctypes.c_float)]
    L.bfvm_field_alloc.argtypes = [_vp, _i32, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_float)]
    L.bfvm_field_free.argtypes = [_vp]
    L.bfvm_batch_create.argtypes = [ctypes.POINTER(_vp), _i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp]
    L.bfvm_batch_destroy.argtypes = [_vp]
    L.bfvm_batch_set_fields.argtypes = [_vp, _i32, ctypes.POINTER(_vp)]
    L.bfvm_batch_step.argtypes = [_vp, _i64]
    L.bfvm_batch_step_eager.argtypes = [_vp, _i64]
    L.bfvm_batch_step_adjoint.argtypes = [_vp, _i32, _i32p, _f64p, _f64p]
    L.bfvm_batch_autotune.argtypes = [_vp, ctypes.c_char_p, _f64p]
    L.bfvm_batch_get_plan.argtypes = [_vp, _i32, _i32, _i32p, _i32p]
    L.bfvm_batch_set_plan.argtypes = [_vp, _i32, _i32, _i32, _i32]
    L.bfvm_batch_info.argtypes = [_vp, _i64p, _i32p, _i64p]
    L.bfvm_status_string.argtypes = [ctypes.c_int]
    L.bfvm_status_string.restype = ctypes.c_char_p
    L.bfvm_last_error.argtypes = []
    L.bfvm_last_error.restype = ctypes.c_char_p
    L.bfvm_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        fn = getattr(L, name)
        if fn.restype is ctypes.c_int or name not in ("bfvm_status_string", "bfvm_last_error", "bfvm_version"):
            fn.restype = ctypes.c_int
    _lib = L
    return L


def last_error() -> str:
    return lib().bfvm_last_error().decode()


def _check(status: int, what: str):
    if status != 0:
        raise BfvmError(status, what, last_error())


def _f64arr(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _ptr(a, t=_f64p):
    return a.ctypes.data_as(t) if a is not None and a.size else None


def _current_stream():
    import torch
    if not torch.cuda.is_available():
        return None    # no device: every call fails validation or reports EDEVICE
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class _FieldBuffer:
    """Owner of a bfvm_field_alloc allocation, exposed to torch through the
    CUDA array interface; torch keeps a reference for the tensor's lifetime,
    and the memory is freed when the last reference goes."""

    def __init__(self, ptr: int, shape, typestr: str):
        self.ptr = ptr
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (ptr, False),
                                         "strides": None, "version": 2}

    def __del__(self):
        try:
            if self.ptr:
                lib().bfvm_field_free(_vp(self.ptr))
        except Exception:
            pass
        self.ptr = 0


class Grid:
    """nx*ny*nz voxels x nsub substrates, spacings h (um), storage dtype."""

    def __init__(self, nx: int, ny: int, nz: int, nsub: int, h: Sequence[float] = (10.0, 10.0, 10.0),
                 dtype: str = "f64", stream=None):
        self.nx, self.ny, self.nz, self.nsub = int(nx), int(ny), int(nz), int(nsub)
        self.h = tuple(float(v) for v in h)
        if dtype not in DTYPES:
            raise ValueError(f"dtype must be one of {list(DTYPES)}")
        self.dtype = dtype
        self._handle = _vp()
        _check(lib().bfvm_create(ctypes.byref(self._handle), self.nx, self.ny, self.nz, self.nsub,
                                 self.h[0], self.h[1], self.h[2], DTYPES[dtype],
                                 stream if stream is not None else None), "bfvm_create")
        self._explicit_stream = stream is not None

    # -------------------------------------------------------------- helpers
    @property
    def handle(self):
        return self._handle

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx, self.nsub)

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.dtype == "f64" else torch.float32

    def _sync_stream(self):
        if not self._explicit_stream:
            _check(lib().bfvm_set_stream(self._handle, _current_stream()), "bfvm_set_stream")

    def _field_ptr(self, t):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("field must be a CUDA tensor")
        if t.dtype != self.torch_dtype:
            raise TypeError(f"field dtype {t.dtype} does not match grid dtype {self.dtype}")
        if not t.is_contiguous() or t.numel() != self.nx * self.ny * self.nz * self.nsub:
            raise ValueError("field must be contiguous with nz*ny*nx*nsub elements")
        return ctypes.c_void_p(t.data_ptr())

    def empty_field(self):
        import torch
        return torch.empty(self.shape, dtype=self.torch_dtype, device="cuda")

    def alloc_field(self, candidates: int = 4):
        """A field tensor in device memory whose placement the library chose
        by timing the sweeps on `candidates` allocations (bfvm_field_alloc).
        Returns (tensor, ms per candidate); the memory is released with the
        last reference to the tensor.  Contents are unspecified."""
        import torch
        ptr = _vp()
        ms = (ctypes.c_float * int(candidates))()
        self._sync_stream()
        _check(lib().bfvm_field_alloc(self._handle, int(candidates), ctypes.byref(ptr), ms), "bfvm_field_alloc")
        buf = _FieldBuffer(ptr.value, self.shape, "<f8" if self.dtype == "f64" else "<f4")
        t = torch.as_tensor(buf, device="cuda")
        if t.data_ptr() != ptr.value or tuple(t.shape) != self.shape:
            raise RuntimeError("field tensor does not wrap the allocation")
        return t, [float(x) for x in ms]

    # -------------------------------------------------------------- setup
    def set_params(self, D, lam, dt: float):
        D = _f64arr(D, self.nsub)
        lam = _f64arr(lam, self.nsub)
        self._sync_stream()
        _check(lib().bfvm_set_params(self._handle, _ptr(D), _ptr(lam), float(dt)), "bfvm_set_params")

    def set_sources(self, voxel, secretion, saturation, uptake):
        voxel = np.ascontiguousarray(voxel, dtype=np.int64).reshape(-1)
        n = voxel.size
        sec = _f64arr(secretion, n * self.nsub)
        sat = _f64arr(saturation, n * self.nsub)
        upt = _f64arr(uptake, n * self.nsub)
        self._sync_stream()
        _check(lib().bfvm_set_sources(self._handle, n, _ptr(voxel, _i64p), _ptr(sec), _ptr(sat), _ptr(upt)),
               "bfvm_set_sources")

    def set_dirichlet(self, voxel, value, active):
        voxel = np.ascontiguousarray(voxel, dtype=np.int64).reshape(-1)
        n = voxel.size
        val = _f64arr(value, n * self.nsub)
        act = np.ascontiguousarray(active, dtype=np.uint8).reshape(-1)
        if act.size != n * self.nsub:
            raise ValueError("active must have count*nsub entries")
        self._sync_stream()
        _check(lib().bfvm_set_dirichlet(self._handle, n, _ptr(voxel, _i64p), _ptr(val), _ptr(act, _u8p)),
               "bfvm_set_dirichlet")

    # -------------------------------------------------------------- compute
    def step(self, field, nsteps: int = 1):
        p = self._field_ptr(field)
        self._sync_stream()
        _check(lib().bfvm_step(self._handle, p, int(nsteps)), "bfvm_step")
        return field

    def sweep(self, field, axis: int):
        p = self._field_ptr(field)
        self._sync_stream()
        _check(lib().bfvm_sweep(self._handle, p, int(axis)), "bfvm_sweep")
        return field

    def _slab_args(self, slab, x0, x1, l0, l1, carry_in, carry_out):
        import torch
        for t in (slab, carry_out) + ((carry_in,) if carry_in is not None else ()):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
                raise TypeError("slab and carries must be contiguous CUDA tensors")
        if slab.dtype != self.torch_dtype or slab.numel() != (x1 - x0) * self.ny * self.nz * self.nsub:
            raise ValueError("slab must hold nz*ny*(x1-x0)*nsub elements of the grid's dtype")
        cdt = torch.float32 if self.dtype == "f32fast" else torch.float64
        for t in (carry_out,) + ((carry_in,) if carry_in is not None else ()):
            if t.dtype != cdt or t.numel() < l1 - l0:
                raise ValueError(f"carries must hold l1 - l0 values of {cdt}")
        cin = ctypes.c_void_p(carry_in.data_ptr()) if carry_in is not None else None
        return (ctypes.c_void_p(slab.data_ptr()), int(x0), int(x1), int(l0), int(l1), cin,
                ctypes.c_void_p(carry_out.data_ptr()))

    def xslab_forward(self, slab, x0, x1, l0, l1, carry_in, carry_out):
        """Forward share of the x sweep on slab [x0, x1), lines [l0, l1) (bfvm_xslab_forward)."""
        a = self._slab_args(slab, x0, x1, l0, l1, carry_in, carry_out)
        self._sync_stream()
        _check(lib().bfvm_xslab_forward(self._handle, *a), "bfvm_xslab_forward")

    def xslab_backward(self, slab, x0, x1, l0, l1, carry_in, carry_out):
        """Backward share of the x sweep on slab [x0, x1), lines [l0, l1) (bfvm_xslab_backward)."""
        a = self._slab_args(slab, x0, x1, l0, l1, carry_in, carry_out)
        self._sync_stream()
        _check(lib().bfvm_xslab_backward(self._handle, *a), "bfvm_xslab_backward")

    def step_adjoint(self, field_in, grad, grad_D=None, grad_lambda=None):
        """One reverse step; returns (grad_D, grad_lambda) accumulators (numpy)."""
        pin = self._field_ptr(field_in)
        pg = self._field_ptr(grad)
        gD = np.zeros(self.nsub) if grad_D is None else grad_D
        gL = np.zeros(self.nsub) if grad_lambda is None else grad_lambda
        self._sync_stream()
        _check(lib().bfvm_step_adjoint(self._handle, pin, pg, _ptr(gD), _ptr(gL)), "bfvm_step_adjoint")
        return gD, gL

    def device_bytes(self) -> int:
        """Device memory held by the library for this grid (fields excluded)."""
        b = ctypes.c_int64()
        _check(lib().bfvm_device_bytes(self._handle, ctypes.byref(b)), "bfvm_device_bytes")
        return b.value

    def fill_uniform(self, field, seed: int, stream: int = 0, lo: float = 0.0, hi: float = 1.0):
        """Seeded uniform values in [lo, hi) written on the device (SplitMix64 counter stream)."""
        p = self._field_ptr(field)
        self._sync_stream()
        _check(lib().bfvm_fill_uniform(self._handle, p, ctypes.c_uint64(seed), ctypes.c_uint32(stream),
                                       ctypes.c_double(lo), ctypes.c_double(hi)), "bfvm_fill_uniform")

    def fill_gaussian(self, field, center, sigma: float, peak: float = 1.0, noise: float = 0.0, seed: int = 0,
                      stream: int = 0):
        """Gaussian profile (voxel-centre coordinates) plus noise * U, written on the device.
        center = (cx, cy, cz) in voxel units."""
        p = self._field_ptr(field)
        self._sync_stream()
        cx, cy, cz = (float(c) for c in center)
        _check(lib().bfvm_fill_gaussian(self._handle, p, _dbl(cx), _dbl(cy), _dbl(cz), _dbl(sigma), _dbl(peak),
                                        _dbl(noise), ctypes.c_uint64(seed), ctypes.c_uint32(stream)),
               "bfvm_fill_gaussian")

    def read_field(self, field) -> np.ndarray:
        p = self._field_ptr(field)
        out = np.empty(self.shape, dtype=np.float64 if self.dtype == "f64" else np.float32)
        self._sync_stream()
        _check(lib().bfvm_read_field(self._handle, p, out.ctypes.data_as(_vp)), "bfvm_read_field")
        return out

    def save_npy(self, field, path):
        """Write a device field to a NumPy .npy file (shape (nz, ny, nx, nsub))."""
        p = self._field_ptr(field)
        self._sync_stream()
        _check(lib().bfvm_save_npy(self._handle, p, os.fsencode(str(path))), "bfvm_save_npy")

    def load_npy(self, field, path):
        """Read a NumPy .npy file of this grid's shape and element type into a device field."""
        p = self._field_ptr(field)
        self._sync_stream()
        _check(lib().bfvm_load_npy(self._handle, p, os.fsencode(str(path))), "bfvm_load_npy")

    # -------------------------------------------------------------- plans, timing
    def get_plan(self, axis: int):
        v = [ctypes.c_int32() for _ in range(4)]
        _check(lib().bfvm_get_plan(self._handle, axis, *[ctypes.byref(x) for x in v]), "bfvm_get_plan")
        return tuple(x.value for x in v)

    def set_plan(self, axis: int, kind: int, m: int = 0, w: int = 0, lpw: int = 0):
        _check(lib().bfvm_set_plan(self._handle, axis, kind, m, w, lpw), "bfvm_set_plan")

    def autotune(self, field, reps: int = 3):
        """Time candidate plans on `field` (overwritten) and keep the fastest per axis.
        Returns ([plan per axis], [ms per sweep per axis])."""
        p = self._field_ptr(field)
        self._sync_stream()
        ms = (ctypes.c_float * 3)()
        _check(lib().bfvm_autotune(self._handle, p, reps, ms), "bfvm_autotune")
        return [self.get_plan(a) for a in range(3)], [float(x) for x in ms]

    def set_schedule(self, schedule: int, slab_width: int = 0):
        _check(lib().bfvm_set_schedule(self._handle, schedule, slab_width), "bfvm_set_schedule")

    def get_schedule(self):
        sc = ctypes.c_int32()
        w = ctypes.c_int64()
        _check(lib().bfvm_get_schedule(self._handle, ctypes.byref(sc), ctypes.byref(w)), "bfvm_get_schedule")
        return sc.value, w.value

    def timing_elements(self, stage: int) -> int:
        n = ctypes.c_int64()
        _check(lib().bfvm_timing_elements(self._handle, stage, ctypes.byref(n)), "bfvm_timing_elements")
        return n.value

    def timing(self, enable: bool):
        _check(lib().bfvm_timing_enable(self._handle, 1 if enable else 0), "bfvm_timing_enable")

    def timing_reset(self):
        _check(lib().bfvm_timing_reset(self._handle), "bfvm_timing_reset")

    def timing_read(self, stage: int):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().bfvm_timing_read(self._handle, stage, ctypes.byref(ms), ctypes.byref(n)),
               "bfvm_timing_read")
        return ms.value, n.value

    def close(self):
        if self._handle:
            lib().bfvm_destroy(self._handle)
            self._handle = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


STAGES = {"source": 0, "dirichlet": 1, "x": 2, "y": 3, "z": 4}


BATCH_MODES = {"grouped": 0, "persistent": 1}


class Batch:
    """Many grids stepped together, one graph replay per step.

    grids: configured Grid objects (params, sources, Dirichlet set); fields: their
    CUDA field tensors.  The grids and fields must outlive the batch.  mode:
    "grouped" (one launch per stage over all domains); "persistent" is switched
    off in the library and raises BfvmError (EOFF)."""

    def __init__(self, grids, fields, stream=None, mode="grouped"):
        n = len(grids)
        if n != len(fields) or n == 0:
            raise ValueError("need one field per grid")
        self.grids = list(grids)
        self.fields = list(fields)
        hs = (_vp * n)(*[g.handle for g in grids])
        fs = (_vp * n)(*[g._field_ptr(f) for g, f in zip(grids, fields)])
        self._handle = _vp()
        import torch
        torch.cuda.synchronize()     # the batch runs on its own stream
        _check(lib().bfvm_batch_create(ctypes.byref(self._handle), n, hs, fs, stream), "bfvm_batch_create")
        if mode != "grouped":
            try:
                _check(lib().bfvm_batch_set_mode(self._handle, BATCH_MODES[mode]), "bfvm_batch_set_mode")
            except Exception:
                self.close()
                raise

    def _ptrs(self, tensors):
        n = len(self.grids)
        return (_vp * n)(*[g._field_ptr(t) if t is not None else None for g, t in zip(self.grids, tensors)])

    def set_fields(self, fields):
        self.fields = list(fields)
        _check(lib().bfvm_batch_set_fields(self._handle, 0, self._ptrs(fields)), "bfvm_batch_set_fields")

    def set_grads(self, grads):
        _check(lib().bfvm_batch_set_fields(self._handle, 1, self._ptrs(grads)), "bfvm_batch_set_fields")

    def step(self, nsteps: int = 1, graph: bool = True):
        import torch
        torch.cuda.synchronize()
        fn = lib().bfvm_batch_step if graph else lib().bfvm_batch_step_eager
        _check(fn(self._handle, int(nsteps)), "bfvm_batch_step")

    def step_adjoint(self, subset, grad_D=None, grad_lambda=None):
        import torch
        torch.cuda.synchronize()
        subset = np.ascontiguousarray(subset, dtype=np.int32)
        tot = sum(self.grids[i].nsub for i in subset)
        gD = np.zeros(tot) if grad_D is None else grad_D
        gL = np.zeros(tot) if grad_lambda is None else grad_lambda
        _check(lib().bfvm_batch_step_adjoint(self._handle, subset.size, subset.ctypes.data_as(_i32p),
                                             _ptr(gD), _ptr(gL)), "bfvm_batch_step_adjoint")
        return gD, gL

    def autotune(self, cache_path=None) -> float:
        import torch
        torch.cuda.synchronize()
        ms = ctypes.c_double()
        path = cache_path.encode() if cache_path else None
        _check(lib().bfvm_batch_autotune(self._handle, path, ctypes.byref(ms)), "bfvm_batch_autotune")
        return ms.value

    def plan(self, domain: int, axis: int):
        m, l = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().bfvm_batch_get_plan(self._handle, domain, axis, ctypes.byref(m), ctypes.byref(l)),
               "bfvm_batch_get_plan")
        return m.value, l.value

    def set_plan(self, domain: int, axis: int, m: int, lpw: int):
        _check(lib().bfvm_batch_set_plan(self._handle, domain, axis, m, lpw), "bfvm_batch_set_plan")

    def info(self):
        it, bl, ch = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().bfvm_batch_info(self._handle, ctypes.byref(it), ctypes.byref(bl), ctypes.byref(ch)),
               "bfvm_batch_info")
        return {"items": it.value, "launches": bl.value, "chunk_elems": ch.value}

    def close(self):
        if self._handle:
            lib().bfvm_batch_destroy(self._handle)
            self._handle = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
