"""Python binding of the fftb C ABI (include/fftb.h): argument marshalling only.

Every step of the transform runs in the HIP kernels of libfftb.so; this module
only converts Python/torch arguments to pointers and sizes. PyTorch supplies
device memory and streams. The library must be built (paper_2406_05577_amd.build);
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; FFTB_LIB may name another build of the same library
LIB_PATH = os.environ.get("FFTB_LIB") or os.path.join(_PKG, "libfftb.so")

FFTB_OK = 0
FFTB_ERR_INVALID = -1
FFTB_ERR_UNSUPPORTED = -2
FFTB_ERR_NOMEM = -3
FFTB_ERR_HIP = -4

FFTB_C128 = 0
FFTB_C64 = 1

PLAN_PLAIN = 0
PLAN_BATCHED = 1
PLAN_AUTOTUNE = 2
PLAN_GRAPH = 4
PLAN_HOST_ONLY = 8
PLAN_MFMA = 16

EXPORTS = [
    "fftb_plan_create", "fftb_sphere_to_grid", "fftb_grid_to_sphere", "fftb_plan_get_info",
    "fftb_plan_workspace_size", "fftb_plan_sphere_stats", "fftb_plan_sphere_columns",
    "fftb_plan_destroy", "fftb_status_string", "fftb_last_error",
    "fftb_plan_set_profiling", "fftb_plan_get_profile", "fftb_apply_potential",
    "fftb_plan_create_cuboid", "fftb_sphere_to_grid_static",
]


class Sphere_t(C.Structure):
    _fields_ = [("n_coeffs", C.c_int64), ("map", C.POINTER(C.c_int32)),
                ("kpt", C.c_double * 3), ("nbands", C.c_int32)]


DIR_FIELDS = ["band_chunk", "y_classes", "x_rows", "col_tile", "threads", "path", "acc", "splits",
              "lanes"]


class DirTuning_t(C.Structure):
    _fields_ = [(f, C.c_int32) for f in DIR_FIELDS]


class Tuning_t(C.Structure):
    _fields_ = [("inv", DirTuning_t), ("fwd", DirTuning_t)]


def make_tuning(d: dict) -> Tuning_t:
    """Flat dict -> per-direction struct: plain keys set both directions,
    inv_<key> / fwd_<key> set one; acc and splits apply to the forward."""
    t = Tuning_t()
    for k, v in d.items():
        if k.startswith("inv_") or k.startswith("fwd_"):
            continue
        if k not in DIR_FIELDS:
            raise KeyError(f"unknown tuning key {k}")
        if k not in ("acc", "splits"):
            setattr(t.inv, k, int(v))
        setattr(t.fwd, k, int(v))
    for k, v in d.items():
        for pre, part in (("inv_", t.inv), ("fwd_", t.fwd)):
            if k.startswith(pre):
                key = k[len(pre):]
                if key not in DIR_FIELDS:
                    raise KeyError(f"unknown tuning key {k}")
                setattr(part, key, int(v))
    return t


class Info_t(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("nspheres", C.c_int32), ("dtype", C.c_int32),
                ("flags", C.c_uint32), ("total_coeffs", C.c_int64), ("sphere_elems", C.c_int64),
                ("grid_elems", C.c_int64), ("total_columns", C.c_int64),
                ("max_columns", C.c_int32), ("max_slab", C.c_int32),
                ("workspace_bytes", C.c_int64), ("radix_x", C.c_int32 * 8),
                ("radix_y", C.c_int32 * 8), ("radix_z", C.c_int32 * 8), ("tuning", Tuning_t),
                ("autotuned", C.c_int32)]


class Profile_t(C.Structure):
    _fields_ = [("launches", C.c_int64 * 5), ("total_ms", C.c_double * 5)]


KERNEL_NAMES = ["column_inverse", "plane_inverse", "plane_forward", "column_forward",
                "combine_forward"]


class FftbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fftb status {status}: {msg}")
        self.status = status


_lib = None


def lib() -> C.CDLL:
    """Load libfftb.so (built in-tree). Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2406_05577_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.fftb_plan_create.argtypes = [C.POINTER(vp), C.POINTER(C.c_int32), C.POINTER(Sphere_t),
                                   C.c_int32, C.c_int, C.c_uint32, C.POINTER(Tuning_t), vp]
    L.fftb_plan_create.restype = C.c_int
    L.fftb_sphere_to_grid.argtypes = [vp, vp, vp, vp]
    L.fftb_sphere_to_grid.restype = C.c_int
    L.fftb_grid_to_sphere.argtypes = [vp, vp, vp, vp]
    L.fftb_grid_to_sphere.restype = C.c_int
    L.fftb_sphere_to_grid_static.argtypes = [vp, vp, vp, vp]
    L.fftb_sphere_to_grid_static.restype = C.c_int
    L.fftb_apply_potential.argtypes = [vp, vp, vp, vp, vp, vp]
    L.fftb_apply_potential.restype = C.c_int
    L.fftb_plan_create_cuboid.argtypes = [C.POINTER(vp), C.POINTER(C.c_int32), C.c_int32, C.c_int,
                                          C.c_uint32, C.POINTER(Tuning_t), vp]
    L.fftb_plan_create_cuboid.restype = C.c_int
    L.fftb_plan_get_info.argtypes = [vp, C.POINTER(Info_t)]
    L.fftb_plan_get_info.restype = C.c_int
    L.fftb_plan_workspace_size.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.fftb_plan_workspace_size.restype = C.c_int
    L.fftb_plan_sphere_stats.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.fftb_plan_sphere_stats.restype = C.c_int
    ip = C.POINTER(C.c_int32)
    L.fftb_plan_sphere_columns.argtypes = [vp, C.c_int32, ip, ip, ip, ip]
    L.fftb_plan_sphere_columns.restype = C.c_int
    L.fftb_plan_set_profiling.argtypes = [vp, C.c_int32]
    L.fftb_plan_set_profiling.restype = C.c_int
    L.fftb_plan_get_profile.argtypes = [vp, C.POINTER(Profile_t)]
    L.fftb_plan_get_profile.restype = C.c_int
    L.fftb_plan_destroy.argtypes = [vp]
    L.fftb_plan_destroy.restype = C.c_int
    L.fftb_status_string.argtypes = [C.c_int]
    L.fftb_status_string.restype = C.c_char_p
    L.fftb_last_error.argtypes = []
    L.fftb_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(st: int):
    if st != FFTB_OK:
        L = lib()
        raise FftbError(st, f"{L.fftb_status_string(st).decode()}: {L.fftb_last_error().decode()}")


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Plan:
    """A sphere<->grid transform plan (create / execute / destroy).

    dims    -- (nx, ny, nz)
    maps    -- list of int32 arrays, one per sphere (k-point): wrapped linear
               grid index x + nx*(y + ny*z) of each coefficient
    nbands  -- int or list of ints (bands per sphere)
    kpts    -- optional list of k-points (metadata)
    dtype   -- "c128" or "c64"
    flags   -- PLAN_* bits
    tuning  -- optional dict of tiling knobs (band_chunk, y_classes, x_rows, col_tile,
               threads, path, acc, splits); plain keys set both directions,
               inv_<key> / fwd_<key> one of them
    """

    def __init__(self, dims: Sequence[int], maps, nbands, kpts=None, dtype: str = "c128",
                 flags: int = 0, tuning: Optional[dict] = None, stream=None):
        L = lib()
        if isinstance(maps, np.ndarray) and maps.ndim == 1:
            maps = [maps]
        nsph = len(maps)
        if isinstance(nbands, int):
            nbands = [nbands] * nsph
        if kpts is None:
            kpts = [(0.0, 0.0, 0.0)] * nsph
        self._maps = [np.ascontiguousarray(m, dtype=np.int32) for m in maps]
        arr = (Sphere_t * nsph)()
        for i, m in enumerate(self._maps):
            arr[i].n_coeffs = m.shape[0]
            arr[i].map = m.ctypes.data_as(C.POINTER(C.c_int32))
            arr[i].kpt[:] = [float(v) for v in kpts[i]]
            arr[i].nbands = int(nbands[i])
        d = (C.c_int32 * 3)(*[int(v) for v in dims])
        tun = make_tuning(tuning) if tuning else None
        self.dtype = dtype
        dt = FFTB_C128 if dtype == "c128" else FFTB_C64
        self._h = C.c_void_p()
        st = None
        if not (flags & PLAN_HOST_ONLY):
            st = _stream_ptr(stream)
        _check(L.fftb_plan_create(C.byref(self._h), d, arr, nsph, dt, flags,
                                  C.byref(tun) if tun is not None else None, st))
        self.dims = tuple(int(v) for v in dims)
        self.nbands = list(nbands)
        self.flags = flags
        self.info = self.get_info()

    @classmethod
    def cuboid(cls, dims: Sequence[int], nbands: int, dtype: str = "c128", flags: int = 0,
               tuning: Optional[dict] = None, stream=None) -> "Plan":
        """The batched cuboid 3D FFT: every grid point is a coefficient, both
        buffers hold G[z][y][x][b] (fftb_plan_create_cuboid)."""
        L = lib()
        self = cls.__new__(cls)
        n = int(dims[0]) * int(dims[1]) * int(dims[2])
        self._maps = [np.arange(n, dtype=np.int32)]
        d = (C.c_int32 * 3)(*[int(v) for v in dims])
        tun = make_tuning(tuning) if tuning else None
        self.dtype = dtype
        self._h = C.c_void_p()
        st = None if (flags & PLAN_HOST_ONLY) else _stream_ptr(stream)
        _check(L.fftb_plan_create_cuboid(C.byref(self._h), d, int(nbands),
                                         FFTB_C128 if dtype == "c128" else FFTB_C64, flags,
                                         C.byref(tun) if tun is not None else None, st))
        self.dims = tuple(int(v) for v in dims)
        self.nbands = [int(nbands)]
        self.flags = flags
        self.info = self.get_info()
        return self

    def get_info(self) -> dict:
        inf = Info_t()
        _check(lib().fftb_plan_get_info(self._h, C.byref(inf)))
        out = {f: getattr(inf, f) for f, _ in Info_t._fields_}
        out["dims"] = tuple(inf.dims)
        out["tuning"] = {d: {f: getattr(getattr(inf.tuning, d), f) for f in DIR_FIELDS}
                         for d in ("inv", "fwd")}
        for k in ("radix_x", "radix_y", "radix_z"):
            out[k] = [v for v in getattr(inf, k) if v]
        return out

    def sphere_stats(self, s: int):
        nc, ns = C.c_int32(), C.c_int32()
        _check(lib().fftb_plan_sphere_stats(self._h, s, C.byref(nc), C.byref(ns)))
        return nc.value, ns.value

    def sphere_columns(self, s: int):
        ncol, _ = self.sphere_stats(s)
        ns = self._maps[s].shape[0]
        cx = np.zeros(ncol, np.int32)
        cy = np.zeros(ncol, np.int32)
        ec = np.zeros(ns, np.int32)
        ez = np.zeros(ns, np.int32)
        ip = C.POINTER(C.c_int32)
        _check(lib().fftb_plan_sphere_columns(self._h, s, cx.ctypes.data_as(ip),
                                              cy.ctypes.data_as(ip), ec.ctypes.data_as(ip),
                                              ez.ctypes.data_as(ip)))
        return cx, cy, ec, ez

    def set_profiling(self, on: bool):
        _check(lib().fftb_plan_set_profiling(self._h, 1 if on else 0))

    def get_profile(self) -> dict:
        """Per-kernel launches and total milliseconds since the last call."""
        pr = Profile_t()
        _check(lib().fftb_plan_get_profile(self._h, C.byref(pr)))
        return {n: (pr.launches[i], pr.total_ms[i]) for i, n in enumerate(KERNEL_NAMES)}

    @property
    def torch_dtype(self):
        import torch
        return torch.complex128 if self.dtype == "c128" else torch.complex64

    def _check_tensor(self, t, numel, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
        if t.dtype != self.torch_dtype:
            raise TypeError(f"{name} has dtype {t.dtype}, plan expects {self.torch_dtype}")
        if not t.is_contiguous() or t.numel() != numel:
            raise ValueError(f"{name} must be contiguous with {numel} elements")

    def sphere_to_grid(self, sphere, grid=None, stream=None):
        import torch
        self._check_tensor(sphere, self.info["sphere_elems"], "sphere")
        if grid is None:
            grid = torch.empty(self.info["grid_elems"], dtype=self.torch_dtype, device=sphere.device)
        self._check_tensor(grid, self.info["grid_elems"], "grid")
        _check(lib().fftb_sphere_to_grid(self._h, sphere.data_ptr(), grid.data_ptr(),
                                         _stream_ptr(stream)))
        return grid

    def sphere_to_grid_static(self, sphere, grid, stream=None):
        """sphere_to_grid with the library's static device scratch instead of
        the plan's (fftb_sphere_to_grid_static): allocates nothing, so `grid`
        must be given."""
        self._check_tensor(sphere, self.info["sphere_elems"], "sphere")
        self._check_tensor(grid, self.info["grid_elems"], "grid")
        _check(lib().fftb_sphere_to_grid_static(self._h, sphere.data_ptr(), grid.data_ptr(),
                                                _stream_ptr(stream)))
        return grid

    def grid_to_sphere(self, grid, sphere=None, stream=None):
        import torch
        self._check_tensor(grid, self.info["grid_elems"], "grid")
        if sphere is None:
            sphere = torch.empty(self.info["sphere_elems"], dtype=self.torch_dtype, device=grid.device)
        self._check_tensor(sphere, self.info["sphere_elems"], "sphere")
        _check(lib().fftb_grid_to_sphere(self._h, grid.data_ptr(), sphere.data_ptr(),
                                         _stream_ptr(stream)))
        return sphere

    def apply_potential(self, sphere, potential, grid=None, out=None, stream=None):
        """c' = grid_to_sphere(V * sphere_to_grid(c)) for a real potential V
        (N values in [z][y][x] order, float64 for c128 plans, float32 for c64),
        fused into the inverse kernel. `grid` receives V * psi."""
        import torch
        self._check_tensor(sphere, self.info["sphere_elems"], "sphere")
        rdt = torch.float64 if self.info["dtype"] == 0 else torch.float32
        nx, ny, nz = self.info["dims"]
        if not (potential.is_cuda and potential.dtype == rdt and potential.is_contiguous()
                and potential.numel() == nx * ny * nz):
            raise ValueError(f"potential must be a contiguous {rdt} CUDA tensor of {nx * ny * nz} values")
        if grid is None:
            grid = torch.empty(self.info["grid_elems"], dtype=self.torch_dtype, device=sphere.device)
        self._check_tensor(grid, self.info["grid_elems"], "grid")
        if out is None:
            out = torch.empty(self.info["sphere_elems"], dtype=self.torch_dtype, device=sphere.device)
        self._check_tensor(out, self.info["sphere_elems"], "sphere")
        _check(lib().fftb_apply_potential(self._h, sphere.data_ptr(), potential.data_ptr(),
                                          grid.data_ptr(), out.data_ptr(), _stream_ptr(stream)))
        return out

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().fftb_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
