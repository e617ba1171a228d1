"""A-term image-domain gridding for AMD MI355X (gfx950).

Thin Python binding of ``libaidg.so`` (see ``include/aidg.h``): argument
marshalling only.  Every step of gridding and degridding runs in the library's
HIP kernels; PyTorch supplies device memory (tensors) and the HIP stream.  When
the library has not been built, importing works but every call raises
``RuntimeError`` -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaidg.so")

AIDG_OK, AIDG_E_INVALID, AIDG_E_NOMEM, AIDG_E_DEVICE, AIDG_E_UNSUPPORTED, AIDG_E_RANGE, AIDG_E_BUSY = range(7)
STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "NOMEM", 3: "DEVICE", 4: "UNSUPPORTED", 5: "RANGE", 6: "BUSY"}
FP32, FP64 = 0, 1
ATERM_ADJOINT, ATERM_INVERSE = 0, 1  # A-term of gridding: A^H (adjoint of degridding) or normalised A^-1
DEGRID_AUTO, DEGRID_RECURRENCE, DEGRID_PER_VIS, DEGRID_DIRECT = 0, 1, 2, 3  # degridder form per subgrid

# aidg_subgrid (64 bytes), see include/aidg.h
SUBGRID_DTYPE = np.dtype([
    ("bl", "<i4"), ("st1", "<i4"), ("st2", "<i4"), ("t0", "<i4"), ("nt", "<i4"),
    ("c0", "<i4"), ("nc", "<i4"), ("U0", "<i4"), ("V0", "<i4"), ("wlayer", "<i4"),
    ("aint", "<i4"), ("folded", "<i4"), ("w0", "<f8"), ("vis_offset", "<i8")])


class AidgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"aidg {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class _Geometry(ctypes.Structure):
    _fields_ = [("grid_size", ctypes.c_int32), ("subgrid_size", ctypes.c_int32),
                ("kernel_support", ctypes.c_int32), ("aterm_interval", ctypes.c_int32),
                ("pixel_scale", ctypes.c_double), ("w_step", ctypes.c_double),
                ("taper_beta", ctypes.c_double), ("precision", ctypes.c_int32),
                ("reseed_channels", ctypes.c_int32), ("strict_range", ctypes.c_int32),
                ("max_subgrid_vis", ctypes.c_int32), ("center_lattice", ctypes.c_int32),
                ("w_fold", ctypes.c_int32), ("aterm_mode", ctypes.c_int32),
                ("stokes_i", ctypes.c_int32), ("degrid_form", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("workspace_bytes", ctypes.c_int64)]


class _PlanInfo(ctypes.Structure):
    _fields_ = [("n_subgrids", ctypes.c_int64), ("n_vis", ctypes.c_int64),
                ("n_excluded", ctypes.c_int64), ("n_wlayers", ctypes.c_int32),
                ("subgrid_size", ctypes.c_int32), ("w_step", ctypes.c_double),
                ("device_bytes", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("grid_bytes", ctypes.c_int64), ("vis_bytes", ctypes.c_int64),
                ("n_batches", ctypes.c_int64), ("max_subgrid_vis", ctypes.c_int64),
                ("n_groups", ctypes.c_int64), ("n_subgrids_pervis", ctypes.c_int64),
                ("n_subgrids_direct", ctypes.c_int64)]


class _Footprint(ctypes.Structure):
    _fields_ = [("n_wlayers", ctypes.c_int32), ("n_pol", ctypes.c_int32), ("w_step", ctypes.c_double),
                ("n_subgrids", ctypes.c_int64), ("n_excluded", ctypes.c_int64), ("grid_bytes", ctypes.c_int64),
                ("vis_bytes", ctypes.c_int64), ("aterm_bytes", ctypes.c_int64), ("plan_bytes", ctypes.c_int64),
                ("n_groups", ctypes.c_int64), ("n_subgrids_pervis", ctypes.c_int64),
                ("n_subgrids_direct", ctypes.c_int64)]


KERNEL_CLASSES = ("grid_dft", "fft_add", "split_ifft", "degrid_dft", "zero_vis", "image_fft",
                  "image_wstack")
DIR_GRID, DIR_DEGRID = 0, 1


class _Work(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("direction", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("in_", ctypes.c_void_p), ("out", ctypes.c_void_p), ("sg_begin", ctypes.c_int64),
                ("sg_end", ctypes.c_int64)]


class _KernelTimes(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 7), ("launches", ctypes.c_int64 * 7),
                ("vis_pixels", ctypes.c_int64 * 7), ("subgrids", ctypes.c_int64 * 7)]


@dataclasses.dataclass
class Geometry:
    """Mirror of ``aidg_geometry``."""

    grid_size: int
    subgrid_size: int
    kernel_support: int
    pixel_scale: float
    aterm_interval: int = 1
    w_step: float = 0.0
    taper_beta: float = 0.0
    precision: int = FP32
    reseed_channels: int = 0
    strict_range: int = 0
    max_subgrid_vis: int = 0
    workspace_bytes: int = 0
    center_lattice: int = 0
    w_fold: int = 0
    aterm_mode: int = ATERM_ADJOINT
    stokes_i: int = 0
    degrid_form: int = 0  # DEGRID_AUTO, DEGRID_RECURRENCE, DEGRID_PER_VIS or DEGRID_DIRECT

    @property
    def n_pol(self) -> int:
        """Grid and image planes: 4 (XX, XY, YX, YY), or 1 for Stokes-I grids."""
        return 1 if self.stokes_i else 4

    def to_c(self) -> _Geometry:
        return _Geometry(self.grid_size, self.subgrid_size, self.kernel_support, self.aterm_interval,
                         self.pixel_scale, self.w_step, self.taper_beta, self.precision,
                         self.reseed_channels, self.strict_range, self.max_subgrid_vis,
                         self.center_lattice, self.w_fold, self.aterm_mode, self.stokes_i,
                         self.degrid_form, 0, self.workspace_bytes)


_lib = None
ABI_VERSION = 8  # the structure layouts above follow include/aidg.h at this version


def library() -> ctypes.CDLL:
    """Load libaidg.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2502_17789_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "aidg_abi_version": (I32, []),
        "aidg_last_error": (ctypes.c_char_p, []),
        "aidg_partition": (I32, [P, I32, I32, I32, I32, P, P, P, P, I64, P, P]),
        "aidg_plan_create": (I32, [P, I32, I32, I32, I32, P, P, P, P, P, I64, P, P]),
        "aidg_plan_info_get": (I32, [P, P]),
        "aidg_plan_subgrids": (I32, [P, P, I64]),
        "aidg_plan_wlayers": (I32, [P, P, I32]),
        "aidg_plan_set_aterms": (I32, [P, P, P]),
        "aidg_plan_aterm_norm": (I32, [P, P, I64]),
        "aidg_grid": (I32, [P, P, P, P]),
        "aidg_degrid": (I32, [P, P, P, P]),
        "aidg_grid_adjoint": (I32, [P, P, P, P]),
        "aidg_degrid_adjoint": (I32, [P, P, P, P]),
        "aidg_footprint_estimate": (I32, [P, I32, I32, I32, I32, P, P, P]),
        "aidg_plan_set_profiling": (I32, [P, I32]),
        "aidg_plan_kernel_times": (I32, [P, P]),
        "aidg_plan_destroy": (None, [P]),
        "aidg_executor_create": (I32, [I64, P]),
        "aidg_execute": (I32, [P, P, I32, P]),
        "aidg_executor_destroy": (None, [P]),
        "aidg_execute_static": (I32, [P, I32, I64, P]),
        "aidg_image_workspace_bytes": (I32, [P, P]),
        "aidg_invert": (I32, [P, P, P, P, I64, P]),
        "aidg_predict": (I32, [P, P, P, P, I64, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if lib.aidg_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{LIB_PATH} has ABI version {lib.aidg_abi_version()}, this binding "
                           f"expects {ABI_VERSION}: rebuild with `python -m paper_2502_17789_amd.build`")
    _lib = lib
    return lib


def _check(status: int):
    if status != AIDG_OK:
        raise AidgError(status, library().aidg_last_error().decode())


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def partition(geometry: Geometry, n_stations: int, baselines, uvw, freqs):
    """The library's own partition (host only, no GPU needed)."""
    lib = library()
    bl, u, f = _host(baselines, np.int32), _host(uvw, np.float64), _host(freqs, np.float64)
    g = geometry.to_c()
    n = ctypes.c_int64(0)
    w = ctypes.c_double(0)
    args = [ctypes.byref(g), n_stations, bl.shape[0], u.shape[1], f.shape[0], _ptr(bl), _ptr(u), _ptr(f)]
    st = lib.aidg_partition(*args, None, 0, ctypes.byref(n), ctypes.byref(w))
    if st not in (AIDG_OK, AIDG_E_INVALID) or (st == AIDG_E_INVALID and n.value == 0):
        _check(st)
    out = np.zeros(max(n.value, 1), SUBGRID_DTYPE)
    _check(lib.aidg_partition(*args, _ptr(out), out.shape[0], ctypes.byref(n), ctypes.byref(w)))
    return out[:n.value].copy(), w.value


def footprint(geometry: Geometry, n_stations: int, baselines, uvw, freqs) -> dict:
    """Device memory a plan of this observation and its data would take, estimated on the
    host without building the plan (``aidg_footprint_estimate``): n_wlayers, grid_bytes,
    vis_bytes, aterm_bytes, plan_bytes and the estimated subgrid and same-centre group
    counts."""
    lib = library()
    u, f = _host(uvw, np.float64), _host(freqs, np.float64)
    nbl = int(np.asarray(baselines).shape[0])
    g = geometry.to_c()
    out = _Footprint()
    _check(lib.aidg_footprint_estimate(ctypes.byref(g), int(n_stations), nbl, u.shape[1], f.shape[0],
                                       _ptr(u), _ptr(f), ctypes.byref(out)))
    return {name: getattr(out, name) for name, _ in _Footprint._fields_}


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A gridding/degridding plan on the current HIP device (``aidg_plan``)."""

    def __init__(self, geometry: Geometry, n_stations: int, baselines, uvw, freqs, aterms,
                 table=None, stream=None):
        import torch
        lib = library()
        self.geometry = geometry
        self._cdtype = torch.complex64 if geometry.precision == FP32 else torch.complex128
        if not (isinstance(aterms, torch.Tensor) and aterms.is_cuda and aterms.dtype == self._cdtype
                and aterms.is_contiguous()):
            raise TypeError("aterms must be a contiguous device tensor of the plan's complex dtype")
        self.baselines = _host(baselines, np.int32)
        self.uvw = _host(uvw, np.float64)
        self.freqs = _host(freqs, np.float64)
        self.n_stations = int(n_stations)
        self.nbl, self.nt, self.nc = self.baselines.shape[0], self.uvw.shape[1], self.freqs.shape[0]
        n_int = (self.nt + geometry.aterm_interval - 1) // geometry.aterm_interval
        L = geometry.subgrid_size
        if tuple(aterms.shape) != (n_int, self.n_stations, L, L, 4):
            raise ValueError(f"aterms shape {tuple(aterms.shape)} != {(n_int, self.n_stations, L, L, 4)}")
        tab = None if table is None else _host(table, SUBGRID_DTYPE)
        g = geometry.to_c()
        h = ctypes.c_void_p()
        _check(lib.aidg_plan_create(ctypes.byref(g), self.n_stations, self.nbl, self.nt, self.nc,
                                    _ptr(self.baselines), _ptr(self.uvw), _ptr(self.freqs), _dptr(aterms),
                                    None if tab is None else _ptr(tab), 0 if tab is None else tab.shape[0],
                                    _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        info = _PlanInfo()
        _check(lib.aidg_plan_info_get(h, ctypes.byref(info)))
        self.info = {name: getattr(info, name) for name, _ in _PlanInfo._fields_}
        self.n_wlayers = info.n_wlayers

    # ------------------------------------------------------------ queries
    def subgrids(self) -> np.ndarray:
        out = np.zeros(max(self.info["n_subgrids"], 1), SUBGRID_DTYPE)
        _check(library().aidg_plan_subgrids(self._h, _ptr(out), out.shape[0]))
        return out[:self.info["n_subgrids"]].copy()

    def wlayers(self) -> np.ndarray:
        out = np.zeros(self.n_wlayers)
        _check(library().aidg_plan_wlayers(self._h, _ptr(out), self.n_wlayers))
        return out

    def grid_shape(self):
        N = self.geometry.grid_size
        return (self.n_wlayers, self.geometry.n_pol, N, N)

    def vis_shape(self):
        return (self.nbl, self.nt, self.nc, 4)

    # ------------------------------------------------------------ operations
    def _check_tensor(self, t, shape, name):
        if not (t.is_cuda and t.dtype == self._cdtype and t.is_contiguous() and tuple(t.shape) == shape):
            raise ValueError(f"{name} must be a contiguous {self._cdtype} device tensor of shape {shape}")

    def set_aterms(self, aterms, stream=None):
        L = self.geometry.subgrid_size
        n_int = (self.nt + self.geometry.aterm_interval - 1) // self.geometry.aterm_interval
        self._check_tensor(aterms, (n_int, self.n_stations, L, L, 4), "aterms")
        _check(library().aidg_plan_set_aterms(self._h, _dptr(aterms), _stream_handle(stream)))

    def aterm_norm(self):
        """Inverse A-term mode: the weighted-average normalisation map [L, L] (float64,
        host) that ``invert`` divides the image by (after bilinear interpolation)."""
        L = self.geometry.subgrid_size
        out = np.zeros((L, L), np.float64)
        _check(library().aidg_plan_aterm_norm(self._h, out.ctypes.data_as(ctypes.c_void_p), L * L))
        return out

    def grid(self, vis, out=None, stream=None):
        """Grid ``vis`` [nbl, nt, nc, 4]; accumulates into ``out`` (zeros if None)."""
        import torch
        self._check_tensor(vis, self.vis_shape(), "vis")
        if out is None:
            out = torch.zeros(self.grid_shape(), dtype=self._cdtype, device=vis.device)
        self._check_tensor(out, self.grid_shape(), "grid")
        _check(library().aidg_grid(self._h, _dptr(vis), _dptr(out), _stream_handle(stream)))
        return out

    def degrid(self, grid, out=None, stream=None):
        """Degrid ``grid`` [W, P, N, N] into ``out`` [nbl, nt, nc, 4] (overwritten)."""
        import torch
        self._check_tensor(grid, self.grid_shape(), "grid")
        if out is None:
            out = torch.empty(self.vis_shape(), dtype=self._cdtype, device=grid.device)
        self._check_tensor(out, self.vis_shape(), "vis")
        _check(library().aidg_degrid(self._h, _dptr(grid), _dptr(out), _stream_handle(stream)))
        return out

    def grid_adjoint(self, vis, out=None, stream=None):
        """The exact adjoint of ``degrid`` applied to ``vis`` (aidg_grid_adjoint), accumulated
        into ``out`` (zeros if None); equal to ``grid`` except on Stokes-I plans."""
        import torch
        self._check_tensor(vis, self.vis_shape(), "vis")
        if out is None:
            out = torch.zeros(self.grid_shape(), dtype=self._cdtype, device=vis.device)
        self._check_tensor(out, self.grid_shape(), "grid")
        _check(library().aidg_grid_adjoint(self._h, _dptr(vis), _dptr(out), _stream_handle(stream)))
        return out

    def degrid_adjoint(self, grid, out=None, stream=None):
        """The exact adjoint of ``grid`` applied to ``grid`` (aidg_degrid_adjoint), written to
        ``out``; equal to ``degrid`` except on Stokes-I plans."""
        import torch
        self._check_tensor(grid, self.grid_shape(), "grid")
        if out is None:
            out = torch.empty(self.vis_shape(), dtype=self._cdtype, device=grid.device)
        self._check_tensor(out, self.vis_shape(), "vis")
        _check(library().aidg_degrid_adjoint(self._h, _dptr(grid), _dptr(out), _stream_handle(stream)))
        return out

    def image_shape(self):
        N = self.geometry.grid_size
        return (self.geometry.n_pol, N, N)

    def _image_workspace(self, device):
        import torch
        n = ctypes.c_int64()
        _check(library().aidg_image_workspace_bytes(self._h, ctypes.byref(n)))
        ws = getattr(self, "_img_ws", None)
        if ws is None or ws.numel() < n.value or ws.device != device:
            ws = self._img_ws = torch.empty(n.value, dtype=torch.uint8, device=device)
        return ws

    def invert(self, grid, out=None, stream=None):
        """Image ``grid`` [W, P, N, N] by w-stacking into ``out`` [P, N, N] (overwritten)."""
        import torch
        self._check_tensor(grid, self.grid_shape(), "grid")
        if out is None:
            out = torch.empty(self.image_shape(), dtype=self._cdtype, device=grid.device)
        self._check_tensor(out, self.image_shape(), "image")
        ws = self._image_workspace(grid.device)
        _check(library().aidg_invert(self._h, _dptr(grid), _dptr(out), _dptr(ws), ws.numel(),
                                     _stream_handle(stream)))
        return out

    def predict(self, image, out=None, stream=None):
        """Grid layers [W, 4, N, N] (``out``, overwritten) predicted from ``image`` [4, N, N]."""
        import torch
        self._check_tensor(image, self.image_shape(), "image")
        if out is None:
            out = torch.empty(self.grid_shape(), dtype=self._cdtype, device=image.device)
        self._check_tensor(out, self.grid_shape(), "grid")
        ws = self._image_workspace(image.device)
        _check(library().aidg_predict(self._h, _dptr(image), _dptr(out), _dptr(ws), ws.numel(),
                                      _stream_handle(stream)))
        return out

    def set_profiling(self, enable: bool = True):
        """Time every kernel launch with HIP events on its stream (aidg_plan_set_profiling)."""
        _check(library().aidg_plan_set_profiling(self._h, 1 if enable else 0))

    def kernel_times(self) -> dict:
        """Per kernel class: summed ms, launches, vis x pixels, subgrids; resets the sums."""
        kt = _KernelTimes()
        _check(library().aidg_plan_kernel_times(self._h, ctypes.byref(kt)))
        return {name: {"ms": kt.ms[i], "launches": kt.launches[i], "vis_pixels": kt.vis_pixels[i],
                       "subgrids": kt.subgrids[i]} for i, name in enumerate(KERNEL_CLASSES)}

    def close(self):
        if getattr(self, "_h", None):
            library().aidg_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


STATIC_WORKSPACE_BYTES = 128 << 20   # AIDG_STATIC_WORKSPACE_BYTES


def _work_array(items):
    items = list(items)
    arr = (_Work * max(len(items), 1))()
    for i, (plan, direction, tin, tout, b, e) in enumerate(items):
        arr[i] = _Work(plan._h.value, int(direction), 0, tin.data_ptr(), tout.data_ptr(), int(b), int(e))
    return arr, len(items)


def execute_static(items, workspace_bytes: int = 0, stream=None):
    """Grouped execution without an executor (``aidg_execute_static``): the group images
    go to the library's static device workspace, so the call allocates nothing.
    items as for ``Executor.execute``; workspace_bytes: budget within the static
    workspace (0 = all of it)."""
    arr, n = _work_array(items)
    _check(library().aidg_execute_static(arr, n, int(workspace_bytes), _stream_handle(stream)))


class Executor:
    """Grouped execution of subgrid ranges from many plans (``aidg_execute``)."""

    def __init__(self, workspace_bytes: int = 0):
        h = ctypes.c_void_p()
        _check(library().aidg_executor_create(int(workspace_bytes), ctypes.byref(h)))
        self._h = h

    def execute(self, items, stream=None):
        """items: iterable of (plan, direction, in_tensor, out_tensor, sg_begin, sg_end)."""
        arr, n = _work_array(items)
        _check(library().aidg_execute(self._h, arr, n, _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None):
            library().aidg_executor_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
