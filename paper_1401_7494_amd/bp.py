"""ctypes binding of ``libbp.so`` (the C ABI in ``include/bp.h``).

Argument marshalling only: torch tensors are checked for device, dtype and
layout, and their device pointers and the current HIP stream are passed to
the library.  Every step of the back projection runs in the library's HIP
kernels.  If the library is missing this module raises on import of the
library (``lib()``) -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbp.so")

BP_OK, BP_ERR_INVALID_ARG, BP_ERR_UNSUPPORTED, BP_ERR_OUT_OF_MEMORY, BP_ERR_DEVICE, BP_ERR_LAUNCH = range(6)
DTYPES = {"f32": 0, "f16": 1, "bf16": 2}
PATHS = {"auto": 0, "plain": 1, "fused": 2, "fused_direct": 3}
PATH_NAMES = {v: k for k, v in PATHS.items()}

# Every function the header declares, with its ctypes signature.
_c_int, _c_float, _c_double, _vp = ctypes.c_int, ctypes.c_float, ctypes.c_double, ctypes.c_void_p


class BpConfig(ctypes.Structure):
    _fields_ = [
        ("device", _c_int),
        ("det_width", _c_int),
        ("det_height", _c_int),
        ("proj_dtype", _c_int),
        ("path", _c_int),
        ("views_per_pass", _c_int),
        ("z_unroll", _c_int),
        ("tile_x", _c_int),
    ]


class BpFdkConfig(ctypes.Structure):
    _fields_ = [
        ("device", _c_int),
        ("det_width", _c_int),
        ("det_height", _c_int),
        ("pitch", _c_double),
        ("sid", _c_double),
        ("sdd", _c_double),
    ]


SIGNATURES = {
    "bp_config_default": (None, [ctypes.POINTER(BpConfig)]),
    "bp_create": (_c_int, [ctypes.POINTER(BpConfig), ctypes.POINTER(_vp)]),
    "bp_destroy": (_c_int, [_vp]),
    "bp_backproject": (_c_int, [_vp, _vp, _vp, _vp, _c_int, _c_int, _c_float, ctypes.POINTER(_c_float), _vp]),
    "bp_backproject_box": (_c_int, [_vp, _vp, _c_int, _c_int, _c_int, _vp, _vp, _c_int, _c_float,
                                    ctypes.POINTER(_c_float), _vp]),
    "bp_backproject_noalloc": (_c_int, [_vp, _vp, _c_int, _c_int, _c_int, _vp, _vp, _c_int, _c_float,
                                        ctypes.POINTER(_c_float), _vp]),
    "bp_set_tuning": (_c_int, [_vp, _c_int, _c_int, _c_int, _c_int]),
    "bp_set_options": (_c_int, [_vp, _c_int]),
    "bp_set_tap_split": (_c_int, [_vp, _c_int]),
    "bp_query_plan": (_c_int, [_vp, _c_int, _c_int, _c_int, _c_int, ctypes.POINTER(_c_int),
                               ctypes.POINTER(_c_int), ctypes.POINTER(_c_int), ctypes.POINTER(_c_int),
                               ctypes.POINTER(_c_int)]),
    "bp_query_scratch": (_c_int, [_vp, _c_int, _c_int, _c_int, _c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "bp_circular_matrices": (_c_int, [_vp, _c_int, _c_double, _c_double, _c_double, _c_int, _c_int, _vp, _vp]),
    "bp_enable_timing": (_c_int, [_vp, _c_int]),
    "bp_kernel_timing": (_c_int, [_vp, _c_int, ctypes.POINTER(_c_double), ctypes.POINTER(ctypes.c_longlong)]),
    "bp_status_string": (ctypes.c_char_p, [_c_int]),
    "bp_last_error": (ctypes.c_char_p, [_vp]),
    "bp_version": (ctypes.c_char_p, []),
    "bp_fdk_config_default": (None, [ctypes.POINTER(BpFdkConfig)]),
    "bp_fdk_create": (_c_int, [ctypes.POINTER(BpFdkConfig), ctypes.POINTER(_vp)]),
    "bp_fdk_filter": (_c_int, [_vp, _vp, _vp, _c_int, _c_int, _vp]),
    "bp_fdk_destroy": (_c_int, [_vp]),
    "bp_fdk_last_error": (ctypes.c_char_p, [_vp]),
}

_lib = None


class BPError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


def lib():
    """The loaded ``libbp.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1401_7494_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def status_string(st: int) -> str:
    return lib().bp_status_string(st).decode()


def circular_matrices(angles, sid, sdd, pitch, W, H):
    """Host FP64 composition of circular-orbit matrices; returns (P64 (N,3,4), P32 (N,3,4))."""
    a = np.ascontiguousarray(angles, dtype=np.float64)
    n = a.shape[0]
    p64 = np.empty((n, 3, 4), dtype=np.float64)
    p32 = np.empty((n, 3, 4), dtype=np.float32)
    st = lib().bp_circular_matrices(a.ctypes.data, n, float(sid), float(sdd), float(pitch), int(W), int(H),
                                    p64.ctypes.data, p32.ctypes.data)
    if st != BP_OK:
        raise BPError(st, f"bp_circular_matrices: {status_string(st)}")
    return p64, p32


@dataclass
class Plan:
    path: str
    views_per_pass: int
    z_unroll: int
    tile_x: int
    direct_taps: bool = False


class Context:
    """One library context (one device, detector size and projection dtype)."""

    def __init__(self, det_width=1248, det_height=960, dtype="f32", device=0, path="auto",
                 views_per_pass=0, z_unroll=0, tile_x=0):
        L = lib()
        cfg = BpConfig()
        L.bp_config_default(ctypes.byref(cfg))
        cfg.device = int(device)
        cfg.det_width = int(det_width)
        cfg.det_height = int(det_height)
        cfg.proj_dtype = DTYPES[dtype]
        cfg.path = PATHS[path]
        cfg.views_per_pass = int(views_per_pass)
        cfg.z_unroll = int(z_unroll)
        cfg.tile_x = int(tile_x)
        h = _vp()
        st = L.bp_create(ctypes.byref(cfg), ctypes.byref(h))
        if st != BP_OK:
            raise BPError(st, f"bp_create: {status_string(st)}")
        self._h = h
        self.det_width, self.det_height, self.dtype, self.device = det_width, det_height, dtype, device

    def close(self):
        if getattr(self, "_h", None):
            lib().bp_destroy(self._h)
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

    @property
    def handle(self):
        return self._h

    def last_error(self) -> str:
        return lib().bp_last_error(self._h).decode()

    def _check(self, st: int, what: str):
        if st != BP_OK:
            raise BPError(st, f"{what}: {status_string(st)}: {self.last_error()}")

    def set_tuning(self, path="auto", views_per_pass=0, z_unroll=0, tile_x=0):
        self._check(lib().bp_set_tuning(self._h, PATHS[path], int(views_per_pass), int(z_unroll), int(tile_x)),
                    "bp_set_tuning")

    OPT_NO_CULL = 1
    OPT_NO_COLUMN = 2
    OPT_XCD_ORDER = 4
    OPT_WIDE_STAGING = 8
    OPT_PLAIN_ORDER = 16
    OPT_XCD_REGION_SHIFT = 5
    OPT_DIRECT_TAPS = 1 << 9
    OPT_SERIAL_STAGING = 1 << 10
    OPT_OVERLAP_STAGING = 1 << 11
    OPT_STAGE_RECORDS = 1 << 12
    OPT_POISON_STAGING = 1 << 13
    OPT_SINGLE_TAPS = 1 << 14
    OPT_COMPACT_STAGING = 1 << 15
    ORDERS = ("region", "plain", "zslices")

    def set_options(self, no_cull: bool = False, no_column: bool = False, wide_staging: bool = False,
                    order: str = "region", region_ax: int = 0, direct_taps: bool = False,
                    staging: str = "auto", stage_records: bool = False, poison_staging: bool = False,
                    single_taps: bool = False, compact_staging: bool = False):
        """Switch off the clipping mask or the column specialisation (on by default); stage 16-bit
        projections as compact FP16 coefficients (``compact_staging``) instead of as FP32 projections
        (the default, which ``wide_staging`` names); choose the tile order ("region": XCD-private regions of
        each z-layer, ``region_ax`` regions along x (0 = default); "plain"; "zslices"); read every tap
        of the fused path directly instead of staging most views' footprints through LDS; stage the
        next pass while one runs ("overlap"), just before it ("serial") or as tuned ("auto":
        overlapped for compact 16-bit records); ``poison_staging`` (testing aid) fills the staging copy
        and the LDS stage with NaN before each is written; ``single_taps`` reads the caller's
        pixels one load per tap (instead of one load per row pair: 8 bytes of FP32, 4 of FP16/BF16)."""
        flags = ((self.OPT_NO_CULL if no_cull else 0) | (self.OPT_NO_COLUMN if no_column else 0)
                 | (self.OPT_WIDE_STAGING if wide_staging else 0))
        if order == "plain":
            flags |= self.OPT_PLAIN_ORDER
        elif order == "zslices":
            flags |= self.OPT_XCD_ORDER
        elif order != "region":
            raise ValueError(f"order must be one of {self.ORDERS}")
        flags |= int(region_ax) << self.OPT_XCD_REGION_SHIFT
        if direct_taps:
            flags |= self.OPT_DIRECT_TAPS
        if staging not in ("auto", "serial", "overlap"):
            raise ValueError(f"staging must be auto, serial or overlap, not {staging!r}")
        if staging == "serial":
            flags |= self.OPT_SERIAL_STAGING
        elif staging == "overlap":
            flags |= self.OPT_OVERLAP_STAGING
        if stage_records:
            flags |= self.OPT_STAGE_RECORDS
        if poison_staging:
            flags |= self.OPT_POISON_STAGING
        if single_taps:
            flags |= self.OPT_SINGLE_TAPS
        if compact_staging:
            flags |= self.OPT_COMPACT_STAGING
        self._check(lib().bp_set_options(self._h, flags), "bp_set_options")

    def set_tap_split(self, direct_eighths: int = -1):
        """Of every 8 views of a staged pass, how many read their taps directly (-1 = tuned)."""
        self._check(lib().bp_set_tap_split(self._h, int(direct_eighths)), "bp_set_tap_split")

    KERNELS = {"backproject": 0, "pad": 1, "views": 2}

    def enable_timing(self, on: bool = True):
        """Bracket every kernel launch with HIP events (resets the totals)."""
        self._check(lib().bp_enable_timing(self._h, int(bool(on))), "bp_enable_timing")

    def kernel_timing(self, kind: str = "backproject"):
        """(total milliseconds, launches) of one kernel kind since timing was enabled."""
        ms, n = _c_double(), ctypes.c_longlong()
        self._check(lib().bp_kernel_timing(self._h, self.KERNELS[kind], ctypes.byref(ms), ctypes.byref(n)),
                    "bp_kernel_timing")
        return ms.value, n.value

    def plan(self, nx, ny, nz, n_views) -> Plan:
        p, k, z, t, d = _c_int(), _c_int(), _c_int(), _c_int(), _c_int()
        self._check(lib().bp_query_plan(self._h, nx, ny, nz, n_views, ctypes.byref(p), ctypes.byref(k),
                                        ctypes.byref(z), ctypes.byref(t), ctypes.byref(d)), "bp_query_plan")
        return Plan(PATH_NAMES[p.value], k.value, z.value, t.value, bool(d.value))

    def scratch_bytes(self, nx, ny, nz, n_views) -> int:
        """Device scratch (bytes) a call of this size needs with the context's current settings."""
        b = ctypes.c_size_t()
        self._check(lib().bp_query_scratch(self._h, nx, ny, nz, n_views, ctypes.byref(b)), "bp_query_scratch")
        return b.value

    def backproject(self, volume, projections, matrices, voxel_size, origin, stream=None, cubic=False) -> None:
        """Accumulate ``projections`` (N, H, W) into ``volume`` (nz, ny, nx), asynchronously on ``stream``.

        cubic: call the cubic entry ``bp_backproject`` (volume L x L x L) instead of
        ``bp_backproject_box`` (the two compute the same).

        volume: contiguous float32 CUDA tensor.  projections: contiguous CUDA
        tensor of the context's dtype.  matrices: (N, 3, 4) or (N, 12)
        contiguous float32 CUDA tensor.  stream: torch stream or raw handle;
        default torch's current stream.
        """
        import torch

        _need(volume, torch.float32, "volume", 3)
        _need(projections, {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[self.dtype],
              "projections", 3)
        _need(matrices, torch.float32, "matrices", None)
        n = projections.shape[0]
        if projections.shape[1:] != (self.det_height, self.det_width):
            raise ValueError(f"projections must be (N, {self.det_height}, {self.det_width})")
        if matrices.numel() != 12 * n:
            raise ValueError("matrices must hold 12 floats per view")
        for t in (volume, projections, matrices):
            if t.device.index != self.device:
                raise ValueError("tensor is not on the context's device")
        nz, ny, nx = volume.shape
        o = (ctypes.c_float * 3)(*[float(v) for v in origin])
        if cubic:
            if not nx == ny == nz:
                raise ValueError("the cubic entry takes an L x L x L volume")
            st = lib().bp_backproject(self._h, volume.data_ptr(), projections.data_ptr(), matrices.data_ptr(), n,
                                      nx, float(voxel_size), o, _stream_handle(stream, self.device))
            self._check(st, "bp_backproject")
            return
        st = lib().bp_backproject_box(self._h, volume.data_ptr(), nx, ny, nz, projections.data_ptr(),
                                      matrices.data_ptr(), n, float(voxel_size), o, _stream_handle(stream, self.device))
        self._check(st, "bp_backproject_box")


class FdkFilter:
    """FDK pre-processing on one device for one detector geometry (``bp_fdk_*``).

    ``filter(raw, out_dtype)`` weights and ramp-filters raw projections
    (N, H, W) FP32 into a new tensor of ``out_dtype`` ("f32", "f16", "bf16"),
    or into ``out`` (which may be ``raw`` itself for FP32).
    """

    def __init__(self, det_width=1248, det_height=960, pitch=0.32, sid=800.0, sdd=1200.0, device=0):
        L = lib()
        cfg = BpFdkConfig()
        L.bp_fdk_config_default(ctypes.byref(cfg))
        cfg.device, cfg.det_width, cfg.det_height = int(device), int(det_width), int(det_height)
        cfg.pitch, cfg.sid, cfg.sdd = float(pitch), float(sid), float(sdd)
        h = _vp()
        st = L.bp_fdk_create(ctypes.byref(cfg), ctypes.byref(h))
        if st != BP_OK:
            raise BPError(st, f"bp_fdk_create: {status_string(st)}")
        self._h = h
        self.det_width, self.det_height, self.device = det_width, det_height, device

    @classmethod
    def for_scanner(cls, scanner, device=0):
        return cls(scanner.W, scanner.H, scanner.pitch, scanner.sid, scanner.sdd, device)

    def close(self):
        if getattr(self, "_h", None):
            lib().bp_fdk_destroy(self._h)
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

    def last_error(self) -> str:
        return lib().bp_fdk_last_error(self._h).decode()

    def filter(self, raw, out_dtype="f32", out=None, stream=None):
        import torch

        tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[out_dtype]
        _need(raw, torch.float32, "raw", 3)
        if raw.shape[1:] != (self.det_height, self.det_width):
            raise ValueError(f"raw must be (N, {self.det_height}, {self.det_width})")
        if raw.device.index != self.device:
            raise ValueError("raw is not on the filter's device")
        if out is None:
            out = torch.empty(raw.shape, dtype=tdt, device=raw.device)
        _need(out, tdt, "out", 3)
        if out.shape != raw.shape or out.device != raw.device:
            raise ValueError("out must match raw in shape and device")
        st = lib().bp_fdk_filter(self._h, raw.data_ptr(), out.data_ptr(), DTYPES[out_dtype], raw.shape[0],
                                 _stream_handle(stream, self.device))
        if st != BP_OK:
            raise BPError(st, f"bp_fdk_filter: {status_string(st)}: {self.last_error()}")
        return out


def _need(t, dtype, name, ndim):
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if ndim is not None and t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions")


def _stream_handle(stream, device):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream(device)
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def backproject(volume, projections, matrices, voxel_size, origin, dtype=None, stream=None, **ctx_kw):
    """One-shot convenience: create a context for the projections' shape, back project, destroy."""
    import torch

    if dtype is None:
        dtype = {torch.float32: "f32", torch.float16: "f16", torch.bfloat16: "bf16"}[projections.dtype]
    n, H, W = projections.shape
    with Context(W, H, dtype, device=volume.device.index or 0, **ctx_kw) as ctx:
        ctx.backproject(volume, projections, matrices, voxel_size, origin, stream)
        torch.cuda.current_stream(volume.device).synchronize() if stream is None else stream.synchronize()
