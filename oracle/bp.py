"""FP64 back projector (ctypes over ``bp_oracle.c``) -- TEST INFRASTRUCTURE.

The computation is the RabbitCT reference back projection of Hofmann et al.
(WPMVP'14), Sec. 4.1 and Listing 1, with the readings stated in the header of
``bp_oracle.c`` (floor indices, W columns by H rows, row-major 3x4 matrices,
zero contribution unless w > 0, zero-extended image).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bp_oracle.c")
_LIB = os.path.join(_HERE, "_bp_oracle.so")
_lib = None

# -ffp-contract=off: every product and sum is rounded separately, as written.
GCC_FLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-pthread", "-ffp-contract=off", "-fno-fast-math"]


def build_library(src: str = _SRC, out: str = _LIB, defines: tuple = ()) -> str:
    """Compile ``bp_oracle.c`` (or a copy of it) with gcc into a shared object."""
    cmd = ["gcc", *GCC_FLAGS, *[f"-D{d}" for d in defines], src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _bind(lib):
    lib.oracle_backproject.restype = ctypes.c_int
    lib.oracle_backproject.argtypes = [
        ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
        ctypes.c_int, ctypes.c_int, ctypes.c_int,
        ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
        ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_int,
    ]
    lib.oracle_backproject_points.restype = ctypes.c_int
    lib.oracle_backproject_points.argtypes = [
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_long,
        ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
        ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_int,
    ]
    lib.oracle_backproject_abs.restype = ctypes.c_int
    lib.oracle_backproject_abs.argtypes = lib.oracle_backproject.argtypes
    lib.oracle_backproject_points_abs.restype = ctypes.c_int
    lib.oracle_backproject_points_abs.argtypes = lib.oracle_backproject_points.argtypes
    lib.oracle_interpolate.restype = ctypes.c_double
    lib.oracle_interpolate.argtypes = [
        ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
    ]
    return lib


def load_library(path: str | None = None):
    """Load the compiled oracle; build it first only if no build exists."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB):
            build_library()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def default_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def backproject(proj, P, L, voxel_size, origin, block=None, vol=None, threads=None, lib=None, absolute=False):
    """Back project ``proj`` into (a block of) an L^3 volume, in FP64.

    proj        (N, H, W) array; widened exactly to FP32 storage (the values the
                GPU reads).  FP16/BF16 data is passed already widened.
    P           (N, 3, 4) or (N, 12) matrices; widened to FP64.
    L           edge length of the volume.
    voxel_size  MM of Listing 1 (world units per voxel).
    origin      world position of the centre of voxel (0, 0, 0), per axis.
    block       ((x0, x1), (y0, y1), (z0, z1)) half-open voxel ranges; whole
                volume if None.
    vol         optional FP64 array (nz, ny, nx) to accumulate into.
    absolute    sum |contribution| of every view instead (the magnitude of the
                summands, which sets the sum's conditioning).
    Returns the FP64 block, indexed [z, y, x].
    """
    lib = lib or load_library()
    proj = np.ascontiguousarray(proj, dtype=np.float32)
    if proj.ndim != 3:
        raise ValueError("proj must be (N, H, W)")
    n, H, W = proj.shape
    P = np.ascontiguousarray(np.asarray(P, dtype=np.float64).reshape(n, 12))
    if block is None:
        block = ((0, L), (0, L), (0, L))
    (x0, x1), (y0, y1), (z0, z1) = block
    nx, ny, nz = x1 - x0, y1 - y0, z1 - z0
    if vol is None:
        vol = np.zeros((nz, ny, nx), dtype=np.float64)
    else:
        vol = np.ascontiguousarray(vol, dtype=np.float64).copy()
        if vol.shape != (nz, ny, nx):
            raise ValueError("vol has the wrong shape")
    o = np.ascontiguousarray(np.asarray(origin, dtype=np.float64).reshape(3))
    fn = lib.oracle_backproject_abs if absolute else lib.oracle_backproject
    rc = fn(
        vol.ctypes.data, x0, y0, z0, nx, ny, nz,
        proj.ctypes.data, W, H, n,
        P.ctypes.data, float(voxel_size), o.ctypes.data,
        int(threads if threads is not None else default_threads()),
    )
    if rc != 0:
        raise ValueError("oracle_backproject rejected its arguments")
    return vol


def backproject_points(proj, P, voxel_size, origin, xyz, threads=None, lib=None, absolute=False):
    """FP64 back projection of a list of voxels ``xyz`` (M, 3) integer (x, y, z); returns (M,) FP64
    (``absolute``: the sum of |contribution| instead)."""
    lib = lib or load_library()
    proj = np.ascontiguousarray(proj, dtype=np.float32)
    n, H, W = proj.shape
    P = np.ascontiguousarray(np.asarray(P, dtype=np.float64).reshape(n, 12))
    xyz = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1, 3)
    out = np.zeros(xyz.shape[0], dtype=np.float64)
    o = np.ascontiguousarray(np.asarray(origin, dtype=np.float64).reshape(3))
    fn = lib.oracle_backproject_points_abs if absolute else lib.oracle_backproject_points
    rc = fn(out.ctypes.data, xyz.ctypes.data, xyz.shape[0], proj.ctypes.data, W, H, n,
                                       P.ctypes.data, float(voxel_size), o.ctypes.data,
                                       int(threads if threads is not None else default_threads()))
    if rc != 0:
        raise ValueError("oracle_backproject_points rejected its arguments")
    return out


def interpolate(img, ix, iy, lib=None):
    """Bilinear interpolant of the zero-extended FP32 image at (ix, iy) (C oracle)."""
    lib = lib or load_library()
    img = np.ascontiguousarray(img, dtype=np.float32)
    H, W = img.shape
    return lib.oracle_interpolate(img.ctypes.data, W, H, float(ix), float(iy))


def tent_interpolate(img, ix, iy):
    """Brute-force interpolant: the double sum over all pixels of I[j][i] * tent(ix-i) * tent(iy-j).

    The tent is tent(r) = max(0, 1 - |r|).  This is a second, independent
    formula for the bilinear interpolant of the zero-extended image of Sec. 4.1
    (every pixel, on or off the detector, weighted by its hat function), so it
    pins the four-tap evaluation, the floor convention and the edges.  Works on
    Fractions for exact arithmetic.  Pure Python: tiny images only.
    """
    H = len(img)
    W = len(img[0])
    exact = isinstance(ix, Fraction) or isinstance(iy, Fraction)
    zero = Fraction(0) if exact else 0.0
    one = Fraction(1) if exact else 1.0
    total = zero
    for j in range(H):
        ty = one - abs(iy - j)
        if ty <= 0:
            continue
        for i in range(W):
            tx = one - abs(ix - i)
            if tx <= 0:
                continue
            pix = Fraction(float(img[j][i])) if exact else float(img[j][i])
            total += pix * tx * ty
    return total
