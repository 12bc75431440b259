"""Oracle for voxel-driven cone-beam back projection -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never imports,
links or calls it, and the two share no code: the product must fail loudly
when its HIP library is missing instead of falling back to anything here.

Contents
  bp          FP64 multithreaded back projector (C, ``bp_oracle.c``) and its
              ctypes loader; a pure-Python brute-force tent-sum interpolant.
  geometry    FP64 projection matrices of a circular cone-beam trajectory,
              and an independent ray/detector-plane intersection used to pin
              them.
  closed      closed-form back projections (constant, affine, impulse images,
              orthographic identity) used to pin the oracle.
  fdk         FP64 cosine weighting and Ram-Lak row filtering: the pre-processing
              that turns raw projections into the filtered, weighted input of
              the back projection.

Every function cites the passage of Hofmann, Treibig, Hager and Wellein,
"Comparing the Performance of Different x86 SIMD Instruction Sets for a
Medical Imaging Application on Modern Multi- and Manycore Chips" (WPMVP'14)
that it follows.
"""
from .bp import backproject, backproject_points, interpolate, tent_interpolate, load_library, build_library
from . import geometry, closed, fdk

__all__ = [
    "backproject",
    "backproject_points",
    "interpolate",
    "tent_interpolate",
    "load_library",
    "build_library",
    "geometry",
    "closed",
    "fdk",
]
