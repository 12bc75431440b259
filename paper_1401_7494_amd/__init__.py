"""MI355X-native voxel-driven cone-beam back projection.

The hot path -- back projecting filtered projections into an FP32 volume,
as in FDK reconstruction -- runs in hand-written HIP kernels for gfx950
behind a C ABI (``include/bp.h``, ``libbp.so``).  ``bp`` is the thin ctypes
binding; ``synth`` makes seeded synthetic inputs.  Submodules load lazily so
input generation works without the native library.
"""
import importlib

__all__ = ["bp", "synth", "autotune", "serve"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
