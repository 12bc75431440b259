"""The C ABI library on the host: it loads, exports what the header declares,
and its host-only parts behave (CPU only; no kernel is launched)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import geometry
from paper_1401_7494_amd import bp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bp_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_create_backproject_destroy_entry_points():
    names = declared_functions()
    for n in ("bp_create", "bp_backproject", "bp_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(bp.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    assert set(declared_functions()) == set(bp.SIGNATURES), "binding and header disagree"


def test_status_strings_and_version():
    assert bp.status_string(bp.BP_OK) == "ok"
    assert "invalid" in bp.status_string(bp.BP_ERR_INVALID_ARG)
    assert bp.status_string(99) == "unknown status"
    assert re.fullmatch(r"\d+\.\d+\.\d+", bp.lib().bp_version().decode())


def test_config_default():
    cfg = bp.BpConfig()
    bp.lib().bp_config_default(ctypes.byref(cfg))
    assert (cfg.det_width, cfg.det_height, cfg.proj_dtype, cfg.path) == (1248, 960, 0, 0)


def test_create_rejects_bad_config_without_touching_a_device():
    L = bp.lib()
    cfg = bp.BpConfig()
    L.bp_config_default(ctypes.byref(cfg))
    h = ctypes.c_void_p()
    assert L.bp_create(None, ctypes.byref(h)) == bp.BP_ERR_INVALID_ARG
    assert L.bp_create(ctypes.byref(cfg), None) == bp.BP_ERR_INVALID_ARG
    cfg.det_width = 0
    assert L.bp_create(ctypes.byref(cfg), ctypes.byref(h)) == bp.BP_ERR_INVALID_ARG
    L.bp_config_default(ctypes.byref(cfg))
    cfg.z_unroll = 3
    assert L.bp_create(ctypes.byref(cfg), ctypes.byref(h)) == bp.BP_ERR_INVALID_ARG
    L.bp_config_default(ctypes.byref(cfg))
    cfg.proj_dtype = 7
    assert L.bp_create(ctypes.byref(cfg), ctypes.byref(h)) == bp.BP_ERR_INVALID_ARG
    assert not h.value
    assert L.bp_destroy(None) == bp.BP_OK
    assert L.bp_backproject(None, None, None, None, 1, 1, 1.0, None, None) == bp.BP_ERR_INVALID_ARG


def test_create_without_gpu_reports_device_error():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = bp.lib()
    cfg = bp.BpConfig()
    L.bp_config_default(ctypes.byref(cfg))
    h = ctypes.c_void_p()
    assert L.bp_create(ctypes.byref(cfg), ctypes.byref(h)) == bp.BP_ERR_DEVICE


@pytest.mark.parametrize("n_views", [1, 7, 496])
def test_circular_matrices_match_the_oracle_geometry(n_views):
    """Host FP64 composition (K[R|t]/SID) vs the oracle's composition from the pinhole definition."""
    from paper_1401_7494_amd import synth

    sc = synth.Scanner(n_views=n_views)
    p64, p32 = bp.circular_matrices(*sc.geometry_args())
    ref = geometry.circular_matrices(*sc.geometry_args())
    assert np.abs(p64 - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.array_equal(p32, ref.astype(np.float32)), "FP32 rounding of the FP64 matrices differs"
    assert np.array_equal(p32, p64.astype(np.float32))


def test_circular_matrices_reject_bad_geometry():
    a = np.zeros(3)
    for args in [(0.0, 1200.0, 0.32), (800.0, -1.0, 0.32), (800.0, 1200.0, 0.0), (float("nan"), 1200.0, 0.32)]:
        with pytest.raises(bp.BPError):
            bp.circular_matrices(a, *args, 1248, 960)
    with pytest.raises(bp.BPError):
        bp.circular_matrices(np.array([np.inf]), 800.0, 1200.0, 0.32, 1248, 960)
