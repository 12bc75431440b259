"""The FP64 oracle against its pins (CPU only)."""
import numpy as np
import pytest

import oracle_pins as pins
from oracle import geometry


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin, oracle_lib):
    pin(oracle_lib)


def test_geometry_matches_ray_plane_intersection():
    """Composed matrices reproduce an explicit ray/detector-plane intersection (Sec. 4: A_i maps world to detector)."""
    angles = np.deg2rad([0.0, 17.0, 90.0, 133.3, 200.0 - 200.0 / 496])
    args = dict(sid=800.0, sdd=1200.0, pitch=0.32, W=1248, H=960)
    P = geometry.circular_matrices(angles, **args)
    rng = np.random.default_rng(0)
    X = rng.uniform(-128, 128, size=(40, 3))
    s, t, w = geometry.apply(P, X)
    s2, t2, w2 = geometry.project_by_intersection(angles, X=X, **args)
    assert np.abs(s - s2).max() < 1e-9
    assert np.abs(t - t2).max() < 1e-9
    assert np.abs(w - w2).max() < 1e-12


def test_geometry_isocentre_and_normalisation():
    """The isocentre lands on the detector centre with w = 1 in every view."""
    angles = np.linspace(0, np.deg2rad(200), 17)
    P = geometry.circular_matrices(angles, 800.0, 1200.0, 0.32, 1248, 960)
    s, t, w = geometry.apply(P, np.zeros((1, 3)))
    assert np.allclose(s, 623.5, atol=1e-12) and np.allclose(t, 479.5, atol=1e-12)
    assert np.allclose(w, 1.0, atol=1e-15)
    # magnification SDD/SID: 1 mm along e_v at the isocentre moves 1.5 mm = 1.5/0.32 px on the detector
    s, t, w = geometry.apply(P, np.array([[0.0, 0.0, 1.0]]))
    assert np.allclose(t - 479.5, 1.5 / 0.32, atol=1e-9)


def test_oracle_rejects_bad_arguments(oracle_lib):
    import ctypes

    rc = oracle_lib.oracle_backproject(None, 0, 0, 0, 1, 1, 1, None, 1, 1, 1, None, 1.0, None, 1)
    assert rc == -1
    buf = (ctypes.c_double * 1)()
    img = (ctypes.c_float * 1)()
    P = (ctypes.c_double * 12)()
    o = (ctypes.c_double * 3)()
    assert oracle_lib.oracle_backproject(buf, 0, 0, 0, 1, 1, 1, img, 0, 1, 1, P, 1.0, o, 1) == -1
    assert oracle_lib.oracle_backproject(buf, 0, 0, 0, 1, 1, 1, img, 1, 1, 1, P, 1.0, o, 1) == 0
