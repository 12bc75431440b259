"""The per-voxel FP32 error bound of ``fp32_bounds`` against an FP32 emulation (CPU).

The emulation evaluates the back projection with FP32 rounding after every
operation in the order the fused kernel uses (Part 1 by fused multiply-adds,
the reciprocal of w, the bilinear patch of the zero-padded image, Part 3,
FP32 accumulation); the bound must hold for every voxel against the FP64
oracle, and it must be tight enough that a wrong tap breaks it.
"""
import numpy as np
import pytest

import fp32_bounds
import oracle
from oracle import closed
from paper_1401_7494_amd import synth

SC_INSIDE = synth.Scanner(n_views=13, W=96, H=72, pitch=3.0, sid=60.0, sdd=160.0)  # source inside the box
BOX = (21, 37, 70)  # (nz, ny, nx)
VS = 3.0


def _origin(shape, vs):
    nz, ny, nx = shape
    return (-(nx - 1) / 2 * vs, -(ny - 1) / 2 * vs, -(nz - 1) / 2 * vs)


@pytest.fixture(scope="module")
def inside_case():
    proj = synth.filtered_projections(SC_INSIDE, synth.random_ellipsoids(1401)).numpy()
    P32 = closed_matrices(SC_INSIDE)
    origin = _origin(BOX, VS)
    nz, ny, nx = BOX
    ref = oracle.backproject(proj, P32.astype(np.float64), max(BOX), VS, origin,
                             block=((0, nx), (0, ny), (0, nz)))
    pts = closed.voxel_centres(max(BOX), VS, origin, block=((0, nx), (0, ny), (0, nz)))
    E, S = fp32_bounds.error_bound(proj, P32, pts)
    return proj, P32, origin, ref, E, S


def closed_matrices(sc):
    from oracle import geometry

    return geometry.circular_matrices(*sc.geometry_args()).astype(np.float32)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_bound_holds_for_an_fp32_evaluation(inside_case, sign):
    proj, P32, origin, ref, E, S = inside_case
    if sign < 0:
        P32 = -P32
        nz, ny, nx = BOX
        ref = oracle.backproject(proj, P32.astype(np.float64), max(BOX), VS, origin,
                                 block=((0, nx), (0, ny), (0, nz)))
        pts = closed.voxel_centres(max(BOX), VS, origin, block=((0, nx), (0, ny), (0, nz)))
        E, S = fp32_bounds.error_bound(proj, P32, pts)
    got = fp32_bounds.emulate_fp32(proj, P32, BOX, VS, origin)
    fin = np.isfinite(E)
    err = np.abs(got - ref)
    print(f"\nsign {sign}: finite bound on {fin.mean():.3f} of the voxels; max err/bound "
          f"{np.max(err[fin] / np.maximum(E[fin], 1e-300)):.3e}")
    assert fin.mean() > 0.9
    assert (err[fin] <= E[fin]).all()
    # the band where FP32 in the kernel's order meets the bar: a few mm, and some voxels stay
    d = fp32_bounds.band_for_bar(proj, P32, BOX, VS, origin, SC_INSIDE.sid, ref, 1e-5)
    pts = closed.voxel_centres(max(BOX), VS, origin, block=((0, BOX[2]), (0, BOX[1]), (0, BOX[0])))
    keep = fp32_bounds.min_source_distance(P32, pts, SC_INSIDE.sid) > d
    print(f"band {d} mm keeps {keep.mean():.3f}")
    assert d is not None and 1 <= d <= 20 and keep.mean() > 0.25
    dd = got[keep] - ref[keep]
    assert np.linalg.norm(dd) <= 0.5e-5 * np.linalg.norm(ref[keep])


def test_bound_catches_a_wrong_tap(inside_case):
    proj, P32, origin, ref, E, S = inside_case
    bad = fp32_bounds.emulate_fp32(proj, P32, BOX, VS, origin, swap_taps=True)
    fin = np.isfinite(E)
    assert (np.abs(bad - ref)[fin] > E[fin]).mean() > 0.05
