"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each pin takes a loaded oracle library and raises AssertionError on a
mismatch, so the same pins run against the real oracle (``test_oracle_pins``)
and against deliberately broken copies of it (``test_oracle_mutants``).

The back projection is the RabbitCT reference of Hofmann et al., WPMVP'14,
Sec. 4.1 (Listing 1).  Pins:
  handworked     values worked out by hand from the definition (tests/golden)
  tent           four-tap interpolant == brute-force double sum of pixel * tent * tent
  bruteforce     whole back projection == exact rational evaluation on tiny inputs
  constant       constant image: closed form sum c * ramp(s) * ramp(t) / w^2
  affine         affine image: interior closed form sum (a + b s + c t) / w^2
  impulse        single-pixel image: sum tent(s - i*) tent(t - j*) / w^2
  orthographic   w = 1, integer positions: V[z,y,x] = sum_k I_k[y][x], bit-exact
  invariants     linearity, view additivity, P -> 2P gives V/4, origin shift, w < 0 gives 0
"""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np

import oracle
from oracle import closed, geometry

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "bilinear_handworked.txt")


def read_golden(path=GOLDEN):
    image = None
    interps = []
    volumes = []
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            kind, *vals = line.split()
            if kind == "image":
                H, W = int(vals[0]), int(vals[1])
                image = np.array([float(v) for v in vals[2:]], dtype=np.float32).reshape(H, W)
            elif kind == "interp":
                interps.append(tuple(float(v) for v in vals))
            elif kind == "volume":
                L = int(vals[0])
                vs = float(vals[1])
                origin = [float(v) for v in vals[2:5]]
                P = np.array([float(v) for v in vals[5:17]]).reshape(1, 3, 4)
                expect = np.array([float(v) for v in vals[17:]]).reshape(L, L, L)
                volumes.append((L, vs, origin, P, expect))
    return image, interps, volumes


# A small circular scan with the proportions of the paper's C-arm workload
# (SID 800, SDD 1200, 200 degree arc) but a 48 x 40 detector whose pitch is
# scaled so a 256 mm field of view still fits partly on it.
SMALL_SCAN = dict(sid=800.0, sdd=1200.0, pitch=6.0, W=48, H=40)


def small_scan(n_views=7, arc_deg=200.0):
    angles = np.deg2rad(arc_deg) / n_views * np.arange(n_views)
    P = geometry.circular_matrices(angles, **SMALL_SCAN)
    return angles, P


def _P32(P):
    """The FP32 matrices a GPU consumes, widened back to FP64."""
    return np.asarray(P, dtype=np.float32).astype(np.float64)


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def pin_handworked(lib):
    image, interps, volumes = read_golden()
    for s, t, expect in interps:
        got = oracle.interpolate(image, s, t, lib=lib)
        assert got == expect, f"interp({s},{t}) = {got}, hand-worked {expect}"
    for L, vs, origin, P, expect in volumes:
        proj = image[None]
        got = oracle.backproject(proj, P, L, vs, origin, lib=lib)
        assert np.array_equal(got, expect), f"hand-worked volume mismatch: {got.ravel()} vs {expect.ravel()}"


def pin_tent(lib):
    rng = np.random.default_rng(11)
    img = rng.integers(-9, 10, size=(4, 5)).astype(np.float32)
    pts = [(Fraction(int(a), 8), Fraction(int(b), 8)) for a, b in rng.integers(-24, 48, size=(160, 2))]
    pts += [(Fraction(-1), Fraction(1)), (Fraction(-1, 2), Fraction(3, 2)), (Fraction(4), Fraction(0)),
            (Fraction(5), Fraction(3)), (Fraction(9, 2), Fraction(7, 2)), (Fraction(0), Fraction(-1, 4))]
    for s, t in pts:
        want = oracle.tent_interpolate(img, s, t)
        got = oracle.interpolate(img, float(s), float(t), lib=lib)
        assert Fraction(got) == want, f"interp({s},{t}) = {got} vs tent sum {float(want)}"


def _bruteforce_volume(proj, P, L, vs, origin):
    """Exact rational back projection: tent sums, exact division, w > 0 rule."""
    n = proj.shape[0]
    P = [[[Fraction(float(P[k, r, c])) for c in range(4)] for r in range(3)] for k in range(n)]
    o = [Fraction(float(x)) for x in origin]
    vsf = Fraction(float(vs))
    out = np.zeros((L, L, L))
    for z in range(L):
        for y in range(L):
            for x in range(L):
                X = (o[0] + vsf * x, o[1] + vsf * y, o[2] + vsf * z, Fraction(1))
                acc = Fraction(0)
                for k in range(n):
                    u, v, w = (sum(P[k][r][c] * X[c] for c in range(4)) for r in range(3))
                    if w <= 0:
                        continue
                    acc += oracle.tent_interpolate(proj[k], u / w, v / w) / (w * w)
                out[z, y, x] = float(acc)
    return out


def pin_bruteforce(lib):
    rng = np.random.default_rng(5)
    n, H, W, L = 3, 6, 7, 3
    proj = rng.uniform(-1, 1, size=(n, H, W)).astype(np.float32)
    # random perspective matrices that spread the 3^3 voxels over and past the detector
    P = np.zeros((n, 3, 4))
    for k in range(n):
        P[k, 0] = [rng.uniform(0.8, 2.2), rng.uniform(-0.6, 0.6), rng.uniform(-0.4, 0.4), rng.uniform(-1.5, 1.0)]
        P[k, 1] = [rng.uniform(-0.6, 0.6), rng.uniform(0.8, 2.0), rng.uniform(-0.4, 0.4), rng.uniform(-1.5, 1.0)]
        P[k, 2] = [rng.uniform(-0.05, 0.05), rng.uniform(-0.05, 0.05), rng.uniform(-0.05, 0.05), rng.uniform(0.6, 1.2)]
    P = _P32(P)
    origin = (-0.5, -0.25, 0.5)
    want = _bruteforce_volume(proj, P, L, 1.25, origin)
    got = oracle.backproject(proj, P, L, 1.25, origin, lib=lib, threads=2)
    assert _rel(got, want) < 1e-13, f"brute force mismatch {_rel(got, want)}"
    # a view behind the source (w < 0 for every voxel) adds nothing
    Pn = P.copy()
    Pn[1] *= -1.0
    want_n = _bruteforce_volume(proj, Pn, L, 1.25, origin)
    got_n = oracle.backproject(proj, Pn, L, 1.25, origin, lib=lib, threads=2)
    assert _rel(got_n, want_n) < 1e-13


def pin_constant(lib):
    _, P = small_scan()
    P = _P32(P)
    L, vs = 12, 256.0 / 12
    origin = [-(L - 1) / 2 * vs] * 3
    c = 0.75
    proj = np.full((P.shape[0], SMALL_SCAN["H"], SMALL_SCAN["W"]), c, dtype=np.float32)
    got = oracle.backproject(proj, P, L, vs, origin, lib=lib)
    want = closed.constant_image(P, c, SMALL_SCAN["W"], SMALL_SCAN["H"], L, vs, origin)
    assert _rel(got, want) < 1e-12, f"constant image {_rel(got, want)}"
    assert (want > 0).any() and (want == 0).any(), "scan must cover on- and off-detector voxels"


def pin_affine(lib):
    _, P = small_scan()
    P = _P32(P)
    W, H = SMALL_SCAN["W"], SMALL_SCAN["H"]
    L, vs = 10, 160.0 / 10
    origin = [-(L - 1) / 2 * vs] * 3
    a, b, c = 0.5, -0.125, 0.0625
    j, i = np.mgrid[0:H, 0:W]
    img = (a + b * i + c * j).astype(np.float32)
    proj = np.broadcast_to(img, (P.shape[0], H, W)).copy()
    got = oracle.backproject(proj, P, L, vs, origin, lib=lib)
    want, mask = closed.affine_image(P, a, b, c, W, H, L, vs, origin)
    assert mask.sum() > 50
    assert _rel(got[mask], want[mask]) < 1e-12, f"affine image {_rel(got[mask], want[mask])}"


def pin_impulse(lib):
    _, P = small_scan(n_views=5)
    P = _P32(P)
    W, H = SMALL_SCAN["W"], SMALL_SCAN["H"]
    L, vs = 14, 256.0 / 14
    origin = [-(L - 1) / 2 * vs] * 3
    for (i_star, j_star) in [(23, 19), (0, 7), (W - 1, 0), (5, H - 1), (0, 0)]:
        proj = np.zeros((P.shape[0], H, W), dtype=np.float32)
        proj[:, j_star, i_star] = 2.0
        got = oracle.backproject(proj, P, L, vs, origin, lib=lib)
        want = closed.impulse_image(P, i_star, j_star, W, H, L, vs, origin, amplitude=2.0)
        assert _rel(got, want) < 1e-12, f"impulse at ({i_star},{j_star}) {_rel(got, want)}"
        assert np.array_equal(got != 0, want != 0), "impulse support differs"


def pin_orthographic(lib):
    rng = np.random.default_rng(3)
    n, H, W, L, vs = 4, 9, 11, 8, 2.0
    origin = (-7.0, -7.0, -7.0)
    proj = rng.integers(0, 16, size=(n, H, W)).astype(np.float32)
    P = closed.orthographic_matrices(n, vs, origin)
    got = oracle.backproject(proj, P, L, vs, origin, lib=lib)
    want = closed.orthographic_volume(proj, L)
    assert np.array_equal(got, want), "orthographic identity not exact"


def pin_invariants(lib):
    _, P = small_scan(n_views=6)
    P = _P32(P)
    W, H = SMALL_SCAN["W"], SMALL_SCAN["H"]
    L, vs = 9, 22.0  # dyadic voxel size: shifted origins stay exact
    origin = [-(L - 1) / 2 * vs] * 3
    rng = np.random.default_rng(9)
    I1 = rng.uniform(-1, 1, size=(6, H, W)).astype(np.float32)
    I2 = rng.uniform(-1, 1, size=(6, H, W)).astype(np.float32)
    V1 = oracle.backproject(I1, P, L, vs, origin, lib=lib)
    V2 = oracle.backproject(I2, P, L, vs, origin, lib=lib)
    # linearity in the images (exact inputs: 2*I2 and I1 + 2*I2 rounded once)
    I3 = (I1.astype(np.float64) + 2.0 * I2.astype(np.float64))
    V3 = oracle.backproject(I3.astype(np.float32), P, L, vs, origin, lib=lib)
    assert _rel(V3, V1 + 2 * V2) < 1e-6  # I3 is rounded to FP32 once
    # additivity over views: a split run, accumulated, equals one run
    Va = oracle.backproject(I1[:2], P[:2], L, vs, origin, lib=lib)
    Vb = oracle.backproject(I1[2:], P[2:], L, vs, origin, vol=Va, lib=lib)
    assert _rel(Vb, V1) < 1e-13
    # P -> 2P: same positions, weight / 4, exact in binary floating point
    V4 = oracle.backproject(I1, 2.0 * P, L, vs, origin, lib=lib)
    assert np.array_equal(V4 * 4.0, V1)
    # origin shifted by one voxel along z == the block shifted by one plane
    o2 = [origin[0], origin[1], origin[2] + vs]
    Vs = oracle.backproject(I1, P, L, vs, o2, block=((0, L), (0, L), (0, L - 1)), lib=lib)
    assert np.array_equal(Vs, V1[1:])
    # a block of the volume equals the same voxels of the whole volume
    Vblk = oracle.backproject(I1, P, L, vs, origin, block=((2, 7), (1, 9), (3, 5)), lib=lib)
    assert np.array_equal(Vblk, V1[3:5, 1:9, 2:7])
    # view order permuted: same sum up to rounding
    perm = rng.permutation(6)
    Vp = oracle.backproject(I1[perm], P[perm], L, vs, origin, lib=lib)
    assert _rel(Vp, V1) < 1e-13
    # matrices that put every voxel behind the source (w < 0) contribute nothing
    Vneg = oracle.backproject(I1, -P, L, vs, origin, lib=lib)
    assert not Vneg.any() and V1.any()
    # thread count does not change the result
    Vt = oracle.backproject(I1, P, L, vs, origin, lib=lib, threads=1)
    assert np.array_equal(Vt, V1)


ALL_PINS = [pin_handworked, pin_tent, pin_bruteforce, pin_constant, pin_affine, pin_impulse,
            pin_orthographic, pin_invariants]


def pin_points_equal_blocks(lib):
    """The voxel-list entry computes exactly what the block entry computes for the same voxels."""
    _, P = small_scan(n_views=4)
    P = _P32(P)
    L, vs = 11, 20.0
    origin = [-(L - 1) / 2 * vs] * 3
    rng = np.random.default_rng(12)
    proj = rng.uniform(-1, 1, size=(4, SMALL_SCAN["H"], SMALL_SCAN["W"])).astype(np.float32)
    V = oracle.backproject(proj, P, L, vs, origin, lib=lib)
    xyz = rng.integers(0, L, size=(50, 3))
    got = oracle.backproject_points(proj, P, vs, origin, xyz, lib=lib)
    assert np.array_equal(got, V[xyz[:, 2], xyz[:, 1], xyz[:, 0]])


ALL_PINS.append(pin_points_equal_blocks)


def pin_absolute(lib):
    """The magnitude mode adds |contribution| of every view: the sum of the single-view
    magnitudes, equal to the back projection itself for non-negative images, unchanged when the
    images change sign, never below |V| and above it where signed contributions cancel; the
    voxel-list entry agrees with the block entry."""
    _, P = small_scan(n_views=5)
    P = _P32(P)
    W, H = SMALL_SCAN["W"], SMALL_SCAN["H"]
    L, vs = 9, 22.0
    origin = [-(L - 1) / 2 * vs] * 3
    rng = np.random.default_rng(21)
    I = rng.uniform(-1, 1, size=(5, H, W)).astype(np.float32)
    V = oracle.backproject(I, P, L, vs, origin, lib=lib)
    A = oracle.backproject(I, P, L, vs, origin, lib=lib, absolute=True)
    singles = [np.abs(oracle.backproject(I[k:k + 1], P[k:k + 1], L, vs, origin, lib=lib)) for k in range(5)]
    want = np.zeros_like(A)
    for a in singles:  # the same order of additions as the oracle's views
        want = want + a
    assert np.array_equal(A, want), "magnitude mode is not the sum of single-view magnitudes"
    assert np.array_equal(oracle.backproject(-I, P, L, vs, origin, lib=lib, absolute=True), A)
    assert (A >= np.abs(V)).all() and (A > np.abs(V) * (1 + 1e-9)).any()
    Ipos = np.abs(I)
    assert np.array_equal(oracle.backproject(Ipos, P, L, vs, origin, lib=lib, absolute=True),
                          oracle.backproject(Ipos, P, L, vs, origin, lib=lib))
    xyz = rng.integers(0, L, size=(40, 3))
    got = oracle.backproject_points(I, P, vs, origin, xyz, lib=lib, absolute=True)
    assert np.array_equal(got, A[xyz[:, 2], xyz[:, 1], xyz[:, 0]])


ALL_PINS.append(pin_absolute)
