"""Per-voxel bound on the error of an FP32 evaluation of the back projection.

The back projection of Sec. 4.1 (voxel -> (u, v, w) = P (X, 1), bilinear
interpolant at (u/w, v/w) of the zero-extended image, weight 1/w^2,
accumulate) is evaluated by the GPU in FP32 and by the oracle in FP64 on the
same FP32 inputs.  Near the source plane (w -> 0) the weight 1/w^2 amplifies
the rounding of w without limit, so a relative-L2 bar over a box that holds
the source cannot be met there by any FP32 evaluation.  This module derives,
from the standard rounding-error model (each FP32 operation rounds with
relative error at most U = 2^-24; the hardware reciprocal with at most 2U), an
upper bound E on |V_fp32 - V_exact| for every voxel, so that a test can

  * check every voxel against its own bound (an element-wise gate), and
  * apply the relative-L2 bar exactly where the bound shows FP32 can meet it,
    instead of on a hand-picked distance from the source.

Model, per view k and voxel X (first order in U):
  |du| <= g (|P00 X| + |P01 Y| + |P02 Z| + |P03|)       g = 8 U (X rounded, products, sums)
  |dv|, |dw| likewise with rows 1 and 2
  w within 2 |dw| of 0: the sign of w may flip (contribution 0 or 1/w^2-large): E = inf
  (also E = inf where |ds| or |dt| >= 1/2 or |dr| / r >= 1/4: outside the first-order model)
  r = 1/w:           |dr| / r <= |dw| / |w| + 2 U
  s = u r (+1):      |ds| <= |du| r + |s| |dr| / r + U (|s| + 2)     likewise t
  B(s, t):           Lipschitz in s and t with constant <= 2 M, M = max |pixel| of the 4 x 4
                     pixels around (floor s, floor t) (zero off the detector; |ds|, |dt| < 1);
                     its evaluation from four taps rounds by at most 16 U M
  c = B r^2:         |dc| <= (2 M (|ds| + |dt|) + 16 U M) r^2 + M r^2 (2 |dr| / r + 2 U)
  V = sum_k c_k:     plus (N + 2) U sum_k M_k r_k^2 for the FP32 summation.
The bound is a worst case (about 1000 times the typical error), so it serves
as the element-wise gate; where the relative-L2 bar applies near the source
is found from an FP32 emulation of the fused pass (``emulate_fp32``, every
operation rounded to FP32 in the kernel's order): the smallest distance from
the source plane beyond which that emulation meets half the bar
(``band_for_bar``).  Only test infrastructure uses this module.
"""
from __future__ import annotations

import numpy as np

U = 2.0 ** -24
GAMMA = 8.0 * U


def _local_max(img: np.ndarray) -> np.ndarray:
    """M[j + 1, i + 1] = max |img| over rows j-1..j+2 and columns i-1..i+2 (zero-extended), for
    j in -1..H-1 and i in -1..W-1 (the window of a position with floor (i, j))."""
    a = np.abs(np.asarray(img, dtype=np.float64))
    H, W = a.shape
    p = np.zeros((H + 5, W + 5))
    p[2:H + 2, 2:W + 2] = a  # p[j + 2, i + 2] = |img[j, i]|
    # rows j-1..j+2 of the image are p rows j+1..j+4; index j+1 in 0..H: start rows 0..H
    rows = np.maximum.reduce([p[d:d + H + 1, :] for d in range(4)])
    return np.maximum.reduce([rows[:, d:d + W + 1] for d in range(4)])


def error_bound(proj, P32, pts) -> tuple[np.ndarray, np.ndarray]:
    """(E, S) for voxels at world positions pts (..., 3): E bounds |V_fp32 - V_exact| (inf where
    some view may put the voxel on the wrong side of the source plane); S = sum_k M_k / w_k^2 is
    the magnitude scale of the voxel's contributions (E <= 1e-5 S: FP32 can meet a 1e-5 bar)."""
    proj = np.asarray(proj, dtype=np.float32)
    n, H, W = proj.shape
    P = np.asarray(P32, dtype=np.float32).astype(np.float64).reshape(n, 3, 4)
    pts = np.asarray(pts, dtype=np.float64)
    shape = pts.shape[:-1]
    X = pts.reshape(-1, 3)
    E = np.zeros(X.shape[0])
    S = np.zeros(X.shape[0])
    for k in range(n):
        M4 = _local_max(proj[k])
        rows = []
        for r in range(3):
            val = X @ P[k, r, :3] + P[k, r, 3]
            scale = np.abs(X) @ np.abs(P[k, r, :3]) + abs(P[k, r, 3])
            rows.append((val, GAMMA * scale))
        (u, du), (v, dv), (w, dw) = rows
        flip = np.abs(w) <= 2.0 * dw
        front = (w > 2.0 * dw)
        E[flip] = np.inf
        if not front.any():
            continue
        wf, uf, vf = w[front], u[front], v[front]
        r = 1.0 / wf
        drr = dw[front] / wf + 2.0 * U
        s, t = uf * r, vf * r
        ds = du[front] * r + np.abs(s) * drr + U * (np.abs(s) + 2.0)
        dt = dv[front] * r + np.abs(t) * drr + U * (np.abs(t) + 2.0)
        # window of the position (floor in -1..W-1 / -1..H-1; beyond that every tap is 0)
        i0 = np.floor(np.clip(s, -3.0, W + 2.0)).astype(np.int64)
        j0 = np.floor(np.clip(t, -3.0, H + 2.0)).astype(np.int64)
        inside = (i0 >= -1) & (i0 <= W - 1) & (j0 >= -1) & (j0 <= H - 1)
        M = np.zeros(wf.shape)
        M[inside] = M4[j0[inside] + 1, i0[inside] + 1]
        # a position just outside the window range can still reach the detector's edge pixels
        near = ~inside & (s > -3.0) & (s < W + 2.0) & (t > -3.0) & (t < H + 2.0)
        if near.any():
            ic = np.clip(i0[near], -1, W - 1)
            jc = np.clip(j0[near], -1, H - 1)
            M[near] = M4[jc + 1, ic + 1]
        r2 = r * r
        e = (2.0 * M * (ds + dt) + 16.0 * U * M) * r2 + M * r2 * (2.0 * drr + 2.0 * U)
        e[(ds >= 0.5) | (dt >= 0.5) | (drr >= 0.25)] = np.inf  # beyond the first-order model
        E[front] += e
        S[front] += M * r2
    E += (n + 2) * U * S
    return E.reshape(shape), S.reshape(shape)


def _f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def _fma(a, b, c):
    # products of FP32 values are exact in FP64; one rounding to FP32 after the sum
    return _f32(np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64))


def emulate_fp32(proj, P32, shape, vs, origin, swap_taps=False):
    """The guarded branch of the fused pass in FP32 (every operation rounded), views in order."""
    proj = np.asarray(proj, dtype=np.float32)
    n, H, W = proj.shape
    P = np.asarray(P32, dtype=np.float32).astype(np.float64).reshape(n, 3, 4)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = _fma(vs, x, origin[0])
    Y = _fma(vs, y, origin[1])
    Z = _fma(vs, z, origin[2])
    acc = np.zeros(shape)
    for k in range(n):
        pad = np.zeros((H + 3, W + 3))
        pad[1:H + 1, 1:W + 1] = proj[k]
        a = pad[:-1, :-1]
        b = pad[:-1, 1:]
        c = pad[1:, :-1]
        d = pad[1:, 1:]
        if swap_taps:
            b, c = c, b
        dx = _f32(b - a)
        dx2 = _f32(d - c)
        p = P[k]
        uu = _fma(p[0, 2], Z, _fma(p[0, 1], Y, _fma(p[0, 0], X, p[0, 3])))
        vv = _fma(p[1, 2], Z, _fma(p[1, 1], Y, _fma(p[1, 0], X, p[1, 3])))
        ww = _fma(p[2, 2], Z, _fma(p[2, 1], Y, _fma(p[2, 0], X, p[2, 3])))
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            r = _f32(1.0 / ww)
            s = _fma(uu, r, 1.0)
            t = _fma(vv, r, 1.0)
        ok = (ww > 0) & (s > 0) & (s < W + 1) & (t > 0) & (t < H + 1)
        s = np.where(ok, s, 0.0)
        t = np.where(ok, t, 0.0)
        c0 = np.floor(s).astype(np.int64)
        r0 = np.floor(t).astype(np.int64)
        fx = _f32(s - c0)
        fy = _f32(t - r0)
        top = _fma(fx, dx[r0, c0], a[r0, c0])
        bot = _fma(fx, dx2[r0, c0], c[r0, c0])
        val = _fma(fy, _f32(bot - top), top)
        with np.errstate(invalid="ignore", over="ignore"):
            contrib = np.where(ok, _f32(val * _f32(r * r)), 0.0)
        acc = _f32(acc + contrib)
    return acc


def min_source_distance(P32, pts, sid):
    """Over all views, the smallest |w| SID (distance from the source plane in the normalised
    geometry, mm) of each voxel at world positions pts (..., 3)."""
    P = np.asarray(P32, dtype=np.float32).astype(np.float64).reshape(-1, 3, 4)
    w = np.einsum("kc,...c->k...", P[:, 2, :3], pts) + P[:, 2, 3].reshape(-1, *([1] * (pts.ndim - 1)))
    return (np.abs(w) * sid).min(axis=0)


def band_for_bar(proj, P32, shape, vs, origin, sid, ref, bar, grid=(1, 2, 3, 4, 6, 8, 10, 12, 15, 20, 25, 30)):
    """Smallest distance d (mm, from ``grid``) such that the FP32 emulation meets bar / 2 in
    relative L2 against ``ref`` (the FP64 oracle) over the voxels at least d from every view's
    source plane; None if no d of the grid does."""
    from oracle import closed

    nz, ny, nx = shape
    got = emulate_fp32(proj, P32, shape, vs, origin)
    pts = closed.voxel_centres(max(shape), vs, origin, block=((0, nx), (0, ny), (0, nz)))
    dist = min_source_distance(P32, pts, sid)
    for d in grid:
        keep = dist > d
        if not keep.any():
            return None
        den = np.linalg.norm(ref[keep])
        num = np.linalg.norm(got[keep] - ref[keep])
        if (den == 0 and num == 0) or (den > 0 and num <= 0.5 * bar * den):
            return d
    return None
