"""Closed-form back projections used to pin the oracle -- TEST INFRASTRUCTURE.

For special images the bilinear interpolant of the zero-extended image
(Hofmann et al., WPMVP'14, Sec. 4.1, Listing 1) has a closed form, so the
whole back projection sum_k B_k(u/w, v/w) / w^2 can be written without any
taps, floors or fractions.  These functions evaluate those closed forms in
FP64 with numpy; they share nothing with the four-tap code of the oracle
except the affine map (u, v, w) = P (X, 1), which is pinned on its own by
ray/plane intersection in ``geometry``.
"""
from __future__ import annotations

import numpy as np


def voxel_centres(L, voxel_size, origin, block=None):
    """World coordinates (nz, ny, nx, 3) of the voxel centres of a block."""
    if block is None:
        block = ((0, L), (0, L), (0, L))
    (x0, x1), (y0, y1), (z0, z1) = block
    o = np.asarray(origin, dtype=np.float64)
    xs = o[0] + voxel_size * np.arange(x0, x1, dtype=np.float64)
    ys = o[1] + voxel_size * np.arange(y0, y1, dtype=np.float64)
    zs = o[2] + voxel_size * np.arange(z0, z1, dtype=np.float64)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def _stw(P, pts):
    P = np.asarray(P, dtype=np.float64).reshape(-1, 3, 4)
    u = np.einsum("kc,...c->k...", P[:, 0, :3], pts) + P[:, 0, 3].reshape(-1, *([1] * (pts.ndim - 1)))
    v = np.einsum("kc,...c->k...", P[:, 1, :3], pts) + P[:, 1, 3].reshape(-1, *([1] * (pts.ndim - 1)))
    w = np.einsum("kc,...c->k...", P[:, 2, :3], pts) + P[:, 2, 3].reshape(-1, *([1] * (pts.ndim - 1)))
    with np.errstate(divide="ignore", invalid="ignore"):
        return u / w, v / w, w


def edge_ramp(s, n):
    """Interpolant of a constant-1 row of n pixels, zero outside: a trapezoid.

    1 on [0, n-1], falling linearly to 0 at -1 and at n, 0 beyond.
    """
    return np.clip(np.minimum(s + 1.0, n - s), 0.0, 1.0)


def constant_image(P, c, W, H, L, voxel_size, origin, block=None):
    """V for images that all equal c on the detector: sum_k c * ramp_W(s) * ramp_H(t) / w^2 (w > 0)."""
    pts = voxel_centres(L, voxel_size, origin, block)
    s, t, w = _stw(P, pts)
    ok = w > 0
    with np.errstate(divide="ignore", invalid="ignore"):
        val = np.where(ok, c * edge_ramp(s, W) * edge_ramp(t, H) / (w * w), 0.0)
    return val.sum(axis=0)


def affine_image(P, a, b, c, W, H, L, voxel_size, origin, block=None):
    """V for I[j][i] = a + b*i + c*j, and the mask of voxels where it is exact.

    Where every view puts the voxel inside [0, W-1] x [0, H-1] (and w > 0) the
    interpolant reproduces the affine function exactly, so
    V = sum_k (a + b s_k + c t_k) / w_k^2.  Returns (V, mask).
    """
    pts = voxel_centres(L, voxel_size, origin, block)
    s, t, w = _stw(P, pts)
    inside = (w > 0) & (s >= 0) & (s <= W - 1) & (t >= 0) & (t <= H - 1)
    with np.errstate(divide="ignore", invalid="ignore"):
        val = np.where(inside, (a + b * s + c * t) / (w * w), 0.0)
    return val.sum(axis=0), inside.all(axis=0)


def tent(r):
    return np.maximum(0.0, 1.0 - np.abs(r))


def impulse_image(P, i_star, j_star, W, H, L, voxel_size, origin, block=None, amplitude=1.0):
    """V for images with a single non-zero pixel (i*, j*): sum_k A tent(s-i*) tent(t-j*) / w^2."""
    pts = voxel_centres(L, voxel_size, origin, block)
    s, t, w = _stw(P, pts)
    ok = w > 0
    with np.errstate(divide="ignore", invalid="ignore"):
        val = np.where(ok, amplitude * tent(s - i_star) * tent(t - j_star) / (w * w), 0.0)
    return val.sum(axis=0)


def orthographic_matrices(n_views, voxel_size, origin):
    """Matrices with w = 1, u/w = x index, v/w = y index of the voxel (orthographic identity).

    Under these matrices voxel (x, y, z) lands exactly on pixel (x, y) of every
    view with zero fractions and unit weight, so V[z, y, x] = sum_k I_k[y][x].
    """
    o = np.asarray(origin, dtype=np.float64)
    P = np.zeros((n_views, 3, 4))
    P[:, 0, 0] = 1.0 / voxel_size
    P[:, 0, 3] = -o[0] / voxel_size
    P[:, 1, 1] = 1.0 / voxel_size
    P[:, 1, 3] = -o[1] / voxel_size
    P[:, 2, 3] = 1.0
    return P


def orthographic_volume(proj, L):
    """V[z, y, x] = sum_k I_k[y][x] for x, y < L (requires L <= W and L <= H)."""
    s = np.asarray(proj, dtype=np.float64).sum(axis=0)[:L, :L]
    return np.broadcast_to(s, (L, L, L)).copy()
