"""Projection matrices of a circular cone-beam trajectory, FP64 -- TEST INFRASTRUCTURE.

Each view of RabbitCT carries a 3x4 matrix A_i that maps a homogeneous world
point to homogeneous detector coordinates (Hofmann et al., WPMVP'14, Sec. 4 and
Sec. 4.1): (u, v, w) = A_i (X, 1), detector position (u/w, v/w).  The paper's
dataset supplies these matrices; here they are composed from a circular orbit
so that synthetic workloads have the same structure.

Trajectory convention (angle theta per view, distances in mm):
  source            S = SID * (cos t, sin t, 0)
  detector centre   D = -(SDD - SID) * (cos t, sin t, 0)
  principal ray     n = -(cos t, sin t, 0)          unit, source -> detector
  detector axes     e_u = (-sin t, cos t, 0)  (columns, index i)
                    e_v = (0, 0, 1)           (rows,    index j)
  pixel (i, j)      D + (i - c_u) * pitch * e_u + (j - c_v) * pitch * e_v,
                    c_u = (W - 1) / 2, c_v = (H - 1) / 2  (integer index = pixel centre)

The matrix is scaled so that w = n . (X - S) / SID: the depth of X along the
principal ray in units of SID, so w = 1 at the isocentre and 1/w^2 is the
inverse-square weight of Listing 1.
"""
from __future__ import annotations

import numpy as np


def frame(theta: float, sid: float, sdd: float):
    """Source, detector centre, principal ray and detector axes for one view."""
    c, s = np.cos(theta), np.sin(theta)
    S = sid * np.array([c, s, 0.0])
    D = -(sdd - sid) * np.array([c, s, 0.0])
    n = -np.array([c, s, 0.0])
    e_u = np.array([-s, c, 0.0])
    e_v = np.array([0.0, 0.0, 1.0])
    return S, D, n, e_u, e_v


def circular_matrices(angles, sid, sdd, pitch, W, H) -> np.ndarray:
    """(N, 3, 4) FP64 matrices of the pinhole projection, written from its definition.

    A point X hits the detector plane at Q = S + (X - S) * SDD / d with
    d = n . (X - S).  Its column index is i = c_u + e_u . (Q - D) / pitch; since
    e_u . (S - D) = 0 this is i = c_u + (SDD / pitch) e_u . (X - S) / d.  With
    w = d / SID, u = i * w is affine in X:
        u = ((SDD/pitch) e_u + c_u n) . (X - S) / SID
        v = ((SDD/pitch) e_v + c_v n) . (X - S) / SID
        w = n . (X - S) / SID
    """
    cu, cv = (W - 1) / 2.0, (H - 1) / 2.0
    f = sdd / pitch
    out = np.zeros((len(angles), 3, 4), dtype=np.float64)
    for k, th in enumerate(angles):
        S, _D, n, e_u, e_v = frame(th, sid, sdd)
        rows = [f * e_u + cu * n, f * e_v + cv * n, n]
        for r, a in enumerate(rows):
            out[k, r, :3] = a / sid
            out[k, r, 3] = -np.dot(a, S) / sid
    return out


def project_by_intersection(angles, sid, sdd, pitch, W, H, X):
    """Detector position and depth of world points by explicit ray/plane intersection.

    Solves S + lam (X - S) = D + a e_u + b e_v for (lam, a, b) with a 3x3
    linear solve per point and view, independently of the matrix composition.
    Returns (s, t, w) arrays of shape (N, M) for M points: s = c_u + a/pitch,
    t = c_v + b/pitch, w = n.(X - S)/SID.
    """
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    cu, cv = (W - 1) / 2.0, (H - 1) / 2.0
    N, M = len(angles), X.shape[0]
    s = np.empty((N, M))
    t = np.empty((N, M))
    w = np.empty((N, M))
    for k, th in enumerate(angles):
        S, D, n, e_u, e_v = frame(th, sid, sdd)
        for m in range(M):
            A = np.stack([X[m] - S, -e_u, -e_v], axis=1)
            lam, a, b = np.linalg.solve(A, D - S)
            s[k, m] = cu + a / pitch
            t[k, m] = cv + b / pitch
            w[k, m] = np.dot(n, X[m] - S) / sid
    return s, t, w


def apply(P, X):
    """(u/w, v/w, w) of world points X (M, 3) under matrices P (N, 3, 4), FP64."""
    P = np.asarray(P, dtype=np.float64).reshape(-1, 3, 4)
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    Xh = np.concatenate([X, np.ones((X.shape[0], 1))], axis=1)
    uvw = np.einsum("krc,mc->krm", P, Xh)
    return uvw[:, 0] / uvw[:, 2], uvw[:, 1] / uvw[:, 2], uvw[:, 2]
