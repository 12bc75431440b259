"""FDK pre-processing of cone-beam projections, FP64 -- TEST INFRASTRUCTURE.

The back projection of Hofmann et al. (WPMVP'14, Sec. 4.1) consumes projections
that have already been weighted and filtered (Sec. 4 describes the RabbitCT
input as filtered, weighted projection images).  The paper does not spell the
two steps out; this module follows the standard Feldkamp-Davis-Kress
pre-processing, with these readings:

  weight   each pixel is multiplied by the cosine of the angle between its ray
           and the principal ray, SDD / sqrt(SDD^2 + u^2 + v^2), where (u, v)
           are the pixel's offsets (mm) from the detector centre along the
           column and row axes; pixel (i, j) has u = (i - (W-1)/2) * pitch and
           v = (j - (H-1)/2) * pitch.
  filter   every detector row is convolved with the discrete band-limited
           ramp (Ram-Lak) kernel of Kak and Slaney, h(0) = 1/(4 tau^2),
           h(n) = -1/(pi n tau)^2 for odd n, h(n) = 0 for even n != 0, where
           tau = pitch * SID / SDD is the pixel spacing scaled to the
           isocentre; the result is scaled by tau (the quadrature weight of
           the convolution integral).  The convolution is linear: samples
           beyond either end of the row are zero.

So, for view k, row j and column i,

    q[k, j, i] = tau * sum_{m=0}^{W-1} h(i - m) * c[j, m] * p[k, j, m].

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module.  It shares no code with the GPU library.
The functions are the definition written out: the convolution is one dense
product with the Toeplitz matrix T[m, i] = h(i - m).
"""
from __future__ import annotations

import numpy as np


def isocentre_spacing(pitch: float, sid: float, sdd: float) -> float:
    """tau: the detector pixel pitch scaled to the isocentre (magnification SDD / SID)."""
    return pitch * sid / sdd


def cosine_weights(W: int, H: int, pitch: float, sdd: float) -> np.ndarray:
    """(H, W) weights SDD / sqrt(SDD^2 + u^2 + v^2) of the pixel centres."""
    u = (np.arange(W, dtype=np.float64) - (W - 1) / 2.0) * pitch
    v = (np.arange(H, dtype=np.float64) - (H - 1) / 2.0) * pitch
    return sdd / np.sqrt(sdd * sdd + u[None, :] ** 2 + v[:, None] ** 2)


def ramp_taps(n, tau: float) -> np.ndarray:
    """h(n) of the discrete Ram-Lak kernel for integer offsets n (any shape)."""
    n = np.asarray(n, dtype=np.int64)
    h = np.zeros(n.shape, dtype=np.float64)
    h[n == 0] = 1.0 / (4.0 * tau * tau)
    odd = (np.abs(n) % 2) == 1
    nf = n[odd].astype(np.float64)
    h[odd] = -1.0 / (np.pi * np.pi * nf * nf * tau * tau)
    return h


def ramp_matrix(W: int, tau: float) -> np.ndarray:
    """(W, W) Toeplitz matrix T[m, i] = h(i - m): row-vector times T convolves a row."""
    m = np.arange(W)
    return ramp_taps(m[None, :] - m[:, None], tau)


def ramp_filter_rows(x: np.ndarray, tau: float) -> np.ndarray:
    """tau * sum_m h(i - m) x[..., m] along the last axis (linear convolution, zeros beyond the row)."""
    x = np.asarray(x, dtype=np.float64)
    return tau * (x @ ramp_matrix(x.shape[-1], tau))


def fdk_filter(p: np.ndarray, pitch: float, sid: float, sdd: float) -> np.ndarray:
    """Weighted, ramp-filtered projections (N, H, W) in FP64 from raw projections (N, H, W)."""
    p = np.asarray(p, dtype=np.float64)
    _, H, W = p.shape
    tau = isocentre_spacing(pitch, sid, sdd)
    return ramp_filter_rows(p * cosine_weights(W, H, pitch, sdd)[None], tau)


def fdk_filter_rows(p: np.ndarray, rows, pitch: float, sid: float, sdd: float) -> np.ndarray:
    """The same for selected (view, row) pairs of a large stack: returns (len(rows), W)."""
    p = np.asarray(p)
    _, H, W = p.shape
    tau = isocentre_spacing(pitch, sid, sdd)
    c = cosine_weights(W, H, pitch, sdd)
    rows = list(rows)
    x = np.stack([p[k, j].astype(np.float64) * c[j] for k, j in rows])
    return ramp_filter_rows(x, tau)
