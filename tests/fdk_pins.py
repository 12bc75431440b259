"""Pins of the FP64 FDK pre-processing oracle (``oracle.fdk``).

Each pin takes a module with the interface of ``oracle.fdk`` and raises
AssertionError on a mismatch, so the same pins run against the real oracle
(``test_fdk_pins``) and against copies of it with planted mistakes.

The pre-processing produces the filtered, weighted projections that the back
projection of Hofmann et al., WPMVP'14 (Sec. 4) consumes: cosine weighting and
row-wise convolution with the discrete Ram-Lak kernel.  Pins:
  handworked   impulse and constant rows, and single weights, worked out by hand (tests/golden)
  geometry     weight == cosine of the angle between the pixel's ray and the principal
               ray, from the explicit source and pixel positions of the orbit
  spectrum     a sampled cosine of frequency omega comes out scaled by |omega| / (2 pi tau)
               (the frequency response of the kernel), within the exact bound of the
               taps that fall beyond the row
  fft          linear convolution == FFT circular convolution with zero padding to
               >= 2W - 1 samples (an independent library route)
  rows         the selected-rows entry equals the whole-stack entry
"""
from __future__ import annotations

import os

import numpy as np

from oracle import geometry

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fdk_handworked.txt")


def read_golden(path=GOLDEN):
    ramps, weights = [], []
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            kind, rest = line.split(None, 1)
            lhs, rhs = rest.split("->")
            a = [float(v) for v in lhs.split()]
            b = [float(v) for v in rhs.split()]
            if kind == "ramp":
                ramps.append((a[0], np.array(a[1:]), np.array(b)))
            elif kind == "weight":
                weights.append((int(a[0]), int(a[1]), a[2], a[3], int(a[4]), int(a[5]), b[0]))
    return ramps, weights


def pin_handworked(m):
    ramps, weights = read_golden()
    assert len(ramps) >= 4 and len(weights) >= 5
    for tau, x, want in ramps:
        got = m.ramp_filter_rows(x[None], tau)[0]
        assert np.allclose(got, want, rtol=0, atol=1e-15), (tau, x, got, want)
    for W, H, pitch, sdd, i, j, want in weights:
        got = m.cosine_weights(W, H, pitch, sdd)[j, i]
        assert abs(got - want) <= 1e-15, (W, H, i, j, got, want)


def pin_geometry(m):
    W, H, pitch, sid, sdd = 13, 9, 1.7, 800.0, 1200.0
    c = m.cosine_weights(W, H, pitch, sdd)
    cu, cv = (W - 1) / 2.0, (H - 1) / 2.0
    for theta in (0.0, 0.7, 2.9):
        S, D, n, e_u, e_v = geometry.frame(theta, sid, sdd)
        for j in range(H):
            for i in range(W):
                X = D + (i - cu) * pitch * e_u + (j - cv) * pitch * e_v
                r = X - S
                want = np.dot(n, r) / np.linalg.norm(r)
                assert abs(c[j, i] - want) <= 1e-14, (theta, i, j, c[j, i], want)


def _odd_tail(a):
    """Upper bound of sum over odd n >= a of 1/n^2 (exact head plus an integral bound)."""
    a = max(int(a), 1)
    if a % 2 == 0:
        a += 1
    head = sum(1.0 / (n * n) for n in range(a, a + 4000, 2))
    return head + 1.0 / (2.0 * (a + 4000 - 2))


def pin_spectrum(m):
    """tau * sum_n h(n) cos(omega (i - n) + phi) = |omega| / (2 pi tau) cos(omega i + phi) for |omega| <= pi.

    A row of W samples misses the taps with i - n outside [0, W); with |x| <= 1 their
    sum is at most tau * sum |h(n)| over those n, which the pin bounds exactly.
    """
    W = 1501
    i = np.arange(W)
    for tau in (1.0, 0.2133):
        for omega, phi in ((0.0, 0.0), (0.05, 0.3), (0.9, -1.1), (2.0, 0.5), (np.pi, 0.0)):
            x = np.cos(omega * i + phi)
            got = m.ramp_filter_rows(x[None], tau)[0]
            want = abs(omega) / (2.0 * np.pi * tau) * np.cos(omega * i + phi)
            for ii in (W // 4, W // 2, 3 * W // 4, W // 2 + 1):
                bound = (_odd_tail(ii + 1) + _odd_tail(W - ii)) / (np.pi * np.pi * tau) + 1e-12
                assert abs(got[ii] - want[ii]) <= bound, (tau, omega, ii, got[ii], want[ii], bound)
    # the same through the whole pre-processing: rows that are cosines after weighting,
    # with tau composed from pitch and the magnification SDD / SID
    pitch, sid, sdd, H = 0.32, 800.0, 1200.0, 3
    c = m.cosine_weights(W, H, pitch, sdd)
    omega = 1.3
    p = np.cos(omega * i)[None, None, :] / c[None]
    got = m.fdk_filter(p, pitch, sid, sdd)
    tau = pitch * sid / sdd
    want = omega / (2.0 * np.pi * tau) * np.cos(omega * i[W // 2])
    bound = (_odd_tail(W // 2 + 1) + _odd_tail(W - W // 2)) / (np.pi * np.pi * tau) + 1e-12
    assert np.all(np.abs(got[0, :, W // 2] - want) <= bound), (got[0, :, W // 2], want)


def pin_fft(m):
    rng = np.random.default_rng(20140301)
    for W in (1, 2, 37, 100):
        tau = 0.37
        x = rng.standard_normal((3, W))
        N = 1 << int(np.ceil(np.log2(max(2 * W - 1, 1))))
        N = max(N, 1)
        n = np.arange(-(W - 1), W)
        h = m.ramp_taps(n, tau)
        wrapped = np.zeros(N)
        wrapped[n % N] = h
        want = tau * np.real(np.fft.ifft(np.fft.fft(x, N) * np.fft.fft(wrapped)))[:, :W]
        got = m.ramp_filter_rows(x, tau)
        assert np.allclose(got, want, rtol=0, atol=1e-12 * max(1.0, np.abs(want).max())), W


def pin_rows(m):
    rng = np.random.default_rng(7)
    p = rng.standard_normal((3, 5, 21))
    full = m.fdk_filter(p, 0.5, 600.0, 900.0)
    rows = [(0, 0), (2, 4), (1, 3)]
    part = m.fdk_filter_rows(p.astype(np.float32), rows, 0.5, 600.0, 900.0)
    full32 = m.fdk_filter(p.astype(np.float32), 0.5, 600.0, 900.0)
    for r, (k, j) in enumerate(rows):
        assert np.allclose(part[r], full32[k, j], rtol=0, atol=1e-13), (k, j)
    assert np.abs(full - full32).max() < 1e-5  # only the input rounding differs


ALL_PINS = [pin_handworked, pin_geometry, pin_spectrum, pin_fft, pin_rows]
