"""Seeded synthetic inputs for back-projection workloads.

This module only makes input data: a circular scan description, a phantom
of random ellipsoids, its analytic cone-beam line integrals, the FDK
cosine weighting and ramp filtering that turn them into "filtered and
weighted" projections, noise, and storage rounding.  It holds none of the
back-projection arithmetic (no projection matrices, no interpolation, no
accumulation), so both the HIP path and the FP64 oracle can consume what it
makes.

The paper's workload (Hofmann et al., WPMVP'14, Sec. 4) is the RabbitCT
rabbit dataset: 496 filtered, weighted C-arm projections of 1248 x 960 FP32
pixels, one 3x4 matrix per view, reconstructed into 512^3 voxels.  That
dataset is not available here; the seeded phantom below stands in for it at
the same shapes and value structure (signed, edge-dominated filtered images
that are zero off the object).

Torch is used for the pixel arithmetic so that large stacks can be made on
the GPU; the random parameters come from numpy's PCG64 so a seed means the
same phantom on any device.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch


@dataclass(frozen=True)
class Scanner:
    """Circular cone-beam scan: angles, distances (mm) and detector size.

    Convention (shared by the product's and the oracle's matrix code, each
    written separately): source S = SID (cos t, sin t, 0); detector centre
    D = -(SDD - SID)(cos t, sin t, 0); detector columns along
    e_u = (-sin t, cos t, 0), rows along e_v = (0, 0, 1); pixel (i, j) centred
    at D + (i - (W-1)/2) pitch e_u + (j - (H-1)/2) pitch e_v.
    """

    n_views: int = 496
    arc_deg: float = 200.0
    start_deg: float = 0.0
    sid: float = 800.0
    sdd: float = 1200.0
    pitch: float = 0.32
    W: int = 1248
    H: int = 960

    def angles(self) -> np.ndarray:
        """theta_k = start + k * arc / N, k = 0 .. N-1 (radians, FP64)."""
        step = math.radians(self.arc_deg) / self.n_views
        return math.radians(self.start_deg) + step * np.arange(self.n_views, dtype=np.float64)

    def geometry_args(self):
        """(angles, sid, sdd, pitch, W, H) in the order the matrix builders take them."""
        return self.angles(), self.sid, self.sdd, self.pitch, self.W, self.H


@dataclass(frozen=True)
class Volume:
    """An L^3 grid of voxels of edge ``voxel_size`` mm, centred on the isocentre."""

    L: int
    voxel_size: float

    @property
    def origin(self) -> tuple:
        """World position of the centre of voxel (0,0,0): -(L-1)/2 * voxel_size per axis."""
        o = -(self.L - 1) / 2.0 * self.voxel_size
        return (o, o, o)

    @property
    def n_voxels(self) -> int:
        return self.L ** 3


@dataclass(frozen=True)
class Ellipsoids:
    centres: np.ndarray  # (n, 3) mm
    axes: np.ndarray  # (n, 3) semi-axes, mm
    rotations: np.ndarray  # (n, 3, 3) columns = principal axes
    densities: np.ndarray  # (n,)


def random_ellipsoids(seed: int, n: int = 10, ball_radius: float = 70.0,
                      axis_range=(10.0, 60.0), density_range=(0.0, 1.0)) -> Ellipsoids:
    """n ellipsoids: centres uniform in a ball, semi-axes uniform, uniform random rotation, densities U[0,1]."""
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = ball_radius * rng.uniform(size=(n, 1)) ** (1.0 / 3.0)
    centres = d * r
    axes = rng.uniform(axis_range[0], axis_range[1], size=(n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    a, b, c, e = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    rot = np.stack([
        np.stack([1 - 2 * (c * c + e * e), 2 * (b * c - a * e), 2 * (b * e + a * c)], -1),
        np.stack([2 * (b * c + a * e), 1 - 2 * (b * b + e * e), 2 * (c * e - a * b)], -1),
        np.stack([2 * (b * e - a * c), 2 * (c * e + a * b), 1 - 2 * (b * b + c * c)], -1),
    ], axis=1)
    dens = rng.uniform(density_range[0], density_range[1], size=n)
    return Ellipsoids(centres, axes, rot, dens)


def _frames(scanner: Scanner, views, device):
    th = torch.as_tensor(scanner.angles()[list(views)], dtype=torch.float64, device=device)
    c, s = torch.cos(th), torch.sin(th)
    z = torch.zeros_like(c)
    src = scanner.sid * torch.stack([c, s, z], -1)
    det = -(scanner.sdd - scanner.sid) * torch.stack([c, s, z], -1)
    e_u = torch.stack([-s, c, z], -1)
    e_v = torch.stack([z, z, torch.ones_like(c)], -1)
    return src, det, e_u, e_v


def _detector_offsets(scanner: Scanner, device):
    i = torch.arange(scanner.W, dtype=torch.float64, device=device) - (scanner.W - 1) / 2.0
    j = torch.arange(scanner.H, dtype=torch.float64, device=device) - (scanner.H - 1) / 2.0
    return i * scanner.pitch, j * scanner.pitch  # mm along e_u, e_v


_SYNTH_LIB = None


def _synth_lib():
    """The generator's GPU kernels (libbpsynth.so), or None if not built."""
    global _SYNTH_LIB
    if _SYNTH_LIB is None:
        import ctypes
        import os

        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbpsynth.so")
        if not os.path.exists(path):
            return None
        lib = ctypes.CDLL(path)
        lib.bpsynth_line_integrals.restype = ctypes.c_int
        lib.bpsynth_line_integrals.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_int,
                                               ctypes.c_void_p]
        _SYNTH_LIB = lib
    return _SYNTH_LIB


def line_integrals_fast(scanner: Scanner, phantom: Ellipsoids, views, device) -> torch.Tensor:
    """Same as ``line_integrals`` by one GPU kernel per call (libbpsynth.so) on torch's current stream."""
    lib = _synth_lib()
    if lib is None:
        raise RuntimeError("libbpsynth.so is not built")
    views = list(views)
    src, det, e_u, e_v = _frames(scanner, views, device)
    frames = torch.cat([src, det, e_u, e_v], dim=1).contiguous()
    ell = []
    for e in range(len(phantom.densities)):
        R = phantom.rotations[e]
        M = R @ np.diag(1.0 / phantom.axes[e] ** 2) @ R.T
        ell.append(np.concatenate([phantom.centres[e], M.ravel(), [phantom.densities[e]]]))
    ell = torch.as_tensor(np.array(ell, dtype=np.float64).reshape(-1, 13), device=device).contiguous()
    out = torch.empty((len(views), scanner.H, scanner.W), dtype=torch.float64, device=device)
    stream = torch.cuda.current_stream(out.device).cuda_stream
    rc = lib.bpsynth_line_integrals(out.data_ptr(), frames.data_ptr(), len(views), scanner.W, scanner.H,
                                    float(scanner.pitch), ell.data_ptr(), len(phantom.densities), stream)
    if rc != 0:
        raise RuntimeError(f"bpsynth_line_integrals failed ({rc})")
    return out


def line_integrals(scanner: Scanner, phantom: Ellipsoids, views, device="cpu") -> torch.Tensor:
    """Analytic line integrals (V, H, W) FP64 of the phantom along source -> pixel-centre rays.

    For an ellipsoid (x - c)^T M (x - c) = 1 and a unit ray x = S + lam d the
    chord length is 2 sqrt(B^2 - A C) / A with A = d^T M d, B = d^T M (S - c),
    C = (S - c)^T M (S - c) - 1; densities add.
    """
    views = list(views)
    src, det, e_u, e_v = _frames(scanner, views, device)
    du, dv = _detector_offsets(scanner, device)
    pix = (det[:, None, None, :]
           + du[None, None, :, None] * e_u[:, None, None, :]
           + dv[None, :, None, None] * e_v[:, None, None, :])
    d = pix - src[:, None, None, :]
    d = d / torch.linalg.norm(d, dim=-1, keepdim=True)
    out = torch.zeros(d.shape[:-1], dtype=torch.float64, device=device)
    for e in range(len(phantom.densities)):
        R = torch.as_tensor(phantom.rotations[e], dtype=torch.float64, device=device)
        inv_ax2 = torch.as_tensor(1.0 / phantom.axes[e] ** 2, dtype=torch.float64, device=device)
        M = R @ torch.diag(inv_ax2) @ R.T
        q = src - torch.as_tensor(phantom.centres[e], dtype=torch.float64, device=device)
        Mq = q @ M  # (V, 3)
        C = (q * Mq).sum(-1) - 1.0  # (V,)
        Md = d @ M
        A = (d * Md).sum(-1)
        B = (d * Mq[:, None, None, :]).sum(-1)
        disc = B * B - A * C[:, None, None]
        chord = 2.0 * torch.sqrt(torch.clamp(disc, min=0.0)) / A
        out += float(phantom.densities[e]) * chord
        del Md, A, B, disc, chord
    return out


def ramp_kernel(n_pad: int, tau: float, device="cpu") -> torch.Tensor:
    """Discrete Ram-Lak kernel h[n] (Kak & Slaney): 1/(4 tau^2) at 0, -1/(pi n tau)^2 at odd n, 0 at even n.

    Laid out circularly over n_pad samples for FFT convolution.
    """
    n = torch.arange(n_pad, device=device, dtype=torch.float64)
    n = torch.where(n < n_pad // 2, n, n - n_pad)
    h = torch.zeros(n_pad, dtype=torch.float64, device=device)
    h[0] = 1.0 / (4.0 * tau * tau)
    odd = (n.abs().remainder(2) == 1)
    h[odd] = -1.0 / (math.pi * math.pi * n[odd] * n[odd] * tau * tau)
    return h


def fdk_filter(p: torch.Tensor, scanner: Scanner) -> torch.Tensor:
    """Cosine weighting SDD / sqrt(SDD^2 + u^2 + v^2), then row-wise ramp filtering, FP64.

    The ramp runs along detector rows (the e_u direction) with the pixel
    pitch scaled to the isocentre, tau = pitch * SID / SDD, by zero-padded FFT.
    """
    device = p.device
    du, dv = _detector_offsets(scanner, device)
    cosw = scanner.sdd / torch.sqrt(scanner.sdd ** 2 + du[None, :] ** 2 + dv[:, None] ** 2)
    q = p * cosw[None]
    W = scanner.W
    n_pad = 1 << int(math.ceil(math.log2(2 * W)))
    tau = scanner.pitch * scanner.sid / scanner.sdd
    H = torch.fft.rfft(ramp_kernel(n_pad, tau, device))
    Q = torch.fft.rfft(q, n=n_pad, dim=-1)
    return torch.fft.irfft(Q * H, n=n_pad, dim=-1)[..., :W] * tau


def filtered_projections(scanner: Scanner, phantom: Ellipsoids, device="cpu", views=None,
                         chunk: int = 8, out_dtype=torch.float32, noise_frac: float = 0.0,
                         noise_seed: int = 0, fast: bool = False) -> torch.Tensor:
    """Filtered, weighted projections (V, H, W) as ``out_dtype`` (FP32/FP16/BF16, round-to-nearest-even).

    noise_frac > 0 adds Gaussian noise of sigma = noise_frac * max|p| over the
    whole stack to the filtered FP64 pixels before rounding (separate seed).
    fast: compute the line integrals with the generator's GPU kernel (device
    must be a GPU; equal to the torch path up to FP64 rounding order).
    """
    views = list(range(scanner.n_views)) if views is None else list(views)
    integrals = line_integrals_fast if fast else line_integrals
    out64 = [] if noise_frac > 0 else None
    out = torch.empty((len(views), scanner.H, scanner.W), dtype=out_dtype, device=device)
    for a in range(0, len(views), chunk):
        vs = views[a:a + chunk]
        f = fdk_filter(integrals(scanner, phantom, vs, device), scanner)
        if out64 is not None:
            out64.append(f.to(torch.float32))  # keeps memory bounded; noise is added below
        else:
            out[a:a + len(vs)] = f.to(out_dtype)
    if out64 is not None:
        stack = torch.cat(out64, 0)
        sigma = noise_frac * float(stack.abs().max())
        g = torch.Generator(device=device)
        g.manual_seed(noise_seed)
        noise = torch.randn(stack.shape, generator=g, device=device, dtype=torch.float32) * sigma
        out.copy_((stack + noise).to(out_dtype))
    return out


def uniform_images(shape, seed: int, low=-1.0, high=1.0, dtype=torch.float32) -> torch.Tensor:
    """Seeded uniform random images (numpy PCG64), for parity cases that need no phantom."""
    rng = np.random.default_rng(seed)
    return torch.from_numpy(rng.uniform(low, high, size=shape).astype(np.float32)).to(dtype)


def integer_images(shape, seed: int, high=8) -> torch.Tensor:
    """Seeded small-integer FP32 images in [0, high): sums of them are exact in FP32."""
    rng = np.random.default_rng(seed)
    return torch.from_numpy(rng.integers(0, high, size=shape).astype(np.float32))


@dataclass
class Request:
    """One reconstruction request of a serving stream."""

    rid: int
    arrival_s: float
    L: int
    n_views: int
    dtype: str  # "f32" | "f16" | "bf16"
    phantom_seed: int
    cancel_s: float = None  # the client withdraws the request at this time (None: never)


def poisson_requests(n: int, rate_per_s: float, seed: int,
                     L_choices=(128, 256, 512), view_choices=(124, 248, 496),
                     dtype_choices=("f32", "f16"), seed_base: int = 100000) -> list:
    """A seeded Poisson stream: exponential inter-arrival gaps, uniform choices per request."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    t = np.cumsum(gaps) - gaps[0]
    Ls = rng.choice(L_choices, size=n)
    vs = rng.choice(view_choices, size=n)
    ds = rng.choice(dtype_choices, size=n)
    return [Request(i, float(t[i]), int(Ls[i]), int(vs[i]), str(ds[i]), seed_base + i) for i in range(n)]


FOV_MM = 256.0  # every standard volume spans 256 mm: L * voxel_size


def standard_volume(L: int) -> Volume:
    """The volume of edge L used by the standard workloads: voxel size 256 mm / L (2.0 mm at L=128)."""
    return Volume(L, FOV_MM / L)


@dataclass(frozen=True)
class Workload:
    name: str
    volume: Volume
    scanner: Scanner = field(default_factory=Scanner)
    phantom_seed: int = 1401
    dtype: str = "f32"
    noise_frac: float = 0.0
    noise_seed: int = 7494


WORKLOADS = {
    "fdk_l128_v496_f32": Workload("fdk_l128_v496_f32", Volume(128, 2.0), phantom_seed=1401),
    "fdk_l512_v496_f32": Workload("fdk_l512_v496_f32", Volume(512, 0.5), phantom_seed=1402),
    "fdk_l1024_v496_f32": Workload("fdk_l1024_v496_f32", Volume(1024, 0.25), phantom_seed=1403),
    "fdk_l512_v496_f16_noisy": Workload("fdk_l512_v496_f16_noisy", Volume(512, 0.5), phantom_seed=1404,
                                        dtype="f16", noise_frac=0.01),
    "fdk_l512_v496_bf16_noisy": Workload("fdk_l512_v496_bf16_noisy", Volume(512, 0.5), phantom_seed=1404,
                                         dtype="bf16", noise_frac=0.01),
}
