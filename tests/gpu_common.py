"""Shared helpers of the GPU tests: run the HIP path and the oracle on the same inputs."""
from __future__ import annotations

import functools

import numpy as np
import torch

import oracle
from oracle import geometry
from paper_1401_7494_amd import bp, synth

TORCH_DTYPE = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}

# FP32 parity bar against the FP64 oracle on identical inputs: relative L2 over
# the compared voxels.
REL_L2_TOL = 1e-5

# Element-wise companion of the relative-L2 bar (reading R12): max |error| over max |V_ref|.
MAX_ABS_TOL = 1e-4

# Compact staging rounds the bilinear-patch coefficients (pixel differences) to
# FP16: unit roundoff u = 2^-11 on each of dx, dy, dxy.  The interpolated value
# moves by at most u (|dx| + |dy| + |dxy|), which is of the order of u times the
# local pixel magnitude; the bar on relative L2 is 2u.
COMPACT_REL_L2_TOL = 2.0 ** -10
# ... and its element-wise companion, in the same ratio to the relative-L2 bar as for FP32.
COMPACT_MAX_ABS_TOL = COMPACT_REL_L2_TOL * (MAX_ABS_TOL / REL_L2_TOL)


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / den) if den > 0 else float(np.linalg.norm(got))


def error_stats(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = got - ref
    return {
        "rel_l2": rel_l2(got, ref),
        "max_abs_over_max": float(np.abs(d).max() / max(np.abs(ref).max(), 1e-300)),
        "rms": float(np.sqrt(np.mean(d * d))),
    }


def oracle_matrices(scanner):
    """The oracle's own FP32 matrices (composed in FP64 from the pinhole definition, rounded once)."""
    return geometry.circular_matrices(*scanner.geometry_args()).astype(np.float32)


def product_matrices(scanner):
    return bp.circular_matrices(*scanner.geometry_args())[1]


def run_gpu(proj, P32, shape, voxel_size, origin, dtype="f32", path="auto", k=0, zu=0, init=None,
            stream=None, tx=0, compact=False, cubic=False):
    """Back project on cuda:0 through the C ABI; returns the volume as a float32 numpy array."""
    dev = torch.device("cuda:0")
    nz, ny, nx = shape
    vol = torch.zeros(shape, dtype=torch.float32, device=dev) if init is None else \
        torch.as_tensor(init, dtype=torch.float32).to(dev).contiguous()
    p = proj.to(dev).contiguous() if isinstance(proj, torch.Tensor) else torch.from_numpy(proj).to(dev)
    m = torch.as_tensor(np.ascontiguousarray(P32, dtype=np.float32)).to(dev)
    H, W = p.shape[1:]
    with bp.Context(W, H, dtype) as ctx:  # FP32 staging unless the caller asks for the compact form
        ctx.set_tuning(path, k, zu, tx)
        ctx.set_options(compact_staging=compact)
        ctx.backproject(vol, p, m, voxel_size, origin, stream, cubic=cubic)
        torch.cuda.synchronize()
    return vol.cpu().numpy()


def run_oracle(proj, P32, L, voxel_size, origin, block=None, vol=None):
    """The oracle on the data the GPU read (FP16/BF16 widened exactly to FP32)."""
    if isinstance(proj, torch.Tensor):
        proj = proj.float().cpu().numpy()
    return oracle.backproject(proj, np.asarray(P32, dtype=np.float32).astype(np.float64), L, voxel_size,
                              origin, block=block, vol=vol)


@functools.lru_cache(maxsize=4)
def full_projections(phantom_seed: int, dtype: str = "f32", noise_frac: float = 0.0, noise_seed: int = 7494,
                     n_views: int = 496):
    """The paper-shaped stack (n_views x 960 x 1248) of a seeded phantom, made on the GPU."""
    sc = synth.Scanner(n_views=n_views)
    return synth.filtered_projections(sc, synth.random_ellipsoids(phantom_seed), device="cuda:0",
                                      out_dtype=TORCH_DTYPE[dtype], noise_frac=noise_frac,
                                      noise_seed=noise_seed)
