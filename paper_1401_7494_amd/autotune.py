"""Autotuner for the fused back-projection pass.

For one problem shape -- box (nx, ny, nz), views, storage dtype, detector --
it times every candidate (path, views per pass K, z-unroll ZU) on the device
and keeps the fastest, as the median of a few timed runs after a warm-up.
Results are cached in a JSON file keyed by device name and shape, and applied
to a context with ``bp_set_tuning``.

The timing function is injectable, so the search logic is testable without a
GPU.
"""
from __future__ import annotations

import json
import os
import statistics
from dataclasses import asdict, dataclass, field

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")

K_CANDIDATES = (1, 2, 4, 8, 16, 32, 64)
ZU_CANDIDATES = (1, 2, 4, 8)


@dataclass(frozen=True)
class Candidate:
    path: str
    views_per_pass: int
    z_unroll: int


@dataclass(frozen=True)
class Problem:
    nx: int
    ny: int
    nz: int
    n_views: int
    dtype: str
    det_width: int
    det_height: int

    def key(self, device: str) -> str:
        return (f"{device}|{self.nx}x{self.ny}x{self.nz}|v{self.n_views}|{self.dtype}|"
                f"{self.det_width}x{self.det_height}")


@dataclass
class Result:
    best: Candidate
    timings_ms: dict = field(default_factory=dict)  # "path/K/ZU" -> median ms


def candidates(problem: Problem, ks=K_CANDIDATES, zus=ZU_CANDIDATES, include_plain=True):
    out = []
    if include_plain:
        out += [Candidate("plain", 1, zu) for zu in zus if zu <= max(problem.nz, 1)]
    out += [Candidate("fused", k, zu) for k in ks if k <= problem.n_views for zu in zus if zu <= max(problem.nz, 1)]
    return out


def search(problem: Problem, time_fn, cands=None, reps: int = 3, warmup: int = 1) -> Result:
    """Time every candidate with ``time_fn(candidate) -> ms`` and return the fastest (median of ``reps``)."""
    cands = cands if cands is not None else candidates(problem)
    if not cands:
        raise ValueError("no candidates to time")
    timings = {}
    for c in cands:
        for _ in range(warmup):
            time_fn(c)
        ms = statistics.median(time_fn(c) for _ in range(reps))
        timings[f"{c.path}/{c.views_per_pass}/{c.z_unroll}"] = ms
    best_key = min(timings, key=timings.get)
    path, k, zu = best_key.split("/")
    return Result(Candidate(path, int(k), int(zu)), timings)


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def store(key: str, result: Result, path: str = DEFAULT_CACHE) -> None:
    cache = load_cache(path)
    cache[key] = {"best": asdict(result.best), "timings_ms": result.timings_ms}
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(key: str, path: str = DEFAULT_CACHE):
    entry = load_cache(path).get(key)
    return Candidate(**entry["best"]) if entry else None


def device_timer(ctx, volume, projections, matrices, voxel_size, origin, torch):
    """A ``time_fn`` that runs one call on the device and returns its time in ms (HIP events)."""

    def run(c: Candidate) -> float:
        ctx.set_tuning(c.path, c.views_per_pass, c.z_unroll)
        s = torch.cuda.current_stream()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s)
        ctx.backproject(volume, projections, matrices, voxel_size, origin, s)
        b.record(s)
        b.synchronize()
        return a.elapsed_time(b)

    return run


def tune_on_device(ctx, volume, projections, matrices, voxel_size, origin, cands=None, reps=3,
                   cache_path: str | None = DEFAULT_CACHE) -> Result:
    """Search on the GPU for this shape, store the winner in the cache and apply it to ``ctx``."""
    import torch

    nz, ny, nx = volume.shape
    n, H, W = projections.shape
    problem = Problem(nx, ny, nz, n, ctx.dtype, W, H)
    result = search(problem, device_timer(ctx, volume, projections, matrices, voxel_size, origin, torch),
                    cands=cands, reps=reps)
    if cache_path:
        store(problem.key(torch.cuda.get_device_name(volume.device)), result, cache_path)
    apply(ctx, result.best)
    return result


def apply(ctx, cand: Candidate) -> None:
    ctx.set_tuning(cand.path, cand.views_per_pass, cand.z_unroll)
