"""Autotuner for the fused back-projection pass.

For one problem shape -- box (nx, ny, nz), views, storage dtype, detector --
it times every candidate (path, views per pass K, z-unroll ZU) on the device
and keeps the fastest, as the median of a few timed runs after a warm-up.
Results are cached in a JSON file keyed by device name and shape, and applied
to a context with ``bp_set_tuning`` (and the tap options).  ``ensure_tuned``
is what the benchmark and the serving executor call: it reads the cache for
the call's shape and device, searches only on a miss, and applies the winner.
The library's own automatic choice (``AUTO``) is always one of the timed
candidates, so a tuned launch is never slower than it on the timed runs, and
it is kept when another launch is faster only by the timing noise.

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
TX_CANDIDATES = (8, 16, 32, 64)


@dataclass(frozen=True)
class Candidate:
    path: str
    views_per_pass: int
    z_unroll: int
    tile_x: int = 64
    tap_split: int = -1        # fused path: views of every 8 read directly (-1 = tuned, 8 = all)
    direct_taps: bool = False  # fused path: no LDS stage at all
    no_column: bool = False    # Part 1 per voxel even where u and w do not vary along z

    def key(self) -> str:
        return (f"{self.path}/{self.views_per_pass}/{self.z_unroll}/{self.tile_x}/"
                f"{'direct' if self.direct_taps else self.tap_split}" + ("/nocol" if self.no_column else ""))


# The library's own choice for the call (BP_PATH_AUTO with every parameter tuned by the library).
AUTO = Candidate("auto", 0, 0, 0, -1, False)


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
    timings_ms: dict = field(default_factory=dict)  # "path/K/ZU/TX" -> median ms


def candidates(problem: Problem, ks=K_CANDIDATES, zus=ZU_CANDIDATES, txs=TX_CANDIDATES, include_plain=True,
               splits=(-1,), include_direct_taps=True):
    """Plain passes (64-wide tiles), fused passes over K x ZU x tile width x share of directly read
    views (and with no LDS stage), and fused passes on the caller's images (16- and 64-wide tiles)."""
    zus = [zu for zu in zus if zu <= max(problem.nz, 1)]
    out = []
    if include_plain:
        out += [Candidate("plain", 1, zu, 64) for zu in zus]
    fused = [(k, zu, tx) for k in ks if k <= problem.n_views for zu in zus for tx in txs]
    out += [Candidate("fused", k, zu, tx, sp) for k, zu, tx in fused for sp in splits]
    if include_direct_taps:
        out += [Candidate("fused", k, zu, tx, -1, True) for k, zu, tx in fused]
    out += [Candidate("fused_direct", k, zu, tx) for k in ks if k <= problem.n_views for zu in zus
            for tx in txs if tx in (16, 64)]
    return out


def search(problem: Problem, time_fn, cands=None, reps: int = 3, warmup: int = 1, refine: float = 0.02,
           rounds: int = 7, tie: float = 0.01) -> Result:
    """Time every candidate with ``time_fn(candidate) -> ms`` (median of ``reps`` after ``warmup``)
    and return the fastest.  The candidates within ``refine`` (a fraction) of the fastest are then
    timed ``rounds`` more times, interleaved (in alternating order), so that a drift of the clocks
    over the search does not decide between near-equal launches; the medians of those interleaved
    runs decide between them.  Among the
    candidates within ``tie`` of the fastest, the library's own choice (``AUTO``) is kept when it
    is one of them: timing noise does not move a shape off the library's default (at L = 512 two
    identical launches still differ by up to 1% after three such rounds)."""
    cands = cands if cands is not None else candidates(problem)
    if not cands:
        raise ValueError("no candidates to time")
    samples = {}
    by_key = {}
    for c in cands:
        for _ in range(warmup):
            time_fn(c)
        samples[c.key()] = [time_fn(c) for _ in range(reps)]
        by_key[c.key()] = c
    timings = {k: statistics.median(v) for k, v in samples.items()}
    first = min(timings.values())
    close = [k for k in timings if timings[k] <= first * (1.0 + refine)]
    if len(close) > 1 and rounds > 0:
        again = {k: [] for k in close}
        for r in range(rounds):
            for k in (close if r % 2 == 0 else close[::-1]):
                again[k].append(time_fn(by_key[k]))
        for k in close:
            timings[k] = statistics.median(again[k])
    best_key = min(timings, key=timings.get)
    auto = AUTO.key()
    if auto in timings and timings[auto] <= timings[best_key] * (1.0 + tie):
        best_key = auto
    return Result(by_key[best_key], timings)


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
        apply(ctx, c)
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


def apply(ctx, cand: Candidate, **options) -> None:
    """Set the candidate's choices on a context; its options are reset to ``options`` plus the
    candidate's tap mode."""
    ctx.set_tuning(cand.path, cand.views_per_pass, cand.z_unroll, cand.tile_x)
    ctx.set_options(direct_taps=cand.direct_taps, no_column=cand.no_column, **options)
    ctx.set_tap_split(cand.tap_split)


def problem_of(ctx, volume_shape, n_views) -> Problem:
    nz, ny, nx = volume_shape
    return Problem(nx, ny, nz, n_views, ctx.dtype, ctx.det_width, ctx.det_height)


def ensure_tuned(ctx, volume, projections, matrices, voxel_size, origin, cands=None, reps=2, warmup=1,
                 cache_path: str | None = DEFAULT_CACHE, device_name: str | None = None, time_fn=None,
                 include_auto: bool = True, tag: str = ""):
    """The tuned launch for this call's shape on this device, applied to ``ctx``.

    Reads the cache (key: device name and problem shape); on a miss times ``cands`` (plus the
    library's automatic choice) on the device, stores the result and applies the winner.
    ``volume`` is used as scratch by the search (its contents are left undefined).  Returns
    ``(candidate, info)`` with info = {"source": "cache" | "search", "auto_ms", "best_ms",
    "timings_ms"} (times only for a search).  ``time_fn`` replaces the device timer (tests).
    ``include_auto = False`` searches only ``cands`` (e.g. the launches of one path, such as the
    plain form's); ``tag`` then keeps such a search apart in the cache."""
    problem = problem_of(ctx, volume.shape, projections.shape[0])
    if device_name is None:
        import torch

        device_name = torch.cuda.get_device_name(volume.device)
    dev = device_name
    key = problem.key(dev) + (f"|{tag}" if tag else "")
    if cache_path:
        hit = lookup(key, cache_path)
        if hit is not None:
            apply(ctx, hit)
            return hit, {"source": "cache", "key": key}
    cands = list(cands) if cands is not None else candidates(problem)
    if include_auto and AUTO not in cands:
        cands.insert(0, AUTO)
    if time_fn is None:
        import torch

        time_fn = device_timer(ctx, volume, projections, matrices, voxel_size, origin, torch)
    res = search(problem, time_fn, cands, reps=reps, warmup=warmup)
    if cache_path:
        store(key, res, cache_path)
    apply(ctx, res.best)
    return res.best, {"source": "search", "key": key, "auto_ms": res.timings_ms.get(AUTO.key()),
                      "best_ms": res.timings_ms[res.best.key()], "timings_ms": res.timings_ms}


def lookup_and_apply(ctx, volume_shape, n_views, device_name: str, cache_path: str = DEFAULT_CACHE):
    """Apply the cached tuned launch for this shape if there is one (else the library's automatic
    choice); returns the candidate applied."""
    hit = lookup(problem_of(ctx, volume_shape, n_views).key(device_name), cache_path) if cache_path else None
    apply(ctx, hit or AUTO)
    return hit or AUTO


def _csv_ints(s):
    return tuple(int(v) for v in s.split(",") if v)


def main(argv=None):
    """Tune one standard workload on the GPU: ``python -m paper_1401_7494_amd.autotune --workload ...``."""
    import argparse
    import sys

    import torch

    from . import bp, synth

    ap = argparse.ArgumentParser(description="autotune the fused back projection for one workload")
    ap.add_argument("--workload", default="fdk_l512_v496_f32")
    ap.add_argument("--dtype", default=None, help="storage dtype (default: the workload's)")
    ap.add_argument("--ks", default="8,16,32,64")
    ap.add_argument("--zus", default="4,8")
    ap.add_argument("--txs", default="8,16,32,64")
    ap.add_argument("--plain", action="store_true", help="also time the plain path")
    ap.add_argument("--splits", default="-1", help="shares of directly read views to try (-1 = tuned)")
    ap.add_argument("--no-direct-taps", action="store_true", help="skip the candidates without an LDS stage")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    args = ap.parse_args(argv)
    wl = synth.WORKLOADS[args.workload]
    dtype = args.dtype or wl.dtype
    dev = torch.device("cuda:0")
    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dtype]
    proj = synth.filtered_projections(wl.scanner, synth.random_ellipsoids(wl.phantom_seed), device=dev,
                                      out_dtype=tdt)
    _, P32 = bp.circular_matrices(*wl.scanner.geometry_args())
    mats = torch.from_numpy(P32).to(dev)
    v = wl.volume
    vol = torch.zeros((v.L,) * 3, dtype=torch.float32, device=dev)
    problem = Problem(v.L, v.L, v.L, wl.scanner.n_views, dtype, wl.scanner.W, wl.scanner.H)
    cands = candidates(problem, _csv_ints(args.ks), _csv_ints(args.zus), _csv_ints(args.txs), args.plain,
                       _csv_ints(args.splits), not args.no_direct_taps)
    with bp.Context(wl.scanner.W, wl.scanner.H, dtype) as ctx:
        res = search(problem, device_timer(ctx, vol, proj, mats, v.voxel_size, v.origin, torch), cands, args.reps)
    updates = v.L ** 3 * wl.scanner.n_views
    for key, ms in sorted(res.timings_ms.items(), key=lambda kv: kv[1]):
        print(f"autotune {wl.name} {dtype} {key}: {ms:.3f} ms  {updates / ms / 1e6:.1f} GUPS", flush=True)
    print(f"autotune best: {res.best}", flush=True)
    if args.cache:
        store(problem.key(torch.cuda.get_device_name(dev)), res, args.cache)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
