"""Serving loop: continuous batching of reconstruction requests on one GPU.

Requests (volume edge L, number of views, storage dtype, phantom seed) arrive
over time.  A request's ingest makes its raw projections on the device (line
integrals of its phantom, standing in for detector data) and runs the
library's FDK pre-processing on them; then its volume is back projected.  The server keeps a FIFO of arrived requests and admits the oldest
ones that fit -- in both the HBM budget (volume + projections + library
scratch) and the in-flight limit -- whenever a slot and memory free up, not
in fixed batches.  Every admitted request gets its own HIP stream and library
context, so the back projections of different requests overlap on the device;
a request whose inputs are still being made does not hold up the others.
Latency is measured from arrival to the volume being ready; the device time
of the ingest and of the back projection are recorded separately (HIP events
on the request's stream).

A request can be withdrawn (``Request.cancel_s``, or ``Server.cancel(rid)``
from another thread): one still waiting leaves the queue at once; one in
flight is handed to the executor's ``cancel``, its result is dropped, and its
memory is released when the executor reports its device work over (work
already enqueued on the GPU runs to its end).

The executor does the device work; ``FakeExecutor`` stands in for it with
simulated durations so the scheduling logic is testable on the CPU.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import synth

GIB = 1 << 30


@dataclass
class Completed:
    rid: int
    arrival_s: float
    admitted_s: float
    done_s: float
    updates: float
    footprint: int
    result: object = None
    ingest_ms: float = None  # device time of the ingest (raw projections + FDK pre-processing)
    bp_ms: float = None      # device time of the back projection
    gen_ms: float = None     # of the ingest: the generator making the raw projections (the detector's stand-in)
    fdk_ms: float = None     # of the ingest: the library's FDK pre-processing and zeroing the volume

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s

    @property
    def queue_s(self) -> float:
        return self.admitted_s - self.arrival_s


@dataclass
class Report:
    completed: list
    makespan_s: float
    peak_bytes: int
    peak_inflight: int
    rejected: list = field(default_factory=list)
    cancelled: list = field(default_factory=list)  # (rid, "waiting" | "inflight", time s)

    def latencies(self):
        return np.array([c.latency_s for c in self.completed])

    def summary(self) -> dict:
        lat = self.latencies()
        upd = sum(c.updates for c in self.completed)
        timed = [c for c in self.completed if c.bp_ms is not None]
        dev = {}
        if timed:
            ing = np.array([c.ingest_ms for c in timed])
            bpm = np.array([c.bp_ms for c in timed])
            dev = {"p50_ingest_ms": float(np.percentile(ing, 50)), "p99_ingest_ms": float(np.percentile(ing, 99)),
                   "sum_generator_ms": float(sum(c.gen_ms or 0.0 for c in timed)),
                   "sum_fdk_ms": float(sum(c.fdk_ms or 0.0 for c in timed)),
                   "sum_backprojection_ms": float(bpm.sum()),
                   "p50_backprojection_ms": float(np.percentile(bpm, 50)),
                   "p99_backprojection_ms": float(np.percentile(bpm, 99)),
                   "backprojection_gups": float(sum(c.updates for c in timed) / (bpm.sum() * 1e-3) / 1e9)}
        return {
            "requests": len(self.completed),
            "rejected": len(self.rejected),
            "cancelled": len(self.cancelled),
            "p50_latency_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else None,
            "p99_latency_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else None,
            "mean_queue_ms": float(np.mean([c.queue_s for c in self.completed]) * 1e3) if len(lat) else None,
            "aggregate_gups": float(upd / self.makespan_s / 1e9) if self.makespan_s > 0 else None,
            "makespan_s": self.makespan_s,
            "peak_hbm_gib": self.peak_bytes / GIB,
            "peak_inflight": self.peak_inflight,
            **dev,
        }


class Server:
    """Admission by HBM budget and in-flight limit, FIFO among arrived requests."""

    def __init__(self, executor, budget_bytes: int, max_inflight: int = 8, clock=time.perf_counter,
                 sleep=time.sleep, poll_s: float = 2e-4):
        import threading

        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_inflight = int(max_inflight)
        self.clock = clock
        self.sleep = sleep
        self.poll_s = poll_s
        self._lock = threading.Lock()
        self._cancel = set()

    def cancel(self, rid: int) -> None:
        """Withdraw request ``rid`` (safe to call from another thread while ``run`` is going)."""
        with self._lock:
            self._cancel.add(rid)

    def _withdrawn(self, r, now) -> bool:
        if r.cancel_s is not None and r.cancel_s <= now:
            return True
        with self._lock:
            return r.rid in self._cancel

    def run(self, requests) -> Report:
        pending = sorted(requests, key=lambda r: (r.arrival_s, r.rid))
        waiting = []  # arrived, not admitted (FIFO)
        inflight = {}  # rid -> (handle, request, footprint, admitted_s)
        draining = {}  # cancelled in flight: rid -> (handle, footprint), memory held until the work ends
        used = peak = peak_n = 0
        done, rejected, cancelled = [], [], []
        t0 = self.clock()
        i = 0
        while i < len(pending) or waiting or inflight or draining:
            now = self.clock() - t0
            while i < len(pending) and pending[i].arrival_s <= now:
                r = pending[i]
                i += 1
                if self.ex.footprint(r) > self.budget:
                    rejected.append(r)  # can never fit
                else:
                    waiting.append(r)
            progressed = False
            # withdrawn requests: waiting ones leave the queue, running ones are told to stop
            for r in [r for r in waiting if self._withdrawn(r, now)]:
                waiting.remove(r)
                cancelled.append((r.rid, "waiting", now))
                progressed = True
            for rid in list(inflight):
                h, r, fp, adm = inflight[rid]
                if self._withdrawn(r, now):
                    self.ex.cancel(h)
                    draining[rid] = (h, fp)
                    del inflight[rid]
                    cancelled.append((rid, "inflight", now))
                    progressed = True
            for rid in list(draining):
                h, fp = draining[rid]
                if self.ex.poll(h):
                    self.ex.discard(h)
                    used -= fp
                    del draining[rid]
                    progressed = True
            # completions free memory and slots
            for rid in list(inflight):
                h, r, fp, adm = inflight[rid]
                if self.ex.poll(h):
                    res, tm = self.ex.finish(h)
                    done.append(Completed(r.rid, r.arrival_s, adm, self.clock() - t0, self.ex.updates(r), fp, res,
                                          tm.get("ingest_ms"), tm.get("bp_ms"), tm.get("gen_ms"), tm.get("fdk_ms")))
                    used -= fp
                    del inflight[rid]
                    progressed = True
            # admit the oldest arrived requests that fit (a large one does not block smaller ones behind it)
            for r in list(waiting):
                if len(inflight) + len(draining) >= self.max_inflight:
                    break
                fp = self.ex.footprint(r)
                if used + fp <= self.budget:
                    waiting.remove(r)
                    adm = self.clock() - t0
                    inflight[r.rid] = (self.ex.start(r), r, fp, adm)
                    used += fp
                    peak = max(peak, used)
                    peak_n = max(peak_n, len(inflight) + len(draining))
                    progressed = True
            if not progressed:
                nxt = pending[i].arrival_s - (self.clock() - t0) if i < len(pending) else None
                wait = self.poll_s if (inflight or nxt is None) else min(max(nxt, 0.0), 0.01)
                if inflight and nxt is not None:
                    wait = min(self.poll_s, max(nxt, 0.0))
                self.sleep(max(wait, 0.0))
        return Report(done, self.clock() - t0, peak, peak_n, rejected, cancelled)


# ---------------------------------------------------------------------------
# Executors
# ---------------------------------------------------------------------------

def request_scanner(req) -> synth.Scanner:
    """The orbit of a request: the standard 200 degree C-arm orbit sampled with its view count."""
    return synth.Scanner(n_views=req.n_views)


def request_volume(req) -> synth.Volume:
    return synth.standard_volume(req.L)


class FakeExecutor:
    """Simulated device for scheduler tests: a request takes ``t_fixed + updates / rate`` seconds."""

    def __init__(self, clock, rate_ups: float = 1e12, t_fixed: float = 0.0, bytes_per_pixel=None):
        self.clock = clock
        self.rate = rate_ups
        self.t_fixed = t_fixed
        self.started = []
        self.discarded = []
        self.bytes_per_pixel = bytes_per_pixel or {"f32": 4, "f16": 2, "bf16": 2}

    def updates(self, r) -> float:
        return float(r.L) ** 3 * r.n_views

    def footprint(self, r) -> int:
        sc = request_scanner(r)
        return 4 * r.L ** 3 + r.n_views * sc.W * sc.H * self.bytes_per_pixel[r.dtype]

    def start(self, r):
        self.started.append(r.rid)
        return (r, self.clock() + self.t_fixed + self.updates(r) / self.rate, {"stop": None})

    def poll(self, h) -> bool:
        return self.clock() >= (h[1] if h[2]["stop"] is None else h[2]["stop"])

    def finish(self, h):
        return h[0].rid, {}

    def cancel(self, h):
        """The simulated device stops a cancelled request at once."""
        h[2]["stop"] = self.clock()

    def discard(self, h):
        self.discarded.append(h[0].rid)


class GpuExecutor:
    """Per request: its own stream and context.  At admission its raw projections are made on
    the device (line integrals, FP32) and weighted and filtered by the library's FDK
    pre-processing into the request's storage dtype; then one back projection of all its
    views is accumulated into a zeroed volume.

    keep_results: return each volume (on the host) from ``finish``; otherwise a checksum."""

    def __init__(self, device=0, keep_results=False, views_per_pass=0, z_unroll=0, tile_x=0,
                 scanner_fn=request_scanner, volume_fn=request_volume, fast_inputs=True, tuning_cache=None):
        import torch

        from . import bp

        self.torch = torch
        self.bp = bp
        self.dev = torch.device(f"cuda:{device}")
        self.dev_name = torch.cuda.get_device_name(self.dev)
        self.keep = keep_results
        self.tuning = (views_per_pass, z_unroll, tile_x)
        # autotune cache (path): a request whose shape has a tuned launch on this device runs it
        self.tuning_cache = tuning_cache
        self.scanner_fn = scanner_fn
        self.volume_fn = volume_fn
        self.fast_inputs = fast_inputs
        self._mats = {}
        # Free library contexts per (dtype, W, H).  A context's scratch is reused by every
        # call on it, so one context serves one in-flight request at a time; contexts are
        # kept for the executor's lifetime (destroying one synchronises the device).
        self._free_ctx = {}
        self._probe = {}  # one context per (dtype, W, H) that only answers scratch queries
        self._fdk = {}  # FDK handles per detector geometry (safe to share between streams)

    def updates(self, r) -> float:
        return float(r.L) ** 3 * r.n_views

    def _tune(self, ctx, r, sc):
        """The request's launch: the autotuner's for its shape if cached, else the executor's
        fixed choices (0 = the library's)."""
        if self.tuning_cache:
            from . import autotune

            hit = autotune.lookup(autotune.Problem(r.L, r.L, r.L, r.n_views, r.dtype, sc.W, sc.H).key(self.dev_name),
                                  self.tuning_cache)
            if hit is not None:
                autotune.apply(ctx, hit)
                return hit
        ctx.set_tuning("auto", *self.tuning)
        ctx.set_options()
        ctx.set_tap_split(-1)
        return None

    def footprint(self, r) -> int:
        """Device bytes the request holds while in flight: volume, projections, raw input, the
        generator's work arrays and the library's scratch for the call (as the library reports it
        for the launch the request will run)."""
        sc = self.scanner_fn(r)
        bpp = 4 if r.dtype == "f32" else 2
        vol = 4 * r.L ** 3
        proj = r.n_views * sc.W * sc.H * bpp
        raw = r.n_views * sc.W * sc.H * 4 if self.fast_inputs else 0
        key = (r.dtype, sc.W, sc.H)
        if key not in self._probe:
            self._probe[key] = self.bp.Context(sc.W, sc.H, r.dtype, device=self.dev.index or 0)
        probe = self._probe[key]
        self._tune(probe, r, sc)
        scratch = probe.scratch_bytes(r.L, r.L, r.L, r.n_views)
        gen = 6 * 62 * sc.W * sc.H * 8  # FP64 work arrays of the input generator (62 views at a time)
        return vol + proj + raw + scratch + gen

    def _matrices(self, sc):
        key = sc.geometry_args()[1:] + (sc.n_views, sc.arc_deg, sc.start_deg)
        if key not in self._mats:
            _, P32 = self.bp.circular_matrices(*sc.geometry_args())
            self._mats[key] = self.torch.from_numpy(P32).to(self.dev)
        return self._mats[key]

    def _fdk_for(self, sc):
        key = (sc.W, sc.H, sc.pitch, sc.sid, sc.sdd)
        if key not in self._fdk:
            self._fdk[key] = self.bp.FdkFilter.for_scanner(sc, device=self.dev.index or 0)
        return self._fdk[key]

    def start(self, r):
        torch = self.torch
        stream = torch.cuda.Stream(device=self.dev)  # default priority
        sc, v = self.scanner_fn(r), self.volume_fn(r)
        tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[r.dtype]
        mats = self._matrices(sc)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        raw = None
        with torch.cuda.stream(stream):
            ev[0].record(stream)
            ph = synth.random_ellipsoids(r.phantom_seed)
            if self.fast_inputs:
                # ingest: raw projections arrive (made here by the generator), the library filters them
                raw = torch.empty((sc.n_views, sc.H, sc.W), dtype=torch.float32, device=self.dev)
                for a in range(0, sc.n_views, 62):
                    views = list(range(a, min(a + 62, sc.n_views)))
                    raw[a:a + len(views)] = synth.line_integrals_fast(sc, ph, views, self.dev).to(torch.float32)
                ev[3].record(stream)
                proj = self._fdk_for(sc).filter(raw, r.dtype, stream=stream)
            else:
                proj = synth.filtered_projections(sc, ph, device=self.dev, out_dtype=tdt, chunk=62)
            vol = torch.zeros((v.L,) * 3, dtype=torch.float32, device=self.dev)
            ev[1].record(stream)
        key = (r.dtype, sc.W, sc.H)
        pool = self._free_ctx.setdefault(key, [])
        ctx = pool.pop() if pool else self.bp.Context(sc.W, sc.H, r.dtype, device=self.dev.index or 0)
        self._tune(ctx, r, sc)
        ctx.backproject(vol, proj, mats, v.voxel_size, v.origin, stream)
        ev[2].record(stream)
        return {"r": r, "stream": stream, "ctx": ctx, "key": key, "vol": vol, "proj": proj, "raw": raw,
                "done": ev[2], "ev": ev}

    def poll(self, h) -> bool:
        return h["done"].query()

    def finish(self, h):
        h["done"].synchronize()
        ev = h["ev"]
        tm = {"ingest_ms": ev[0].elapsed_time(ev[1]), "bp_ms": ev[1].elapsed_time(ev[2])}
        if self.fast_inputs:
            tm.update(gen_ms=ev[0].elapsed_time(ev[3]), fdk_ms=ev[3].elapsed_time(ev[1]))
        out = h["vol"].cpu().numpy() if self.keep else float(h["vol"].double().sum())
        self._free_ctx[h["key"]].append(h["ctx"])
        h.clear()
        return out, tm

    def cancel(self, h):
        """Work already enqueued for a cancelled request runs to its end (a kernel cannot be
        stopped midway); its result is dropped by ``discard``."""
        h["cancelled"] = True

    def discard(self, h):
        h["done"].synchronize()
        self._free_ctx[h["key"]].append(h["ctx"])
        h.clear()

    def close(self):
        for ctx in self._probe.values():
            ctx.close()
        self._probe.clear()
        for pool in self._free_ctx.values():
            for ctx in pool:
                ctx.close()
        self._free_ctx.clear()
        for f in self._fdk.values():
            f.close()
        self._fdk.clear()


def serve_mix(ex, n_requests=200, seed=1405, budget_bytes=200 * GIB, max_inflight=8, load=0.8, rate=0.0,
              warmup=True, log=None):
    """The serving measurement: first every request of the seeded mix is offered at time 0
    (back-to-back capacity), then the same mix arrives as a Poisson stream at ``load`` times that
    capacity (or at ``rate`` requests/s).  Returns (capacity summary or None, Poisson summary)."""
    if warmup:
        # not reported: contexts, FDK handles, scratch and the allocator reach their largest sizes
        # for every storage dtype of the mix
        warm = [synth.Request(-1 - i, 0.0, 512, 496, dt, 99999 - i) for i, dt in enumerate(("f32", "f16"))]
        Server(ex, budget_bytes, max_inflight).run(warm)
    base = synth.poisson_requests(n_requests, 1.0, seed)
    cap_summary = None
    if not rate:
        burst = [synth.Request(r.rid, 0.0, r.L, r.n_views, r.dtype, r.phantom_seed) for r in base]
        rep = Server(ex, budget_bytes, max_inflight).run(burst)
        cap = len(rep.completed) / rep.makespan_s
        cap_summary = rep.summary()
        cap_summary.update(phase="back_to_back", capacity_rps=cap)
        if log:
            log(f"serve: capacity {cap_summary}")
        rate = load * cap
    stream = synth.poisson_requests(n_requests, rate, seed)
    rep = Server(ex, budget_bytes, max_inflight).run(stream)
    s = rep.summary()
    s.update(phase="poisson", rate_rps=rate, load=load, budget_gib=budget_bytes / GIB, max_inflight=max_inflight)
    if log:
        log(f"serve: poisson {s}")
    return cap_summary, s


def main(argv=None):
    """Serve a seeded Poisson stream on the GPU: ``python -m paper_1401_7494_amd.serve``.

    First every request is offered at time 0 to measure back-to-back capacity,
    then the stream is replayed with Poisson arrivals at ``load`` times that
    capacity.  Prints one JSON line per phase.
    """
    import argparse
    import json

    ap = argparse.ArgumentParser(description="continuous-batching serving run on one GPU")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--seed", type=int, default=1405)
    ap.add_argument("--budget-gib", type=float, default=200.0)
    ap.add_argument("--max-inflight", type=int, default=8)
    ap.add_argument("--load", type=float, default=0.8, help="arrival rate as a fraction of measured capacity")
    ap.add_argument("--rate", type=float, default=0.0, help="arrival rate (requests/s); 0 = load x capacity")
    ap.add_argument("--tuning-cache", default=None, help="autotune cache to take each request's launch from")
    args = ap.parse_args(argv)
    ex = GpuExecutor(tuning_cache=args.tuning_cache)
    cap, poi = serve_mix(ex, args.requests, args.seed, int(args.budget_gib * GIB), args.max_inflight, args.load,
                         args.rate)
    ex.close()
    for s in (cap, poi):
        if s is not None:
            print(json.dumps(s), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
