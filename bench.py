#!/usr/bin/env python3
"""Throughput of the HIP back projector on one MI355X, over every workload of the measurement plan.

A step is one full reconstruction: all views of the workload back projected
into the volume (per-view constants, staging, footprints and the
back-projection passes), inputs resident in HBM.  GUPS = voxels x views /
step time.  The seeded random-ellipsoid phantom stands in for the RabbitCT
rabbit scan (496 filtered, weighted projections of 1248 x 960, Sec. 4); the
orbit is a 200 degree circle with SID 800 mm, SDD 1200 mm and pitch 0.32 mm.

Headline (`value`): L=512 (512^3 FP32, voxel 0.5 mm), 496 views of FP32, the
fused form with the autotuner's launch.  Beside it on the same GPU and inputs:
the plain form (one volume pass per view), BF16 and FP16 storage.  Every form
states its error against the FP64 oracle on the centre block that the CPU
baseline times.

`configs` holds the other workloads:
  C1  plain FP32, L=128 (voxel 2 mm), 496 views; error over the whole volume
  C3  batched fused, L=1024 (4 GiB), 496 views streamed K per pass, K / z-unroll / tile width
      chosen by the autotuner (K over 1, 2, 4, 8, 16 and wider); sampled error
  C4  FP16 and BF16 storage of the phantom + 1% Gaussian noise, L=512; throughput and error of the
      default FP32 staging and of the compact FP16 records, against the oracle on the FP32 data
      and on the rounded data
  C5  the serving mix: 200 seeded requests (L in 128/256/512, 124/248/496 views, FP32/FP16),
      first all at once (capacity), then Poisson at 0.8 x capacity; p50/p99 latency,
      aggregate GUPS, ingest and back-projection device times, peak admitted HBM
  general  the L=512 workload through a tilted orbit (every view off the column branch), in the
           autotuner's launch for that geometry; sampled error

`roofline`: the dominant kernel of the headline form -- the paper's 38 FP32
operations per voxel update (Sec. 4.2) times the updates of one launch over
its mean duration (HIP events on the launch's stream), against the 157.3
TFLOP/s FP32 vector peak; beside it the VALU issue rate from the committed
counter record, the algorithmic and counter-measured HBM bytes, and the share
of (tile, view) pairs the clipping mask skips.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_UPDATE = 38          # Sec. 4.2: 13 additions, 5 subtractions, 17 multiplications, 3 divisions
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector peak (packed FMA: 2 x 2 flops per lane per clock)
VALU_PEAK_T = 256 * 64 * 2.4e9 / 1e12  # 256 CUs x 64 lanes x 2.4 GHz: VALU lane-instructions/s (no packed FP32)
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("paper_1401_7494_amd/csrc/bp_kernels.hip", "paper_1401_7494_amd/csrc/bp_internal.h")
COUNTERS_MD = "profiles/backproject_fused_f32_l512_v496_counters.md"
TILT_DEG = 7.0                 # gantry tilt of the general-branch workload


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_sha():
    """SHA-256 of the kernel sources with comments and white space removed (an edit of a comment
    keeps a counter record valid, any change of the code does not)."""
    import hashlib
    import re

    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def tilt_matrices(P64, deg):
    """The orbit tilted by ``deg`` degrees about x (P T, T the rotation of the world frame), composed
    in FP64 and rounded once to FP32: every view then has P[0][2] and P[2][2] non-zero."""
    a = np.radians(deg)
    T = np.eye(4)
    T[1, 1], T[1, 2], T[2, 1], T[2, 2] = np.cos(a), -np.sin(a), np.sin(a), np.cos(a)
    return (np.asarray(P64, dtype=np.float64) @ T).astype(np.float32)


def counter_record(kernel: str, launch: str, workload: str):
    """The committed rocprofv3 counter record of this kernel, launch and workload (the file holds one
    per profiled launch), or None when the kernel sources changed since it was taken or no record is
    for this kernel and launch."""
    path = os.path.join(ROOT, COUNTERS_MD)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if "```json" not in text:
        return None
    recs = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    sha = kernel_source_sha()
    for rec in recs if isinstance(recs, list) else [recs]:
        if (rec.get("kernel_source_sha256") == sha and rec.get("kernel") == kernel and
                rec.get("launch_key") == launch and rec.get("workload") == workload):
            return rec
    return None


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed reconstructions of the headline forms")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config-steps", type=int, default=5, help="timed reconstructions of the other workloads")
    ap.add_argument("--configs", default="roofs,C1,C3,C4,C5,general",
                    help="workloads beside the headline (roofs, C1, C3, C4, C5, general; empty: none)")
    ap.add_argument("--forms", default="fused_f32,plain_f32,fused_bf16,fused_f16",
                    help="headline forms (path_dtype; path in fused, plain, direct, auto)")
    ap.add_argument("--no-tune", action="store_true", help="headline forms on the library's automatic choice")
    ap.add_argument("--tuning-cache", default=None,
                    help="autotune cache file (default: a fresh one under gpurun_out/ or the temp folder)")
    ap.add_argument("--k", type=int, default=0, help="views per pass for fused forms (0 = tuned)")
    ap.add_argument("--zu", type=int, default=0, help="z-unroll (0 = tuned)")
    ap.add_argument("--tx", type=int, default=0, help="block tile width along x (0 = tuned)")
    ap.add_argument("--direct-taps", action="store_true", help="fused forms read every tap directly (no LDS stage)")
    ap.add_argument("--tap-split", type=int, default=-1, help="views of every 8 read directly (-1 = tuned)")
    ap.add_argument("--no-fdk", action="store_true", help="skip timing the FDK pre-processing of the stack")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-block", type=int, default=320,
                    help="edge of the centre block the oracle times (about 10 s of FP64 work on 16 threads)")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--no-clocks", action="store_true", help="do not query clocks with rocm-smi (profiled runs)")
    ap.add_argument("--tilt", type=float, default=0.0,
                    help="headline forms on the orbit tilted by this many degrees about x (the general branch; "
                         "for profiling it: the workload is then named with the tilt)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device 3 times (a known-size kernel for HBM counters)")
    return ap.parse_args()


def device_info(torch):
    p = torch.cuda.get_device_properties(0)
    return {"name": torch.cuda.get_device_name(0), "arch": getattr(p, "gcnArchName", None),
            "compute_units": p.multi_processor_count, "memory_gib": round(p.total_memory / 2 ** 30, 1)}


NO_CLOCKS = False  # --no-clocks: under a profiler, whose preloaded library makes the query's exec fail


def clocks():
    """Current shader and memory clocks as rocm-smi reports them (None if it cannot)."""
    if NO_CLOCKS:
        return None
    try:
        out = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True, timeout=20)
        data = json.loads(out.stdout[out.stdout.index("{"):])
    except Exception:
        return None
    card = next(iter(data.values()), {}) if isinstance(data, dict) else {}
    return {k: v for k, v in card.items() if "sclk" in k.lower() or "mclk" in k.lower()} or None


def stats(step_ms, updates):
    ms = np.asarray(step_ms, dtype=np.float64)
    return {"ms_per_step": round(float(ms.mean()), 3),
            "gups_mean": round(updates / (ms.mean() * 1e-3) / 1e9, 2),
            "gups_p50": round(updates / (np.percentile(ms, 50) * 1e-3) / 1e9, 2),
            "gups_p99": round(updates / (np.percentile(ms, 99) * 1e-3) / 1e9, 2)}


def error_stats(got, ref):
    got = np.asarray(got, dtype=np.float64)
    d = got - ref
    return {"rel_l2": float(np.linalg.norm(d) / np.linalg.norm(ref)),
            "max_abs_over_max": float(np.abs(d).max() / np.abs(ref).max()),
            "rms": float(np.sqrt(np.mean(d * d)))}


class Bench:
    def __init__(self, args):
        import torch

        from paper_1401_7494_amd import autotune, bp, synth

        self.args, self.torch, self.bp, self.synth, self.at = args, torch, bp, synth, autotune
        self.dev = torch.device("cuda:0")
        self.dev_name = torch.cuda.get_device_name(self.dev)
        if args.tuning_cache:
            self.cache = args.tuning_cache
        else:
            d = os.path.join(ROOT, "gpurun_out") if os.path.isdir(os.path.join(ROOT, "gpurun_out")) else \
                os.environ.get("TMPDIR", "/tmp")
            self.cache = os.path.join(d, f"bench_tuning_{os.getpid()}.json")

    # ------------------------------------------------------------------ inputs
    def stack(self, wl, dtype="f32"):
        t = time.perf_counter()
        p = self.synth.filtered_projections(wl.scanner, self.synth.random_ellipsoids(wl.phantom_seed),
                                            device=self.dev, noise_frac=wl.noise_frac, noise_seed=wl.noise_seed)
        self.torch.cuda.synchronize()
        log(f"bench: {wl.name} inputs made on the GPU in {time.perf_counter() - t:.1f} s")
        return p

    def matrices(self, sc):
        P64, P32 = self.bp.circular_matrices(*sc.geometry_args())
        return P64, self.torch.from_numpy(P32).to(self.dev)

    def free(self):
        self.torch.cuda.synchronize()
        self.torch.cuda.empty_cache()

    # ------------------------------------------------------------------ runs
    def context(self, W, H, dtype, cand=None, **options):
        ctx = self.bp.Context(W, H, dtype)
        if cand is not None:
            self.at.apply(ctx, cand, **options)
        elif options:
            ctx.set_options(**options)
        return ctx

    def tune(self, ctx, vol, proj, P, v, cands, label, include_auto=True, tag="", **options):
        """The autotuner's launch for this shape (from the cache, or searched and stored), applied."""
        t = time.perf_counter()
        best, info = self.at.ensure_tuned(ctx, vol, proj, P, v.voxel_size, v.origin, cands=cands,
                                          cache_path=self.cache, device_name=self.dev_name,
                                          include_auto=include_auto, tag=tag)
        if options:
            self.at.apply(ctx, best, **options)
        out = {"source": info["source"], "choice": best.key(), "path": best.path, "views_per_pass": best.views_per_pass,
               "z_unroll": best.z_unroll, "tile_x": best.tile_x, "tap_split": best.tap_split,
               "direct_taps": best.direct_taps, "no_column": best.no_column}
        if info["source"] == "search":
            out.update(candidates=len(info["timings_ms"]), tuned_ms=round(info["best_ms"], 3),
                       search_s=round(time.perf_counter() - t, 1))
            if info.get("auto_ms"):
                out.update(auto_ms=round(info["auto_ms"], 3), margin_over_auto=round(info["auto_ms"] / info["best_ms"], 4))
        log(f"bench: tuned {label}: {out}")
        return best, out

    def run(self, ctx, proj, P, v, steps, warmup, shape=None, timing="inside", graph=False):
        """warmup + steps reconstructions into one volume; returns the step times (HIP events around
        each step), the library's per-kernel timings (HIP events around each launch, on the stream
        of the launch) over the timed steps (``timing="inside"``) or over up to 3 further steps
        ("after": the timed steps carry no per-launch events; None: no kernel timings), and the
        volume of one reconstruction.  ``graph``: each step replays one reconstruction captured in
        a HIP graph (launch costs paid once; kernel timings then come "after")."""
        torch = self.torch
        shape = shape or (v.L,) * 3
        vol = torch.zeros(shape, dtype=torch.float32, device=self.dev)
        stream = torch.cuda.current_stream(self.dev)
        for _ in range(max(warmup, 1 if graph else 0)):
            ctx.backproject(vol, proj, P, v.voxel_size, v.origin, stream)
        torch.cuda.synchronize()
        g = None
        if graph:
            g = torch.cuda.CUDAGraph()
            cs = torch.cuda.Stream(device=self.dev)
            cs.wait_stream(stream)
            with torch.cuda.stream(cs):
                g.capture_begin()
                ctx.backproject(vol, proj, P, v.voxel_size, v.origin, cs)
                g.capture_end()
            torch.cuda.synchronize()
        vol.zero_()
        if graph and timing == "inside":
            timing = "after"
        if timing == "inside":
            ctx.enable_timing(True)
        starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        torch.cuda.synchronize()
        for i in range(steps):
            starts[i].record(stream)
            if g is not None:
                g.replay()
            else:
                ctx.backproject(vol, proj, P, v.voxel_size, v.origin, stream)
            ends[i].record(stream)
        torch.cuda.synchronize()
        step_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
        vol /= float(steps)
        kern = None
        if timing == "inside":
            kern = {k: ctx.kernel_timing(k) for k in ("backproject", "pad", "views")}
            kern["reconstructions"] = steps
            ctx.enable_timing(False)
        elif timing == "after":
            scratch = torch.zeros(shape, dtype=torch.float32, device=self.dev)
            ctx.enable_timing(True)
            for _ in range(min(steps, 3)):
                ctx.backproject(scratch, proj, P, v.voxel_size, v.origin, stream)
            torch.cuda.synchronize()
            kern = {k: ctx.kernel_timing(k) for k in ("backproject", "pad", "views")}
            kern["reconstructions"] = min(steps, 3)
            ctx.enable_timing(False)
            del scratch
        return step_ms, kern, vol

    def plan_of(self, ctx, v, n):
        p = ctx.plan(v.L, v.L, v.L, n)
        return {"path": p.path, "views_per_pass": p.views_per_pass, "z_unroll": p.z_unroll, "tile_x": p.tile_x,
                "direct_taps": p.direct_taps}

    # ------------------------------------------------------------------ candidates
    def cands_l512(self, n):
        C = self.at.Candidate
        out = [C("fused", k, zu, tx, sp) for k in (32, 64, 128) for zu in (4, 8) for tx in (8, 16, 32)
               for sp in (-1, 0, 1, 2, 4)]
        # wider passes, up to every view in one, in the shapes that lead at K = 64 and 128
        out += [C("fused", k, 8, tx, sp) for k in (256, n) for tx in (16, 32) for sp in (-1, 0)]
        out += [C("fused", k, 8, 16, -1, True) for k in (32, 64)]
        return [c for c in out if c.views_per_pass <= n]

    def cands_l1024(self):
        C = self.at.Candidate
        out = [C("fused", k, 8, 16) for k in (1, 2, 4)]  # HBM-bound: the tile shape hardly matters
        out += [C("fused", k, zu, tx) for k in (8, 16) for zu in (4, 8) for tx in (16, 32)]
        out += [C("fused", k, 8, tx, sp) for k in (32, 64, 128) for tx in (16, 32) for sp in (-1, 0, 1, 2, 4)]
        out += [C("fused", k, 8, tx, sp) for k in (256, 496) for tx in (16, 32) for sp in (-1, 0)]
        out += [C("fused", k, 8, 16, -1, True) for k in (64, 128)]
        return out

    def cands_plain(self):
        """The plain form (one volume pass per view) over its z-unroll, tile width and the column
        branch (hoisting Part 1 out of the z loop, or not)."""
        C = self.at.Candidate
        return [C("plain", 1, zu, tx, -1, False, nc) for zu in (1, 2, 4, 8) for tx in (16, 64) for nc in (False, True)]

    def cands_serving(self, L, n):
        C = self.at.Candidate
        out = [C("fused_direct", 64, 8, 16), C("fused_direct", 32, 8, 16), C("fused_direct", 64, 8, 64)]
        if L >= 256:
            out += [C("fused", k, 8, 16) for k in (64, 128)]
        return [c for c in out if c.views_per_pass <= n]


# ---------------------------------------------------------------------------- legs

def headline(b: Bench, res: dict):
    args, torch, synth = b.args, b.torch, b.synth
    wl = synth.WORKLOADS["fdk_l512_v496_f32"]
    v, sc = wl.volume, wl.scanner
    proj32 = b.stack(wl)
    if args.copy_calibration:
        src = torch.empty(args.copy_calibration << 18, dtype=torch.float32, device=b.dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copy calibration: 3 x {args.copy_calibration} MiB device-to-device")
        del src, dst
    P64, P = b.matrices(sc)
    wname = wl.name
    if args.tilt:
        P = torch.from_numpy(tilt_matrices(P64, args.tilt)).to(b.dev)
        wname = f"{wl.name}_tilt{args.tilt:g}"
    res["workload"] = wname
    updates = float(v.L) ** 3 * sc.n_views
    forms = [f for f in args.forms.split(",") if f]
    projs = {"f32": proj32}
    fixed = args.k or args.zu or args.tx or args.direct_taps or args.tap_split >= 0
    out, vols = {}, {}
    for form in forms:
        path, dt = form.rsplit("_", 1)
        path = {"direct": "fused_direct"}.get(path, path)
        if dt not in projs:
            projs[dt] = proj32.to({"bf16": torch.bfloat16, "f16": torch.float16}[dt])
        proj = projs[dt]
        ctx = b.context(sc.W, sc.H, dt)
        tuning = None
        if path in ("fused", "plain") and not args.no_tune and not fixed:
            scratch = torch.zeros((v.L,) * 3, dtype=torch.float32, device=b.dev)
            geo = f"tilt{args.tilt:g}" if args.tilt else ""  # another geometry: its own cache entries
            if path == "fused":
                _, tuning = b.tune(ctx, scratch, proj, P, v, b.cands_l512(sc.n_views), f"L=512 {dt}", tag=geo)
            else:
                _, tuning = b.tune(ctx, scratch, proj, P, v, b.cands_plain(), f"L=512 plain {dt}",
                                   include_auto=False, tag="plain" + (f"|{geo}" if geo else ""))
            del scratch
        else:
            ctx.set_tuning(path, args.k, args.zu, args.tx)
            ctx.set_options(direct_taps=args.direct_taps)
            ctx.set_tap_split(args.tap_split)
        plan = b.plan_of(ctx, v, sc.n_views)
        step_ms, kern, vol = b.run(ctx, proj, P, v, args.steps, args.warmup)
        ctx.close()
        r = {**plan, "dtype": dt, **stats(step_ms, updates), "kernels": kern, "tuning": tuning,
             "tap_split": tuning["tap_split"] if tuning else args.tap_split}
        log(f"bench: {form}: {r['ms_per_step']} ms/step, p50 {r['gups_p50']} GUPS, plan {plan}, kernels {kern}")
        out[form] = r
        vols[form] = vol
    res["clocks_after_headline"] = clocks()

    # FDK pre-processing of a stack of this shape (the step before the path)
    if not args.no_fdk:
        with b.bp.FdkFilter.for_scanner(sc) as f:
            o = torch.empty_like(proj32)
            for _ in range(2):
                f.filter(proj32, "f32", out=o)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                f.filter(proj32, "f32", out=o)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            del o
        pix = float(sc.n_views) * sc.H * sc.W
        res["fdk_preprocessing"] = {"kernel": "fdk_kernel", "ms_per_stack": round(ms, 3),
                                    "gpixel_per_s": round(pix / ms / 1e6, 2),
                                    "hbm_gbs_algorithmic": round(pix * 8 / ms / 1e6, 1),
                                    "hbm_frac": round(pix * 8 / ms / 1e6 / HBM_PEAK_GBS, 4)}
        log(f"bench: FDK {res['fdk_preprocessing']}")

    # errors and the CPU baseline: the oracle on the centre block
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        from oracle.bp import default_threads

        bl = args.cpu_block
        lo = (v.L - bl) // 2
        blk = ((lo, lo + bl),) * 3
        P_or = oracle.geometry.circular_matrices(*sc.geometry_args())
        P_or = (tilt_matrices(P_or, args.tilt) if args.tilt else P_or.astype(np.float32)).astype(np.float64)
        thr = default_threads()
        t = time.perf_counter()
        ref = oracle.backproject(proj32.cpu().numpy(), P_or, v.L, v.voxel_size, v.origin, block=blk, threads=thr)
        dt = time.perf_counter() - t
        n_upd = float(bl) ** 3 * sc.n_views
        cpu = {"value": round(n_upd / dt / 1e9, 4), "unit": "GUPS", "cores": thr, "kind": "oracle",
               "sample": f"centre {bl}^3 block of the {v.L}^3 volume x {sc.n_views} views "
                         f"({n_upd:.3g} voxel updates, FP64, {dt:.1f} s)"}
        log(f"bench: oracle {cpu}")
        for form, vol in vols.items():
            out[form]["error_vs_fp64_oracle"] = error_stats(vol[lo:lo + bl, lo:lo + bl, lo:lo + bl].double().cpu().numpy(),
                                                            ref)
        del ref
    res["cpu_baseline"] = cpu
    res["forms"] = out

    # roofline of the dominant kernel of the headline form
    head = out.get("fused_f32") or next(iter(out.values()))
    ms_bp, n_bp = head["kernels"]["backproject"]
    per_launch_ms = ms_bp / max(n_bp, 1)
    upl = updates * head["kernels"]["reconstructions"] / max(n_bp, 1)
    tflops = FLOPS_PER_UPDATE * upl / (per_launch_ms * 1e-3) / 1e12
    if head["path"] == "fused" and not head["direct_taps"]:
        kernel = "backproject_lds_kernel"
    else:
        kernel = "backproject_kernel"
    k = head["views_per_pass"]
    split = head["tap_split"]
    if split < 0 and kernel == "backproject_lds_kernel":
        split = 0  # the library's share of directly read views for FP32 pixel stages
    launch = f"K={k} ZU={head['z_unroll']} TX={head['tile_x']} split={split}"
    rec = counter_record(kernel, launch, wname)
    views_per_launch = upl / float(v.L) ** 3
    alg_bytes = upl * (8.0 / views_per_launch + sc.W * sc.H * 4.0 / float(v.L) ** 3)
    traffic = None
    valu = None
    if rec:
        traffic = (rec["fetch_kib_per_launch"] * rec["fetch_scale"] + rec["write_kib_per_launch"] * rec["write_scale"]) * 1024
        if rec.get("valu_per_update"):
            vpu = rec["valu_per_update"]
            valu = {"instr_per_update": vpu, "issue_frac": round(vpu * upl / (per_launch_ms * 1e-3) / 1e12 / VALU_PEAK_T, 4),
                    "peak_tinstr_per_s": round(VALU_PEAK_T, 2)}
    res["roofline"] = {
        "bound": "alu", "achieved": round(tflops, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
        "frac": round(tflops / FP32_PEAK_TFLOPS, 4), "traffic": round(traffic) if traffic else None,
        "kernel": kernel, "launch": launch, "avg_launch_ms": round(per_launch_ms, 4),
        "updates_per_launch": upl, "flops_per_update": FLOPS_PER_UPDATE,
        "valu_issue": valu,
        "hbm_algorithmic_bytes": round(alg_bytes),
        "traffic_over_algorithmic": round(traffic / alg_bytes, 3) if traffic else None,
        "hbm_frac_algorithmic": round(alg_bytes / (per_launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "culled_share": culled_share(b, P, v, sc, head["tile_x"], head["z_unroll"]),
    }
    log(f"bench: roofline {res['roofline']}")
    del projs, vols, proj32
    b.free()
    return P64


def culled_share(b, P, v, sc, tx, zu):
    """Share of (block tile, view) pairs whose tile projects wholly beyond one detector edge (the
    clipping mask's test on the tile's 8 corners, FP64), for the tile shape of the launch; such
    pairs still count as updates (their contribution is exactly 0)."""
    torch = b.torch
    ty = 256 // tx
    gx, gy, gz = -(-v.L // tx), -(-v.L // ty), -(-v.L // zu)
    dev = b.dev

    def corners(g, t, o):
        lo = torch.arange(g, device=dev, dtype=torch.float64) * t
        hi = torch.clamp(lo + t - 1, max=v.L - 1)
        return torch.stack([lo, hi], 1) * v.voxel_size + o  # (g, 2)

    X = corners(gx, tx, v.origin[0])
    Y = corners(gy, ty, v.origin[1])
    Z = corners(gz, zu, v.origin[2])
    Pm = P.double().reshape(-1, 3, 4)
    skipped = 0
    for k0 in range(0, Pm.shape[0], 32):
        p = Pm[k0:k0 + 32].view(-1, 3, 4, 1, 1, 1)
        allc = None
        for cz in range(2):
            for cy in range(2):
                for cx in range(2):
                    xx = X[:, cx].view(1, 1, 1, gx)
                    yy = Y[:, cy].view(1, 1, gy, 1)
                    zz = Z[:, cz].view(1, gz, 1, 1)
                    u = p[:, 0, 0] * xx + p[:, 0, 1] * yy + p[:, 0, 2] * zz + p[:, 0, 3]
                    vv = p[:, 1, 0] * xx + p[:, 1, 1] * yy + p[:, 1, 2] * zz + p[:, 1, 3]
                    w = p[:, 2, 0] * xx + p[:, 2, 1] * yy + p[:, 2, 2] * zz + p[:, 2, 3]
                    c = torch.stack([u <= -2.0 * w, u >= (sc.W + 1.0) * w, vv <= -2.0 * w, vv >= (sc.H + 1.0) * w])
                    allc = c if allc is None else allc & c
        skipped += int(allc.any(0).sum())
    return round(skipped / (gx * gy * gz * Pm.shape[0]), 4)


VALU_CLASSES = ("v_fma_f32", "v_mul_f32", "v_add_f32", "v_rcp_f32", "v_cvt_flr_i32_f32", "v_fract_f32",
                "v_med3_f32", "v_mad_u32_u24", "v_floor_f32", "v_cvt_i32_f32", "v_cvt_f32_i32", "v_add_u32",
                "v_and_b32", "v_lshl_add_u32", "v_mul_u32_u24", "v_max_f32", "v_sub_f32", "v_fma_mix_f32",
                "v_cndmask_b32", "v_fmac_f32", "v_add_lshl_u32")


def probe_lib():
    """libbpprobe.so (the roof microbenchmarks), bound with ctypes."""
    import ctypes

    from paper_1401_7494_amd import build

    if not os.path.exists(build.PROBE_LIB):
        raise RuntimeError(f"{build.PROBE_LIB} is missing: build it with `python -m paper_1401_7494_amd.build`")
    lib = ctypes.CDLL(build.PROBE_LIB)
    vp, ci, cl, cf = ctypes.c_void_p, ctypes.c_int, ctypes.c_long, ctypes.c_float
    lib.probe_update.argtypes = [vp, cl, cf, ci, vp]
    lib.probe_copy.argtypes = [vp, vp, cl, ci, vp]
    lib.probe_valu.argtypes = [ci, vp, ci, ci, vp]
    lib.probe_valu_per_lane.argtypes = [ci]
    lib.probe_valu_per_lane.restype = ctypes.c_longlong
    lib.probe_valu_threads.argtypes = [ci]
    lib.probe_valu_threads.restype = ctypes.c_longlong
    for f in (lib.probe_update, lib.probe_copy, lib.probe_valu):
        f.restype = ci
    return lib


def leg_roofs(b: Bench):
    """Measured roofs: streaming FP32 read-modify-write of a 512^3 array (the 8 bytes per update of
    the plain form; the "Node Update" benchmark of Table 1), a copy of the same size, and the issue
    rate of each VALU instruction class the pass uses (lane-instructions/s; peak 39.3 T)."""
    torch = b.torch
    lib = probe_lib()
    s = torch.cuda.current_stream(b.dev)
    n = 512 ** 3
    a = torch.zeros(n, dtype=torch.float32, device=b.dev)
    c = torch.empty_like(a)

    def timed(fn, reps=5):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = []
        for _ in range(reps):
            e0.record(s)
            fn()
            e1.record(s)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms))

    out = {"array": "512^3 FP32 (537 MB)"}
    best = {}
    for blocks in (1024, 2048, 4096, 8192, 32768, n // 4 // 256):
        t = timed(lambda: lib.probe_update(a.data_ptr(), n, 1.0, blocks, s.cuda_stream))
        best["update", blocks] = 8.0 * n / (t * 1e-3) / 1e9
        t = timed(lambda: lib.probe_copy(a.data_ptr(), c.data_ptr(), n, blocks, s.cuda_stream))
        best["copy", blocks] = 8.0 * n / (t * 1e-3) / 1e9
    for kind in ("update", "copy"):
        bb = max((v, k[1]) for k, v in best.items() if k[0] == kind)
        out[f"{kind}_gbs"] = round(bb[0], 1)
        out[f"{kind}_blocks"] = bb[1]
    out["update_frac_of_8tbs"] = round(out["update_gbs"] / HBM_PEAK_GBS, 4)
    out["plain_gups_ceiling_l512"] = round(out["update_gbs"] / 8.036, 1)  # 8 B RMW + 0.036 B of pixels per update
    del a, c
    blocks, iters = 4096, 2048
    o = torch.empty(int(lib.probe_valu_threads(blocks)), dtype=torch.float32, device=b.dev)
    lanes = float(lib.probe_valu_threads(blocks)) * float(lib.probe_valu_per_lane(iters))
    rates = {}
    for k, name in enumerate(VALU_CLASSES):
        t = timed(lambda: lib.probe_valu(k, o.data_ptr(), blocks, iters, s.cuda_stream))
        rates[name] = round(lanes / (t * 1e-3) / 1e12, 2)
    out["valu_tinstr_per_s"] = rates
    out["valu_peak_tinstr_per_s"] = round(VALU_PEAK_T, 2)
    del o
    b.free()
    log(f"bench: roofs {out}")
    return out


def leg_c1(b: Bench):
    args, torch, synth = b.args, b.torch, b.synth
    wl = synth.WORKLOADS["fdk_l128_v496_f32"]
    v, sc = wl.volume, wl.scanner
    proj = b.stack(wl)
    _, P = b.matrices(sc)
    updates = float(v.L) ** 3 * sc.n_views
    out = {"workload": wl.name, "L": v.L, "voxel_mm": v.voxel_size, "views": sc.n_views}
    vols = {}
    for name, path in (("plain_f32", "plain"), ("tuned_f32", None)):
        ctx = b.context(sc.W, sc.H, "f32")
        tuning = None
        if path:
            scratch = torch.zeros((v.L,) * 3, dtype=torch.float32, device=b.dev)
            _, tuning = b.tune(ctx, scratch, proj, P, v, b.cands_plain(), "L=128 plain f32", include_auto=False,
                               tag="plain")
            del scratch
        else:
            scratch = torch.zeros((v.L,) * 3, dtype=torch.float32, device=b.dev)
            C = b.at.Candidate
            cands = [C("fused_direct", k, 8, tx) for k in (32, 64, 128) for tx in (16, 64)]
            cands += [C("fused", 64, 8, 16)]
            _, tuning = b.tune(ctx, scratch, proj, P, v, cands, "L=128 f32")
            del scratch
        plan = b.plan_of(ctx, v, sc.n_views)
        steps = max(args.config_steps, 10)
        step_ms, kern, vol = b.run(ctx, proj, P, v, steps, 2, timing="after")
        # the same reconstruction captured once in a HIP graph and replayed (launch costs paid once)
        g_ms, _, g_vol = b.run(ctx, proj, P, v, steps, 2, timing=None, graph=True)
        ctx.close()
        out[name] = {**plan, **stats(step_ms, updates), "tuning": tuning,
                     "backproject_ms_per_launch": round(kern["backproject"][0] / max(kern["backproject"][1], 1), 4),
                     "launches_per_step": kern["backproject"][1] // kern["reconstructions"],
                     "graph_replay": {**stats(g_ms, updates), "equal_to_eager": bool(torch.equal(g_vol, vol))}}
        vols[name] = vol
        log(f"bench: C1 {name}: {out[name]}")
    pl = out["plain_f32"]
    # K = 1: 8 B of volume read-modify-write per update (Sec. 4.2) + the view's pixels once per pass
    out["plain_f32"]["hbm_gbs_algorithmic"] = round(updates * (8.0 + sc.W * sc.H * 4.0 / v.L ** 3)
                                                    / (pl["ms_per_step"] * 1e-3) / 1e9, 1)
    import oracle

    P_or = oracle.geometry.circular_matrices(*sc.geometry_args()).astype(np.float32).astype(np.float64)
    t = time.perf_counter()
    ref = oracle.backproject(proj.cpu().numpy(), P_or, v.L, v.voxel_size, v.origin)
    out["oracle_s"] = round(time.perf_counter() - t, 2)
    for name, vol in vols.items():
        out[name]["error_vs_fp64_oracle"] = error_stats(vol.double().cpu().numpy(), ref)
    out["error_region"] = "whole 128^3 volume"
    del proj, vols, ref
    b.free()
    return out


def strided(L, stride, offset):
    idx = np.arange(offset, L, stride)
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def leg_c3(b: Bench):
    args, torch, synth = b.args, b.torch, b.synth
    wl = synth.WORKLOADS["fdk_l1024_v496_f32"]
    v, sc = wl.volume, wl.scanner
    proj = b.stack(wl)
    _, P = b.matrices(sc)
    updates = float(v.L) ** 3 * sc.n_views
    ctx = b.context(sc.W, sc.H, "f32")
    vol = torch.zeros((v.L,) * 3, dtype=torch.float32, device=b.dev)
    _, tuning = b.tune(ctx, vol, proj, P, v, b.cands_l1024(), "L=1024 f32")
    del vol
    b.free()
    plan = b.plan_of(ctx, v, sc.n_views)
    step_ms, kern, vol = b.run(ctx, proj, P, v, args.config_steps, 1)
    ctx.close()
    out = {"workload": wl.name, "L": v.L, "voxel_mm": v.voxel_size, "views": sc.n_views,
           "fused_f32": {**plan, **stats(step_ms, updates), "tuning": tuning,
                         "backproject_ms_per_launch": round(kern["backproject"][0] / max(kern["backproject"][1], 1), 4)}}
    # the search's per-K best (the required set K = 1, 2, 4, 8, 16 and wider)
    cache = b.at.load_cache(b.cache)
    key = b.at.Problem(v.L, v.L, v.L, sc.n_views, "f32", sc.W, sc.H).key(b.dev_name)
    timings = cache.get(key, {}).get("timings_ms", {})
    per_k = {}
    for ck, ms in timings.items():
        parts = ck.split("/")
        if parts[0] != "fused":
            continue
        kk = int(parts[1])
        if kk not in per_k or ms < per_k[kk][0]:
            per_k[kk] = (ms, ck)
    out["search_best_per_k"] = {str(kk): {"ms": round(ms, 2), "gups": round(updates / (ms * 1e-3) / 1e9, 1),
                                          "choice": ck} for kk, (ms, ck) in sorted(per_k.items())}
    import oracle

    xyz = strided(v.L, 16, 7)
    P_or = oracle.geometry.circular_matrices(*sc.geometry_args()).astype(np.float32).astype(np.float64)
    ref = oracle.backproject_points(proj.cpu().numpy(), P_or, v.voxel_size, v.origin, xyz)
    got = vol[xyz[:, 2], xyz[:, 1], xyz[:, 0]].double().cpu().numpy()
    out["fused_f32"]["error_vs_fp64_oracle"] = error_stats(got, ref)
    out["error_region"] = "every 16th voxel per axis (64^3 voxels spread over the volume)"
    log(f"bench: C3 {out}")
    del proj, vol
    b.free()
    return out


def leg_c4(b: Bench):
    args, torch, synth = b.args, b.torch, b.synth
    import oracle

    out = {}
    bl = 128
    for dt in ("f16", "bf16"):
        wl = synth.WORKLOADS[f"fdk_l512_v496_{dt}_noisy"]
        v, sc = wl.volume, wl.scanner
        if not out:
            proj32 = b.stack(wl)  # the same noisy FP32 stack for both storage types
            _, P = b.matrices(sc)
            lo = (v.L - bl) // 2
            blk = ((lo, lo + bl),) * 3
            P_or = oracle.geometry.circular_matrices(*sc.geometry_args()).astype(np.float32).astype(np.float64)
            ref32 = oracle.backproject(proj32.cpu().numpy(), P_or, v.L, v.voxel_size, v.origin, block=blk)
        tdt = {"f16": torch.float16, "bf16": torch.bfloat16}[dt]
        proj = proj32.to(tdt)
        ref_r = oracle.backproject(proj.float().cpu().numpy(), P_or, v.L, v.voxel_size, v.origin, block=blk)
        updates = float(v.L) ** 3 * sc.n_views
        ctx = b.context(sc.W, sc.H, dt)
        scratch = torch.zeros((v.L,) * 3, dtype=torch.float32, device=b.dev)
        cand, tuning = b.tune(ctx, scratch, proj, P, v, b.cands_l512(sc.n_views), f"L=512 {dt}")
        del scratch
        plan = b.plan_of(ctx, v, sc.n_views)
        step_ms, kern, vol = b.run(ctx, proj, P, v, args.config_steps, 1)
        # FP32 staging (the default: the 16-bit pixels widened exactly): storage rounding alone
        r = {**plan, **stats(step_ms, updates), "staging": "fp32 (16-bit pixels widened)", "tuning": tuning}
        g = vol[lo:lo + bl, lo:lo + bl, lo:lo + bl].double().cpu().numpy()
        r["error_vs_oracle_fp32_data"] = error_stats(g, ref32)
        r["error_vs_oracle_rounded_data"] = error_stats(g, ref_r)
        # compact FP16 records (K = 128, the library's split for them), timed as well
        b.at.apply(ctx, b.at.Candidate("fused", 128, 8, 16, -1), compact_staging=True)
        step_c, _, volc = b.run(ctx, proj, P, v, args.config_steps, 1, timing=None)
        gc_ = volc[lo:lo + bl, lo:lo + bl, lo:lo + bl].double().cpu().numpy()
        r["compact"] = {"launch": "fused/128/8/16, 3 of 8 views direct", **stats(step_c, updates),
                        "error_vs_oracle_fp32_data": error_stats(gc_, ref32),
                        "error_vs_oracle_rounded_data": error_stats(gc_, ref_r)}
        ctx.close()
        r["error_region"] = f"centre {bl}^3 block"
        out[f"fused_{dt}"] = r
        log(f"bench: C4 {dt}: {r}")
        del proj, vol, volc
    out.update(workload="fdk_l512_v496_{f16,bf16}_noisy", L=512, views=496, noise="N(0, (0.01 max|p|)^2) on the "
               "filtered pixels, then rounded to FP16 / BF16")
    del proj32
    b.free()
    return out


def leg_general(b: Bench, P64_c2):
    """The benchmark workload through a tilted orbit: the gantry tilted by TILT_DEG about x, so that
    every view has P[0][2] and P[2][2] non-zero (no column branch).  The projections are the
    circular orbit's; the tilt rotates the reconstructed object, not the throughput."""
    args, torch, synth = b.args, b.torch, b.synth
    wl = synth.WORKLOADS["fdk_l512_v496_f32"]
    v, sc = wl.volume, wl.scanner
    proj = b.stack(wl)
    Pt32 = tilt_matrices(P64_c2, TILT_DEG)
    share = float(np.mean((Pt32[:, 0, 2] != 0) & (Pt32[:, 2, 2] != 0)))
    P = torch.from_numpy(Pt32).to(b.dev)
    updates = float(v.L) ** 3 * sc.n_views
    ctx = b.context(sc.W, sc.H, "f32")
    tuning = None
    if not args.no_tune:  # the autotuner's launch for this geometry, cached apart from the circular orbit's
        scratch = torch.zeros((v.L,) * 3, dtype=torch.float32, device=b.dev)
        _, tuning = b.tune(ctx, scratch, proj, P, v, b.cands_l512(sc.n_views), "L=512 tilted f32",
                           tag=f"tilt{TILT_DEG:g}")
        del scratch
    plan = b.plan_of(ctx, v, sc.n_views)
    step_ms, kern, vol = b.run(ctx, proj, P, v, args.config_steps, 1)
    ctx.close()
    import oracle

    xyz = strided(v.L, 8, 3)
    ref = oracle.backproject_points(proj.cpu().numpy(), Pt32.astype(np.float64), v.voxel_size, v.origin, xyz)
    got = vol[xyz[:, 2], xyz[:, 1], xyz[:, 0]].double().cpu().numpy()
    out = {"workload": f"{wl.name} with the orbit tilted {TILT_DEG} degrees about x",
           "views_off_the_column_branch": share, "fused_f32": {**plan, **stats(step_ms, updates), "tuning": tuning,
           "backproject_ms_per_launch": round(kern["backproject"][0] / max(kern["backproject"][1], 1), 4),
           "error_vs_fp64_oracle": error_stats(got, ref)},
           "error_region": "every 8th voxel per axis (64^3 voxels)"}
    log(f"bench: general branch {out}")
    del proj, vol
    b.free()
    return out


def leg_c5(b: Bench):
    from paper_1401_7494_amd import serve

    torch, synth = b.torch, b.synth
    # the autotuner's launch for every shape of the mix, into the cache the executor reads
    t = time.perf_counter()
    tuned = {}
    sc0 = synth.Scanner()
    for n in (124, 248, 496):
        sc = synth.Scanner(n_views=n)
        _, P = b.matrices(sc)
        for dt in ("f32", "f16"):
            proj = (torch.rand((n, sc.H, sc.W), device=b.dev) - 0.5).to({"f32": torch.float32, "f16": torch.float16}[dt])
            for L in (128, 256, 512):
                v = synth.standard_volume(L)
                vol = torch.zeros((L,) * 3, dtype=torch.float32, device=b.dev)
                ctx = b.context(sc.W, sc.H, dt)
                best, info = b.at.ensure_tuned(ctx, vol, proj, P, v.voxel_size, v.origin, cands=b.cands_serving(L, n),
                                               cache_path=b.cache, device_name=b.dev_name)
                ctx.close()
                tuned[f"L{L}_v{n}_{dt}"] = {"choice": best.key(), "source": info["source"],
                                            "margin_over_auto": round(info["auto_ms"] / info["best_ms"], 3)
                                            if "auto_ms" in info else None}
                del vol
            del proj
    b.free()
    tune_s = time.perf_counter() - t
    log(f"bench: serving shapes tuned in {tune_s:.1f} s: {tuned}")
    ex = serve.GpuExecutor(tuning_cache=b.cache)
    cap, poi = serve.serve_mix(ex, n_requests=b.args.serve_requests, log=log)
    ex.close()
    b.free()
    return {"workload": f"{b.args.serve_requests} seeded requests (seed 1405): L in 128/256/512, 124/248/496 views "
                        f"of {sc0.W}x{sc0.H}, FP32/FP16; raw projections made on the device and filtered by the "
                        "library's FDK row at admission; 200 GiB HBM budget, 8 in flight",
            "capacity": cap, "poisson": poi, "tuned_shapes": tuned, "tuning_s": round(tune_s, 1)}


def main():
    args = parse()
    global NO_CLOCKS
    NO_CLOCKS = args.no_clocks
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (sharding the volume into z-slabs "
              "across GPUs is designed but not implemented)", file=sys.stderr)
        sys.exit(2)
    b = Bench(args)
    torch = b.torch
    t_all = time.perf_counter()
    log(f"bench: {b.dev_name}, autotune cache {b.cache}")
    res = {"clocks_before": clocks()}
    P64 = headline(b, res)
    configs = {}
    want = [c for c in args.configs.split(",") if c]
    for name in want:
        t = time.perf_counter()
        if name == "C1":
            configs["C1"] = leg_c1(b)
        elif name == "C3":
            configs["C3"] = leg_c3(b)
        elif name == "C4":
            configs["C4"] = leg_c4(b)
        elif name == "C5":
            configs["C5"] = leg_c5(b)
        elif name == "general":
            configs["general_branch"] = leg_general(b, P64)
        elif name == "roofs":
            res["measured_roofs"] = leg_roofs(b)
        else:
            raise SystemExit(f"unknown config {name}")
        log(f"bench: {name} done in {time.perf_counter() - t:.1f} s")
    head = res["forms"].get("fused_f32") or next(iter(res["forms"].values()))
    line = {
        "metric": "GUPS (voxel updates/s) at L=512, 496 views: fused/BF16 vs plain FP32; p50/p99",
        "value": head["gups_mean"],
        "unit": "GUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded random-ellipsoid phantom standing in for the RabbitCT dataset)",
        "config": {"workload": res.get("workload", "fdk_l512_v496_f32"), "L": 512, "voxel_mm": 0.5, "views": 496,
                   "detector": [1248, 960], "form": "fused_f32", "parallelism": "single GPU"},
        "p50_gups": head["gups_p50"],
        "p99_gups": head["gups_p99"],
        "forms": res["forms"],
        "roofline": res["roofline"],
        "measured_roofs": res.get("measured_roofs"),
        "cpu_baseline": res["cpu_baseline"],
        "configs": configs,
        "fdk_preprocessing": res.get("fdk_preprocessing"),
        "device": device_info(torch),
        "clocks": {"before": res["clocks_before"], "after_headline": res.get("clocks_after_headline"),
                   "end": clocks()},
        "bench_s": round(time.perf_counter() - t_all, 1),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
