#!/usr/bin/env python3
"""Throughput of the HIP back projector on one MI355X.

Workload: L=512 volume (512^3 FP32, voxel 0.5 mm, centred), 496 filtered
projections of 1248 x 960 from a seeded random-ellipsoid phantom on a 200
degree circular orbit (SID 800 mm, SDD 1200 mm, pitch 0.32 mm).  A step is
one full reconstruction: all 496 views back projected into the volume
(per-view constants, zero-padded staging and the back-projection passes),
inputs resident in HBM.  GUPS = L^3 * views / step time.

Forms timed on the same GPU and inputs:
  fused_f32    K views per volume pass, FP32 projections (the headline `value`)
  plain_f32    one volume pass per view (the paper's one-call-per-projection form)
  fused_bf16   fused, projections stored as BF16 (FP32 interpolation and accumulation)
  fused_f16    fused, projections stored as FP16
  direct_f32   fused, taps from the caller's images (no staging copy; small volumes)
  auto_f32     the library's own choice of path

Prints one JSON line.  Each form's error is stated against the FP64 oracle on
the FP32 data over the centre 128^3 block (the CPU-baseline sample).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Minimal VALU instructions per voxel update of the fused pass on a column view
# (row FMA, clamp, convert, fraction, index mad, three patch FMAs, accumulate),
# counted in the gfx950 ISA of backproject_kernel.
VALU_PER_UPDATE = 9
VALU_PEAK_T = 256 * 64 * 2.4e9 / 1e12  # 256 CUs x 64 lanes/clk x 2.4 GHz, lane-instructions/s (no packed FP32)
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("paper_1401_7494_amd/csrc/bp_kernels.hip", "paper_1401_7494_amd/csrc/bp_internal.h")
COUNTERS_MD = "profiles/backproject_fused_f32_l512_v496_counters.md"


def kernel_source_sha():
    """SHA-256 of the kernel sources with comments and white space removed (so that an edit of a
    comment keeps a counter record valid, while any change of the code does not)."""
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


def measured_traffic(kernel: str, launch: str, workload: str):
    """HBM-side bytes per launch of the fused FP32 pass from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a copy of known size), or None when the kernel sources
    have changed since the counters were taken or the summary is for another kernel or launch."""
    path = os.path.join(ROOT, COUNTERS_MD)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if "```json" not in text:
        return None
    rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    if rec.get("kernel_source_sha256") != kernel_source_sha() or rec.get("kernel") != kernel:
        return None
    if rec.get("launch_key") != launch or rec.get("workload") != workload:
        return None
    return (rec["fetch_kib_per_launch"] * rec["fetch_scale"] + rec["write_kib_per_launch"] * rec["write_scale"]) * 1024


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--forms", default="fused_f32,plain_f32,fused_bf16,fused_f16")
    ap.add_argument("--workload", default="fdk_l512_v496_f32")
    ap.add_argument("--k", type=int, default=0, help="views per pass for fused forms (0 = tuned)")
    ap.add_argument("--zu", type=int, default=0, help="z-unroll (0 = tuned)")
    ap.add_argument("--tx", type=int, default=0, help="block tile width along x (0 = tuned)")
    ap.add_argument("--order", default="region", choices=("region", "plain", "zslices"), help="tile order")
    ap.add_argument("--region-ax", type=int, default=0, help="XCD regions along x for --order region (0 = default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cull", action="store_true", help="time without the clipping mask")
    ap.add_argument("--no-column", action="store_true", help="time without the column specialisation")
    ap.add_argument("--direct-taps", action="store_true", help="fused forms read every tap directly (no LDS stage)")
    ap.add_argument("--tap-split", type=int, default=-1, help="views of every 8 read directly in a staged pass (-1 = tuned)")
    ap.add_argument("--staging", default="auto", choices=("auto", "serial", "overlap"),
                    help="stage each pass just before it, or the next pass while one runs (auto: tuned)")
    ap.add_argument("--no-fdk", action="store_true", help="skip timing the FDK pre-processing of the stack")
    ap.add_argument("--cpu-block", type=int, default=320,
                    help="edge of the centre block the oracle times (about 10 s of FP64 work on 16 threads)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device 3 times (a known-size kernel for HBM counters)")
    return ap.parse_args()


def _device_info(torch):
    p = torch.cuda.get_device_properties(0)
    return {"name": torch.cuda.get_device_name(0), "arch": getattr(p, "gcnArchName", None),
            "compute_units": p.multi_processor_count, "memory_gib": round(p.total_memory / 2 ** 30, 1)}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_form(bp, torch, form, proj_by_dtype, P, vol_cfg, steps, warmup, k, zu, tx=0, no_cull=False,
              no_column=False, order="region", region_ax=0, direct_taps=False, tap_split=-1, staging="auto"):
    path, dt = form.rsplit("_", 1)
    path = {"direct": "fused_direct"}.get(path, path)
    proj = proj_by_dtype[dt]
    n, H, W = proj.shape
    L = vol_cfg.L
    dev = proj.device
    vol = torch.zeros((L, L, L), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    ctx = bp.Context(W, H, dt)
    ctx.set_tuning(path, k, zu, tx)
    ctx.set_options(no_cull=no_cull, no_column=no_column, order=order, region_ax=region_ax, direct_taps=direct_taps,
                    staging=staging)
    ctx.set_tap_split(tap_split)
    plan = ctx.plan(L, L, L, n)
    for _ in range(warmup):
        ctx.backproject(vol, proj, P, vol_cfg.voxel_size, vol_cfg.origin, stream)
    torch.cuda.synchronize()
    vol.zero_()
    ctx.enable_timing(True)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record(stream)
        ctx.backproject(vol, proj, P, vol_cfg.voxel_size, vol_cfg.origin, stream)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    kern = {kind: ctx.kernel_timing(kind) for kind in ("backproject", "pad", "views")}
    ctx.enable_timing(False)
    ctx.close()
    out = vol / float(steps)  # every step added the same reconstruction
    return {
        "path": plan.path, "dtype": dt, "views_per_pass": plan.views_per_pass, "z_unroll": plan.z_unroll,
        "tile_x": plan.tile_x, "direct_taps": plan.direct_taps,
        "step_ms": step_ms, "wall_s": wall, "kernels": kern, "volume": out,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (sharding the volume into z-slabs "
              "across GPUs is designed but not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1401_7494_amd import bp, synth

    wl = synth.WORKLOADS[args.workload]
    v = wl.volume
    sc = wl.scanner
    dev = torch.device("cuda:0")
    log(f"bench: workload {wl.name} L={v.L} views={sc.n_views} det={sc.W}x{sc.H} on {torch.cuda.get_device_name(0)}")
    t = time.perf_counter()
    proj32 = synth.filtered_projections(sc, synth.random_ellipsoids(wl.phantom_seed), device=dev,
                                        noise_frac=wl.noise_frac, noise_seed=wl.noise_seed)
    torch.cuda.synchronize()
    log(f"bench: inputs generated on the GPU in {time.perf_counter() - t:.1f} s")
    if args.copy_calibration:
        src = torch.empty(args.copy_calibration << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copy calibration: 3 x {args.copy_calibration} MiB device-to-device")
        del src, dst
    forms = [f for f in args.forms.split(",") if f]
    proj_by_dtype = {"f32": proj32}
    if any(f.endswith("bf16") for f in forms):
        proj_by_dtype["bf16"] = proj32.to(torch.bfloat16)
    if any(f.endswith("f16") and not f.endswith("bf16") for f in forms):
        proj_by_dtype["f16"] = proj32.to(torch.float16)
    _, P32 = bp.circular_matrices(*sc.geometry_args())
    P = torch.from_numpy(P32).to(dev)

    updates = float(v.L) ** 3 * sc.n_views
    # FDK pre-processing of a stack of this shape (the step before the path): the FP32 stack
    # stands in for the raw projections (the filter's cost does not depend on the values)
    fdk = None
    if not args.no_fdk:
        with bp.FdkFilter.for_scanner(sc) as f:
            out = torch.empty_like(proj32)
            for _ in range(2):
                f.filter(proj32, "f32", out=out)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(args.steps):
                f.filter(proj32, "f32", out=out)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / args.steps
            del out
        pix = float(sc.n_views) * sc.H * sc.W
        fdk = {"kernel": "fdk_kernel", "ms_per_stack": round(ms, 3), "gpixel_per_s": round(pix / ms / 1e6, 2),
               "hbm_gbs_algorithmic": round(pix * 8 / ms / 1e6, 1),
               "hbm_frac": round(pix * 8 / ms / 1e6 / HBM_PEAK_GBS, 4)}
        log(f"bench: FDK pre-processing {fdk}")
    results = {}
    for form in forms:
        r = time_form(bp, torch, form, proj_by_dtype, P, v, args.steps, args.warmup, args.k, args.zu, args.tx,
                      args.no_cull, args.no_column, args.order, args.region_ax, args.direct_taps, args.tap_split,
                      args.staging)
        ms = r["step_ms"]
        r["gups_mean"] = updates / (ms.mean() * 1e-3) / 1e9
        r["gups_p50"] = updates / (np.percentile(ms, 50) * 1e-3) / 1e9
        r["gups_p99"] = updates / (np.percentile(ms, 99) * 1e-3) / 1e9
        log(f"bench: {form}: {ms.mean():.2f} ms/step  p50 {r['gups_p50']:.1f} GUPS  p99 {r['gups_p99']:.1f} GUPS  "
            f"(path {r['path']} K={r['views_per_pass']} ZU={r['z_unroll']} TX={r['tile_x']}"
            f"{' direct taps' if r.get('direct_taps') else ''}) kernels {r['kernels']}")
        results[form] = r

    # CPU baseline: the oracle on the centre block, on this host's cores.
    cpu = None
    errors = {}
    if not args.no_cpu_baseline:
        import oracle
        from oracle.bp import default_threads

        b = args.cpu_block
        lo = (v.L - b) // 2
        blk = ((lo, lo + b),) * 3
        proj_np = proj32.cpu().numpy()
        P_or = oracle.geometry.circular_matrices(*sc.geometry_args()).astype(np.float32).astype(np.float64)
        thr = default_threads()
        t = time.perf_counter()
        ref = oracle.backproject(proj_np, P_or, v.L, v.voxel_size, v.origin, block=blk, threads=thr)
        dt = time.perf_counter() - t
        n_upd = float(b) ** 3 * sc.n_views
        cpu = {"value": round(n_upd / dt / 1e9, 4), "unit": "GUPS", "cores": thr, "kind": "oracle",
               "sample": f"centre {b}^3 block of the {v.L}^3 volume x {sc.n_views} views "
                         f"({n_upd:.3g} voxel updates, FP64, {dt:.1f} s)"}
        log(f"bench: oracle {cpu}")
        for form, r in results.items():
            got = r["volume"][lo:lo + b, lo:lo + b, lo:lo + b].double().cpu().numpy()
            d = got - ref
            errors[form] = {"rel_l2": float(np.linalg.norm(d) / np.linalg.norm(ref)),
                            "max_abs_over_max": float(np.abs(d).max() / np.abs(ref).max()),
                            "rms": float(np.sqrt(np.mean(d * d)))}

    head = results.get("fused_f32") or next(iter(results.values()))
    ms_bp, n_bp = head["kernels"]["backproject"]
    per_launch_ms = ms_bp / max(n_bp, 1)
    updates_per_launch = updates * args.steps / max(n_bp, 1)
    achieved = updates_per_launch * VALU_PER_UPDATE / (per_launch_ms * 1e-3) / 1e12
    kernel = "backproject_kernel" if head.get("direct_taps") else "backproject_lds_kernel"
    launch = f"K={head['views_per_pass']} ZU={head['z_unroll']} TX={head['tile_x']} split={args.tap_split}"
    traffic = measured_traffic(kernel, launch, wl.name) if head is results.get("fused_f32") else None
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_T, 3),
                "unit": "Tinstr/s", "frac": round(achieved / VALU_PEAK_T, 4),
                "traffic": round(traffic) if traffic else None,
                "kernel": kernel, "avg_launch_ms": round(per_launch_ms, 4),
                "updates_per_launch": updates_per_launch, "valu_instr_per_update": VALU_PER_UPDATE}

    forms_out = {}
    for form, r in results.items():
        forms_out[form] = {"path": r["path"], "dtype": r["dtype"], "views_per_pass": r["views_per_pass"],
                           "z_unroll": r["z_unroll"], "tile_x": r["tile_x"], "direct_taps": r.get("direct_taps"),
                           "ms_per_step": round(float(r["step_ms"].mean()), 3),
                           "gups_p50": round(r["gups_p50"], 2), "gups_p99": round(r["gups_p99"], 2),
                           "gups_mean": round(r["gups_mean"], 2),
                           "hbm_frac_algorithmic": round(
                               r["gups_mean"] * 1e9 * (8.0 / r["views_per_pass"] +
                                                       sc.W * sc.H * (4 if r["dtype"] == "f32" else 2) / v.L ** 3)
                               / (HBM_PEAK_GBS * 1e9), 4),
                           "error_vs_fp64_oracle": errors.get(form)}

    line = {
        "metric": "GUPS (voxel updates/s) at L=512, 496 views: fused/BF16 vs plain FP32; p50/p99",
        "value": round(head["gups_mean"], 2),
        "unit": "GUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(float(head["step_ms"].mean()), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded random-ellipsoid phantom standing in for the RabbitCT dataset)",
        "config": {"workload": wl.name, "L": v.L, "voxel_mm": v.voxel_size, "views": sc.n_views,
                   "noise_frac": wl.noise_frac,
                   "detector": [sc.W, sc.H], "form": "fused_f32", "parallelism": "single GPU"},
        "p50_gups": round(head["gups_p50"], 2),
        "p99_gups": round(head["gups_p99"], 2),
        "forms": forms_out,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fdk_preprocessing": fdk,
        "device": _device_info(torch),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
