"""Parity of the HIP back projector with the FP64 oracle, through the C ABI (GPU).

Inputs are seeded and synthetic; both sides read identical projections and
identical FP32 matrices (the product's host composition and the oracle's are
checked bit-identical first).  The bar is relative L2 <= 1e-5 over the
compared voxels for every storage type (FP16/BF16 data is compared with the
oracle run on the same rounded values, so the bar measures the kernel's FP32
arithmetic), and bit-exactness where the arithmetic is exact.
"""
import numpy as np
import pytest
import torch

import gpu_common as gc
import oracle
from paper_1401_7494_amd import bp, synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

# A small scan with the paper's proportions: SID 800, SDD 1200, 200 degree arc,
# on a 96 x 72 detector whose coarse pitch covers a ~200 mm field of view.
SMALL = synth.Scanner(n_views=13, W=96, H=72, pitch=3.0)
# A ragged box: no edge is a multiple of the 64 x 4 x ZU thread tile.
BOX = (21, 37, 70)  # (nz, ny, nx)
VS = 3.0


def _box_origin(shape, vs):
    nz, ny, nx = shape
    return (-(nx - 1) / 2 * vs, -(ny - 1) / 2 * vs, -(nz - 1) / 2 * vs)


def _oracle_box(proj, P32, shape, vs, origin):
    nz, ny, nx = shape
    L = max(shape)
    return gc.run_oracle(proj, P32, L, vs, origin, block=((0, nx), (0, ny), (0, nz)))


@pytest.fixture(scope="module")
def small_inputs():
    ph = synth.random_ellipsoids(1401)
    proj32 = synth.filtered_projections(SMALL, ph)
    P32 = gc.product_matrices(SMALL)
    assert np.array_equal(P32, gc.oracle_matrices(SMALL))
    return proj32, P32


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("path,k,tx", [("plain", 1, 64), ("plain", 1, 16), ("fused", 4, 16), ("fused", 13, 8),
                                       ("fused", 32, 64), ("fused_direct", 5, 16), ("fused_direct", 13, 64)])
@pytest.mark.parametrize("zu", [1, 2, 4, 8])
def test_parity_small_ragged(small_inputs, dtype, path, k, tx, zu):
    proj32, P32 = small_inputs
    proj = proj32.to(gc.TORCH_DTYPE[dtype])
    origin = _box_origin(BOX, VS)
    got = gc.run_gpu(proj, P32, BOX, VS, origin, dtype=dtype, path=path, k=k, zu=zu, tx=tx)
    ref = _oracle_box(proj, P32, BOX, VS, origin)
    err = gc.error_stats(got, ref)
    print(f"\n{dtype} {path} K={k} ZU={zu} TX={tx}: {err}")
    assert np.abs(ref).max() > 0
    assert err["rel_l2"] <= gc.REL_L2_TOL, err


@pytest.mark.parametrize("path,zu,tx", [("plain", 1, 64), ("plain", 8, 16), ("fused", 1, 16), ("fused", 4, 8),
                                         ("fused", 8, 64)])
def test_orthographic_identity_is_bit_exact(path, zu, tx):
    """w = 1 and integer positions: every voxel (x, y, z) is exactly sum_k I_k[y][x]."""
    from oracle import closed

    n, H, W, L, vs = 9, 70, 80, 66, 2.0
    origin = (-65.0, -65.0, -65.0)
    proj = synth.integer_images((n, H, W), seed=3)
    P = closed.orthographic_matrices(n, vs, origin).astype(np.float32)
    got = gc.run_gpu(proj, P, (L, L, L), vs, origin, path=path, k=4, zu=zu, tx=tx)
    want = closed.orthographic_volume(proj.numpy(), L)
    assert np.array_equal(got.astype(np.float64), want)


@pytest.mark.parametrize("path", ["plain", "fused"])
def test_views_behind_the_source_contribute_zero(small_inputs, path):
    """A source inside the volume: views put some voxels at w <= 0 (the guarded branch).

    Near a source plane 1/w^2 amplifies the FP32 rounding of w without limit, so two gates
    derived from FP32 arithmetic replace a fixed distance: every voxel must lie within its own
    rounding-error bound (``fp32_bounds.error_bound``; infinite only where w's sign itself is
    uncertain), and the relative-L2 bar applies beyond the distance from the source planes at
    which an FP32 emulation of the pass meets half the bar (``fp32_bounds.band_for_bar``)."""
    import fp32_bounds
    from oracle import closed

    proj32, _ = small_inputs
    sc = synth.Scanner(n_views=13, W=96, H=72, pitch=3.0, sid=60.0, sdd=160.0)
    P32 = gc.product_matrices(sc)
    origin = _box_origin(BOX, VS)
    pts = closed.voxel_centres(max(BOX), VS, origin, block=((0, BOX[2]), (0, BOX[1]), (0, BOX[0])))
    proj_np = proj32.numpy()
    for sign in (1.0, -1.0):  # negated matrices swap the voxels in front of and behind the source
        P = sign * P32
        got = gc.run_gpu(proj32, P, BOX, VS, origin, path=path, k=5, zu=4)
        ref = _oracle_box(proj32, P, BOX, VS, origin)
        _, _, w = closed._stw(P.astype(np.float64), pts)
        assert (w < 0).any() and (w > 0).any()
        E, _ = fp32_bounds.error_bound(proj_np, P, pts)
        fin = np.isfinite(E)
        err = np.abs(got.astype(np.float64) - ref)
        worst = float(np.max(err[fin] / np.maximum(E[fin], 1e-300)))
        d = fp32_bounds.band_for_bar(proj_np, P, BOX, VS, origin, sc.sid, ref, gc.REL_L2_TOL)
        keep = fp32_bounds.min_source_distance(P, pts, sc.sid) > d
        e = gc.error_stats(got[keep], ref[keep])
        print(f"\nsource inside the volume, {path}, sign {sign}: bound finite on {fin.mean():.3f}, "
              f"max error / bound {worst:.3e}; band {d} mm keeps {keep.mean():.3f}: {e}")
        assert fin.mean() > 0.9 and (err[fin] <= E[fin]).all(), worst
        assert d is not None and keep.mean() > 0.25
        assert gc.rel_l2(got[keep], ref[keep]) <= gc.REL_L2_TOL, e
        if sign < 0:
            assert np.array_equal(got[keep] == 0, ref[keep] == 0)


@pytest.mark.parametrize("path", ["plain", "fused"])
def test_source_outside_negated_matrices_give_zero(small_inputs, path):
    """With the source outside the volume, -P puts every voxel behind it: nothing is added."""
    proj32, P32 = small_inputs
    origin = _box_origin(BOX, VS)
    got = gc.run_gpu(proj32, -P32, BOX, VS, origin, path=path, k=5, zu=4)
    assert not got.any()


@pytest.mark.parametrize("path", ["plain", "fused"])
def test_accumulates_into_the_volume_and_chunks_add_up(small_inputs, path):
    proj32, P32 = small_inputs
    origin = _box_origin(BOX, VS)
    init = synth.uniform_images(BOX, seed=4).numpy()
    whole = gc.run_gpu(proj32, P32, BOX, VS, origin, path=path, k=4, zu=4, init=init)
    ref = _oracle_box(proj32, P32, BOX, VS, origin)
    assert gc.rel_l2(whole - init, ref) <= gc.REL_L2_TOL
    first = gc.run_gpu(proj32[:6], P32[:6], BOX, VS, origin, path=path, k=4, zu=4, init=init)
    both = gc.run_gpu(proj32[6:], P32[6:], BOX, VS, origin, path=path, k=4, zu=4, init=first)
    assert gc.rel_l2(both, whole) <= 1e-6


def test_fused_is_deterministic_and_plain_agrees(small_inputs):
    proj32, P32 = small_inputs
    origin = _box_origin(BOX, VS)
    a = gc.run_gpu(proj32, P32, BOX, VS, origin, path="fused", k=7, zu=8)
    b = gc.run_gpu(proj32, P32, BOX, VS, origin, path="fused", k=7, zu=8)
    c = gc.run_gpu(proj32, P32, BOX, VS, origin, path="plain", zu=8)
    assert np.array_equal(a, b)
    assert gc.rel_l2(a, c) <= 1e-6


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 65), (3, 5, 1), (9, 1, 130)])
def test_degenerate_boxes(small_inputs, shape):
    proj32, P32 = small_inputs
    origin = _box_origin(shape, VS)
    for path in ("plain", "fused"):
        got = gc.run_gpu(proj32[:3], P32[:3], shape, VS, origin, path=path, k=2, zu=8)
        ref = _oracle_box(proj32[:3], P32[:3], shape, VS, origin)
        assert gc.rel_l2(got, ref) <= gc.REL_L2_TOL


def test_single_view_single_pixel_detector():
    proj = torch.tensor([[[2.5]]], dtype=torch.float32)
    P = np.array([[[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1]]], dtype=np.float32)  # w = 1, s = X, t = Y
    shape = (2, 3, 3)
    origin = (-1.0, -1.0, 0.0)
    for path in ("plain", "fused"):
        got = gc.run_gpu(proj, P, shape, 0.5, origin, path=path, zu=2)
        ref = _oracle_box(proj, P, shape, 0.5, origin)
        assert np.array_equal(got.astype(np.float64), ref)


@pytest.mark.parametrize("path", ["plain", "fused", "fused_direct"])
def test_cubic_entry_equals_box_entry(small_inputs, path):
    """bp_backproject (L x L x L, the interface of the paper's framework) and bp_backproject_box
    give the same bits, and both match the oracle."""
    proj32, P32 = small_inputs
    L = 41
    shape = (L, L, L)
    origin = _box_origin(shape, VS)
    a = gc.run_gpu(proj32, P32, shape, VS, origin, path=path, k=5, zu=8, cubic=True)
    b = gc.run_gpu(proj32, P32, shape, VS, origin, path=path, k=5, zu=8, cubic=False)
    assert np.array_equal(a, b)
    ref = gc.run_oracle(proj32, P32, L, VS, origin)
    assert gc.rel_l2(a, ref) <= gc.REL_L2_TOL


def test_invalid_arguments_enqueue_nothing():
    dev = torch.device("cuda:0")
    vol = torch.zeros((4, 4, 4), device=dev)
    proj = torch.zeros((2, 8, 8), device=dev)
    mats = torch.zeros((2, 12), device=dev)
    L = bp.lib()
    o = (bp.ctypes.c_float * 3)(0, 0, 0)
    with bp.Context(8, 8) as ctx:
        h = ctx.handle
        args = dict(v=vol.data_ptr(), p=proj.data_ptr(), m=mats.data_ptr())
        assert L.bp_backproject(h, None, args["p"], args["m"], 2, 4, 1.0, o, None) == bp.BP_ERR_INVALID_ARG
        assert "null" in ctx.last_error()
        assert L.bp_backproject(h, args["v"], args["p"], args["m"], 0, 4, 1.0, o, None) == bp.BP_ERR_INVALID_ARG
        assert L.bp_backproject(h, args["v"], args["p"], args["m"], 2, 0, 1.0, o, None) == bp.BP_ERR_INVALID_ARG
        assert L.bp_backproject(h, args["v"], args["p"], args["m"], 2, 4, 0.0, o, None) == bp.BP_ERR_INVALID_ARG
        assert L.bp_backproject(h, args["v"], args["p"], args["m"], 2, 4, float("nan"), o, None) == bp.BP_ERR_INVALID_ARG
        bad = (bp.ctypes.c_float * 3)(0, float("inf"), 0)
        assert L.bp_backproject(h, args["v"], args["p"], args["m"], 2, 4, 1.0, bad, None) == bp.BP_ERR_INVALID_ARG
        assert L.bp_backproject(h, args["v"] + 2, args["p"], args["m"], 2, 4, 1.0, o, None) == bp.BP_ERR_INVALID_ARG
        assert L.bp_backproject(h, args["v"], args["p"], args["m"], 2, 2000, 1.0, o, None) == bp.BP_ERR_INVALID_ARG
        assert L.bp_set_tuning(h, 9, 0, 0, 0) == bp.BP_ERR_INVALID_ARG
        assert L.bp_set_tuning(h, 0, 0, 3, 0) == bp.BP_ERR_INVALID_ARG
        assert L.bp_set_tuning(h, 0, 0, 0, 12) == bp.BP_ERR_INVALID_ARG
        assert L.bp_set_options(h, 1 << 16) == bp.BP_ERR_INVALID_ARG
        assert L.bp_set_options(h, 3 << 5) == bp.BP_ERR_INVALID_ARG  # region split of 3 along x
        assert L.bp_set_options(h, (1 << 10) | (1 << 11)) == bp.BP_ERR_INVALID_ARG  # serial and overlapped
        torch.cuda.synchronize()
    assert not vol.any()


def test_allocation_failure_is_reported(monkeypatch, small_inputs):
    proj32, P32 = small_inputs
    monkeypatch.setenv("BP_FAULT_INJECT", "alloc")
    with pytest.raises(bp.BPError) as ei:
        gc.run_gpu(proj32, P32, BOX, VS, _box_origin(BOX, VS), path="fused", k=4)
    assert ei.value.status == bp.BP_ERR_OUT_OF_MEMORY


def test_plan_reports_choices():
    with bp.Context(1248, 960, "f32") as ctx:
        p = ctx.plan(512, 512, 512, 496)
        assert p.path == "fused" and p.z_unroll in (1, 2, 4, 8)
        ctx.set_tuning("plain", 0, 4, 16)
        p = ctx.plan(512, 512, 512, 496)
        assert (p.path, p.views_per_pass, p.z_unroll, p.tile_x) == ("plain", 1, 4, 16)
        ctx.set_tuning("plain", 0, 4, 8)
        assert ctx.plan(512, 512, 512, 496).tile_x == 64
        ctx.set_tuning("fused", 500, 2, 8)
        p = ctx.plan(64, 64, 64, 496)
        assert (p.views_per_pass, p.tile_x) == (496, 8)
        ctx.set_tuning("auto", 0, 0, 0)  # coarse boxes read the caller's images, fine ones the staging copy
        assert ctx.plan(128, 128, 128, 496).path == "fused_direct"
        assert ctx.plan(384, 384, 384, 496).path == "fused_direct"
        assert ctx.plan(448, 448, 448, 496).path == "fused"
        ctx.set_tuning("fused_direct", 0, 0, 32)
        p = ctx.plan(128, 128, 128, 496)
        assert (p.path, p.views_per_pass, p.tile_x) == ("fused_direct", 64, 64)
        # staged or direct taps: FP32 pixel stages at every size (K = 64 below 2e8 voxels, every
        # view in one pass above, up to 512); FP32 record stages at L = 512, direct reads on finer,
        # larger grids
        ctx.set_tuning("auto", 0, 0, 0)
        p = ctx.plan(512, 512, 512, 496)
        assert (p.path, p.views_per_pass, p.direct_taps) == ("fused", 64, False)
        p = ctx.plan(1024, 1024, 1024, 496)
        assert (p.path, p.views_per_pass, p.direct_taps) == ("fused", 496, False)
        assert ctx.plan(1024, 1024, 1024, 2000).views_per_pass == 512
        ctx.set_options(stage_records=True)
        p = ctx.plan(640, 640, 640, 496)
        assert (p.path, p.views_per_pass, p.direct_taps) == ("fused", 64, True)
        ctx.set_tap_split(4)  # an explicit split keeps the stage
        assert not ctx.plan(1024, 1024, 1024, 496).direct_taps
        ctx.set_tap_split(-1)
        ctx.set_options(direct_taps=True)
        p = ctx.plan(512, 512, 512, 496)
        assert (p.views_per_pass, p.direct_taps) == (32, True)
    with bp.Context(1248, 960, "bf16") as ctx:
        p = ctx.plan(1024, 1024, 1024, 496)
        assert (p.path, p.views_per_pass, p.direct_taps) == ("fused", 496, False)
        assert ctx.plan(512, 512, 512, 496).views_per_pass == 496  # 16-bit stages: every view in one pass
        assert ctx.plan(320, 320, 320, 496).path == "fused_direct"  # 16-bit pairs: staged a little sooner
        assert ctx.plan(384, 384, 384, 496).path == "fused"


# ---------------------------------------------------------------------------
# The paper-shaped workloads: 496 views of 1248 x 960 FP32, C-arm-like orbit.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("path,cubic,dtype", [("auto", False, "f32"), ("plain", True, "f32"),
                                              ("auto", False, "bf16"), ("plain", False, "f16")])
def test_parity_l128_full_volume(path, cubic, dtype):
    """L=128 (voxel 2 mm), 496 views, every voxel against the oracle: the library's automatic
    choice (the fused pass on the caller's images, each row's pixel pair as one load) and the plain
    form of the 128^3 workload, the FP32 plain form through the cubic entry bp_backproject; 16-bit
    stacks against the oracle on the same rounded values."""
    wl = synth.WORKLOADS["fdk_l128_v496_f32"]
    v = wl.volume
    proj = gc.full_projections(wl.phantom_seed).to(gc.TORCH_DTYPE[dtype])
    P32 = gc.product_matrices(wl.scanner)
    assert np.array_equal(P32, gc.oracle_matrices(wl.scanner))
    got = gc.run_gpu(proj, P32, (v.L,) * 3, v.voxel_size, v.origin, dtype=dtype, path=path, cubic=cubic)
    ref = gc.run_oracle(proj, P32, v.L, v.voxel_size, v.origin)
    err = gc.error_stats(got, ref)
    print(f"\nL=128 full, {path} {dtype}: {err}")
    assert err["rel_l2"] <= gc.REL_L2_TOL, err
    assert err["max_abs_over_max"] <= gc.MAX_ABS_TOL, err


L512_BLOCKS = {
    "centre": ((224, 288), (224, 288), (224, 288)),
    "corner": ((0, 64), (0, 64), (0, 64)),
    "top_edge": ((224, 288), (224, 288), (448, 512)),
}
# A block conditioned like the volume (kappa = ||sum_k |c_k| || / ||sum_k c_k||, the magnitude of
# the summed contributions over the result, at most this multiple of the volume's) is held to the
# bar on its own relative L2 as well.
KAPPA_OWN = 2.0


def strided_sample(L, stride, offset):
    """Voxel (x, y, z) triples on a uniform grid spread over the whole volume."""
    idx = np.arange(offset, L, stride)
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def _kappa(ref, mag):
    n = float(np.linalg.norm(ref))
    return float(np.linalg.norm(mag)) / n if n > 0 else float("inf")


@pytest.mark.parametrize("dtype,compact,path", [("f32", False, "auto"), ("f32", False, "plain"),
                                                ("f16", False, "auto"), ("bf16", False, "auto"),
                                                ("f16", True, "auto"), ("bf16", True, "auto")])
def test_parity_l512_sampled(dtype, compact, path):
    """L=512 (voxel 0.5 mm), 496 views, whole volume on the GPU in the benchmark's configuration
    (the automatic path) and in the plain form.

    The bar (relative L2 <= 1e-5, max |error| / max |V| <= 1e-4) holds over the volume, estimated
    on a uniform sample of 64^3 voxels (every 8th per axis).  On three 64^3 blocks it holds
    against the magnitude of what each block sums, ||V_gpu - V|| <= bar ||A|| with
    A = sum_k |contribution_k| (the oracle's magnitude mode; FP32 accumulation error scales with
    A, not with V where signed contributions cancel), and a block conditioned like the volume
    (A / V at most twice the volume's) is held to its own relative L2 too.  16-bit inputs are
    compared with the oracle on the same rounded values, with FP32 staging (the default) at the 1e-5
    bar and with compact FP16 staging at its derived bar."""
    wl = synth.WORKLOADS["fdk_l512_v496_f32"]
    v = wl.volume
    tol = gc.COMPACT_REL_L2_TOL if compact else gc.REL_L2_TOL
    max_tol = gc.COMPACT_MAX_ABS_TOL if compact else gc.MAX_ABS_TOL
    proj = gc.full_projections(wl.phantom_seed).to(gc.TORCH_DTYPE[dtype])
    P32 = gc.product_matrices(wl.scanner)
    got = gc.run_gpu(proj, P32, (v.L,) * 3, v.voxel_size, v.origin, dtype=dtype, compact=compact, path=path)
    proj_np = proj.float().cpu().numpy()
    P64 = P32.astype(np.float64)
    xyz = strided_sample(v.L, 8, 3)
    ref_s = oracle.backproject_points(proj_np, P64, v.voxel_size, v.origin, xyz)
    mag_s = oracle.backproject_points(proj_np, P64, v.voxel_size, v.origin, xyz, absolute=True)
    got_s = got[xyz[:, 2], xyz[:, 1], xyz[:, 0]]
    err = gc.error_stats(got_s, ref_s)
    k_vol = _kappa(ref_s, mag_s)
    print(f"\nL=512 {dtype} compact={compact} {path} uniform sample (kappa {k_vol:.2f}): {err}")
    assert err["rel_l2"] <= tol, err
    assert err["max_abs_over_max"] <= max_tol, err
    for name, blk in L512_BLOCKS.items():
        (x0, x1), (y0, y1), (z0, z1) = blk
        ref = gc.run_oracle(proj_np, P32, v.L, v.voxel_size, v.origin, block=blk)
        mag = oracle.backproject(proj_np, P64, v.L, v.voxel_size, v.origin, block=blk, absolute=True)
        g = got[z0:z1, y0:y1, x0:x1].astype(np.float64)
        d = g - ref
        e = gc.error_stats(g, ref) if np.abs(ref).max() > 0 else {"max_abs": float(np.abs(d).max())}
        kap = _kappa(ref, mag)
        rel_mag = float(np.linalg.norm(d) / np.linalg.norm(mag)) if np.abs(mag).max() > 0 else float(np.abs(d).max())
        print(f"L=512 {dtype} compact={compact} {path} block {name}: kappa {kap:.2f}, own {e}, "
              f"||error|| / ||A|| {rel_mag:.3e}")
        if np.abs(mag).max() == 0:  # every contribution is exactly 0: so is the result
            assert not d.any(), name
            continue
        assert rel_mag <= tol, (name, rel_mag)
        assert float(np.abs(d).max()) <= max_tol * float(np.abs(mag).max()), name
        if kap <= KAPPA_OWN * k_vol:
            assert e["rel_l2"] <= tol, (name, e)
            assert e["max_abs_over_max"] <= max_tol, (name, e)


# Launches from the benchmark's search space at L = 512 (views per pass, z-unroll, tile width, tap
# split, direct taps): the usual winner, a records split with wide tiles, the tuned split with
# narrow tiles, every view in one pass, and every tap read from the caller's images.
L512_TUNED_LAUNCHES = [(64, 8, 16, 0, False), (32, 4, 32, 4, False), (128, 8, 8, -1, False),
                       (496, 8, 32, 0, False), (64, 8, 16, -1, True)]


def test_parity_l512_tuned_launches_sampled():
    """The L=512 workload in launches the benchmark's autotuner can pick: every 8th voxel per axis
    against the oracle at the 1e-5 bar, and the whole volume against the library's default launch
    (both within the bar of the exact result, so within twice the bar of each other)."""
    wl = synth.WORKLOADS["fdk_l512_v496_f32"]
    v = wl.volume
    proj = gc.full_projections(wl.phantom_seed)
    P32 = gc.product_matrices(wl.scanner)
    shape = (v.L,) * 3
    base = gc.run_gpu(proj, P32, shape, v.voxel_size, v.origin)
    xyz = strided_sample(v.L, 8, 3)
    ref_s = oracle.backproject_points(proj.cpu().numpy(), P32.astype(np.float64), v.voxel_size, v.origin, xyz)
    for k, zu, tx, split, direct in L512_TUNED_LAUNCHES:
        got = _run_opts(proj, P32, shape, v.voxel_size, v.origin, k=k, zu=zu, tx=tx, tap_split=split,
                        direct_taps=direct)
        err = gc.error_stats(got[xyz[:, 2], xyz[:, 1], xyz[:, 0]], ref_s)
        whole = gc.rel_l2(got, base.astype(np.float64))
        print(f"\nL=512 K={k} zu={zu} tx={tx} split={split} direct={direct}: sample {err}, "
              f"whole volume vs default {whole:.3e}")
        assert err["rel_l2"] <= gc.REL_L2_TOL, (k, zu, tx, split, direct, err)
        assert err["max_abs_over_max"] <= gc.MAX_ABS_TOL, (k, zu, tx, split, direct, err)
        assert whole <= 2 * gc.REL_L2_TOL, (k, zu, tx, split, direct, whole)


def tilted(P64, deg):
    """The orbit tilted by ``deg`` degrees about the x axis (P T, T the rotation of the world frame),
    composed in FP64 and rounded once to FP32: every view has P[0][2] and P[2][2] non-zero."""
    a = np.radians(deg)
    T = np.eye(4)
    T[1, 1], T[1, 2], T[2, 1], T[2, 2] = np.cos(a), -np.sin(a), np.sin(a), np.cos(a)
    return (np.asarray(P64, dtype=np.float64) @ T).astype(np.float32)


def test_parity_l512_tilted_orbit_sampled():
    """The L=512 workload through a tilted orbit (7 degrees about x): no view takes the column
    branch, every update runs Part 1 per voxel (the general branch), in the library's automatic
    configuration; every 8th voxel per axis against the oracle, and the centre block."""
    wl = synth.WORKLOADS["fdk_l512_v496_f32"]
    v = wl.volume
    proj = gc.full_projections(wl.phantom_seed)
    P64, _ = bp.circular_matrices(*wl.scanner.geometry_args())
    P32 = tilted(P64, 7.0)
    assert ((P32[:, 0, 2] != 0) & (P32[:, 2, 2] != 0)).mean() > 0.99
    got = gc.run_gpu(proj, P32, (v.L,) * 3, v.voxel_size, v.origin)
    proj_np = proj.cpu().numpy()
    xyz = strided_sample(v.L, 8, 3)
    ref_s = oracle.backproject_points(proj_np, P32.astype(np.float64), v.voxel_size, v.origin, xyz)
    err = gc.error_stats(got[xyz[:, 2], xyz[:, 1], xyz[:, 0]], ref_s)
    print(f"\nL=512 tilted uniform sample: {err}")
    assert err["rel_l2"] <= gc.REL_L2_TOL, err
    assert err["max_abs_over_max"] <= gc.MAX_ABS_TOL, err
    blk = L512_BLOCKS["centre"]
    (x0, x1), (y0, y1), (z0, z1) = blk
    ref = gc.run_oracle(proj_np, P32, v.L, v.voxel_size, v.origin, block=blk)
    e = gc.error_stats(got[z0:z1, y0:y1, x0:x1], ref)
    print(f"L=512 tilted centre block: {e}")
    assert e["rel_l2"] <= gc.REL_L2_TOL, e


def _run_opts(proj, P32, shape, vs, origin, no_cull=False, no_column=False, dtype="f32", k=0, zu=0, tx=0,
              order="region", region_ax=0, direct_taps=False, compact=False, tap_split=-1,
              staging="auto", stage_records=False, poison=False, path="fused", init=None):
    dev = torch.device("cuda:0")
    vol = torch.zeros(shape, dtype=torch.float32, device=dev) if init is None else \
        torch.as_tensor(init, dtype=torch.float32).to(dev).contiguous()
    p = proj.to(dev).contiguous()
    m = torch.as_tensor(np.ascontiguousarray(P32, dtype=np.float32)).to(dev)
    n, H, W = p.shape
    with bp.Context(W, H, dtype) as ctx:
        ctx.set_tuning(path, k, zu, tx)
        ctx.set_options(no_cull=no_cull, no_column=no_column, order=order, region_ax=region_ax,
                        direct_taps=direct_taps, compact_staging=compact, staging=staging,
                        stage_records=stage_records, poison_staging=poison)
        ctx.set_tap_split(tap_split)
        ctx.backproject(vol, p, m, vs, origin)
        torch.cuda.synchronize()
    return vol.cpu().numpy()


def _run_direct(proj, P32, shape, vs, origin, path, single_taps, zu=8, tx=16, k=5, dtype="f32"):
    dev = torch.device("cuda:0")
    vol = torch.zeros(shape, dtype=torch.float32, device=dev)
    p = proj.to(gc.TORCH_DTYPE[dtype]).to(dev).contiguous()
    m = torch.as_tensor(np.ascontiguousarray(P32, dtype=np.float32)).to(dev)
    n, H, W = p.shape
    with bp.Context(W, H, dtype) as ctx:
        ctx.set_tuning(path, k, zu, tx)
        ctx.set_options(single_taps=single_taps)
        ctx.backproject(vol, p, m, vs, origin)
        torch.cuda.synchronize()
    return vol.cpu().numpy()


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("path", ["plain", "fused_direct"])
def test_pair_taps_equal_single_taps(path, dtype):
    """On the caller's images, each row's pixel pair read as one load (8 bytes of FP32, or 4 bytes
    of FP16/BF16 at any 2-byte boundary) gives the same bits as one load per tap: boxes across
    every detector edge and corner (pairs clamped into the row at column 0 and W - 2), even and
    odd detector widths (16-bit rows that start off a 4-byte boundary), views behind the source,
    detectors of two columns and of one."""
    shape, vs = (24, 40, 40), 2.0
    o = _box_origin(shape, vs)
    for W in (96, 97):
        sc = synth.Scanner(n_views=16, W=W, H=64, pitch=2.0)
        proj = synth.filtered_projections(sc, synth.random_ellipsoids(79)).to(gc.TORCH_DTYPE[dtype])
        P32 = gc.product_matrices(sc)
        for shift in ((0.0, 0.0, 0.0), (60.0, 0.0, 43.0), (0.0, 60.0, -43.0), (-60.0, 0.0, -43.0), (0.0, -60.0, 43.0)):
            origin = (o[0] + shift[0], o[1] + shift[1], o[2] + shift[2])
            for zu, tx in ((8, 16), (4, 64)):
                a = _run_direct(proj, P32, shape, vs, origin, path, True, zu, tx, dtype=dtype)
                b = _run_direct(proj, P32, shape, vs, origin, path, False, zu, tx, dtype=dtype)
                assert np.array_equal(a, b), (W, shift, zu, tx)
                assert np.abs(a).max() > 0
        ref = _oracle_box(proj, P32, shape, vs, origin)  # the oracle on the values the GPU read
        assert gc.rel_l2(b, ref) <= gc.REL_L2_TOL, W
    # the source inside the box (guarded contributions)
    sc2 = synth.Scanner(n_views=13, W=96, H=72, pitch=3.0, sid=60.0, sdd=160.0)
    P2 = gc.product_matrices(sc2)
    proj2 = synth.filtered_projections(sc2, synth.random_ellipsoids(1401))
    o2 = _box_origin(BOX, VS)
    assert np.array_equal(_run_direct(proj2, P2, BOX, VS, o2, path, True, dtype=dtype),
                          _run_direct(proj2, P2, BOX, VS, o2, path, False, dtype=dtype))
    # detectors of two columns and of one (single taps, whatever the option)
    for W in (2, 1):
        img = synth.uniform_images((3, 5, W), seed=W).to(gc.TORCH_DTYPE[dtype])
        P = np.array([[[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1]]] * 3, dtype=np.float32)
        shp, org = (2, 6, 4), (-1.0, -1.0, 0.0)
        a = _run_direct(img, P, shp, 0.5, org, path, True, 8, 16, 3, dtype=dtype)
        b = _run_direct(img, P, shp, 0.5, org, path, False, 8, 16, 3, dtype=dtype)
        assert np.array_equal(a, b)
        assert gc.rel_l2(a, _oracle_box(img, P, shp, 0.5, org)) <= gc.REL_L2_TOL


@pytest.mark.parametrize("zu", [1, 8])
def test_clipping_mask_is_exact_and_column_path_matches(zu):
    """Skipping tiles that project off the detector changes no bit; the column branch
    (u, w constant along z) and the general branch both match the oracle."""
    sc = synth.Scanner(n_views=29, W=120, H=64, pitch=2.0)  # small detector: many tiles fall off it
    proj = synth.filtered_projections(sc, synth.random_ellipsoids(77))
    P32 = gc.product_matrices(sc)
    shape, vs = (40, 70, 130), 2.0
    origin = _box_origin(shape, vs)
    full = _run_opts(proj, P32, shape, vs, origin, no_cull=True, k=13, zu=zu)
    culled = _run_opts(proj, P32, shape, vs, origin, k=13, zu=zu)
    assert np.array_equal(culled, full)
    general = _run_opts(proj, P32, shape, vs, origin, no_column=True, k=13, zu=zu)
    ref = _oracle_box(proj, P32, shape, vs, origin)
    for name, got in (("column", culled), ("general", general)):
        err = gc.error_stats(got, ref)
        print(f"\n{name} ZU={zu}: {err}")
        assert err["rel_l2"] <= gc.REL_L2_TOL, (name, err)


@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("path,k,tx", [("plain", 1, 16), ("plain", 1, 64), ("fused_direct", 13, 16)])
def test_clipping_mask_on_the_caller_image_passes(path, k, tx, dtype):
    """Passes on the caller's images skip every (tile, view) pair that misses the detector, and a
    tile that all views of a pass miss is neither read nor written: on a volume that already holds
    values, the result equals the pass without the mask (which adds exact zeros there) bit for bit,
    and the oracle's sum on top of those values."""
    sc = synth.Scanner(n_views=29, W=120, H=64, pitch=2.0)  # small detector: many tiles fall off it
    proj = synth.filtered_projections(sc, synth.random_ellipsoids(83))
    if dtype != "f32":
        proj = proj.to(gc.TORCH_DTYPE[dtype])
    P32 = gc.product_matrices(sc)
    shape, vs = (40, 70, 130), 2.0
    origin = _box_origin(shape, vs)
    init = (0.01 * np.random.default_rng(83).standard_normal(shape)).astype(np.float32)
    full = _run_opts(proj, P32, shape, vs, origin, no_cull=True, k=k, zu=8, tx=tx, dtype=dtype, path=path,
                     init=init)
    culled = _run_opts(proj, P32, shape, vs, origin, k=k, zu=8, tx=tx, dtype=dtype, path=path, init=init)
    assert np.array_equal(culled, full)
    ref = _oracle_box(proj, P32, shape, vs, origin)
    assert gc.rel_l2(culled - init, ref) <= gc.REL_L2_TOL
    # the box reaches beyond the detector in some views, so the mask acts: voxel centres (every 4th
    # per axis) that project off the detector
    nz, ny, nx = shape
    g = [np.arange(0, n, 4) * vs + o for n, o in zip((nx, ny, nz), origin)]
    X, Y, Z = np.meshgrid(*g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel(), np.ones(X.size)])
    uvw = np.asarray(P32, np.float64).reshape(-1, 3, 4) @ pts
    s_, t_ = uvw[:, 0] / uvw[:, 2], uvw[:, 1] / uvw[:, 2]
    assert ((s_ <= -1) | (s_ >= sc.W) | (t_ <= -1) | (t_ >= sc.H)).any()


def test_column_branch_needs_exact_zeros():
    """A matrix with a tiny P[0][2] takes the general branch; results still match the oracle."""
    sc = synth.Scanner(n_views=7, W=96, H=72, pitch=3.0)
    proj = synth.filtered_projections(sc, synth.random_ellipsoids(5))
    P32 = gc.product_matrices(sc).copy()
    P32[:, 0, 2] = 1e-3  # a tilted detector column axis
    origin = _box_origin(BOX, VS)
    got = _run_opts(proj, P32, BOX, VS, origin, k=4, zu=8)
    ref = _oracle_box(proj, P32, BOX, VS, origin)
    assert gc.rel_l2(got, ref) <= gc.REL_L2_TOL


@pytest.mark.parametrize("tx", [8, 16, 32, 64])
@pytest.mark.parametrize("zu", [1, 4, 8])
def test_tile_shapes_and_block_order(small_inputs, tx, zu):
    """Every block tile shape covers the ragged box exactly once; every tile order changes
    no bit; culling stays exact for every shape."""
    proj32, P32 = small_inputs
    origin = _box_origin(BOX, VS)
    a = _run_opts(proj32, P32, BOX, VS, origin, k=5, zu=zu, tx=tx, order="plain")
    for order, ax in (("zslices", 0), ("region", 0), ("region", 1), ("region", 2), ("region", 4)):
        b = _run_opts(proj32, P32, BOX, VS, origin, k=5, zu=zu, tx=tx, order=order, region_ax=ax)
        assert np.array_equal(a, b), (order, ax)
    c = _run_opts(proj32, P32, BOX, VS, origin, k=5, zu=zu, tx=tx, no_cull=True)
    assert np.array_equal(a, c)
    d = _run_opts(proj32, P32, BOX, VS, origin, k=5, zu=zu, tx=tx, direct_taps=True)
    assert np.array_equal(a, d), "direct taps"
    for split in (0, 8):
        e = _run_opts(proj32, P32, BOX, VS, origin, k=5, zu=zu, tx=tx, tap_split=split)
        assert np.array_equal(a, e), ("tap split", split)
    # a box whose tile grid divides into XCD regions takes the region order itself
    shape8 = (9, 8 * (256 // tx), 8 * tx)
    o8 = _box_origin(shape8, VS)
    e = _run_opts(proj32, P32, shape8, VS, o8, k=5, zu=zu, tx=tx, order="plain")
    for ax in (1, 2, 4, 8):
        f = _run_opts(proj32, P32, shape8, VS, o8, k=5, zu=zu, tx=tx, order="region", region_ax=ax)
        assert np.array_equal(e, f), ax
    ref = _oracle_box(proj32, P32, BOX, VS, origin)
    assert gc.rel_l2(a, ref) <= gc.REL_L2_TOL


@pytest.mark.parametrize("dtype,compact", [("f32", False), ("f16", True), ("bf16", True), ("bf16", False), ("f16", False)])
def test_lds_staged_taps_are_bit_identical(dtype, compact):
    """Taps staged through LDS per (tile, view) footprint give the same bits as direct taps, for any
    share of views read directly and with FP32 footprints staged as pixels or as records: column and
    general branches, culled tiles, guarded views (direct inside the staged pass), footprints too
    large for LDS (records read directly, or with a pixel stage the caller's pixels, zero-extended at
    the detector's edges), and footprints at the detector's edges (zero pixels)."""
    sc = synth.Scanner(n_views=29, W=120, H=64, pitch=2.0)
    proj = synth.filtered_projections(sc, synth.random_ellipsoids(77))
    if dtype != "f32":
        proj = proj.to(gc.TORCH_DTYPE[dtype])
    P32 = gc.product_matrices(sc)
    cases = [((40, 70, 130), 2.0, {}), ((40, 70, 130), 2.0, {"no_column": True}),
             ((9, 33, 65), 9.0, {}),  # large voxels: footprints beyond the LDS stage
             ((33, 47, 53), 20.0, {})]  # the source inside the box: guarded views
    for shape, vs, kw in cases:
        origin = _box_origin(shape, vs)
        for tx, zu in ((16, 8), (64, 1), (8, 4)):
            a = _run_opts(proj, P32, shape, vs, origin, dtype=dtype, k=13, zu=zu, tx=tx, compact=compact,
                          direct_taps=True, **kw)
            for split in (-1, 0, 5):  # tuned share of direct views, all staged, 5 of 8 direct
                b = _run_opts(proj, P32, shape, vs, origin, dtype=dtype, k=13, zu=zu, tx=tx, compact=compact,
                              tap_split=split, **kw)
                assert np.array_equal(a, b), (shape, vs, kw, tx, zu, split)
            if dtype == "f32":  # FP32 footprints staged as records instead of pixels
                b = _run_opts(proj, P32, shape, vs, origin, dtype=dtype, k=13, zu=zu, tx=tx, tap_split=0,
                              stage_records=True, **kw)
                assert np.array_equal(a, b), (shape, vs, kw, tx, zu, "records")
            assert np.abs(a).max() > 0


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_pixel_stage_at_the_detector_corners(dtype):
    """Boxes straddling the detector's corners (footprints that reach the bordered frame's first
    and last rows and columns): pixels staged in LDS as FP32 (16-bit ones widened), with every
    pixel off the detector read as 0 -- columns at an offset past the view, the row above the
    detector at one that wraps past 2^32, rows below past the view's end -- give the same bits as
    the records read directly, and match the oracle."""
    sc = synth.Scanner(n_views=16, W=96, H=64, pitch=2.0)
    proj = synth.filtered_projections(sc, synth.random_ellipsoids(79)).to(gc.TORCH_DTYPE[dtype])
    P32 = gc.product_matrices(sc)
    shape, vs = (24, 40, 40), 2.0
    for cx, cy, cz in ((60.0, 0.0, 43.0), (0.0, 60.0, -43.0), (-60.0, 0.0, -43.0), (0.0, -60.0, 43.0)):
        o = _box_origin(shape, vs)
        origin = (o[0] + cx, o[1] + cy, o[2] + cz)
        for tx, zu in ((16, 8), (8, 4), (64, 1)):
            a = _run_opts(proj, P32, shape, vs, origin, dtype=dtype, k=16, zu=zu, tx=tx, direct_taps=True)
            for split in (0, -1):
                b = _run_opts(proj, P32, shape, vs, origin, dtype=dtype, k=16, zu=zu, tx=tx, tap_split=split)
                assert np.array_equal(a, b), ((cx, cy, cz), tx, zu, split)
            assert np.abs(a).max() > 0
        a = _run_opts(proj, P32, shape, vs, origin, dtype=dtype, k=16, zu=8, tx=16, direct_taps=True)
        b = _run_opts(proj, P32, shape, vs, origin, dtype=dtype, k=16, zu=8, tx=16, tap_split=0)
    ref = _oracle_box(proj, P32, shape, vs, origin)  # the oracle on the values the GPU read
    err = gc.error_stats(b, ref)
    assert err["rel_l2"] <= gc.REL_L2_TOL, err


@pytest.mark.parametrize("dtype,compact,records", [("f32", False, False), ("f32", False, True), ("bf16", True, False),
                                                   ("bf16", False, False)])
def test_poisoned_staging_changes_nothing(dtype, compact, records):
    """The staging copy of each pass and the LDS stage of each footprint filled with NaN before
    they are written: the result is finite and bit-identical, so no element the staging did not
    write is ever read -- records of views only some tiles read directly, unused LDS rows and
    columns, footprints at the detector's edges, guarded views, footprints too large for the
    stage; any share of direct views; serial and overlapped staging."""
    sc = synth.Scanner(n_views=29, W=120, H=64, pitch=2.0)
    proj = synth.filtered_projections(sc, synth.random_ellipsoids(77))
    if dtype != "f32":
        proj = proj.to(gc.TORCH_DTYPE[dtype])
    P32 = gc.product_matrices(sc)
    cases = [((40, 70, 130), 2.0, (0.0, 0.0, 0.0)),
             ((24, 40, 40), 2.0, (60.0, 0.0, 43.0)),  # across a detector corner
             ((9, 33, 65), 9.0, (0.0, 0.0, 0.0)),  # large voxels: footprints beyond the stage
             ((33, 47, 53), 20.0, (0.0, 0.0, 0.0))]  # the source inside the box: guarded views
    for shape, vs, shift in cases:
        o = _box_origin(shape, vs)
        origin = (o[0] + shift[0], o[1] + shift[1], o[2] + shift[2])
        for split, staging in ((-1, "serial"), (0, "overlap"), (5, "serial")):
            kw = dict(dtype=dtype, k=13, zu=8, tx=16, compact=compact, stage_records=records, tap_split=split,
                      staging=staging)
            a = _run_opts(proj, P32, shape, vs, origin, **kw)
            b = _run_opts(proj, P32, shape, vs, origin, poison=True, **kw)
            assert np.isfinite(b).all(), (shape, split, staging)
            assert np.array_equal(a, b), (shape, split, staging)
            assert np.abs(a).max() > 0


@pytest.mark.parametrize("dtype,compact", [("f32", False), ("bf16", True), ("bf16", False)])
def test_staging_overlap_is_bit_identical(dtype, compact):
    """Staging the next pass on the context's side stream while the current pass runs gives the same
    bits as staging each pass just before it: many passes (both halves of the staging buffer reused),
    a ragged last pass, LDS-staged and direct taps, and a caller on a non-default stream whose earlier
    work the side stream must wait for."""
    sc = synth.Scanner(n_views=29, W=120, H=64, pitch=2.0)
    proj = synth.filtered_projections(sc, synth.random_ellipsoids(78))
    if dtype != "f32":
        proj = proj.to(gc.TORCH_DTYPE[dtype])
    P32 = gc.product_matrices(sc)
    shape, vs = (40, 70, 130), 2.0
    origin = _box_origin(shape, vs)
    for k in (4, 13, 28):  # 8, 3 and 2 passes
        for direct in (False, True):
            a = _run_opts(proj, P32, shape, vs, origin, dtype=dtype, k=k, zu=8, tx=16, compact=compact,
                          direct_taps=direct, staging="serial")
            b = _run_opts(proj, P32, shape, vs, origin, dtype=dtype, k=k, zu=8, tx=16, compact=compact,
                          direct_taps=direct, staging="overlap")
            assert np.array_equal(a, b), (k, direct)
            assert np.abs(a).max() > 0
    # a side stream of the caller's: the projections are written there just before the call, and two
    # calls accumulate into one volume; against the same two calls staged serially on the default stream
    dev = torch.device("cuda:0")
    m = torch.as_tensor(np.ascontiguousarray(P32, dtype=np.float32)).to(dev)
    src = proj.to(dev).contiguous()
    vols = []
    for serial in (True, False):
        st = torch.cuda.current_stream(dev) if serial else torch.cuda.Stream(device=dev)
        with bp.Context(sc.W, sc.H, dtype) as ctx:
            ctx.set_tuning("fused", 4, 8, 16)
            ctx.set_options(compact_staging=compact, staging="serial" if serial else "overlap")
            vol = torch.zeros(shape, dtype=torch.float32, device=dev)
            torch.cuda.synchronize()
            with torch.cuda.stream(st):
                p = torch.empty_like(src)
                p.copy_(src)
                ctx.backproject(vol, p, m, vs, origin, st)
                ctx.backproject(vol, p, m, vs, origin, st)
            st.synchronize()
        vols.append(vol)
    assert torch.equal(vols[0], vols[1])
    assert float(vols[0].abs().max()) > 0


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
@pytest.mark.parametrize("tx,zu", [(16, 8), (64, 1)])
def test_compact_staging_within_fp16_bound(small_inputs, dtype, tx, zu):
    """Compact staging (FP16 patch coefficients, per-view power-of-two scale) against the
    oracle on the same rounded data, within the bar derived from FP16 rounding of the
    pixel differences; FP32 staging (the default) of the same data meets the FP32 bar."""
    proj32, P32 = small_inputs
    proj = proj32.to(gc.TORCH_DTYPE[dtype]) * 1000.0  # large values: the per-view scale must engage
    origin = _box_origin(BOX, VS)
    ref = _oracle_box(proj, P32, BOX, VS, origin)
    compact = gc.run_gpu(proj, P32, BOX, VS, origin, dtype=dtype, path="fused", k=6, zu=zu, tx=tx, compact=True)
    wide = gc.run_gpu(proj, P32, BOX, VS, origin, dtype=dtype, path="fused", k=6, zu=zu, tx=tx)
    e_c, e_w = gc.error_stats(compact, ref), gc.error_stats(wide, ref)
    print(f"\n{dtype} compact: {e_c}\n{dtype} wide: {e_w}")
    assert e_w["rel_l2"] <= gc.REL_L2_TOL
    assert e_c["rel_l2"] <= gc.COMPACT_REL_L2_TOL
    assert not np.array_equal(compact, wide)


@pytest.mark.parametrize("k", [4, 8])
def test_stream_checkpoint_resume_is_bit_exact(small_inputs, k):
    """Views streamed in chunks (the L=1024 mode): stop after a chunk, save the volume on the
    host, resume into a fresh buffer and context; with the split on a pass boundary the
    result equals the uninterrupted run bit for bit."""
    proj32, P32 = small_inputs
    origin = _box_origin(BOX, VS)
    whole = gc.run_gpu(proj32, P32, BOX, VS, origin, path="fused", k=k, zu=8)
    cut = 2 * k if 2 * k < proj32.shape[0] else k
    ckpt = gc.run_gpu(proj32[:cut], P32[:cut], BOX, VS, origin, path="fused", k=k, zu=8)
    ckpt = np.array(ckpt, copy=True)  # the checkpoint lives on the host
    resumed = gc.run_gpu(proj32[cut:], P32[cut:], BOX, VS, origin, path="fused", k=k, zu=8, init=ckpt)
    assert np.array_equal(resumed, whole)


@pytest.mark.parametrize("dtype,k", [("f32", 0), ("f32", 128), ("bf16", 0)])
def test_parity_l1024_sampled(dtype, k):
    """L=1024 (voxel 0.25 mm, 4 GiB volume), 496 views: every 16th voxel per axis (64^3 voxels
    spread over the volume) against the oracle, in the library's launch (every view in one pass)
    and in passes of 128 views; BF16 against the oracle on the same rounded values."""
    wl = synth.WORKLOADS["fdk_l1024_v496_f32"]
    v = wl.volume
    proj = gc.full_projections(wl.phantom_seed).to(gc.TORCH_DTYPE[dtype])
    P32 = gc.product_matrices(wl.scanner)
    got = gc.run_gpu(proj, P32, (v.L,) * 3, v.voxel_size, v.origin, dtype=dtype, k=k)
    xyz = strided_sample(v.L, 16, 7)
    ref = oracle.backproject_points(proj.float().cpu().numpy(), P32.astype(np.float64), v.voxel_size, v.origin, xyz)
    err = gc.error_stats(got[xyz[:, 2], xyz[:, 1], xyz[:, 0]], ref)
    print(f"\nL=1024 {dtype} K={k or 'library'} uniform sample: {err}")
    assert err["rel_l2"] <= gc.REL_L2_TOL, err
    assert err["max_abs_over_max"] <= gc.MAX_ABS_TOL, err


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_lds_staged_taps_bit_identical_at_l512(dtype):
    """At the benchmark size (512^3, 496 views of 1248 x 960, K = 64) the LDS-staged taps (with the
    tuned share of direct views) reproduce the direct pass bit for bit over the whole volume."""
    wl = synth.WORKLOADS["fdk_l512_v496_f32"]
    v = wl.volume
    proj = gc.full_projections(wl.phantom_seed, dtype)
    P = torch.from_numpy(gc.product_matrices(wl.scanner)).to("cuda:0")
    out = []
    for direct in (True, False):
        vol = torch.zeros((v.L,) * 3, dtype=torch.float32, device="cuda:0")
        with bp.Context(wl.scanner.W, wl.scanner.H, dtype) as ctx:
            ctx.set_tuning("fused", 64, 0, 0)  # the same views per pass: the same summation order
            ctx.set_options(direct_taps=direct)
            ctx.backproject(vol, proj, P, v.voxel_size, v.origin)
            torch.cuda.synchronize()
        out.append(vol)
    assert torch.equal(out[0], out[1])
    assert float(out[0].abs().max()) > 0
