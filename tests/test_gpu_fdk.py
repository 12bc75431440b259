"""FDK pre-processing on the GPU (bp_fdk_*) against the FP64 oracle (``oracle.fdk``).

The kernel computes in FP64 and rounds each output once to FP32 (then to
FP16 / BF16).  The oracle's FP64 values, rounded the same way, are the
expected outputs: the two FP64 results differ by rounding order only (~1e-15
relative), so an output may differ from the expected one only where a
rounding boundary falls between them, and then by one unit in the last place.
The bar: every output within 1 ulp of the expected value (or within 1e-12 of
the row's largest magnitude, for outputs that are nearly zero), and at least
99.9% of outputs bit-equal.
"""
import numpy as np
import pytest
import torch

from oracle import fdk as ofdk
from paper_1401_7494_amd import bp, synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _key(bits):
    """Monotonic integer key of IEEE sign-magnitude bit patterns (adjacent values differ by 1)."""
    b = bits.astype(np.int64)
    top = 1 << (8 * bits.dtype.itemsize - 1)
    return np.where(b >= 0, b, -(b & (top - 1)))


def _round(ref64, dtype):
    r32 = torch.from_numpy(np.ascontiguousarray(ref64, dtype=np.float64)).to(torch.float32)
    return r32 if dtype == "f32" else r32.to({"f16": torch.float16, "bf16": torch.bfloat16}[dtype])


def _check(got, ref64, dtype, min_equal=0.999):
    got = got.cpu()
    want = _round(ref64, dtype)
    ibits = {"f32": torch.int32, "f16": torch.int16, "bf16": torch.int16}[dtype]
    kg = _key(got.view(ibits).numpy())
    kw = _key(want.view(ibits).numpy())
    dk = np.abs(kg - kw)
    near_zero = np.abs(got.double().numpy() - ref64) <= 1e-12 * np.abs(ref64).max()
    bad = (dk > 1) & ~near_zero
    frac_equal = float(np.mean(dk == 0))
    print(f"\nFDK {dtype}: {frac_equal * 100:.4f}% bit-equal, max ulp {int(dk.max())}, {int(bad.sum())} beyond 1 ulp")
    assert not bad.any(), (int(bad.sum()), np.argwhere(bad)[:5])
    assert frac_equal >= min_equal, frac_equal


def _raw(scanner, seed, views=None):
    views = range(scanner.n_views) if views is None else views
    return synth.line_integrals(scanner, synth.random_ellipsoids(seed), views, DEV).to(torch.float32).contiguous()


SMALL = synth.Scanner(n_views=13, W=96, H=72, pitch=3.0)


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_fdk_small_matches_oracle(dtype):
    raw = _raw(SMALL, 1401)
    with bp.FdkFilter.for_scanner(SMALL) as f:
        got = f.filter(raw, dtype)
        torch.cuda.synchronize()
    ref = ofdk.fdk_filter(raw.cpu().double().numpy(), SMALL.pitch, SMALL.sid, SMALL.sdd)
    _check(got, ref, dtype)


@pytest.mark.parametrize("W,H,n", [(1, 5, 3), (2, 3, 1), (7, 7, 3), (255, 2, 1), (257, 3, 5), (1000, 9, 2),
                                   (2048, 4, 3)])
def test_fdk_widths_and_odd_row_counts(W, H, n):
    """Widths from one pixel to the maximum, row counts odd and even (the last workgroup
    then holds one row), random signed data."""
    g = torch.Generator().manual_seed(W * 131 + H)
    raw = torch.randn((n, H, W), generator=g, dtype=torch.float32).to(DEV)
    pitch, sid, sdd = 0.7, 500.0, 900.0
    with bp.FdkFilter(W, H, pitch, sid, sdd) as f:
        got = f.filter(raw, "f32")
        torch.cuda.synchronize()
    ref = ofdk.fdk_filter(raw.cpu().double().numpy(), pitch, sid, sdd)
    _check(got, ref, "f32", min_equal=0.99 if raw.numel() < 1000 else 0.999)


def test_fdk_in_place_equals_out_of_place():
    raw = _raw(SMALL, 7)
    with bp.FdkFilter.for_scanner(SMALL) as f:
        a = f.filter(raw, "f32")
        b = raw.clone()
        f.filter(b, "f32", out=b)
        torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_fdk_full_detector_sampled_rows():
    """496 views of 1248 x 960 (the benchmark's detector) in one call; sampled rows against the oracle."""
    sc = synth.Scanner()
    raw = torch.empty((sc.n_views, sc.H, sc.W), dtype=torch.float32, device=DEV)
    ph = synth.random_ellipsoids(1402)
    for a in range(0, sc.n_views, 62):
        vs = list(range(a, min(a + 62, sc.n_views)))
        raw[a:a + len(vs)] = synth.line_integrals_fast(sc, ph, vs, DEV).to(torch.float32)
    with bp.FdkFilter.for_scanner(sc) as f:
        got = f.filter(raw, "f32")
        torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    rows = [(int(k), int(j)) for k, j in zip(rng.integers(0, sc.n_views, 48), rng.integers(0, sc.H, 48))]
    rows += [(0, 0), (sc.n_views - 1, sc.H - 1), (247, sc.H // 2)]
    ref = ofdk.fdk_filter_rows(raw.cpu().numpy(), rows, sc.pitch, sc.sid, sc.sdd)
    got_rows = torch.stack([got[k, j] for k, j in rows])
    _check(got_rows, ref, "f32")


def test_fdk_then_backprojection_matches_oracle_chain():
    """Raw data -> GPU FDK -> GPU back projection, against the oracle's FDK then back projection."""
    from gpu_common import REL_L2_TOL, oracle_matrices, product_matrices, rel_l2, run_oracle

    raw = _raw(SMALL, 1401)
    with bp.FdkFilter.for_scanner(SMALL) as f:
        q = f.filter(raw, "f32")
    P32 = product_matrices(SMALL)
    shape, vs = (21, 37, 70), 3.0
    origin = (-(70 - 1) / 2 * vs, -(37 - 1) / 2 * vs, -(21 - 1) / 2 * vs)
    vol = torch.zeros(shape, dtype=torch.float32, device=DEV)
    with bp.Context(SMALL.W, SMALL.H, "f32") as ctx:
        ctx.backproject(vol, q, torch.from_numpy(P32).to(DEV), vs, origin)
        torch.cuda.synchronize()
    q_ref = ofdk.fdk_filter(raw.cpu().double().numpy(), SMALL.pitch, SMALL.sid, SMALL.sdd).astype(np.float32)
    nz, ny, nx = shape
    ref = run_oracle(q_ref, oracle_matrices(SMALL), max(shape), vs, origin, block=((0, nx), (0, ny), (0, nz)))
    err = rel_l2(vol.cpu().numpy(), ref)
    print(f"\nFDK + back projection vs oracle chain: rel-L2 {err:.3e}")
    assert err <= REL_L2_TOL


def test_fdk_invalid_arguments():
    L = bp.lib()
    import ctypes

    cfg = bp.BpFdkConfig()
    L.bp_fdk_config_default(ctypes.byref(cfg))
    h = ctypes.c_void_p()
    cfg.det_width = 2049
    assert L.bp_fdk_create(ctypes.byref(cfg), ctypes.byref(h)) == bp.BP_ERR_UNSUPPORTED and not h.value
    L.bp_fdk_config_default(ctypes.byref(cfg))
    cfg.sdd = float("nan")
    assert L.bp_fdk_create(ctypes.byref(cfg), ctypes.byref(h)) == bp.BP_ERR_INVALID_ARG
    with bp.FdkFilter(64, 4, 1.0, 100.0, 200.0) as f:
        raw = torch.zeros((3, 4, 64), dtype=torch.float32, device=DEV)
        out = torch.zeros((4, 4, 64), dtype=torch.float32, device=DEV)
        assert L.bp_fdk_filter(f._h, raw.data_ptr(), out.data_ptr(), 0, 0, None) == bp.BP_ERR_INVALID_ARG
        assert L.bp_fdk_filter(f._h, raw.data_ptr(), out.data_ptr(), 5, 3, None) == bp.BP_ERR_INVALID_ARG
        assert L.bp_fdk_filter(f._h, None, out.data_ptr(), 0, 3, None) == bp.BP_ERR_INVALID_ARG
        # partial overlap (shifted by one row) is refused; exact FP32 aliasing is allowed
        assert L.bp_fdk_filter(f._h, out.data_ptr(), out.data_ptr() + 256, 0, 3, None) == bp.BP_ERR_INVALID_ARG
        assert L.bp_fdk_filter(f._h, out.data_ptr(), out.data_ptr(), 1, 3, None) == bp.BP_ERR_INVALID_ARG
        assert "overlap" in f.last_error()
        torch.cuda.synchronize()
    assert L.bp_fdk_destroy(None) == bp.BP_OK
