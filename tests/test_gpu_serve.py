"""Serving on the GPU: each request's volume is the same alone and in a concurrent mix."""
import numpy as np
import pytest
import torch

from paper_1401_7494_amd import serve, synth

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def small_scanner(r):
    return synth.Scanner(n_views=r.n_views, W=160, H=120, pitch=2.5)


def small_volume(r):
    return synth.Volume(r.L, 192.0 / r.L)


def test_results_are_the_same_alone_and_in_the_mix():
    rng = np.random.default_rng(1405)
    # all arrive at once, so that four run together whatever the device's speed
    reqs = [synth.Request(i, 0.0, int(rng.choice([32, 48, 64])), int(rng.choice([12, 24, 36])),
                          str(rng.choice(["f32", "f16"])), 100000 + i) for i in range(8)]
    kw = dict(keep_results=True, scanner_fn=small_scanner, volume_fn=small_volume)
    mix = serve.Server(serve.GpuExecutor(**kw), budget_bytes=8 * serve.GIB, max_inflight=4).run(reqs)
    assert len(mix.completed) == 8 and mix.peak_inflight == 4
    alone = {}
    for r in reqs:
        rep = serve.Server(serve.GpuExecutor(**kw), budget_bytes=8 * serve.GIB, max_inflight=1).run([r])
        alone[r.rid] = rep.completed[0].result
    for c in mix.completed:
        assert np.array_equal(c.result, alone[c.rid]), f"request {c.rid} differs in the mix"
        assert np.abs(c.result).max() > 0


def test_fast_generator_matches_the_torch_generator():
    """The generator's GPU line-integral kernel equals the torch formulation (FP64 rounding only)."""
    sc = synth.Scanner(n_views=5, W=200, H=150, pitch=1.5)
    ph = synth.random_ellipsoids(100003)
    dev = torch.device("cuda:0")
    a = synth.line_integrals(sc, ph, range(5), device=dev)
    b = synth.line_integrals_fast(sc, ph, range(5), device=dev)
    torch.cuda.synchronize()
    assert float(a.abs().max()) > 10.0
    assert float((a - b).abs().max()) <= 1e-9 * float(a.abs().max())
    fa = synth.filtered_projections(sc, ph, device=dev)
    fb = synth.filtered_projections(sc, ph, device=dev, fast=True)
    assert float((fa - fb).abs().max()) <= 1e-6 * float(fa.abs().max())


def test_cancelled_request_on_the_device():
    """A request withdrawn while its work is on the GPU: its result is dropped, its context and
    memory come back, and the others finish with the results they have alone."""
    kw = dict(keep_results=True, scanner_fn=small_scanner, volume_fn=small_volume)
    reqs = [synth.Request(0, 0.0, 48, 24, "f32", 100000),
            synth.Request(1, 0.0, 64, 36, "f32", 100001, cancel_s=1e-4),
            synth.Request(2, 0.0, 32, 12, "f16", 100002)]
    ex = serve.GpuExecutor(**kw)
    rep = serve.Server(ex, budget_bytes=8 * serve.GIB, max_inflight=4).run(reqs)
    assert sorted(c.rid for c in rep.completed) == [0, 2]
    assert [rid for rid, _, _ in rep.cancelled] == [1]
    for c in rep.completed:
        alone = serve.Server(serve.GpuExecutor(**kw), budget_bytes=8 * serve.GIB, max_inflight=1).run(
            [r for r in reqs if r.rid == c.rid])
        assert np.array_equal(c.result, alone.completed[0].result)
    ex.close()
