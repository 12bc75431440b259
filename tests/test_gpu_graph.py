"""A back projection captured in a HIP graph and replayed (GPU).

The library enqueues only kernels (and, when it stages the next pass on its side stream, event
records and waits that fork from and join the caller's stream), so a caller can capture a call
once its scratch has grown and replay it without launch costs.  Every replay, with the program's
own eager work and synchronisations between replays, must give the eager call's bits.
"""
import numpy as np
import pytest
import torch

import gpu_common as gc
from paper_1401_7494_amd import bp, synth

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

SC = synth.Scanner(n_views=29, W=120, H=64, pitch=2.0)
SHAPE, VS = (40, 70, 130), 2.0


def _origin():
    nz, ny, nx = SHAPE
    return (-(nx - 1) / 2 * VS, -(ny - 1) / 2 * VS, -(nz - 1) / 2 * VS)


@pytest.mark.parametrize("dtype,path,k,staging", [("f32", "plain", 1, "auto"), ("f32", "fused", 8, "serial"),
                                                  ("f32", "fused_direct", 8, "auto"),
                                                  ("bf16", "fused", 8, "overlap"), ("f16", "fused", 13, "auto")])
def test_graph_replays_equal_the_eager_call(dtype, path, k, staging):
    dev = torch.device("cuda:0")
    proj = synth.filtered_projections(SC, synth.random_ellipsoids(81)).to(gc.TORCH_DTYPE[dtype]).to(dev)
    P = torch.from_numpy(gc.product_matrices(SC)).to(dev)
    origin = _origin()
    stream = torch.cuda.current_stream(dev)
    with bp.Context(SC.W, SC.H, dtype) as ctx:
        ctx.set_tuning(path, k, 8, 16)
        ctx.set_options(staging=staging)
        eager = torch.zeros(SHAPE, dtype=torch.float32, device=dev)
        ctx.backproject(eager, proj, P, VS, origin, stream)  # also grows the context's scratch
        torch.cuda.synchronize()
        vol = torch.zeros(SHAPE, dtype=torch.float32, device=dev)
        g = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream(device=dev)
        cs.wait_stream(stream)
        with torch.cuda.stream(cs):
            g.capture_begin()
            ctx.backproject(vol, proj, P, VS, origin, cs)
            g.capture_end()
        torch.cuda.synchronize()
        other = torch.randn(1 << 20, device=dev)
        for rep in range(4):
            vol.zero_()
            other.mul_(1.0001).add_(0.5)  # eager work of the program between replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(vol, eager), (dtype, path, rep)
        # replays accumulate like calls do
        g.replay()
        torch.cuda.synchronize()
        twice = eager.clone()
        ctx.backproject(twice, proj, P, VS, origin, stream)
        torch.cuda.synchronize()
        assert torch.equal(vol, twice)
    assert float(eager.abs().max()) > 0
    ref = gc.run_oracle(proj.float().cpu(), P.cpu().numpy(), max(SHAPE), VS, origin,
                        block=((0, SHAPE[2]), (0, SHAPE[1]), (0, SHAPE[0])))
    tol = gc.COMPACT_REL_L2_TOL if dtype != "f32" else gc.REL_L2_TOL
    assert gc.rel_l2(eager.cpu().numpy(), ref) <= tol
