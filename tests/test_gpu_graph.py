"""Frames captured in a HIP graph (torch.cuda.CUDAGraph) and replayed.  Each
replay runs after eager work that overwrites the outputs, and must equal the
eager frame bit for bit: the one-ray-per-lane form, the persistent form (its
work counter is zeroed by a kernel inside the graph, not by a memset), the
Manko-Novikov tracer, and a ring frame with its redshift in one graph."""
import math

import numpy as np
import pytest

from tests.gpu_util import DEG

pytestmark = pytest.mark.gpu

REPLAYS = 3


@pytest.fixture(scope="module")
def g():
    import paper_2310_15183_amd as g
    return g


def _snapshot(arrays):
    return {k: v.cpu().numpy().copy() for k, v in arrays.items()}


def _scramble(arrays):
    for v in arrays.values():
        if v.dtype.is_floating_point:
            v.fill_(float("nan"))
        else:
            v.fill_(-7)


def _check_replays(run, arrays):
    """Eager run, capture, then REPLAYS replays with eager scrambling and
    synchronisation in between; every replay must reproduce the eager bytes."""
    import torch
    run()
    torch.cuda.synchronize()
    eager = _snapshot(arrays)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side, capture_error_mode="relaxed"):
        run()
    torch.cuda.synchronize()
    for i in range(REPLAYS):
        _scramble(arrays)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = _snapshot(arrays)
        for k, v in eager.items():
            assert got[k].tobytes() == v.tobytes(), (i, k)
    return eager


@pytest.mark.parametrize("launch", [None, (256, 0, 1, 0), (64, 2, 1, 0)])
def test_kerr_newman_frame_replays(g, launch):
    ctx = g.gr_trace_init(0, g.make_integrator(dt=0.01, max_steps=20000))
    try:
        if launch is not None:
            g.gr_trace_set_launch(ctx, g.gr_launch(*launch))
        out = g.alloc_outputs(48 * 40, fields=g.FIELDS)
        metric = g.gr_metric(0.5, 0.24, 0.3)
        cam = g.gr_camera(20.0, 80 * DEG, 0.0, 75 * DEG, 48, 40)
        eager = _check_replays(lambda: g.gr_trace_frame(ctx, metric, cam, out.struct),
                               out.tensors)
        assert (eager["flag"] == g.GR_FLAG_ESCAPE).sum() > 100
        assert (eager["flag"] == g.GR_FLAG_HORIZON).sum() > 10
    finally:
        g.gr_trace_destroy(ctx)


def test_manko_novikov_frame_replays(g):
    ctx = g.gr_trace_init(0, g.make_integrator(dt=0.01, max_steps=20000))
    try:
        out = g.alloc_outputs(24 * 20, fields=g.FIELDS)
        metric = g.gr_metric_mn(0.5, 0.24, 2.0)
        cam = g.gr_camera(8.0, math.pi / 2, 0.0, 75 * DEG, 24, 20)
        eager = _check_replays(lambda: g.gr_trace_frame_mn(ctx, metric, cam, out.struct),
                               out.tensors)
        assert (eager["flag"] == g.GR_FLAG_ESCAPE).sum() > 50
    finally:
        g.gr_trace_destroy(ctx)


def test_ring_frame_and_redshift_replay(g):
    import torch
    ctx = g.gr_trace_init(0, g.make_integrator(dt=0.01, max_steps=20000,
                                               disk=(2.0, 5.0, 0.02)))
    try:
        n = 48 * 32
        out = g.alloc_outputs(n, dtype=g.GR_F32, fields=("t", "r", "theta", "phi", "p_t",
                                                          "p_phi"))
        z = torch.empty(n, dtype=torch.float32, device="cuda")
        metric = g.gr_metric(0.5, 0.49, 0.0)
        cam = g.gr_camera(20.0, 80 * DEG, 0.0, 50 * DEG, 48, 32)

        def run():
            g.gr_trace_frame(ctx, metric, cam, out.struct)
            g.gr_redshift(ctx, metric, cam, out.struct, n, z)

        eager = _check_replays(run, dict(out.tensors, z=z))
        on = eager["flag"] == g.GR_FLAG_DISK
        assert on.sum() > 50 and np.isfinite(eager["z"][on]).mean() > 0.9
    finally:
        g.gr_trace_destroy(ctx)
