"""The solid ring (exit object, flag 4) and the redshift of its light
(paper Sec. 3.3.2-3.3.3) on the GPU against the oracle: frames bit-exact,
redshifts bit-identical (NaN where the oracle has NaN)."""
import math

import numpy as np
import pytest

from tests.gpu_util import DEG, compare

pytestmark = pytest.mark.gpu

M = 0.5
DISK = (2.0, 5.0, 0.02)


@pytest.fixture(scope="module")
def g():
    import paper_2310_15183_amd as g
    return g


def _ref(res):
    return {"t": res.t, "r": res.r, "theta": res.theta, "phi": res.phi, "p_t": res.p0[:, 0],
            "p_r": res.pr, "p_theta": res.ptheta, "p_phi": res.p0[:, 3], "flag": res.flag,
            "steps": res.steps}


def _gpu(g, ctx, metric, cam, n, dtype):
    import torch
    out = g.alloc_outputs(n, dtype=dtype, fields=g.FIELDS)
    if isinstance(metric, g.gr_metric_mn):
        g.gr_trace_frame_mn(ctx, metric, cam, out.struct)
    else:
        g.gr_trace_frame(ctx, metric, cam, out.struct)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("mn", [False, True])
def test_ring_frames_and_redshift_are_bit_exact(g, mn, method):
    import torch

    import oracle
    W, H, r0, th0, fov = 48, 32, 20.0, 80 * DEG, 50 * DEG
    if mn:
        params = (M, 0.1 * M * M, -2.0)          # the paper's Manko-Novikov ring figure
        metric = g.gr_metric_mn(*params)
        trace = oracle.trace_frame_mn
    else:
        params = (M, 0.49, 0.0)                  # Kerr a = 0.98 M, the Kerr ring figure
        metric = g.gr_metric(*params)
        trace = oracle.trace_frame
    ctx = g.gr_trace_init(0, g.make_integrator(dt=0.01, max_steps=20000, method=method,
                                               disk=DISK))
    try:
        cam = g.gr_camera(r0, th0, 0.0, fov, W, H)
        for launch in (None, g.gr_launch(256, 0, 1, 2)):      # the launch shape is ignored
            g.gr_trace_set_launch(ctx, launch)
            out = _gpu(g, ctx, metric, cam, W * H, g.GR_F64)
            gpu = {k: v.cpu().numpy() for k, v in out.tensors.items()}
            res = trace(*params, r0, th0, 0.0, fov, W, H, dt=0.01, max_steps=20000,
                        want_p0=True, form="twin", method=method, disk=DISK)
            st = compare(gpu, _ref(res))
            assert st["bit_identical"] == st["n"]
        assert (res.flag == 4).sum() > 50
        z = torch.empty(W * H, dtype=torch.float64, device="cuda")
        g.gr_redshift(ctx, metric, cam, out.struct, W * H, z)
        torch.cuda.synchronize()
        z = z.cpu().numpy()
        want = oracle.redshift(*params, r0, th0, gpu["r"], gpu["theta"], gpu["p_t"],
                               gpu["p_phi"], gpu["flag"], mn=mn)
        np.testing.assert_array_equal(z, want)
        on = gpu["flag"] == 4
        assert np.isfinite(z[on]).mean() > 0.9 and np.all(np.isnan(z[~on]))
        assert 0.3 < np.nanmin(z) and np.nanmax(z) < 3.0
    finally:
        g.gr_trace_destroy(ctx)


def test_redshift_from_binary32_outputs(g):
    import torch

    import oracle
    W, H, r0, th0, fov = 40, 24, 20.0, 75 * DEG, 50 * DEG
    ctx = g.gr_trace_init(0, g.make_integrator(dt=0.01, max_steps=20000, disk=DISK))
    try:
        metric, cam = g.gr_metric(M, 0.3, 0.2), g.gr_camera(r0, th0, 0.0, fov, W, H)
        out = _gpu(g, ctx, metric, cam, W * H, g.GR_F32)
        z = torch.empty(W * H, dtype=torch.float32, device="cuda")
        g.gr_redshift(ctx, metric, cam, out.struct, W * H, z)
        torch.cuda.synchronize()
        h = {k: v.cpu().numpy().astype(np.float64) for k, v in out.tensors.items()
             if k != "flag"}
        want = oracle.redshift(M, 0.3, 0.2, r0, th0, h["r"], h["theta"], h["p_t"], h["p_phi"],
                               out.tensors["flag"].cpu().numpy()).astype(np.float32)
        np.testing.assert_array_equal(z.cpu().numpy(), want)
    finally:
        g.gr_trace_destroy(ctx)


def test_ring_arguments(g):
    for disk in [(2.0, 5.0, math.pi / 2), (5.0, 2.0, 0.02), (-1.0, 5.0, 0.02), (2.0, 5.0, -0.1)]:
        with pytest.raises(g.GrError) as e:
            g.gr_trace_init(0, g.make_integrator(disk=disk))
        assert e.value.code == g.GR_EINVAL
    with pytest.raises(g.GrError) as e:
        g.gr_trace_init(0, g.make_integrator(disk=DISK, precision=g.GR_MIXED))
    assert e.value.code == g.GR_EUNSUPPORTED
    ctx = g.gr_trace_init(0, g.make_integrator(disk=DISK))
    try:
        out = g.alloc_outputs(16, fields=("r",))
        inst = g.gr_instance(g.gr_metric(M, 0.3, 0.0),
                             g.gr_camera(20.0, math.pi / 2, 0.0, 60 * DEG, 4, 4), out.struct,
                             None, -1)
        with pytest.raises(g.GrError) as e:
            g.gr_trace_batch(ctx, [inst])
        assert e.value.code == g.GR_EUNSUPPORTED
    finally:
        g.gr_trace_destroy(ctx)


def _sample(flag, side, stride, n_edge, seed):
    """Every stride-th pixel in both axes plus n_edge seeded pixels where the
    flag changes between vertical neighbours."""
    f = flag.reshape(side, side)
    edge = np.zeros_like(f, bool)
    edge[1:-1, 1:-1] = (f[1:-1, 1:-1] != f[:-2, 1:-1]) | (f[1:-1, 1:-1] != f[2:, 1:-1])
    edge_pix = np.nonzero(edge.ravel())[0]
    edge_pix = np.random.default_rng(seed).choice(edge_pix, size=min(n_edge, edge_pix.size),
                                                  replace=False)
    grid = (np.arange(stride // 2, side, stride)[:, None] * side +
            np.arange(stride // 2, side, stride)[None, :]).ravel()
    return np.unique(np.concatenate([grid, edge_pix]))


def test_ring_megapixel_sampled(g):
    """The ringed frame in the benchmark's configuration (Kerr M=0.5, a=0.49,
    Q=0, r0=20, theta0=80 deg, fov 50 deg, 1000x1000, dt=0.005, 50000 steps,
    ring r in [2, 5], |theta - pi/2| <= 0.02, binary32 outputs): the oracle
    re-traces every 32nd pixel in both axes plus 256 pixels on flag edges
    (ring rims, shadow edge); then the redshift of the whole frame against the
    oracle's on the same sampled rays."""
    import torch

    import oracle
    side, r0, th0, fov = 1000, 20.0, 80 * DEG, 50 * DEG
    params = (M, 0.49, 0.0)
    ctx = g.gr_trace_init(0, g.make_integrator(dt=0.005, max_steps=50000, disk=DISK))
    try:
        metric, cam = g.gr_metric(*params), g.gr_camera(r0, th0, 0.0, fov, side, side)
        out = g.alloc_outputs(side * side, dtype=g.GR_F32,
                              fields=("t", "r", "theta", "phi", "p_t", "p_phi"))
        g.gr_trace_frame(ctx, metric, cam, out.struct)
        z = torch.empty(side * side, dtype=torch.float32, device="cuda")
        g.gr_redshift(ctx, metric, cam, out.struct, side * side, z)
        torch.cuda.synchronize()
        gpu = {k: v.cpu().numpy() for k, v in out.tensors.items()}
        z = z.cpu().numpy()
    finally:
        g.gr_trace_destroy(ctx)
    assert 0.05 < (gpu["flag"] == 4).mean() < 0.2
    pix = _sample(gpu["flag"], side, 32, 256, seed=11)
    res = oracle.trace_frame(*params, r0, th0, 0.0, fov, side, side, dt=0.005, max_steps=50000,
                             pixels=pix, want_p0=True, form="twin", disk=DISK)
    st = compare({k: v[pix] for k, v in gpu.items()}, _ref(res), angle_tol=0.0, f32=True)
    assert st["bit_identical"] == st["n"]
    assert (res.flag == 4).sum() > 100
    h = {k: gpu[k][pix].astype(np.float64) for k in ("r", "theta", "p_t", "p_phi")}
    want = oracle.redshift(*params, r0, th0, h["r"], h["theta"], h["p_t"], h["p_phi"],
                           gpu["flag"][pix]).astype(np.float32)
    np.testing.assert_array_equal(z[pix], want)
