"""Parity of the HIP Manko-Novikov tracer (paper Sec. 2.2.3) with the CPU
oracle, through the C ABI.

Gate as for Kerr-Newman: flags and step counts bit-exact, end theta/phi
within 1e-9 rad; both sides follow the same IEEE operation sequence (exp
and sin/cos from their series definitions), so every field is expected to
be bit-identical, and that is asserted.
"""
import math

import numpy as np
import pytest

from tests.gpu_util import DEG, compare, fp32_round

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import paper_2310_15183_amd as g
    return g


@pytest.fixture()
def ctx(g):
    c = g.gr_trace_init(0, g.make_integrator(dt=0.01, max_steps=20000))
    yield c
    g.gr_trace_destroy(c)


def gpu_trace_mn(g, ctx, M, S, q, r0, th0, ph0, fov, W, H, dtype=None, fields=None):
    import torch
    dtype = g.GR_F64 if dtype is None else dtype
    kw = {} if fields is None else {"fields": fields}
    out = g.alloc_outputs(W * H, dtype=dtype, **kw)
    g.gr_trace_frame_mn(ctx, g.gr_metric_mn(M, S, q), g.gr_camera(r0, th0, ph0, fov, W, H),
                        out.struct)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.tensors.items()}


def oracle_trace_mn(M, S, q, r0, th0, ph0, fov, W, H, integ, pixels=None):
    import oracle
    res = oracle.trace_frame_mn(M, S, q, r0, th0, ph0, fov, W, H, dt=integ.dt,
                                eps=integ.fd_eps, horizon_norm=integ.horizon_norm,
                                escape_factor=integ.escape_factor, max_steps=integ.max_steps,
                                pixels=pixels, want_p0=True, form="twin")
    return {"t": res.t, "r": res.r, "theta": res.theta, "phi": res.phi,
            "p_t": res.p0[:, 0], "p_r": res.pr, "p_theta": res.ptheta, "p_phi": res.p0[:, 3],
            "flag": res.flag, "steps": res.steps}


M = 0.5


@pytest.mark.parametrize("case", [
    # (M, S, q, r0, theta0, phi0, fov, W, H)
    (M, 0.24, 2.0, 8.0, math.pi / 2, 0.0, 75 * DEG, 24, 24),          # the listing's spacetime
    (M, 0.98 * M * M, 2.0, 15.0, 80 * DEG, 0.0, 60 * DEG, 21, 13),     # chaotic-shadow case
    (M, 0.1 * M * M, -2.0, 12.0, 70 * DEG, 0.3, 70 * DEG, 17, 19),      # prolate (ring figure)
    (M, -0.5 * M * M, 0.5, 20.0, 40 * DEG, 0.0, 50 * DEG, 9, 7),        # counter-rotating, ragged
    (M, 0.6 * M * M, 0.0, 20.0, 80 * DEG, 0.0, 60 * DEG, 16, 8),        # q = 0 (Kerr)
    (M, 0.3 * M * M, 1.0, 10.0, 90 * DEG, 0.0, 75 * DEG, 1, 1),         # single pixel
])
def test_mn_frames_are_bit_exact(g, ctx, case):
    integ = g.make_integrator(dt=0.01, max_steps=20000)
    gpu = gpu_trace_mn(g, ctx, *case)
    ref = oracle_trace_mn(*case, integ)
    st = compare(gpu, ref)
    print(st, np.bincount(ref["flag"], minlength=4))
    assert st["bit_identical"] == st["n"]


def test_mn_step_limit_and_f32_outputs(g, ctx):
    case = (M, 0.24, 2.0, 8.0, math.pi / 2, 0.0, 75 * DEG, 16, 12)
    integ = g.make_integrator(dt=0.01, max_steps=137)
    g.gr_trace_set_integrator(ctx, integ)
    gpu = gpu_trace_mn(g, ctx, *case, dtype=g.GR_F32)
    ref = oracle_trace_mn(*case, integ)
    st = compare(gpu, ref, angle_tol=0.0, f32=True)
    assert st["bit_identical"] == st["n"]
    assert np.all(gpu["steps"] <= 137)
    g.gr_trace_set_integrator(ctx, g.make_integrator(dt=0.01, max_steps=20000))


def test_mn_ignores_launch_shape(g, ctx):
    case = (M, 0.24, 2.0, 8.0, math.pi / 2, 0.0, 75 * DEG, 20, 12)
    base = gpu_trace_mn(g, ctx, *case)
    g.gr_trace_set_launch(ctx, g.gr_launch(256, 0, 1, 2))
    other = gpu_trace_mn(g, ctx, *case)
    g.gr_trace_set_launch(ctx, None)
    for k in base:
        np.testing.assert_array_equal(other[k], base[k], err_msg=k)


def test_mn_invalid_arguments(g, ctx):
    out = g.alloc_outputs(16, fields=("r",))
    cam = g.gr_camera(8.0, math.pi / 2, 0.0, 75 * DEG, 4, 4)
    for m in [g.gr_metric_mn(M, 0.0, 1.0), g.gr_metric_mn(M, M * M, 1.0),
              g.gr_metric_mn(0.0, 0.1, 1.0), g.gr_metric_mn(M, 0.1, float("nan"))]:
        with pytest.raises(g.GrError) as e:
            g.gr_trace_frame_mn(ctx, m, cam, out.struct)
        assert e.value.code == g.GR_EINVAL
    inside = g.gr_camera(0.9, math.pi / 2, 0.0, 75 * DEG, 4, 4)     # r0 < M + k
    with pytest.raises(g.GrError):
        g.gr_trace_frame_mn(ctx, g.gr_metric_mn(M, 0.1, 1.0), inside, out.struct)
    mixed = g.gr_trace_init(0, g.make_integrator(precision=g.GR_MIXED))
    try:
        with pytest.raises(g.GrError) as e:
            g.gr_trace_frame_mn(mixed, g.gr_metric_mn(M, 0.24, 2.0), cam, out.struct)
        assert e.value.code == g.GR_EUNSUPPORTED
    finally:
        g.gr_trace_destroy(mixed)


def test_mn_megapixel_sampled(g, ctx):
    """The benchmark's Manko-Novikov frame at full size in its launch
    configuration: 1000x1000, M=0.5, S=0.24, q=2 (the listing's spacetime),
    r0=8 on the equator, fov 75 deg, dt=0.005, 50000 steps, parameters
    rounded to binary32, binary32 end coordinates.  The oracle re-traces a
    stratified sample (every 40th pixel in both axes) and pixels on the
    shadow edge."""
    f = fp32_round
    case = (f(0.5), f(0.24), f(2.0), f(8.0), f(math.pi / 2), 0.0, f(75 * DEG), 1000, 1000)
    integ = g.make_integrator(dt=0.005, max_steps=50000)
    g.gr_trace_set_integrator(ctx, integ)
    gpu = gpu_trace_mn(g, ctx, *case, dtype=g.GR_F32, fields=("t", "r", "theta", "phi"))
    flag = gpu["flag"].reshape(1000, 1000)
    edge = np.zeros_like(flag, bool)
    edge[1:-1, 1:-1] = (flag[1:-1, 1:-1] != flag[:-2, 1:-1]) | (flag[1:-1, 1:-1] != flag[2:, 1:-1])
    edge_pix = np.nonzero(edge.ravel())[0]
    rng = np.random.default_rng(11)
    edge_pix = rng.choice(edge_pix, size=min(128, edge_pix.size), replace=False)
    grid = (np.arange(20, 1000, 40)[:, None] * 1000 + np.arange(20, 1000, 40)[None, :]).ravel()
    pix = np.unique(np.concatenate([grid, edge_pix]))
    ref = oracle_trace_mn(*case, integ, pixels=pix)
    sub = {k: v[pix] for k, v in gpu.items()}
    st = compare(sub, ref, angle_tol=0.0, f32=True)
    print(st, np.bincount(ref["flag"], minlength=4))
    assert st["bit_identical"] == st["n"]
    g.gr_trace_set_integrator(ctx, g.make_integrator(dt=0.01, max_steps=20000))


def test_mn_euler_frame_is_bit_exact(g, ctx):
    case = (M, 0.24, 2.0, 8.0, math.pi / 2, 0.0, 75 * DEG, 20, 14)
    integ = g.make_integrator(dt=0.01, max_steps=20000, method=g.GR_EULER)
    g.gr_trace_set_integrator(ctx, integ)
    gpu = gpu_trace_mn(g, ctx, *case)
    import oracle
    res = oracle.trace_frame_mn(*case, dt=0.01, max_steps=20000, want_p0=True, form="twin", method=1)
    ref = {"t": res.t, "r": res.r, "theta": res.theta, "phi": res.phi, "p_t": res.p0[:, 0],
           "p_r": res.pr, "p_theta": res.ptheta, "p_phi": res.p0[:, 3], "flag": res.flag,
           "steps": res.steps}
    st = compare(gpu, ref)
    assert st["bit_identical"] == st["n"]
    g.gr_trace_set_integrator(ctx, g.make_integrator(dt=0.01, max_steps=20000))


def test_mn_parked_rays_continue_bit_exact(g, ctx):
    """With a step limit of 4096 or more the tracer parks the rays still running
    after a quarter of it and continues them in a second launch.  On the
    listing's spacetime at dt=0.01 and 20000 steps, many rays pass 5000 steps
    (some to the limit): every field stays bit-identical to the oracle's
    single loop."""
    case = (M, 0.24, 2.0, 8.0, math.pi / 2, 0.0, 75 * DEG, 40, 32)
    integ = g.make_integrator(dt=0.01, max_steps=20000)
    gpu = gpu_trace_mn(g, ctx, *case)
    assert (gpu["steps"] > 5000).sum() > 50          # rays of the second launch
    assert (gpu["flag"] == g.GR_FLAG_TIMEOUT).sum() > 10
    st = compare(gpu, oracle_trace_mn(*case, integ))
    assert st["bit_identical"] == st["n"]


def test_mn_more_parked_rays_than_room(g, ctx):
    """A frame of 2100 x 2048 = 4.3e6 pixels whose rays all outlast a quarter
    of the 4096-step limit (camera at r0 = 50, escape at 75, dt = 0.01): more
    rays want parking than the 2^22 the workspace holds, and those past it are
    finished by the first launch.  Sampled rays from the first and last tiles
    and across the frame are bit-identical to the oracle."""
    import torch
    W, H = 2100, 2048
    case = (M, 0.24, 2.0, 50.0, 70 * DEG, 0.0, 60 * DEG, W, H)
    integ = g.make_integrator(dt=0.01, max_steps=4096)
    g.gr_trace_set_integrator(ctx, integ)
    out = g.alloc_outputs(W * H, fields=g.FIELDS)
    g.gr_trace_frame_mn(ctx, g.gr_metric_mn(*case[:3]), g.gr_camera(*case[3:]), out.struct)
    torch.cuda.synchronize()
    steps = out["steps"].cpu().numpy()
    assert np.all(steps > 1024)                      # every ray passed the parking point
    rng = np.random.default_rng(5)
    tile_rows = [0, 1, H - 2, H - 1]
    pix = np.unique(np.concatenate([
        np.array([j * W + i for j in tile_rows for i in (0, 7, W // 2, W - 9, W - 1)]),
        rng.choice(W * H, size=300, replace=False)]))
    gpu = {k: v[torch.as_tensor(pix, device="cuda")].cpu().numpy()
           for k, v in out.tensors.items()}
    st = compare(gpu, oracle_trace_mn(*case, integ, pixels=pix))
    assert st["bit_identical"] == st["n"]
    g.gr_trace_set_integrator(ctx, g.make_integrator(dt=0.01, max_steps=20000))
