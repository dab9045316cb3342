"""Shading kernels (the sky's three lines, the exit-time map, the sky texture)
against the oracle's shading on the same arrays: every colour identical."""
import math

import numpy as np
import pytest

from tests.gpu_util import DEG

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import paper_2310_15183_amd as g
    return g


def _shade_gpu(g, out, n, mode, t_max=1.0, band=0.0):
    import torch
    rgba = torch.empty(n, dtype=torch.int32, device="cuda")
    g.gr_shade_frame(g.gr_shade(mode, t_max, band), out.struct, n, rgba)
    torch.cuda.synchronize()
    return rgba.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("dtype_name", ["GR_F64", "GR_F32"])
def test_shading_of_a_traced_frame(g, dtype_name):
    import oracle
    W, H = 64, 48
    ctx = g.gr_trace_init(0, g.make_integrator(dt=0.01, max_steps=20000))
    try:
        out = g.alloc_outputs(W * H, dtype=getattr(g, dtype_name),
                              fields=("t", "r", "theta", "phi"))
        g.gr_trace_frame(ctx, g.gr_metric(0.5, 0.24, 0.3),
                         g.gr_camera(20.0, 80 * DEG, 0.0, 75 * DEG, W, H), out.struct)
        import torch
        torch.cuda.synchronize()
        host = {k: v.cpu().numpy() for k, v in out.tensors.items()}
        f64 = {k: host[k].astype(np.float64) for k in ("t", "theta", "phi")}
        bands = _shade_gpu(g, out, W * H, g.GR_SHADE_BANDS)
        want = oracle.shade(0, None, f64["theta"], f64["phi"], host["flag"])
        np.testing.assert_array_equal(bands, want)
        assert len(set(bands.tolist())) >= 4               # black, dark blue and lines
        times = _shade_gpu(g, out, W * H, g.GR_SHADE_TIME, t_max=80.0, band=5.0)
        want = oracle.shade(1, f64["t"], None, None, host["flag"], t_max=80.0, band=5.0)
        np.testing.assert_array_equal(times, want)
    finally:
        g.gr_trace_destroy(ctx)


def test_shading_edges_and_grid_stride(g):
    """Synthetic rays (seeded) over 2^24 + 1000 pixels, more than one pass of
    the capped grid, with values at the band edges, NaN and infinite times."""
    import torch

    import oracle
    n = (1 << 24) + 1000
    rng = np.random.default_rng(5)
    th = rng.uniform(0.0, math.pi, n)
    ph = rng.uniform(-4.0, 4.0, n)
    t = -rng.exponential(40.0, n)
    flag = rng.choice(np.array([0, 1, 1, 1, 2, 3], np.int8), n)
    edge = math.asin(0.1)
    ph[:8] = [edge, -edge, math.pi - edge, math.pi / 2 - edge, 0.0, math.pi, 1e-300, -0.0]
    th[8:12] = [math.pi / 2, 0.5 * math.asin(0.1), 0.0, math.pi]
    t[12:16] = [np.nan, -np.inf, 0.0, -100.0]
    flag[:16] = 1
    out = g.alloc_outputs(n, dtype=g.GR_F64, fields=("t", "theta", "phi"), steps=False)
    out.tensors["t"].copy_(torch.from_numpy(t))
    out.tensors["theta"].copy_(torch.from_numpy(th))
    out.tensors["phi"].copy_(torch.from_numpy(ph))
    out.tensors["flag"].copy_(torch.from_numpy(flag))
    bands = _shade_gpu(g, out, n, g.GR_SHADE_BANDS)
    np.testing.assert_array_equal(bands, oracle.shade(0, None, th, ph, flag))
    times = _shade_gpu(g, out, n, g.GR_SHADE_TIME, t_max=100.0, band=7.5)
    np.testing.assert_array_equal(times, oracle.shade(1, t, None, None, flag, t_max=100.0,
                                                      band=7.5))


def test_shading_invalid_arguments(g):
    out = g.alloc_outputs(16, fields=("r",))          # no theta/phi/t arrays
    import torch
    rgba = torch.empty(16, dtype=torch.int32, device="cuda")
    for sh in [g.gr_shade(g.GR_SHADE_BANDS, 1.0, 0.0), g.gr_shade(g.GR_SHADE_TIME, 1.0, 0.0),
               g.gr_shade(7, 1.0, 0.0)]:
        with pytest.raises(g.GrError) as e:
            g.gr_shade_frame(sh, out.struct, 16, rgba)
        assert e.value.code == g.GR_EINVAL
    out2 = g.alloc_outputs(16, fields=("t",))
    with pytest.raises(g.GrError):
        g.gr_shade_frame(g.gr_shade(g.GR_SHADE_TIME, 0.0, 0.0), out2.struct, 16, rgba)


@pytest.mark.parametrize("n,offset,mode", [((1 << 24) + 1001, 0, 0), ((1 << 24) + 1001, 0, 1),
                                           (4099, 1, 0), ((1 << 26) + 5, 0, 1)])
def test_binary32_paths(g, n, offset, mode):
    """Binary32 arrays: the four-pixel kernel (aligned; a ragged tail; more
    than one pass of the capped grid at 2^26 + 5) and the one-pixel kernel
    (arrays starting one element off a 16-byte boundary)."""
    import torch

    import oracle
    rng = np.random.default_rng(n + offset)
    m = n + offset
    th = torch.from_numpy(rng.uniform(0.0, math.pi, m).astype(np.float32)).cuda()
    ph = torch.from_numpy(rng.uniform(-4.0, 4.0, m).astype(np.float32)).cuda()
    t = torch.from_numpy((-rng.exponential(40.0, m)).astype(np.float32)).cuda()
    fl = torch.from_numpy(rng.choice(np.array([0, 1, 1, 1, 2, 3], np.int8), m)).cuda()
    ptr = lambda x: x[offset:].data_ptr()      # noqa: E731
    out = g.gr_output(ptr(t), None, ptr(th), ptr(ph), None, None, None, None, ptr(fl), None,
                      g.GR_F32)
    rgba = torch.empty(n, dtype=torch.int32, device="cuda")
    sh = g.gr_shade(mode, 100.0, 7.5)
    g.gr_shade_frame(sh, out, n, rgba)
    torch.cuda.synchronize()
    got = rgba.cpu().numpy().view(np.uint32)
    host = lambda x: x.cpu().numpy()[offset:].astype(np.float64)     # noqa: E731
    want = oracle.shade(mode, host(t), host(th), host(ph), fl.cpu().numpy()[offset:],
                        t_max=100.0, band=7.5)
    np.testing.assert_array_equal(got, want)


def _texture(g, w, h, seed):
    import torch

    from paper_2310_15183_amd.workloads import sky_texture
    tex = sky_texture(w, h, seed)
    return tex, torch.from_numpy(tex.view(np.int32)).cuda()


@pytest.mark.parametrize("dtype_name", ["GR_F64", "GR_F32"])
def test_texture_shading_of_a_traced_frame(g, dtype_name):
    """A traced Kerr-Newman frame shaded with a seeded 256 x 128 sky texture
    (bilinear filtering): every colour identical to the oracle's."""
    import torch

    import oracle
    W, H = 64, 48
    tex, tex_dev = _texture(g, 256, 128, 3)
    ctx = g.gr_trace_init(0, g.make_integrator(dt=0.01, max_steps=20000))
    try:
        out = g.alloc_outputs(W * H, dtype=getattr(g, dtype_name),
                              fields=("t", "r", "theta", "phi"))
        g.gr_trace_frame(ctx, g.gr_metric(0.5, 0.24, 0.3),
                         g.gr_camera(20.0, 80 * DEG, 0.0, 75 * DEG, W, H), out.struct)
        rgba = torch.empty(W * H, dtype=torch.int32, device="cuda")
        g.gr_shade_frame(g.shade_texture(tex_dev), out.struct, W * H, rgba)
        torch.cuda.synchronize()
        host = {k: v.cpu().numpy() for k, v in out.tensors.items()}
    finally:
        g.gr_trace_destroy(ctx)
    got = rgba.cpu().numpy().view(np.uint32)
    want = oracle.shade(2, None, host["theta"].astype(np.float64),
                        host["phi"].astype(np.float64), host["flag"], texture=tex)
    np.testing.assert_array_equal(got, want)
    assert len(set(got.tolist())) > 100


@pytest.mark.parametrize("n,offset,f32", [((1 << 22) + 1001, 0, True), (4099, 1, True),
                                          ((1 << 22) + 7, 0, False)])
def test_texture_shading_of_seeded_rays(g, n, offset, f32):
    """Seeded synthetic end directions, theta over [-2 pi, 3 pi] (reflections
    over the poles) and phi over [-30, 30] (wraps), on a 97 x 31 texture (odd
    sides); binary32 through the four-pixel kernel with a ragged tail and
    through the one-pixel kernel (arrays one element off a 16-byte
    boundary), and binary64."""
    import torch

    import oracle
    rng = np.random.default_rng(n + offset)
    m = n + offset
    dt = np.float32 if f32 else np.float64
    th = torch.from_numpy(rng.uniform(-2 * math.pi, 3 * math.pi, m).astype(dt)).cuda()
    ph = torch.from_numpy(rng.uniform(-30.0, 30.0, m).astype(dt)).cuda()
    fl = torch.from_numpy(rng.choice(np.array([0, 1, 1, 1, 2, 3], np.int8), m)).cuda()
    tex, tex_dev = _texture(g, 97, 31, 4)
    ptr = lambda x: x[offset:].data_ptr()      # noqa: E731
    out = g.gr_output(None, None, ptr(th), ptr(ph), None, None, None, None, ptr(fl), None,
                      g.GR_F32 if f32 else g.GR_F64)
    rgba = torch.empty(n, dtype=torch.int32, device="cuda")
    g.gr_shade_frame(g.shade_texture(tex_dev), out, n, rgba)
    torch.cuda.synchronize()
    got = rgba.cpu().numpy().view(np.uint32)
    host = lambda x: x.cpu().numpy()[offset:].astype(np.float64)     # noqa: E731
    want = oracle.shade(2, None, host(th), host(ph), fl.cpu().numpy()[offset:], texture=tex)
    np.testing.assert_array_equal(got, want)


def test_texture_shading_invalid_arguments(g):
    import torch
    out = g.alloc_outputs(16, fields=("theta", "phi"))
    rgba = torch.empty(16, dtype=torch.int32, device="cuda")
    tex = torch.zeros(4, 8, dtype=torch.int32, device="cuda")
    bad = [g.gr_shade(g.GR_SHADE_TEXTURE, 0.0, 0.0, None, 8, 4),
           g.gr_shade(g.GR_SHADE_TEXTURE, 0.0, 0.0, tex.data_ptr(), 0, 4),
           g.gr_shade(g.GR_SHADE_TEXTURE, 0.0, 0.0, tex.data_ptr(), 8, 0)]
    for sh in bad:
        with pytest.raises(g.GrError) as e:
            g.gr_shade_frame(sh, out.struct, 16, rgba)
        assert e.value.code == g.GR_EINVAL
    out2 = g.alloc_outputs(16, fields=("t",))
    with pytest.raises(g.GrError):
        g.gr_shade_frame(g.shade_texture(tex), out2.struct, 16, rgba)
