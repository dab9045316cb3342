"""Parity of the HIP FP64 tracer with the CPU oracle, through the C ABI.

Gate: flags and step counts bit-exact; end theta/phi within 1e-9 rad.  The
kernel and the oracle follow the same IEEE operation sequence, so the rays
are expected to be bit-identical in every field, and that is asserted too.
"""
import math

import numpy as np
import pytest

from tests.gpu_util import DEG, compare, fp32_round, gpu_trace, oracle_trace

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


KERR64 = (0.5, 0.24, 0.0, 20.0, math.pi / 2, 0.0, 75 * DEG, 64, 64)


def _both(g, ctx, case, integ=None, **kw):
    integ = integ or g.make_integrator(dt=0.01, max_steps=20000)
    g.gr_trace_set_integrator(ctx, integ)
    gpu = gpu_trace(ctx, *case, **kw)
    ref = oracle_trace(*case, integ, pixels=kw.get("pixels"))
    return gpu, ref


def test_small_kerr_frame_is_bit_exact(g, ctx):
    """64x64 Kerr frame (M=0.5, a=0.24, r0=20 on the equator, fov 75 deg,
    dt=0.01, 20000 steps)."""
    gpu, ref = _both(g, ctx, KERR64)
    st = compare(gpu, ref)
    print(st)
    assert st["bit_identical"] == st["n"]
    assert (ref["flag"] == g.GR_FLAG_HORIZON).sum() > 0


@pytest.mark.parametrize("method", ["GR_RK4", "GR_RK4_TIME", "GR_EULER"])
def test_camera_next_to_the_pole_is_bit_exact(g, ctx, method):
    """A camera 2e-6 rad from the polar axis: the theta-displaced points of
    the first steps lie within 5e5 eps of the axis, where the reciprocal
    there is divided instead of refined from the base point's, so every ray
    takes the frame's second pass; each integrator bit-identical to the
    twin form (flags, steps and all fields)."""
    case = (0.5, 0.3, 0.1, 20.0, 2e-6, 0.4, 60 * DEG, 16, 16)
    integ = g.make_integrator(dt=0.01, max_steps=20000, method=getattr(g, method))
    g.gr_trace_set_integrator(ctx, integ)
    gpu = gpu_trace(ctx, *case)
    ref = oracle_trace(*case, integ)
    st = compare(gpu, ref)
    print(st)
    assert st["bit_identical"] == st["n"]


def test_camera_initial_state_is_bit_exact(g, ctx):
    integ = g.make_integrator(max_steps=0)
    case = (0.5, 0.24, 0.3, 20.0, 80 * DEG, 0.25, 75 * DEG, 17, 9)
    gpu, ref = _both(g, ctx, case, integ=integ)
    st = compare(gpu, ref)
    assert st["bit_identical"] == st["n"]
    assert np.all(gpu["flag"] == g.GR_FLAG_TIMEOUT) and np.all(gpu["steps"] == 0)
    assert np.all(gpu["t"] == 0.0) and np.all(gpu["r"] == 20.0)


@pytest.mark.parametrize("case", [
    (0.5, 0.24, 0.3, 20.0, 80 * DEG, 0.0, 75 * DEG, 37, 23),     # Kerr-Newman, ragged
    (0.5, 0.49, 0.0, 20.0, 60 * DEG, 0.0, 75 * DEG, 30, 30),     # near-extremal
    (0.5, 0.1, 0.2, 35.0, 20 * DEG, 1.0, 40 * DEG, 19, 41),      # tall image, high latitude
    (0.5, 0.24, 0.0, 20.0, math.pi / 2, 0.0, 75 * DEG, 1, 1),    # single pixel
    (0.0, 0.3, 0.0, 20.0, 70 * DEG, 0.3, 75 * DEG, 13, 7),       # flat space
])
def test_frames_are_bit_exact(g, ctx, case):
    gpu, ref = _both(g, ctx, case)
    st = compare(gpu, ref)
    assert st["bit_identical"] == st["n"]


def test_f32_outputs_are_rounded_fp64(g, ctx):
    case = (0.5, 0.24, 0.3, 20.0, 80 * DEG, 0.0, 75 * DEG, 24, 16)
    gpu, ref = _both(g, ctx, case, dtype=g.GR_F32)
    st = compare(gpu, ref, angle_tol=0.0, f32=True)
    assert st["bit_identical"] == st["n"]


def test_step_limit_is_bit_exact(g, ctx):
    integ = g.make_integrator(max_steps=137)
    gpu, ref = _both(g, ctx, KERR64, integ=integ)
    st = compare(gpu, ref)
    assert st["bit_identical"] == st["n"]
    assert np.all(gpu["flag"] == g.GR_FLAG_TIMEOUT) and np.all(gpu["steps"] == 137)


def test_launch_shape_does_not_change_results(g, ctx):
    g.gr_trace_set_integrator(ctx, g.make_integrator(dt=0.01, max_steps=20000))
    case = (0.5, 0.24, 0.3, 20.0, 80 * DEG, 0.0, 75 * DEG, 48, 40)
    base = gpu_trace(ctx, *case)
    for block, wps, refill in [(64, 1, 1), (128, 2, 1), (256, 4, 1), (256, 0, 0), (64, 0, 0)]:
        g.gr_trace_set_launch(ctx, g.gr_launch(block, wps, refill))
        other = gpu_trace(ctx, *case)
        for k in base:
            np.testing.assert_array_equal(other[k], base[k], err_msg=f"{k} {block} {wps} {refill}")
    g.gr_trace_set_launch(ctx, None)


def test_queue_order_does_not_change_results(g, ctx):
    """Frames of at least 4096 pixels queued near-critical rays first give
    the outputs of pixel order, bit for bit (binary64 and mixed), and so do
    one-ray-per-lane launches (which take 8x8 tiles in row-major order and
    ignore the queue order; the 81x63 frame has ragged edge tiles)."""
    for case in [(0.5, 0.24, 0.3, 20.0, 80 * DEG, 0.0, 75 * DEG, 80, 64),
                 (0.5, 0.3, 0.2, 20.0, 70 * DEG, 0.0, 70 * DEG, 81, 63)]:
        for prec in (g.GR_FP64, g.GR_MIXED):
            g.gr_trace_set_integrator(ctx, g.make_integrator(dt=0.01, max_steps=20000,
                                                             precision=prec))
            g.gr_trace_set_launch(ctx, g.gr_launch(256, 0, 1, 0))
            plain = gpu_trace(ctx, *case)
            for shape in [(256, 0, 1, 2), (64, 0, 0, 2), (128, 0, 0, 2)]:
                g.gr_trace_set_launch(ctx, g.gr_launch(*shape))
                ordered = gpu_trace(ctx, *case)
                for k in plain:
                    np.testing.assert_array_equal(ordered[k], plain[k],
                                                  err_msg=f"{k} {prec} {shape}")
    g.gr_trace_set_launch(ctx, None)
    g.gr_trace_set_integrator(ctx, g.make_integrator(dt=0.01, max_steps=20000))


def test_pixel_list_matches_frame(g, ctx):
    g.gr_trace_set_integrator(ctx, g.make_integrator(dt=0.01, max_steps=20000))
    case = (0.5, 0.24, 0.3, 20.0, 80 * DEG, 0.0, 75 * DEG, 32, 24)
    frame = gpu_trace(ctx, *case)
    rng = np.random.default_rng(3)
    pix = np.concatenate([rng.integers(0, 32 * 24, 200), [0, 0, 32 * 24 - 1]])
    sub = gpu_trace(ctx, *case, pixels=pix)
    for k in frame:
        np.testing.assert_array_equal(sub[k], frame[k][pix], err_msg=k)
    empty = gpu_trace(ctx, *case, pixels=np.zeros(0, np.int32))
    assert empty["flag"].size == 0


def test_spin_reversal_mirror_on_gpu(g, ctx):
    g.gr_trace_set_integrator(ctx, g.make_integrator(dt=0.01, max_steps=20000))
    W, H = 24, 16
    A = gpu_trace(ctx, 0.5, 0.24, 0.3, 20.0, 80 * DEG, 0.0, 75 * DEG, W, H)
    B = gpu_trace(ctx, 0.5, -0.24, 0.3, 20.0, 80 * DEG, 0.0, 75 * DEG, W, H)
    mirror = lambda x: x.reshape(H, W)[:, ::-1].ravel()  # noqa: E731
    np.testing.assert_array_equal(A["phi"], -mirror(B["phi"]))
    np.testing.assert_array_equal(A["p_phi"], -mirror(B["p_phi"]))
    for k in ("t", "r", "theta", "p_t", "p_r", "p_theta", "flag", "steps"):
        np.testing.assert_array_equal(A[k], mirror(B[k]), err_msg=k)


def test_invalid_arguments_launch_nothing(g, ctx):
    import torch
    out = g.alloc_outputs(16, fields=("r",))
    m = g.gr_metric(0.5, 0.24, 0.0)
    bad = g.gr_camera(0.3, math.pi / 2, 0.0, 75 * DEG, 4, 4)          # inside the horizon
    with pytest.raises(g.GrError) as e:
        g.gr_trace_frame(ctx, m, bad, out.struct)
    assert e.value.code == g.GR_EINVAL
    torch.cuda.synchronize()
    assert np.all(out["flag"].cpu().numpy() == -1)


def test_kerr_newman_megapixel_sampled(g, ctx):
    """Full-size Kerr-Newman frame in the benchmark's launch configuration:
    1000x1000, M=0.5, a=0.24, Q=0.3, r0=20, theta0=80 deg, fov 75 deg,
    dt=0.005, 50000 steps, parameters rounded to binary32, binary32 end
    coordinates.  The oracle re-traces a stratified sample (every 32nd pixel
    in both axes) plus pixels on the shadow edge."""
    f = fp32_round
    case = (f(0.5), f(0.24), f(0.3), f(20.0), f(80 * DEG), 0.0, f(75 * DEG), 1000, 1000)
    integ = g.make_integrator(dt=0.005, max_steps=50000)
    g.gr_trace_set_integrator(ctx, integ)
    gpu = gpu_trace(ctx, *case, dtype=g.GR_F32, fields=("t", "r", "theta", "phi"))
    flag = gpu["flag"].reshape(1000, 1000)
    assert np.all((flag == g.GR_FLAG_ESCAPE) | (flag == g.GR_FLAG_HORIZON) |
                  (flag == g.GR_FLAG_TIMEOUT))
    edge = np.zeros_like(flag, bool)
    edge[1:-1, 1:-1] = (flag[1:-1, 1:-1] != flag[:-2, 1:-1]) | (flag[1:-1, 1:-1] != flag[2:, 1:-1])
    edge_pix = np.nonzero(edge.ravel())[0]
    rng = np.random.default_rng(7)
    edge_pix = rng.choice(edge_pix, size=min(256, edge_pix.size), replace=False)
    grid = (np.arange(16, 1000, 32)[:, None] * 1000 + np.arange(16, 1000, 32)[None, :]).ravel()
    pix = np.unique(np.concatenate([grid, edge_pix]))
    ref = oracle_trace(*case, integ, pixels=pix)
    sub = {k: v[pix] for k, v in gpu.items()}
    st = compare(sub, ref, angle_tol=0.0, f32=True)
    print(st, "escape", int((ref["flag"] == 1).sum()), "horizon", int((ref["flag"] == 2).sum()))
    assert st["bit_identical"] == st["n"]


def test_euler_megapixel_sampled(g, ctx):
    """Explicit Euler on the full-size Kerr-Newman frame in the benchmark's
    Euler configuration (the headline frame, dt=0.005, 50000 steps, binary32
    end coordinates): every 32nd pixel in both axes plus 256 pixels on the
    shadow edge, bit-exact against the oracle."""
    import oracle
    f = fp32_round
    case = (f(0.5), f(0.24), f(0.3), f(20.0), f(80 * DEG), 0.0, f(75 * DEG), 1000, 1000)
    g.gr_trace_set_integrator(ctx, g.make_integrator(dt=0.005, max_steps=50000,
                                                     method=g.GR_EULER))
    try:
        gpu = gpu_trace(ctx, *case, dtype=g.GR_F32, fields=("t", "r", "theta", "phi"))
    finally:
        g.gr_trace_set_integrator(ctx, g.make_integrator())
    flag = gpu["flag"].reshape(1000, 1000)
    edge = np.zeros_like(flag, bool)
    edge[1:-1, 1:-1] = (flag[1:-1, 1:-1] != flag[:-2, 1:-1]) | (flag[1:-1, 1:-1] != flag[2:, 1:-1])
    edge_pix = np.nonzero(edge.ravel())[0]
    edge_pix = np.random.default_rng(9).choice(edge_pix, size=min(256, edge_pix.size),
                                               replace=False)
    grid = (np.arange(16, 1000, 32)[:, None] * 1000 + np.arange(16, 1000, 32)[None, :]).ravel()
    pix = np.unique(np.concatenate([grid, edge_pix]))
    res = oracle.trace_frame(*case, dt=0.005, max_steps=50000, pixels=pix, want_p0=True, form="twin",
                             method=1)
    ref = {"t": res.t, "r": res.r, "theta": res.theta, "phi": res.phi, "flag": res.flag,
           "steps": res.steps}
    st = compare({k: v[pix] for k, v in gpu.items()}, ref, angle_tol=0.0, f32=True)
    assert st["bit_identical"] == st["n"]
    assert (res.flag == g.GR_FLAG_ESCAPE).sum() > 100 and (res.flag == g.GR_FLAG_HORIZON).sum() > 50


@pytest.mark.parametrize("case", [
    (0.5, 0.24, 0.3, 20.0, 80 * DEG, 0.0, 75 * DEG, 37, 23),     # Kerr-Newman, ragged
    (0.5, 0.49, 0.0, 20.0, 60 * DEG, 0.0, 75 * DEG, 24, 16),     # near-extremal
])
def test_euler_frames_are_bit_exact(g, ctx, case):
    """Explicit Euler steps (Sec. 3.1.1), whatever the launch shape."""
    integ = g.make_integrator(dt=0.01, max_steps=40000, method=g.GR_EULER)
    g.gr_trace_set_integrator(ctx, integ)
    for shape in [None, g.gr_launch(256, 0, 1, 2)]:
        g.gr_trace_set_launch(ctx, shape)
        gpu = gpu_trace(ctx, *case)
        import oracle
        res = oracle.trace_frame(*case, dt=0.01, max_steps=40000, want_p0=True, form="twin", method=1)
        ref = {"t": res.t, "r": res.r, "theta": res.theta, "phi": res.phi,
               "p_t": res.p0[:, 0], "p_r": res.pr, "p_theta": res.ptheta, "p_phi": res.p0[:, 3],
               "flag": res.flag, "steps": res.steps}
        st = compare(gpu, ref)
        assert st["bit_identical"] == st["n"]
    g.gr_trace_set_launch(ctx, None)
    g.gr_trace_set_integrator(ctx, g.make_integrator(dt=0.01, max_steps=20000))


def test_euler_is_refused_where_it_is_not_built(g):
    import torch
    ctx = g.gr_trace_init(0, g.make_integrator(method=g.GR_EULER))
    try:
        out = g.alloc_outputs(16, fields=("r",))
        inst = g.gr_instance(g.gr_metric(0.5, 0.24, 0.0),
                             g.gr_camera(20.0, math.pi / 2, 0.0, 75 * DEG, 4, 4), out.struct,
                             None, -1)
        with pytest.raises(g.GrError) as e:
            g.gr_trace_batch(ctx, [inst])
        assert e.value.code == g.GR_EUNSUPPORTED
        torch.cuda.synchronize()
    finally:
        g.gr_trace_destroy(ctx)
    with pytest.raises(g.GrError) as e:
        g.gr_trace_init(0, g.make_integrator(method=g.GR_EULER, precision=g.GR_MIXED))
    assert e.value.code == g.GR_EUNSUPPORTED


def test_oversized_frames_are_refused_before_launch(g, ctx):
    """A 2^20 x 2^20 frame (the largest the ABI accepts) has 2^34 8x8 tiles,
    more than one launch's grid holds.  Frames that exist only in the
    one-ray-per-lane form (Euler steps, the ring, the Manko-Novikov metric)
    refuse it before anything is launched: the (deliberately tiny) output
    arrays stay untouched."""
    import torch
    side = 1 << 20
    out = g.alloc_outputs(64, fields=("t",))
    out["flag"].fill_(77)
    cam = g.gr_camera(20.0, 80 * DEG, 0.0, 75 * DEG, side, side)
    for integ in (g.make_integrator(method=g.GR_EULER), g.make_integrator(disk=(2.0, 5.0, 0.02))):
        g.gr_trace_set_integrator(ctx, integ)
        with pytest.raises(g.GrError) as e:
            g.gr_trace_frame(ctx, g.gr_metric(0.5, 0.24, 0.3), cam, out.struct)
        assert e.value.code == g.GR_EUNSUPPORTED
    g.gr_trace_set_integrator(ctx, g.make_integrator())
    with pytest.raises(g.GrError) as e:
        g.gr_trace_frame_mn(ctx, g.gr_metric_mn(0.5, 0.24, 2.0), cam, out.struct)
    assert e.value.code == g.GR_EINVAL
    torch.cuda.synchronize()
    assert np.all(out["flag"].cpu().numpy() == 77)


LARGE_STEP = (0.5, 0.3, 0.2, 12.0, 70 * DEG, 0.0, 60 * DEG, 24, 24)


@pytest.mark.parametrize("launch", [None, (256, 0, 1, 0), (64, 0, 1, 0)])
def test_large_steps_finish_in_the_second_pass(g, ctx, launch):
    """dt = 0.5: steps rotate theta's (sin, cos) by more than 1/32, beyond the
    first pass's series; those rays are traced again by the second pass with
    the general rotation.  Every ray bit-identical to the twin form, whatever
    the launch form (tiles, persistent lanes)."""
    import oracle
    integ = g.make_integrator(dt=0.5, max_steps=20000)
    oracle.halved_rotations(reset=True)
    g.gr_trace_set_integrator(ctx, integ)
    if launch is not None:
        g.gr_trace_set_launch(ctx, g.gr_launch(*launch))
    gpu, ref = gpu_trace(ctx, *LARGE_STEP), oracle_trace(*LARGE_STEP, integ)
    assert oracle.halved_rotations() > 1000
    st = compare(gpu, ref, angle_tol=0.0)
    assert st["bit_identical"] == st["n"]


def test_large_steps_in_a_batch(g, ctx):
    """The same through the batch path (whole frame and a pixel list)."""
    import torch
    integ = g.make_integrator(dt=0.5, max_steps=20000)
    g.gr_trace_set_integrator(ctx, integ)
    M, a, Q, r0, th0, ph0, fov, W, H = LARGE_STEP
    pix = np.arange(0, W * H, 7)[::-1].copy()
    out1 = g.alloc_outputs(W * H, fields=("t", "r", "theta", "phi"))
    out2 = g.alloc_outputs(pix.size, fields=("t", "r", "theta", "phi"))
    pt = torch.as_tensor(pix.astype(np.int32), device="cuda")
    m, c = g.gr_metric(M, a, Q), g.gr_camera(r0, th0, ph0, fov, W, H)
    for launch in (None, g.gr_launch(64, 0, 0, 0)):
        g.gr_trace_set_launch(ctx, launch)
        g.gr_trace_batch(ctx, [g.gr_instance(m, c, out1.struct, None, -1),
                               g.gr_instance(m, c, out2.struct, pt.data_ptr(), pix.size)])
        torch.cuda.synchronize()
        for out, p in ((out1, None), (out2, pix)):
            got = {k: v.cpu().numpy() for k, v in out.tensors.items()}
            ref = oracle_trace(*LARGE_STEP, integ, pixels=p)
            st = compare(got, ref, angle_tol=0.0)
            assert st["bit_identical"] == st["n"]
