"""Seeded random draws over the tracer's whole parameter space, each traced on
the GPU through the C ABI and by the oracle: every field bit-identical.

A draw picks the spacetime (Kerr-Newman with a^2 + Q^2 < M^2, or
Manko-Novikov with |S| < M^2 and q in [-2, 2]), the camera (r0, theta0, phi0,
fov, a small ragged frame), the integrator (dt, now and then large enough
that RK4's carried angle leaves its series range and the second pass takes
the ray; step limit; RK4, Euler or RK4 in coordinate time; with or without
the ring; the forward-difference step, 1e-8 or one whose cosine is below 1),
the output precision and, for Kerr-Newman, the launch shape.  Frames are small so that the oracle finishes each in well
under a second."""
import math

import numpy as np
import pytest

from tests.gpu_util import compare

pytestmark = pytest.mark.gpu

DRAWS = 64


@pytest.fixture(scope="module")
def g():
    import paper_2310_15183_amd as g
    return g


def _draw(rng):
    M = float(rng.uniform(0.3, 1.0))
    mn = bool(rng.random() < 0.35)
    if mn:
        S = float(rng.uniform(0.05, 0.95)) * M * M * (1 if rng.random() < 0.8 else -1)
        q = float(rng.uniform(-2.0, 2.0))
        hole = (M, S, q)
    else:
        a = float(rng.uniform(0.0, 0.98)) * M
        Q = float(rng.uniform(0.0, 0.95)) * math.sqrt(M * M - a * a)
        hole = (M, a, Q)
    r0 = float(rng.uniform(6.0, 25.0)) * M
    th0 = float(rng.uniform(5.0, 175.0)) * math.pi / 180
    ph0 = float(rng.uniform(-math.pi, math.pi))
    fov = float(rng.uniform(20.0, 100.0)) * math.pi / 180
    W, H = int(rng.integers(1, 23)), int(rng.integers(1, 17))
    dt = float(rng.choice([0.02, 0.05, 0.02, 0.05, 0.4])) * M
    max_steps = int(rng.choice([137, 3000, 8000]))
    method = int(rng.choice([0, 0, 0, 0, 1, 2]))      # RK4, Euler, coordinate-time RK4
    disk = (3.0 * M, 8.0 * M, 0.03) if rng.random() < 0.25 else None
    f32 = bool(rng.random() < 0.5)
    launch = None
    if not mn and rng.random() < 0.5:
        launch = (int(rng.choice([64, 128, 256])), int(rng.integers(0, 5)),
                  int(rng.integers(0, 2)), int(rng.integers(0, 3)))
    # forward-difference step: 1e-8 (cos eps rounds to 1, the kernels' first
    # form) or larger (cos eps < 1, the general form)
    eps = float(rng.choice([1e-8, 1e-8, 1e-8, 2e-8, 1e-7]))
    return mn, hole, (r0, th0, ph0, fov, W, H), dt, max_steps, method, disk, f32, launch, eps


@pytest.mark.parametrize("seed", range(DRAWS))
def test_random_draw_is_bit_exact(g, seed):
    import torch

    import oracle
    rng = np.random.default_rng(1000 + seed)
    mn, hole, cam, dt, max_steps, method, disk, f32, launch, eps = _draw(rng)
    print("draw", seed, mn, hole, cam, dt, max_steps, method, disk, f32, launch, eps, flush=True)
    ctx = g.gr_trace_init(0, g.make_integrator(dt=dt, max_steps=max_steps, method=method,
                                               disk=disk, fd_eps=eps))
    try:
        if launch is not None:
            g.gr_trace_set_launch(ctx, g.gr_launch(*launch))
        W, H = cam[4], cam[5]
        out = g.alloc_outputs(W * H, dtype=g.GR_F32 if f32 else g.GR_F64, fields=g.FIELDS)
        camera = g.gr_camera(*cam)
        if mn:
            g.gr_trace_frame_mn(ctx, g.gr_metric_mn(*hole), camera, out.struct)
            trace = oracle.trace_frame_mn
        else:
            g.gr_trace_frame(ctx, g.gr_metric(*hole), camera, out.struct)
            trace = oracle.trace_frame
        torch.cuda.synchronize()
        gpu = {k: v.cpu().numpy() for k, v in out.tensors.items()}
    finally:
        g.gr_trace_destroy(ctx)
    res = trace(*hole, *cam, dt=dt, eps=eps, max_steps=max_steps, want_p0=True, form="twin",
                method=method, disk=disk)
    ref = {"t": res.t, "r": res.r, "theta": res.theta, "phi": res.phi, "p_t": res.p0[:, 0],
           "p_r": res.pr, "p_theta": res.ptheta, "p_phi": res.p0[:, 3], "flag": res.flag,
           "steps": res.steps}
    st = compare(gpu, ref, angle_tol=0.0, f32=f32)
    assert st["bit_identical"] == st["n"]


BATCH_DRAWS = 16


@pytest.mark.parametrize("seed", range(BATCH_DRAWS))
def test_random_batch_is_bit_exact(g, seed):
    """Random batches: 1-6 Kerr-Newman instances of random spacetimes, cameras
    and small ragged frames, some as pixel lists (possibly empty or with
    repeated pixels), traced in one gr_trace_batch call under a random launch
    shape; every instance bit-identical to the oracle."""
    import torch

    import oracle
    rng = np.random.default_rng(7000 + seed)
    dt = float(rng.choice([0.02, 0.05, 0.02, 0.05, 0.3]))    # 0.3: second-pass rays too
    max_steps = int(rng.choice([137, 3000]))
    f32 = bool(rng.random() < 0.5)
    eps = 2e-8 if seed % 4 == 3 else 1e-8        # the kernels' general form on every 4th batch
    ctx = g.gr_trace_init(0, g.make_integrator(dt=dt, max_steps=max_steps, fd_eps=eps))
    keep, insts, outs, spec = [], [], [], []
    try:
        if rng.random() < 0.7:
            g.gr_trace_set_launch(ctx, g.gr_launch(int(rng.choice([64, 128, 256])),
                                                   int(rng.integers(0, 5)),
                                                   int(rng.integers(0, 2)),
                                                   int(rng.integers(0, 3))))
        for _ in range(int(rng.integers(1, 7))):
            M = 0.5
            a = float(rng.uniform(0.0, 0.98)) * M
            Q = float(rng.uniform(0.0, 0.95)) * math.sqrt(M * M - a * a)
            cam = (float(rng.uniform(6.0, 25.0)) * M, float(rng.uniform(5, 175)) * math.pi / 180,
                   float(rng.uniform(-math.pi, math.pi)), float(rng.uniform(20, 100)) * math.pi / 180,
                   int(rng.integers(1, 20)), int(rng.integers(1, 14)))
            pix = None
            if rng.random() < 0.4:
                pix = rng.integers(0, cam[4] * cam[5], int(rng.integers(0, 40))).astype(np.int32)
            n = cam[4] * cam[5] if pix is None else len(pix)
            o = g.alloc_outputs(n, dtype=g.GR_F32 if f32 else g.GR_F64, fields=g.FIELDS)
            p_ptr, npix = None, -1
            if pix is not None:
                t = torch.as_tensor(pix, device="cuda")
                keep.append(t)
                p_ptr, npix = (t.data_ptr() or None), len(pix)
            insts.append(g.gr_instance(g.gr_metric(M, a, Q), g.gr_camera(*cam), o.struct, p_ptr,
                                       npix))
            outs.append(o)
            spec.append(((M, a, Q), cam, pix))
        print("batch draw", seed, dt, max_steps, f32, eps, [(s[0], s[1], None if s[2] is None else
                                                        len(s[2])) for s in spec], flush=True)
        g.gr_trace_batch(ctx, insts)
        torch.cuda.synchronize()
        got = [{k: v.cpu().numpy() for k, v in o.tensors.items()} for o in outs]
    finally:
        g.gr_trace_destroy(ctx)
    for (hole, cam, pix), res in zip(spec, got):
        if pix is not None and len(pix) == 0:
            assert res["flag"].size == 0
            continue
        r = oracle.trace_frame(*hole, *cam, dt=dt, eps=eps, max_steps=max_steps, pixels=pix,
                               want_p0=True, form="twin")
        ref = {"t": r.t, "r": r.r, "theta": r.theta, "phi": r.phi, "p_t": r.p0[:, 0],
               "p_r": r.pr, "p_theta": r.ptheta, "p_phi": r.p0[:, 3], "flag": r.flag,
               "steps": r.steps}
        st = compare(res, ref, angle_tol=0.0, f32=f32)
        assert st["bit_identical"] == st["n"]
