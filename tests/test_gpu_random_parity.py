"""Seeded random draws over the tracer's whole parameter space, each traced on
the GPU through the C ABI and by the oracle: every field bit-identical.

A draw picks the spacetime (Kerr-Newman with a^2 + Q^2 < M^2, or
Manko-Novikov with |S| < M^2 and q in [-2, 2]), the camera (r0, theta0, phi0,
fov, a small ragged frame), the integrator (dt, step limit, RK4 or Euler,
with or without the ring), the output precision and, for Kerr-Newman, the
launch shape.  Frames are small so that the oracle finishes each in well
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
    dt = float(rng.choice([0.02, 0.05])) * M
    max_steps = int(rng.choice([137, 3000, 8000]))
    method = int(rng.random() < 0.25)
    disk = (3.0 * M, 8.0 * M, 0.03) if rng.random() < 0.25 else None
    f32 = bool(rng.random() < 0.5)
    launch = None
    if not mn and rng.random() < 0.5:
        launch = (int(rng.choice([64, 128, 256])), int(rng.integers(0, 5)),
                  int(rng.integers(0, 2)), int(rng.integers(0, 3)))
    return mn, hole, (r0, th0, ph0, fov, W, H), dt, max_steps, method, disk, f32, launch


@pytest.mark.parametrize("seed", range(DRAWS))
def test_random_draw_is_bit_exact(g, seed):
    import torch

    import oracle
    rng = np.random.default_rng(1000 + seed)
    mn, hole, cam, dt, max_steps, method, disk, f32, launch = _draw(rng)
    print("draw", seed, mn, hole, cam, dt, max_steps, method, disk, f32, launch, flush=True)
    ctx = g.gr_trace_init(0, g.make_integrator(dt=dt, max_steps=max_steps, method=method,
                                               disk=disk))
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
    res = trace(*hole, *cam, dt=dt, max_steps=max_steps, want_p0=True, method=method, disk=disk)
    ref = {"t": res.t, "r": res.r, "theta": res.theta, "phi": res.phi, "p_t": res.p0[:, 0],
           "p_r": res.pr, "p_theta": res.ptheta, "p_phi": res.p0[:, 3], "flag": res.flag,
           "steps": res.steps}
    st = compare(gpu, ref, angle_tol=0.0, f32=f32)
    assert st["bit_identical"] == st["n"]
