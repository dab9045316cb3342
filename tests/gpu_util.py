"""Helpers shared by the GPU tests: run the HIP tracer through the C ABI and
the CPU oracle on the same camera, and compare."""
from __future__ import annotations

import math

import numpy as np

FLOAT_FIELDS = ("t", "r", "theta", "phi", "p_t", "p_r", "p_theta", "p_phi")


def gpu_trace(ctx, M, a, Q, r0, th0, ph0, fov, W, H, dtype=None, pixels=None, stream=None,
              fields=FLOAT_FIELDS):
    """Trace a frame (or a pixel list) on the GPU; returns numpy arrays."""
    import torch

    import paper_2310_15183_amd as g
    dtype = g.GR_F64 if dtype is None else dtype
    n = W * H if pixels is None else len(pixels)
    out = g.alloc_outputs(n, dtype=dtype, fields=fields)
    m = g.gr_metric(M, a, Q)
    c = g.gr_camera(r0, th0, ph0, fov, W, H)
    if pixels is None:
        g.gr_trace_frame(ctx, m, c, out.struct, stream)
    else:
        pix = torch.as_tensor(np.asarray(pixels, dtype=np.int32), device="cuda")
        inst = g.gr_instance(m, c, out.struct, pix.data_ptr() or None, n)
        g.gr_trace_batch(ctx, [inst], stream)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.tensors.items()}


def oracle_trace(M, a, Q, r0, th0, ph0, fov, W, H, integ, pixels=None):
    import oracle
    res = oracle.trace_frame(M, a, Q, r0, th0, ph0, fov, W, H, dt=integ.dt,
                             eps=integ.fd_eps, horizon_norm=integ.horizon_norm,
                             escape_factor=integ.escape_factor, max_steps=integ.max_steps,
                             pixels=pixels, want_p0=True, form="twin", method=integ.method)
    return {"t": res.t, "r": res.r, "theta": res.theta, "phi": res.phi,
            "p_t": res.p0[:, 0], "p_r": res.pr, "p_theta": res.ptheta, "p_phi": res.p0[:, 3],
            "flag": res.flag, "steps": res.steps}


def compare(gpu, ref, angle_tol=1e-9, f32=False):
    """Flags and steps must agree exactly; theta/phi within angle_tol (raw,
    unwrapped).  Returns a dict of statistics, including how many rays are
    bit-identical in every floating-point field."""
    np.testing.assert_array_equal(gpu["flag"], ref["flag"])
    if "steps" in gpu:
        np.testing.assert_array_equal(gpu["steps"], ref["steps"])
    stats = {}
    same = np.ones(ref["flag"].shape, bool)
    for k in FLOAT_FIELDS:
        if k not in gpu:
            continue
        want = ref[k].astype(np.float32) if f32 else ref[k]
        got = gpu[k]
        same &= (got == want) | (np.isnan(got) & np.isnan(want))
    for k in ("theta", "phi"):
        want = ref[k].astype(np.float32).astype(np.float64) if f32 else ref[k]
        got = gpu[k].astype(np.float64)
        both_nan = np.isnan(got) & np.isnan(want)           # invalid rays on both sides
        d = np.abs(got - want)[~both_nan]
        stats[f"max_d{k}"] = float(d.max()) if d.size else 0.0
        assert d.size == 0 or d.max() <= angle_tol, (k, float(d.max()))
    stats["bit_identical"] = int(same.sum())
    stats["n"] = int(same.size)
    return stats


def fp32_round(x):
    return float(np.float32(x))


DEG = math.pi / 180.0


from paper_2310_15183_amd.evaluate import mixed_errors, sky_at_escape  # noqa: E402,F401
