"""The HIP binary64 tracer against the listing form of the oracle (the
paper's method written as its plain definitions: the metric evaluated afresh
at each finite-difference point with the C library's sin/cos and its own
divisions, each component difference divided by eps, appendix "Code for
propagation of rays"), ray by ray at each ray's own rounding sensitivity.

The kernel follows a fixed IEEE operation sequence that the oracle's
kernel-twin form reproduces bit for bit (test_gpu_parity.py and the other
parity files); this file checks the kernel against the independent form:
flags and step counts identical on every ray whose one-ulp probes leave them
unchanged, end angles within K_MAX times the ray's sensitivity s
(tests/sens_gate.py), and within 1e-9 rad on every ray the probes find well
conditioned (s <= 1e-10, the conditioning threshold of the paper's
ill-posed near-critical rays, Sec. 3.3).
"""
import math

import numpy as np
import pytest

from tests.gpu_util import DEG, fp32_round, gpu_trace
from tests.sens_gate import compare_at_sensitivity

pytestmark = pytest.mark.gpu

WELL_CONDITIONED = 1e-10     # s at or below this: the absolute 1e-9 rad gate applies
ABS_GATE = 1e-9


@pytest.fixture(scope="module")
def g():
    import paper_2310_15183_amd as g
    return g


def _listing(case, integ, pixels=None, mn=False):
    import oracle
    trace = oracle.trace_frame_mn if mn else oracle.trace_frame
    return trace(*case, dt=integ.dt, eps=integ.fd_eps, horizon_norm=integ.horizon_norm,
                 escape_factor=integ.escape_factor, max_steps=integ.max_steps, pixels=pixels,
                 probe=8)


def _gate(gpu, ref):
    st = compare_at_sensitivity(gpu, ref)
    ok = ~np.asarray(ref.flip, bool)
    well = ok & (ref.sens <= WELL_CONDITIONED) & ~np.isnan(ref.theta)
    d = np.maximum(np.abs(gpu["theta"] - ref.theta), np.abs(gpu["phi"] - ref.phi))[well]
    st["well_conditioned"] = int(well.sum())
    st["well_conditioned_d_max"] = float(d.max()) if d.size else 0.0
    assert d.size == 0 or d.max() <= ABS_GATE, st
    return st


def _edge_sample(flag, side, stride, n_edge, seed):
    """Every stride-th pixel in both axes plus n_edge pixels where the flag
    changes between vertical neighbours (the shadow edge)."""
    f = flag.reshape(side, side)
    edge = np.zeros_like(f, bool)
    edge[1:-1, :] = (f[1:-1, :] != f[:-2, :]) | (f[1:-1, :] != f[2:, :])
    edge_pix = np.nonzero(edge.ravel())[0]
    edge_pix = np.random.default_rng(seed).choice(edge_pix, size=min(n_edge, edge_pix.size),
                                                  replace=False)
    grid = (np.arange(stride // 2, side, stride)[:, None] * side
            + np.arange(stride // 2, side, stride)[None, :]).ravel()
    return np.unique(np.concatenate([grid, edge_pix]))


@pytest.mark.parametrize("case", [
    (0.5, 0.24, 0.0, 20.0, math.pi / 2, 0.0, 75 * DEG, 64, 64),   # the small Kerr frame
    (0.5, 0.24, 0.3, 20.0, 80 * DEG, 0.0, 75 * DEG, 37, 23),      # Kerr-Newman, ragged
    (0.5, 0.49, 0.0, 20.0, 60 * DEG, 0.0, 75 * DEG, 30, 30),      # near-extremal Kerr
])
def test_frames_match_the_listing_form(g, case):
    integ = g.make_integrator(dt=0.01, max_steps=20000)
    ctx = g.gr_trace_init(0, integ)
    try:
        gpu = gpu_trace(ctx, *case)
    finally:
        g.gr_trace_destroy(ctx)
    st = _gate(gpu, _listing(case, integ))
    print(st)


@pytest.mark.parametrize("name", ["kerr_newman", "near_extremal"])
def test_megapixel_frames_match_the_listing_form(g, name):
    """Full-size frames, sampled: the 1000^2 Kerr-Newman frame of the
    benchmark (binary32-rounded inputs, dt = 0.005, 50000 steps) and the
    1000^2 near-extremal Kerr frame (a = 0.98 M, theta0 = 60 deg, same
    integrator)."""
    f = fp32_round
    if name == "kerr_newman":
        case = (f(0.5), f(0.24), f(0.3), f(20.0), f(80 * DEG), 0.0, f(75 * DEG), 1000, 1000)
    else:
        case = (0.5, 0.49, 0.0, 20.0, 60 * DEG, 0.0, 75 * DEG, 1000, 1000)
    integ = g.make_integrator(dt=0.005, max_steps=50000)
    ctx = g.gr_trace_init(0, integ)
    try:
        gpu = gpu_trace(ctx, *case, fields=("t", "r", "theta", "phi"))
    finally:
        g.gr_trace_destroy(ctx)
    pix = _edge_sample(gpu["flag"], 1000, 64, 128, seed=5)
    ref = _listing(case, integ, pixels=pix)
    st = _gate({k: v[pix] for k, v in gpu.items()}, ref)
    print(name, st)
    assert (ref.flag == 1).sum() > 50 and (ref.flag == 2).sum() > 50


def test_manko_novikov_frame_matches_the_listing_form(g):
    """The listing's spacetime (M = 0.5, S = 0.24, q = 2), 24 x 24."""
    case = (0.5, 0.24, 2.0, 8.0, math.pi / 2, 0.0, 75 * DEG, 24, 24)
    integ = g.make_integrator(dt=0.01, max_steps=20000)
    ctx = g.gr_trace_init(0, integ)
    try:
        import torch
        out = g.alloc_outputs(24 * 24, fields=("t", "r", "theta", "phi"))
        g.gr_trace_frame_mn(ctx, g.gr_metric_mn(*case[:3]), g.gr_camera(*case[3:]), out.struct)
        torch.cuda.synchronize()
        gpu = {k: v.cpu().numpy() for k, v in out.tensors.items()}
    finally:
        g.gr_trace_destroy(ctx)
    st = _gate(gpu, _listing(case, integ, mn=True))
    print(st)
