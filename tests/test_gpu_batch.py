"""Batched persistent launch: many instances in one kernel fed by one work
queue.  Results must equal the per-frame path and the oracle bit for bit,
for every queue order, launch shape and autotuned shape."""
import os

import numpy as np
import pytest

from paper_2310_15183_amd.workloads import batch_instances
from tests.gpu_util import compare, oracle_trace

pytestmark = pytest.mark.gpu

FIELDS = ("t", "r", "theta", "phi", "p_t", "p_r", "p_theta", "p_phi")


@pytest.fixture(scope="module")
def g():
    import paper_2310_15183_amd as g
    return g


@pytest.fixture()
def ctx(g):
    c = g.gr_trace_init(0, g.make_integrator(dt=0.01, max_steps=20000))
    yield c
    g.gr_trace_destroy(c)


def _make(g, insts, dtype=None, pixel_lists=None):
    import torch
    dtype = g.GR_F64 if dtype is None else dtype
    outs, structs, keep = [], [], []
    for k, I in enumerate(insts):
        pix = None if pixel_lists is None else pixel_lists[k]
        n = I.width * I.height if pix is None else len(pix)
        o = g.alloc_outputs(n, dtype=dtype, fields=FIELDS)
        if pix is None:
            p_ptr, npix = None, -1
        else:
            t = torch.as_tensor(np.asarray(pix, np.int32), device="cuda")
            keep.append(t)
            p_ptr, npix = (t.data_ptr() or None), len(pix)
        structs.append(g.gr_instance(g.gr_metric(I.M, I.a, I.Q),
                                     g.gr_camera(I.r0, I.theta0, I.phi0, I.fov, I.width,
                                                 I.height), o.struct, p_ptr, npix))
        outs.append(o)
    return outs, structs, keep


def _np(outs):
    import torch
    torch.cuda.synchronize()
    return [{k: v.cpu().numpy() for k, v in o.tensors.items()} for o in outs]


def test_batch_equals_frames_and_oracle(g, ctx):
    insts = batch_instances(8, scale=16)                   # sides 8..32 pixels
    outs, structs, _ = _make(g, insts)
    g.gr_trace_batch(ctx, structs)
    got = _np(outs)
    integ = g.make_integrator(dt=0.01, max_steps=20000)
    for I, res in zip(insts, got):
        one = g.alloc_outputs(I.width * I.height, fields=FIELDS)
        g.gr_trace_frame(ctx, g.gr_metric(I.M, I.a, I.Q),
                         g.gr_camera(I.r0, I.theta0, I.phi0, I.fov, I.width, I.height),
                         one.struct)
        frame = _np([one])[0]
        for k in frame:
            np.testing.assert_array_equal(res[k], frame[k], err_msg=k)
        ref = oracle_trace(I.M, I.a, I.Q, I.r0, I.theta0, I.phi0, I.fov, I.width, I.height,
                           integ)
        st = compare(res, ref)
        assert st["bit_identical"] == st["n"]


def test_batch_with_pixel_lists_and_empty_instances(g, ctx):
    insts = batch_instances(6, seed=5, scale=16)
    rng = np.random.default_rng(11)
    lists = [None, rng.integers(0, insts[1].width * insts[1].height, 50), np.zeros(0, int),
             None, rng.integers(0, insts[4].width * insts[4].height, 7), None]
    outs, structs, keep = _make(g, insts, dtype=g.GR_F32, pixel_lists=lists)
    g.gr_trace_batch(ctx, structs)
    got = _np(outs)
    integ = g.make_integrator(dt=0.01, max_steps=20000)
    for I, res, pix in zip(insts, got, lists):
        if pix is not None and len(pix) == 0:
            assert res["flag"].size == 0
            continue
        ref = oracle_trace(I.M, I.a, I.Q, I.r0, I.theta0, I.phi0, I.fov, I.width, I.height,
                           integ, pixels=pix)
        st = compare(res, ref, angle_tol=0.0, f32=True)
        assert st["bit_identical"] == st["n"]


def test_batch_order_and_shape_do_not_change_results(g, ctx):
    insts = batch_instances(10, seed=9, scale=16)
    outs, structs, _ = _make(g, insts)
    g.gr_trace_batch(ctx, structs)
    base = _np(outs)
    for shape in [(64, 1, 1, 0), (128, 2, 1, 1), (256, 0, 1, 0), (256, 4, 1, 1)]:
        g.gr_trace_set_launch(ctx, g.gr_launch(*shape))
        for o in outs:
            for t in o.tensors.values():
                t.fill_(-7)
        g.gr_trace_batch(ctx, structs)
        other = _np(outs)
        for a, b in zip(base, other):
            for k in a:
                np.testing.assert_array_equal(b[k], a[k], err_msg=f"{k} {shape}")
    g.gr_trace_set_launch(ctx, None)


def test_autotune_picks_a_shape_and_caches_it(g, ctx, tmp_path):
    insts = batch_instances(12, seed=3, scale=16)
    outs, structs, _ = _make(g, insts)
    g.gr_trace_batch(ctx, structs)
    base = _np(outs)
    cache = str(tmp_path / "autotune.jsonl")
    best = g.gr_trace_autotune(ctx, structs, trial_steps=300, cache_path=cache)
    assert best.block in (64, 128, 256) and best.order in (0, 1)
    got = _np(outs)
    for a, b in zip(base, got):
        for k in a:
            np.testing.assert_array_equal(b[k], a[k], err_msg=k)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and '"key": "gfx950/trace_fp64_batch/' in lines[0]
    again = g.gr_trace_autotune(ctx, structs, trial_steps=300, cache_path=cache)
    assert (again.block, again.waves_per_simd, again.order) == (best.block, best.waves_per_simd,
                                                                 best.order)
    assert len(open(cache).read().splitlines()) == 1          # reused, not re-tuned
    cur = g.gr_trace_get_launch(ctx)
    assert (cur.block, cur.order) == (best.block, best.order)


def test_full_size_batch_sampled(g, ctx):
    """All 256 seeded instances at their full sizes (about 3.1e7 rays) in one
    launch; the oracle re-traces 3 rays of every instance."""
    insts = batch_instances(256)
    outs, structs, _ = _make(g, insts, dtype=g.GR_F32)
    g.gr_trace_batch(ctx, structs)
    import torch
    torch.cuda.synchronize()
    integ = g.make_integrator(dt=0.01, max_steps=20000)
    rng = np.random.default_rng(2)
    n_ok = 0
    for I, o in zip(insts, outs):
        n = I.width * I.height
        pix = rng.integers(0, n, 3)
        sub = {k: v[torch.as_tensor(pix, device="cuda")].cpu().numpy()
               for k, v in o.tensors.items()}
        ref = oracle_trace(I.M, I.a, I.Q, I.r0, I.theta0, I.phi0, I.fov, I.width, I.height,
                           integ, pixels=pix)
        st = compare(sub, ref, angle_tol=0.0, f32=True)
        assert st["bit_identical"] == st["n"]
        n_ok += st["n"]
    assert n_ok == 3 * 256
    total = sum(I.width * I.height for I in insts)
    print("rays", total)
