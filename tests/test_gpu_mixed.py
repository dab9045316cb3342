"""Mixed-precision form (binary32 stages, binary64 differences and state
accumulation): accuracy against the binary64 path, which is itself
bit-identical to the oracle.

Error = great-circle angle between where the two runs' rays cross the escape
sphere (rays escaped in both); misclassified = pixels whose flags differ.
Gates: p99.9 <= 1e-4 rad and <= 0.1 % misclassified."""
import math

import numpy as np
import pytest

from tests.gpu_util import DEG, compare, gpu_trace, mixed_errors, oracle_trace

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import paper_2310_15183_amd as g
    return g


def _pair(g, case, dt=0.005, max_steps=50000):
    out = {}
    for prec in (g.GR_FP64, g.GR_MIXED):
        ctx = g.gr_trace_init(0, g.make_integrator(dt=dt, max_steps=max_steps, precision=prec))
        try:
            out[prec] = gpu_trace(ctx, *case)
        finally:
            g.gr_trace_destroy(ctx)
    return out[g.GR_FP64], out[g.GR_MIXED]


@pytest.mark.parametrize("name,case", [
    ("near-extremal Kerr", (0.5, 0.49, 0.0, 20.0, 60 * DEG, 0.0, 75 * DEG, 320, 320)),
    ("Kerr-Newman", (0.5, 0.24, 0.3, 20.0, 80 * DEG, 0.0, 75 * DEG, 320, 320)),
    ("wide Kerr-Newman, far camera", (0.5, 0.3, 0.35, 45.0, 30 * DEG, 0.4, 90 * DEG, 200, 150)),
    ("the benchmark's 1000x1000 Kerr-Newman frame",
     (0.5, 0.24, 0.3, 20.0, 80 * DEG, 0.0, 75 * DEG, 1000, 1000)),
    ("near-extremal Kerr at 1000x1000", (0.5, 0.49, 0.0, 20.0, 60 * DEG, 0.0, 75 * DEG, 1000, 1000)),
    ("near-extremal Kerr at 2048x2048", (0.5, 0.49, 0.0, 20.0, 60 * DEG, 0.0, 75 * DEG, 2048, 2048)),
])
def test_mixed_accuracy_against_fp64(g, name, case):
    """Whole frames, every pixel; the last two are the near-extremal Kerr frames
    of the precision workload (a = 0.98 M, theta0 = 60 deg, dt = 0.005,
    50000 steps) at both of its sizes."""
    ref, mix = _pair(g, case)
    e = mixed_errors(case[0], case[1], case[2], 1.5 * case[3], ref, mix)
    print(name, e)
    assert e["p999"] <= 1e-4
    assert e["flag_mismatch"] <= 1e-3
    assert e["median"] <= 1e-6


def test_fp64_reference_of_mixed_test_is_the_oracle(g):
    """The binary64 run the mixed form is judged against equals the oracle on
    a sample of the same frame."""
    case = (0.5, 0.49, 0.0, 20.0, 60 * DEG, 0.0, 75 * DEG, 320, 320)
    ref, _ = _pair(g, case)
    pix = np.arange(7, 320 * 320, 211)
    integ = g.make_integrator(dt=0.005, max_steps=50000)
    orc = oracle_trace(*case, integ, pixels=pix)
    st = compare({k: v[pix] for k, v in ref.items()}, orc)
    assert st["bit_identical"] == st["n"]


def test_mixed_handles_flat_space_and_step_limit(g):
    case = (0.0, 0.3, 0.0, 20.0, 70 * DEG, 0.3, 75 * DEG, 32, 24)
    ref, mix = _pair(g, case, dt=0.01, max_steps=20000)
    e = mixed_errors(0.0, 0.3, 0.0, 30.0, ref, mix)
    assert e["flag_mismatch"] == 0.0 and e["max"] < 1e-5
    ref, mix = _pair(g, case, dt=0.01, max_steps=50)
    assert np.all(mix["flag"] == g.GR_FLAG_TIMEOUT) and np.all(mix["steps"] == 50)


def test_mixed_batch_is_unsupported(g):
    ctx = g.gr_trace_init(0, g.make_integrator(precision=g.GR_MIXED))
    try:
        out = g.alloc_outputs(4, fields=("r",))
        inst = g.gr_instance(g.gr_metric(0.5, 0.2, 0.0),
                             g.gr_camera(20.0, 1.0, 0.0, 1.0, 2, 2), out.struct, None, -1)
        with pytest.raises(g.GrError) as e:
            g.gr_trace_batch(ctx, [inst])
        assert e.value.code == g.GR_EUNSUPPORTED
    finally:
        g.gr_trace_destroy(ctx)
