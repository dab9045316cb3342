"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/grtrace.h, and validates arguments on the host."""
import math
import os
import re
import subprocess

import pytest

import paper_2310_15183_amd as g

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "grtrace.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gr_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 10
    out = subprocess.run(["nm", "-D", "--defined-only", g.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (gr_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert sorted(g.EXPORTED) == names


def test_strerror_and_horizon():
    assert g.gr_trace_strerror(g.GR_OK) == "success"
    assert g.gr_trace_strerror(g.GR_EINVAL) == "invalid argument"
    assert g.gr_trace_strerror(12345) == "unknown error code"
    assert g.gr_horizon_radius(g.gr_metric(0.5, 0.24, 0.3)) == pytest.approx(
        0.5 + math.sqrt(0.25 - 0.24 ** 2 - 0.09), rel=1e-15)
    assert g.gr_horizon_radius(g.gr_metric(1.0, 0.0, 0.0)) == 2.0


def _valid():
    m = g.gr_metric(0.5, 0.24, 0.3)
    c = g.gr_camera(20.0, math.radians(80), 0.0, math.radians(75), 64, 48)
    i = g.make_integrator()
    o = g.gr_output()
    o.flag = 0x1000                         # any non-null pointer: nothing is dereferenced
    o.dtype = g.GR_F64
    return m, c, i, o


def test_validation_accepts_valid_arguments():
    assert g.gr_trace_validate(*_valid()) == g.GR_OK


@pytest.mark.parametrize("field,value", [
    ("M", -1.0), ("a", 0.49), ("Q", 0.5), ("M", float("nan")), ("a", float("inf"))])
def test_validation_rejects_bad_metric(field, value):
    m, c, i, o = _valid()
    setattr(m, field, value)
    assert g.gr_trace_validate(m, c, i, o) == g.GR_EINVAL


@pytest.mark.parametrize("field,value", [
    ("r0", 0.5), ("r0", float("nan")), ("theta0", 0.0), ("theta0", math.pi), ("fov", 0.0),
    ("fov", math.pi), ("width", 0), ("height", -3)])
def test_validation_rejects_bad_camera(field, value):
    m, c, i, o = _valid()
    setattr(c, field, value)
    assert g.gr_trace_validate(m, c, i, o) == g.GR_EINVAL


@pytest.mark.parametrize("field,value", [
    ("dt", 0.0), ("dt", -1.0), ("fd_eps", 0.0), ("horizon_norm", 0.0),
    ("escape_factor", 1.0), ("max_steps", -1), ("precision", 7)])
def test_validation_rejects_bad_integrator(field, value):
    m, c, i, o = _valid()
    setattr(i, field, value)
    assert g.gr_trace_validate(m, c, i, o) == g.GR_EINVAL


def test_validation_rejects_bad_output():
    m, c, i, o = _valid()
    o.flag = None
    assert g.gr_trace_validate(m, c, i, o) == g.GR_EINVAL
    m, c, i, o = _valid()
    o.dtype = 9
    assert g.gr_trace_validate(m, c, i, o) == g.GR_EINVAL


def test_extremal_and_flat_metrics_are_valid():
    m, c, i, o = _valid()
    for M, a, Q in [(0.5, 0.5, 0.0), (0.0, 0.0, 0.0), (0.5, 0.3, 0.39), (0.0, 0.3, 0.0)]:
        assert g.gr_trace_validate(g.gr_metric(M, a, Q), c, i, o) == g.GR_OK
    assert g.gr_trace_validate(g.gr_metric(0.0, 0.0, 0.1), c, i, o) == g.GR_EINVAL
    assert g.gr_horizon_radius(g.gr_metric(0.0, 0.3, 0.0)) == 0.0


@pytest.mark.parametrize("fields,code", [
    ({"method": 3}, "GR_EINVAL"),
    ({"method": -1}, "GR_EINVAL"),
    ({"method": 1, "precision": 1}, "GR_EUNSUPPORTED"),
    ({"method": 2, "precision": 1}, "GR_EUNSUPPORTED"),
    ({"disk_r_in": 2.0, "disk_r_out": 5.0, "disk_half_angle": math.pi / 2}, "GR_EINVAL"),
    ({"disk_r_in": 5.0, "disk_r_out": 2.0, "disk_half_angle": 0.02}, "GR_EINVAL"),
    ({"disk_r_in": -1.0, "disk_r_out": 2.0, "disk_half_angle": 0.02}, "GR_EINVAL"),
    ({"disk_r_in": 2.0, "disk_r_out": float("inf"), "disk_half_angle": 0.02}, "GR_EINVAL"),
    ({"disk_half_angle": -0.1}, "GR_EINVAL"),
    ({"disk_r_in": 2.0, "disk_r_out": 5.0, "disk_half_angle": 0.02, "precision": 1},
     "GR_EUNSUPPORTED"),
])
def test_validation_of_method_and_ring(fields, code):
    m, c, i, o = _valid()
    for k, v in fields.items():
        setattr(i, k, v)
    assert g.gr_trace_validate(m, c, i, o) == getattr(g, code)


def test_method_and_ring_accepted():
    m, c, _, o = _valid()
    for integ in [g.make_integrator(method=g.GR_EULER),
                  g.make_integrator(method=g.GR_RK4_TIME),
                  g.make_integrator(method=g.GR_RK4_TIME, disk=(2.0, 5.0, 0.3)),
                  g.make_integrator(disk=(0.0, 5.0, 0.02)),
                  g.make_integrator(method=g.GR_EULER, disk=(2.0, 5.0, 0.3))]:
        assert g.gr_trace_validate(m, c, integ, o) == g.GR_OK


@pytest.mark.parametrize("w,h,code", [
    (1 << 20, 1 << 20, 0),                  # 2^40 rays: the largest frame accepted
    ((1 << 20) + 1, 1 << 20, -1),           # one column more
    ((1 << 31) - 1, 1, 0),                  # widest single row
    (1, (1 << 31) - 1, 0),                  # tallest single column
    (1, 1, 0)])                             # a single pixel
def test_frame_size_limits(w, h, code):
    m, c, i, o = _valid()
    c.width, c.height = w, h
    assert g.gr_trace_validate(m, c, i, o) == (g.GR_OK if code == 0 else g.GR_EINVAL)
