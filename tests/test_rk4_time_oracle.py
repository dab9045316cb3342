"""Pins of the oracle's RK4 with coordinate time as the parameter (method 2,
the per-stage reparametrised form of Sec. 3.1.2's RK4 for the coordinate-time
steps of the listing): every stage's derivative is divided by that stage's
own |dt/dtau|, so each step advances t by exactly dt; it is fourth order
(the end azimuth of equatorial Reissner-Nordstrom rays against the sweep
integral to the ray's own end radius: the error falls ~13x per halving of
dt, against ~2x for Euler); it converges to the same rays as the listing's
RK4 (h fixed from the first stage); and the kernel-twin form meets the
listing-form gate with it."""
import math

import numpy as np
import pytest

import oracle
from tests import physics
from tests.sens_gate import compare_at_sensitivity

M, Q, R0, W = 0.5, 0.3, 20.0, 41
FOV = math.radians(60.0)
PIX = np.arange(W // 2 + 3, W)                       # equatorial rays with x > 0


def _sweep_errors(dt, method, form):
    res = oracle.trace_frame(M, 0.0, Q, R0, math.pi / 2, 0.0, FOV, W, 1, dt=dt,
                             max_steps=100000, pixels=PIX, method=method, form=form)
    f = 1 - 2 * M / R0 + Q * Q / R0 ** 2
    x = ((2 * PIX + 1 - W) / W) * math.tan(FOV / 2)
    b = R0 * (x / np.sqrt(1 + x * x)) / math.sqrt(f)
    esc = res.flag == oracle.FLAG_ESCAPE
    assert esc.sum() >= 14 and np.all(esc[2:])       # the two smallest impact parameters are captured
    k = np.arange(2, PIX.size)
    want = np.array([physics.rn_sweep(M, Q, b[i], R0, res.r[i]) for i in k])
    return np.abs(res.phi[k] - want), res


@pytest.mark.parametrize("form", ["listing", "twin"])
def test_coordinate_time_rk4_is_fourth_order(form):
    e = {dt: _sweep_errors(dt, 2, form)[0] for dt in (1.6, 0.8, 0.4)}
    r1 = np.median(e[1.6] / e[0.8])
    r2 = np.median(e[0.8] / e[0.4])
    print(form, r1, r2)
    assert 8.0 < r1 < 24.0 and 8.0 < r2 < 24.0              # 2^4 = 16 (2^1 for Euler)
    eu = {dt: _sweep_errors(dt, 1, form)[0] for dt in (0.1, 0.05)}
    assert 1.5 < np.median(eu[0.1] / eu[0.05]) < 2.6


@pytest.mark.parametrize("form", ["listing", "twin"])
def test_each_step_advances_coordinate_time_by_dt(form):
    _, res = _sweep_errors(0.4, 2, form)
    np.testing.assert_allclose(res.t, -0.4 * res.steps, rtol=0, atol=1e-12)
    assert res.steps.min() > 20


def test_converges_to_the_listing_rk4_rays():
    case = (0.5, 0.3, 0.2, 20.0, math.radians(75.0), 0.0, math.radians(60.0), 16, 12)
    a = oracle.trace_frame(*case, dt=0.01, max_steps=100000, method=2, form="twin")
    b = oracle.trace_frame(*case, dt=0.01, max_steps=100000, method=0, form="twin")
    both = (a.flag == 1) & (b.flag == 1)
    assert both.sum() > 150 and (a.flag == b.flag).mean() > 0.99
    d = np.abs(a.phi[both] - b.phi[both])
    assert np.median(d) < 1e-6


@pytest.mark.parametrize("mn", [False, True])
def test_twin_matches_listing_with_coordinate_time_rk4(mn):
    if mn:
        case = (0.5, 0.24, 2.0, 8.0, math.pi / 2, 0.0, math.radians(75.0), 20, 20)
        trace = oracle.trace_frame_mn
    else:
        case = (0.5, 0.3, 0.2, 20.0, math.radians(75.0), 0.0, math.radians(60.0), 24, 18)
        trace = oracle.trace_frame
    lis = trace(*case, dt=0.01, max_steps=20000, method=2, probe=8)
    twin = trace(*case, dt=0.01, max_steps=20000, method=2, form="twin")
    st = compare_at_sensitivity({"theta": twin.theta, "phi": twin.phi, "flag": twin.flag,
                                 "steps": twin.steps}, lis)
    print(st)
