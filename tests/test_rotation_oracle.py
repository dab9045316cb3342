"""The kernel-twin form's rotation of a (sin, cos) pair (oracle.rotate): the
twin, and the HIP kernels it states, carry sin and cos of theta along a
Kerr-Newman RK4 ray and rotate them by each stage's increment instead of
evaluating sin/cos at every stage point.

Pins: the rotation against 60-digit arithmetic of s cos d + c sin d and
c cos d - s sin d for the same (s, c, d), over increments from 1e-12 to 10
rad of either sign (the series range |d| <= 1/32 and 1 to 9 halvings beyond
it); d = 0 returns the pair unchanged; d = +-pi/2 swaps the pair; rotating
by a then b agrees with rotating by a + b; and a frame traced with steps
large enough to need the halvings still meets the listing-form gate.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle
from tests.sens_gate import compare_at_sensitivity

mpmath.mp.dps = 60
ULP1 = 2.0 ** -52


def _exact(s, c, d):
    S, C, D = mpmath.mpf(s), mpmath.mpf(c), mpmath.mpf(d)
    return (float(S * mpmath.cos(D) + C * mpmath.sin(D)),
            float(C * mpmath.cos(D) - S * mpmath.sin(D)))


def test_rotation_against_high_precision():
    rng = np.random.default_rng(3)
    n = 4000
    x = rng.uniform(0.0, math.pi, n)
    s, c = np.sin(x), np.cos(x)
    d = np.exp(rng.uniform(math.log(1e-12), math.log(10.0), n)) * rng.choice([-1.0, 1.0], n)
    gs, gc = oracle.rotate(s, c, d)
    for k in range(n):
        es, ec = _exact(s[k], c[k], d[k])
        m = max(0, math.ceil(math.log2(abs(d[k]) / 0.03125))) if abs(d[k]) > 0.03125 else 0
        tol = (2.0 + 2.0 ** (m + 1)) * ULP1        # 2 ulp of 1, growing with the doublings
        assert abs(gs[k] - es) <= tol and abs(gc[k] - ec) <= tol, (x[k], d[k], m)


def test_rotation_special_cases():
    s, c = math.sin(0.7), math.cos(0.7)
    gs, gc = oracle.rotate(s, c, 0.0)
    assert gs[()] == s and gc[()] == c
    gs, gc = oracle.rotate(s, c, math.pi / 2)
    assert abs(gs[()] - c) < 4 * ULP1 and abs(gc[()] + s) < 4 * ULP1
    gs, gc = oracle.rotate(s, c, -math.pi / 2)
    assert abs(gs[()] + c) < 4 * ULP1 and abs(gc[()] - s) < 4 * ULP1


def test_rotations_compose():
    rng = np.random.default_rng(4)
    x = rng.uniform(0, math.pi, 500)
    a = rng.uniform(-0.05, 0.05, 500)
    b = rng.uniform(-0.05, 0.05, 500)
    s1, c1 = oracle.rotate(np.sin(x), np.cos(x), a)
    s2, c2 = oracle.rotate(s1, c1, b)
    s3, c3 = oracle.rotate(np.sin(x), np.cos(x), a + b)
    assert np.abs(s2 - s3).max() < 8 * ULP1 and np.abs(c2 - c3).max() < 8 * ULP1


@pytest.mark.parametrize("method", [0, 1, 2])
def test_large_steps_use_halved_rotations_and_meet_the_gate(method):
    """dt = 0.5 on a 24 x 24 Kerr-Newman frame: thousands of rotations by
    more than 1/32 with each integrator (RK4, Euler, coordinate-time RK4);
    the twin still meets the listing-form gate."""
    case = (0.5, 0.3, 0.2, 12.0, math.radians(70.0), 0.0, math.radians(60.0), 24, 24)
    oracle.halved_rotations(reset=True)
    twin = oracle.trace_frame(*case, dt=0.5, max_steps=20000, form="twin", method=method)
    assert oracle.halved_rotations() > 1000
    lis = oracle.trace_frame(*case, dt=0.5, max_steps=20000, probe=8, method=method)
    st = compare_at_sensitivity({"theta": twin.theta, "phi": twin.phi, "flag": twin.flag,
                                 "steps": twin.steps}, lis)
    print(st)
