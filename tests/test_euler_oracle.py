"""Pins of the oracle's explicit Euler integrator (paper Sec. 3.1.1): each
step advances coordinate time by exactly dt (to rounding), it is first
order (the drift of the conserved H halves with dt, where RK4's falls
~16x), and it converges to the RK4 ray."""
import math

import numpy as np

import oracle

M, A_SPIN, Q = 0.5, 0.24, 0.3
CAM = (20.0, math.radians(80.0), 0.0, math.radians(60.0), 16, 12)


def _frame(dt, method, max_steps):
    return oracle.trace_frame(M, A_SPIN, Q, *CAM, dt=dt, max_steps=max_steps, want_p0=True,
                              method=method)


def _hamiltonian(res, k):
    g = oracle.inverse_metric(M, A_SPIN, Q, res.r[k], res.theta[k])
    pt, pph = res.p0[k, 0], res.p0[k, 3]
    pr, pth = res.pr[k], res.ptheta[k]
    return 0.5 * (g[0] * pt * pt + 2 * g[1] * pt * pph + g[2] * pr * pr + g[3] * pth * pth
                  + g[4] * pph * pph)


def test_euler_steps_advance_coordinate_time_by_dt():
    res = _frame(0.02, 1, 300)
    ok = res.flag != 3
    np.testing.assert_allclose(res.t[ok], -0.02 * res.steps[ok], rtol=0, atol=1e-12 * 300)


def test_euler_is_first_order():
    """Median |H| at the end of escaping rays: Euler's halves with dt (first
    order; measured ratio 2.0 from dt = 0.04 to 0.005), while RK4's sits at
    the floor the eps = 1e-8 forward difference leaves (~3e-9 at every dt
    here), five orders below."""
    drift = {}
    for method in (0, 1):
        for dt in (0.02, 0.01):
            res = _frame(dt, method, 100000)
            esc = np.nonzero(res.flag == 1)[0]
            drift[(method, dt)] = np.median([abs(_hamiltonian(res, k)) for k in esc])
    euler_ratio = drift[(1, 0.02)] / drift[(1, 0.01)]
    assert 1.8 < euler_ratio < 2.2, euler_ratio
    assert drift[(0, 0.02)] < 1e-8 and drift[(0, 0.01)] < 1e-8
    assert drift[(1, 0.01)] > 1e4 * drift[(0, 0.01)]


def test_euler_converges_to_the_rk4_ray():
    """Escape directions (end position moved back to the escape sphere along
    the last step) of Euler rays approach RK4's as dt shrinks."""
    ref = _frame(0.01, 0, 100000)

    def err(dt):
        res = _frame(dt, 1, 400000)
        both = (res.flag == 1) & (ref.flag == 1)
        return np.median(np.abs(np.unwrap(res.phi[both]) - np.unwrap(ref.phi[both])))
    e1, e2 = err(0.01), err(0.0025)
    assert e2 < e1 / 2.5, (e1, e2)
