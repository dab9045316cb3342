"""Pins of the oracle's solid ring and its redshift (paper Sec. 3.3.2 exit
objects, Sec. 3.3.3 "Redshift"): the ring's circular orbit has the Kerr
Keplerian angular velocity, the redshift of zero-angular-momentum photons
has its closed form for Schwarzschild and Kerr, and in flat space the rays
that stop on the ring are those whose straight lines cross it."""
import math

import numpy as np
import pytest

import oracle

M = 0.5


@pytest.mark.parametrize("a", [0.0, 0.24, 0.45, -0.3])
def test_ring_orbit_is_keplerian(a):
    """dphi/dt = sqrt(M) / (r^{3/2} + a sqrt(M)) (Bardeen, Press and
    Teukolsky), the orbit turning toward +phi."""
    for r in (3.0, 4.5, 6.0, 9.0, 12.0):
        st, sp, om = oracle.disk_orbit(M, a, 0.0, r)
        want = math.sqrt(M) / (r ** 1.5 + a * math.sqrt(M))
        assert om == pytest.approx(want, rel=5e-6)
        # timelike, future-directed four-velocity with the Kerr u^t
        ut = (r ** 1.5 + a * math.sqrt(M)) / (
            r ** 0.75 * math.sqrt(r ** 1.5 - 3 * M * r ** 0.5 + 2 * a * math.sqrt(M)))
        assert st == pytest.approx(ut, rel=5e-6)


@pytest.mark.parametrize("a", [0.0, 0.3])
def test_redshift_of_zero_angular_momentum_photons(a):
    """A photon with p_phi = 0 scaled to dt/dtau = -1 at a camera (r0,
    theta0) has p_t = -1/g^tt(camera); the ring's matter sees it at
    frequency p_t u^t and the camera's observer at sqrt(-1/g^tt), so
    z = sqrt(-1/g^tt(camera)) u^t (Schwarzschild: sqrt(1 - 2M/r0) /
    sqrt(1 - 3M/r))."""
    r0, th0 = 20.0, math.radians(70.0)
    g0 = oracle.inverse_metric(M, a, 0.0, r0, th0)
    r = np.array([3.0, 4.0, 6.0, 10.0, 15.0])
    pt = np.full(r.size, -1.0 / g0[0])
    z = oracle.redshift(M, a, 0.0, r0, th0, r, np.full(r.size, math.pi / 2), pt,
                        np.zeros(r.size), np.full(r.size, 4, np.int8))
    ut = (r ** 1.5 + a * math.sqrt(M)) / (
        r ** 0.75 * np.sqrt(r ** 1.5 - 3 * M * r ** 0.5 + 2 * a * math.sqrt(M)))
    np.testing.assert_allclose(z, math.sqrt(-1.0 / g0[0]) * ut, rtol=5e-6)
    if a == 0.0:
        np.testing.assert_allclose(z, math.sqrt(1 - 2 * M / r0) / np.sqrt(1 - 3 * M / r),
                                   rtol=5e-6)


def test_redshift_is_nan_off_the_ring_and_inside_the_photon_orbit():
    z = oracle.redshift(M, 0.0, 0.0, 20.0, 1.2, np.array([6.0, 6.0, 1.4]),
                        np.full(3, math.pi / 2), np.full(3, -0.9), np.zeros(3),
                        np.array([1, 4, 4], np.int8))
    assert np.isnan(z[0]) and np.isfinite(z[1]) and np.isnan(z[2])      # r < 3M: no orbit


def test_flat_space_rays_stop_where_their_lines_cross_the_ring():
    W, H, r0, th0, fov = 40, 30, 20.0, math.radians(60.0), math.radians(50.0)
    r_in, r_out, dth = 4.0, 8.0, 0.01
    res = oracle.trace_frame(0.0, 0.0, 0.0, r0, th0, 0.0, fov, W, H, dt=0.01,
                             max_steps=20000, disk=(r_in, r_out, dth))
    # the camera's pixel directions in Cartesian coordinates (phi0 = 0)
    tan_h = math.tan(fov / 2)
    tan_v = tan_h * H / W
    i, j = np.meshgrid(np.arange(W), np.arange(H))
    x = (2 * i + 1 - W) / W * tan_h
    y = (H - 2 * j - 1) / H * tan_v
    n = np.stack([-np.ones_like(x), -y, x], -1) / np.sqrt(1 + x * x + y * y)[..., None]
    st, ct = math.sin(th0), math.cos(th0)
    e_r, e_t, e_p = np.array([st, 0, ct]), np.array([ct, 0, -st]), np.array([0, 1.0, 0])
    d = n[..., :1] * e_r + n[..., 1:2] * e_t + n[..., 2:] * e_p
    x0 = r0 * e_r
    s = -x0[2] / d[..., 2]
    hit = x0 + s[..., None] * d
    rho = np.hypot(hit[..., 0], hit[..., 1]).ravel()
    crosses = (s > 0).ravel()
    inside = crosses & (rho > r_in + 0.3) & (rho < r_out - 0.3)
    outside = ~crosses | (rho < r_in - 0.3) | (rho > r_out + 0.3)
    assert inside.sum() > 50 and outside.sum() > 50
    assert np.all(res.flag[inside] == 4)
    assert np.all(res.flag[outside] != 4)
    # and they stop inside the ring's volume
    on = res.flag == 4
    assert np.all((res.r[on] >= r_in) & (res.r[on] <= r_out))
    assert np.all(np.abs(res.theta[on] - math.pi / 2) <= dth)
