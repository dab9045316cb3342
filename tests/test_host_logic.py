"""Host-side logic without a GPU: seeded workloads, the error metrics the
bench and tests report, and the surrogate's online error bookkeeping."""
import math

import numpy as np

import paper_2310_15183_amd as g
from paper_2310_15183_amd import surrogate as S
from paper_2310_15183_amd.evaluate import angle_between, sky_at_escape, sky_direction
from paper_2310_15183_amd.workloads import SIDES, batch_instances


def test_batch_instances_follow_the_stated_ranges_and_seed():
    a1 = batch_instances(256)
    assert a1 == batch_instances(256)                    # seeded
    assert a1 != batch_instances(256, seed=1)
    for I in a1:
        assert I.M == 0.5 and 0.0 <= I.a <= 0.49
        assert 0.0 <= I.Q <= 0.95 * math.sqrt(I.M ** 2 - I.a ** 2)
        assert 10.0 <= I.r0 <= 50.0
        assert math.radians(5) <= I.theta0 <= math.radians(90)
        assert math.radians(30) <= I.fov <= math.radians(90)
        assert I.width == I.height and I.width in SIDES
    # every side occurs and the expected total is near 256 x mean side^2
    assert {I.width for I in a1} == set(SIDES)
    n = sum(I.width * I.height for I in a1)
    assert 0.8 * 256 * np.mean(np.square(SIDES)) < n < 1.2 * 256 * np.mean(np.square(SIDES))
    # scale shrinks the sides only
    small = batch_instances(256, scale=8)
    assert [(I.a, I.Q, I.r0) for I in small] == [(I.a, I.Q, I.r0) for I in a1]
    assert all(s.width == I.width // 8 for s, I in zip(small, a1))


def test_angle_between_is_accurate_for_tiny_and_large_angles():
    rng = np.random.default_rng(0)
    u = rng.normal(size=(100, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    axis = np.cross(u, rng.normal(size=(100, 3)))
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    for ang in (1e-9, 1e-4, 0.3, 2.5, math.pi - 1e-3):
        # rotate u about axis (perpendicular to u) by ang
        v = u * math.cos(ang) + np.cross(axis, u) * math.sin(ang)
        np.testing.assert_allclose(angle_between(u, v), ang, rtol=1e-6, atol=1e-15)


def _state_at_sphere(n, r_esc, rng):
    th = rng.uniform(0.2, math.pi - 0.2, n)
    ph = rng.uniform(-math.pi, math.pi, n)
    return {"r": np.full(n, r_esc), "theta": th, "phi": ph, "p_t": np.full(n, -1.0),
            "p_r": np.full(n, 0.9), "p_theta": rng.normal(size=n), "p_phi": rng.normal(size=n)}


def test_sky_at_escape_is_identity_on_the_sphere_and_moves_back_along_the_velocity():
    rng = np.random.default_rng(1)
    M, a, Q, r_esc = 0.5, 0.3, 0.2, 30.0
    st = _state_at_sphere(50, r_esc, rng)
    th, ph = sky_at_escape(M, a, Q, r_esc, st)
    np.testing.assert_array_equal(th, st["theta"])
    np.testing.assert_array_equal(ph, st["phi"])
    # a state a little beyond the sphere maps back to within O(step^2) of it
    dlam = 1e-3
    s = np.sin(st["theta"]) ** 2
    rho2 = r_esc ** 2 + a * a * np.cos(st["theta"]) ** 2
    Delta = r_esc ** 2 - 2 * M * r_esc + a * a + Q * Q
    dr = Delta / rho2 * st["p_r"]
    dth = st["p_theta"] / rho2
    dph = -a * (2 * M * r_esc - Q * Q) / (rho2 * Delta) * st["p_t"] + \
        (Delta - a * a * s) / (rho2 * Delta * s) * st["p_phi"]
    beyond = dict(st, r=st["r"] + dr * dlam, theta=st["theta"] + dth * dlam,
                  phi=st["phi"] + dph * dlam)
    th2, ph2 = sky_at_escape(M, a, Q, r_esc, beyond)
    assert np.abs(th2 - st["theta"]).max() < 1e-6 and np.abs(ph2 - st["phi"]).max() < 1e-6


def test_frame_errors_counts_classes_and_measures_directions():
    rng = np.random.default_rng(2)
    n, r_esc = 400, 30.0
    ref = _state_at_sphere(n, r_esc, rng)
    ref["flag"] = np.where(rng.uniform(size=n) < 0.8, g.GR_FLAG_ESCAPE, g.GR_FLAG_HORIZON).astype(np.int8)
    u = sky_direction(ref["theta"], ref["phi"])
    # rotate every direction by a known angle about a perpendicular axis
    ang = 10.0 ** rng.uniform(-6, -2, n)
    axis = np.cross(u, rng.normal(size=(n, 3)))
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    direc = (u * np.cos(ang)[:, None] + np.cross(axis, u) * np.sin(ang)[:, None]).astype(np.float32)
    flag = ref["flag"].copy()
    flag[:10] = np.where(flag[:10] == g.GR_FLAG_ESCAPE, g.GR_FLAG_HORIZON, g.GR_FLAG_ESCAPE)
    e = S.frame_errors(0.5, 0.3, 0.2, r_esc, ref, flag, direc)
    assert e["misclassified_frac"] == 10 / n
    both = (ref["flag"] == g.GR_FLAG_ESCAPE) & (flag == g.GR_FLAG_ESCAPE)
    assert e["n_escaped_both"] == both.sum()
    want = np.quantile(ang[both], [0.5, 0.99])
    # binary32 storage of the unit vectors adds ~1e-7 rad
    assert abs(e["angle_err_rad"]["median"] - want[0]) < 2e-7 + 1e-3 * want[0]
    assert abs(e["angle_err_rad"]["p99"] - want[1]) < 2e-7 + 1e-3 * want[1]


def test_online_errors_use_only_the_retraced_pixels():
    rng = np.random.default_rng(3)
    n = 1000
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    net_flag = np.full(n, g.GR_FLAG_ESCAPE, np.int8)
    flag = net_flag.copy()
    fb = np.zeros(n, np.int8)
    fb[:100] = 1
    flag[:5] = g.GR_FLAG_HORIZON                          # 5 re-traced pixels change class
    direc = d.copy()
    direc[5:100] = -d[5:100]                              # re-traced escaping ones point away
    o = S.online_errors(net_flag, d, flag, direc, fb)
    assert o["pixels"] == 100 and o["class_changed_frac"] == 0.05
    assert abs(o["angle_err_rad"]["median"] - math.pi) < 1e-6
    assert S.online_errors(net_flag, d, flag, direc, np.zeros(n, np.int8)) == {"pixels": 0}


def test_frame_errors_set_axis_grazing_rays_apart():
    """Rays with |L_z| / sqrt(Q + L_z^2) below 1e-3 pass within ~1e-3 rad of
    the polar axis; their errors are reported apart."""
    rng = np.random.default_rng(4)
    n, r_esc = 300, 30.0
    ref = _state_at_sphere(n, r_esc, rng)
    ref["flag"] = np.full(n, g.GR_FLAG_ESCAPE, np.int8)
    ref["p_theta"] = rng.choice([-1.0, 1.0], n) * rng.uniform(0.5, 2.0, n)   # physical: Q + L^2 > 0
    ref["p_phi"][:40] = 1e-7                       # grazing the axis
    u = sky_direction(ref["theta"], ref["phi"])
    direc = u.astype(np.float32).copy()
    direc[:40] = -direc[:40]                       # wildly wrong there only
    e = S.frame_errors(0.5, 0.3, 0.2, r_esc, ref, np.full(n, g.GR_FLAG_ESCAPE, np.int8), direc)
    assert e["axis_grazing_rays"] == 40
    assert abs(e["angle_err_rad"]["max"] - math.pi) < 1e-3
    assert e["angle_err_rad_off_axis"]["max"] < 1e-6
