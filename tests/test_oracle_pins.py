"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these retype the oracle's own formulas: each compares it with an
independent closed form (textbook covariant metric, Schwarzschild and
Reissner-Nordstrom critical impact parameters, the Schwarzschild deflection
integral, Bardeen's critical curve, the Kerr-Newman radial potential), an
invariant (H, Carter constant), a symmetry, flat space, or a convergence
order.  Tolerances are stated next to each check with what sets them.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from tests import physics

FOV75 = math.radians(75.0)


@pytest.fixture(scope="module")
def kerr64():
    """Small Kerr frame: M=0.5, a=0.24, camera r0=20 on the equator, 64x64, 75 deg,
    dt=0.01, eps=1e-8, 20000 steps, horizon at |dt/dtau| > 1e4, escape r > 30."""
    return oracle.trace_frame(0.5, 0.24, 0.0, 20.0, math.pi / 2, 0.0, FOV75, 64, 64,
                              dt=0.01, max_steps=20000, want_p0=True)


# --------------------------------------------------------------------------- trig
def test_sincos_definition_is_within_1p5_ulp():
    rng = np.random.default_rng(1)
    x = np.concatenate([np.linspace(-7.0, 7.0, 4001), rng.uniform(0.0, math.pi, 4000),
                        [math.pi / 2, math.pi, 1e-300]])
    s, c = oracle.sincos(x)
    mp.mp.prec = 120
    worst = 0.0
    for xi, si, ci in zip(x, s, c):
        for got, ref in ((si, mp.sin(mp.mpf(xi))), (ci, mp.cos(mp.mpf(xi)))):
            if ref == 0:
                continue
            ulp = np.spacing(abs(float(ref)))
            worst = max(worst, float(abs(mp.mpf(got) - ref)) / ulp)
    assert worst <= 1.5
    s0, c0 = oracle.sincos([0.0])
    assert s0[0] == 0.0 and c0[0] == 1.0


def test_newton_reciprocal_is_correctly_rounded_for_small_displacements():
    """The displaced points' reciprocals (two Newton steps from the base
    point's exact reciprocal) are correctly rounded for relative
    displacements up to 3e-5 and within 1.5 ulp up to 1e-4, the largest the
    forward differences produce (at the horizon cutoff)."""
    rng = np.random.default_rng(3)
    x0 = 10.0 ** rng.uniform(-6, 6, 4000)
    rel = np.concatenate([rng.uniform(-1e-4, 1e-4, 2000), 10.0 ** rng.uniform(-12, -4, 2000)])
    x = x0 * (1.0 + rel)
    y0 = 1.0 / x0
    got = oracle.recip_newton(x, y0)
    mp.mp.prec = 120
    err = np.array([float(abs(mp.mpf(g) - 1 / mp.mpf(xi))) / np.spacing(float(1 / mp.mpf(xi)))
                    for g, xi in zip(got, x)])
    assert err[np.abs(rel) <= 3e-5].max() <= 0.5 + 1e-9
    assert err.max() <= 1.5
    # a large displacement is not what the refinement is for: two steps leave e0^4
    far = oracle.recip_newton(np.array([1.1]), np.array([1.0]))
    assert abs(far[0] - 1 / 1.1) > 1e-5


def test_three_newton_steps_reach_rounding_from_two_to_the_minus_8():
    """The theta-displaced point's 1/(rho^2 Delta sin^2), three Newton steps
    from the base point's reciprocal: within 1.5 ulp of 1/x (against 120-bit
    arithmetic) for starting residuals up to 2^-8, the largest the kernels
    refine from; two steps from 2^-8 leave ~2^-32, far from rounding."""
    rng = np.random.default_rng(5)
    x0 = 10.0 ** rng.uniform(-6, 6, 3000)
    rel = np.concatenate([rng.uniform(-2.0 ** -8, 2.0 ** -8, 2000),
                          np.array([2.0 ** -8, -(2.0 ** -8)] * 50),
                          10.0 ** rng.uniform(-14, -4, 900)])
    x = x0 * (1.0 + rel)
    y0 = 1.0 / x0
    got = oracle.recip_newton(x, y0, steps=3)
    mp.mp.prec = 120
    err = np.array([float(abs(mp.mpf(g) - 1 / mp.mpf(xi))) / np.spacing(float(1 / mp.mpf(xi)))
                    for g, xi in zip(got, x)])
    assert err.max() <= 1.5
    assert np.mean(err <= 0.5 + 1e-9) > 0.9
    two = oracle.recip_newton(np.array([1.0 + 2.0 ** -8]), np.array([1.0]))
    assert abs(two[0] - 1 / (1.0 + 2.0 ** -8)) > 1e-11


# --------------------------------------------------------------------------- metric
@pytest.mark.parametrize("M,a,Q", [(0.5, 0.24, 0.0), (0.5, 0.24, 0.3), (0.5, 0.49, 0.0),
                                   (0.0, 0.3, 0.0), (0.5, 0.0, 0.0)])
def test_inverse_metric_inverts_textbook_metric(M, a, Q):
    for r in (0.9, 1.7, 5.0, 20.0, 47.0):
        for th in (0.3, 1.0, math.pi / 2 - 0.1, 2.5):
            if M > 0 and r <= physics.horizon_radius(M, a, Q) * 1.05:
                continue
            g5 = oracle.inverse_metric(M, a, Q, r, th)
            gi = np.zeros((4, 4))
            gi[0, 0], gi[0, 3], gi[3, 0] = g5[0], g5[1], g5[1]
            gi[1, 1], gi[2, 2], gi[3, 3] = g5[2], g5[3], g5[4]
            prod = gi @ physics.covariant_metric(M, a, Q, r, th)
            assert np.abs(prod - np.eye(4)).max() < 1e-12


def test_flat_metric_is_exact():
    r, th = 7.0, 1.1
    g = oracle.inverse_metric(0.0, 0.0, 0.0, r, th)
    s, _ = oracle.sincos([th])
    assert g[0] == -1.0 and g[1] == 0.0 and g[2] == 1.0
    assert g[3] == pytest.approx(1.0 / (r * r), rel=4e-16)         # Delta / (rho^2 Delta)
    assert g[4] == pytest.approx(1.0 / (r * r * s[0] ** 2), rel=6e-16)


# --------------------------------------------------------------------------- camera
@pytest.mark.parametrize("M,a,Q,th0", [(0.5, 0.24, 0.0, math.pi / 2),
                                        (0.5, 0.24, 0.3, math.radians(80)),
                                        (0.5, 0.49, 0.0, math.radians(60))])
def test_camera_rays_are_null_and_past_directed(M, a, Q, th0):
    W, H = 9, 7
    init = oracle.camera(M, a, Q, 20.0, th0, 0.0, FOV75, W, H)
    gi = physics.inverse_metric_numeric(M, a, Q, 20.0, th0)
    for q_p in init:
        p = q_p[4:]
        v = gi @ p
        assert v[0] == pytest.approx(-1.0, abs=4e-15)          # dt/dtau = -1
        terms = np.abs(np.outer(p, p) * gi).sum()
        assert abs(0.5 * p @ gi @ p) / terms < 1e-15           # H = 0
        assert v[1] < 0                                        # looks inward
    centre = init[(H // 2) * W + W // 2, 4:]
    assert centre[2] == 0.0 and centre[3] == 0.0               # central ray is radial
    right = init[(H // 2) * W + W - 1, 4:]
    top = init[W // 2, 4:]
    assert right[3] > 0 and right[2] == 0.0                    # image right = +phi
    assert top[2] < 0 and top[3] == 0.0                        # image up = -theta


# --------------------------------------------------------------------------- flat space
def _flat_deviation(a, eps, form="listing"):
    th0, ph0 = math.radians(70), 0.3
    W, H = 16, 12
    res = oracle.trace_frame(0.0, a, 0.0, 20.0, th0, ph0, FOV75, W, H, dt=0.01, eps=eps,
                             form=form)
    init = oracle.camera(0.0, a, 0.0, 20.0, th0, ph0, FOV75, W, H)
    gi = physics.inverse_metric_numeric(0.0, a, 0.0, 20.0, th0)
    v = init[:, 4:] @ gi.T
    x0 = physics.bl_to_cartesian(a, 20.0, th0, ph0)
    d = physics.bl_velocity_to_cartesian(a, 20.0, th0, ph0, v[:, 1], v[:, 2], v[:, 3])
    speed = np.linalg.norm(d, axis=1)
    dhat = d / speed[:, None]
    rel = physics.bl_to_cartesian(a, res.r, res.theta, res.phi) - x0
    along = (rel * dhat).sum(1)
    angle = np.linalg.norm(np.cross(rel, dhat), axis=1) / along
    return res, speed, along, angle


@pytest.mark.parametrize("form", ["listing", "twin"])
@pytest.mark.parametrize("a", [0.0, 0.3])
def test_flat_space_rays_are_straight_lines(a, form):
    """M = 0: Boyer-Lindquist coordinates are flat (oblate spheroidal for a != 0),
    so every ray is a straight line travelled at unit speed in coordinate time.
    The forward difference's O(eps) truncation (about 3e-7 rad here) sets the
    1e-6 rad gate.  Both forms: the twin's t and phi come from its own RK4
    sums of g^tt, g^tphi and g^phph."""
    res, speed, along, angle = _flat_deviation(a, 1e-8, form)
    assert np.all(res.flag == oracle.FLAG_ESCAPE)
    np.testing.assert_allclose(speed, 1.0, atol=1e-14)
    assert angle.max() < 1e-6
    np.testing.assert_allclose(along, -res.t, rtol=1e-7)       # |dx| = |dt|


def test_forward_difference_is_first_order():
    """The flat-space deviation is the one-sided difference's truncation error,
    linear in eps: ten times the step gives about ten times the error."""
    e5 = _flat_deviation(0.3, 1e-5)[3].max()
    e6 = _flat_deviation(0.3, 1e-6)[3].max()
    assert 8.0 < e5 / e6 < 12.0


# --------------------------------------------------------------------------- Schwarzschild
def _critical_b(M, Q, lo, hi, rounds=4):
    for _ in range(rounds):
        bs = np.linspace(lo, hi, 65)
        init = np.array([physics.equatorial_state(M, Q, 20.0, b) for b in bs])
        res = oracle.trace_rays(M, 0.0, Q, init, dt=0.01, max_steps=200000)
        assert np.all((res.flag == 1) | (res.flag == 2))
        k = int(np.nonzero(res.flag == oracle.FLAG_ESCAPE)[0][0])
        assert k > 0 and np.all(res.flag[:k] == oracle.FLAG_HORIZON)
        lo, hi = bs[k - 1], bs[k]
    return 0.5 * (lo + hi)


def test_schwarzschild_critical_impact_parameter():
    """Equatorial rays with b < 3 sqrt(3) M fall in, b > 3 sqrt(3) M escape."""
    M = 0.5
    b = _critical_b(M, 0.0, 2.4, 2.8)
    assert abs(b - 3 * math.sqrt(3) * M) / (3 * math.sqrt(3) * M) < 1e-6


def test_reissner_nordstrom_critical_impact_parameter():
    """The charge term: b_c = r_ph / sqrt(1 - 2M/r_ph + Q^2/r_ph^2) with
    r_ph = (3M + sqrt(9M^2 - 8Q^2))/2."""
    M, Q = 0.5, 0.3
    _, bc = physics.rn_critical_b(M, Q)
    b = _critical_b(M, Q, 2.0, 2.8)
    assert abs(b - bc) / bc < 1e-6


@pytest.mark.parametrize("form", ["listing", "twin"])
@pytest.mark.parametrize("b", [3.0, 4.0, 6.0, 10.0])
def test_schwarzschild_deflection_and_travel_time(b, form):
    """End phi and t of an equatorial ray equal the deflection and time
    integrals taken to the oracle's own end radius.  Gate 4e-7 rad / 2e-6 in t:
    the forward-difference step fl(r+eps)-r exceeds eps by 8.3e-8 (relative)
    for 8 <= r < 64, which biases the centrifugal term at that level."""
    M = 0.5
    init = physics.equatorial_state(M, 0.0, 20.0, b)[None]
    res = oracle.trace_rays(M, 0.0, 0.0, init, dt=0.01, max_steps=200000, form=form)
    assert res.flag[0] == oracle.FLAG_ESCAPE
    phi, t = physics.schwarzschild_deflection(M, b, 20.0, res.r[0])
    assert abs(res.phi[0] - phi) < 4e-7
    assert abs(-res.t[0] - t) < 2e-6


def test_rk4_is_fourth_order():
    """Halving dt at steps where truncation dominates divides the deflection
    error by about 16 (a second-order slip would give 4)."""
    M, b = 0.5, 4.0
    init = physics.equatorial_state(M, 0.0, 20.0, b)[None]
    errs = []
    for dt in (0.8, 0.4):
        res = oracle.trace_rays(M, 0.0, 0.0, init, dt=dt, max_steps=10000)
        phi, _ = physics.schwarzschild_deflection(M, b, 20.0, res.r[0])
        errs.append(abs(res.phi[0] - phi))
    assert 11.0 < errs[0] / errs[1] < 22.0


# --------------------------------------------------------------------------- Kerr(-Newman)
@pytest.mark.parametrize("M,a,Q,th0,W", [(0.5, 0.24, 0.3, math.radians(80), 40),
                                          (0.5, 0.49, 0.0, math.radians(60), 40)])
def test_capture_matches_radial_potential(M, a, Q, th0, W):
    """A ray is captured exactly when the radial potential R(r) built from its
    conserved E, L and Carter constant stays positive on (r_+, r0]."""
    res = oracle.trace_frame(M, a, Q, 20.0, th0, 0.0, FOV75, W, W, dt=0.01, want_p0=True)
    _check_capture(M, a, Q, th0, res)


def test_capture_matches_radial_potential_kerr64(kerr64):
    _check_capture(0.5, 0.24, 0.0, math.pi / 2, kerr64)


def _check_capture(M, a, Q, th0, res):
    n_checked = n_captured = 0
    for k in range(res.flag.size):
        pred = physics.captured(M, a, Q, 20.0, res.p0[k], th0)
        if pred is None:
            continue
        n_checked += 1
        n_captured += pred
        assert res.flag[k] == (oracle.FLAG_HORIZON if pred else oracle.FLAG_ESCAPE), k
    assert n_checked >= 0.98 * res.flag.size and n_captured > 0


@pytest.mark.parametrize("a", [0.24, 0.49])
def test_bardeen_critical_curve(a):
    """Rays whose (xi, eta) sit just outside Bardeen's critical curve escape,
    just inside fall in (equatorial camera, so eta = p_theta^2 / p_t^2)."""
    M = 0.5
    r1, r2 = physics.photon_orbit_radii(M, a)
    gi = physics.inverse_metric_numeric(M, a, 0.0, 20.0, math.pi / 2)
    init, want = [], []
    for rp in np.linspace(r1, r2, 7)[1:-1]:
        xi, eta = physics.bardeen_curve(M, a, rp)
        for sign in (+1, -1):
            e = eta * (1 + sign * 1e-6)
            pt, pph, pth = 1.0, -xi, math.sqrt(e)
            rest = gi[0, 0] * pt * pt + 2 * gi[0, 3] * pt * pph + gi[2, 2] * pth ** 2 \
                + gi[3, 3] * pph ** 2
            pr = -math.sqrt(-rest / gi[1, 1])
            init.append([0.0, 20.0, math.pi / 2, 0.0, pt, pr, pth, pph])
            want.append(oracle.FLAG_ESCAPE if sign > 0 else oracle.FLAG_HORIZON)
    res = oracle.trace_rays(M, a, 0.0, np.array(init), dt=0.01, max_steps=100000)
    np.testing.assert_array_equal(res.flag, want)


def test_conserved_quantities(kerr64):
    """p_t, p_phi are constant by construction; H stays ~0 and the Carter
    constant is kept to the forward-difference noise (random walk of ~1e-8
    per unit force over thousands of steps)."""
    M, a = 0.5, 0.24
    res = kerr64
    hs, cs = [], []
    for k in range(0, res.flag.size, 3):
        if res.flag[k] != oracle.FLAG_ESCAPE:
            continue
        p0 = res.p0[k]
        pe = np.array([p0[0], res.pr[k], res.ptheta[k], p0[3]])
        gi = physics.inverse_metric_numeric(M, a, 0.0, res.r[k], res.theta[k])
        hs.append(abs(0.5 * pe @ gi @ pe) / np.abs(np.outer(pe, pe) * gi).sum())
        c0 = physics.carter(a, math.pi / 2, p0)
        c1 = physics.carter(a, res.theta[k], pe)
        cs.append(abs(c1 - c0) / (abs(c0) + a * a * p0[0] ** 2))
    assert max(hs) < 1e-7
    assert max(cs) < 1e-6 and np.median(cs) < 1e-7


# --------------------------------------------------------------------------- symmetries
def test_spin_reversal_mirrors_phi_bit_exactly():
    """a -> -a with the image mirrored left-right maps phi_end -> -phi_end and
    leaves everything else unchanged, bit for bit (only signs flip)."""
    W, H = 24, 16
    kw = dict(dt=0.01, max_steps=20000)
    A = oracle.trace_frame(0.5, 0.24, 0.3, 20.0, math.radians(80), 0.0, FOV75, W, H, **kw)
    B = oracle.trace_frame(0.5, -0.24, 0.3, 20.0, math.radians(80), 0.0, FOV75, W, H, **kw)
    mirror = lambda x: x.reshape(H, W)[:, ::-1].ravel()  # noqa: E731
    np.testing.assert_array_equal(A.phi, -mirror(B.phi))
    for f in ("t", "r", "theta", "pr", "ptheta", "flag", "steps"):
        np.testing.assert_array_equal(getattr(A, f), mirror(getattr(B, f)))


def test_equatorial_mirror(kerr64):
    """Equatorial camera: flipping the image top-bottom maps theta -> pi - theta.
    The one-sided difference breaks this reflection at O(eps): its truncation
    term eps/2 d^2g keeps its sign under theta -> pi - theta while the
    derivative flips, the same ~1e-7 rad level as the flat-space check."""
    W = H = 64
    A = kerr64
    flip = lambda x: x.reshape(H, W)[::-1, :].ravel()  # noqa: E731
    np.testing.assert_array_equal(A.flag, flip(A.flag))
    esc = A.flag == oracle.FLAG_ESCAPE
    # great-circle angle between the end direction and the mirrored one (raw
    # phi is ill-conditioned for rays that pass near the axis)
    u = physics.sky_direction(A.theta, A.phi)
    v = physics.sky_direction(flip(A.theta), flip(A.phi)) * np.array([1.0, 1.0, -1.0])
    ang = physics.angle_between(u, v)[esc]
    assert np.median(ang) < 1e-7
    # rays that wrap over the pole: the theta-difference of g^phph ~ 1/sin^2
    # has truncation error ~ eps/sin^4, the axis weakness of these coordinates
    assert ang.max() < 5e-6


# --------------------------------------------------------------------------- termination
def test_termination_flags_and_counts(kerr64):
    res = kerr64
    esc = res.flag == oracle.FLAG_ESCAPE
    hor = res.flag == oracle.FLAG_HORIZON
    assert esc.sum() + hor.sum() == res.flag.size
    assert np.all(res.r[esc] > 30.0)
    rp = physics.horizon_radius(0.5, 0.24, 0.0)
    assert np.all(res.r[hor] < 30.0) and np.all(res.r[hor] < rp * 1.01)
    assert np.all(res.t < 0)                                  # traced backward in time
    assert np.all((res.steps > 0) & (res.steps < 20000))

    short = oracle.trace_frame(0.5, 0.24, 0.0, 20.0, math.pi / 2, 0.0, FOV75, 8, 8,
                               dt=0.01, max_steps=100)
    assert np.all(short.flag == oracle.FLAG_TIMEOUT) and np.all(short.steps == 100)

    init = oracle.camera(0.5, 0.24, 0.0, 20.0, math.pi / 2, 0.0, FOV75, 2, 1)
    init[0, 5] = np.nan
    bad = oracle.trace_rays(0.5, 0.24, 0.0, init, dt=0.01, max_steps=50)
    assert bad.flag[0] == oracle.FLAG_INVALID and bad.steps[0] == 0


def test_escape_factor_is_relative_to_start_radius():
    res = oracle.trace_frame(0.5, 0.24, 0.0, 12.0, math.pi / 2, 0.0, FOV75, 8, 8,
                             dt=0.01, escape_factor=2.0)
    esc = res.flag == oracle.FLAG_ESCAPE
    assert esc.any() and np.all(res.r[esc] > 24.0) and np.all(res.r[esc] < 24.1)


# --------------------------------------------------------------------------- trig choice
def test_library_trig_changes_only_the_noise_floor(kerr64):
    """sin/cos from the C library instead of the series definition moves end
    angles only at the forward-difference noise floor; flags and steps agree."""
    oracle.set_trig_mode(1)
    try:
        lib = oracle.trace_frame(0.5, 0.24, 0.0, 20.0, math.pi / 2, 0.0, FOV75, 64, 64,
                                 dt=0.01, max_steps=20000, pixels=np.arange(0, 4096, 4))
    finally:
        oracle.set_trig_mode(0)
    sel = np.arange(0, 4096, 4)
    np.testing.assert_array_equal(lib.flag, kerr64.flag[sel])
    np.testing.assert_array_equal(lib.steps, kerr64.steps[sel])
    esc = lib.flag == oracle.FLAG_ESCAPE
    d = np.maximum(np.abs(lib.theta - kerr64.theta[sel]), np.abs(lib.phi - kerr64.phi[sel]))
    assert d[esc].max() < 2e-7


def test_reissner_nordstrom_sweep_reference():
    """The sweep integral the surrogate's baseline is checked against: equal to
    the Schwarzschild deflection for Q = 0, to the straight line in flat space,
    and to equatorial Reissner-Nordstrom rays traced by the oracle."""
    assert abs(physics.rn_sweep(0.5, 0.0, 5.0, 20.0, 30.0) -
               physics.schwarzschild_deflection(0.5, 5.0, 20.0, 30.0)[0]) < 1e-12
    b = 7.0
    assert abs(physics.rn_sweep(0.0, 0.0, b, 20.0, 30.0) -
               (math.acos(b / 20.0) + math.acos(b / 30.0))) < 1e-12
    assert physics.rn_sweep(0.5, 0.3, 1.0, 20.0, 30.0) is None          # captured
    # oracle: one equatorial row of an RN frame, a = 0, camera on the equator
    M, Q, r0, W = 0.5, 0.3, 20.0, 41
    fov = math.radians(60.0)
    pix = np.arange(W // 2 + 3, W)                                      # rays with x > 0
    res = oracle.trace_frame(M, 0.0, Q, r0, math.pi / 2, 0.0, fov, W, 1, dt=0.002, eps=1e-8,
                             horizon_norm=1e4, escape_factor=1.5, max_steps=100000, pixels=pix,
                             want_p0=True)
    f = 1 - 2 * M / r0 + Q * Q / r0 ** 2
    x = ((2 * pix + 1 - W) / W) * math.tan(fov / 2)
    b = r0 * (x / np.sqrt(1 + x * x)) / math.sqrt(f)
    st = {"r": res.r, "theta": res.theta, "phi": res.phi, "p_t": res.p0[:, 0], "p_r": res.pr,
          "p_theta": res.ptheta, "p_phi": res.p0[:, 3]}
    esc = res.flag == oracle.FLAG_ESCAPE
    pcov = np.stack([st["p_t"], st["p_r"], st["p_theta"], st["p_phi"]], axis=1)[esc]
    th, ph = physics.escape_crossing(M, 0.0, Q, 1.5 * r0, st["r"][esc], st["theta"][esc],
                                     st["phi"][esc], pcov)
    assert esc.sum() >= 10 and np.allclose(th, math.pi / 2, atol=1e-12)
    want = np.array([physics.rn_sweep(M, Q, bb, r0, 1.5 * r0) for bb in b[esc]])
    assert np.abs(ph - want).max() < 1e-6
