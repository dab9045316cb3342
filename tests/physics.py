"""Independent physics used to pin the oracle (no code shared with it).

Everything here comes from textbook closed forms of the Kerr-Newman geometry,
evaluated with numpy (covariant metric, then a numerical 4x4 inverse) or with
mpmath quadrature, never from the oracle's own inverse-metric expressions.
"""
from __future__ import annotations

import math

import mpmath as mp
import numpy as np


def covariant_metric(M, a, Q, r, theta):
    """Kerr-Newman g_{mu nu} in Boyer-Lindquist coordinates (t, r, theta, phi),
    textbook line element:
      ds^2 = -(1 - (2Mr - Q^2)/rho^2) dt^2 - 2 a sin^2 (2Mr - Q^2)/rho^2 dt dphi
             + rho^2/Delta dr^2 + rho^2 dtheta^2
             + sin^2 ((r^2+a^2)^2 - a^2 Delta sin^2)/rho^2 dphi^2."""
    s2, c2 = math.sin(theta) ** 2, math.cos(theta) ** 2
    rho2 = r * r + a * a * c2
    Delta = r * r - 2 * M * r + a * a + Q * Q
    f = 2 * M * r - Q * Q
    g = np.zeros((4, 4))
    g[0, 0] = -(1 - f / rho2)
    g[0, 3] = g[3, 0] = -a * s2 * f / rho2
    g[1, 1] = rho2 / Delta
    g[2, 2] = rho2
    g[3, 3] = s2 * ((r * r + a * a) ** 2 - a * a * Delta * s2) / rho2
    return g


def inverse_metric_numeric(M, a, Q, r, theta):
    """g^{mu nu} as the numerical inverse of the covariant metric."""
    return np.linalg.inv(covariant_metric(M, a, Q, r, theta))


def hamiltonian(M, a, Q, r, theta, p):
    gi = inverse_metric_numeric(M, a, Q, r, theta)
    p = np.asarray(p, float)
    return 0.5 * p @ gi @ p


def carter(a, theta, p):
    """Carter constant Q = p_theta^2 + cos^2(theta) (p_phi^2/sin^2 - a^2 p_t^2)."""
    pt, _, pth, pph = p
    s2, c2 = math.sin(theta) ** 2, math.cos(theta) ** 2
    return pth * pth + c2 * (pph * pph / s2 - a * a * pt * pt)


def horizon_radius(M, a, Q):
    return M + math.sqrt(M * M - a * a - Q * Q)


def radial_potential_coeffs(M, a, Q, E, L, K):
    """R(r) = ((r^2+a^2)E - aL)^2 - Delta ((L - aE)^2 + K), as polynomial
    coefficients in r (highest first); Delta = r^2 - 2Mr + a^2 + Q^2."""
    A = np.polynomial.polynomial
    first = A.polypow([a * a * E - a * L, 0.0, E], 2)          # ((r^2+a^2)E - aL)^2
    Delta = [a * a + Q * Q, -2 * M, 1.0]
    second = A.polymul(Delta, [(L - a * E) ** 2 + K])
    c = A.polysub(first, second)
    return c[::-1]


def captured(M, a, Q, r0, p, theta0, margin=1e-6):
    """Classify an ingoing photon starting at r0 with covector p (either time
    orientation): True if it reaches the horizon, False if it meets a turning
    point and escapes, None if the radial potential's interior minimum is
    within margin (relative to E^2 r^4) of zero (near-critical ray).
    R(r0) >= 0 and R(r_+) >= 0 always hold, so the ray is captured exactly
    when every interior minimum of R on (r_+, r0) is positive."""
    pt, _, _, pph = p
    E, L = -pt, pph
    K = carter(a, theta0, p)
    coeffs = radial_potential_coeffs(M, a, Q, E, L, K)
    rp = horizon_radius(M, a, Q)
    crit = np.roots(np.polyder(coeffs))
    crit = crit[np.abs(crit.imag) < 1e-9].real
    crit = crit[(crit > rp) & (crit < r0)]
    captured_ = True
    for rc in crit:
        val = np.polyval(coeffs, rc)
        if abs(val) < margin * E * E * rc ** 4:
            return None
        if val < 0:
            captured_ = False
    return captured_


def bardeen_curve(M, a, rp):
    """Critical impact parameters (xi, eta) of the spherical photon orbit at
    radius rp (Bardeen 1973; Q = 0)."""
    xi = (rp * rp * (3 * M - rp) - a * a * (rp + M)) / (a * (rp - M))
    eta = rp ** 3 * (4 * a * a * M - rp * (rp - 3 * M) ** 2) / (a * a * (rp - M) ** 2)
    return xi, eta


def photon_orbit_radii(M, a):
    """Prograde and retrograde equatorial circular photon orbit radii (Kerr)."""
    r1 = 2 * M * (1 + math.cos(2.0 / 3.0 * math.acos(-abs(a) / M)))
    r2 = 2 * M * (1 + math.cos(2.0 / 3.0 * math.acos(abs(a) / M)))
    return min(r1, r2), max(r1, r2)


def rn_critical_b(M, Q):
    """Reissner-Nordstrom photon sphere radius and critical impact parameter."""
    rph = 0.5 * (3 * M + math.sqrt(9 * M * M - 8 * Q * Q))
    f = 1 - 2 * M / rph + Q * Q / (rph * rph)
    return rph, rph / math.sqrt(f)


def equatorial_state(M, Q, r0, b, ingoing=True):
    """Initial (q, p) of an equatorial Schwarzschild/Reissner-Nordstrom photon
    traced backward (dt/dtau < 0) with impact parameter b = p_phi/p_t, p_t = 1."""
    f = 1 - 2 * M / r0 + Q * Q / (r0 * r0)
    pt, pph = 1.0, b
    pr2 = (pt * pt / f - pph * pph / (r0 * r0)) / f
    pr = -math.sqrt(pr2) if ingoing else math.sqrt(pr2)
    return np.array([0.0, r0, math.pi / 2, 0.0, pt, pr, 0.0, pph])


def schwarzschild_deflection(M, b, r0, r_end, dps=30):
    """(Delta phi, Delta t) of an equatorial Schwarzschild photon with impact
    parameter b > 3 sqrt(3) M that starts inward at r0, passes periapsis and
    leaves to r_end: with u = 1/r, (du/dphi)^2 = F(u) = 1/b^2 - u^2 + 2 M u^3,
    dt/dphi = 1/(b u^2 (1 - 2 M u)).  The inverse-square-root endpoint at the
    turning point u_t is removed by u = u_t - s^2."""
    with mp.workdps(dps):
        M_, b_ = mp.mpf(M), mp.mpf(b)
        roots = mp.polyroots([2 * M_, -1, 0, 1 / b_ ** 2], maxsteps=200, extraprec=100)
        pos = sorted([mp.re(x) for x in roots if abs(mp.im(x)) < mp.mpf(10) ** (-dps // 2)
                      and mp.re(x) > 0])
        ut = pos[0]

        # F(u_t - s^2) = s^2 G(s) exactly, since F(u_t) = 0 (Taylor series of a cubic)
        g0 = 2 * ut - 6 * M_ * ut * ut
        g1 = 6 * M_ * ut - 1

        def G(s):
            return g0 + g1 * s * s - 2 * M_ * s ** 4

        def dphi(s):
            return 2 / mp.sqrt(G(s))

        def dt(s):
            u = ut - s * s
            return 2 / mp.sqrt(G(s)) / (b_ * u * u * (1 - 2 * M_ * u))

        s_in = mp.sqrt(ut - 1 / mp.mpf(r0))
        s_out = mp.sqrt(ut - 1 / mp.mpf(r_end))
        phi = mp.quad(dphi, [0, s_in]) + mp.quad(dphi, [0, s_out])
        t = mp.quad(dt, [0, s_in]) + mp.quad(dt, [0, s_out])
        return float(phi), float(t)


def rn_sweep(M, Q, b, r0, r_end, dps=30):
    """Azimuth swept by an equatorial Reissner-Nordstrom photon with impact
    parameter b that starts inward at r0, passes periapsis and leaves to r_end:
    (du/dphi)^2 = F(u) = 1/b^2 - u^2 + 2 M u^3 - Q^2 u^4 with u = 1/r; the
    turning point u_t is the smallest positive root of F, and u = u_t - s^2
    removes the endpoint singularity (mpmath quadrature).  None if the photon
    does not turn (captured)."""
    with mp.workdps(dps):
        M_, Q2, b_ = mp.mpf(M), mp.mpf(Q) ** 2, mp.mpf(b)
        coeffs = [-Q2, 2 * M_, -1, 0, 1 / b_ ** 2] if Q2 > 0 else [2 * M_, -1, 0, 1 / b_ ** 2]
        if M_ == 0 and Q2 == 0:
            pos = [1 / b_]
        else:
            roots = mp.polyroots(coeffs, maxsteps=400, extraprec=200)
            pos = sorted([mp.re(x) for x in roots if abs(mp.im(x)) < mp.mpf(10) ** (-dps // 2)
                          and mp.re(x) > 0])
        if not pos or pos[0] <= 1 / mp.mpf(r0):
            return None
        ut = pos[0]
        if M_ > 0:
            # a root beyond the photon sphere lies inside the hole: no turning point
            uph = (3 * M_ - mp.sqrt(9 * M_ ** 2 - 8 * Q2)) / (4 * Q2) if Q2 > 0 else 1 / (3 * M_)
            if ut >= uph:
                return None

        # F(u_t - s^2) = s^2 G(s) exactly (Taylor series of the quartic about its root)
        F1 = -2 * ut + 6 * M_ * ut ** 2 - 4 * Q2 * ut ** 3
        F2 = -2 + 12 * M_ * ut - 12 * Q2 * ut ** 2
        F3 = 12 * M_ - 24 * Q2 * ut
        F4 = -24 * Q2

        def dphi(s):
            z = s * s
            return 2 / mp.sqrt(-F1 + F2 / 2 * z - F3 / 6 * z * z + F4 / 24 * z ** 3)

        return float(mp.quad(dphi, [0, mp.sqrt(ut - 1 / mp.mpf(r0))]) +
                     mp.quad(dphi, [0, mp.sqrt(ut - 1 / mp.mpf(r_end))]))


def bl_to_cartesian(a, r, theta, phi):
    """Flat-space oblate-spheroidal map x = sqrt(r^2+a^2) sin cos, y = ..., z = r cos."""
    rr = np.sqrt(r * r + a * a)
    return np.stack([rr * np.sin(theta) * np.cos(phi), rr * np.sin(theta) * np.sin(phi),
                     r * np.cos(theta)], axis=-1)


def bl_velocity_to_cartesian(a, r, theta, phi, vr, vth, vph):
    """Jacobian of bl_to_cartesian applied to (dr, dtheta, dphi)."""
    rr = np.sqrt(r * r + a * a)
    st, ct, sp, cp = np.sin(theta), np.cos(theta), np.sin(phi), np.cos(phi)
    drr = r / rr
    dx = drr * st * cp * vr + rr * ct * cp * vth - rr * st * sp * vph
    dy = drr * st * sp * vr + rr * ct * sp * vth + rr * st * cp * vph
    dz = ct * vr - r * st * vth
    return np.stack([dx, dy, dz], axis=-1)


def sky_direction(theta, phi):
    """Unit vector (sin th cos ph, sin th sin ph, cos th)."""
    theta, phi = np.asarray(theta), np.asarray(phi)
    return np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi),
                     np.cos(theta)], axis=-1)


def angle_between(u, v):
    """Great-circle angle between unit vectors (accurate for tiny angles)."""
    return 2.0 * np.arctan2(np.linalg.norm(u - v, axis=-1), np.linalg.norm(u + v, axis=-1))


# ------------------------------------------------------------------ curvature
def covariant_from_inverse(g5):
    """4x4 covariant metric (t, r, theta, phi) from the five independent
    inverse components (g^tt, g^tphi, g^rr, g^thth, g^phph)."""
    gtt, gtp, grr, ghh, gpp = g5
    det = gtt * gpp - gtp * gtp
    g = np.zeros((4, 4))
    g[0, 0] = gpp / det
    g[0, 3] = g[3, 0] = -gtp / det
    g[3, 3] = gtt / det
    g[1, 1] = 1.0 / grr
    g[2, 2] = 1.0 / ghh
    return g


def _d(fn, x, h):
    """Fourth-order central difference of fn at x."""
    return (8.0 * (fn(x + h) - fn(x - h)) - (fn(x + 2 * h) - fn(x - 2 * h))) / (12.0 * h)


def ricci(inverse_fn, r, theta, h=2e-3):
    """Ricci tensor R_{mu nu} at (r, theta) of a stationary axisymmetric metric
    given by inverse_fn(r, theta) -> (g^tt, g^tphi, g^rr, g^thth, g^phph),
    from Christoffel symbols and their derivatives by nested fourth-order
    central differences in r and theta (the metric depends on no other
    coordinate).  R = d_l G^l_mn - d_n G^l_lm + G^l_ls G^s_mn - G^l_ns G^s_lm."""
    def gcov(rr, tt):
        return covariant_from_inverse(inverse_fn(rr, tt))

    def christoffel(rr, tt):
        g = gcov(rr, tt)
        gi = np.linalg.inv(g)
        dg = np.zeros((4, 4, 4))                   # dg[s, m, n] = d_s g_mn
        dg[1] = _d(lambda x: gcov(x, tt), rr, h)
        dg[2] = _d(lambda x: gcov(rr, x), tt, h)
        # G^l_mn = 1/2 g^ls (d_m g_sn + d_n g_sm - d_s g_mn)
        t1 = np.einsum('msn->smn', dg)             # d_m g_sn indexed [s, m, n]
        t2 = np.einsum('nsm->smn', dg)             # d_n g_sm
        return 0.5 * np.einsum('ls,smn->lmn', gi, t1 + t2 - dg)

    G = christoffel(r, theta)
    dG = np.zeros((4, 4, 4, 4))                    # dG[s, l, m, n] = d_s G^l_mn
    dG[1] = _d(lambda x: christoffel(x, theta), r, h)
    dG[2] = _d(lambda x: christoffel(r, x), theta, h)
    R = (np.einsum('llmn->mn', dG) - np.einsum('nllm->mn', dG)
         + np.einsum('lls,smn->mn', G, G) - np.einsum('lns,slm->mn', G, G))
    return R


def mn_quadrupole_moment(M, S, q):
    """Mass quadrupole of the Manko-Novikov spacetime: the Kerr value -S^2/M
    plus the deviation -q M^3."""
    return -(S * S) / M - q * M ** 3


def escape_crossing(M, a, Q, r_esc, r, theta, phi, p):
    """(theta, phi) where each ray crosses r = r_esc: its end state (r, theta,
    phi, covector p of shape (n, 4)) moved back along its velocity
    dq/dtau = g^{mu nu} p_nu, with g^{mu nu} the numerical inverse of the
    textbook covariant metric (linear over the last part of a step)."""
    th_out, ph_out = [], []
    for rk, tk, fk, pk in zip(r, theta, phi, np.asarray(p, float)):
        v = inverse_metric_numeric(M, a, Q, rk, tk) @ pk
        lam = (r_esc - rk) / v[1]
        th_out.append(tk + v[2] * lam)
        ph_out.append(fk + v[3] * lam)
    return np.array(th_out), np.array(ph_out)
