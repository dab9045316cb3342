"""Accuracy of one tracing run against another (e.g. the mixed-precision form
against binary64): where each escaped ray crossed the escape sphere, and how
many pixels changed class.  Host-side numpy on the tracer's outputs."""
from __future__ import annotations

import numpy as np


def sky_at_escape(M, a, Q, r_esc, res):
    """Boyer-Lindquist (theta, phi) where each escaped ray crossed r = r_esc:
    its end state moved back along its own velocity dq/dtau = g^{mu nu} p_nu
    (linear over the last fraction of a step; error ~1e-9 rad).  Two runs that
    agree on the trajectory but stop one step apart give the same answer."""
    r, th, ph = (np.asarray(res[k], np.float64) for k in ("r", "theta", "phi"))
    pt, pr, pth, pph = (np.asarray(res[k], np.float64) for k in ("p_t", "p_r", "p_theta", "p_phi"))
    s2, c2 = np.sin(th) ** 2, np.cos(th) ** 2
    rho2 = r * r + a * a * c2
    Delta = r * r - 2 * M * r + a * a + Q * Q
    grr = Delta / rho2
    ghh = 1.0 / rho2
    gtp = -a * (2 * M * r - Q * Q) / (rho2 * Delta)
    gpp = (Delta - a * a * s2) / (rho2 * Delta * s2)
    dr, dth, dph = grr * pr, ghh * pth, gtp * pt + gpp * pph
    lam = (r_esc - r) / dr
    return th + dth * lam, ph + dph * lam


def mixed_errors(M, a, Q, r_esc, ref, got):
    """Great-circle angle between the escape-sphere crossings of two runs
    (rays escaped in both) and the fraction of pixels whose flags differ."""
    both = (ref["flag"] == 1) & (got["flag"] == 1)
    t1, p1 = sky_at_escape(M, a, Q, r_esc, {k: v[both] for k, v in ref.items()})
    t2, p2 = sky_at_escape(M, a, Q, r_esc, {k: v[both] for k, v in got.items()})
    ang = angle_between(sky_direction(t1, p1), sky_direction(t2, p2))
    mism = float((ref["flag"] != got["flag"]).mean())
    q = np.quantile(ang, [0.5, 0.99, 0.999, 1.0]) if ang.size else np.zeros(4)
    return {"median": float(q[0]), "p99": float(q[1]), "p999": float(q[2]), "max": float(q[3]),
            "flag_mismatch": mism, "n_escaped_both": int(both.sum())}


def sky_direction(theta, phi):
    """Unit vector (sin th cos ph, sin th sin ph, cos th)."""
    theta, phi = np.asarray(theta), np.asarray(phi)
    return np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi),
                     np.cos(theta)], axis=-1)


def angle_between(u, v):
    """Great-circle angle between unit vectors (accurate for tiny angles)."""
    return 2.0 * np.arctan2(np.linalg.norm(u - v, axis=-1), np.linalg.norm(u + v, axis=-1))
