"""Comparison of a traced frame with the listing form of the oracle at each
ray's own rounding sensitivity.

The forward difference of step eps = 1e-8 divides the rounding of the metric
by eps, so two correct implementations whose roundings differ (the listing
form with the C library's sin/cos and a division per component, against the
kernel's fixed sequence) end their rays ~1e-9 rad apart, about as far as the
same implementation started one ulp away.  The listing form measures that
per ray (oracle probe=8: p_theta scaled by 1 + 2^-52 and by 1 - 2^-53, the
camera latitude moved one ulp up and down, p_r scaled by 1 + 2^-52 and by
1 - 2^-53, and the whole covector scaled by 1 + 2^-52 and 1 - 2^-53, which
leaves the ray unchanged in coordinate time but changes every rounding); s
is the largest end-angle change of the probes.  (With the first four probes
alone s was underestimated on some rays: on the 1000^2 frame's far-field
grid rays the largest d / s fell from 25 to 7 with all eight.)  A ray's flag and step count
are ill-conditioned (ref.flip) when a probe changes them or when its exit was
a tie: the escape or horizon test decided by a margin within 64 times the
probes' spread of the tested quantity (r, or |dt/dtau|), so that rounding
differently could end it one step earlier or later.

Gate: flags and step counts identical on every ray not so marked, and d = max(|d theta|, |d phi|) <= K_MAX * s on each such ray,
with the median and 99th percentile of d / s at most K_MED and K_P99; a
planted mistake (a dropped factor, a sign, the listing's 0.1667 in place of
1/6) gives ratios of 1e3 or more.
"""
from __future__ import annotations

import numpy as np

K_MAX, K_MED, K_P99 = 64.0, 3.0, 16.0
S_FLOOR = 1e-14   # a ray whose probes agree to this is compared at this floor


def compare_at_sensitivity(got, ref, k_max=K_MAX, k_med=K_MED, k_p99=K_P99, check=True):
    """got: mapping with theta, phi, flag, steps (binary64); ref: oracle Result
    of the listing form traced with probe > 0.  Returns statistics; with
    check=True asserts the gate."""
    flip = np.asarray(ref.flip, bool)
    ok = ~flip
    st = {"n": int(flip.size), "probe_flipped": int(flip.sum())}
    flags_same = np.asarray(got["flag"])[ok] == ref.flag[ok]
    steps_same = np.asarray(got["steps"])[ok] == ref.steps[ok]
    st["flag_mismatch"] = int((~flags_same).sum())
    st["steps_mismatch"] = int((~steps_same).sum())
    th = np.asarray(got["theta"], np.float64)
    ph = np.asarray(got["phi"], np.float64)
    d = np.maximum(np.abs(th - ref.theta), np.abs(ph - ref.phi))
    both_nan = np.isnan(th) & np.isnan(ref.theta)
    use = ok & ~both_nan
    ratio = d[use] / np.maximum(ref.sens[use], S_FLOOR)
    if ratio.size:
        st.update(ratio_median=float(np.median(ratio)), ratio_p99=float(np.percentile(ratio, 99)),
                  ratio_max=float(ratio.max()), d_median=float(np.median(d[use])),
                  d_max=float(d[use].max()), s_median=float(np.median(ref.sens[use])))
    if check:
        assert st["flag_mismatch"] == 0, st
        assert st["steps_mismatch"] == 0, st
        assert not np.isnan(ratio).any(), st
        assert ratio.size == 0 or (st["ratio_max"] <= k_max and st["ratio_median"] <= k_med
                                   and st["ratio_p99"] <= k_p99), st
    return st
