"""Pins of the oracle's Manko-Novikov metric (paper Sec. 2.2.3) and of its
exp definition.

The printed formulas are garbled in places; the readings the oracle takes
are fixed here by what the spacetime must satisfy, not by retyping them:
q = 0 must give the Kerr metric (coded independently in the Kerr-Newman
oracle), every member must be a vacuum solution (Ricci tensor zero, from
finite differences of the oracle's own metric), asymptotically flat, with
the quadrupole deviation -q M^3 in the Newtonian far field, and reflection
symmetric about the equator.  Mutants of the oracle source (a sign, a term,
a constant changed) are compiled and must each fail one of these checks.
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests import physics

M = 0.5
CASES = [(0.5 * M * M, 0.5), (0.1 * M * M, -2.0), (0.98 * M * M, 2.0)]   # (S, q)
POINTS = [(2.0, 0.7), (3.5, 1.3), (6.0, 2.2)]


def _mn(S, q, fn=None):
    fn = fn or oracle.inverse_metric_mn
    return lambda r, th: fn(M, S, q, r, th)


def test_exp_definition_within_one_ulp_of_libm():
    x = np.concatenate([np.linspace(-745.0, 709.0, 200001), np.linspace(-1.0, 1.0, 20001),
                        [0.0, -0.0, 1e-300, -1e-300, 0.34657359, -0.34657359]])
    got = oracle.exp_def(x)
    ref = np.exp(x)
    ok = ref > 0
    ulp = np.abs(got[ok] - ref[ok]) / np.spacing(ref[ok])
    assert ulp.max() <= 1.0
    assert oracle.exp_def(np.array([0.0]))[0] == 1.0
    sp = oracle.exp_def(np.array([np.nan, 800.0, -800.0, np.inf, -np.inf]))
    assert np.isnan(sp[0]) and sp[1] == np.inf and sp[2] == 0.0 and sp[3] == np.inf
    assert sp[4] == 0.0


def test_constants_reduce_to_kerr_values():
    """k = sqrt(M^2 - a^2) with a = S/M (the Kerr horizon r+ = M + k), and
    beta = q M^3 / k^3."""
    for S, q in CASES:
        alpha, k, beta = oracle.mn_consts(M, S, q)
        a = S / M
        assert k == pytest.approx(math.sqrt(M * M - a * a), rel=1e-14)
        assert beta == pytest.approx(q * M ** 3 / k ** 3, rel=1e-14)
        assert -1.0 < alpha < 0.0


@pytest.mark.parametrize("S", [0.1 * M * M, 0.5 * M * M, 0.98 * M * M, -0.6 * M * M])
def test_q_zero_is_kerr(S):
    for r in (1.2, 2.0, 5.0, 40.0):
        for th in (0.2, 0.9, 1.5707, 2.4):
            if r <= M + math.sqrt(M * M - (S / M) ** 2):
                continue
            g_mn = oracle.inverse_metric_mn(M, S, 0.0, r, th)
            g_kerr = oracle.inverse_metric(M, S / M, 0.0, r, th)
            np.testing.assert_allclose(g_mn, g_kerr, rtol=1e-12, atol=0.0)


def _max_ricci(fn):
    return max(np.abs(physics.ricci(fn, r, th, h=4e-3)).max() for r, th in POINTS)


def test_ricci_check_separates_vacuum_from_non_vacuum():
    """The curvature check itself: Kerr is a vacuum solution, Kerr-Newman is
    not (its Ricci tensor is the electromagnetic stress)."""
    kerr = lambda r, th: oracle.inverse_metric(M, 0.3, 0.0, r, th)          # noqa: E731
    kn = lambda r, th: oracle.inverse_metric(M, 0.24, 0.3, r, th)           # noqa: E731
    assert _max_ricci(kerr) < 1e-8
    assert _max_ricci(kn) > 1e-3


@pytest.mark.parametrize("S,q", CASES)
def test_manko_novikov_is_a_vacuum_solution(S, q):
    assert _max_ricci(_mn(S, q)) < 2e-6


@pytest.mark.parametrize("S,q", CASES)
def test_asymptotically_flat(S, q):
    r, th = 1e5, 1.0
    g = oracle.inverse_metric_mn(M, S, q, r, th)
    assert abs(g[0] + 1.0 + 2.0 * M / r) < 1e-8          # g^tt = -(1 + 2M/r + ...)
    assert abs(g[2] - 1.0 + 2.0 * M / r) < 1e-8          # g^rr = 1 - 2M/r + ...
    assert abs(g[3] * r * r - 1.0) < 1e-8
    assert abs(g[4] * (r * math.sin(th)) ** 2 - 1.0) < 1e-8


@pytest.mark.parametrize("S,q", CASES)
def test_far_field_quadrupole(S, q):
    """-g_tt differs from Kerr's by 2 q M^3 P2(cos theta) / r^3 (the mass
    quadrupole -q M^3 on top of Kerr's), up to O(M/r) relative."""
    r = 2000.0
    for th in (0.4, 1.0, 1.5):
        gq = physics.covariant_from_inverse(oracle.inverse_metric_mn(M, S, q, r, th))
        g0 = physics.covariant_from_inverse(oracle.inverse_metric_mn(M, S, 0.0, r, th))
        p2 = 1.5 * math.cos(th) ** 2 - 0.5
        ratio = -(gq[0, 0] - g0[0, 0]) * r ** 3 / (2.0 * q * M ** 3 * p2)
        assert abs(ratio - 1.0) < 1e-3


@pytest.mark.parametrize("S,q", CASES)
def test_equatorial_reflection_symmetry(S, q):
    for r, th in POINTS:
        a = oracle.inverse_metric_mn(M, S, q, r, th)
        b = oracle.inverse_metric_mn(M, S, q, r, math.pi - th)
        np.testing.assert_allclose(a, b, rtol=1e-12)


MUTANTS = [
    ("const double Sb = -((x + y) * L2);", "const double Sb = (x + y) * L2;"),
    ("const double L2 = fma(P2, iR3, fma(-P1, iR2, iR));", "const double L2 = fma(P2, iR3, fma(P1, iR2, iR));"),
    ("beta * (Sg - 2.0)", "beta * Sg"),
    ("const double P3 = u * fma(2.5 * u, u, -1.5);", "const double P3 = u * fma(2.5 * u, u, -0.5);"),
    ("const double psi = (beta * P2) * iR3;", "const double psi = (beta * P2) * iR2;"),
    ("const double B2 = fma(1.0 + y, am, (1.0 - y) * bm);", "const double B2 = fma(1.0 + y, am, (1.0 + y) * bm);"),
    ("fma(-y, apb, bma)", "fma(y, apb, bma)"),
    ("(K->twok * C) / fA - K->om0", "(K->twok * C) / fA + K->om0"),
    ("fma((1.5 * (beta * beta)) * iR6,", "fma((3.0 * (beta * beta)) * iR6,"),
    ("K->beta = (q * (M * M * M)) / (K->k * K->k * K->k);", "K->beta = (q * (M * M)) / (K->k * K->k);"),
]


def _mutant_lib(tmp_path, k, old, new):
    src = open(oracle._SRCS[0]).read()   # oracle.c, the kernel-twin form
    assert src.count(old) == 1, old
    path = tmp_path / f"mutant{k}.c"
    path.write_text(src.replace(old, new))
    lib_path = tmp_path / f"libmutant{k}.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", str(lib_path), str(path), "-lm"])
    lib = ctypes.CDLL(str(lib_path))
    d = ctypes.c_double
    lib.oracle_inverse_metric_mn.argtypes = [d, d, d, d, d, ctypes.c_void_p]
    lib.oracle_inverse_metric_mn.restype = None

    def fn(M_, S, q, r, th):
        g = np.empty(5)
        lib.oracle_inverse_metric_mn(M_, S, q, float(r), float(th), g.ctypes.data_as(ctypes.c_void_p))
        return g
    return fn


def _pins_pass(fn):
    for S, q in CASES:
        if _max_ricci(_mn(S, q, fn)) >= 2e-6:
            return False
        g = fn(M, S, q, 1e5, 1.0)
        if abs(g[3] * 1e10 - 1.0) >= 1e-8 or abs(g[2] - 1.0 + 2.0 * M / 1e5) >= 1e-8:
            return False
        r = 2000.0
        gq = physics.covariant_from_inverse(fn(M, S, q, r, 1.0))
        g0 = physics.covariant_from_inverse(fn(M, S, 0.0, r, 1.0))
        p2 = 1.5 * math.cos(1.0) ** 2 - 0.5
        if abs(-(gq[0, 0] - g0[0, 0]) * r ** 3 / (2.0 * q * M ** 3 * p2) - 1.0) >= 1e-3:
            return False
        g_kerr = oracle.inverse_metric(M, S / M, 0.0, 3.0, 0.8)
        if not np.allclose(fn(M, S, 0.0, 3.0, 0.8), g_kerr, rtol=1e-12, atol=0.0):
            return False
    return True


def test_unmutated_source_passes_the_pins(tmp_path):
    assert _pins_pass(_mutant_lib(tmp_path, 0, "const double P1 = u;", "const double P1 = u;"))


@pytest.mark.parametrize("k", range(len(MUTANTS)))
def test_mutants_fail_the_pins(tmp_path, k):
    old, new = MUTANTS[k]
    assert not _pins_pass(_mutant_lib(tmp_path, k + 1, old, new))


# ---------------------------------------------------------------- whole rays
def _frame(S, q, W=20, H=14, **kw):
    return oracle.trace_frame_mn(M, S, q, 20.0, math.radians(80.0), 0.0, math.radians(60.0),
                                 W, H, dt=0.01, max_steps=20000, want_p0=True, **kw)


def test_camera_and_frame_reduce_to_kerr_at_q_zero():
    """With q = 0 the Manko-Novikov path (camera, right-hand side, RK4) traces
    the Kerr frame of the independently coded Kerr-Newman path: the same
    flags and end points up to the rounding differences the forward
    differences amplify."""
    S = 0.6 * M * M
    mn = _frame(S, 0.0)
    kerr = oracle.trace_frame(M, S / M, 0.0, 20.0, math.radians(80.0), 0.0, math.radians(60.0),
                              20, 14, dt=0.01, max_steps=20000, want_p0=True)
    np.testing.assert_allclose(mn.p0, kerr.p0, rtol=1e-13, atol=1e-15)
    assert np.array_equal(mn.flag, kerr.flag)
    esc = kerr.flag == 1
    assert esc.sum() > 50 and (kerr.flag == 2).sum() > 10
    assert np.abs(mn.theta[esc] - kerr.theta[esc]).max() < 1e-6
    assert np.abs(mn.phi[esc] - kerr.phi[esc]).max() < 1e-6


@pytest.mark.parametrize("S,q,med,mx", [(CASES[0][0], CASES[0][1], 5e-8, 1e-5),
                                        (CASES[1][0], CASES[1][1], 5e-8, 1e-5),
                                        (CASES[2][0], CASES[2][1], 2e-5, 1e-4)])
def test_null_condition_holds_at_the_end(S, q, med, mx):
    """H = 1/2 g^{mu nu} p_mu p_nu stays ~0 along escaping rays (p_t and p_phi
    are carried unchanged).  For S = 0.98 M^2, q = 2 (beta = 254) the
    exponentials' arguments reach ~500, so their rounding gives the metric
    ~1e-13 relative noise, which the eps = 1e-8 forward difference turns
    into ~1e-5 relative noise in the forces: H then drifts ~1e-5 whatever
    the step (halving dt changes it by less than 2x)."""
    res = _frame(S, q)
    esc = np.nonzero(res.flag == 1)[0]
    assert esc.size > 50
    hs = []
    for k in esc:
        g = oracle.inverse_metric_mn(M, S, q, res.r[k], res.theta[k])
        pt, pph = res.p0[k, 0], res.p0[k, 3]
        pr, pth = res.pr[k], res.ptheta[k]
        hs.append(0.5 * (g[0] * pt * pt + 2 * g[1] * pt * pph + g[2] * pr * pr
                         + g[3] * pth * pth + g[4] * pph * pph))
    hs = np.abs(hs)
    # Kerr-Newman rays of this frame: median 3e-9, max 1.5e-8
    assert np.median(hs) < med and hs.max() < mx


def test_spin_reversal_mirrors_the_frame_exactly():
    S, q = 0.5 * M * M, 0.5
    W, H = 20, 14
    A = _frame(S, q, W, H)
    B = _frame(-S, q, W, H)
    mirror = lambda x: x.reshape(H, W)[:, ::-1].ravel()          # noqa: E731
    np.testing.assert_array_equal(A.phi, -mirror(B.phi))
    for k in ("t", "r", "theta", "flag", "steps"):
        np.testing.assert_array_equal(getattr(A, k), mirror(getattr(B, k)), err_msg=k)
