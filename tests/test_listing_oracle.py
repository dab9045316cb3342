"""The listing form of the oracle (oracle/listing.c, the default form) and
the kernel-twin form (oracle/oracle.c) that the HIP kernels follow bit for bit.

The listing form is pinned like any oracle: the physics pins of
test_oracle_pins.py run on it (it is the default), and here its metric is
checked against the textbook covariant metric, the vacuum equations and the
Kerr limit, and its camera (built from the locally non-rotating frame's
vectors and the covariant metric) against the twin's camera (built from the
null condition of the inverse metric): two independent constructions of the
same initial states, equal to a few ulp.

The twin form is then tied to the listing form ray by ray at each ray's own
rounding sensitivity (tests/sens_gate.py), and a mistake planted in the
twin's source fails that gate.
"""
import ctypes
import math
import subprocess

import numpy as np
import pytest

import oracle
from tests import physics
from tests.sens_gate import compare_at_sensitivity

DEG = math.pi / 180.0
KERR64 = (0.5, 0.24, 0.0, 20.0, math.pi / 2, 0.0, 75 * DEG, 64, 64)
FRAMES = {
    "kn40": (0.5, 0.24, 0.3, 20.0, 80 * DEG, 0.0, 75 * DEG, 40, 40),
    "near_extremal40": (0.5, 0.49, 0.0, 20.0, 60 * DEG, 0.0, 75 * DEG, 40, 40),
    "high_latitude": (0.5, 0.1, 0.2, 35.0, 20 * DEG, 0.3, 40 * DEG, 19, 41),
    # 2e-6 rad from the pole: theta-displaced points divided, not refined
    "next_to_pole": (0.5, 0.3, 0.1, 20.0, 2e-6, 0.4, 60 * DEG, 16, 16),
}
MN_FRAMES = {
    "mn_listing_spacetime": (0.5, 0.24, 2.0, 8.0, math.pi / 2, 0.0, 75 * DEG, 24, 24),
    "mn_prolate": (0.5, 0.1, -1.0, 10.0, 1.2, 0.0, 75 * DEG, 24, 24),
}


def _as_dict(res):
    return {"theta": res.theta, "phi": res.phi, "flag": res.flag, "steps": res.steps}


# ------------------------------------------------------------------- metric
@pytest.mark.parametrize("M,a,Q", [(0.5, 0.24, 0.0), (0.5, 0.24, 0.3), (0.5, 0.49, 0.0),
                                   (0.0, 0.3, 0.0), (0.5, 0.0, 0.0)])
@pytest.mark.parametrize("r,th", [(1.3, 0.4), (3.0, 1.2), (20.0, 80 * DEG), (7.0, 2.9)])
def test_listing_metric_is_the_textbook_kerr_newman(M, a, Q, r, th):
    inv, cov = oracle.listing_metric(M, a, Q, r, th)
    ref = physics.covariant_metric(M, a, Q, r, th)
    np.testing.assert_allclose(cov, ref, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(inv @ ref, np.eye(4), rtol=0, atol=1e-12)


@pytest.mark.parametrize("S,q", [(0.5 * 0.25, 0.5), (0.1 * 0.25, -2.0), (0.98 * 0.25, 2.0)])
def test_listing_manko_novikov_metric(S, q):
    """Inverse and covariant forms agree, q = 0 is Kerr (the listing form's own
    Kerr-Newman branch with Q = 0), and the spacetime is vacuum."""
    M = 0.5
    for r, th in [(2.0, 0.7), (3.5, 1.3), (6.0, 2.2)]:
        inv, cov = oracle.listing_metric(M, S, q, r, th, mn=True)
        np.testing.assert_allclose(inv @ cov, np.eye(4), rtol=0, atol=1e-11)
        inv0, _ = oracle.listing_metric(M, S, 0.0, r, th, mn=True)
        kerr, _ = oracle.listing_metric(M, S / M, 0.0, r, th)
        np.testing.assert_allclose(inv0, kerr, rtol=1e-12, atol=1e-300)

        def five(rr, tt):
            g, _ = oracle.listing_metric(M, S, q, rr, tt, mn=True)
            return np.array([g[0, 0], g[0, 3], g[1, 1], g[2, 2], g[3, 3]])
        R = physics.ricci(five, r, th)
        assert np.abs(R).max() < 2e-6


# ------------------------------------------------------------------- camera
@pytest.mark.parametrize("case", [KERR64] + list(FRAMES.values()))
def test_two_camera_constructions_agree(case):
    """Listing camera (zero-angular-momentum frame vectors, velocity lowered
    with g_{mu nu}) and twin camera (p_t from the null condition of g^{mu nu},
    rescaled to dt/dtau = -1): the same covectors to a few ulp."""
    lis = oracle.camera(*case)
    twin = oracle.camera(*case, form="twin")
    np.testing.assert_array_equal(lis[:, :4], twin[:, :4])
    scale = np.abs(twin[:, 4:]).max(axis=1, keepdims=True)
    err = np.abs(lis[:, 4:] - twin[:, 4:]) / scale
    assert err.max() < 8 * 2.0 ** -52


@pytest.mark.parametrize("case", [KERR64, FRAMES["kn40"]])
def test_listing_camera_is_null_and_normalised(case):
    M, a, Q, r0, th0 = case[:5]
    init = oracle.camera(*case)
    gi = physics.inverse_metric_numeric(M, a, Q, r0, th0)
    p = init[:, 4:]
    H = np.einsum("ki,ij,kj->k", p, gi, p)
    terms = np.einsum("ki,ij,kj->k", np.abs(p), np.abs(gi), np.abs(p))
    assert np.abs(H / terms).max() < 1e-15
    tdot = p @ gi[0]
    np.testing.assert_allclose(tdot, -1.0, rtol=0, atol=4e-15)


def test_listing_mn_camera_matches_twin():
    case = MN_FRAMES["mn_listing_spacetime"]
    twin = oracle.trace_frame_mn(*case, max_steps=0, form="twin", want_p0=True)
    lis = oracle.trace_frame_mn(*case, max_steps=0, want_p0=True)
    scale = np.abs(twin.p0).max(axis=1, keepdims=True)
    assert (np.abs(lis.p0 - twin.p0) / scale).max() < 16 * 2.0 ** -52


# ------------------------------------------------- twin form vs listing form
@pytest.fixture(scope="module")
def kerr64_listing():
    return oracle.trace_frame(*KERR64, dt=0.01, max_steps=20000, probe=8)


def test_twin_matches_listing_on_small_kerr_frame(kerr64_listing):
    twin = oracle.trace_frame(*KERR64, dt=0.01, max_steps=20000, form="twin")
    st = compare_at_sensitivity(_as_dict(twin), kerr64_listing)
    print(st)
    # rays set apart as ill-conditioned (a probe changed flag or steps, or
    # the exit was a tie within the probes' spread) stay a small minority
    assert st["probe_flipped"] <= 0.005 * st["n"]
    assert (kerr64_listing.flag == 2).sum() > 50


@pytest.mark.parametrize("name", sorted(FRAMES))
def test_twin_matches_listing_on_other_frames(name):
    case = FRAMES[name]
    lis = oracle.trace_frame(*case, dt=0.01, max_steps=20000, probe=8)
    twin = oracle.trace_frame(*case, dt=0.01, max_steps=20000, form="twin")
    print(name, compare_at_sensitivity(_as_dict(twin), lis))


def test_twin_matches_listing_on_headline_frame_sample():
    """The 1000^2 Kerr-Newman frame of the benchmark (binary32-rounded inputs,
    dt = 0.005, 50000 steps): every 50th pixel in both axes, plus the pixels
    within two of each capture/escape transition along the middle row."""
    f = lambda x: float(np.float32(x))                                   # noqa: E731
    case = (f(0.5), f(0.24), f(0.3), f(20.0), f(80 * DEG), 0.0, f(75 * DEG), 1000, 1000)
    kw = dict(dt=0.005, max_steps=50000)
    row = 500 * 1000 + np.arange(1000)
    flags = oracle.trace_frame(*case, pixels=row, form="twin", **kw).flag
    cut = np.nonzero(flags[1:] != flags[:-1])[0]
    assert cut.size >= 2
    edge = (row[0] + cut[:, None] + np.arange(-1, 3)[None, :]).ravel()
    grid = (np.arange(25, 1000, 50)[:, None] * 1000 + np.arange(25, 1000, 50)[None, :]).ravel()
    pix = np.unique(np.concatenate([grid, edge]))
    lis = oracle.trace_frame(*case, pixels=pix, probe=8, **kw)
    twin = oracle.trace_frame(*case, pixels=pix, form="twin", **kw)
    st = compare_at_sensitivity(_as_dict(twin), lis)
    print(st)
    assert (lis.flag == 2).sum() >= 8 and (lis.flag == 1).sum() > 300


@pytest.mark.parametrize("name", sorted(MN_FRAMES))
def test_twin_matches_listing_manko_novikov(name):
    case = MN_FRAMES[name]
    lis = oracle.trace_frame_mn(*case, dt=0.01, max_steps=20000, probe=8)
    twin = oracle.trace_frame_mn(*case, dt=0.01, max_steps=20000, form="twin")
    print(name, compare_at_sensitivity(_as_dict(twin), lis))


@pytest.mark.parametrize("method,disk", [(1, None), (0, (2.0, 5.0, 0.02))])
def test_twin_matches_listing_euler_and_ring(method, disk):
    case = (0.5, 0.49, 0.0, 20.0, 80 * DEG, 0.0, 50 * DEG, 32, 32)
    lis = oracle.trace_frame(*case, dt=0.01, max_steps=20000, probe=8, method=method,
                             disk=disk)
    twin = oracle.trace_frame(*case, dt=0.01, max_steps=20000, form="twin", method=method,
                              disk=disk)
    st = compare_at_sensitivity(_as_dict(twin), lis)
    print(st)
    if disk is not None:
        assert (lis.flag == 4).sum() > 20


# ------------------------------------------------------- the gate has teeth
MUTANTS = [
    ("const double wtt = pt * pt, wtp = (2.0 * pt) * pph, wpp = pph * pph;",
     "const double wtt = pt * pt, wtp = pt * pph, wpp = pph * pph;"),        # drop the 2 of g^{t phi}
    ("const double h6 = h * (1.0 / 6.0);", "const double h6 = h * 0.1667;"),   # listing's 0.1667
    ("return fma(P->a * (2.0 * P->M), r, -(P->a * (P->Q * P->Q)));",
     "return -fma(P->a * (2.0 * P->M), r, -(P->a * (P->Q * P->Q)));"),      # sign of g^{t phi}
    ("return -0.5 * (1.0 / P->eps);", "return -0.5 * (1.0 / 1.01e-8);"),          # eps off by 1%
    ("const double rho2 = (r * r + a2) - a2 * s2;",
     "const double rho2 = (r * r + a2) + a2 * s2;"),                         # rho^2 from sin^2: sign
    ("G[m] = ((g1[m] + 2.0 * g2[m]) + 2.0 * g3[m]) + g4[m];",
     "G[m] = ((g1[m] + g2[m]) + 2.0 * g3[m]) + g4[m];"),                    # RK4 weight of phi's sum
]


def _mutant_twin(tmp_path, k, old, new):
    src = open(oracle._SRCS[0]).read()
    assert src.count(old) == 1, old
    path = tmp_path / f"twin_mutant{k}.c"
    path.write_text(src.replace(old, new))
    lib_path = tmp_path / f"libtwin_mutant{k}.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", str(lib_path), str(path), "-lm"])
    lib = ctypes.CDLL(str(lib_path))
    lib.oracle_trace_frame.restype = ctypes.c_int64
    lib.oracle_trace_frame.argtypes = oracle._load().oracle_trace_frame.argtypes
    return lib


@pytest.mark.parametrize("k", range(len(MUTANTS)))
def test_planted_mistake_in_twin_fails_the_gate(tmp_path, k):
    case = (0.5, 0.24, 0.3, 20.0, 80 * DEG, 0.0, 75 * DEG, 16, 16)
    lis = oracle.trace_frame(*case, dt=0.01, max_steps=20000, probe=8)
    lib = _mutant_twin(tmp_path, k, *MUTANTS[k])
    n = 16 * 16
    out = {f: np.empty(n) for f in ("t", "r", "theta", "phi", "pr", "pth")}
    flag, steps = np.empty(n, np.int8), np.empty(n, np.int32)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)   # noqa: E731
    lib.oracle_trace_frame(*case, 0.01, 1e-8, 1e4, 1.5, 20000, None, n, P(out["t"]), P(out["r"]),
                           P(out["theta"]), P(out["phi"]), P(out["pr"]), P(out["pth"]), None,
                           P(flag), P(steps), 4, 0, None)
    st = compare_at_sensitivity({"theta": out["theta"], "phi": out["phi"], "flag": flag,
                                 "steps": steps}, lis, check=False)
    print(st)
    failed = (st["flag_mismatch"] > 0 or st["steps_mismatch"] > 0
              or st.get("ratio_max", 0) > 64 or st.get("ratio_median", 0) > 3)
    assert failed
