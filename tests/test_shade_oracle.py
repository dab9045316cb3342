"""Pins of the oracle's shading (Sec. 4's figures): the three lines on the
sky (a vertical great circle, a circle around the hole as seen from the
camera, the equator) at points where the answer is fixed by the trigonometry
or the lines' precedence; the exit-time map; and the bilinearly filtered sky
texture against functions bilinear filtering reproduces exactly, texel
centres, midpoints, the wrap in phi, the clamp at the poles and the
reflection of theta beyond [0, pi]."""
import math

import numpy as np

import oracle

RED, GREEN, BLUE, DARK, BLACK, CYAN = (0xff0000ff, 0xff00ff00, 0xffff0000, 0xff3c0000,
                                       0xff000000, 0xffffff00)


def test_band_colours():
    pi = math.pi
    #                theta,      phi,          flag, want
    cases = [(pi / 4, 0.0, 1, RED),               # sin phi = 0
             (pi / 4, pi, 1, RED),
             (pi / 4, 0.05, 1, RED),              # sin^2 = 0.0025
             (pi / 4, 0.2, 1, DARK),              # sin^2 = 0.039, cos^2 = 0.96, sin 2th = 1
             (pi / 4, pi / 2, 1, GREEN),          # cos phi = 0
             (pi / 4, -pi / 2 + 0.05, 1, GREEN),
             (pi / 2, pi / 4, 1, BLUE),           # sin 2 theta = sin pi
             (0.02, pi / 4, 1, BLUE),             # near the pole
             (pi / 3, pi / 4, 1, DARK),
             (0.0, 0.0, 1, RED),                  # red is tested first
             (pi / 4, 0.0, 2, BLACK),             # captured
             (pi / 4, 0.0, 0, BLACK),             # step limit
             (pi / 4, 0.0, 3, BLACK)]             # invalid
    th, ph, fl, want = map(np.array, zip(*cases))
    got = oracle.shade(0, None, th, ph, fl.astype(np.int8))
    np.testing.assert_array_equal(got, want.astype(np.uint32))


def test_band_threshold_is_sin_squared_one_percent():
    edge = math.asin(0.1)                         # sin^2 = 0.01 exactly at the edge
    ph = np.array([edge * (1 - 1e-9), edge * (1 + 1e-9)])
    got = oracle.shade(0, None, np.full(2, math.pi / 3), ph, np.ones(2, np.int8))
    assert got[0] == RED and got[1] == DARK


def test_exit_time_colours():
    t = np.array([0.0, -50.0, -99.99, -100.0, -150.0, -10.0, -10.0, np.nan])
    flag = np.array([1, 1, 1, 1, 1, 2, 0, 3], np.int8)
    got = oracle.shade(1, t, None, None, flag, t_max=100.0)
    level = [0, 127, 254]
    want = [0xff000000 | ((64 + l * 191 // 255) << 16) | (l << 8) for l in level]
    want += [CYAN, CYAN, CYAN, CYAN, BLACK]
    np.testing.assert_array_equal(got, np.array(want, np.uint32))
    # banding: every other band of width 10 is dimmed to 7/8
    t = -np.array([5.0, 15.0, 25.0])
    got = oracle.shade(1, t, None, None, np.ones(3, np.int8), t_max=100.0, band=10.0)
    lv = [int(255 * 0.05), int(255 * 0.15) * 7 // 8, int(255 * 0.25)]
    want = [0xff000000 | ((64 + l * 191 // 255) << 16) | (l << 8) for l in lv]
    np.testing.assert_array_equal(got, np.array(want, np.uint32))


# ---------------------------------------------------------------- texture
TW, TH = 16, 8


def _dir(x, y):
    """End direction (theta, phi) whose texel coordinates are (x, y):
    x = u TW - 1/2 with u = phi / 2 pi, y = v TH - 1/2 with v = theta / pi."""
    return math.pi * (y + 0.5) / TH, 2 * math.pi * (x + 0.5) / TW


def _shade_tex(tex, theta, phi, flag=None):
    theta, phi = np.atleast_1d(theta), np.atleast_1d(phi)
    flag = np.ones(theta.size, np.int8) if flag is None else flag
    return oracle.shade(2, None, theta, phi, flag, texture=tex)


def _channels(c):
    c = np.asarray(c, np.uint32)
    return np.stack([(c >> (8 * k)) & 255 for k in range(4)], axis=-1).astype(np.int64)


def _pack(r, g=0, b=0, a=255):
    return (np.uint32(a) << 24) | (np.uint32(b) << 16) | (np.uint32(g) << 8) | np.uint32(r)


def test_texture_reproduces_bilinear_functions_exactly():
    """Bilinear filtering reproduces any A + B x + C y + D x y sampled at the
    texel centres: texture R = 2 + 3i + 5j + ij, G = 200 - 7i - 3j; at random
    interior points the bytes are those values, rounded."""
    i, j = np.meshgrid(np.arange(TW), np.arange(TH))
    tex = _pack((2 + 3 * i + 5 * j + i * j).astype(np.uint32),
                (200 - 7 * i - 3 * j).astype(np.uint32), 17)
    rng = np.random.default_rng(5)
    x = rng.uniform(0.0, TW - 1.0, 500)
    y = rng.uniform(0.0, TH - 1.0, 500)
    th, ph = _dir(x, y)
    got = _channels(_shade_tex(tex, th, ph))
    want_r = 2 + 3 * x + 5 * y + x * y
    want_g = 200 - 7 * x - 3 * y
    assert np.abs(got[:, 0] - want_r).max() <= 0.5 + 1e-9
    assert np.abs(got[:, 1] - want_g).max() <= 0.5 + 1e-9
    assert np.all(got[:, 2] == 17) and np.all(got[:, 3] == 255)


def test_texel_centres_and_midpoints():
    rng = np.random.default_rng(6)
    tex = (rng.integers(0, 128, (TH, TW, 4)) * 2).astype(np.uint32)      # even bytes
    tex = tex[..., 0] | (tex[..., 1] << 8) | (tex[..., 2] << 16) | (tex[..., 3] << 24)
    c = _channels(tex)
    for jj in range(TH):
        for ii in range(TW):
            th, ph = _dir(ii, jj)
            assert _shade_tex(tex, th, ph)[0] == tex[jj, ii]
    # halfway between columns ii and ii + 1 (and between the last and the first)
    for ii in range(TW):
        th, ph = _dir(ii + 0.5, 3)
        want = (c[3, ii] + c[3, (ii + 1) % TW]) // 2
        np.testing.assert_array_equal(_channels(_shade_tex(tex, th, ph))[0], want)


def test_texture_wraps_in_phi_and_clamps_at_the_poles():
    rng = np.random.default_rng(7)
    tex = rng.integers(0, 2 ** 32, (TH, TW), dtype=np.uint64).astype(np.uint32)
    # phi = 0 is halfway between the last column and the first
    th = math.pi * 2.5 / TH
    np.testing.assert_array_equal(
        _channels(_shade_tex(tex, th, 0.0))[0],
        np.floor((_channels(tex[2, TW - 1]) + _channels(tex[2, 0])) / 2 + 0.5).astype(np.int64))
    # phi and phi + 2 pi k are the same direction
    ph = rng.uniform(-20, 20, 200)
    ths = rng.uniform(0.1, 3.0, 200)
    np.testing.assert_array_equal(_shade_tex(tex, ths, ph), _shade_tex(tex, ths, ph + 4 * math.pi))
    # the pole rows clamp: theta = 0 samples row 0 only, theta = pi the last row only
    x = 5.0
    for theta, row in ((0.0, 0), (math.pi, TH - 1)):
        got = _channels(_shade_tex(tex, theta, 2 * math.pi * (x + 0.5) / TW))[0]
        np.testing.assert_array_equal(got, _channels(tex[row, 5]))


def test_texture_theta_outside_zero_pi_is_the_reflected_direction():
    rng = np.random.default_rng(8)
    tex = rng.integers(0, 2 ** 32, (TH, TW), dtype=np.uint64).astype(np.uint32)
    th = rng.uniform(0.05, 3.0, 300)
    ph = rng.uniform(-3, 3, 300)
    a = _shade_tex(tex, -th, ph)                    # over the pole theta = 0
    b = _shade_tex(tex, th, ph + math.pi)
    assert (a == b).mean() > 0.99                   # equal up to a rounding at a byte boundary
    assert np.abs(_channels(a) - _channels(b)).max() <= 1


def test_texture_constant_and_non_escaped_rays():
    tex = np.full((TH, TW), _pack(10, 20, 30, 40), np.uint32)
    th = np.linspace(-1, 4, 50)
    ph = np.linspace(-7, 7, 50)
    flag = np.array([1, 2, 0, 3, 4] * 10, np.int8)
    got = _shade_tex(tex, th, ph, flag)
    np.testing.assert_array_equal(got[flag == 1], np.full((flag == 1).sum(), tex[0, 0]))
    assert np.all(got[flag != 1] == BLACK)
