"""Pins of the oracle's shading (the appendix listing's colour kernel and
the exit-time map): the colours the rules assign at points where the answer
is fixed by the trigonometry or the ordering of the tests."""
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
