"""The oracle reproduces its recorded end states bit for bit (regression
record written by tests/golden/make_oracle_golden.py)."""
import math
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "oracle_kerr64_sample.txt")


def test_oracle_matches_its_record():
    rows = [ln.split() for ln in open(GOLDEN) if not ln.startswith("#")]
    pixels = np.array([int(r[0]) for r in rows])
    res = oracle.trace_frame(0.5, 0.24, 0.0, 20.0, math.pi / 2, 0.0, math.radians(75.0),
                             64, 64, dt=0.01, eps=1e-8, horizon_norm=1e4, escape_factor=1.5,
                             max_steps=20000, pixels=pixels)
    for k, r in enumerate(rows):
        assert res.flag[k] == int(r[1]) and res.steps[k] == int(r[2])
        got = [res.t[k], res.r[k], res.theta[k], res.phi[k], res.pr[k], res.ptheta[k]]
        assert [float(v).hex() for v in got] == r[3:9]
