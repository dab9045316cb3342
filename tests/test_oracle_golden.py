"""Both forms of the oracle reproduce their recorded end states bit for bit
(regression records written by tests/golden/make_oracle_golden.py)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_oracle_golden as mk  # noqa: E402


@pytest.mark.parametrize("form", mk.FORMS)
def test_oracle_matches_its_record(form):
    rows = [ln.split() for ln in open(mk.record_path(form)) if not ln.startswith("#")]
    pixels = np.array([int(r[0]) for r in rows])
    res = mk.trace(form, pixels)
    for k, r in enumerate(rows):
        assert res.flag[k] == int(r[1]) and res.steps[k] == int(r[2])
        got = [res.t[k], res.r[k], res.theta[k], res.phi[k], res.pr[k], res.ptheta[k]]
        assert [float(v).hex() for v in got] == r[3:9]
