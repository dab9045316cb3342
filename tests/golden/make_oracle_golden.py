"""Write the oracle's regression records: end states of a fixed sample of rays
of the small Kerr frame (M=0.5, a=0.24, Q=0, r0=20, theta0=pi/2, phi0=0,
64x64, fov 75 deg, dt=0.01, eps=1e-8, 20000 steps), one file per form of the
CPU oracle: oracle_kerr64_listing_sample.txt (the listing form, the default)
and oracle_kerr64_twin_sample.txt (the kernel-twin form).

The paper prints no per-pixel values, so these files are regression records
of the oracle itself (any change to its arithmetic shows up here), not pins.
Calls only the oracle package.  Run from the repository root:
    python tests/golden/make_oracle_golden.py
"""
import math
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import oracle  # noqa: E402

PIXELS = [0, 63, 1000, 2016, 2047, 2080, 2111, 3000, 4032, 4095] + list(range(1900, 1910))
FORMS = ("listing", "twin")


def record_path(form):
    return os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        f"oracle_kerr64_{form}_sample.txt")


def trace(form, pixels):
    return oracle.trace_frame(0.5, 0.24, 0.0, 20.0, math.pi / 2, 0.0, math.radians(75.0),
                              64, 64, dt=0.01, eps=1e-8, horizon_norm=1e4, escape_factor=1.5,
                              max_steps=20000, pixels=np.asarray(pixels), form=form)


def main():
    for form in FORMS:
        res = trace(form, PIXELS)
        with open(record_path(form), "w") as f:
            f.write("# pixel flag steps t r theta phi p_r p_theta (binary64 as hex)\n")
            for k, pix in enumerate(PIXELS):
                vals = [res.t[k], res.r[k], res.theta[k], res.phi[k], res.pr[k], res.ptheta[k]]
                f.write(f"{pix} {int(res.flag[k])} {int(res.steps[k])} "
                        + " ".join(float(v).hex() for v in vals) + "\n")


if __name__ == "__main__":
    main()
