"""Write oracle_kerr64_sample.txt: end states of a fixed sample of rays of the
small Kerr frame (M=0.5, a=0.24, Q=0, r0=20, theta0=pi/2, phi0=0, 64x64, fov 75
deg, dt=0.01, eps=1e-8, 20000 steps), as produced by the CPU oracle.

The paper prints no per-pixel values, so this file is a regression record of
the oracle itself (any change to its arithmetic shows up here), not a pin.
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


def main():
    res = oracle.trace_frame(0.5, 0.24, 0.0, 20.0, math.pi / 2, 0.0, math.radians(75.0),
                             64, 64, dt=0.01, eps=1e-8, horizon_norm=1e4, escape_factor=1.5,
                             max_steps=20000, pixels=np.array(PIXELS))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_kerr64_sample.txt")
    with open(out, "w") as f:
        f.write("# pixel flag steps t r theta phi p_r p_theta (binary64 as hex)\n")
        for k, pix in enumerate(PIXELS):
            vals = [res.t[k], res.r[k], res.theta[k], res.phi[k], res.pr[k], res.ptheta[k]]
            f.write(f"{pix} {int(res.flag[k])} {int(res.steps[k])} "
                    + " ".join(float(v).hex() for v in vals) + "\n")


if __name__ == "__main__":
    main()
