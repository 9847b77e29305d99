"""Write c2_self_divergence.json: how far the FP64 oracle drifts from itself
on the 256 x 512 SL-MPP7 workloads (nonlinear Landau damping and the
two-stream instability, x-CFL 3) when every non-zero cell of f0 moves by
one ulp (up or down, seeded).  The GPU-vs-oracle bound at step 2000 of
these workloads is derived from it: both differences start at the rounding
level, and the instability amplifies whatever differs.

Calls only the oracle and the seeded input generators.  Run from the
repository root:  python tests/golden/make_c2_self_divergence.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_1702_08521_amd import workloads as W  # noqa: E402

SEED = 1702
STOPS = (100, 200, 500, 1000, 1500, 2000)


def l1rel(a, b):
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def main():
    out = {"what": "L1 relative difference between two FP64 oracle runs whose initial f "
                   "differ by one ulp in every non-zero cell (direction drawn with the seed)",
           "seed": SEED, "command": "python tests/golden/make_c2_self_divergence.py",
           "workloads": {}}
    for which in ("landau_nl_1d1v", "twostream_1d1v"):
        spec = getattr(W, which)()
        g = O.make_grid(spec)
        f0 = O.init_separable(g, *W.separable_factors(spec))
        up = np.random.default_rng(SEED).random(f0.shape) < 0.5
        f1 = np.where(up, np.nextafter(f0, np.inf), np.nextafter(f0, -np.inf))
        f1[f0 == 0.0] = 0.0
        a, b = O.Run(spec, f0), O.Run(spec, f1)
        done, rec = 0, {}
        t0 = time.time()
        for stop in STOPS:
            a.step(spec["dt"], stop - done)
            b.step(spec["dt"], stop - done)
            done = stop
            rec[str(stop)] = l1rel(b.f, a.f)
            print(which, stop, rec[str(stop)], f"{time.time() - t0:.1f} s", flush=True)
        out["workloads"][which] = {"dt": spec["dt"], "l1_rel_by_step": rec}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_self_divergence.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
