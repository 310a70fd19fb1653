"""Writes fullsize_samples.npz: FP64 oracle densities at seeded fluid nodes
of the two single-instance benchmark workloads at their full sizes,
  d2q9: the 1024x512 disc-medium drainage (MRT, M = 10), after 200 steps;
  d3q19: the 384^3 sphere-pack drainage (TRT, M = 10), after 200 steps.
Calls only the oracle and the seeded input generators.  The 384^3 oracle
holds about 40 GB of FP64 state and takes a few seconds per step.

    python tests/golden/make_fullsize_samples.py [d2q9] [d3q19]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O                                    # noqa: E402
from paper_2111_08666_amd import inputs as I          # noqa: E402

OUT = os.path.join(HERE, "fullsize_samples.npz")
CASES = {"d2q9": (I.large_drainage, 200), "d3q19": (I.drainage_3d, 200)}
SAMPLES = 2048


def main(names):
    out = {}
    if os.path.exists(OUT):
        with np.load(OUT, allow_pickle=False) as z:
            out = {k: z[k] for k in z.files}
    rng = np.random.default_rng(77)
    for name, (make, steps) in CASES.items():
        p = make()
        fluid = np.flatnonzero(p.mask.ravel() == 0)
        idx = np.sort(rng.choice(fluid, size=SAMPLES, replace=False)).astype(np.int64)
        if name not in names:
            continue
        t0 = time.time()
        s = O.OracleSim(p)
        print(f"[fullsize] {name}: oracle ready ({time.time() - t0:.0f}s)", flush=True)
        for k in range(steps):
            s.step(1)
            if (k + 1) % max(1, steps // 10) == 0:
                print(f"[fullsize] {name}: step {k + 1}/{steps} ({time.time() - t0:.0f}s)", flush=True)
        out[f"{name}_idx"] = idx
        out[f"{name}_rho"] = s.density().reshape(2, -1)[:, idx]
        out[f"{name}_steps"] = np.array(steps)
        del s
    np.savez_compressed(OUT, **out)
    print(f"[fullsize] wrote {OUT}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
