"""Writes batch64_step200_samples.npz: FP64 oracle densities after 200 steps
at 1024 seeded fluid nodes of each of the 64 uneven drainage instances
(256x128 .. 1024x512, contact angle and pressure step per instance).  Calls
only the oracle and the seeded input generators.

    python tests/golden/make_batch64_samples.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O                                    # noqa: E402
from paper_2111_08666_amd import inputs as I          # noqa: E402

STEPS = 200
SAMPLES = 1024


def main():
    probs = I.batch_instances(64)
    rng = np.random.default_rng(2024)
    out = {"steps": STEPS}
    t0 = time.time()
    for k, p in enumerate(probs):
        fluid = np.flatnonzero(p.mask.ravel() == 0)
        idx = np.sort(rng.choice(fluid, size=SAMPLES, replace=False)).astype(np.int64)
        s = O.OracleSim(p)
        s.step(STEPS)
        rho = s.density().reshape(2, -1)[:, idx]
        out[f"idx{k}"] = idx
        out[f"rho{k}"] = rho
        out[f"shape{k}"] = np.array(p.mask.shape)
        print(f"[batch64] instance {k} {p.nx}x{p.ny} done ({time.time() - t0:.0f}s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "batch64_step200_samples.npz"), **out)


if __name__ == "__main__":
    main()
