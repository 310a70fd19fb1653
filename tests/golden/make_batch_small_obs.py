"""Writes batch64_small_step10k_obs.npz: FP64 oracle observables after
10 000 steps of the eight smallest of the 64 uneven drainage instances
(256x128 and 320x160, each with its own medium, contact angle and pressure
step): window saturations (count and weighted), the capillary pressure and
the face pressures (Eq. 14), and both masses.  Calls only the oracle and the
seeded input generators.

    python tests/golden/make_batch_small_obs.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O                                    # noqa: E402
from paper_2111_08666_amd import inputs as I          # noqa: E402

STEPS = 10000
COUNT = 8
KEYS = ("s_w", "s_w_weighted", "pc", "p_in", "p_out")


def smallest(probs, n=COUNT):
    """Indices of the n smallest instances (ties by index)."""
    return sorted(range(len(probs)), key=lambda k: (probs[k].n_nodes, k))[:n]


def main():
    probs = I.batch_instances(64)
    idx = smallest(probs)
    out = {"steps": STEPS, "index": np.array(idx)}
    t0 = time.time()
    for k in idx:
        s = O.OracleSim(probs[k])
        s.step(STEPS)
        o = s.observables()
        for key in KEYS:
            out[f"{key}{k}"] = np.float64(o[key])
        out[f"mass{k}"] = np.array(o["mass"], np.float64)
        print(f"[batch-small] instance {k} {probs[k].nx}x{probs[k].ny}: S_w {o['s_w']:.5f} "
              f"P_c {o['pc']:+.6f} ({time.time() - t0:.0f}s, {O.num_threads()} threads)", flush=True)
    np.savez_compressed(os.path.join(HERE, "batch64_small_step10k_obs.npz"), **out)


if __name__ == "__main__":
    main()
