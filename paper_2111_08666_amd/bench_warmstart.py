"""Time to steady state with and without the learned warm start, on one MI355X.

    python -m paper_2111_08666_amd.bench_warmstart [--first 2000] [--count 32] [--cap 300000]

Held-out drainage instances (256x256 disc media, contact angle and pressure
step drawn per instance; training used other indices) whose contact angle
is below 90 degrees run twice as one batch each: from the plain cold start,
and from the densities the trained U-Net's predicted saturation sets.  Each
run stops when every instance's window saturation changes by less than
1e-6 per 1000 steps (or at the cap).  Prints one JSON line: the steps to
steady state per instance for both starts, the median ratio over the
instances where both settle and agree within 0.01 in saturation, the wall
time of each batch, and the network's inference time for the whole set.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WEIGHTS = os.path.join(ROOT, "paper_2111_08666_amd", "weights", "unet_drainage256.npz")


def measure(first=2000, count=32, cap=300000, s_tol=0.01, log=None):
    """Runs the comparison and returns the result record (see the module
    docstring); `log` receives the progress lines."""
    import torch
    from paper_2111_08666_amd import inputs as I
    from paper_2111_08666_amd import surrogate as S
    from paper_2111_08666_amd import train_surrogate as T

    log = log or (lambda m: print(m, file=sys.stderr, flush=True))
    probs = [p for p in (I.surrogate_instance(k) for k in range(first, first + count)) if p.theta < 90.0]
    net = S.UNet.load(WEIGHTS)
    S.predict(net, probs[:1])  # first call loads the kernels
    torch.cuda.synchronize()
    t0 = time.time()
    sat = S.predict(net, probs)
    torch.cuda.synchronize()
    infer_s = time.time() - t0
    warm = []
    for p, s in zip(probs, sat):
        q = I.Problem(**{f: getattr(p, f) for f in p.__dataclass_fields__})
        q.rho0 = S.warm_start_density(p, s)
        warm.append(q)
    log(f"[warmstart] {len(probs)} instances; inference {infer_s * 1e3:.1f} ms")
    t0 = time.time()
    cs, cc, cS, _, _ = T.run_to_steady(probs, cap, tag=" cold")
    cold_s = time.time() - t0
    t0 = time.time()
    ws, wc, wS, _, _ = T.run_to_steady(warm, cap, tag=" warm")
    warm_s = time.time() - t0
    both = [i for i in range(len(probs)) if cc[i] and wc[i]]
    agree = [i for i in both if abs(cS[i] - wS[i]) <= s_tol]
    ratios = [cs[i] / ws[i] for i in agree]
    return {
        "metric": "time to steady state, cold start / U-Net warm start (steps, median over settled instances)",
        "value": round(float(np.median(ratios)), 3) if ratios else None, "unit": "x",
        "higher_is_better": True,
        "config": {"workload": f"{len(probs)} held-out D2Q9 drainage instances 256x256, contact angle < 90 deg",
                   "indices": [first, first + count], "cap": cap, "check": 1000, "tol": 1e-6,
                   "s_tol": s_tol},
        "settled_both": len(both), "agree_within_s_tol": len(agree),
        "cold_steps": cs, "warm_steps": ws,
        "abs_dS": [round(abs(cS[i] - wS[i]), 5) for i in range(len(probs))],
        "steps_total": {"cold": int(sum(cs)), "warm": int(sum(ws))},
        "wall_s": {"cold_batch": round(cold_s, 2), "warm_batch": round(warm_s, 2),
                   "inference": round(infer_s, 4)},
    }


def summary(w):
    """The record's headline fields, as bench.py reports them."""
    return {"cold_over_warm_steps_median": w["value"], "unit": "x", "workload": w["config"]["workload"],
            "criterion": "window saturation change < 1e-6 per 1000 steps; cold and warm S within 0.01",
            "settled_both": w["settled_both"], "agree_within_s_tol": w["agree_within_s_tol"],
            "steps_total": w["steps_total"], "wall_s": w["wall_s"], "cap": w["config"]["cap"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--first", type=int, default=2000)
    ap.add_argument("--count", type=int, default=32)
    ap.add_argument("--cap", type=int, default=300000)
    ap.add_argument("--s-tol", type=float, default=0.01)
    a = ap.parse_args()
    print(json.dumps(measure(a.first, a.count, a.cap, a.s_tol)), flush=True)


if __name__ == "__main__":
    main()
