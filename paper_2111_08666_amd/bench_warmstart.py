"""Time to steady state with and without the learned warm start, on one MI355X.

    python -m paper_2111_08666_amd.bench_warmstart [--first 2000] [--count 32] [--cap 300000]

Held-out drainage instances (256x256 disc media, contact angle and pressure
step drawn per instance; training used other indices) whose contact angle is
below 90 degrees each run on their own solver, one after another:

- cold: the plain method from its cold start, until the window saturation
  changes by less than 1e-6 per 1000 steps (or the cap);
- warm: the plain method from the densities the trained U-Net's predicted
  saturation sets.  The warm run gets a step budget; a warm run that has not
  settled within it, or whose density becomes non-finite, falls back to the
  cold start, and its cost is then the budget spent plus the whole cold run.

The plain method also judges the warm result: it is compared with the cold
steady saturation.  Every time is wall clock on the GPU's stream, from the
first step to the settle check that stops the run; the warm side adds the
network's inference time (the batch's, shared equally).  Instances with a
contact angle of 90 degrees or more are left out: there the non-wetting phase
imbibes spontaneously and neither start settles within the cap.

The same comparison also runs batched, as a production sweep would: all
cold starts in one batch, all warm starts in another, each instance retired
from its batch (lbm_batch_set_active) as it settles or goes non-finite, so
the batch's wall time is that of its slowest instance at a shrinking cost per
step; the warm runs not settled within the budget then run cold in a third
batch, whose wall time is counted on the warm side.  Batch set-up (which
uploads the initial densities) is outside the timed region on both sides.

Prints one JSON line with the per-instance steps and times, the fallbacks,
the saturation differences and the totals.
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


def settle(solver, cap, check=1000, tol=1e-6, min_steps=2000):
    """Advance one solver in graph replays of `check` steps until its window
    saturation (weighted, non-wetting) changes by less than tol per check.
    Returns (steps, settled, S_nw, wall seconds); a non-finite density ends
    the run unsettled."""
    import torch
    torch.cuda.synchronize()
    t0 = time.time()
    prev = 1.0 - solver.observables()["s_w_weighted"]
    t = 0
    while t < cap:
        solver.step_graph(check, 1)
        t += check
        o = solver.observables(allow_unstable=True)
        if o["flags"] & 1:
            return t, False, float("nan"), time.time() - t0
        s = 1.0 - o["s_w_weighted"]
        if t >= min_steps and abs(s - prev) < tol:
            return t, True, s, time.time() - t0
        prev = s
    return t, False, prev, time.time() - t0


def settle_batch(batch, cap, check=1000, tol=1e-6, min_steps=2000):
    """settle() for every instance of a batch at once: an instance is retired
    from the batch as soon as it settles or its density becomes non-finite,
    and the batch runs until none is left or the cap.  Returns per-instance
    steps, settled flags and S_nw (NaN where non-finite), and the wall
    seconds."""
    import torch
    torch.cuda.synchronize()
    t0 = time.time()
    prev = [1.0 - o["s_w_weighted"] for o in batch.observables()]
    k = len(prev)
    steps, ok, snw, done = [cap] * k, [False] * k, list(prev), [False] * k
    t = 0
    while t < cap and not all(done):
        batch.step_graph(check, 1)
        t += check
        changed = False
        for i, o in enumerate(batch.observables(allow_unstable=True)):
            if done[i]:
                continue
            if o["flags"] & 1:
                done[i], steps[i], snw[i], changed = True, t, float("nan"), True
                continue
            s = 1.0 - o["s_w_weighted"]
            if t >= min_steps and abs(s - prev[i]) < tol:
                done[i], ok[i], steps[i], snw[i], changed = True, True, t, s, True
            prev[i] = s
        if changed and not all(done):
            batch.set_active([not d for d in done])
    for i in range(k):
        if not done[i]:
            snw[i] = prev[i]
    return steps, ok, snw, time.time() - t0


def measure_batched(probs, sat, infer_s, cap, budget, s_tol, log):
    """The batched comparison (see the module docstring)."""
    from paper_2111_08666_amd import inputs as I
    from paper_2111_08666_amd import lbm
    from paper_2111_08666_amd import surrogate as S

    n = len(probs)
    warm_probs = []
    for p, s in zip(probs, sat):
        q = I.Problem(**{f: getattr(p, f) for f in p.__dataclass_fields__})
        q.rho0 = S.warm_start_density(p, s)
        warm_probs.append(q)
    b = lbm.BatchSolver(probs)
    cs, cok, cS, cw = settle_batch(b, cap)
    b.close()
    b = lbm.BatchSolver(warm_probs)
    ws, wok, wS, ww = settle_batch(b, budget)
    b.close()
    back = [i for i in range(n) if not wok[i]]
    fw, fS = 0.0, {}
    if back:
        b = lbm.BatchSolver([probs[i] for i in back])
        fs, fok, fSs, fw = settle_batch(b, cap)
        b.close()
        fS = dict(zip(back, fSs))
    final = [fS[i] if i in fS else wS[i] for i in range(n)]
    agree = [i for i in range(n) if cok[i] and abs(final[i] - cS[i]) <= s_tol]
    warm_total = ww + fw + infer_s
    log(f"[warmstart] batched: cold {cw:.2f} s (max {max(cs)} steps), warm {ww:.2f} s + fallback {fw:.2f} s "
        f"({len(back)} instances) + inference {infer_s * 1e3:.1f} ms")
    return {"cold_over_warm_wall": round(cw / warm_total, 3) if warm_total > 0 else None,
            "wall_s": {"cold": round(cw, 3), "warm": round(ww, 3), "fallback_cold": round(fw, 3),
                       "inference": round(infer_s, 4), "warm_with_fallback": round(warm_total, 3)},
            "steps_max": {"cold": int(max(cs)), "warm": int(max(ws))},
            "cold_settled": int(sum(cok)), "fallbacks": len(back), "agree_within_s_tol": len(agree)}


def measure(first=2000, count=32, cap=300000, budget=100000, s_tol=0.01, log=None, batched=True):
    """Runs the comparison and returns the result record (see the module
    docstring); `log` receives the progress lines."""
    import torch
    from paper_2111_08666_amd import inputs as I
    from paper_2111_08666_amd import lbm
    from paper_2111_08666_amd import surrogate as S

    log = log or (lambda m: print(m, file=sys.stderr, flush=True))
    probs = [p for p in (I.surrogate_instance(k) for k in range(first, first + count)) if p.theta < 90.0]
    n = len(probs)
    net = S.UNet.load(WEIGHTS)
    S.predict(net, probs[:1])  # first call loads the kernels
    torch.cuda.synchronize()
    t0 = time.time()
    sat = S.predict(net, probs)
    torch.cuda.synchronize()
    infer_s = time.time() - t0
    log(f"[warmstart] {n} instances; inference {infer_s * 1e3:.1f} ms")
    rec = []
    for i, p in enumerate(probs):
        cold = lbm.Solver(p)
        cs, cok, cS, cw = settle(cold, cap)
        cold.close()
        warm = lbm.Solver(p)
        warm.init_from_saturation(S.full_saturation(p, sat[i]))
        ws, wok, wS, ww = settle(warm, budget)
        warm.close()
        fell_back = not wok
        r = {"theta": round(float(p.theta), 2), "cold_steps": cs, "cold_settled": cok, "cold_s": round(cw, 4),
             "warm_steps": ws, "warm_settled": wok, "fell_back": fell_back,
             "warm_total_steps": ws + (cs if fell_back else 0),
             "warm_total_s": round(ww + (cw if fell_back else 0.0) + infer_s / n, 4),
             "abs_dS": round(abs(cS - (cS if fell_back else wS)), 5) if cok else None}
        rec.append(r)
        log(f"[warmstart] {i}: theta {r['theta']} cold {cs} steps {cw:.2f} s ({'settled' if cok else 'cap'}), "
            f"warm {ws} steps {ww:.2f} s ({'settled' if wok else 'fallback'}), |dS| {r['abs_dS']}")
    both = [r for r in rec if r["cold_settled"]]
    agree = [r for r in both if r["abs_dS"] is not None and r["abs_dS"] <= s_tol]
    ratios = [r["cold_steps"] / r["warm_total_steps"] for r in both]
    cold_s = sum(r["cold_s"] for r in rec)
    warm_s = sum(r["warm_total_s"] for r in rec)
    bat = measure_batched(probs, sat, infer_s, cap, budget, s_tol, log) if batched else None
    return {
        "metric": "time to steady state, cold start / U-Net warm start with fallback (wall, all instances)",
        "value": round(cold_s / warm_s, 3) if warm_s > 0 else None, "unit": "x", "higher_is_better": True,
        "config": {"workload": f"{n} held-out D2Q9 drainage instances 256x256, contact angle < 90 deg",
                   "excluded": "contact angle >= 90 deg: neither start settles within the cap",
                   "indices": [first, first + count], "cap": cap, "warm_budget": budget, "check": 1000,
                   "tol": 1e-6, "s_tol": s_tol},
        "cold_settled": len(both), "fallbacks": sum(r["fell_back"] for r in rec),
        "agree_within_s_tol": len(agree),
        "steps_median_ratio": round(float(np.median(ratios)), 3) if ratios else None,
        "steps_total": {"cold": int(sum(r["cold_steps"] for r in rec)),
                        "warm_with_fallback": int(sum(r["warm_total_steps"] for r in rec))},
        "wall_s": {"cold": round(cold_s, 3), "warm_with_fallback": round(warm_s, 3),
                   "inference": round(infer_s, 4)},
        "instances": rec,
        "batched": bat,
    }


def summary(w):
    """The record's headline fields, as bench.py reports them."""
    return {"cold_over_warm_wall": w["value"], "unit": "x", "workload": w["config"]["workload"],
            "excluded": w["config"]["excluded"],
            "criterion": "window saturation change < 1e-6 per 1000 steps; a warm run not settled within "
                         f"{w['config']['warm_budget']} steps falls back to the cold start (cost counted)",
            "cold_settled": w["cold_settled"], "fallbacks": w["fallbacks"],
            "agree_within_s_tol": w["agree_within_s_tol"], "s_tol": w["config"]["s_tol"],
            "steps_median_ratio": w["steps_median_ratio"], "steps_total": w["steps_total"],
            "wall_s": w["wall_s"], "cap": w["config"]["cap"], "batched": w.get("batched")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--first", type=int, default=2000)
    ap.add_argument("--count", type=int, default=32)
    ap.add_argument("--cap", type=int, default=300000)
    ap.add_argument("--budget", type=int, default=100000)
    ap.add_argument("--s-tol", type=float, default=0.01)
    a = ap.parse_args()
    print(json.dumps(measure(a.first, a.count, a.cap, a.budget, a.s_tol)), flush=True)


if __name__ == "__main__":
    main()
