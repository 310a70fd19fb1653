"""Capillary pressure - water saturation curve of the 1024x512 disc medium
(its one-node throats closed): primary drainage, then imbibition, by
stepwise pressure increments (Sec. 4.2, Figs. 10 and 12), on one GPU.

    python -m paper_2111_08666_amd.pc_sw_curve [--size 1024x512] [--steps 200000] [--audit 1000] [--out curve.json]
        [--all-increments] [--raw-medium] [--locate-blowup] [--collision 2] [--lam 0.1875]

Drainage raises the inlet density of component 1 (the invading oil) over
ten levels, rho_in1 = 1 + 3 dP with dP from 1e-3 to 2e-2 (geometric), each
level continuing from the state the previous one left (Sec. 4.2.1).
Imbibition then lowers rho_in1 back to 1 in five levels (P_c down to zero:
spontaneous imbibition) and raises the outlet density of component 2 in five
levels (negative P_c: forced imbibition), the sequence Sec. 4.2.2 describes.

At the end of each increment the measured P_c = P_in - P_out (Eq. 14
pressures at the faces) and the window saturations are recorded.  Every
`audit` steps the FP64 GPU sums are read: both components' masses and the
flags word (a non-finite or negative density).  Prints one progress line per
increment and one JSON line.
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

from paper_2111_08666_amd import inputs as I   # noqa: E402
from paper_2111_08666_amd import lbm           # noqa: E402

DRAIN_DP = tuple(float(v) for v in np.geomspace(1e-3, 2e-2, 10))
IMB_IN_DP = (1e-2, 5e-3, 2e-3, 1e-3, 0.0)        # rho_in1 = 1 + 3 dP, rho_out2 = 1
IMB_OUT_DP = (1e-3, 2e-3, 5e-3, 1e-2, 2e-2)      # rho_in1 = 1, rho_out2 = 1 + 3 dP


def schedule():
    """[(phase, rho_in1, rho_out2)] of the twenty increments."""
    s = [("drainage", 1.0 + 3 * dp, 1.0) for dp in DRAIN_DP]
    s += [("imbibition", 1.0 + 3 * dp, 1.0) for dp in IMB_IN_DP]
    s += [("imbibition", 1.0, 1.0 + 3 * dp) for dp in IMB_OUT_DP]
    return s


def study_problem(nx=1024, ny=512, xi=-0.4, close=True):
    """The drainage medium (1024x512: the benchmark's; other sizes: the same
    recipe, radii 4-20, porosity 0.55, seed 2) with its under-resolved pores
    closed (inputs.close_narrow_throats).  In the unmodified 1024x512
    medium the first imbibition increment went non-finite twice: the water
    density grew to 3.9 in a one-node throat at x = 236, then (throats
    closed) to 1.4 beside a negative oil density in a 2x2 pocket reached
    only through diagonal links at x = 625.  close=False keeps the medium as
    generated."""
    if (nx, ny) == (1024, 512):
        p = I.large_drainage()
    else:
        p = I.drainage_2d(nx=nx, ny=ny, r=(4.0, 20.0), porosity=0.55, seed=2, G=3.5,
                          theta=I.theta_of_xi(xi), tau=I.TAU_M10, rho_in1=1.0 + 3 * 1e-3, rho_out2=1.0,
                          minor=0.027, collision=1, name=f"d2q9_{nx}x{ny}_drainage_M10")
    p.xi = xi
    if close:
        p.mask = I.close_narrow_throats(p.mask)
        p.rho0 = I.reservoir_front(p.mask, p.porous_x0, 1.0, 0.027)
        p.name += "_throats_closed"
    return p


def _reservoir_fraction(rho, fl, cols, c):
    """Mean share of component c over the fluid nodes of columns `cols`."""
    r = rho[:, :, cols]
    f = fl[:, cols]
    return float((r[c][f] / (r[0][f] + r[1][f])).mean())


def _extremes(rho, fl):
    """Where each component's density is largest and smallest over the fluid."""
    out = {}
    for c in (0, 1):
        r = np.where(fl, rho[c], np.nan)
        for name, f in (("max", np.nanargmax), ("min", np.nanargmin)):
            y, x = np.unravel_index(int(f(r)), r.shape)
            out[f"rho{c + 1}_{name}"] = {"value": float(r[y, x]), "x": int(x), "y": int(y)}
    return out


def locate_blowup(s, blob, fl, audit):
    """Replays the audit interval that went non-finite one step at a time from
    the checkpoint `blob` taken at its start.  Returns the first step with a
    non-finite density, the nodes that hold one then, and where the densities
    were extreme one step and `audit` steps before."""
    s.load(blob)
    t0 = s.t
    first = s.density()
    prev = first
    for k in range(audit):
        s.step(1)
        o = s.observables(allow_unstable=True)
        if o["flags"] & 1:
            rho = s.density()
            bad = ~np.isfinite(rho).all(axis=0) & fl
            ys, xs = np.nonzero(bad)
            return {"step": t0 + k + 1, "count": int(bad.sum()),
                    "nodes": [[int(x), int(y)] for x, y in list(zip(xs, ys))[:16]],
                    "extremes_one_step_before": _extremes(prev, fl),
                    "extremes_at_interval_start": _extremes(first, fl)}
        prev = s.density()
    return None


def run(steps=200000, audit=1000, problem=None, log=print, stop_at_breakthrough=True, locate=False):
    """Breakthrough ends a phase: drainage when component 1 makes up a
    quarter of the outlet reservoir, imbibition when component 2 makes up a
    quarter of the inlet reservoir (checked at every audit).  Past it the
    displacing phase reaches the face where Set-3 imposes the other
    component's density.  stop_at_breakthrough=False records breakthrough
    but runs every increment in full (only a non-finite density stops).
    locate=True checkpoints the state at every audit, so that a blow-up can
    be replayed step by step (locate_blowup)."""
    if steps % audit:
        raise ValueError("steps must be a multiple of the audit interval")
    p = problem if problem is not None else study_problem()
    s = lbm.Solver(p)
    fl = p.mask == 0
    res_in = slice(0, p.porous_x0)
    res_out = slice(p.porous_x1, p.nx)
    rec = []
    t0 = time.time()
    done = set()
    try:
        kernel = s.kernel_info()[0]
        for k, (phase, rin, rout) in enumerate(schedule()):
            if phase in done:
                continue
            s.set_bc(rin, rout)
            m1, m2, flags, sw_hist, through, blowup = [], [], 0, [], False, None
            for a in range(steps // audit):
                blob = s.save() if locate else None
                s.step_graph(audit, 1)
                o = s.observables(allow_unstable=True)
                m1.append(o["mass"][0])
                m2.append(o["mass"][1])
                flags |= o["flags"]
                sw_hist.append(o["s_w_weighted"])
                if o["flags"] & 1:
                    if locate:
                        blowup = locate_blowup(s, blob, fl, audit)
                        log(f"[pc_sw] blow-up: {json.dumps(blowup)}")
                    break
                rho = s.density()
                if phase == "drainage":
                    through = _reservoir_fraction(rho, fl, res_out, 0) > 0.25
                else:
                    through = _reservoir_fraction(rho, fl, res_in, 1) > 0.25
                if through and stop_at_breakthrough:
                    done.add(phase)
                    break
            o = s.observables(allow_unstable=True)
            rho = s.density().astype(np.float64)
            fl = p.mask == 0
            inlet = {f"x{x}": [float(rho[c][:, x][fl[:, x]].mean()) for c in (0, 1)] for x in (0, 1, 8, 16)}
            bad = ~np.isfinite(rho).all(axis=0) & fl
            where = None
            if bad.any():
                ys, xs = np.nonzero(bad)
                where = {"count": int(bad.sum()), "x": [int(xs.min()), int(xs.max())],
                         "y": [int(ys.min()), int(ys.max())]}
            r = {"increment": k, "phase": phase, "rho_in1": rin, "rho_out2": rout,
                 "pc_set": (rin - rout) / 3.0, "pc": o["pc"], "p_in": o["p_in"], "p_out": o["p_out"],
                 "s_w": o["s_w"], "s_w_weighted": o["s_w_weighted"], "step": o["step"],
                 "ds_w_last_10k": abs(sw_hist[-1] - sw_hist[-11]) if len(sw_hist) > 10 else None,
                 "mass_audit": {"n": len(m1), "mass1_min": min(m1), "mass1_max": max(m1),
                                "mass2_min": min(m2), "mass2_max": max(m2),
                                "finite": bool(np.all(np.isfinite(m1 + m2))), "flags": flags},
                 "column_means": inlet, "non_finite": where, "breakthrough": through, "blowup": blowup,
                 "stag": o["stag"]}
            rec.append(r)
            log(f"[pc_sw] {k:2d} {phase:10s} rho_in1 {rin:.4f} rho_out2 {rout:.4f}: P_c {r['pc']:+.5f} "
                f"S_w {r['s_w']:.4f} (weighted {r['s_w_weighted']:.4f}) stag_x {o['stag'][0]:+.1e} flags {flags}"
                f"{' breakthrough' if through else ''} ({time.time() - t0:.0f}s)")
            if flags & 1:
                break
    finally:
        s.close()
    return {"workload": p.name, "nx": p.nx, "ny": p.ny, "steps_per_increment": steps, "audit_every": audit,
            "kernel": kernel, "G": p.G, "xi": p.xi, "tau": list(p.tau), "collision": p.collision, "lam": p.lam,
            "stop_at_breakthrough": stop_at_breakthrough, "wall_s": round(time.time() - t0, 1), "increments": rec}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=200000)
    ap.add_argument("--audit", type=int, default=1000)
    ap.add_argument("--size", default="1024x512", help="medium size NXxNY (1024x512: the benchmark's)")
    ap.add_argument("--xi", type=float, default=-0.4,
                    help="adhesion (-0.4: about 50 degrees, Sec. 4.2.1; -0.55: about 22; 0.2: about 110)")
    ap.add_argument("--out", default="")
    ap.add_argument("--all-increments", action="store_true",
                    help="run all twenty increments in full, past breakthrough")
    ap.add_argument("--raw-medium", action="store_true", help="keep the medium's narrow throats open")
    ap.add_argument("--locate-blowup", action="store_true",
                    help="checkpoint every audit and replay a blow-up step by step")
    ap.add_argument("--collision", type=int, default=None, help="0 SRT, 1 MRT (the default), 2 TRT")
    ap.add_argument("--lam", type=float, default=None, help="TRT/MRT magic parameter (default 3/16)")
    a = ap.parse_args()
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    nx, ny = (int(v) for v in a.size.split("x"))
    prob = study_problem(nx, ny, a.xi, close=not a.raw_medium)
    if a.collision is not None:
        prob.collision = a.collision
    if a.lam is not None:
        prob.lam = a.lam
    res = run(a.steps, a.audit, problem=prob, log=log, stop_at_breakthrough=not a.all_increments,
              locate=a.locate_blowup)
    print(json.dumps(res), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
