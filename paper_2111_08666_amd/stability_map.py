"""Stability map of the collision operators against the viscosity ratio M
and the cohesion G, on the GPU.

    python -m paper_2111_08666_amd.stability_map [--steps 20000] [--out map.json] [--tune-mrt]

Each (collision, M, G) cell is one instance of a small pressure-driven
drainage (127 x 37 disc medium, porosity 0.7, 45 degrees, inlet density
1.02, Set-3) with the wetting component at nu = 0.04 (tau = 0.62, the
paper's water) and the invading component at M times that.  All cells of
one collision operator run as one batch; a cell counts as stable when no
density became non-finite or negative within the run, and its final
window saturation is reported.  D2Q9 SRT, MRT (Lallemand-Luo moments,
s_e = s_eps = 1, s_q from Lambda = 3/16, component-momentum rate
s_j = min(s_nu, s_q)) and TRT (Lambda = 3/16).  Prints one progress line per
operator and one JSON line.

--tune-mrt adds a sweep of the MRT operator's free rates at high viscosity
ratio (G = 3.5): the energy rates s_e = s_eps and the magic parameter
Lambda (which sets s_q), with the wetting viscosity 0.04, 0.01 or 0.005.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2111_08666_amd import inputs as I   # noqa: E402
from paper_2111_08666_amd import lbm           # noqa: E402

MS = (1, 10, 25, 100, 1000)
GS = (2.5, 3.0, 3.5, 4.0, 4.5)
NU_WET = 0.04


def tau_of_nu(nu):
    return 0.5 + 3.0 * nu


def cell(collision, M, G, nu_wet=NU_WET):
    p = I.drainage_2d(nx=127, ny=37, r=(2.0, 5.0), porosity=0.7, seed=11, G=G, theta=45.0,
                      tau=(tau_of_nu(M * nu_wet), tau_of_nu(nu_wet)), rho_in1=1.02, minor=0.027,
                      collision=collision, name=f"stab_c{collision}_M{M}_G{G}")
    return p


def tune_mrt(steps=20000, log=print):
    """Stable MRT rate choices at M = 100 and 1000, G = 3.5."""
    cells = [(M, nu, se, lam) for M in (100, 1000) for nu in (0.04, 0.01, 0.005)
             for se in (0.6, 0.8, 1.0, 1.2, 1.5) for lam in (1 / 12, 3 / 16, 1 / 4)]
    probs = []
    for M, nu, se, lam in cells:
        p = cell(1, M, 3.5, nu)
        p.s_e = p.s_eps = se
        p.lam = lam
        probs.append(p)
    t0 = time.time()
    b = lbm.BatchSolver(probs)
    b.step_graph(1000, steps // 1000)
    obs = b.observables(allow_unstable=True)
    b.close()
    out = [{"M": M, "nu_wetting": nu, "s_e": se, "lambda": lam, "stable": o["flags"] == 0,
            "flags": o["flags"], "s_w": o["s_w"] if o["flags"] == 0 else None}
           for (M, nu, se, lam), o in zip(cells, obs)]
    log(f"[stability] MRT rate sweep: {sum(c['stable'] for c in out)}/{len(out)} stable "
        f"({time.time() - t0:.1f}s)")
    return out


def run(steps=20000, log=print):
    out = {}
    for collision, name in ((0, "SRT"), (1, "MRT"), (2, "TRT")):
        cells = [(M, G) for M in MS for G in GS]
        t0 = time.time()
        b = lbm.BatchSolver([cell(collision, M, G) for M, G in cells])
        b.step_graph(1000, steps // 1000)
        obs = b.observables(allow_unstable=True)
        b.close()
        out[name] = {f"M{M}_G{G}": {"stable": o["flags"] == 0, "flags": o["flags"],
                                    "s_w": o["s_w"] if o["flags"] == 0 else None}
                     for (M, G), o in zip(cells, obs)}
        n_ok = sum(v["stable"] for v in out[name].values())
        log(f"[stability] {name}: {n_ok}/{len(cells)} cells stable after {steps} steps "
            f"({time.time() - t0:.1f}s)")
    return {"steps": steps, "M": MS, "G": GS, "nu_wetting": NU_WET, "map": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--out", default="")
    ap.add_argument("--tune-mrt", action="store_true")
    a = ap.parse_args()
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    res = run(a.steps, log=log)
    if a.tune_mrt:
        res["mrt_rates"] = tune_mrt(a.steps, log=log)
    print(json.dumps(res), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
