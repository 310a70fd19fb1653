"""A benchmark workload run as a simulation: the named drainage advanced for
`--steps` steps (autotuned variant, HIP-graph replays), with the FP64 GPU
observables read every `--every` steps: window saturations, face pressures
and capillary pressure (Eq. 14), both masses, and the flags word.

    python -m paper_2111_08666_amd.drainage_run --workload d3q19_384 --steps 50000 --every 5000

Workloads are bench.py's.  Prints one progress line per record and one JSON
line (the records, the kernel, the wall time and the step rate).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def run(workload, steps, every, chunk=100, log=print):
    import torch
    from bench import workload as make
    from paper_2111_08666_amd import lbm
    p = make(workload)
    if isinstance(p, list):
        raise ValueError("a single-instance workload is needed")
    if every % chunk or steps % every:
        raise ValueError("steps must be a multiple of every, every a multiple of chunk")
    s = lbm.Solver(p)
    recs = []
    try:
        tune = s.autotune(10)
        kernel = s.kernel_info()[0]
        t_tuned = s.t
        torch.cuda.synchronize()
        t0 = time.time()

        def record():
            o = s.observables(allow_unstable=True)
            recs.append({k: o[k] for k in ("step", "s_w", "s_w_weighted", "p_in", "p_out", "pc", "mass", "flags")})
            log(f"[drainage_run] {workload} step {o['step']}: S_w {o['s_w']:.5f} (weighted "
                f"{o['s_w_weighted']:.5f}) P_c {o['pc']:+.6f} mass {o['mass'][0]:.6e} {o['mass'][1]:.6e} "
                f"flags {o['flags']} ({time.time() - t0:.0f}s)")
            return o["flags"]

        record()
        while s.t - t_tuned < steps:
            s.step_graph(chunk, every // chunk)
            if record() & 1:
                break
        torch.cuda.synchronize()
        wall = time.time() - t0
        done = s.t - t_tuned
    finally:
        s.close()
    return {"workload": workload, "nx": p.nx, "ny": p.ny, "nz": p.nz, "n_fluid": p.n_fluid, "kernel": kernel,
            "autotune": tune.strip().splitlines(), "steps": done, "every": every, "wall_s": round(wall, 2),
            "mlups_incl_observables": round(p.n_nodes * done / wall / 1e6, 1), "records": recs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="d3q19_384")
    ap.add_argument("--steps", type=int, default=50000)
    ap.add_argument("--every", type=int, default=5000)
    ap.add_argument("--chunk", type=int, default=100)
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    res = run(a.workload, a.steps, a.every, a.chunk, log=log)
    print(json.dumps(res), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
