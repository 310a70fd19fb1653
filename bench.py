"""Benchmark of the two-component LBM step on one MI355X.

Headline workload (default): D3Q19 on a 384^3 Boolean sphere pack (radii
6-14, porosity 0.4, seed 5), viscosity ratio 10, contact angle 60 degrees,
pressure-driven drainage (Set-3 inlet/outlet), with the state resident in
HBM (about 15 GB of populations).  The timed region replays HIP graphs of the
step on the solver's stream.

Prints one JSON line: MLUPS over all lattice nodes (both components per
node), the roofline of the step (algorithmic bytes per step / step duration
from HIP events on the solver's stream around the timed replays), the FP64
oracle timed on the host cores as a CPU baseline, and side measurements
(an all-fluid periodic 384^3 box, the 64-instance D2Q9 batch and the
cache-resident D2Q9 1024x512 drainage).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per fluid node and step: every population read once and
# written once (two components)
BYTES_PER_NODE = {(9, 0): 2 * 9 * 2 * 4, (9, 1): 2 * (8 * 2 + 4) * 2,
                  (19, 0): 2 * 19 * 2 * 4, (19, 1): 2 * (18 * 2 + 4) * 2}
METRIC = "MLUPS (2-component step) + % HBM roofline; time-to-steady w/ vs w/o warm start"


def kernel_source_hash():
    from paper_2111_08666_amd.build import kernel_source_hash as h
    return h()


def workload(name):
    """A Problem, or a list of Problems for a batched workload."""
    from paper_2111_08666_amd import inputs as I
    if name == "batch64":
        return I.batch_instances(64)
    if name == "d2q9_1024x512":
        return I.large_drainage(collision=1)
    if name == "d2q9_128x64":
        return I.small_drainage()
    if name.startswith("d3q19_box"):
        return I.fluid_box_3d(n=int(name[len("d3q19_box"):] or 384))
    if name.startswith("d3q19_"):
        return I.drainage_3d(n=int(name.split("_")[1]))
    raise SystemExit(f"unknown workload {name}")


def traffic_for(kernel, wl):
    """Measured HBM bytes per step from committed counter summaries, if they
    were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    rec = data.get(f"{kernel}|{wl}")
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(problem, sample, seconds=12.0):
    import oracle as O
    s = O.OracleSim(problem)
    s.step(2)  # warm
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        s.step(5)
        steps += 5
    dt = time.perf_counter() - t0
    return {"value": round(problem.n_nodes * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} steps of {sample} ({problem.nx}x{problem.ny}x{problem.nz}, FP64 oracle, "
                      f"OpenMP over nodes, {dt:.1f} s)"}


def make_solver(lbm, problem, args, dev, math=None):
    kw = dict(storage=args.storage, device=dev, math=args.math if math is None else math,
              strategy=args.strategy, tile_rows=args.tile_rows)
    if isinstance(problem, list):
        return lbm.BatchSolver(problem, **kw)
    return lbm.Solver(problem, **kw)


def time_steps(torch, solver, steps, warmup, chunk, eager):
    """Run `warmup` steps, then time exactly `steps` steps: graph replays of
    `chunk` steps (chunk even) plus an eager remainder.  Returns (wall s,
    event ms on the solver's stream)."""
    def run(n):
        full = 0 if eager else n // chunk
        if full:
            solver.step_graph(chunk, full)
        if n - full * chunk:
            solver.step(n - full * chunk)

    from paper_2111_08666_amd.roctx import rng
    with rng(f"warmup {warmup} steps"):
        run(warmup)
        torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with rng(f"timed {steps} steps"):
        t0 = time.perf_counter()
        e0.record(solver.stream)
        run(steps)
        e1.record(solver.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    return wall, e0.elapsed_time(e1)


def side_line(torch, lbm, name, args, dev, steps, warmup, chunk, math=None):
    """A shorter measurement of another workload, or of the same one with the
    other node arithmetic (same protocol)."""
    problem = workload(name)
    batch = isinstance(problem, list)
    solver = make_solver(lbm, problem, args, dev, math=math)
    try:
        if not args.no_autotune and args.strategy == 0:
            solver.autotune(10)
        wall, ev_ms = time_steps(torch, solver, steps, warmup, chunk, args.eager)
        kname = solver.kernel_info()[0]
        n_nodes = solver.n_nodes if batch else problem.n_nodes
        n_fluid = solver.n_fluid if batch else problem.n_fluid
        q = problem[0].q if batch else problem.q
        alg = BYTES_PER_NODE[(q, args.storage)] * n_fluid
        step_ms = ev_ms / steps
        out = {"workload": (f"batch of {len(problem)} D2Q9 drainage instances" if batch else problem.name),
               "n_nodes": n_nodes, "n_fluid": n_fluid, "steps": steps, "warmup": warmup,
               "ms_per_step": round(wall * 1e3 / steps, 5), "value": round(n_nodes * steps / wall / 1e6, 1),
               "unit": "MLUPS", "kernel": kname,
               "roofline_frac": round(alg / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "alg_bytes_per_step": alg, "traffic": traffic_for(kname, name),
               "math": "f32" if (args.math if math is None else math) == 0 else "f64"}
        if name == "d2q9_1024x512":
            out["note"] = ("both population buffers (75 MB) stay in the 256 MB last-level cache: "
                           "the fraction is of on-chip bandwidth, not of HBM")
        return out
    finally:
        solver.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--workload", default="d3q19_384")
    ap.add_argument("--chunk", type=int, default=20, help="steps per captured graph (even)")
    ap.add_argument("--storage", type=int, default=0, help="0 FP32, 1 BF16 deviations")
    ap.add_argument("--math", type=int, default=0, help="node arithmetic: 0 FP32 (default), 1 FP64")
    ap.add_argument("--strategy", type=int, default=0,
                    help="0 auto (autotuned), 1 fused, 2 split, 3 compact, 4 fused with listed collision, "
                         "5 compacted fused (D2Q9)")
    ap.add_argument("--tile-rows", type=int, default=0, help="fused D2Q9 tile height 8, 12 or 16 (0: 12)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--eager", action="store_true", help="plain launches instead of graphs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-side", action="store_true", help="skip the side workloads")
    ap.add_argument("--no-warm-start", action="store_true",
                    help="skip the time-to-steady comparison of a cold start and the U-Net warm start")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        raise SystemExit("--steps must be >= 1 and --warmup >= 0")

    import torch
    from paper_2111_08666_amd import lbm
    from paper_2111_08666_amd.roctx import rng

    dev = torch.device("cuda:0")
    chunk = max(2, args.chunk - args.chunk % 2)
    problem = workload(args.workload)
    batch = isinstance(problem, list)
    if batch:
        problems = problem
        solver = make_solver(lbm, problems, args, dev)
        n_nodes, n_fluid = solver.n_nodes, solver.n_fluid
        sizes = sorted({(p.nx, p.ny) for p in problems})
        q = problems[0].q
        print(f"[bench] workload {args.workload}: {len(problems)} instances, {sizes[0]} .. {sizes[-1]}, "
              f"{n_nodes} nodes, fluid {n_fluid}", file=sys.stderr, flush=True)
    else:
        print(f"[bench] workload {args.workload}: {problem.nx}x{problem.ny}x{problem.nz}, "
              f"fluid {problem.n_fluid}, collision {problem.collision}", file=sys.stderr, flush=True)
        solver = make_solver(lbm, problem, args, dev)
        n_nodes, n_fluid, q = problem.n_nodes, problem.n_fluid, problem.q
    tune = None
    if not args.no_autotune and args.strategy == 0:
        with rng("autotune"):
            tune = solver.autotune(10)
        print("[bench] autotune:\n" + tune, file=sys.stderr, flush=True)
    with rng(f"workload {args.workload}"):
        wall, ev_ms = time_steps(torch, solver, args.steps, args.warmup, chunk, args.eager)
    ms_per_step = wall * 1e3 / args.steps
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.4f} ms/step", file=sys.stderr, flush=True)

    # eager single launches bracketed by events, beside the timed replays
    n_samples = 20
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_samples)]
    for a, b in evs:
        a.record(solver.stream)
        solver.step(1)
        b.record(solver.stream)
    torch.cuda.synchronize()
    k_ms = sorted(a.elapsed_time(b) for a, b in evs)
    obs = solver.observables()
    mass = [sum(o["mass"][c] for o in obs) for c in range(2)] if batch else obs["mass"]
    kname, grid, block = solver.kernel_info()
    solver.close()

    bpn = BYTES_PER_NODE[(q, args.storage)]
    alg_bytes = bpn * n_fluid
    step_ms = ev_ms / args.steps
    achieved = alg_bytes / (step_ms * 1e-3) / 1e9
    traffic = traffic_for(kname, args.workload)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": kname,
                "step_ms_timed": round(step_ms, 5),
                "eager_launch_ms_median": round(k_ms[len(k_ms) // 2], 5),
                "alg_bytes_per_step": alg_bytes, "bytes_per_fluid_node": bpn}
    mlups = n_nodes * args.steps / wall / 1e6
    out = {
        "metric": METRIC,
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": ("f32" if args.math == 0 else "f64") + " node arithmetic, "
                 + ("f32" if args.storage == 0 else "bf16-deviation") + " storage",
        "data": "synthetic (seeded sphere/disc media; the paper's geometry is not available)",
        "config": {"workload": (f"batch of {len(problems)} D2Q9 drainage instances "
                                f"{sizes[0][0]}x{sizes[0][1]} .. {sizes[-1][0]}x{sizes[-1][1]}"
                                if batch else problem.name),
                   "q": q, "nx": None if batch else problem.nx, "ny": None if batch else problem.ny,
                   "nz": None if batch else problem.nz, "n_nodes": n_nodes, "n_fluid": n_fluid,
                   "collision": ["SRT", "MRT", "TRT"][(problems[0] if batch else problem).collision],
                   "storage": "f32" if args.storage == 0 else "bf16-dev",
                   "launch": "eager" if args.eager else f"hipGraph x{chunk}",
                   "mflups_fluid": round(n_fluid * args.steps / wall / 1e6, 1),
                   "mass_after": mass, "grid_blocks": grid, "block_threads": block,
                   "autotune": tune.strip().splitlines() if tune else None},
        "roofline": roofline,
    }
    if not args.no_side:
        side = {}
        for name, steps in (("d3q19_box384", 100), ("batch64", 400), ("d2q9_1024x512", 2000)):
            if name == args.workload:
                continue
            print(f"[bench] side workload {name}", file=sys.stderr, flush=True)
            with rng(f"side workload {name}"):
                side[name] = side_line(torch, lbm, name, args, dev, steps, max(10, steps // 10), chunk)
        other = 1 - args.math
        print(f"[bench] side: {args.workload} with {'FP64' if other else 'FP32'} node arithmetic",
              file=sys.stderr, flush=True)
        side[f"{args.workload}_{'f64' if other else 'f32'}_arithmetic"] = side_line(
            torch, lbm, args.workload, args, dev, min(args.steps, 200), 20, chunk, math=other)
        out["side"] = side
    if not args.no_cpu_baseline:
        if not batch and q == 19 and problem.nx > 64:
            from paper_2111_08666_amd import inputs as I
            sample, cpu_problem = "the same sphere-pack generator on a 64^3 domain", I.drainage_3d(n=64)
        elif batch:
            sample = "the median-size instance of the batch"
            cpu_problem = sorted(problems, key=lambda p: p.n_nodes)[len(problems) // 2]
        else:
            sample, cpu_problem = "the same workload", problem
        with rng("cpu baseline (oracle)"):
            out["cpu_baseline"] = cpu_baseline(cpu_problem, sample)
    if not args.no_warm_start:
        # after the timed region: held-out instances run to steady state from
        # the cold start and from the trained network's prediction
        from paper_2111_08666_amd import bench_warmstart
        with rng("time to steady state"):
            w = bench_warmstart.measure(log=lambda m: print(m, file=sys.stderr, flush=True))
        out["time_to_steady"] = bench_warmstart.summary(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
