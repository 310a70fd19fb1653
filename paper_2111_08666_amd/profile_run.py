"""Driver for hardware-counter and trace runs of the step kernel.

    python -m paper_2111_08666_amd.profile_run --workload d2q9_1024x512 --steps 20

Creates the solver for a named workload (the same inputs as bench.py), runs
one warm-up step and then `--steps` steps, then (with --copy-mib) a plain
device-to-device copy of a known size, whose counters calibrate the memory
traffic counters.  Prints one progress line per stage.
"""
import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="d2q9_1024x512")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--math", type=int, default=0)
    ap.add_argument("--storage", type=int, default=0)
    ap.add_argument("--strategy", type=int, default=0, help="0 auto, 1 fused, 2 split")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--copy-mib", type=int, default=0)
    args = ap.parse_args()
    import torch
    from bench import workload
    from paper_2111_08666_amd import lbm
    t0 = time.time()
    p = workload(args.workload)
    if isinstance(p, list):
        s = lbm.BatchSolver(p, storage=args.storage, math=args.math, strategy=args.strategy,
                            tile_rows=args.tile_rows)
    else:
        s = lbm.Solver(p, storage=args.storage, math=args.math, strategy=args.strategy,
                       tile_rows=args.tile_rows)
    print(f"[profile_run] {args.workload} ready in {time.time() - t0:.1f}s; kernel {s.kernel_info()}",
          flush=True)
    s.step(1)
    torch.cuda.synchronize()
    s.step(args.steps)
    torch.cuda.synchronize()
    print(f"[profile_run] {args.steps} steps done", flush=True)
    if args.copy_mib:
        n = args.copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"[profile_run] copied {args.copy_mib} MiB x3", flush=True)


if __name__ == "__main__":
    main()
