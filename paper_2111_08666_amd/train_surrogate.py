"""Data generation, training and the warm-start evaluation of the U-Net
surrogate, all on the GPU through liblbm.so.

    python -m paper_2111_08666_amd.train_surrogate gen   --first 0 --count 2000 --out data.npz
    python -m paper_2111_08666_amd.train_surrogate train --data data.npz --out weights.npz
    python -m paper_2111_08666_amd.train_surrogate eval  --weights weights.npz --first 2000 --count 32

gen:   runs instances (inputs.surrogate_instance) from the cold start, many
       per launch (BatchSolver), until the window saturation changes by less
       than --tol per --check steps, and stores the steady non-wetting
       fraction rho1 / (rho1 + rho2) per node (uint8, 1/255 steps).
train: Adam on the masked cross-entropy, mini-batches of --batch fields,
       vertical mirror images as augmentation (a symmetry of the problem).
eval:  the same held-out instances from the cold start and from the
       network's prediction, both to the same steadiness criterion; reports
       steps to steady and the saturation difference.

Each stage prints one progress line per unit of work.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2111_08666_amd import inputs as I          # noqa: E402
from paper_2111_08666_amd import lbm                  # noqa: E402
from paper_2111_08666_amd import surrogate as S       # noqa: E402


def log(msg):
    print(msg, flush=True)


def make_masks(idx, n=256, workers=8):
    """Solid maps of the given instances.  Worker processes are forked here,
    before this process touches the GPU."""
    idx = [int(k) for k in idx]
    if workers > 1 and len(idx) > 8:
        from multiprocessing import Pool
        with Pool(workers) as pool:
            return pool.starmap(I.surrogate_mask, [(k, 40000, n) for k in idx])
    return [I.surrogate_mask(k, 40000, n) for k in idx]


def make_instances(idx, masks, n=256):
    return [I.surrogate_instance(int(k), 40000, n, mask=m) for k, m in zip(idx, masks)]


def run_to_steady(problems, cap, check=1000, tol=1e-6, min_steps=2000, storage=lbm.STORE_F32, tag="",
                  run_all=False):
    """Advance all problems in one batch until each one's window saturation
    (weighted, non-wetting) changes by less than tol over `check` steps.
    A settled instance is retired from the batch (it costs nothing more and
    its state stays as it settled) unless run_all asks for trajectories to the
    cap; an instance whose density becomes non-finite is retired at once and
    reported as None, and the rest go on.  Returns per-instance (steps,
    converged, S_nw, density) and the S_nw trajectory (k x checks, constant
    after an instance settles, NaN for a failed one)."""
    k = len(problems)
    b = lbm.BatchSolver(problems, storage=storage)
    prev = [1.0 - o["s_w_weighted"] for o in b.observables()]
    traj = [list(prev)]
    steps = [cap] * k
    conv = [False] * k
    failed = [False] * k
    snw = list(prev)
    dens = [None] * k
    t = 0
    t0 = time.time()
    while t < cap and (run_all or not all(c or f for c, f in zip(conv, failed))):
        b.step_graph(check, 1)
        t += check
        obs = b.observables(allow_unstable=True)
        bad = [i for i, o in enumerate(obs) if o["flags"] & 1 and not failed[i]]
        if bad:
            log(f"[steady{tag}] non-finite density in instances {bad} at t={t}: retired")
            for i in bad:
                failed[i] = True
        changed = bool(bad)
        for i, o in enumerate(obs):
            if failed[i]:
                continue
            s = 1.0 - o["s_w_weighted"]
            if not conv[i] and t >= min_steps and abs(s - prev[i]) < tol:
                conv[i], steps[i], snw[i] = True, t, s
                dens[i] = b.density(i)
                changed = changed or not run_all
            prev[i] = s
        if changed:
            b.set_active([not f and (run_all or not c) for c, f in zip(conv, failed)])
        traj.append(list(prev))
        if t % (10 * check) == 0:
            log(f"[steady{tag}] t={t} converged {sum(conv)}/{k} ({time.time() - t0:.0f}s)")
    for i in range(k):
        if not conv[i] and not failed[i]:
            snw[i] = prev[i]
            dens[i] = b.density(i)
    b.close()
    traj = np.array(traj).T
    for i in range(k):
        if failed[i]:
            steps[i] = conv[i] = snw[i] = dens[i] = None
            traj[i] = np.nan
    return steps, conv, snw, dens, traj


def cmd_gen(a):
    t0 = time.time()
    all_idx = list(range(a.first, a.first + a.count))
    masks = make_masks(all_idx, a.n, a.workers)
    log(f"[gen] {a.count} media built ({time.time() - t0:.0f}s)")
    for g0 in range(a.first, a.first + a.count, a.batch):
        idx_all, tgt_all, steps_all, conv_all, s_all = [], [], [], [], []
        cnt = min(a.batch, a.first + a.count - g0)
        probs = make_instances(range(g0, g0 + cnt), masks[g0 - a.first:g0 - a.first + cnt], a.n)
        steps, conv, snw, dens, traj = run_to_steady(probs, a.cap, a.check, a.tol, tag=f" {g0}",
                                                     run_all=a.run_all)
        for i, p in enumerate(probs):
            if dens[i] is None:
                continue
            sat = S.saturation_field(dens[i])
            idx_all.append(g0 + i)
            tgt_all.append(np.rint(np.clip(sat, 0, 1) * 255).astype(np.uint8))
            steps_all.append(steps[i])
            conv_all.append(conv[i])
            s_all.append(snw[i])
        log(f"[gen] batch {g0}: converged {sum(conv_all)}/{cnt}, kept {len(idx_all)}, median steps "
            f"{int(np.median(steps_all))}, S_nw range [{min(s_all):.3f}, {max(s_all):.3f}] "
            f"({time.time() - t0:.0f}s)")
        out = a.out.replace(".npz", "") + f"_{g0}.npz"
        np.savez_compressed(out, idx=np.array(idx_all), target=np.stack(tgt_all), steps=np.array(steps_all),
                            converged=np.array(conv_all), s_nw=np.array(s_all), n=a.n, cap=a.cap,
                            traj=traj[[i for i in range(cnt) if dens[i] is not None]].astype(np.float32),
                            check=a.check, tol=a.tol)
        log(f"[gen] wrote {out}: {len(idx_all)} fields")


def load_data(paths, workers):
    idx, tgt = [], []
    for p in paths:
        with np.load(p, allow_pickle=False) as z:
            idx.append(z["idx"])
            tgt.append(z["target"])
            n = int(z["n"])
    idx = np.concatenate(idx)
    tgt = np.concatenate(tgt)
    probs = make_instances(idx, make_masks(idx, n, workers), n)
    x = np.stack([S.features(p.mask, p.theta, p.dp) for p in probs])
    m = np.stack([(p.mask == 0).astype(np.uint8) for p in probs])
    return idx, x, tgt.astype(np.float32) / 255.0, m


def cmd_train(a):
    import torch
    t0 = time.time()
    idx, x, t, m = load_data(a.data, a.workers)
    nval = max(1, int(len(idx) * a.val_frac))
    log(f"[train] {len(idx)} fields ({nval} for validation) loaded in {time.time() - t0:.0f}s")
    dev = torch.device("cuda:0")
    X = torch.from_numpy(S.bf16_bits(x).view(np.int16)).to(dev)
    T = torch.from_numpy(t).to(dev)
    M = torch.from_numpy(m).to(dev)
    counts = m.reshape(len(idx), -1).sum(axis=1).astype(np.int64)
    tr = np.arange(nval, len(idx))
    va = np.arange(nval)
    net = S.UNet(seed=a.seed)
    rng = np.random.default_rng(a.seed)
    steps_per_epoch = len(tr) // a.batch
    total = steps_per_epoch * a.epochs
    flops = 3 * net.flops_per_image(x.shape[1], x.shape[2]) * a.batch
    it = 0
    history = []
    t_start = time.time()
    for ep in range(a.epochs):
        if a.max_minutes and time.time() - t_start > 60 * a.max_minutes:
            log(f"[train] time budget of {a.max_minutes} min reached after {ep} epochs")
            break
        perm = rng.permutation(tr)
        torch.cuda.synchronize()
        te = time.time()
        losses = []
        for s in range(steps_per_epoch):
            sel = torch.from_numpy(perm[s * a.batch:(s + 1) * a.batch]).to(dev)
            xb, tb, mb = X.index_select(0, sel), T.index_select(0, sel), M.index_select(0, sel)
            if rng.uniform() < 0.5:                   # mirror in y
                xb, tb, mb = xb.flip(1), tb.flip(1), mb.flip(1)
            xb, tb, mb = xb.contiguous(), tb.contiguous(), mb.contiguous()
            lr = a.lr * 0.5 * (1 + np.cos(np.pi * it / total))
            cnt = int(counts[perm[s * a.batch:(s + 1) * a.batch]].sum())
            losses.append(net.train_step(xb, tb, mb, lr=lr, count=cnt).clone())
            it += 1
        torch.cuda.synchronize()
        dt = time.time() - te
        tl = float(torch.stack(losses).mean().item())
        vl, vacc, vs = evaluate(net, X, T, M, va, a.batch)
        history.append({"epoch": ep, "train_loss": tl, "val_loss": vl, "val_acc": vacc, "val_sat_err": vs,
                        "s_per_epoch": dt, "tflops": flops * steps_per_epoch / dt / 1e12})
        log(f"[train] epoch {ep}: loss {tl:.4f}, val loss {vl:.4f}, val pixel acc {vacc:.4f}, "
            f"val |dS| {vs:.4f}, {dt:.1f}s ({history[-1]['tflops']:.1f} TFLOP/s)")
    net.save(a.out)
    with open(a.out + ".json", "w") as f:
        json.dump({"history": history, "fields": int(len(idx)), "val": int(nval), "batch": a.batch,
                   "epochs": a.epochs, "lr": a.lr}, f, indent=1)
    log(f"[train] wrote {a.out}")


def evaluate(net, X, T, M, sel_idx, batch):
    """Masked loss, pixel accuracy (threshold 0.5) and mean |S_pred - S_true|
    over the window, for the given rows."""
    import torch
    losses, accs, serr = [], [], []
    for s in range(0, len(sel_idx), batch):
        sel = torch.from_numpy(sel_idx[s:s + batch]).to(X.device)
        xb, tb, mb = X.index_select(0, sel), T.index_select(0, sel), M.index_select(0, sel)
        pred = net.forward(xb.contiguous())
        p = pred.clamp(1e-6, 1 - 1e-6)
        mf = mb.float()
        bce = -(tb * p.log() + (1 - tb) * (1 - p).log())
        losses.append(float((bce * mf).sum() / mf.sum()))
        accs.append(float((((p > 0.5) == (tb > 0.5)).float() * mf).sum() / mf.sum()))
        w = mf[:, :, 8:-8]
        sp = (p[:, :, 8:-8] * w).sum(dim=(1, 2)) / w.sum(dim=(1, 2))
        st = (tb[:, :, 8:-8] * w).sum(dim=(1, 2)) / w.sum(dim=(1, 2))
        serr += (sp - st).abs().tolist()
    return float(np.mean(losses)), float(np.mean(accs)), float(np.mean(serr))


def cmd_eval(a):
    t0 = time.time()
    idx = list(range(a.first, a.first + a.count))
    probs = make_instances(idx, make_masks(idx, a.n, a.workers), a.n)
    net = S.UNet.load(a.weights)
    sat = S.predict(net, probs)
    warm = []
    for p, s in zip(probs, sat):
        q = I.Problem(**{k: getattr(p, k) for k in p.__dataclass_fields__})
        q.rho0 = S.warm_start_density(p, s)
        q.theta, q.dp = p.theta, p.dp
        warm.append(q)
    log(f"[eval] {a.count} instances, predictions ready ({time.time() - t0:.0f}s)")
    steps, conv, snw, _, _ = run_to_steady(probs + warm, a.cap, a.check, a.tol, tag=" eval")
    k = a.count
    rows = []
    for i in range(k):
        if steps[i] is None or steps[k + i] is None:
            log(f"[eval] instance {a.first + i} dropped (non-finite density)")
            continue
        rows.append({"idx": a.first + i, "theta": probs[i].theta, "dp": probs[i].dp,
                     "cold_steps": steps[i], "cold_conv": conv[i], "cold_S": snw[i],
                     "warm_steps": steps[k + i], "warm_conv": conv[k + i], "warm_S": snw[k + i],
                     "pred_S": float(sat[i][:, probs[i].porous_x0:probs[i].porous_x1][
                         probs[i].mask[:, probs[i].porous_x0:probs[i].porous_x1] == 0].mean())})
    both = [r for r in rows if r["cold_conv"] and r["warm_conv"]]
    ok = [r for r in both if abs(r["warm_S"] - r["cold_S"]) <= a.s_tol]
    summary = {
        "instances": k, "both_converged": len(both), "within_s_tol": len(ok), "s_tol": a.s_tol,
        "cold_steps_median": float(np.median([r["cold_steps"] for r in rows])),
        "warm_steps_median": float(np.median([r["warm_steps"] for r in rows])),
        "cold_steps_total": int(sum(r["cold_steps"] for r in rows)),
        "warm_steps_total": int(sum(r["warm_steps"] for r in rows)),
        "speedup_total_steps": sum(r["cold_steps"] for r in rows) / max(1, sum(r["warm_steps"] for r in rows)),
        "speedup_median_within_tol": float(np.median([r["cold_steps"] / r["warm_steps"] for r in ok])) if ok
        else None,
        "mean_abs_dS": float(np.mean([abs(r["warm_S"] - r["cold_S"]) for r in rows])),
        "cap": a.cap, "check": a.check, "tol": a.tol,
    }
    log("[eval] " + json.dumps(summary))
    if a.out:
        with open(a.out, "w") as f:
            json.dump({"summary": summary, "rows": rows}, f, indent=1)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("gen")
    g.add_argument("--first", type=int, default=0)
    g.add_argument("--count", type=int, default=2000)
    g.add_argument("--batch", type=int, default=128)
    g.add_argument("--n", type=int, default=256)
    g.add_argument("--cap", type=int, default=100000)
    g.add_argument("--check", type=int, default=1000)
    g.add_argument("--tol", type=float, default=1e-6)
    g.add_argument("--workers", type=int, default=8)
    g.add_argument("--run-all", action="store_true", help="keep stepping to the cap (full trajectories)")
    g.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--data", nargs="+", required=True)
    t.add_argument("--epochs", type=int, default=30)
    t.add_argument("--batch", type=int, default=16)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--val-frac", type=float, default=0.05)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--workers", type=int, default=8)
    t.add_argument("--max-minutes", type=float, default=0.0, help="stop starting epochs after this")
    t.add_argument("--out", required=True)
    e = sub.add_parser("eval")
    e.add_argument("--weights", required=True)
    e.add_argument("--first", type=int, default=2000)
    e.add_argument("--count", type=int, default=32)
    e.add_argument("--n", type=int, default=256)
    e.add_argument("--cap", type=int, default=200000)
    e.add_argument("--check", type=int, default=1000)
    e.add_argument("--tol", type=float, default=1e-6)
    e.add_argument("--s-tol", type=float, default=0.01)
    e.add_argument("--workers", type=int, default=8)
    e.add_argument("--out", default="")
    a = ap.parse_args()
    {"gen": cmd_gen, "train": cmd_train, "eval": cmd_eval}[a.cmd](a)


if __name__ == "__main__":
    main()
