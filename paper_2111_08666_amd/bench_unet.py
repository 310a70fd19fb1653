"""Benchmark of the U-Net surrogate's kernels on one MI355X.

    python -m paper_2111_08666_amd.bench_unet [--batch 16] [--size 256] [--steps 20]

Times full training steps (forward, masked cross-entropy, backward, Adam) and
inference passes of the 4-level U-Net on synthetic 256x256 inputs, with HIP
events on the current stream, and prints one JSON line: TFLOP/s of the
convolutions (2 x multiply-adds; a training step counts three passes) against
the dense BF16 MFMA peak of 2.5 PFLOP/s, and the step time against the sum of
the convolution passes' own rooflines (the MFMA or the HBM bound of each).
"""
import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MFMA_BF16_PEAK_TFLOPS = 2500.0
HBM_PEAK_TBS = 8.0


def conv_roofline_ms(specs, n, h, w):
    """Lower bound on the convolutions of one training step: each layer's
    forward, data-gradient (not for the input layer) and weight-gradient
    pass takes at least the larger of its multiply-adds at the BF16 MFMA
    peak and its minimal HBM bytes at the HBM peak (BF16 operands read once
    and results written once, weight gradients in FP32).  Returns (ms,
    passes bound by the matrix cores, passes bound by HBM)."""
    total, n_mfma, n_hbm = 0.0, 0, 0
    for name, kind, ci, co in specs:
        lvl = int(name[3]) if name.startswith(("enc", "dec")) else int(name[2:])
        p_out = n * (h >> lvl) * (w >> lvl)
        p_in = p_out if kind == "conv" else p_out // 4
        taps = 9 if kind == "conv" else 4
        flops = 2 * p_out * (9 if kind == "conv" else 1) * ci * co
        io = 2 * (p_in * ci + p_out * co)
        passes = [io + 2 * taps * ci * co, io + 4 * taps * ci * co]
        if name != "enc0a":
            passes.append(io + 2 * taps * ci * co)
        for nbytes in passes:
            t_m, t_h = flops / (MFMA_BF16_PEAK_TFLOPS * 1e12), nbytes / (HBM_PEAK_TBS * 1e12)
            total += max(t_m, t_h)
            n_mfma += t_m >= t_h
            n_hbm += t_h > t_m
    return total * 1e3, n_mfma, n_hbm


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    a = ap.parse_args()
    import torch
    from paper_2111_08666_amd import surrogate as S

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(0)
    n, h = a.batch, a.size
    x = np.zeros((n, h, h, S.IN_CH), np.float32)
    x[..., 0] = rng.uniform(size=(n, h, h)) < 0.45
    x[..., 1] = rng.uniform(-1, 1, size=(n, 1, 1))
    x[..., 2] = rng.uniform(-1, 1, size=(n, 1, 1))
    xb = torch.from_numpy(S.bf16_bits(x).view(np.int16)).to(dev)
    t = torch.from_numpy((rng.uniform(size=(n, h, h)) < 0.3).astype(np.float32)).to(dev)
    m = torch.from_numpy((x[..., 0] == 0).astype(np.uint8)).to(dev)
    count = int(m.sum().item())
    net = S.UNet(seed=0, device=dev)
    for _ in range(a.warmup):
        net.train_step(xb, t, m, lr=1e-4, count=count)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream(dev)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(s)
    for _ in range(a.steps):
        net.train_step(xb, t, m, lr=1e-4, count=count)
    e1.record(s)
    for _ in range(a.steps):
        net.forward(xb)
    e2.record(s)
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1) / a.steps
    infer_ms = e1.elapsed_time(e2) / a.steps
    f = net.flops_per_image(h, h)
    train_tf = 3 * f * n / (train_ms * 1e-3) / 1e12
    roof_ms, n_m, n_h = conv_roofline_ms(net.specs, n, h, h)
    infer_tf = f * n / (infer_ms * 1e-3) / 1e12
    out = {
        "metric": "U-Net training step throughput (BF16 MFMA, FP32 accumulate)",
        "value": round(n / (train_ms * 1e-3), 1), "unit": "images/s", "higher_is_better": True,
        "config": {"workload": f"4-level U-Net 32/64/128/256, {n} x {h}x{h} fields", "batch": n,
                   "params": int(sum(np.prod(v) for v in net.shapes.values())),
                   "gflop_per_image_forward": round(f / 1e9, 2)},
        "train_ms_per_step": round(train_ms, 3), "infer_ms_per_batch": round(infer_ms, 3),
        "infer_images_per_s": round(n / (infer_ms * 1e-3), 1),
        "roofline": {"bound": "mfma", "achieved": round(train_tf, 1), "peak": MFMA_BF16_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(train_tf / MFMA_BF16_PEAK_TFLOPS, 4),
                     "infer_achieved": round(infer_tf, 1)},
        "layer_roofline": {"conv_ms": round(roof_ms, 3), "passes_mfma_bound": n_m, "passes_hbm_bound": n_h,
                           "frac_of_step": round(roof_ms / train_ms, 4)},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
