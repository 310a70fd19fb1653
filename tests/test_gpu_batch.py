"""The batched workload at full size: 64 uneven D2Q9 drainage instances
(256x128 .. 1024x512), each with its own medium, contact angle and pressure
step, advanced together by one launch per step in HIP graphs after the
autotuner has picked the variant -- the configuration bench.py times.

Per-instance error against the FP64 oracle after 200 steps at 1024 seeded
fluid nodes per instance (tests/golden/batch64_step200_samples.npz, written
by tests/golden/make_batch64_samples.py from the oracle alone):
  FP32 storage: every sampled density within 1e-5 relative, with FP32 (the
  default) and with FP64 node arithmetic;
  BF16-deviation storage: within 2e-2 (measured values printed).
"""
import os

import numpy as np
import pytest

from paper_2111_08666_amd import inputs as I

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
FIXTURE = os.path.join(HERE, "golden", "batch64_step200_samples.npz")


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_08666_amd import lbm as L
    L.lib()
    return L


@pytest.fixture(scope="module")
def problems():
    return I.batch_instances(64)


@pytest.fixture(scope="module")
def ref():
    with np.load(FIXTURE, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def _advance_like_bench(b, steps=200):
    """Autotune (ordinary steps), then graph replays up to `steps`."""
    rep = b.autotune(10)
    done = 2 * 12 * len(rep.strip().splitlines())  # two passes of 2 + 10 steps per variant
    rest = steps - done
    assert rest > 0 and rest % 2 == 0
    b.step_graph(2, rest // 2)
    return rep


# storage 0 FP32, 1 BF16 deviations; math 0 FP32 node arithmetic (the
# default), 1 FP64
@pytest.mark.parametrize("storage,math,bound", [(0, 0, 1e-5), (0, 1, 1e-5), (1, 0, 2e-2)])
def test_batch64_per_instance_error_vs_oracle(lbm, problems, ref, storage, math, bound):
    assert int(ref["steps"]) == 200
    b = lbm.BatchSolver(problems, storage=storage, math=math)
    rep = _advance_like_bench(b)
    print(f"[batch64] storage={storage} math={math} autotune: {rep.strip().splitlines()}", flush=True)
    errs = []
    for k, p in enumerate(problems):
        assert tuple(ref[f"shape{k}"]) == p.mask.shape
        g = b.density(k).reshape(2, -1)[:, ref[f"idx{k}"]].astype(np.float64)
        r = ref[f"rho{k}"]
        errs.append(float(np.max(np.abs(g - r) / np.abs(r))))
    errs = np.array(errs)
    print(f"[batch64] storage={storage} math={math} per-instance max relative error: "
          + " ".join(f"{e:.1e}" for e in errs), flush=True)
    print(f"[batch64] storage={storage} math={math} worst {errs.max():.2e} median {np.median(errs):.2e}",
          flush=True)
    assert errs.max() <= bound


def test_batch64_equals_single_instance_runs(lbm, problems):
    """Batching changes nothing: each instance of the batch is bitwise equal
    to the same instance advanced alone with the same variant."""
    b = lbm.BatchSolver(problems, strategy=lbm.FUSED, tile_rows=12)
    b.step_graph(10, 3)
    for k in (0, 17, 41, 63):
        s = lbm.Solver(problems[k], strategy=lbm.FUSED, tile_rows=12)
        s.step(30)
        assert np.array_equal(b.density(k), s.density()), k


def test_auto_layout_follows_the_cache_size(lbm, problems):
    """AUTO keeps the dense layout while both population buffers of a context
    fit in the 256 MB last-level cache and compacts beyond it: the 64
    instances (2.4 GB dense) step on the compacted fused kernel, one
    1024x512 instance (75 MB) on the dense one; an explicit strategy is
    kept."""
    b = lbm.BatchSolver(problems)
    assert "compact" in b.kernel_info()[0]
    b.close()
    b = lbm.BatchSolver(problems, strategy=lbm.FUSED)
    assert "compact" not in b.kernel_info()[0]
    b.close()
    s = lbm.Solver(I.large_drainage())
    assert "compact" not in s.kernel_info()[0]
    s.close()


SMALL = os.path.join(HERE, "golden", "batch64_small_step10k_obs.npz")


def test_batch64_small_instances_saturation_and_pc_vs_oracle(lbm, problems):
    """The eight smallest of the 64 instances after 10 000 steps of the
    whole batch, advanced as bench.py runs it (autotune, then graph
    replays), against the FP64 oracle's observables
    (tests/golden/batch64_small_step10k_obs.npz, written by
    tests/golden/make_batch_small_obs.py from the oracle alone): window
    saturation and capillary pressure within 1 %, FP32 storage."""
    with np.load(SMALL, allow_pickle=False) as z:
        ref = {k: z[k] for k in z.files}
    steps = int(ref["steps"])
    b = lbm.BatchSolver(problems)
    try:
        _advance_like_bench(b, steps)
        obs = b.observables()
        kernel = b.kernel_info()[0]
    finally:
        b.close()
    rows = []
    for k in (int(i) for i in ref["index"]):
        o = obs[k]
        e_s = abs(o["s_w"] - float(ref[f"s_w{k}"])) / float(ref[f"s_w{k}"])
        e_sw = abs(o["s_w_weighted"] - float(ref[f"s_w_weighted{k}"])) / float(ref[f"s_w_weighted{k}"])
        e_pc = abs(o["pc"] - float(ref[f"pc{k}"])) / abs(float(ref[f"pc{k}"]))
        rows.append((k, e_s, e_sw, e_pc))
    print(f"[batch64-small] {kernel}, {steps} steps, relative errors (instance: S_w, S_w weighted, P_c): "
          + "  ".join(f"{k}: {a:.1e} {b_:.1e} {c:.1e}" for k, a, b_, c in rows), flush=True)
    for k, a, b_, c in rows:
        assert a <= 0.01 and b_ <= 0.01 and c <= 0.01, (k, a, b_, c)
