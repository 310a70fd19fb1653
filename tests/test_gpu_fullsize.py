"""The two single-instance benchmark workloads at their full sizes, in the
launch configuration bench.py times (the autotuner picks the variant, then
HIP-graph replays), against FP64 oracle densities at 2048 seeded fluid nodes
each (tests/golden/fullsize_samples.npz, written by
tests/golden/make_fullsize_samples.py from the oracle alone):
  D2Q9 1024x512 disc-medium drainage, MRT, after 200 steps;
  D3Q19 384^3 sphere-pack drainage, TRT, after 200 steps.
Every sampled density within 1e-5 relative (FP32 storage, FP32 and FP64
node arithmetic)."""
import os

import numpy as np
import pytest

from paper_2111_08666_amd import inputs as I

pytestmark = pytest.mark.gpu

FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_samples.npz")
REL_TOL = 1e-5


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_08666_amd import lbm as L
    L.lib()
    return L


@pytest.fixture(scope="module")
def ref():
    with np.load(FIXTURE, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


# lbm_params.math: 0 FP32 node arithmetic (the default), 1 FP64
@pytest.mark.parametrize("name,make,math", [("d2q9", I.large_drainage, 0), ("d2q9", I.large_drainage, 1),
                                            ("d3q19", I.drainage_3d, 0), ("d3q19", I.drainage_3d, 1)])
def test_full_size_workload_matches_oracle_samples(lbm, ref, name, make, math):
    """Both node arithmetics on the full-size MRT drainage (D2Q9) and TRT
    sphere-pack drainage (D3Q19), held to the same 1e-5 bar."""
    if f"{name}_rho" not in ref:
        pytest.skip(f"no {name} samples in the fixture")
    steps = int(ref[f"{name}_steps"])
    p = make()
    s = lbm.Solver(p, math=math)
    try:
        rep = s.autotune(10)
        rest = steps - s.t
        assert rest > 0 and rest % 2 == 0
        s.step_graph(2, rest // 2)
        assert s.t == steps
        got = s.density().astype(np.float64).reshape(2, -1)[:, ref[f"{name}_idx"]]
        kernel = s.kernel_info()[0]
    finally:
        s.close()
    want = ref[f"{name}_rho"]
    err = float(np.max(np.abs(got - want) / np.abs(want)))
    print(f"[fullsize] {name} math={math} {p.nx}x{p.ny}x{p.nz} ({kernel}; autotune: {len(rep.strip().splitlines())} "
          f"variants), {steps} steps: worst relative error over {want.shape[1]} nodes x 2 components "
          f"{err:.2e}", flush=True)
    assert err <= REL_TOL
