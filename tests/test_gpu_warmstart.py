"""What the trained surrogate gains, with the plain method as its judge and
its fallback.

Held-out drainage instances (256x256, contact angle and pressure step drawn
per instance; indices 2000-2031, training used 0-1999) whose contact angle is
below 90 degrees run on their own solver, from the plain cold start and from
the network's predicted saturation (lbm_init_from_saturation), each until the
window saturation changes by less than 1e-6 per 1000 steps.  A warm run that
has not settled within its step budget falls back to the cold start and is
charged the budget plus the whole cold run.  Counting inference and
fallbacks, the warm starts must reach steady state in less wall time than the
cold starts, and every warm result must lie within 0.01 in saturation of the
cold steady state.  The same comparison batched (cold starts in one batch,
warm starts in another, settled instances retired from their batch, the
fallbacks in a third batch) must reach the same steady states.  Above 90 degrees the non-wetting phase imbibes
spontaneously and neither start settles within 3e5 steps (see
weights/unet_drainage256.eval.json), so those instances are left out.

The weights are the committed result of
    python -m paper_2111_08666_amd.train_surrogate train ...
on fields the solver generated with
    python -m paper_2111_08666_amd.train_surrogate gen ..."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2111_08666_amd", "weights", "unet_drainage256.npz")


@pytest.fixture(scope="module")
def mods():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(WEIGHTS):
        pytest.skip("no trained weights committed")
    from paper_2111_08666_amd import inputs as I
    from paper_2111_08666_amd import lbm
    from paper_2111_08666_amd import surrogate as S
    return I, S, lbm


def test_init_from_saturation_equals_the_host_warm_start(mods):
    """lbm_init_from_saturation from a device (and a host) saturation field
    sets the same state, bit for bit, as a context created from the warm
    densities the host builds, and both continue alike."""
    import torch
    I, S, lbm = mods
    p = I.surrogate_instance(2003)
    rng = np.random.default_rng(7)
    sat = rng.random(p.mask.shape).astype(np.float32)
    q = I.Problem(**{f: getattr(p, f) for f in p.__dataclass_fields__})
    q.rho0 = S.warm_start_density(p, sat)
    ref = lbm.Solver(q)
    dev = lbm.Solver(p)
    dev.step(7)
    dev.init_from_saturation(torch.from_numpy(S.full_saturation(p, sat)).cuda())
    host = lbm.Solver(p)
    host.init_from_saturation(S.full_saturation(p, sat))
    assert dev.t == 0 and host.t == 0
    for s in (ref, dev, host):
        s.step(50)
    assert np.array_equal(dev.density(), ref.density())
    assert np.array_equal(host.density(), ref.density())
    with pytest.raises(lbm.LbmError) as e:
        host.init_from_saturation(S.full_saturation(p, sat), rho_major=-1.0)
    assert e.value.status == lbm.LBM_EINVAL


def test_warm_start_with_fallback_reaches_steady_state_sooner(mods):
    from paper_2111_08666_amd import bench_warmstart as B
    w = B.measure(first=2000, count=32, cap=300000, budget=100000)
    for r in w["instances"]:
        print(f"[warm] {r}", flush=True)
    print(f"[warm] wall {w['wall_s']}, steps {w['steps_total']}, fallbacks {w['fallbacks']}", flush=True)
    assert len(w["instances"]) >= 8
    assert w["cold_settled"] == len(w["instances"])
    assert w["agree_within_s_tol"] == w["cold_settled"]
    assert w["wall_s"]["warm_with_fallback"] < w["wall_s"]["cold"]
    assert w["steps_total"]["warm_with_fallback"] < w["steps_total"]["cold"]
    # batched, with settled instances retired: the same steady states
    bt = w["batched"]
    print(f"[warm] batched {bt}", flush=True)
    assert bt["cold_settled"] == w["cold_settled"]
    assert bt["agree_within_s_tol"] == bt["cold_settled"]
    assert bt["fallbacks"] == w["fallbacks"]
