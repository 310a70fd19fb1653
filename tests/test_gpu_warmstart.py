"""What the trained surrogate gains: held-out drainage instances (256x256,
contact angle and pressure step drawn per instance) run from the plain cold
start and from the network's predicted saturation, both until the window
saturation changes by less than 1e-6 per 1000 steps.  The warm start must
reach that steady state in fewer steps in total, and on the instances where
both runs settle, land within 0.01 of the cold start's saturation on most of
them (a different metastable state counts against the surrogate).

Instances: the held-out indices 2000-2031 (training used 0-1999) whose
contact angle is below 90 degrees.  In that water-wet regime the cold start
settles within the cap (about 0.8e5-2.2e5 steps); above 90 degrees the
non-wetting phase imbibes spontaneously and neither start settles within
4e5 steps (see weights/unet_drainage256.eval.json for all 32).

The weights are the committed result of
    python -m paper_2111_08666_amd.train_surrogate train ...
on fields the solver generated with
    python -m paper_2111_08666_amd.train_surrogate gen ..."""
import os

import pytest

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2111_08666_amd", "weights", "unet_drainage256.npz")
HELD_OUT = list(range(2000, 2032))
CAP = 300000


@pytest.fixture(scope="module")
def mods():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(WEIGHTS):
        pytest.skip("no trained weights committed")
    from paper_2111_08666_amd import inputs as I
    from paper_2111_08666_amd import surrogate as S
    from paper_2111_08666_amd import train_surrogate as T
    return I, S, T


def test_warm_start_reaches_the_same_steady_state_sooner(mods):
    I, S, T = mods
    probs = [p for p in (I.surrogate_instance(k) for k in HELD_OUT) if p.theta < 90.0]
    assert len(probs) >= 8
    net = S.UNet.load(WEIGHTS)
    sat = S.predict(net, probs)
    warm = []
    for p, s in zip(probs, sat):
        q = I.Problem(**{f: getattr(p, f) for f in p.__dataclass_fields__})
        q.rho0 = S.warm_start_density(p, s)
        warm.append(q)
    steps, conv, snw, _, _ = T.run_to_steady(probs + warm, CAP)
    k = len(probs)
    cold_steps, warm_steps = steps[:k], steps[k:]
    ds = [abs(snw[k + i] - snw[i]) for i in range(k)]
    both = [i for i in range(k) if conv[i] and conv[k + i]]
    agree = [i for i in both if ds[i] <= 0.01]
    print(f"[warm] cold steps {cold_steps}", flush=True)
    print(f"[warm] warm steps {warm_steps}", flush=True)
    print(f"[warm] |dS| {['%.4f' % d for d in ds]}; both settled {len(both)}, within 0.01: {len(agree)}",
          flush=True)
    assert sum(warm_steps) < sum(cold_steps)
    assert len(agree) >= max(1, (len(both) + 1) // 2)
