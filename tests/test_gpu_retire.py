"""Retiring instances from a batch (lbm_batch_set_active).

A batch of uneven instances in which some settle (or fail) early can drop
them from the launches: the block table of the one-launch strategies and the
per-instance launches of the split ones leave retired instances out.  The
checks, on the GPU through the C-ABI:
  * the instances that keep advancing are bit-identical to single-instance
    runs of the same number of steps, and so is a retired instance after it
    is re-admitted (its state, read while retired, is the one it was left in,
    and its step count stops).  The compacted 3D fused step is the exception:
    a change of the active set rebuilds the psi it carries between steps,
    which rounds differently from the carried one in the last FP32 place, so
    there the densities agree within 1e-6 relative (as after any other
    change of state outside a step);
  * a batch with every instance retired steps (eagerly and in graphs)
    without launching anything and without error;
  * an instance whose densities went non-finite stops the batch until it is
    retired; the rest then advance as if it had never been there.
"""
import numpy as np
import pytest

from paper_2111_08666_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_08666_amd import lbm as L
    L.lib()
    return L


def _d2(nx, ny, seed, theta):
    return I.drainage_2d(nx=nx, ny=ny, r=(2.0, 4.0), porosity=0.7, seed=seed, G=3.5, theta=theta,
                         tau=I.TAU_M10, rho_in1=1.02, minor=0.027, collision=2)


def _d3(nx, ny, nz, seed):
    m = I.sphere_medium(nx, ny, nz, 2.0, 4.0, 0.6, seed=seed)
    r0 = I.reservoir_front(m, 8, 1.0, 0.027)
    return I.Problem(q=19, mask=m, rho0=r0, periodic=0, open_x=1, porous_x0=8, porous_x1=nx - 8,
                     tau=I.TAU_M10, G=3.5, xi=I.xi_of_theta(60), rho_in1=1.015, collision=2)


D2 = [_d2(130, 40, 41, 45), _d2(70, 26, 42, 120), _d2(96, 37, 43, 60)]
D3 = [_d3(40, 20, 18, 51), _d3(36, 18, 14, 52), _d3(44, 22, 16, 53)]


def _single(lbm, p, strategy, n):
    s = lbm.Solver(p, strategy=strategy)
    s.step(n)
    return s.density()


@pytest.mark.parametrize("q,strategy", [(9, "FUSED"), (9, "FUSED_LIST"), (9, "SPLIT"), (9, "COMPACT_FUSED"),
                                        (19, "COMPACT"), (19, "COMPACT_FUSED"), (19, "SPLIT")])
def test_retired_instance_is_frozen_and_resumes(lbm, q, strategy):
    ps = D2 if q == 9 else D3
    st = getattr(lbm, strategy)
    b = lbm.BatchSolver(ps, strategy=st)
    b.step(11)
    held = b.density(1)
    b.set_active([True, False, True])
    b.set_active([True, False, True])  # no change: a no-op
    b.step_graph(6, 2)
    b.step(5)
    assert np.array_equal(b.density(1), held)
    steps = [o["step"] for o in b.observables()]
    assert steps == [28, 11, 28], steps
    b.set_active([True, True, True])
    b.step(7)
    b.step_graph(2, 3)
    want = [41, 24, 41]
    assert [o["step"] for o in b.observables()] == want
    for i, p in enumerate(ps):
        ref = _single(lbm, p, st, want[i])
        got = b.density(i)
        if q == 19 and strategy == "COMPACT_FUSED":
            fluid = ~p.mask.astype(bool)
            r = ref.astype(np.float64)
            err = float((np.abs(got - r) / np.abs(r))[:, fluid].max())
            assert err <= 1e-6, (strategy, i, err)
        else:
            assert np.array_equal(got, ref), (strategy, i)
    print(f"[retire] q={q} {strategy}: {b.kernel_info()[0]} ok", flush=True)


@pytest.mark.parametrize("q", [9, 19])
def test_all_retired_steps_are_empty(lbm, q):
    ps = D2 if q == 9 else D3
    st = lbm.FUSED if q == 9 else lbm.COMPACT
    b = lbm.BatchSolver(ps, strategy=st)
    b.step(4)
    before = [b.density(i) for i in range(len(ps))]
    b.set_active([False] * len(ps))
    b.step(3)
    b.step_graph(4, 2)
    for i in range(len(ps)):
        assert np.array_equal(b.density(i), before[i])
    assert [o["step"] for o in b.observables()] == [4] * len(ps)
    b.set_active([False, True, False])
    b.step(6)
    assert np.array_equal(b.density(1), _single(lbm, ps[1], st, 10))
    assert np.array_equal(b.density(0), before[0])


def test_failed_instance_is_retired_and_the_rest_continue(lbm):
    bad = _d2(64, 30, 31, 100)
    bad.G = 400.0  # far beyond any stable cohesion: densities blow up
    ps = [D2[0], bad, D2[2]]
    b = lbm.BatchSolver(ps, strategy=lbm.FUSED)
    b.step(50)
    with pytest.raises(lbm.LbmError) as e:
        b.observables()
    assert e.value.status == lbm.LBM_EUNSTABLE
    with pytest.raises(lbm.LbmError):
        b.step(1)
    b.set_active([True, False, True])
    obs = b.observables()  # the retired instance no longer fails the call
    assert obs[1]["flags"] & 1 and not obs[0]["flags"] & 1
    b.step(20)
    for i in (0, 2):
        assert np.array_equal(b.density(i), _single(lbm, ps[i], lbm.FUSED, 70)), i
    b.set_active([True, True, True])  # re-admitting it stops the batch again
    with pytest.raises(lbm.LbmError) as e:
        b.step(1)
    assert e.value.status == lbm.LBM_EUNSTABLE
