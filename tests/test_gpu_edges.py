"""Degenerate inputs through the C ABI, against the oracle where there is
physics to compare:
  - periodic boxes smaller than a tile and its halo (down to 1 x 1), where
    a tile's halo wraps around the period several times, for every strategy
    on both lattices;
  - an all-solid domain (no fluid node at all), where every strategy must
    step, report zero mass and leave the densities at zero."""
import numpy as np
import pytest

import oracle as O
from paper_2111_08666_amd import inputs as I

pytestmark = pytest.mark.gpu
REL_TOL = 1e-5


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_08666_amd import lbm as L
    L.lib()
    return L


def _box(q, shape, seed):
    rng = np.random.default_rng(seed)
    mask = np.zeros(shape, np.uint8)
    rho0 = rng.uniform(0.4, 0.6, size=(2,) + shape)
    periodic = 3 if q == 9 else 7
    return I.Problem(q=q, mask=mask, rho0=rho0, periodic=periodic, open_x=0, tau=(0.9, 1.3), G=0.9,
                     collision=0 if q == 9 else 2, name=f"box{shape}")


D2_CASES = [((1, 1), 1), ((1, 5), 2), ((2, 3), 3), ((4, 2), 4), ((7, 5), 5), ((13, 3), 6)]
D2_STRATEGIES = [(1, 8), (1, 16), (2, 0), (3, 0), (4, 12), (5, 8)]


@pytest.mark.parametrize("strategy,ty", D2_STRATEGIES)
@pytest.mark.parametrize("shape,seed", D2_CASES)
def test_tiny_periodic_d2q9_boxes_match_oracle(lbm, shape, seed, strategy, ty):
    p = _box(9, shape, seed)
    o = O.OracleSim(p)
    o.step(50)
    s = lbm.Solver(p, strategy=strategy, tile_rows=ty)
    s.step(50)
    ref = o.density()
    err = float(np.max(np.abs(s.density() - ref) / ref))
    assert err <= REL_TOL, (shape, strategy, err)


@pytest.mark.parametrize("strategy", [1, 2, 3])
@pytest.mark.parametrize("shape,seed", [((1, 1, 1), 7), ((3, 2, 1), 8), ((1, 4, 3), 9), ((5, 3, 2), 10)])
def test_tiny_periodic_d3q19_boxes_match_oracle(lbm, shape, seed, strategy):
    p = _box(19, shape, seed)
    o = O.OracleSim(p)
    o.step(30)
    s = lbm.Solver(p, strategy=strategy)
    s.step(30)
    ref = o.density()
    err = float(np.max(np.abs(s.density() - ref) / ref))
    assert err <= REL_TOL, (shape, strategy, err)


@pytest.mark.parametrize("q,strategies", [(9, [1, 2, 3, 4, 5]), (19, [1, 2, 3])])
def test_all_solid_domain_steps_with_zero_mass(lbm, q, strategies):
    shape = (12, 70) if q == 9 else (6, 10, 70)
    mask = np.ones(shape, np.uint8)
    p = I.Problem(q=q, mask=mask, rho0=np.zeros((2,) + shape), periodic=0, open_x=0,
                  collision=0 if q == 9 else 2, name="all_solid")
    for strategy in strategies:
        s = lbm.Solver(p, strategy=strategy)
        s.step(6)
        s.step_graph(4, 2)
        obs = s.observables()
        assert obs["n_fluid"] == 0 and obs["mass"] == [0.0, 0.0] and obs["flags"] == 0, strategy
        assert not np.any(s.density()), strategy
        s.close()
