"""lbm_debug_poke: the failure path forced from the host, and the poke's own
addressing on every layout.

A NaN written into one population of one fluid node must make the next
observables report LBM_EUNSTABLE (flags bit 0) and later steps refuse, on
every strategy and storage, with every kernel exiting normally.  A finite
poke must land exactly where the layout keeps that population: replacing
f*_i of node n by v and then by v + delta changes the density the next step
streams into n + e_i (node n itself for the rest link) by delta and no other
density.  Bad arguments (a solid node, a node outside the grid, a component
or link out of range) are refused with LBM_EINVAL."""
import numpy as np
import pytest

from cases import problems
from paper_2111_08666_amd import inputs as I

pytestmark = pytest.mark.gpu

P2 = problems()


def _p3():
    m = I.sphere_medium(40, 20, 18, 2.0, 4.0, 0.6, seed=5)
    r0 = I.reservoir_front(m, 8, 1.0, 0.027)
    return I.Problem(q=19, mask=m, rho0=r0, periodic=0, open_x=1, porous_x0=8, porous_x1=32,
                     tau=I.TAU_M10, G=3.5, xi=I.xi_of_theta(60), rho_in1=1.015, collision=2)


P3 = _p3()


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_08666_amd import lbm as L
    L.lib()
    return L


def _interior_fluid(p, link=None):
    """A fluid node away from the faces whose neighbour along `link` (if
    given) is fluid too, and that neighbour's coordinates."""
    from paper_2111_08666_amd.inputs import Problem  # noqa: F401
    m = p.mask
    e = {9: [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]}
    if p.q == 9:
        ny, nx = m.shape
        for y in range(2, ny - 2):
            for x in range(10, nx - 10):
                dx, dy = e[9][link or 0]
                if m[y, x] == 0 and m[y + dy, x + dx] == 0:
                    return (x, y, 0), (x + dx, y + dy, 0)
    else:
        nz, ny, nx = m.shape
        for z in range(2, nz - 2):
            for y in range(2, ny - 2):
                for x in range(10, nx - 10):
                    if m[z, y, x] == 0 and m[z, y, x + 1] == 0:
                        return (x, y, z), (x + 1, y, z)
    raise AssertionError("no interior fluid node")


CASES = [("drain_mrt", 1, 0), ("drain_mrt", 2, 0), ("drain_mrt", 3, 0), ("drain_mrt", 4, 0), ("drain_mrt", 5, 0),
         ("drain_mrt", 1, 1), ("drain_mrt", 3, 1), ("d3", 2, 0), ("d3", 3, 0), ("d3", 5, 0), ("d3", 3, 1)]


@pytest.mark.parametrize("name,strategy,storage", CASES)
def test_nan_poke_is_reported_unstable(lbm, name, strategy, storage):
    p = P3 if name == "d3" else P2[name]
    if strategy == 5 and name == "d3" and storage:
        pytest.skip("the compacted 3D fused step needs FP32 storage")
    s = lbm.Solver(p, strategy=strategy, storage=storage)
    s.step(3)
    assert s.observables()["flags"] == 0
    (x, y, z), _ = _interior_fluid(p)
    print(f"[poke] {name} strategy {strategy} storage {storage} NaN at {(x, y, z)}", flush=True)
    s.debug_poke(x, y, z, 1, 0, float("nan"))
    s.step(1)
    o = s.observables(allow_unstable=True)
    assert o["flags"] & 1
    with pytest.raises(lbm.LbmError) as e:
        s.step(1)
    assert e.value.status == lbm.LBM_EUNSTABLE


# (name, strategy, link): D2Q9 link 1 is +x, D3Q19 link 1 is +x as well
ADDR = [("drain_mrt", 1, 0), ("drain_mrt", 1, 1), ("drain_mrt", 2, 1), ("drain_mrt", 3, 0), ("drain_mrt", 3, 1),
        ("drain_mrt", 5, 1), ("d3", 2, 1), ("d3", 3, 0), ("d3", 3, 1), ("d3", 5, 1)]


@pytest.mark.parametrize("name,strategy,link", ADDR)
def test_poke_lands_on_the_population(lbm, name, strategy, link):
    p = P3 if name == "d3" else P2[name]
    s = lbm.Solver(p, strategy=strategy)
    s.step(5)
    node, dest = _interior_fluid(p, link)
    if link == 0:
        dest = node
    base = s.density().astype(np.float64)
    s.debug_poke(*node, 0, link, 0.25)
    a = s.density().astype(np.float64)
    s.debug_poke(*node, 0, link, 0.75)
    b = s.density().astype(np.float64)
    d = b - a
    dx, dy, dz = dest
    idx = (0, dy, dx) if p.q == 9 else (0, dz, dy, dx)
    assert abs(d[idx] - 0.5) < 1e-6, d[idx]
    d[idx] = 0.0
    assert np.abs(d).max() < 1e-7
    # the first poke only touched the same density
    c = a - base
    c[idx] = 0.0
    assert np.abs(c).max() < 1e-7


def test_poke_refuses_bad_arguments(lbm):
    p = P2["drain_mrt"]
    s = lbm.Solver(p)
    ys, xs = np.nonzero(p.mask)
    bad = [(int(xs[0]), int(ys[0]), 0, 0, 0),  # solid
           (p.nx, 0, 0, 0, 0), (0, -1, 0, 0, 0), (0, 0, 1, 0, 0),  # outside
           (10, 10, 0, 2, 0), (10, 10, 0, 0, 9)]  # component, link
    for x, y, z, c, i in bad:
        with pytest.raises(lbm.LbmError) as e:
            s.debug_poke(x, y, z, c, i, 1.0)
        assert e.value.status == lbm.LBM_EINVAL
    s.step(2)
    assert s.observables()["flags"] == 0
