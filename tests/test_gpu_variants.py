"""D3Q19 against the FP64 oracle (1e-5 relative over 200 steps), FP32 node
arithmetic held to the same bar on every D2Q9 and D3Q19 case, and
BF16-deviation storage, whose error against the oracle is measured and
bounded here."""
import numpy as np
import pytest

import oracle as O
from cases import problems
from paper_2111_08666_amd import inputs as I

pytestmark = pytest.mark.gpu

REL_TOL = 1e-5
CHECKPOINTS = (1, 10, 50, 100, 200)


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_08666_amd import lbm as L
    L.lib()
    return L


def problems3d():
    out = {}
    # open drainage through Boolean spheres; 40 x 20 x 18 is one ragged x tile,
    # 3 ragged y tiles and one z chunk
    m = I.sphere_medium(40, 20, 18, 2.0, 4.0, 0.6, seed=5)
    r0 = I.reservoir_front(m, 8, 1.0, 0.027)
    out["d3_drain_trt"] = I.Problem(q=19, mask=m, rho0=r0, periodic=0, open_x=1, porous_x0=8,
                                    porous_x1=32, tau=I.TAU_M10, G=3.5, xi=I.xi_of_theta(60),
                                    rho_in1=1.015, collision=2)
    out["d3_drain_srt"] = I.Problem(q=19, mask=m, rho0=r0, periodic=0, open_x=1, porous_x0=8,
                                    porous_x1=32, tau=(1.0, 0.8), G=3.5, xi=I.xi_of_theta(45),
                                    rho_in1=1.02, collision=0)
    out["d3_drain_mrt"] = I.Problem(q=19, mask=m, rho0=r0, periodic=0, open_x=1, porous_x0=8,
                                    porous_x1=32, tau=I.TAU_M10, G=3.5, xi=I.xi_of_theta(60),
                                    rho_in1=1.015, collision=1)
    # fully periodic droplet with z chunks (nz = 72 -> several chunks)
    n = (24, 20, 72)
    mask = np.zeros(n[::-1], np.uint8)
    r0 = I.tanh_droplet(n[::-1], (12, 10, 36), 7, (1.0, 0.027), (0.027, 1.0))
    out["d3_droplet_periodic_chunks"] = I.Problem(q=19, mask=mask, rho0=r0, periodic=7, open_x=0,
                                                  tau=(1.0, 1.0), G=3.5, collision=0)
    # closed y/z walls, periodic x, sessile droplet on the z = 0 wall, TRT
    mask = np.zeros((26, 18, 66), np.uint8)
    mask[0] = mask[-1] = 1
    mask[:, 0] = mask[:, -1] = 1
    r0 = I.tanh_droplet(mask.shape, (33, 9, 0.5), 8, (1.0, 0.027), (0.027, 1.0), mask=mask)
    out["d3_sessile_trt"] = I.Problem(q=19, mask=mask, rho0=r0, periodic=1, open_x=0,
                                      tau=(1.7, 0.62), G=3.5, xi=-0.3, collision=2)
    return out


P3 = problems3d()


def _series(p, solver, checkpoints):
    o = O.OracleSim(p)
    t = 0
    errs = []
    fluid = ~p.mask.astype(bool)
    for c in checkpoints:
        o.step(c - t)
        solver.step(c - t)
        t = c
        ref = o.density()
        g = solver.density().astype(np.float64)
        errs.append(float((np.abs(g - ref) / np.abs(ref))[:, fluid].max()))
    return errs


STRATEGIES = {"fused": 1, "split": 2, "compact": 3}


@pytest.mark.parametrize("strategy", sorted(STRATEGIES))
@pytest.mark.parametrize("name", sorted(P3))
def test_d3q19_density_parity_200_steps(lbm, name, strategy):
    p = P3[name]
    print(f"[parity3d] {name} {p.mask.shape} {strategy}", flush=True)
    s = lbm.Solver(p, strategy=STRATEGIES[strategy])
    errs = _series(p, s, CHECKPOINTS)
    print(f"[parity3d] {name} {strategy} errors {['%.1e' % e for e in errs]}", flush=True)
    assert max(errs) <= REL_TOL, errs


def test_d3q19_observables(lbm):
    p = P3["d3_drain_trt"]
    o, s = O.OracleSim(p), lbm.Solver(p)
    o.step(100)
    s.step(100)
    a, b = o.observables(), s.observables()
    assert a["n_in"] == b["n_in"] and a["n_window"] == b["n_window"]
    for c in range(2):
        assert abs(a["mass"][c] - b["mass"][c]) <= 1e-6 * a["mass"][c]
    assert abs(a["pc"] - b["pc"]) <= 1e-6


def _drain2d():
    return I.drainage_2d(nx=127, ny=37, r=(2.0, 5.0), porosity=0.7, seed=12, G=3.5, theta=60,
                         tau=I.TAU_M10, rho_in1=1.01, minor=0.027, collision=1)


# FP32 node arithmetic (deviation-form collision, FP64 density sums) holds
# the FP64 path's bar; BF16-deviation storage has a stated bound of its own
# (200 steps, fluid nodes, relative to the FP64 oracle).  Measured values are
# printed by the tests.
F32_MATH_BOUND = REL_TOL
BF16_BOUND = 2e-2


@pytest.mark.parametrize("q", [9, 19])
def test_fp32_math_error_is_bounded(lbm, q):
    p = _drain2d() if q == 9 else P3["d3_drain_trt"]
    errs = _series(p, lbm.Solver(p, math=lbm.MATH_F32), CHECKPOINTS)
    print(f"[fp32-math] q={q} errors {['%.1e' % e for e in errs]}", flush=True)
    assert max(errs) <= F32_MATH_BOUND, errs


P2D = problems()


@pytest.mark.parametrize("name", sorted(P2D))
def test_fp32_math_d2q9_parity(lbm, name):
    """FP32 node arithmetic on every D2Q9 parity case, at the 1e-5 bar: the
    collision works on departures from w_i rho (f - w_i rho and
    feq - w_i rho, both small) and closes mass on the rest population, so
    FP32 rounding stays relative to the departures, not to rho."""
    p = P2D[name]
    errs = _series(p, lbm.Solver(p, math=lbm.MATH_F32), CHECKPOINTS)
    print(f"[fp32-math-2d] {name} errors {['%.1e' % e for e in errs]}", flush=True)
    assert max(errs) <= F32_MATH_BOUND, errs


@pytest.mark.parametrize("name", sorted(P3))
@pytest.mark.parametrize("strategy", ["split", "compact"])
def test_fp32_math_d3q19_parity(lbm, name, strategy):
    """FP32 node arithmetic on every D3Q19 parity case and both 3D layouts."""
    p = P3[name]
    st = lbm.SPLIT if strategy == "split" else lbm.COMPACT
    errs = _series(p, lbm.Solver(p, math=lbm.MATH_F32, strategy=st), CHECKPOINTS)
    print(f"[fp32-math-3d] {name} {strategy} errors {['%.1e' % e for e in errs]}", flush=True)
    assert max(errs) <= F32_MATH_BOUND, errs


@pytest.mark.parametrize("strategy", sorted(STRATEGIES))
@pytest.mark.parametrize("q", [9, 19])
def test_bf16_deviation_storage_error_is_bounded(lbm, q, strategy):
    p = _drain2d() if q == 9 else P3["d3_drain_trt"]
    s = lbm.Solver(p, storage=lbm.STORE_BF16DEV, strategy=STRATEGIES[strategy])
    errs = _series(p, s, CHECKPOINTS)
    print(f"[bf16-dev] q={q} {strategy} errors {['%.1e' % e for e in errs]}", flush=True)
    assert max(errs) <= BF16_BOUND, errs


def test_bf16_storage_conserves_mass_in_a_closed_box(lbm):
    """Densities are stored exactly (FP32) and f0 is implied by them, so a
    closed box keeps each component's mass to FP32 rounding of the sums."""
    p = I.drainage_2d(nx=96, ny=40, r=(2.0, 5.0), porosity=0.7, seed=9, G=3.5, theta=60,
                      tau=I.TAU_M10, minor=0.027, collision=1)
    p.open_x, p.periodic = 0, 1
    drift = {}
    for st in (lbm.STORE_BF16DEV, lbm.STORE_F32):
        s = lbm.Solver(p, storage=st)
        m0 = s.observables()["mass"]
        s.step(1000)
        m1 = s.observables()["mass"]
        drift[st] = [abs(m1[c] - m0[c]) / m0[c] for c in range(2)]
    print(f"[mass] relative drift over 1000 steps: bf16-dev {drift[lbm.STORE_BF16DEV]}, "
          f"f32 {drift[lbm.STORE_F32]}", flush=True)
    assert max(drift[lbm.STORE_BF16DEV]) <= 1e-5


def test_bf16_batch_matches_single(lbm):
    ps = [_drain2d(), I.drainage_2d(nx=64, ny=30, r=(2.0, 4.0), porosity=0.7, seed=31, G=3.5,
                                    theta=100, tau=I.TAU_M10, rho_in1=1.015, minor=0.027,
                                    collision=1)]
    b = lbm.BatchSolver(ps, storage=lbm.STORE_BF16DEV)
    b.step(30)
    for i, p in enumerate(ps):
        s = lbm.Solver(p, storage=lbm.STORE_BF16DEV)
        s.step(30)
        assert np.array_equal(b.density(i), s.density())


@pytest.mark.parametrize("name", sorted(P3))
def test_d3q19_fused_matches_compact_step(lbm, name):
    """The compacted 3D fused step (LBM_COMPACT_FUSED: tile march with the
    next step's densities summed on chip and carried between steps) does the
    compacted split step's node arithmetic but carries psi in FP32: with FP64
    node arithmetic its densities stay within 1e-6 of the split step's over
    eager steps and graph replays, ragged tiles and z chunks, and the
    observables' counts agree exactly."""
    p = P3[name]
    a = lbm.Solver(p, strategy=lbm.COMPACT, math=lbm.MATH_F64)
    b = lbm.Solver(p, strategy=lbm.COMPACT_FUSED, math=lbm.MATH_F64)
    assert "fwd_step_d3q19" in b.kernel_info()[0] and b.kernel_info()[2] == 256
    fluid = ~p.mask.astype(bool)
    for n in (1, 36, 63):
        a.step(n)
        if n % 2 == 0:
            b.step_graph(n, 1)
        else:
            b.step(n)
        ra, rb = a.density().astype(np.float64), b.density().astype(np.float64)
        err = float((np.abs(ra - rb) / np.abs(ra))[:, fluid].max())
        print(f"[fused3d-vs-compact] {name} t={a.t} {err:.1e}", flush=True)
        assert err <= 1e-6, (name, n, err)
    oa, ob = a.observables(), b.observables()
    for k in ("n_fluid", "n_window", "n_in", "n_out"):
        assert oa[k] == ob[k]


@pytest.mark.parametrize("name", sorted(P3))
def test_d3q19_fused_parity_200_steps(lbm, name):
    """The compacted 3D fused step against the FP64 oracle, both node arithmetics."""
    p = P3[name]
    for math in (lbm.MATH_F64, lbm.MATH_F32):
        s = lbm.Solver(p, strategy=lbm.COMPACT_FUSED, math=math)
        errs = _series(p, s, CHECKPOINTS)
        print(f"[fused3d] {name} math={math} errors {['%.1e' % e for e in errs]}", flush=True)
        assert max(errs) <= (REL_TOL if math == lbm.MATH_F64 else F32_MATH_BOUND), errs


def test_d3q19_fused_carried_psi_follows_the_state(lbm):
    """The carried psi is rebuilt whenever the state changes outside a step:
    a pressure increment between graph replays, a host density read-out
    (staged through the psi buffer) and a checkpoint restored into a fresh
    context all continue exactly like an uninterrupted context that took the
    same increments, and a checkpoint resumes bit for bit."""
    p = P3["d3_drain_trt"]
    a = lbm.Solver(p, strategy=lbm.COMPACT_FUSED)
    b = lbm.Solver(p, strategy=lbm.COMPACT)
    for s in (a, b):
        s.step_graph(10, 2)
        s.set_bc(1.02, 1.0)
        s.step_graph(10, 1)
    fluid = ~p.mask.astype(bool)
    ra, rb = a.density().astype(np.float64), b.density().astype(np.float64)
    assert float((np.abs(ra - rb) / np.abs(ra))[:, fluid].max()) <= 1e-6
    blob = a.save()
    a.step(17)
    ref = a.density()
    c = lbm.Solver(p, strategy=lbm.COMPACT_FUSED)
    c.load(blob)
    c.step(17)
    assert np.array_equal(c.density(), ref)


def test_d3q19_compact_equals_split_bitwise(lbm):
    p = P3["d3_drain_trt"]
    a = lbm.Solver(p, strategy=lbm.SPLIT)
    b = lbm.Solver(p, strategy=lbm.COMPACT)
    a.step(40)
    b.step_graph(20, 2)
    assert np.array_equal(a.density(), b.density())


@pytest.mark.parametrize("strategy", ["compact", "compact_fused"])
def test_d3q19_banded_numbering_changes_nothing(lbm, strategy):
    """Fluid nodes numbered in bands of 8 rows (three bands over ny = 20, the
    last one ragged), z-slice by z-slice within a band, instead of row by row
    (what a grid this small gets by default): the node arithmetic is the same,
    so the densities are bit-identical, and they follow the oracle."""
    p = P3["d3_drain_trt"]
    st = lbm.COMPACT if strategy == "compact" else lbm.COMPACT_FUSED
    a = lbm.Solver(p, strategy=st)
    b = lbm.Solver(p, strategy=st, tile_rows=8)
    a.step(60)
    b.step(60)
    assert np.array_equal(a.density(), b.density())
    errs = _series(p, lbm.Solver(p, strategy=st, tile_rows=8), CHECKPOINTS)
    assert max(errs) <= REL_TOL, errs
