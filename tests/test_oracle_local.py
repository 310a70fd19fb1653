"""Pins of the oracle's node-local arithmetic: lattice, equilibrium (Eq. 2),
forcing (Eqs. 10-11), collision (Eq. 1 and its MRT/TRT variants) and the
Zou-He completion (Eqs. 18-25).  Every expected value comes from a closed
form or an identity, never from the oracle itself."""
import itertools

import numpy as np
import pytest

import oracle as O

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("q", [9, 19])
def test_lattice_moment_identities(q):
    e, w, opp = O.lattice(q)
    e = e.astype(float)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs(w @ e).max() < 1e-15
    I = np.eye(3)
    dim = 2 if q == 9 else 3
    I[dim:, dim:] = 0
    assert np.abs(np.einsum("i,ia,ib->ab", w, e, e) - CS2 * I).max() < 1e-15
    assert np.abs(np.einsum("i,ia,ib,ic->abc", w, e, e, e)).max() < 1e-15
    four = np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
                      + np.einsum("ad,bc->abcd", I, I))
    assert np.abs(four - iso).max() < 1e-15
    for i in range(q):
        assert np.all(e[opp[i]] == -e[i])
    if q == 9:  # the paper's D2Q9 order and weights (Sec. 2.1)
        assert e[:, :2].T.tolist() == [[0, 1, 0, -1, 0, 1, -1, -1, 1], [0, 0, 1, 0, -1, 1, 1, -1, -1]]
        assert np.allclose(w, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, rtol=0, atol=1e-16)


@pytest.mark.parametrize("q", [9, 19])
def test_equilibrium_moments(q):
    rng = np.random.default_rng(0)
    e, w, _ = O.lattice(q)
    e = e.astype(float)
    for _ in range(20):
        rho = rng.uniform(0.01, 1.5)
        u = rng.uniform(-0.1, 0.1, 3)
        if q == 9:
            u[2] = 0
        feq = O.equilibrium(q, rho, u)
        assert abs(feq.sum() - rho) < 1e-14
        assert np.abs(feq @ e - rho * u).max() < 1e-14
        P = np.einsum("i,ia,ib->ab", feq, e, e)
        dim = 2 if q == 9 else 3
        exp = rho * (CS2 * np.eye(3) + np.outer(u, u))
        assert np.abs(P[:dim, :dim] - exp[:dim, :dim]).max() < 1e-14


@pytest.mark.parametrize("q", [9, 19])
def test_forcing_moments_and_eq10_form(q):
    """Eq. 11's source has zeroth moment 0, first moment F and second moment
    uF + Fu; and it equals the Eq. 10 form, evaluated here independently."""
    rng = np.random.default_rng(1)
    e, w, _ = O.lattice(q)
    e = e.astype(float)
    dim = 2 if q == 9 else 3
    for _ in range(20):
        u = rng.uniform(-0.1, 0.1, 3)
        F = rng.uniform(-1e-2, 1e-2, 3)
        if q == 9:
            u[2] = F[2] = 0
        S = O.forcing(q, u, F)
        assert abs(S.sum()) < 1e-16
        assert np.abs(S @ e - F).max() < 1e-16
        second = np.einsum("i,ia,ib->ab", S, e, e)
        assert np.abs(second - (np.outer(u, F) + np.outer(F, u)))[:dim, :dim].max() < 1e-16
        # Eq. 10: w_i [ e.F / cs2 + (e e - cs2 I) : (u F + F u) / (2 cs2^2) ]
        uF = np.outer(u, F) + np.outer(F, u)
        eq10 = np.array([w[i] * (e[i] @ F / CS2 +
                                 np.sum((np.outer(e[i], e[i]) - CS2 * np.eye(3)) * uF)
                                 / (2 * CS2 ** 2)) for i in range(q)])
        if q == 9:  # the identity tensor is 2D there
            eq10 = np.array([w[i] * (e[i] @ F / CS2 +
                                     np.sum((np.outer(e[i], e[i])[:2, :2] - CS2 * np.eye(2)) * uF[:2, :2])
                                     / (2 * CS2 ** 2)) for i in range(q)])
        assert np.abs(eq10 - S).max() < 1e-16


def _params(q, collision, tau=(0.8, 1.7), **kw):
    return O.make_params(q=q, nx=1, ny=1, nz=1, collision=collision, tau=tau, **kw)


def _random_node(q, rng, minority=False):
    e, w, _ = O.lattice(q)
    rho = (1.0, 0.02) if minority else (rng.uniform(0.2, 1.0), rng.uniform(0.2, 1.0))
    fin = np.stack([w * r * (1 + rng.uniform(-0.2, 0.2, q)) for r in rho])
    F = rng.uniform(-1e-3, 1e-3, (2, 3))
    if q == 9:
        F[:, 2] = 0
    return fin, F


COLLISIONS = [(9, 0), (9, 1), (9, 2), (19, 0), (19, 1), (19, 2)]


@pytest.mark.parametrize("q,coll", COLLISIONS)
def test_collision_conserves_component_mass_and_adds_force(q, coll):
    """Each component's mass is conserved at the node; with the half-force
    velocity the total momentum grows by exactly F = F1 + F2 per step."""
    rng = np.random.default_rng(2)
    e, _, _ = O.lattice(q)
    e = e.astype(float)
    P = _params(q, coll)
    for trial in range(10):
        fin, F = _random_node(q, rng, minority=trial % 2 == 0)
        out = O.collide_node(P, fin, F)
        assert np.abs(out.sum(axis=1) - fin.sum(axis=1)).max() < 1e-14
        j0 = (fin @ e).sum(axis=0)
        j1 = (out @ e).sum(axis=0)
        assert np.abs(j1 - (j0 + F.sum(axis=0))).max() < 1e-15


def test_literal_velocity_reading_adds_reduced_force():
    """Without the F/2 velocity shift, Eq. 1 adds only (1 - 1/2 tau_s) F of
    momentum per step: the reason for the half-force reading."""
    rng = np.random.default_rng(3)
    e, _, _ = O.lattice(9)
    e = e.astype(float)
    P = _params(9, 0, tau=(1.0, 1.0), half_force_shift=0)
    fin, F = _random_node(9, rng)
    out = O.collide_node(P, fin, F)
    gain = (out @ e).sum(axis=0) - (fin @ e).sum(axis=0)
    assert np.abs(gain - 0.5 * F.sum(axis=0)).max() < 1e-15


@pytest.mark.parametrize("q,coll", COLLISIONS)
def test_equilibrium_is_fixed_point(q, coll):
    e, w, _ = O.lattice(q)
    u = np.array([0.03, -0.02, 0.01 if q == 19 else 0.0])
    fin = np.stack([O.equilibrium(q, r, u) for r in (0.7, 0.3)])
    out = O.collide_node(_params(q, coll), fin, np.zeros((2, 3)))
    assert np.abs(out - fin).max() < 1e-15


def test_srt_matches_closed_form():
    """SRT at one node against Eq. 1 evaluated from the closed-form moments
    of a hand-built state: both components at rest equilibrium plus a
    single perturbed population; tau_s = (rho1 tau1 + rho2 tau2)/rho."""
    q = 9
    e, w, _ = O.lattice(q)
    tau = (0.8, 1.7)
    rho = np.array([0.6, 0.4])
    fin = np.stack([w * r for r in rho])
    fin[0, 1] += 0.01  # component 1 gains mass 0.01 and momentum +0.01 x
    rho[0] += 0.01
    F = np.zeros((2, 3))
    out = O.collide_node(_params(q, 0, tau=tau), fin, F)
    tau_s = (rho[0] * tau[0] + rho[1] * tau[1]) / rho.sum()
    u = np.array([0.01 / rho.sum(), 0.0, 0.0])
    for c in range(2):
        feq = w * rho[c] * (1 + 3 * (e[:, 0] * u[0]) + 4.5 * (e[:, 0] * u[0]) ** 2 - 1.5 * u[0] ** 2)
        exp = fin[c] - (fin[c] - feq) / tau_s
        assert np.abs(out[c] - exp).max() < 1e-15


@pytest.mark.parametrize("q", [9, 19])
def test_mrt_with_equal_rates_is_srt(q):
    rng = np.random.default_rng(4)
    Pm = _params(q, 1, s_e=-1.0, s_eps=-1.0, lam=-1.0, mrt_sj_mode=0)
    Ps = _params(q, 0)
    for _ in range(10):
        fin, F = _random_node(q, rng)
        assert np.abs(O.collide_node(Pm, fin, F) - O.collide_node(Ps, fin, F)).max() < 1e-14


@pytest.mark.parametrize("q", [9, 19])
def test_mrt_with_trt_rates_is_trt(q):
    """MRT with even-moment rates s_nu and odd-moment rates s- (s_j = s_q)
    collapses to the two-relaxation-time operator."""
    rng = np.random.default_rng(5)
    Pm = _params(q, 1, s_e=-1.0, s_eps=-1.0, lam=3 / 16, mrt_sj_mode=1)
    Pt = _params(q, 2, lam=3 / 16)
    for _ in range(10):
        fin, F = _random_node(q, rng)
        assert np.abs(O.collide_node(Pm, fin, F) - O.collide_node(Pt, fin, F)).max() < 1e-14


def test_d3q19_mrt_basis_is_the_textbook_moments():
    """The D3Q19 moment matrix: its rows are mutually orthogonal; the
    conserved rows are the density and momentum; the energy row weighted by
    w gives 19 c_s^2 - 30 = -23... of the equilibrium (checked through
    sum_i w_i M_ki = <M_k> of the rest state): only rho, e and eps have a
    nonzero rest-state mean, with e = -11 and eps = 3 (per unit density)."""
    M = O.mrt_matrix(19)
    e, w, _ = O.lattice(19)
    G = M @ M.T
    assert np.abs(G - np.diag(np.diag(G))).max() == 0.0
    assert np.array_equal(M[0], np.ones(19))
    assert np.array_equal(M[3], e[:, 0]) and np.array_equal(M[5], e[:, 1]) and np.array_equal(M[7], e[:, 2])
    mean = M @ w
    assert abs(mean[0] - 1) < 1e-15 and abs(mean[1] + 11) < 1e-14 and abs(mean[2] - 3) < 1e-14
    assert np.abs(mean[3:]).max() < 1e-15
    # second-order rows: the shear moments are the traceless products of c
    c2 = (e ** 2).sum(axis=1)
    assert np.array_equal(M[9], 3 * e[:, 0] ** 2 - c2) and np.array_equal(M[13], e[:, 0] * e[:, 1])


@pytest.mark.parametrize("q", [9, 19])
def test_trt_with_equal_rates_is_srt(q):
    rng = np.random.default_rng(6)
    Pt = _params(q, 2, lam=-1.0)
    Ps = _params(q, 0)
    for _ in range(10):
        fin, F = _random_node(q, rng)
        assert np.abs(O.collide_node(Pt, fin, F) - O.collide_node(Ps, fin, F)).max() < 1e-14


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("normal", [1, -1])
def test_zouhe_identities(q, normal):
    """After completion: density equals the prescribed one, the tangential
    momentum vanishes, and the normal link obeys the non-equilibrium
    bounce-back f_n - f_opp(n) = 6 w_n j_n (Zou & He's closure)."""
    rng = np.random.default_rng(7)
    e, w, opp = O.lattice(q)
    missing = [i for i in range(q) if e[i, 0] == normal]
    axis = [i for i in missing if abs(e[i]).sum() == 1][0]
    for _ in range(10):
        f = w * rng.uniform(0.9, 1.1, q)
        f[missing] = 1e3  # garbage to be overwritten
        rho_bc = rng.uniform(0.95, 1.05)
        g = O.zouhe(q, f, rho_bc, normal)
        assert abs(g.sum() - rho_bc) < 1e-14
        j = g @ e.astype(float)
        assert abs(j[1]) < 1e-15 and abs(j[2]) < 1e-15
        assert abs((g[axis] - g[opp[axis]]) - 6 * w[axis] * (j @ e[axis])) < 1e-15
        for i in range(q):
            if i not in missing:
                assert g[i] == f[i]


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("normal", [1, -1])
def test_zouhe_recovers_equilibrium(q, normal):
    """An equilibrium with zero tangential velocity is a fixed point of the
    completion: the construction is exact for it."""
    e, w, _ = O.lattice(q)
    for rho_bc, ux in itertools.product([0.97, 1.0, 1.04], [-0.02, 0.0, 0.03]):
        feq = O.equilibrium(q, rho_bc, [ux, 0.0, 0.0])
        f = feq.copy()
        f[e[:, 0] == normal] = -5.0
        g = O.zouhe(q, f, rho_bc, normal)
        assert np.abs(g - feq).max() < 1e-15


def test_zouhe_d2q9_matches_printed_inlet_and_outlet_equations():
    """D2Q9 completion against Eqs. 22-25 (inlet) and 18-21 (outlet),
    evaluated from the paper's printed coefficients."""
    rng = np.random.default_rng(8)
    _, w, _ = O.lattice(9)
    f = w * rng.uniform(0.9, 1.1, 9)
    r = 1.02
    g = O.zouhe(9, f, r, +1)
    u = 1 - (f[0] + f[2] + f[4] + 2 * (f[3] + f[6] + f[7])) / r
    assert abs(g[1] - (f[3] + 2 / 3 * r * u)) < 1e-15
    assert abs(g[5] - (f[7] - 0.5 * (f[2] - f[4]) + r * u / 6)) < 1e-15
    assert abs(g[8] - (f[6] + 0.5 * (f[2] - f[4]) + r * u / 6)) < 1e-15
    g = O.zouhe(9, f, r, -1)
    u = -1 + (f[0] + f[2] + f[4] + 2 * (f[1] + f[5] + f[8])) / r
    assert abs(g[3] - (f[1] - 2 / 3 * r * u)) < 1e-15
    assert abs(g[6] - (f[8] - 0.5 * (f[2] - f[4]) - r * u / 6)) < 1e-15
    assert abs(g[7] - (f[5] + 0.5 * (f[2] - f[4]) - r * u / 6)) < 1e-15


def test_viscosity_reading_matches_printed_pairs(paper):
    """nu = c_s^2 (tau - 1/2): the paper's tau/nu pairs and M = 25."""
    for tau, nu in paper["viscosity_from_tau"]["pairs"]:
        assert abs(CS2 * (tau - 0.5) - nu) < 1e-15
    (t1, _), (t2, _) = paper["viscosity_from_tau"]["pairs"]
    assert abs((t1 - 0.5) / (t2 - 0.5) - paper["viscosity_from_tau"]["viscosity_ratio"]) < 1e-12


def test_mrt_momentum_rate_moves_components_not_the_total():
    """The MRT component-momentum rate s_j (mrt_sj_mode 2: s_nu; 1: s_q)
    leaves the total momentum change at F but changes how the two
    components share it: each component's momentum relaxes towards
    rho^s u at rate s_j.  Mode 0 takes the smaller of the two."""
    rng = np.random.default_rng(9)
    e, _, _ = O.lattice(9)
    e = e.astype(float)
    outs = []
    for sj in (2, 1, 0):
        P = _params(9, 1)
        P.mrt_sj_mode = sj
        fin, F = _random_node(9, np.random.default_rng(9))
        out = O.collide_node(P, fin, F)
        j0, j1 = fin @ e, out @ e
        assert np.abs(j1.sum(axis=0) - (j0.sum(axis=0) + F.sum(axis=0))).max() < 1e-15
        outs.append(j1)
    # the per-component momenta differ between the two rates, and mode 0 is
    # the one with the smaller rate
    assert np.abs(outs[0] - outs[1]).max() > 1e-6
    fin, _ = _random_node(9, np.random.default_rng(9))
    r1, r2 = fin[0].sum(), fin[1].sum()
    tau_s = (0.8 * r1 + 1.7 * r2) / (r1 + r2)
    s_nu, s_q = 1 / tau_s, (tau_s - 0.5) / ((tau_s - 0.5) / 2 + 3 / 16)
    assert np.array_equal(outs[2], outs[1] if s_q < s_nu else outs[0])
