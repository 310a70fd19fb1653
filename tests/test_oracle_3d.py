"""Pins of the oracle's D3Q19 path (the 3D generalisation of Sec. 2: Eq. 1
streaming with half-way bounce-back, the Eq. 13 stencil, Eq. 17 and the
collision) against the mathematics, so that a mistake in the z branch of the
neighbour and wrap logic fails a test:
  - a momentum pulse streams one node along its velocity, across a periodic
    z edge, or comes back reversed off a z wall;
  - translation on a periodic box of unequal sides is bitwise;
  - a box closed by z walls conserves each component's mass to round-off;
  - the force of a pseudopotential linear in z is the exact gradient, and the
    virtual solid density of a z wall is the weighted mean of Eq. 17;
  - pressure-free channel flow between z walls (and y walls) is the exact
    parabola for TRT at the magic parameter 3/16."""
import numpy as np
import pytest

import oracle as O

CS2 = 1.0 / 3.0


def _box(shape, periodic, mask=None, rho0=None, **kw):
    nz, ny, nx = shape
    if mask is None:
        mask = np.zeros(shape, np.uint8)
    if rho0 is None:
        rho0 = np.zeros((2,) + shape)
        rho0[0] = 1.0
    P = O.make_params(q=19, nx=nx, ny=ny, nz=nz, periodic=periodic, open_x=0, **kw)
    return O.OracleSim(params=P, mask=mask, rho0=rho0)


def _pulse_momentum(shape, periodic, mask, node, i):
    """Rest state (rho = 1 of component 1 on fluid nodes) plus 1/10 in
    post-collision population i at `node`; one step of SRT at tau = 1 with
    no force makes each node's post-collision state its equilibrium, whose
    momentum is the streamed momentum.  Returns the momentum field (3, ...)."""
    e, w, _ = O.lattice(19)
    s = _box(shape, periodic, mask=mask, G=0.0, tau=(1.0, 1.0), collision=0)
    fs = np.zeros((2, 19) + shape)
    fluid = ~mask.astype(bool)
    fs[0] = w[:, None, None, None] * fluid[None]
    fs[(0, i) + node] += 0.1
    s.set_fstar(fs)
    s.step(1)
    out = s.fstar()
    return np.einsum("cqzyx,qd->dzyx", out, e.astype(float))


@pytest.mark.parametrize("i", range(1, 19))
def test_pulse_streams_across_the_periodic_z_edge(i):
    """Every link from a node on the last z plane (and the last x, y
    column) lands on x + e_i, wrapped in x, y and z (sides 5, 6, 7)."""
    shape = (7, 6, 5)
    e, _, _ = O.lattice(19)
    mask = np.zeros(shape, np.uint8)
    node = (6, 5, 4)  # (z, y, x)
    j = _pulse_momentum(shape, 7, mask, node, i)
    dest = tuple((node[k] + e[i][2 - k]) % shape[k] for k in range(3))
    exp = np.zeros_like(j)
    exp[(slice(None),) + dest] = 0.1 * e[i]
    assert np.abs(j - exp).max() < 1e-15


@pytest.mark.parametrize("i", range(1, 19))
def test_pulse_bounces_back_off_a_z_wall(i):
    """Solid planes z = 0 and z = nz - 1, periodic x and y: a link leaving
    plane z = 1 towards the wall (e_z = -1) comes back reversed at the same
    node (half-way bounce-back); other links stream on."""
    shape = (6, 5, 4)
    e, _, opp = O.lattice(19)
    mask = np.zeros(shape, np.uint8)
    mask[0] = mask[-1] = 1
    node = (1, 2, 3)
    j = _pulse_momentum(shape, 3, mask, node, i)
    exp = np.zeros_like(j)
    if e[i][2] == -1:
        exp[(slice(None),) + node] = 0.1 * e[opp[i]]
    else:
        dest = (node[0] + e[i][2], (node[1] + e[i][1]) % 5, (node[2] + e[i][0]) % 4)
        exp[(slice(None),) + dest] = 0.1 * e[i]
    assert np.abs(j - exp).max() < 1e-15


def test_periodic_translation_is_bitwise_3d():
    rng = np.random.default_rng(5)
    shape = (9, 8, 7)
    mask = (rng.uniform(size=shape) < 0.12).astype(np.uint8)
    rho0 = np.stack([rng.uniform(0.05, 1.0, shape), rng.uniform(0.05, 1.0, shape)])
    rho0[:, mask.astype(bool)] = 0
    kw = dict(G=3.5, xi=-0.3, tau=(0.8, 1.3), collision=2)
    shift = (4, 3, 5)
    a = _box(shape, 7, mask=mask, rho0=rho0, **kw)
    b = _box(shape, 7, mask=np.roll(mask, shift, (0, 1, 2)), rho0=np.roll(rho0, shift, (1, 2, 3)), **kw)
    a.step(25)
    b.step(25)
    assert np.array_equal(np.roll(a.density(), shift, (1, 2, 3)), b.density())


def test_box_closed_by_z_walls_conserves_mass():
    rng = np.random.default_rng(6)
    shape = (10, 9, 8)
    mask = (rng.uniform(size=shape) < 0.1).astype(np.uint8)
    mask[0] = mask[-1] = 1
    rho0 = np.zeros((2,) + shape)
    rho0[0] = np.where(np.arange(8)[None, None, :] < 4, 1.0, 0.027)
    rho0[1] = np.where(np.arange(8)[None, None, :] < 4, 0.027, 1.0)
    rho0[:, mask.astype(bool)] = 0
    s = _box(shape, 3, mask=mask, rho0=rho0, G=3.5, xi=-0.3, tau=(1.7, 0.62), collision=2)
    m0 = s.observables()["mass"]
    s.step(300)
    m1 = s.observables()["mass"]
    for c in range(2):
        assert abs(m1[c] - m0[c]) / m0[c] < 1e-12


def test_force_of_pseudopotential_linear_in_z_is_exact_gradient():
    """With psi linear in z, sum_i w_i psi(x + e_i) e_i = c_s^2 grad psi, so
    F^s = -G rho^s c_s^2 dpsi^sbar/dz, with no x or y component."""
    shape = (12, 5, 4)
    z = np.arange(12)[:, None, None] * np.ones(shape)
    rho0 = np.stack([0.5 + 0.01 * z, 0.8 - 0.02 * z])
    mask = np.zeros(shape, np.uint8)
    mask[0] = mask[-1] = 1
    rho0[:, mask.astype(bool)] = 0
    G = 2.0
    s = _box(shape, 3, mask=mask, rho0=rho0, G=G, tau=(1.0, 1.0))
    F = s.force()
    rho = s.density()
    # planes whose neighbours z - 1 .. z + 1 all lie in 2 .. 9, where the
    # streamed density is still linear (planes 1 and 10 receive bounce-back)
    inner = slice(3, 9)
    for c, slope_other in ((0, -0.02), (1, 0.01)):
        exp = -G * rho[c, inner] * CS2 * slope_other
        assert np.abs(F[c, 2, inner] - exp).max() < 1e-15
        assert np.abs(F[c, 0, inner]).max() < 1e-15 and np.abs(F[c, 1, inner]).max() < 1e-15


@pytest.mark.parametrize("xi", [-0.4, 0.3])
def test_ivsd_of_a_z_wall_is_the_weighted_mean(xi):
    """At a solid node of the wall z = 0 the fluid neighbours are the five
    links with e_z = +1: (0,0,1) with weight 1/18 and (+-1,0,1), (0,+-1,1)
    with 1/36.  Eq. 17 gives chi^s times their weighted mean."""
    shape = (6, 5, 8)
    x = np.arange(8)[None, None, :] * np.ones(shape)
    rho0 = np.stack([0.2 + 0.05 * x, 1.0 - 0.03 * x])
    mask = np.zeros(shape, np.uint8)
    mask[0] = mask[-1] = 1
    rho0[:, mask.astype(bool)] = 0
    s = _box(shape, 3, mask=mask, rho0=rho0, G=3.5, xi=xi, tau=(1.0, 1.0))
    psi = s.psi()
    rho = s.density()
    for c, chi in ((0, 1 + xi), (1, 1 - xi)):
        r = rho[c, 1, 2]  # plane z = 1, row y = 2
        mean = (r / 18 + (np.roll(r, 1) + np.roll(r, -1)) / 36 + 2 * r / 36) / (1 / 18 + 4 / 36)
        assert np.abs(psi[c, 0, 2] - chi * mean).max() < 1e-15


def _channel3d_error(wall_axis, collision, tau, n=21, steps=20000):
    """Channel between two solid planes normal to `wall_axis` ('z' or 'y'),
    periodic otherwise, driven by F^s = rho^s g along x.  A uniform mixture
    (1, 0.03) at G = 3.5, xi = 0 is force-free, so only the body force acts.
    Analytic: u(s) = g/(2 nu) (s - 1/2)(n - 3/2 - s), nu = (tau - 1/2)/3."""
    shape = (n, 4, 4) if wall_axis == "z" else (4, n, 4)
    mask = np.zeros(shape, np.uint8)
    if wall_axis == "z":
        mask[0] = mask[-1] = 1
        per = 3
    else:
        mask[:, 0] = mask[:, -1] = 1
        per = 5
    rho0 = np.zeros((2,) + shape)
    rho0[0], rho0[1] = 1.0, 0.03
    rho0[:, mask.astype(bool)] = 0
    g = 1e-6
    s = _box(shape, per, mask=mask, rho0=rho0, G=3.5, xi=0.0, tau=(tau, tau), collision=collision,
             g=(g, 0.0, 0.0), lam=3 / 16)
    s.step(steps)
    fs = s.fstar()
    e, _, _ = O.lattice(19)
    rho = fs.sum(axis=(0, 1))
    jx = np.einsum("cqzyx,q->zyx", fs, e[:, 0].astype(float))
    u = (jx - 0.5 * g * rho) / np.where(rho > 0, rho, 1.0)
    prof = u[1:-1, 1, 1] if wall_axis == "z" else u[1, 1:-1, 1]
    sc = np.arange(1, n - 1)
    ua = g / (2 * (tau - 0.5) / 3) * (sc - 0.5) * (n - 1.5 - sc)
    return np.abs(prof - ua).max() / ua.max()


@pytest.mark.parametrize("wall_axis", ["z", "y"])
@pytest.mark.parametrize("tau", [1.7, 1.0])
def test_channel_flow_exact_for_trt_at_magic_lambda_3d(wall_axis, tau):
    assert _channel3d_error(wall_axis, 2, tau, steps=25000) < 1e-7


@pytest.mark.parametrize("tau", [1.7, 1.0])
def test_channel_flow_exact_for_mrt_at_magic_lambda_3d(tau):
    """The D3Q19 MRT (d'Humieres moments, default component-momentum rate)
    gives the exact parabola between z walls at the magic parameter."""
    assert _channel3d_error("z", 1, tau, steps=25000) < 1e-7


def test_channel_flow_exact_for_srt_at_magic_tau_3d():
    assert _channel3d_error("z", 0, 0.5 + np.sqrt(3) / 4, steps=30000) < 1e-9
