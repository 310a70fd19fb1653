"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module holds no part of the lattice Boltzmann arithmetic.  It only
draws geometries (solid masks), initial density fields and parameter sets,
with the shapes and value ranges of the paper's workloads:

* 2D porous media bounded by solid walls, with solid-free inlet and outlet
  reservoirs (Sec. 4.2.1: a heterogeneous medium between two walls, with
  the first and last layers cleared to act as fluid reservoirs).  The
  paper's own block geometry is not available, so non-overlapping random
  discs stand in for it.
* 3D media of overlapping random spheres (the 3D extension named as future
  work in Sec. 5).
* Initial densities: a sharp non-wetting reservoir front (Sec. 4.2.1) and the
  tanh droplet profile of Eq. 29 (Sec. 3.1).
* The contact angle to wettability parameter conversion, by inverting the
  cubic fit of Sec. 3.3 (Fig. 6 caption text).

Arrays are numpy, C order, with x the fastest index: a 2D field has shape
(ny, nx) and a 3D field (nz, ny, nx).  Masks are uint8 with 1 = solid.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict

import numpy as np

# ---------------------------------------------------------------------------
# contact angle <-> xi (Sec. 3.3 cubic fit)
# ---------------------------------------------------------------------------
FIT_COEFFS = (47.5487, -13.9067, 92.0987, 90.8074)  # theta = a xi^3 + b xi^2 + c xi + d


def theta_of_xi(xi: float) -> float:
    """Contact angle in degrees (through component 2) from the Sec. 3.3 fit."""
    a, b, c, d = FIT_COEFFS
    return ((a * xi + b) * xi + c) * xi + d


def xi_of_theta(theta_deg: float) -> float:
    """Invert the Sec. 3.3 cubic fit.  Its derivative 3a xi^2 + 2b xi + c has
    a negative discriminant, so the fit is strictly increasing and the
    inverse is unique; bisection on [-1, 1]."""
    lo, hi = -1.0, 1.0
    if not (theta_of_xi(lo) <= theta_deg <= theta_of_xi(hi)):
        raise ValueError(f"theta={theta_deg} outside the fit range")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if theta_of_xi(mid) < theta_deg:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


# ---------------------------------------------------------------------------
# geometry
# ---------------------------------------------------------------------------
def disc_medium(nx: int, ny: int, r_min: float, r_max: float, porosity: float,
                seed: int, reservoir: int = 8, gap: float = 1.0,
                walls: bool = True, max_attempts: int = 200000) -> np.ndarray:
    """Random sequential addition of non-overlapping discs.

    Discs (radius ~ U[r_min, r_max]) are placed with their whole extent inside
    the porous window reservoir <= x < nx - reservoir and at least `gap`
    lattice units from the walls and from each other, until the window's
    porosity drops to `porosity` or `max_attempts` draws fail.
    Rows y = 0 and y = ny - 1 are solid walls when `walls`.
    """
    rng = np.random.default_rng(seed)
    mask = np.zeros((ny, nx), dtype=np.uint8)
    if walls:
        mask[0, :] = 1
        mask[-1, :] = 1
    x_lo, x_hi = reservoir, nx - reservoir
    y_lo, y_hi = (1, ny - 1) if walls else (0, ny)
    win = (slice(y_lo, y_hi), slice(x_lo, x_hi))
    n_win = (y_hi - y_lo) * (x_hi - x_lo)
    cx = np.empty(0)
    cy = np.empty(0)
    cr = np.empty(0)
    yy, xx = np.mgrid[0:ny, 0:nx]
    solid_win = 0
    attempts = 0
    while attempts < max_attempts:
        if 1.0 - solid_win / n_win <= porosity:
            break
        batch = 256
        r = rng.uniform(r_min, r_max, batch)
        x = rng.uniform(x_lo + r + gap * 0.5, x_hi - r - gap * 0.5)
        y = rng.uniform(y_lo + r + gap, y_hi - 1 - r - gap)
        for k in range(batch):
            attempts += 1
            if x[k] - r[k] < x_lo or x[k] + r[k] > x_hi - 1:
                continue
            if y[k] - r[k] < y_lo + gap or y[k] + r[k] > y_hi - 1 - gap:
                continue
            if cx.size:
                d2 = (cx - x[k]) ** 2 + (cy - y[k]) ** 2
                if np.any(d2 < (cr + r[k] + gap) ** 2):
                    continue
            cx = np.append(cx, x[k])
            cy = np.append(cy, y[k])
            cr = np.append(cr, r[k])
            x0, x1 = int(math.floor(x[k] - r[k])), int(math.ceil(x[k] + r[k])) + 1
            y0, y1 = int(math.floor(y[k] - r[k])), int(math.ceil(y[k] + r[k])) + 1
            sub = (slice(y0, y1), slice(x0, x1))
            inside = (xx[sub] - x[k]) ** 2 + (yy[sub] - y[k]) ** 2 <= r[k] ** 2
            mask[sub][inside] = 1
            solid_win = int(mask[win].sum())
            if 1.0 - solid_win / n_win <= porosity:
                break
    return mask


def sphere_medium(nx: int, ny: int, nz: int, r_min: float, r_max: float,
                  porosity: float, seed: int, reservoir: int = 8) -> np.ndarray:
    """Boolean (overlapping) random spheres in the window reservoir <= x <
    nx - reservoir, added until the window porosity drops to `porosity`.
    The lateral faces y, z in {0, n-1} are solid walls.  Returns (nz, ny, nx)."""
    rng = np.random.default_rng(seed)
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    mask[:, 0, :] = 1
    mask[:, -1, :] = 1
    mask[0, :, :] = 1
    mask[-1, :, :] = 1
    x_lo, x_hi = reservoir, nx - reservoir
    win = mask[1:-1, 1:-1, x_lo:x_hi]
    n_win = win.size
    solid = int(win.sum())
    while 1.0 - solid / n_win > porosity:
        r = rng.uniform(r_min, r_max)
        c = (rng.uniform(x_lo, x_hi), rng.uniform(1, ny - 1), rng.uniform(1, nz - 1))
        x0, x1 = max(x_lo, int(math.floor(c[0] - r))), min(x_hi, int(math.ceil(c[0] + r)) + 1)
        y0, y1 = max(1, int(math.floor(c[1] - r))), min(ny - 1, int(math.ceil(c[1] + r)) + 1)
        z0, z1 = max(1, int(math.floor(c[2] - r))), min(nz - 1, int(math.ceil(c[2] + r)) + 1)
        if x0 >= x1 or y0 >= y1 or z0 >= z1:
            continue
        zz, yy, xx = np.ogrid[z0:z1, y0:y1, x0:x1]
        inside = (xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2 <= r * r
        sub = mask[z0:z1, y0:y1, x0:x1]
        solid += int(np.count_nonzero(inside & (sub == 0)))
        sub[inside] = 1
    return mask


# ---------------------------------------------------------------------------
# initial densities
# ---------------------------------------------------------------------------
def close_narrow_throats(mask: np.ndarray) -> np.ndarray:
    """2D mask with its under-resolved pores closed, for long runs that
    reverse the flow:
    - every one-node-wide passage (a fluid node with solid on both sides
      along x or along y), repeated until none is left;
    - every fluid region not side-connected (4-connectivity) to the region
      that holds the inlet column (pockets reached only through diagonal
      links where two discs nearly touch).
    A diffuse interface (about five nodes wide) cannot resolve such pores;
    with strong wetting the wetting density in them can grow without bound."""
    from scipy import ndimage
    m = mask.astype(bool).copy()
    while True:
        pad = np.pad(m, 1, constant_values=False)
        sx = pad[1:-1, :-2] & pad[1:-1, 2:]
        sy = pad[:-2, 1:-1] & pad[2:, 1:-1]
        fill = ~m & (sx | sy)
        if not fill.any():
            break
        m |= fill
    lab, _ = ndimage.label(~m)  # 4-connectivity
    keep = np.unique(lab[:, 0][lab[:, 0] > 0])
    m |= ~np.isin(lab, keep)
    return m.astype(np.uint8)


def reservoir_front(mask: np.ndarray, front_x: int, rho_major: float = 1.0,
                    rho_minor: float = 0.01) -> np.ndarray:
    """Sharp initial front (Sec. 4.2.1): component 1 (non-wetting, invading)
    is the major component for x < front_x and the minor one elsewhere;
    component 2 is the reverse.  Returns (2, *mask.shape) float64, with
    zeros on solid nodes."""
    shape = mask.shape
    x = np.broadcast_to(np.arange(shape[-1]), shape)
    rho1 = np.where(x < front_x, rho_major, rho_minor)
    rho2 = np.where(x < front_x, rho_minor, rho_major)
    out = np.stack([rho1, rho2]).astype(np.float64)
    out[:, mask.astype(bool)] = 0.0
    return out


def tanh_droplet(shape, center, r0: float, rho_in=(1.0, 0.02), rho_out=(0.02, 1.0),
                 width: float = 5.0, mask: np.ndarray | None = None) -> np.ndarray:
    """Eq. 29 (Sec. 3.1): diffuse droplet of component 1 in component 2.
    rho_in[s] / rho_out[s] are component s's densities inside / outside."""
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    # grids are in (.., y, x) order; center is given as (x, y[, z])
    d2 = np.zeros(shape)
    for axis, c in enumerate(reversed(center)):
        d2 = d2 + (grids[axis] - c) ** 2
    t = np.tanh(2.0 * (np.sqrt(d2) - r0) / width)
    out = np.empty((2,) + tuple(shape))
    for s in range(2):
        out[s] = 0.5 * (rho_in[s] + rho_out[s]) - 0.5 * (rho_in[s] - rho_out[s]) * t
    if mask is not None:
        out[:, mask.astype(bool)] = 0.0
    return out


# ---------------------------------------------------------------------------
# problem descriptions
# ---------------------------------------------------------------------------
@dataclass
class Problem:
    """Everything either solver needs to run one instance."""
    q: int
    mask: np.ndarray            # (ny, nx) or (nz, ny, nx), uint8, 1 = solid
    rho0: np.ndarray            # (2, *mask.shape) float64
    periodic: int = 0           # bit0 x, bit1 y, bit2 z
    open_x: int = 1             # pressure inlet at x = 0, outlet at x = nx - 1
    porous_x0: int = 0
    porous_x1: int = 0          # 0 -> nx
    bc_set: int = 3
    collision: int = 0          # 0 SRT, 1 MRT (D2Q9), 2 TRT
    half_force_shift: int = 1
    mrt_sj_mode: int = 0
    tau: tuple = (1.0, 1.0)
    G: float = 3.5
    xi: float = 0.0
    rho_in1: float = 1.0
    rho_out2: float = 1.0
    rho_in2: float = 0.0
    rho_out1: float = 0.0
    g: tuple = (0.0, 0.0, 0.0)
    lam: float = 3.0 / 16.0
    s_e: float = 1.0
    s_eps: float = 1.0
    eq26_mode: int = 0          # Eqs. 26-27: 0 held initial values, 1 own post-collision values
    ivsd_frozen: int = 0        # Eq. 17: 0 every step, 1 once on the initial densities
    name: str = ""

    @property
    def nx(self):
        return self.mask.shape[-1]

    @property
    def ny(self):
        return self.mask.shape[-2]

    @property
    def nz(self):
        return self.mask.shape[0] if self.mask.ndim == 3 else 1

    @property
    def n_nodes(self):
        return int(self.mask.size)

    @property
    def n_fluid(self):
        return int(self.mask.size - np.count_nonzero(self.mask))


TAU_M10 = (1.7, 0.62)  # nu = 0.4 / 0.04: viscosity ratio 10 (tau - 1/2 reading of Eq. 7)


def drainage_2d(nx=128, ny=64, r=(3.0, 8.0), porosity=0.60, seed=1, G=0.9,
                theta=45.0, tau=(0.8, 1.0), rho_in1=1.05, rho_out2=1.0,
                reservoir=8, minor=0.01, collision=0, name="drainage_2d") -> Problem:
    """2D primary drainage in a disc medium: non-wetting component 1 in the
    inlet reservoir, the medium saturated with wetting component 2."""
    mask = disc_medium(nx, ny, r[0], r[1], porosity, seed, reservoir=reservoir)
    rho0 = reservoir_front(mask, reservoir, 1.0, minor)
    return Problem(q=9, mask=mask, rho0=rho0, periodic=0, open_x=1,
                   porous_x0=reservoir, porous_x1=nx - reservoir, tau=tuple(tau),
                   G=G, xi=xi_of_theta(theta), rho_in1=rho_in1, rho_out2=rho_out2,
                   collision=collision, name=name)


def small_drainage() -> Problem:
    """D2Q9 128x64 disc medium (radii 3-8, porosity 0.6, seed 1), G = 0.9,
    45 degree adhesion, tau_w = 1.0, tau_nw = 0.8; 5000-step run."""
    return drainage_2d(name="d2q9_128x64_drainage_G0.9")


def large_drainage(collision=1) -> Problem:
    """D2Q9 1024x512 disc medium (radii 4-20, porosity 0.55, seed 2), viscosity
    ratio 10 with the MRT collision, G = 3.5, xi = -0.4 (about 50 degrees)."""
    p = drainage_2d(nx=1024, ny=512, r=(4.0, 20.0), porosity=0.55, seed=2, G=3.5,
                    theta=theta_of_xi(-0.4), tau=TAU_M10, rho_in1=1.0 + 3 * 1e-3,
                    rho_out2=1.0, minor=0.027, collision=collision,
                    name="d2q9_1024x512_drainage_M10")
    p.xi = -0.4
    return p


def drainage_3d(n=384, r=(6.0, 14.0), porosity=0.40, seed=5, theta=60.0,
                dp=5e-3, reservoir=8, collision=2, nxyz=None) -> Problem:
    """D3Q19 Boolean-sphere medium (radii 6-14, porosity 0.4, seed 5),
    viscosity ratio 10 (TRT), G = 3.5, 60 degrees, pressure step dp."""
    nx, ny, nz = nxyz if nxyz is not None else (n, n, n)
    mask = sphere_medium(nx, ny, nz, r[0], r[1], porosity, seed, reservoir=reservoir)
    rho0 = reservoir_front(mask, reservoir, 1.0, 0.027)
    return Problem(q=19, mask=mask, rho0=rho0, periodic=0, open_x=1,
                   porous_x0=reservoir, porous_x1=nx - reservoir, tau=TAU_M10,
                   G=3.5, xi=xi_of_theta(theta), rho_in1=1.0 + 3 * dp,
                   rho_out2=1.0, collision=collision,
                   name=f"d3q19_{nx}x{ny}x{nz}_drainage_M10")


def fluid_box_3d(n=384, tau=TAU_M10, collision=2) -> Problem:
    """D3Q19 all-fluid periodic n^3 box holding two flat layers (component 1
    in x < n/2): the upper bound of the 3D step, every node a fluid node."""
    mask = np.zeros((n, n, n), dtype=np.uint8)
    rho0 = np.empty((2, n, n, n))
    rho0[0], rho0[1] = 0.027, 1.0
    rho0[0, :, :, : n // 2], rho0[1, :, :, : n // 2] = 1.0, 0.027
    return Problem(q=19, mask=mask, rho0=rho0, periodic=7, open_x=0, tau=tau, G=3.5,
                   collision=collision, name=f"d3q19_{n}^3_fluid_box_M10")


def batch_instances(k_count=64, seed0=300, nx_range=(256, 1024), collision=1):
    """Uneven batch: instance k has NX a multiple of 64 in nx_range, NY = NX/2,
    its own disc medium (radii 4-20, porosity 0.55, seed seed0 + k), a contact
    angle ~ U[30, 150] and a pressure step log-uniform on [1e-4, 5e-3]."""
    rng = np.random.default_rng(seed0)
    out = []
    for k in range(k_count):
        nx = int(rng.integers(nx_range[0] // 64, nx_range[1] // 64 + 1)) * 64
        theta = float(rng.uniform(30.0, 150.0))
        dp = float(10 ** rng.uniform(math.log10(1e-4), math.log10(5e-3)))
        p = drainage_2d(nx=nx, ny=nx // 2, r=(4.0, 20.0), porosity=0.55,
                        seed=seed0 + k, G=3.5, theta=theta, tau=TAU_M10,
                        rho_in1=1.0 + 3 * dp, rho_out2=1.0, minor=0.027,
                        collision=collision, name=f"batch{k}_{nx}x{nx // 2}")
        p.theta = theta
        p.dp = dp
        out.append(p)
    return out


def surrogate_mask(k: int, seed0: int = 40000, n: int = 256) -> np.ndarray:
    """Solid map of surrogate instance k (radii 4-20, porosity 0.55)."""
    return disc_medium(n, n, 4.0, 20.0, 0.55, seed0 + k, reservoir=8)


def surrogate_instance(k: int, seed0: int = 40000, n: int = 256, collision: int = 1,
                       mask: np.ndarray | None = None) -> Problem:
    """Instance k of the surrogate's data set: an n x n disc medium (seed
    seed0 + k) with a contact angle ~ U[30, 150] and a pressure step
    log-uniform on [1e-4, 5e-3], drawn from their own stream so that instance
    k does not depend on how many are generated.  `mask` may pass a solid map
    already made by surrogate_mask(k, seed0, n)."""
    rng = np.random.default_rng([seed0, k])
    theta = float(rng.uniform(30.0, 150.0))
    dp = float(10 ** rng.uniform(math.log10(1e-4), math.log10(5e-3)))
    if mask is None:
        mask = surrogate_mask(k, seed0, n)
    rho0 = reservoir_front(mask, 8, 1.0, 0.027)
    p = Problem(q=9, mask=mask, rho0=rho0, periodic=0, open_x=1, porous_x0=8, porous_x1=n - 8,
                tau=TAU_M10, G=3.5, xi=xi_of_theta(theta), rho_in1=1.0 + 3 * dp, rho_out2=1.0,
                collision=collision, name=f"surrogate{k}_{n}x{n}")
    # the trained network's fields were generated with s_j = s_nu
    p.mrt_sj_mode = 2
    p.theta = theta
    p.dp = dp
    return p


# U-shaped obstacle of the trapped-volume study (Sec. 4.1).  The paper gives
# the channel (800 x 200), the droplet radius (30) and the parameters, not the
# obstacle's dimensions; these are chosen so that the cup is well inside the
# channel with two open passages of equal width.
U_TRAP = dict(nx=800, ny=200, bar_x=300, thick=6, y0=50, y1=150, arm=120, drop_r=30.0)


def u_trap_mask(nx=800, ny=200, bar_x=300, thick=6, y0=50, y1=150, arm=120, **_) -> np.ndarray:
    """Channel with solid top and bottom rows and a U-shaped wall: a vertical
    bar facing the inlet and two arms pointing downstream, so the cup opens
    towards the outlet."""
    m = np.zeros((ny, nx), np.uint8)
    m[0] = m[-1] = 1
    m[y0:y1, bar_x:bar_x + thick] = 1                       # bar
    m[y0:y0 + thick, bar_x:bar_x + arm] = 1                 # lower arm
    m[y1 - thick:y1, bar_x:bar_x + arm] = 1                 # upper arm
    return m


def u_trap_cup(nx=800, ny=200, bar_x=300, thick=6, y0=50, y1=150, arm=120, **_) -> np.ndarray:
    """Boolean map of the cup's interior (where component 2 gets trapped)."""
    cup = np.zeros((ny, nx), bool)
    cup[y0 + thick:y1 - thick, bar_x + thick:bar_x + arm] = True
    return cup


def u_trap(bc_set: int = 3, collision: int = 0, minor: float = 0.027, **geom) -> Problem:
    """Trapped-volume case of Sec. 4.1: the channel starts full of component 2
    (wetting), with a semicircular droplet of component 1 (radius 30, tanh
    profile) on the inlet face of the U's bar and an 8-column inlet
    reservoir of component 1; tau = (3.5, 0.62) (M = 25), G = 3.5,
    xi = -0.4, inlet density 1.01 (component 1) and outlet density 1
    (component 2).  Set-1 also fixes component 2 at the inlet and component 1
    at the outlet to the minor density."""
    g = dict(U_TRAP)
    g.update(geom)
    mask = u_trap_mask(**g)
    rho0 = reservoir_front(mask, 8, 1.0, minor)
    cy = 0.5 * (g["y0"] + g["y1"])
    drop = tanh_droplet(mask.shape, (g["bar_x"], cy), g["drop_r"], (1.0, minor), (minor, 1.0), mask=mask)
    x = np.arange(mask.shape[1])[None, :]
    upstream = np.broadcast_to(x < g["bar_x"], mask.shape)
    for s in range(2):
        rho0[s] = np.where(upstream & (x >= 8), drop[s], rho0[s])
    rho0[:, mask.astype(bool)] = 0.0
    p = Problem(q=9, mask=mask, rho0=rho0, periodic=0, open_x=1, porous_x0=8, porous_x1=g["nx"] - 8,
                bc_set=bc_set, collision=collision, tau=(3.5, 0.62), G=3.5, xi=-0.4, rho_in1=1.01,
                rho_out2=1.0, rho_in2=minor, rho_out1=minor, name=f"u_trap_set{bc_set}")
    return p


def as_dict(p: Problem) -> dict:
    d = asdict(p)
    d.pop("mask")
    d.pop("rho0")
    d.update(nx=p.nx, ny=p.ny, nz=p.nz)
    return d
