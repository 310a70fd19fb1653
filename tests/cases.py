"""Shared GPU parity cases: D2Q9 problems covering every boundary set,
collision operator and tile edge case, at sizes the oracle runs in seconds."""
import numpy as np

from paper_2111_08666_amd import inputs as I


def _channel(nx, ny, periodic_x=True):
    m = np.zeros((ny, nx), np.uint8)
    m[0] = m[-1] = 1
    return m


def problems():
    out = {}
    # open drainage, ragged tiles (127 = 2*60 + 7 columns, 37 = 3*12 + 1 rows)
    out["drain_srt"] = I.drainage_2d(nx=127, ny=37, r=(2.0, 5.0), porosity=0.7, seed=11, G=3.5,
                                     theta=45, tau=(1.0, 0.8), rho_in1=1.02, minor=0.027)
    out["drain_mrt"] = I.drainage_2d(nx=127, ny=37, r=(2.0, 5.0), porosity=0.7, seed=12, G=3.5,
                                     theta=60, tau=I.TAU_M10, rho_in1=1.01, minor=0.027, collision=1)
    out["drain_trt"] = I.drainage_2d(nx=127, ny=37, r=(2.0, 5.0), porosity=0.7, seed=13, G=3.5,
                                     theta=120, tau=I.TAU_M10, rho_in1=1.01, minor=0.027, collision=2)
    out["small_drainage_G0.9"] = I.small_drainage()
    for s in (1, 2):
        p = I.drainage_2d(nx=70, ny=26, r=(2.0, 4.0), porosity=0.75, seed=20 + s, G=3.5, theta=50,
                          rho_in1=1.02, minor=0.027)
        p.bc_set = s
        p.rho_in2, p.rho_out1 = 0.027, 0.027
        out[f"set{s}"] = p
    # the post-collision reading of Eqs. 26-27, Set-2 and Set-3
    for s in (2, 3):
        p = I.drainage_2d(nx=70, ny=26, r=(2.0, 4.0), porosity=0.75, seed=30 + s, G=3.5, theta=50,
                          rho_in1=1.02, minor=0.027)
        p.bc_set, p.eq26_mode = s, 1
        out[f"set{s}_eq26_post"] = p
    # periodic droplet (Laplace case), both axes periodic
    n = 64
    out["droplet_periodic"] = I.Problem(
        q=9, mask=np.zeros((n, n), np.uint8),
        rho0=I.tanh_droplet((n, n), (n / 2, n / 2), 14, (1.0, 0.027), (0.027, 1.0)),
        periodic=3, open_x=0, tau=(1.0, 1.0), G=3.5, collision=0)
    # sessile droplet on a wall, periodic x (contact-angle case)
    m = _channel(96, 48)
    out["droplet_wall_mrt"] = I.Problem(
        q=9, mask=m, rho0=I.tanh_droplet((48, 96), (48, 0.5), 15, (1.0, 0.027), (0.027, 1.0), mask=m),
        periodic=1, open_x=0, tau=(1.7, 0.62), G=3.5, xi=-0.3, collision=1)
    # smaller than one tile, body-force driven channel
    m = _channel(10, 8)
    r0 = np.zeros((2, 8, 10))
    r0[0], r0[1] = 1.0, 0.03
    r0[:, m.astype(bool)] = 0
    out["tiny_poiseuille"] = I.Problem(q=9, mask=m, rho0=r0, periodic=1, open_x=0, tau=(0.9, 0.9),
                                       G=3.5, g=(1e-5, 0.0, 0.0), collision=2)
    # exact multiple of the tile, literal velocity reading
    p = I.drainage_2d(nx=120, ny=24, r=(2.0, 4.0), porosity=0.75, seed=14, G=3.5, theta=45,
                      rho_in1=1.02, minor=0.027)
    p.half_force_shift = 0
    out["tile_multiple_literal"] = p
    return out
