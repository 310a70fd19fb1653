"""Measurements taken on density fields, shared by the oracle's physics pins
and the GPU runs of the same benchmarks: the Laplace-law point (Sec. 3.2)
and the contact angle of a sessile droplet (Sec. 3.3).  They read fields
only; neither the oracle nor the library is called from here."""
import numpy as np


def laplace_point(r, G):
    """(1/R, dP with the ordered-pair reading of Eq. 14, dP with the
    unordered-pair reading) of a droplet of component 1 centred in a
    periodic n x n box: pressure P = (rho1 + rho2)/3 + k G rho1 rho2 / 3
    inside (centre node) minus outside (corner node), R from the droplet's
    area, counting each node by its interpolated component-1 fraction."""
    n = r.shape[-1]
    dP = {k: ((r[0] + r[1]) / 3 + k * G / 3 * r[0] * r[1]) for k in (1.0, 0.5)}
    inside, outside = r[0, n // 2, n // 2], r[0, 0, 0]
    R = np.sqrt(((r[0] - outside) / (inside - outside)).sum() / np.pi)
    return 1.0 / R, dP[1.0][n // 2, n // 2] - dP[1.0][0, 0], dP[0.5][n // 2, n // 2] - dP[0.5][0, 0]


def contact_angle(r, ywall=0.5, h=5.0):
    """Contact angle through component 2 of a droplet of component 1 sitting
    on the bottom wall: circle through the apex and the chord h lattice units
    above the half-way wall plane, interface at rho1 = rho2 by linear
    interpolation (Sec. 3.3)."""
    d = r[0] - r[1]
    ny, nx = d.shape
    prof = (d > 0).sum(axis=0)
    xc = int(round((prof * np.arange(nx)).sum() / prof.sum()))
    c = d[:, xc]
    H = None
    for y in range(1, ny - 1):
        if c[y] > 0 >= c[y + 1]:
            H = y + c[y] / (c[y] - c[y + 1])
            break
    yh = ywall + h
    y0 = int(np.floor(yh))
    t = yh - y0
    row = (1 - t) * d[y0] + t * d[y0 + 1]
    xl = xr = None
    for x in range(xc, 0, -1):
        if row[x] > 0 >= row[x - 1]:
            xl = x - row[x] / (row[x] - row[x - 1])
            break
    for x in range(xc, nx - 1):
        if row[x] > 0 >= row[x + 1]:
            xr = x + row[x] / (row[x] - row[x + 1])
            break
    a = 0.5 * (xr - xl)
    yc = (H ** 2 - yh ** 2 - a ** 2) / (2 * (H - yh))
    R = H - yc
    theta_drop = np.degrees(np.arccos(np.clip((ywall - yc) / R, -1, 1)))
    return 180.0 - theta_drop
