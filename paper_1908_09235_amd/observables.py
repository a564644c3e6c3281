"""Observables read from the fields the library returns: the steady flow
past a cylinder of Sec. 4.2 (Table 1) and the contact angle a virtual wall
density sets (Sec. 3.2).  Plain numpy post-processing of moments and wall
forces; nothing here is part of the time step.

Flow past a cylinder:

  wake length  2L/D, with L from the rearmost point of the cylinder to the
               end of the recirculation on the wake axis (where u_x turns
               from negative to positive, linear between nodes);
  separation   theta_s, the angle from the rear stagnation point at which
               the tangential velocity next to the wall changes sign.  It is
               read on circles of radius R + delta (bilinear interpolation,
               solid nodes at rest) and extrapolated linearly to delta = 0;
  drag         C_d = F_x / (0.5 rho U0^2 D) with rho = 1.

Contact angle:

  The interface is the level set rho = (rho_l + rho_v) / 2, located by linear
  interpolation on every lattice edge it crosses between two fluid nodes.  A
  circle is fitted to the interface points at least `cut` above the wall (the
  layer next to a wall with a virtual density is not part of the cap) by
  algebraic least squares, and the angle through the liquid follows from
  where the circle meets the wall line: cos(theta) = -(y_c - y_w) / R.  A
  circle that does not reach the wall (a detached droplet) gives 180 degrees,
  one whose centre lies more than R below it gives 0.
"""
import math

import numpy as np


def drag_coefficient(fx, u0, d, rho=1.0):
    return fx / (0.5 * rho * u0 * u0 * d)


def wake_length(ux, cx, cy, r):
    """2L/D from the row through the cylinder's centre (cy on a node row)."""
    row = ux[int(round(cy))]
    x0 = cx + r
    i = int(np.floor(x0)) + 1
    if row[i] >= 0:
        return 0.0
    while i < len(row) and row[i] < 0:
        i += 1
    if i == len(row):
        return float("inf")
    a, b = row[i - 1], row[i]
    xr = (i - 1) + a / (a - b)
    return 2.0 * (xr - x0) / (2.0 * r)


def _bilinear(f, x, y):
    x0 = np.floor(x).astype(int)
    y0 = np.floor(y).astype(int)
    tx, ty = x - x0, y - y0
    return ((1 - tx) * (1 - ty) * f[y0, x0] + tx * (1 - ty) * f[y0, x0 + 1] +
            (1 - tx) * ty * f[y0 + 1, x0] + tx * ty * f[y0 + 1, x0 + 1])


def separation_angle(ux, uy, solid, cx, cy, r, deltas=(1.0, 1.5, 2.0, 2.5, 3.0)):
    """theta_s in degrees (upper and lower halves averaged): where the wall
    shear changes sign.  At each angle phi from the rear stagnation point
    the tangential velocity u_t on circles of radius r + delta (bilinear,
    solid nodes at rest) is fitted by u_t = a delta + b delta^2, which
    vanishes at the wall; the separation point is where a(phi) turns
    negative (reverse flow along the wall), linear between samples."""
    fl = ~solid.astype(bool)
    u = np.where(fl, ux, 0.0)
    v = np.where(fl, uy, 0.0)
    phi = np.radians(np.linspace(1.0, 120.0, 11901))
    dl = np.asarray(deltas, dtype=np.float64)
    basis = np.c_[dl, dl * dl]
    out = []
    for sgn in (1.0, -1.0):
        ut = []
        for d in dl:
            x = cx + (r + d) * np.cos(phi)
            y = cy + sgn * (r + d) * np.sin(phi)
            # the lower half is the mirror image: v changes sign
            ut.append(-_bilinear(u, x, y) * np.sin(phi) + sgn * _bilinear(v, x, y) * np.cos(phi))
        a = np.linalg.lstsq(basis, np.array(ut), rcond=None)[0][0]
        k = int(np.argmax(a < 0))
        if k == 0:
            out.append(0.0)
            continue
        t = a[k - 1] / (a[k - 1] - a[k])
        out.append(np.degrees(phi[k - 1] + t * (phi[k] - phi[k - 1])))
    return 0.5 * (out[0] + out[1])


def interface_points(rho, solid, level):
    fl = ~solid.astype(bool)
    d = rho - level
    pts = []
    # horizontal edges (x, y) - (x + 1, y); the domain is periodic in x
    dr = np.roll(d, -1, axis=1)
    ok = fl & np.roll(fl, -1, axis=1) & (d * dr < 0)
    ys, xs = np.nonzero(ok)
    t = d[ys, xs] / (d[ys, xs] - dr[ys, xs])
    pts.append(np.c_[xs + t, ys])
    du = np.roll(d, -1, axis=0)
    ok = fl & np.roll(fl, -1, axis=0) & (d * du < 0)
    ok[-1, :] = False  # no edge across the y wrap
    ys, xs = np.nonzero(ok)
    t = d[ys, xs] / (d[ys, xs] - du[ys, xs])
    pts.append(np.c_[xs, ys + t])
    return np.concatenate(pts)


def fit_circle(x, y):
    A = np.c_[2 * x, 2 * y, np.ones_like(x)]
    c, *_ = np.linalg.lstsq(A, x * x + y * y, rcond=None)
    xc, yc = c[0], c[1]
    return xc, yc, math.sqrt(c[2] + xc * xc + yc * yc)


def contact_angle(rho, solid, wall_y, level, cut=3.0, y_max=None):
    """(theta in degrees, circle radius, centre height above the wall).
    y_max bounds the points kept from above (a wall with a large virtual
    density carries a dense film, also on the ceiling)."""
    P = interface_points(rho, solid, level)
    keep = P[:, 1] >= wall_y + cut
    if y_max is not None:
        keep &= P[:, 1] <= y_max
    P = P[keep]
    xc, yc, R = fit_circle(P[:, 0], P[:, 1])
    c = -(yc - wall_y) / R
    return math.degrees(math.acos(min(1.0, max(-1.0, c)))), R, yc - wall_y
