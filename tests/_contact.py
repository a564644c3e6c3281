"""Contact angle of a droplet on a flat wall, read from the density field.

The interface is the level set rho = (rho_l + rho_v) / 2, located by linear
interpolation on every lattice edge it crosses between two fluid nodes.  A
circle is fitted to the interface points at least `cut` above the wall (the
layer next to a wall with a virtual density is not part of the cap) by
algebraic least squares, and the angle through the liquid follows from
where the circle meets the wall line: cos(theta) = -(y_c - y_w) / R.  A
circle that does not reach the wall (a detached droplet) gives 180 degrees,
one whose centre lies more than R below it gives 0."""
import math

import numpy as np


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
