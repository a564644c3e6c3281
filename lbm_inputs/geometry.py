"""Geometry: solid masks and cut links with exact wall fractions.

A cut link joins a fluid node x_b to a solid neighbour x_s = x_b + e_a; its
wall fraction is q = |x_b - x_w| / |x_b - x_s| (Eq. 6), where x_w is the point
where the wall crosses the link.  For circles q is the exact root of
|x_b + q e_a - c| = R, taken in FP64 with the cancellation-free form of the
quadratic formula.  Solid nodes are those with |x - c|^2 <= R^2 (so q = 1 can
occur, and 0 < q <= 1 always).  The domain is periodic in x and y.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np

from .problem import LINK_DTYPE

# D2Q9 lattice directions (geometry only: which neighbour a link points to)
EX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
EY = (0, 0, 1, 0, -1, 1, 1, -1, -1)


class Circle:
    """Solid disc |x - c| <= R; may rotate about c at angular speed omega."""

    def __init__(self, cx: float, cy: float, R: float, omega: float = 0.0):
        self.cx, self.cy, self.R, self.omega = float(cx), float(cy), float(R), float(omega)

    def contains(self, X, Y):
        return (X - self.cx) ** 2 + (Y - self.cy) ** 2 <= self.R ** 2

    def bbox(self):
        """Row and column ranges that hold every solid node of the disc."""
        return (int(math.floor(self.cy - self.R)) - 1, int(math.ceil(self.cy + self.R)) + 2,
                int(math.floor(self.cx - self.R)) - 1, int(math.ceil(self.cx + self.R)) + 2)

    def fraction(self, xb, yb, ex, ey):
        dx, dy = xb - self.cx, yb - self.cy
        a = ex * ex + ey * ey
        b = dx * ex + dy * ey                       # < 0: moving inwards
        c = dx * dx + dy * dy - self.R ** 2          # > 0: x_b outside
        disc = np.maximum(b * b - a * c, 0.0)
        q = c / (-b + np.sqrt(disc))                # smaller root, stable
        return np.minimum(q, 1.0)

    def wall_velocity(self, xw, yw):
        return -self.omega * (yw - self.cy), self.omega * (xw - self.cx)

    def fits(self, nx, ny):
        return (self.cx - self.R > 1 and self.cx + self.R < nx - 2 and
                self.cy - self.R > 1 and self.cy + self.R < ny - 2)


class OuterCircle:
    """Solid outside a circle: |x - c| >= R (the fixed outer Couette wall)."""

    def __init__(self, cx: float, cy: float, R: float):
        self.cx, self.cy, self.R = float(cx), float(cy), float(R)

    def contains(self, X, Y):
        return (X - self.cx) ** 2 + (Y - self.cy) ** 2 >= self.R ** 2

    def fraction(self, xb, yb, ex, ey):
        dx, dy = xb - self.cx, yb - self.cy
        a = ex * ex + ey * ey
        b = dx * ex + dy * ey
        c = dx * dx + dy * dy - self.R ** 2          # < 0: x_b inside
        sq = np.sqrt(np.maximum(b * b - a * c, 0.0))
        q = np.where(b >= 0.0, -c / np.where(b + sq > 0, b + sq, 1.0),
                     (-b + sq) / a)
        return np.minimum(q, 1.0)

    def wall_velocity(self, xw, yw):
        return np.zeros_like(xw), np.zeros_like(yw)

    def fits(self, nx, ny):
        return True


class Band:
    """Solid rows y0 <= y < y1 across the whole width (a flat wall).

    Links entering from above get wall fraction q_top, links entering from
    below (through the periodic y wrap if y0 == 0) get q_bottom.  With the
    wall half-way between the last solid and first fluid row, q = 1/2.
    """

    def __init__(self, y0: int, y1: int, q_top: float = 0.5,
                 q_bottom: float = 0.5):
        self.y0, self.y1 = int(y0), int(y1)
        self.q_top, self.q_bottom = float(q_top), float(q_bottom)

    def contains(self, X, Y):
        return (Y >= self.y0) & (Y < self.y1)

    def fraction(self, xb, yb, ex, ey):
        return np.where(np.asarray(ey) < 0, self.q_top, self.q_bottom) + 0.0 * xb

    def wall_velocity(self, xw, yw):
        return np.zeros_like(xw), np.zeros_like(yw)

    def fits(self, nx, ny):
        return 0 <= self.y0 < self.y1 <= ny


class SlopedBand:
    """Solid band between two parallel straight walls of slope 1/2 in a
    periodic nx = 2n by ny = n lattice: a node is solid where
    s = y - x/2, taken modulo n into [s0, s0 + n), lies in [s0, s1).  The
    walls are the lines s = s0 (+ n) and s = s1; since s changes by
    e_y - e_x/2 along a link, the fraction of a cut link is linear in s.
    The walls are not lattice-aligned, so the fractions vary along them
    (with the same pattern at every n when s0 and s1 keep their
    fractional parts)."""

    def __init__(self, n: int, s0: float, s1: float):
        self.n, self.s0, self.s1 = int(n), float(s0), float(s1)

    def coordinate(self, X, Y):
        return np.mod(Y - 0.5 * X - self.s0, self.n) + self.s0

    def contains(self, X, Y):
        s = self.coordinate(X, Y)
        return (s >= self.s0) & (s < self.s1)

    def fraction(self, xb, yb, ex, ey):
        s = self.coordinate(xb, yb)          # in [s1, s0 + n) on fluid nodes
        ds = ey - 0.5 * ex
        q = np.where(ds > 0, (self.s0 + self.n - s) / np.where(ds > 0, ds, 1.0),
                     (self.s1 - s) / np.where(ds < 0, ds, -1.0))
        return np.minimum(q, 1.0)

    def wall_velocity(self, xw, yw):
        return np.zeros_like(xw), np.zeros_like(yw)

    def fits(self, nx, ny):
        return nx == 2 * self.n and ny == self.n


def build(nx: int, ny: int, shapes: Sequence):
    """Solid mask (uint8 [ny, nx]), owner index per node, and the cut links.

    Links are sorted by (y, x, dir).  Shapes must not overlap.
    """
    Y, X = np.mgrid[0:ny, 0:nx]
    owner = np.full((ny, nx), -1, dtype=np.int32)
    for k, sh in enumerate(shapes):
        assert sh.fits(nx, ny), f"shape {k} does not fit the {nx}x{ny} domain"
        if hasattr(sh, "bbox"):   # a shape that fits lies inside its box
            y0, y1, x0, x1 = sh.bbox()
            y0, y1, x0, x1 = max(y0, 0), min(y1, ny), max(x0, 0), min(x1, nx)
            m = sh.contains(X[y0:y1, x0:x1], Y[y0:y1, x0:x1])
            sub = owner[y0:y1, x0:x1]
            assert not np.any(sub[m] >= 0), "overlapping shapes"
            sub[m] = k
            continue
        m = sh.contains(X, Y)
        assert not np.any(owner[m] >= 0), "overlapping shapes"
        owner[m] = k
    solid = owner >= 0
    parts = []
    for a in range(1, 9):
        ys = (Y + EY[a]) % ny
        xs = (X + EX[a]) % nx
        cut = (~solid) & solid[ys, xs]
        if not cut.any():
            continue
        yb, xb = np.nonzero(cut)
        own = owner[ys[cut], xs[cut]]
        for k in np.unique(own):
            sel = own == k
            xk = xb[sel].astype(np.float64)
            yk = yb[sel].astype(np.float64)
            q = shapes[k].fraction(xk, yk, float(EX[a]), float(EY[a]))
            q = np.asarray(q, dtype=np.float64) * np.ones_like(xk)
            uwx, uwy = shapes[k].wall_velocity(xk + q * EX[a], yk + q * EY[a])
            rec = np.zeros(sel.sum(), dtype=LINK_DTYPE)
            rec["x"], rec["y"], rec["dir"] = xb[sel], yb[sel], a
            rec["q"] = q
            rec["uwx"] = np.asarray(uwx, dtype=np.float64) * np.ones_like(xk)
            rec["uwy"] = np.asarray(uwy, dtype=np.float64) * np.ones_like(xk)
            parts.append(rec)
    links = np.concatenate(parts) if parts else np.zeros(0, dtype=LINK_DTYPE)
    order = np.lexsort((links["dir"], links["x"], links["y"]))
    return solid.astype(np.uint8), owner, links[order]


def tanh_disc(nx: int, ny: int, cx: float, cy: float, R: float,
              rho_in: float, rho_out: float, width: float) -> np.ndarray:
    """rho = (in+out)/2 + (in-out)/2 * tanh(2 (R - r)/width), periodic r."""
    Y, X = np.mgrid[0:ny, 0:nx].astype(np.float64)
    dx = X - cx
    dy = Y - cy
    dx = dx - nx * np.round(dx / nx)
    dy = dy - ny * np.round(dy / ny)
    r = np.sqrt(dx * dx + dy * dy)
    return 0.5 * (rho_in + rho_out) + 0.5 * (rho_in - rho_out) * np.tanh(
        2.0 * (R - r) / width)


def tanh_slab(nx: int, ny: int, y0: float, y1: float, rho_in: float,
              rho_out: float, width: float) -> np.ndarray:
    """A liquid slab y0 < y < y1 with two flat tanh interfaces."""
    y = np.arange(ny, dtype=np.float64)
    prof = 0.5 * (rho_in + rho_out) + 0.5 * (rho_in - rho_out) * (
        np.tanh(2.0 * (y - y0) / width) - np.tanh(2.0 * (y - y1) / width) - 1.0)
    return np.repeat(prof[:, None], nx, axis=1)


def no_overlap(circles, clearance: float) -> bool:
    for i in range(len(circles)):
        for j in range(i + 1, len(circles)):
            (x1, y1, r1), (x2, y2, r2) = circles[i], circles[j]
            if math.hypot(x1 - x2, y1 - y2) < r1 + r2 + clearance:
                return False
    return True
