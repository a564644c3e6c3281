"""Readers of the flow past a cylinder, pinned on synthetic fields whose
answers are known by construction."""
import math

import numpy as np
import pytest

from paper_1908_09235_amd import observables as obs


def _separated_field(phi_up, phi_lo, r=20.0, n=160):
    """Velocity around a cylinder of radius r at the centre of an n x n
    grid.  Its tangential component, along increasing angle phi from the
    rear stagnation point (each half measured on its own side of the wake
    axis), is u_t = (phi0 - phi) delta (1 - delta / 20): zero on the wall,
    with a wall shear that changes sign at phi0 (phi_up above the axis,
    phi_lo below)."""
    c = (n - 1) / 2.0
    Y, X = np.mgrid[0:n, 0:n].astype(np.float64)
    dx, dy = X - c, Y - c
    rad = np.hypot(dx, dy)
    phi = np.arctan2(np.abs(dy), dx)
    sgn = np.where(dy >= 0, 1.0, -1.0)
    phi0 = np.radians(np.where(dy >= 0, phi_up, phi_lo))
    delta = rad - r
    ut = (phi0 - phi) * delta * (1.0 - delta / 20.0)
    ux = -ut * np.sin(phi)
    uy = ut * np.cos(phi) * sgn
    solid = (rad <= r).astype(np.uint8)
    return np.where(solid, 0.0, ux), np.where(solid, 0.0, uy), solid, c, r


# bilinear sampling of a field curved on the grid scale costs a few
# hundredths of a degree here; the readings it serves are compared at 2 degrees
TOL = 0.1


@pytest.mark.parametrize("phi0", [35.0, 41.4, 53.9, 70.0])
def test_separation_angle_is_the_sign_change_of_the_wall_shear(phi0):
    ux, uy, solid, c, r = _separated_field(phi0, phi0)
    got = obs.separation_angle(ux, uy, solid, c, c, r)
    assert abs(got - phi0) < TOL, (got, phi0)


def test_separation_angle_averages_the_two_halves():
    ux, uy, solid, c, r = _separated_field(40.0, 50.0)
    got = obs.separation_angle(ux, uy, solid, c, c, r)
    assert abs(got - 45.0) < TOL, got


def test_attached_flow_has_no_separation():
    # u_t positive everywhere on [1, 120] degrees: no sign change
    ux, uy, solid, c, r = _separated_field(150.0, 150.0)
    assert obs.separation_angle(ux, uy, solid, c, c, r) == 0.0
