"""Contact angle by a constant virtual wall density (Sec. 3.2): the reading
of the angle from a density field, and the oracle's wetting trend.

The paper gives no map between the virtual wall density and the angle, so
the angles themselves are parity unpinned; pinned are the reader (ideal
caps of known angle) and the direction of the mechanism (a denser virtual
wall wets more)."""
import math

import numpy as np
import pytest

from lbm_inputs import configs as cfg
from oracle import core as ora
from paper_1908_09235_amd import observables as ca


def _cap_field(theta_deg, R=30.0, nx=200, ny=100, floor=4, lo=0.02, hi=0.27, w=4.0):
    """Density of an ideal circular cap meeting the wall at theta."""
    yw = floor - 0.5
    yc = yw - R * math.cos(math.radians(theta_deg))
    Y, X = np.mgrid[0:ny, 0:nx].astype(float)
    r = np.hypot(X - nx / 2, Y - yc)
    rho = 0.5 * (hi + lo) - 0.5 * (hi - lo) * np.tanh(2 * (r - R) / w)
    solid = np.zeros((ny, nx), np.uint8)
    solid[:floor] = 1
    return rho, solid, yw, 0.5 * (hi + lo)


@pytest.mark.parametrize("theta", [35.0, 60.0, 90.0, 120.0, 150.0])
def test_reader_recovers_the_angle_of_an_ideal_cap(theta):
    rho, solid, yw, lvl = _cap_field(theta)
    got, R, h = ca.contact_angle(rho, solid, yw, lvl)
    assert abs(got - theta) < 0.3
    assert abs(R - 30.0) < 0.3


def test_reader_reports_a_detached_droplet_as_180():
    rho, solid, yw, lvl = _cap_field(90.0)
    rho = np.roll(rho, 40, axis=0)  # lift the disc off the wall
    rho[:4] = rho[4]
    got, _, h = ca.contact_angle(rho, solid, yw, lvl, y_max=95)
    assert got == 180.0 and h > 30


def test_denser_virtual_wall_wets_more():
    """Oracle, CS at 0.86 Tc, a small droplet on a flat floor: the angle
    falls as the virtual wall density rises through the vapour-liquid
    range."""
    th = {}
    for rw in (0.12, 0.18):
        p = cfg.sessile_droplet(rw, nx=120, ny=64, r0=18.0)
        o = ora.Oracle(p)
        o.step(1500)
        r, _, _ = o.moments()
        lvl = 0.5 * (p.meta["rho_l"] + p.meta["rho_v"])
        th[rw] = ca.contact_angle(r, p.solid, p.meta["wall_y"], lvl,
                                  y_max=p.ny - 0.5 - 3.0)[0]
    assert 60.0 < th[0.12] < 150.0 and th[0.18] < th[0.12] - 20.0, th
