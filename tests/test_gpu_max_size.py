"""The largest domain each storage form accepts: a state buffer just below
4 GiB, addressed by the kernels with 32-bit byte offsets.  A droplet on a
cylinder sits in the domain's last rows and columns (the highest offsets)
inside vapour at rest; after a few steps the window around it must equal,
bit for bit, the same case run as a small domain of the window's size:
vapour at rest evolves alike in both, the disturbance has not reached the
window's edge, and the fields do not depend on the launch shape."""
import sys

import numpy as np
import pytest

from lbm_inputs import configs as cfg
from tests._limits import buffer_bytes, max_rows, LIMIT

pytestmark = pytest.mark.gpu

NX = 16384
WIN = 256
# the state at x depends on nodes up to two away per step (psi of the
# neighbours' new densities): the initial disturbance (radius 63 about the
# droplet centre, where the tanh profile differs from the vapour) grows to
# 103, inside the window's half width of 128
STEPS = 20


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    from paper_1908_09235_amd import lbm
    lbm.lib()
    return lbm


def _small():
    # no floor: the window has vapour on every side; the droplet's tanh
    # profile is exactly the vapour density at the window's edges
    return cfg.droplet_on_cylinder(side_x=WIN, side_y=WIN, floor=0,
                                   centre=(128.0, 100.0), rc=20.0, rd=25.0,
                                   tau=0.8, rule="mls", fix="B", name="win256")


def _embed(s, nx, ny):
    """The small problem placed in the last WIN rows and columns of an
    nx x ny domain filled with its edge vapour."""
    x0, y0 = nx - WIN, ny - WIN
    vap = s.rho0[0, 0]
    assert np.all(s.rho0[0, :] == vap) and np.all(s.rho0[:, 0] == vap)
    solid = np.zeros((ny, nx), np.uint8)
    solid[y0:, x0:] = s.solid
    rho0 = np.full((ny, nx), vap)
    rho0[y0:, x0:] = s.rho0
    rw = np.full((ny, nx), s.rho_wall[0, 0])
    links = s.links.copy()
    links["x"] += x0
    links["y"] += y0
    return s.with_(nx=nx, ny=ny, solid=solid, rho0=rho0, rho_wall=rw, links=links,
                   name=f"max_{nx}x{ny}")


@pytest.mark.parametrize("storage", ["f64", "f32", "f16node"])
def test_largest_domain_matches_small_window(L, storage):
    ny = max_rows(storage, NX)
    assert buffer_bytes(storage, NX, ny) < LIMIT <= buffer_bytes(storage, NX, ny + 1)
    s = _small()
    rho_ref = 0.1  # the deviation reference is fixed, not drawn from the domain
    say(f"[gpu] window {WIN}^2 {storage} {STEPS} steps")
    with L.Domain(s, storage=storage, rho_ref=rho_ref) as d:
        d.step(STEPS)
        ref = d.moments()
    big = _embed(s, NX, ny)
    say(f"[gpu] {NX} x {ny} {storage}: {buffer_bytes(storage, NX, ny)} B per state buffer")
    with L.Domain(big, storage=storage, rho_ref=rho_ref) as d:
        d.step(STEPS)
        got = d.moments()
    del big
    for i in range(3):
        w = got[i][ny - WIN:, NX - WIN:]
        assert np.array_equal(w, ref[i]), (storage, i, float(np.max(np.abs(w - ref[i]))))
    # the disturbance stayed inside the window: the rest is uniform vapour
    r = got[0]
    fl = r[:ny - WIN, :] != 0
    assert np.all(r[:ny - WIN, :][fl] == r[0, 0])
