"""Pins of the oracle's flow-past-a-cylinder parts (Sec. 4.2): the Zou-He
velocity inlet, the fully developed outlet and the momentum-exchange force
on the walls.  Each is checked against a property fixed by the mathematics,
not against its own formula: the inlet node's moments come out as the
prescribed velocity, a uniform stream is an exact fixed point, and the wall
force closes the momentum balance of every step."""
import numpy as np
import pytest

from lbm_inputs import configs as cfg
from lbm_inputs import geometry as geo
from lbm_inputs.problem import Problem
from oracle import core as ora


def _small_cylinder(fix="A", re=20.0, rule="mls"):
    # 48 x 32 nodes, D = 8 at (18, 16)
    return cfg.cylinder_flow(re, fix=fix, d=8.0, nx_d=6.0, ny_d=4.0, rule=rule)


def test_uniform_stream_is_a_fixed_point():
    """No obstacle: f = f_eq(1, (U, 0)) everywhere passes through the
    inlet, the bulk and the outlet unchanged."""
    U = 0.08
    nx, ny = 24, 10
    solid = np.zeros((ny, nx), np.uint8)
    p = Problem(nx=nx, ny=ny, solid=solid, links=np.zeros(0, geo.LINK_DTYPE),
                rho0=np.ones((ny, nx)), rho_wall=np.ones((ny, nx)), tau=0.7,
                ux0=np.full((ny, nx), U), uy0=np.zeros((ny, nx)), open_x=True,
                inlet_u=U)
    o = ora.Oracle(p)
    o.step(300)
    r, ux, uy = o.moments()
    assert np.abs(r - 1).max() < 1e-13
    assert np.abs(ux - U).max() < 1e-14 and np.abs(uy).max() < 1e-14


def test_inlet_node_carries_the_prescribed_velocity():
    """Zou and He choose the three unknown populations so that the node's
    own moments give u = (U, 0); from any state of the interior."""
    p = _small_cylinder()
    rs = np.random.default_rng(3)
    fl = ~p.solid.astype(bool)
    p = p.with_(rho0=np.where(fl, 1 + 0.02 * rs.standard_normal(p.solid.shape), 1.0),
                uy0=np.where(fl, 0.02 * rs.standard_normal(p.solid.shape), 0.0))
    o = ora.Oracle(p)
    U = p.inlet_u
    for n in (1, 7, 40):
        o.step(n)
        r, ux, uy = o.moments()
        assert np.abs(ux[:, 0] - U).max() < 1e-14
        assert np.abs(uy[:, 0]).max() < 1e-15
        # nothing else is forced to U
        assert np.abs(ux[:, 1] - U).max() > 1e-6


def test_outlet_takes_incoming_populations_from_its_neighbour():
    p = _small_cylinder()
    o = ora.Oracle(p)
    o.step(25)
    f = o.get_f()
    for a in (3, 6, 7):  # the populations that enter from x = nx
        assert np.array_equal(f[a, :, -1], f[a, :, -2])
    for a in (1, 5, 8, 0, 2, 4):  # the others stream as in the bulk
        assert not np.array_equal(f[a, :, -1], f[a, :, -2])


def _periodic_cylinder(rule, fix, gx=2e-5):
    nx, ny, R = 40, 36, 9.3
    solid, owner, links = geo.build(nx, ny, [geo.Circle(19.6, 17.2, R)])
    fl = ~solid.astype(bool)
    rs = np.random.default_rng(11)
    return Problem(nx=nx, ny=ny, solid=solid, links=links,
                   rho0=np.where(fl, 1 + 0.01 * rs.standard_normal((ny, nx)), 1.0),
                   rho_wall=np.ones((ny, nx)), tau=0.8, rule=rule, fix=fix,
                   gravity=(gx, 0.0),
                   ux0=np.where(fl, 0.01 * rs.standard_normal((ny, nx)), 0.0),
                   uy0=np.where(fl, 0.01 * rs.standard_normal((ny, nx)), 0.0))


@pytest.mark.parametrize("rule,fix", [("halfway", "none"), ("mls", "none"), ("mls", "A"),
                                      ("mls", "B"), ("ibb_quadratic", "none"),
                                      ("zhao_yong", "none"), ("fh", "bao")])
def test_wall_force_closes_the_momentum_balance(rule, fix):
    """Collision with Guo forcing adds exactly F = rho g per node and step;
    streaming between fluid nodes moves momentum without changing it; what a
    cut link takes out (f*_a toward the wall) and puts back (the incoming
    f_abar) is the momentum handed to the wall.  With Sum e f = Sum rho u -
    g M / 2 (Eq. 5), every step satisfies
        Sum rho u(t+1) - g M(t+1)/2 = Sum rho u(t) - g M(t)/2 + g M(t) - F_w(t)."""
    p = _periodic_cylinder(rule, fix)
    gx = p.gravity[0]
    o = ora.Oracle(p)
    fl = ~p.solid.astype(bool)

    def state():
        r, ux, uy = o.moments()
        m = r[fl].sum()
        return m, (r * ux)[fl].sum() - 0.5 * gx * m, (r * uy)[fl].sum()

    m, px, py = state()
    for k in range(12):
        o.step(1 + 5 * (k % 3))
        if k % 3:  # the force is that of the last step only
            m, px, py = state()
            continue
        F = o.wall_force()
        m1, px1, py1 = state()
        assert abs(px1 - (px + gx * m - F[0])) < 1e-12 * max(1.0, abs(F[0]))
        assert abs(py1 - (py - F[1])) < 1e-12 * max(1.0, abs(F[1]))
        assert abs(F[0]) > 1e-4  # the balance is not trivially met
        m, px, py = m1, px1, py1


def test_wall_force_is_zero_before_the_first_step():
    o = ora.Oracle(_small_cylinder())
    assert np.array_equal(o.wall_force(), [0.0, 0.0])


def test_drag_points_downstream_and_lift_vanishes_on_the_axis():
    """Symmetric about the channel axis: F_y of the symmetric state stays
    at rounding level while F_x grows positive."""
    p = _small_cylinder()
    o = ora.Oracle(p)
    o.step(200)
    F = o.wall_force()
    assert F[0] > 0 and abs(F[1]) < 1e-10 * F[0]


def _with_post(p, x):
    """p with one more solid node at (x, 5), a post of radius 0.5 with its
    own cut links."""
    m = p.meta
    solid, _, links = geo.build(p.nx, p.ny, [geo.Circle(m["cx"], m["cy"], 0.5 * m["d"]),
                                             geo.Circle(float(x), 5.0, 0.5)])
    assert solid[5, x] == 1 and solid.sum() == p.solid.sum() + 1
    return p.with_(solid=solid, links=links)


def test_open_x_accepts_a_wall_three_columns_from_the_outlet():
    p = _with_post(_small_cylinder(), 44)
    o = ora.Oracle(p)
    o.step(3)


@pytest.mark.parametrize("bad", ["eos", "speed", "solid_edge", "narrow"])
def test_open_x_rejects_what_it_does_not_support(bad):
    p = _small_cylinder()
    if bad == "eos":
        p = p.with_(eos="cs", eos_params=(1.0, 4.0, 1.0, 0.08), G=-1.0)
    elif bad == "speed":
        p = p.with_(inlet_u=1.0)
    elif bad == "solid_edge":
        p = _with_post(p, p.nx - 3)
    else:
        s = np.zeros((8, 7), np.uint8)
        p = Problem(nx=7, ny=8, solid=s, links=np.zeros(0, geo.LINK_DTYPE),
                    rho0=np.ones((8, 7)), rho_wall=np.ones((8, 7)), open_x=True,
                    inlet_u=0.05)
    with pytest.raises(ora.OracleError):
        ora.Oracle(p)
