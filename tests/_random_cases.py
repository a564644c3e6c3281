"""Seeded random small problems for the randomized parity sweep: lattice
size, discs (some rotating) and a flat wall with arbitrary fractions, rule
and mass fix, EOS with a droplet, BGK or MRT, body force.  Case k draws
everything from numpy's PCG64 seeded with 1000 + k."""
import numpy as np

from lbm_inputs import configs as cfg
from lbm_inputs import geometry as geo
from lbm_inputs.problem import RULES, Problem

MOVING = ("halfway", "fh", "mls")  # the rules that take a wall velocity
# (and not with Bao's fix, which has no moving-wall form)


def _discs(rng, nx, ny, band_rows, n):
    """n non-overlapping discs clear of each other and of the flat wall."""
    out = []
    for _ in range(200):
        if len(out) == n:
            break
        R = rng.uniform(3.0, max(3.5, min(nx, ny) / 5.0))
        cx = rng.uniform(R + 3.0, nx - R - 4.0)
        cy = rng.uniform(band_rows + R + 4.0, ny - R - 5.0)
        if any(np.hypot(cx - c.cx, cy - c.cy) < R + c.R + 4.0 for c in out):
            continue
        out.append(geo.Circle(cx, cy, R))
    return out


def random_case(k):
    rng = np.random.default_rng(1000 + k)
    nx, ny = int(rng.integers(32, 97)), int(rng.integers(40, 97))
    rule = str(rng.choice(RULES))
    fixes = ["none", "A"] + (["B", "bao"] if rule in ("fh", "mls") else [])
    fix = str(rng.choice(fixes))
    eos = str(rng.choice(["none", "exp", "cs"]))
    collision = str(rng.choice(["bgk", "mrt"]))
    # two-phase cases below tau = 0.8 mostly break down within a few dozen
    # steps at a density ratio near 11
    tau = float(rng.uniform(0.6 if eos == "none" else 0.8, 1.3))
    if rule == "fh" and abs(tau - 1.0) < 0.1:
        tau = 0.8  # Eq. 9 is singular at tau = 1
    band_rows = int(rng.integers(0, 4))
    shapes = []
    if band_rows:
        shapes.append(geo.Band(0, band_rows, q_top=rng.uniform(0.05, 1.0),
                               q_bottom=rng.uniform(0.05, 1.0)))
    discs = _discs(rng, nx, ny, band_rows, int(rng.integers(1, 3)))
    if rule in MOVING and fix != "bao" and rng.random() < 0.5:
        d = discs[0]
        discs[0] = geo.Circle(d.cx, d.cy, d.R, omega=rng.uniform(-1e-3, 1e-3))
    shapes += discs
    solid, owner, links = geo.build(nx, ny, shapes)
    g = tuple(float(v) for v in rng.uniform(-1e-5, 1e-5, 2) * (rng.random() < 0.5))
    kw = dict(eos=eos, collision=collision, tau=tau, mrt_s=cfg.mrt_rates(tau), rule=rule,
              fix=fix, gravity=g)
    if eos == "none":
        rho0 = 1.0 + 0.02 * rng.random((ny, nx))
        rw = 1.0
    else:
        if eos == "exp":
            rho_l, rho_v = cfg.EXP_INIT
            kw.update(eos_params=(1.0, 1.0, 0.0, 0.0), G=-10.0 / 3.0)
        else:
            rho_l, rho_v = cfg.cs_init_densities(0.86)
            kw.update(eos_params=cfg.cs_params(0.86), G=-1.0)
        # a droplet on the first disc's top point
        d = discs[0]
        rho0 = geo.tanh_disc(nx, ny, d.cx, d.cy + d.R, rng.uniform(0.8, 1.3) * d.R,
                             rho_l, rho_v, 4.0)
        rw = float(rng.uniform(rho_v + 0.2 * (rho_l - rho_v), rho_l - 0.2 * (rho_l - rho_v)))
    rho_wall = np.full((ny, nx), rw)
    rho0 = np.where(solid.astype(bool), rw, rho0)
    tile_w = int(rng.choice([64, 128, 256]))
    tile_h = int(rng.integers(1, 21))
    p = Problem(nx=nx, ny=ny, solid=solid, links=links, rho0=rho0, rho_wall=rho_wall,
                name=f"random{k}", **kw)
    return p, tile_w, tile_h


def random_open_case(k):
    """Flow past one or two discs between a velocity inlet (x = 0) and a
    fully developed outlet, periodic in y, single phase: lattice size,
    discs (clear of the three columns next to either end), inlet speed,
    rule and fix, BGK or MRT, tau.  Seeded with 2000 + k."""
    rng = np.random.default_rng(2000 + k)
    nx, ny = int(rng.integers(40, 121)), int(rng.integers(32, 97))
    rule = str(rng.choice(RULES))
    fixes = ["none", "A"] + (["B", "bao"] if rule in ("fh", "mls") else [])
    fix = str(rng.choice(fixes))
    collision = str(rng.choice(["bgk", "mrt"]))
    tau = float(rng.uniform(0.55, 1.2))
    if rule == "fh" and abs(tau - 1.0) < 0.1:
        tau = 0.8  # Eq. 9 is singular at tau = 1
    U = float(rng.uniform(0.01, 0.1))
    discs, n = [], int(rng.integers(1, 3))
    for _ in range(200):
        if len(discs) == n:
            break
        R = rng.uniform(3.0, max(3.5, min(nx, ny) / 6.0))
        cx = rng.uniform(R + 6.0, nx - R - 7.0)
        cy = rng.uniform(R + 2.0, ny - R - 3.0)
        if any(np.hypot(cx - c.cx, cy - c.cy) < R + c.R + 4.0 for c in discs):
            continue
        discs.append(geo.Circle(cx, cy, R))
    solid, owner, links = geo.build(nx, ny, discs)
    fl = ~solid.astype(bool)
    tile_w = int(rng.choice([64, 128, 256]))
    tile_h = int(rng.integers(1, 21))
    p = Problem(nx=nx, ny=ny, solid=solid, links=links,
                rho0=1.0 + 0.01 * rng.random((ny, nx)), rho_wall=np.ones((ny, nx)),
                eos="none", collision=collision, tau=tau, mrt_s=cfg.mrt_rates(tau),
                rule=rule, fix=fix, ux0=np.where(fl, U, 0.0), uy0=np.zeros((ny, nx)),
                open_x=True, inlet_u=U, name=f"random_open{k}")
    return p, tile_w, tile_h
