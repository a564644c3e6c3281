"""HIP library vs the FP64 CPU oracle, element by element, on the same seeded
inputs.  Bar: FP64 storage within 1e-12 (max-norm relative, rho and u over
fluid nodes) after 1000 steps; FP32 storage within 1e-5; mass histories
within 1e-13 relative in FP64.  Full-size (2048^2) cases are checked through
properties that hold at any size.  Storage "f32" keeps FP32 populations with
FP64 arithmetic; "f32_arith32" computes in FP32 and has a stated bound."""
import os
import sys

import numpy as np
import pytest

from lbm_inputs import configs as cfg
from lbm_inputs import geometry as geo
from lbm_inputs.problem import Problem
from oracle import core as ora
from tests._lib import rel_err

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
F32_TOL = 1e-5
MASS_TOL = 1e-13


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    from paper_1908_09235_amd import lbm
    lbm.lib()  # raises if the library is missing
    return lbm


def gpu_run(L, p, steps, storage="f64", **kw):
    say(f"[gpu] {p.name} rule={p.rule} fix={p.fix} {storage} steps={steps} {kw}")
    with L.Domain(p, storage=storage, **kw) as d:
        d.step(steps)
        r, ux, uy = d.moments()
        hist = d.mass_history()
    return r, ux, uy, hist


_ORACLE = {}


def oracle_run(p, steps, key=None):
    key = key or (p.name, p.rule, p.fix, p.collision, p.tau, steps)
    if key not in _ORACLE:
        o = ora.Oracle(p)
        m0 = o.total_mass()
        h = o.step(steps)
        r, ux, uy = o.moments()
        _ORACLE[key] = (r, ux, uy, np.concatenate([[m0], h]))
    return _ORACLE[key]


def compare(p, g, o, tol, mass_tol=None):
    fl = ~p.solid.astype(bool)
    e = [rel_err(g[i], o[i], fl) for i in range(3)]
    say(f"    rel err rho {e[0]:.3e} ux {e[1]:.3e} uy {e[2]:.3e}")
    assert max(e) <= tol, e
    assert np.all(g[0][~fl] == 0)
    if mass_tol is not None:
        gh, oh = g[3], o[3]
        assert len(gh) == len(oh)
        dm = np.max(np.abs(gh - oh) / np.abs(oh))
        say(f"    mass history rel diff {dm:.3e}")
        assert dm <= mass_tol


CFG1_CASES = [("mls", "A"), ("mls", "B"), ("ibb_linear", "A"),
              ("ibb_quadratic", "A"), ("halfway", "none"), ("mls", "none"),
              ("ibb_linear", "none"), ("ibb_quadratic", "none"), ("mls", "bao")]


@pytest.mark.parametrize("rule,fix", CFG1_CASES)
def test_cfg1_fp64_1000_steps(L, rule, fix):
    """Droplet on a cylinder, 128^2, CS EOS at 0.86 Tc, BGK tau = 1."""
    p = cfg.cfg1(rule, fix)
    compare(p, gpu_run(L, p, 1000), oracle_run(p, 1000), F64_TOL, MASS_TOL)


@pytest.mark.parametrize("fix,steps", [("none", 25), ("A", 5)])
def test_cfg1_zhao_yong_before_breakdown(L, fix, steps):
    """Zhao-Yong drives this droplet unstable within a few steps (the oracle
    breaks at steps 31 and 7); compare over the stable window."""
    p = cfg.cfg1("zhao_yong", fix)
    compare(p, gpu_run(L, p, steps), oracle_run(p, steps), F64_TOL, MASS_TOL)


@pytest.mark.parametrize("rule,fix", [("mls", "A"), ("mls", "B"),
                                      ("ibb_quadratic", "A"), ("mls", "none")])
def test_cfg1_fp32_1000_steps(L, rule, fix):
    p = cfg.cfg1(rule, fix)
    g = gpu_run(L, p, 1000, storage="f32")
    compare(p, g, oracle_run(p, 1000), F32_TOL)
    m0 = g[3][0]
    say(f"    fp32 mass drift {(g[3][-1] - m0) / m0:.3e}")


@pytest.mark.parametrize("rule,fix", [("mls", "A"), ("mls", "B")])
def test_cfg1_fp32_arithmetic_error_is_stated(L, rule, fix):
    """FP32 storage with FP32 arithmetic: faster, with a larger error that
    is measured against the oracle and bounded here at 3e-5."""
    p = cfg.cfg1(rule, fix)
    g = gpu_run(L, p, 1000, storage="f32_arith32")
    compare(p, g, oracle_run(p, 1000), 3e-5)


def test_moments_at_time_zero(L):
    p = cfg.cfg1("mls", "B")
    o = ora.Oracle(p)
    r, ux, uy = o.moments()
    with L.Domain(p) as d:
        g = d.moments()
        m = d.total_mass()
    compare(p, (*g, None), (r, ux, uy, None), 1e-13)
    assert abs(m - o.total_mass()) / m < 1e-14


@pytest.mark.parametrize("rule,q", [("zhao_yong", 0.3), ("ibb_quadratic", 0.3),
                                    ("mls", 0.7), ("ibb_linear", 0.8)])
def test_static_gravity_parity(L, rule, q):
    """Sec. 3.1's single-phase test: flat walls with fraction q, gravity."""
    p = cfg.static_gravity(q, rule=rule)
    compare(p, gpu_run(L, p, 1000), oracle_run(p, 1000), F64_TOL, MASS_TOL)


@pytest.mark.parametrize("fix", ["none", "A", "B"])
def test_couette_moving_wall_parity(L, fix):
    p = cfg.couette(10, rule="mls", fix=fix)
    compare(p, gpu_run(L, p, 1000), oracle_run(p, 1000), F64_TOL, MASS_TOL)


def test_fh_couette_parity(L):
    p = cfg.couette(10, rule="fh", fix="A", tau=0.7)
    compare(p, gpu_run(L, p, 1000), oracle_run(p, 1000), F64_TOL, MASS_TOL)


def test_mrt_droplet_parity(L):
    """The 2048^2 MRT workload scaled down to 256^2 (MLS + B, tau = 0.8)."""
    p = cfg.cfg2a(scale=2.0)
    compare(p, gpu_run(L, p, 400), oracle_run(p, 400), F64_TOL, MASS_TOL)
    compare(p, gpu_run(L, p, 400, storage="f32"), oracle_run(p, 400), F32_TOL)


def test_exp_eos_free_droplet_parity(L):
    """psi = exp(-1/rho), G = -10/3 (Sec. 3.2); no walls.  In this flow the
    FP64 rounding differences between two evaluation orders grow by about
    2e-15 per step, so the 1e-12 bar is checked at 300 steps."""
    p = cfg.free_droplet(64, 14.0, eos="exp")
    compare(p, gpu_run(L, p, 300), oracle_run(p, 300), F64_TOL, MASS_TOL)


def _ragged_problem(nx=67, ny=53, rule="ibb_quadratic", fix="A"):
    shapes = [geo.Circle(20.3, 17.6, 8.4), geo.Circle(47.1, 33.2, 11.7)]
    solid, owner, links = geo.build(nx, ny, shapes)
    rho0 = geo.tanh_disc(nx, ny, 20.3, 17.6 + 8.4, 10.0, 0.269941, 0.024515, 4.0)
    rho0 = np.where(solid.astype(bool), 0.05, rho0)
    return Problem(nx=nx, ny=ny, solid=solid, links=links, rho0=rho0,
                   rho_wall=np.full((ny, nx), 0.05), eos="cs",
                   eos_params=cfg.cs_params(0.86), G=-1.0, tau=0.9,
                   mrt_s=cfg.mrt_rates(0.9), rule=rule, fix=fix, name="ragged")


@pytest.mark.parametrize("tw,th", [(64, 16), (128, 7), (256, 53), (64, 1)])
def test_ragged_tiles_parity(L, tw, th):
    """67 x 53: a 3-column strip tail and a short last segment."""
    p = _ragged_problem()
    compare(p, gpu_run(L, p, 300, tile_w=tw, tile_h=th), oracle_run(p, 300),
            F64_TOL, MASS_TOL)


@pytest.mark.parametrize("storage", ["f64", "f32", "f32_arith32", "f32dev", "f16dev", "f16node"])
def test_results_do_not_depend_on_tiling(L, storage):
    """rho and u are bit-identical for every launch shape (a row lands in
    a different unrolled copy of the row loop at each tile height)."""
    p = cfg.cfg1("mls", "B")
    ref = gpu_run(L, p, 200, storage=storage, tile_w=128, tile_h=16)
    for tw, th in [(64, 16), (64, 5), (128, 128), (256, 3), (64, 1)]:
        g = gpu_run(L, p, 200, storage=storage, tile_w=tw, tile_h=th)
        for i in range(3):
            assert np.array_equal(g[i], ref[i]), (tw, th, i)


# FP16 per-node storage against the oracle: (rho, u) bounds, as for the
# deviation forms
F16NODE_TOL = (1e-3, 1e-2)


def test_ragged_tiles_fp16_per_node(L):
    """The FP16 per-node form on the 67 x 53 case: the same fields at every
    ragged launch shape (strip tails of 3 columns, one-row segments), and
    within its bounds of the oracle."""
    p = _ragged_problem()
    runs = [gpu_run(L, p, 300, storage="f16node", tile_w=tw, tile_h=th)
            for tw, th in [(64, 16), (128, 7), (256, 53), (64, 1)]]
    for g in runs[1:]:
        for i in range(3):
            assert np.array_equal(g[i], runs[0][i])
    o = oracle_run(p, 300)
    fl = ~p.solid.astype(bool)
    e = [rel_err(runs[0][i], o[i], fl) for i in range(3)]
    say(f"    rel err rho {e[0]:.3e} ux {e[1]:.3e} uy {e[2]:.3e}")
    assert e[0] <= F16NODE_TOL[0] and max(e[1:]) <= F16NODE_TOL[1]


def test_tiny_domain_without_walls(L):
    """3 x 3, the smallest lattice: every neighbour wraps.  Compared at t = 2
    (the velocity falls by 100x per 4 steps and reaches round-off by t ~ 50,
    where a relative norm means nothing)."""
    rng = np.random.default_rng(3)
    n = 3
    rho0 = 0.1 + 0.02 * rng.random((n, n))
    p = cfg.free_droplet(n, 1.0).with_(rho0=rho0, name="tiny3")
    compare(p, gpu_run(L, p, 2), oracle_run(p, 2), F64_TOL, MASS_TOL)
    # FP16 per-node storage: every density the decode reads wraps too
    g = gpu_run(L, p, 2, storage="f16node")
    fl = ~p.solid.astype(bool)
    o = oracle_run(p, 2)
    e = [rel_err(g[i], o[i], fl) for i in range(3)]
    say(f"    f16node rel err rho {e[0]:.3e} ux {e[1]:.3e} uy {e[2]:.3e}")
    assert e[0] <= F16NODE_TOL[0] and max(e[1:]) <= F16NODE_TOL[1]


@pytest.mark.parametrize("storage,rule", [("f64", "mls"), ("f32", "mls"), ("f16node", "mls"),
                                          ("f64", "zhao_yong")])
def test_checkpoint_resume_is_bit_exact(L, storage, rule):
    p = cfg.cfg1(rule, "A")
    steps = 37 if rule == "mls" else 3  # Zhao-Yong with A breaks down at 7
    with L.Domain(p, storage=storage) as a:
        a.step(steps)
        st = L.lbm_get_state(a.h)
        a.step(25 if rule == "mls" else 2)
        ra = a.moments()
        ha = a.mass_history()
    with L.Domain(p, storage=storage) as b:
        L.lbm_set_state(b.h, st)
        assert b.t == steps
        b.step(25 if rule == "mls" else 2)
        rb = b.moments()
        hb = b.mass_history()
    for i in range(3):
        assert np.array_equal(ra[i], rb[i])
    assert np.array_equal(ha, hb)


def test_instability_is_reported_at_the_oracles_step(L):
    p = cfg.cfg1("zhao_yong", "none")
    o = ora.Oracle(p)
    with pytest.raises(ora.OracleError):
        o.step(200)
    bad = o.t  # step index whose mass was not finite
    with L.Domain(p) as d:
        with pytest.raises(L.LbmError) as e:
            d.step(200)
        assert e.value.code == L.LBM_EUNSTABLE
        assert L.lbm_unstable_step(d.h) == bad


def test_long_run_mass_drift_fp64(L):
    """Schemes A and B: |M(t) - M(0)| / M(0) <= 1e-10 over 1e5 steps."""
    for fix in ("A", "B"):
        p = cfg.cfg1("mls", fix)
        with L.Domain(p, history_capacity=1 << 17) as d:
            d.step(100000)
            h = d.mass_history()
        drift = np.max(np.abs(h - h[0])) / h[0]
        say(f"    {fix}: max drift over 1e5 steps {drift:.3e}")
        assert len(h) == 100001
        assert drift <= 1e-10


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_full_size_2048_properties(L, storage):
    """The 2048^2 MRT workload in the launch shape the benchmark times:
    scheme B conserves mass to round-off (FP64), the mirror symmetry about
    x = 1024 holds, and FP32 tracks FP64."""
    p = cfg.cfg2a()
    with L.Domain(p, storage=storage) as d:
        d.step(300)
        r, ux, uy = d.moments()
        h = d.mass_history()
        info = d.info()
    say(f"    {storage} info {info}")
    drift = np.max(np.abs(h - h[0])) / h[0]
    say(f"    {storage} mass drift {drift:.3e}")
    assert drift < (1e-13 if storage == "f64" else 1e-5)
    mir = lambda a: np.roll(a[:, ::-1], 1, axis=1)
    sym = np.max(np.abs(r - mir(r))) / r.max()
    say(f"    {storage} mirror asymmetry {sym:.3e}")
    assert sym < (1e-11 if storage == "f64" else 1e-5)
    assert np.max(np.abs(ux + mir(ux))) < (1e-11 if storage == "f64" else 1e-5)
    key = "full2048"
    if storage == "f64":
        _ORACLE[key] = (r, ux, uy)
    elif key in _ORACLE:
        fl = ~p.solid.astype(bool)
        e = [rel_err((r, ux, uy)[i], _ORACLE[key][i], fl) for i in range(3)]
        say(f"    fp32 vs fp64 {e}")
        assert max(e) < 1e-4


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_full_size_2048_matches_oracle(L, storage):
    """The 2048^2 MRT workload, MLS + B, in the benchmark's launch shape,
    against the oracle over its whole field for 16 steps (about 20 s of
    oracle time): FP64 within 1e-12, FP32 within the 1e-5 gate, every
    total mass on the way."""
    p = cfg.cfg2a()
    steps = 16
    key = ("full2048", steps)
    if key not in _ORACLE:
        o = ora.Oracle(p)
        m0 = o.total_mass()
        hist = o.step(steps)
        _ORACLE[key] = (*o.moments(), np.concatenate([[m0], hist]))
    ref = _ORACLE[key]
    g = gpu_run(L, p, steps, storage)
    compare(p, g, ref, F64_TOL if storage == "f64" else F32_TOL,
            MASS_TOL if storage == "f64" else 1e-7)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_full_size_8192_matches_oracle(L, storage):
    """The 8192 x 4096 many-cylinder workload (96 cylinders with droplets,
    BGK, MLS + B) against the oracle over its whole field for 2 steps
    (33.5 M nodes; about 15 s of oracle time)."""
    p = cfg.many_cylinders()
    steps = 2
    key = ("full8192", steps)
    if key not in _ORACLE:
        o = ora.Oracle(p)
        m0 = o.total_mass()
        hist = o.step(steps)
        _ORACLE[key] = (*o.moments(), np.concatenate([[m0], hist]))
    ref = _ORACLE[key]
    g = gpu_run(L, p, steps, storage)
    compare(p, g, ref, F64_TOL if storage == "f64" else F32_TOL,
            MASS_TOL if storage == "f64" else 1e-7)


def _couette_error(p, ux, uy):
    m = p.meta
    Y, X = np.mgrid[0:p.ny, 0:p.nx].astype(float)
    dx, dy = X - m["c"], Y - m["c"]
    r = np.maximum(np.hypot(dx, dy), 1e-9)
    r1, r2, U = m["r1"], m["r2"], m["U"]
    ut = U * r1 * (r2 ** 2 / r - r) / (r2 ** 2 - r1 ** 2)
    ax, ay = -ut * dy / r, ut * dx / r
    fl = ~p.solid.astype(bool)
    return float(np.sqrt(((ux - ax) ** 2 + (uy - ay) ** 2)[fl].sum() / (ax ** 2 + ay ** 2)[fl].sum()))


@pytest.mark.parametrize("fix", ["none", "A", "B"])
def test_couette_convergence_on_gpu(L, fix):
    """Circular Couette flow, r1 = 10, 20, 40, 80 (r2 = 2 r1, inner wall at
    surface speed 0.01), MLS, FP64, from rest to steady state: L2 error of
    the velocity against the analytic profile and its order.  The moving
    wall's momentum term changes the mass in every scheme (A and B correct
    only the rule's own leak); the change is reported."""
    errs = []
    for r1 in (10, 20, 40, 80):
        p = cfg.couette(r1, rule="mls", fix=fix, tau=0.8)
        steps = int(60 * r1 * r1)  # several viscous times (r2 - r1)^2 / nu
        with L.Domain(p, history_capacity=1 << 10) as d:
            m0 = d.total_mass()
            d.step(steps)
            _, ux, uy = d.moments()
            d.step(1000)
            _, ux2, uy2 = d.moments()
            du = float(np.max(np.abs(ux2 - ux)) + np.max(np.abs(uy2 - uy))) / 0.01
            drift = abs(d.total_mass() - m0) / m0
        e = _couette_error(p, ux2, uy2)
        errs.append(e)
        say(f"    {fix} r1={r1}: steps {steps + 1000}, L2 error {e:.3e}, "
            f"change over the last 1000 steps {du:.1e} U, mass change {drift:.1e}")
        assert du < 1e-9  # steady
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    mean = np.log2(errs[0] / errs[-1]) / 3
    say(f"    {fix}: orders {np.round(orders, 2)}, mean {mean:.2f}")
    assert np.all(np.diff(errs) < 0)
    if fix == "none":
        assert np.all(orders > 1.5) and 1.7 < mean < 2.5


@pytest.mark.parametrize("case", ["cfg1_zy", "wet_zy", "wet_ibbq", "cfg1_mls"])
def test_scheme_a_negative_rest_population_count(L, case):
    """Scheme A leaves some rest populations negative (counted, not
    clamped); the library counts the same (node, step) pairs as the oracle.
    In these cases it happens only as a run breaks down, so both run to the
    oracle's first unstable step; the stable MLS case counts none."""
    rl, _ = cfg.cs_init_densities(0.86)
    p = {"cfg1_zy": lambda: cfg.cfg1("zhao_yong", "A"),
         "wet_zy": lambda: cfg.droplet_on_cylinder(rule="zhao_yong", fix="A", rho_wall=rl,
                                                   tau=1.0, name="wet_zy"),
         "wet_ibbq": lambda: cfg.droplet_on_cylinder(rule="ibb_quadratic", fix="A",
                                                     rho_wall=0.25, tau=1.0, name="wet_ibbq"),
         "cfg1_mls": lambda: cfg.cfg1("mls", "A")}[case]()
    o = ora.Oracle(p)
    steps = 300
    try:
        o.step(steps)
    except ora.OracleError:
        steps = o.t
    want = int(o.counters()[4])
    with L.Domain(p, storage="f64") as d:
        try:
            d.step(steps)
        except L.LbmError as e:
            assert e.code == L.LBM_EUNSTABLE and steps < 300
        got = d.negative_rest()
    say(f"[gpu] {case}: {steps} steps, negative rest populations {got} (oracle {want})")
    assert got == want
    assert (want == 0) == (case == "cfg1_mls")


# ------------------------------------------ schemes A and B on resting walls
@pytest.mark.parametrize("fix", ["none", "A", "B"])
@pytest.mark.parametrize("case", ["sloped_channel16", "cylinder_array8"])
def test_resting_wall_cases_match_oracle(L, case, fix):
    """The resting-wall convergence cases at their smallest size, MLS with
    each fix, FP64, 1000 steps: fields and mass history against the
    oracle.  The body force is 100 times that of the convergence runs, so
    that the velocities (about 0.03) stand well above the FP64 rounding of
    the populations in the max-norm of each component."""
    p = (cfg.sloped_channel(16, fix=fix, g0=1e-3) if case == "sloped_channel16"
         else cfg.cylinder_array(8.0, fix=fix, g0=1e-3))
    g = gpu_run(L, p, 1000, history_capacity=2048)
    compare(p, g, oracle_run(p, 1000, key=(case, fix, "g0=1e-3")), F64_TOL, MASS_TOL)


def _sloped_error(p, ux, uy):
    Y, X = np.mgrid[0:p.ny, 0:p.nx].astype(np.float64)
    m = p.meta
    s = geo.SlopedBand(m["n"], m["s0"], m["s1"]).coordinate(X, Y)
    k = 2.0 / np.sqrt(5.0)
    z, h = (s - m["s1"]) * k, (m["n"] - (m["s1"] - m["s0"])) * k
    U = m["g"] / (2.0 * (p.tau - 0.5) / 3.0) * z * (h - z)
    tx, ty = m["direction"]
    fl = ~p.solid.astype(bool)
    return float(np.sqrt((((ux - U * tx) ** 2 + (uy - U * ty) ** 2)[fl]).sum()
                         / ((U ** 2)[fl]).sum()))


@pytest.mark.parametrize("fix", ["none", "A", "B"])
def test_resting_sloped_walls_convergence_on_gpu(L, fix):
    """The sloped channel at n = 16 ... 128 in FP64 to steady state: MLS
    alone converges at second order; A and B at first order, with the
    total mass constant to round-off (the oracle measures the same orders
    at n = 16, 32, 48)."""
    ns = (16, 32, 64, 128)
    errs, drifts = [], []
    for n in ns:
        p = cfg.sloped_channel(n, fix=fix)
        with L.Domain(p, history_capacity=1 << 10) as d:
            m0 = d.total_mass()
            d.step(12 * n * n)
            _, ux, uy = d.moments()
            drifts.append(abs(d.total_mass() - m0) / m0)
        errs.append(_sloped_error(p, ux, uy))
        say(f"    {fix} n={n}: L2 error {errs[-1]:.4e}, mass change {drifts[-1]:.1e}")
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    say(f"    {fix}: orders {np.round(orders, 3)}")
    if fix == "none":
        assert np.all((orders > 1.85) & (orders < 2.2))
    else:
        assert np.all((orders > 0.8) & (orders < 1.2))
        assert max(drifts) < 1e-16 * 12 * ns[-1] ** 2


@pytest.mark.parametrize("fix", ["none", "A", "B"])
def test_resting_cylinder_array_convergence_on_gpu(L, fix):
    """The cylinder array at d = 8 ... 128 in FP64 to steady state:
    permeabilities k/d^2, the differences between successive resolutions,
    and the mass change (reported; A and B to round-off)."""
    ds = (8.0, 16.0, 32.0, 64.0, 128.0)
    ks = []
    for d in ds:
        p = cfg.cylinder_array(d, fix=fix)
        with L.Domain(p, history_capacity=1 << 10) as dom:
            m0 = dom.total_mass()
            dom.step(int(25 * d * d))
            _, ux, _ = dom.moments()
            drift = abs(dom.total_mass() - m0) / m0
        nu = (p.tau - 0.5) / 3.0
        ks.append(nu * ux[~p.solid.astype(bool)].sum() / (p.nx * p.ny) / (p.meta["g"] * d * d))
        say(f"    {fix} d={d:g}: k/d^2 {ks[-1]:.8f}, mass change {drift:.1e}")
        if fix != "none":
            assert drift < 1e-16 * 25 * d * d
    diffs = np.abs(np.diff(ks))
    say(f"    {fix}: |k(2d) - k(d)| {np.array2string(diffs, precision=3)}")
    assert diffs[-1] < diffs[0]


@pytest.mark.parametrize("storage,steps_per_pass", [("f64", 1), ("f32", 1), ("f32", 2)])
def test_scheme_b_cancelling_sums_count(L, storage, steps_per_pass):
    """The (node, step) pairs where the sums of Eq. (22) cancel, counted by
    the library as by the oracle (eight nodes per step in the constructed
    case), also when two steps are made per pass."""
    from tests.test_oracle_physics import _cancelling_b_case
    p = _cancelling_b_case()
    o = ora.Oracle(p)
    o.step(10)
    want = int(o.counters()[3])
    say(f"[gpu] cancelling scheme-B sums, {storage}, {steps_per_pass} steps per pass")
    with L.Domain(p, storage=storage) as d:
        L.lbm_set_steps_per_pass(d.h, steps_per_pass)
        d.step(10)
        assert d.degenerate_b() == want == 80
        r, ux, uy = d.moments()
    fl = ~p.solid.astype(bool)
    assert np.abs(r[fl] - 1.0).max() < 1e-6 and np.abs(ux[fl]).max() < 1e-12
