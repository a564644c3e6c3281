"""Pins of the oracle's pure functions against mathematics, not against
themselves: moment identities, interpolation properties, special cases."""
import numpy as np
import pytest

from oracle import core as ora
from oracle import eos as oeos
from lbm_inputs.problem import LINK_DTYPE, Problem

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], float)
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]
RNG = np.random.default_rng(12345)


def _states(n=20):
    for _ in range(n):
        yield (RNG.uniform(0.02, 3.0), RNG.uniform(-0.1, 0.1),
               RNG.uniform(-0.1, 0.1), RNG.uniform(-0.01, 0.01),
               RNG.uniform(-0.01, 0.01))


def test_equilibrium_moments():
    """Eq. (4): zeroth, first and second moments are rho, rho u and
    rho c_s^2 I + rho u u."""
    for rho, ux, uy, _, _ in _states():
        f = ora.feq(rho, ux, uy)
        assert np.isclose(f.sum(), rho, rtol=1e-15, atol=0)
        assert np.isclose(f @ EX, rho * ux, rtol=1e-13, atol=1e-17)
        assert np.isclose(f @ EY, rho * uy, rtol=1e-13, atol=1e-17)
        assert np.isclose(f @ (EX * EX), rho / 3 + rho * ux * ux, rtol=1e-14)
        assert np.isclose(f @ (EY * EY), rho / 3 + rho * uy * uy, rtol=1e-14)
        assert np.isclose(f @ (EX * EY), rho * ux * uy, rtol=1e-12, atol=1e-17)


def test_equilibrium_weights_at_rest():
    f = ora.feq(1.0, 0.0, 0.0)
    assert np.allclose(f, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, rtol=0, atol=1e-17)


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_guo_forcing_moments(tau):
    """Guo et al. (2002): sum F_a = 0, sum F_a e = (1 - 1/2tau) F,
    sum F_a e e = (1 - 1/2tau)(u F + F u)."""
    for _, ux, uy, Fx, Fy in _states():
        g = ora.guo(tau, ux, uy, Fx, Fy)
        k = 1 - 0.5 / tau
        assert abs(g.sum()) < 1e-17
        assert np.isclose(g @ EX, k * Fx, rtol=1e-13, atol=1e-19)
        assert np.isclose(g @ EY, k * Fy, rtol=1e-13, atol=1e-19)
        assert np.isclose(g @ (EX * EX), k * 2 * ux * Fx, rtol=1e-11, atol=1e-18)
        assert np.isclose(g @ (EY * EY), k * 2 * uy * Fy, rtol=1e-11, atol=1e-18)
        assert np.isclose(g @ (EX * EY), k * (ux * Fy + uy * Fx), rtol=1e-11, atol=1e-18)


def _pre_collision(rho, ux, uy, Fx, Fy):
    """A random pre-collision state whose Eq. (5) velocity is (ux, uy)."""
    f = ora.feq(rho, ux, uy) + RNG.normal(0, 1e-3, 9) * rho
    # restore rho and rho u - F/2 exactly enough for the identities
    f[0] += rho - f.sum()
    jx, jy = rho * ux - Fx / 2, rho * uy - Fy / 2
    dx, dy = jx - f @ EX, jy - f @ EY
    f[1] += dx / 2; f[3] -= dx / 2
    f[2] += dy / 2; f[4] -= dy / 2
    return f


@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_collision_conserves_mass_and_adds_force(collision):
    """Eq. (2) with Guo forcing: mass unchanged, momentum sum f e changes by
    exactly F (for BGK and for MRT with any rates)."""
    tau = 0.8
    s = [1.0, 1.3, 1.1, 1.0, 1.7, 1.0, 1.7, 1 / tau, 1 / tau]
    for rho, ux, uy, Fx, Fy in _states():
        f = _pre_collision(rho, ux, uy, Fx, Fy)
        out = ora.collide(collision, tau, s, f, rho, ux, uy, Fx, Fy)
        assert np.isclose(out.sum(), f.sum(), rtol=1e-14)
        assert np.isclose(out @ EX - f @ EX, Fx, rtol=1e-9, atol=1e-15)
        assert np.isclose(out @ EY - f @ EY, Fy, rtol=1e-9, atol=1e-15)


def test_mrt_matrix_is_invertible_and_orthogonal():
    M, Mi = ora.mrt_matrix()
    assert np.allclose(M @ Mi, np.eye(9), atol=1e-15)
    G = M @ M.T
    assert np.allclose(G - np.diag(np.diag(G)), 0)
    # Lallemand & Luo (2000): |rows|^2 = 9, 36, 36, 6, 12, 6, 12, 4, 4
    assert np.allclose(np.diag(G), [9, 36, 36, 6, 12, 6, 12, 4, 4])
    # conserved rows: density and momentum
    assert np.allclose(M[0], 1) and np.allclose(M[3], EX) and np.allclose(M[5], EY)


@pytest.mark.parametrize("tau", [0.55, 0.8, 1.0, 1.6])
def test_mrt_with_equal_rates_is_bgk(tau):
    """Special case: every rate 1/tau reduces MRT to BGK."""
    s = [1 / tau] * 9
    for rho, ux, uy, Fx, Fy in _states(10):
        f = _pre_collision(rho, ux, uy, Fx, Fy)
        a = ora.collide("mrt", tau, s, f, rho, ux, uy, Fx, Fy)
        b = ora.collide("bgk", tau, s, f, rho, ux, uy, Fx, Fy)
        assert np.allclose(a, b, rtol=1e-13, atol=1e-16)


def test_cs_critical_point_matches_literature(golden):
    """The oracle's Carnahan-Starling pressure has its critical point at the
    published constants b rho_c = 0.5218, R T_c b / a = 0.3773,
    Z_c = 0.3590."""
    g = golden["cs_critical_point"]
    a, b, R = 1.0, 4.0, 1.0
    Tc = g["RTc_b_over_a"] * a / (b * R)
    rc = g["b_rho_c"] / b
    p = lambda r, T: ora.pressure_eos("cs", (a, b, R, T), r)
    h = 1e-4
    # scan T near the literature T_c for the temperature where the
    # spinodal closes: dp/drho has its minimum exactly at zero
    def min_slope(T):
        rs = np.linspace(0.08, 0.18, 2001)
        d = [(p(r + h, T) - p(r - h, T)) / (2 * h) for r in rs]
        i = int(np.argmin(d))
        return d[i], rs[i]
    lo, hi = Tc * 0.99, Tc * 1.01
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        if min_slope(mid)[0] < 0:
            lo = mid
        else:
            hi = mid
    T_found = 0.5 * (lo + hi)
    r_found = min_slope(T_found)[1]
    assert abs(T_found * b * R / a - g["RTc_b_over_a"]) < 2e-4
    assert abs(r_found * b - g["b_rho_c"]) < 2e-3
    Zc = p(r_found, T_found) / (r_found * R * T_found)
    assert abs(Zc - g["Z_c"]) < 2e-3


def test_psi_model_pressure_recovers_cs():
    """psi for CS is defined so that rho c_s^2 + G psi^2/2 is the EOS."""
    prm = (1.0, 4.0, 1.0, 0.08)
    for r in np.linspace(0.01, 0.4, 17):
        ps = ora.psi("cs", prm, -1.0, r)
        assert np.isclose(r / 3 - 0.5 * ps * ps, ora.pressure_eos("cs", prm, r), rtol=1e-12, atol=1e-16)


# ---------------------------------------------------------------- rules
def _rule(rule, q, tau=0.8, **kw):
    return ora.rule_incoming(rule, kw.pop("dir", 1), q, tau, **kw)[0]


@pytest.mark.parametrize("q", [0.05, 0.2, 0.37, 0.49])
def test_linear_bouzidi_q_lt_half_interpolates(q):
    """Eq. (12), q < 1/2: the value that reaches x_b after reflection left
    from s = 2q - 1 (s = 0 at x_b, -1 at x_f); linear interpolation of a
    linear field is exact."""
    for _ in range(5):
        c0, c1 = RNG.normal(size=2)
        h = lambda s: c0 + c1 * s
        got = _rule("ibb_linear", q, fa_b=h(0), fa_f=h(-1), fab_b=7.0)
        assert np.isclose(got, h(2 * q - 1), rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("q", [0.5, 0.63, 0.8, 1.0])
def test_linear_bouzidi_q_ge_half_interpolates(q):
    """Eq. (12), q >= 1/2: f_abar at x_b interpolated between the reflected
    particle at s = 2q - 1 (value f*_a(x_b)) and f_abar one node back at
    s = -1 (value f*_abar(x_b) after streaming)."""
    for _ in range(5):
        c0, c1 = RNG.normal(size=2)
        h = lambda s: c0 + c1 * s
        got = _rule("ibb_linear", q, fa_b=h(2 * q - 1), fab_b=h(-1), fa_f=9.0)
        assert np.isclose(got, h(0.0), rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("q", [0.05, 0.2, 0.37, 0.49])
def test_quadratic_bouzidi_q_lt_half_interpolates(q):
    for _ in range(5):
        c = RNG.normal(size=3)
        h = lambda s: c[0] + c[1] * s + c[2] * s * s
        got = _rule("ibb_quadratic", q, fa_b=h(0), fa_f=h(-1), fa_ff=h(-2))
        assert np.isclose(got, h(2 * q - 1), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("q", [0.5, 0.63, 0.8, 1.0])
def test_quadratic_bouzidi_q_ge_half_interpolates(q):
    """Nodes s = 2q - 1 (reflected f*_a(x_b)), -1 (f*_abar(x_b)),
    -2 (f*_abar(x_f)); evaluated at s = 0."""
    for _ in range(5):
        c = RNG.normal(size=3)
        h = lambda s: c[0] + c[1] * s + c[2] * s * s
        got = _rule("ibb_quadratic", q, fa_b=h(2 * q - 1), fab_b=h(-1), fab_f=h(-2))
        assert np.isclose(got, h(0.0), rtol=1e-12, atol=1e-13)


def test_quadratic_bouzidi_falls_back_when_x_ff_is_solid():
    q = 0.3
    a = _rule("ibb_quadratic", q, fa_b=1.3, fa_f=0.7, fa_ff=5.0, ff_ok=0)
    b = _rule("ibb_linear", q, fa_b=1.3, fa_f=0.7)
    assert a == b


@pytest.mark.parametrize("dir", range(1, 9))
def test_half_q_reduces_to_halfway(dir):
    """Sec. 2.2: at q = 1/2 (chi = 0) FH, MLS and both Bouzidi schemes give
    f*_a(x_b) exactly; Zhao-Yong does not (text after Eq. 14)."""
    kw = dict(fa_b=0.123, fab_b=0.456, fa_f=0.2, fab_f=0.3, fa_ff=0.1,
              fpre_a=0.777, rho_b=1.1, ubx=0.03, uby=-0.02, ufx=0.01,
              ufy=0.02, dir=dir)
    for rule in ("fh", "mls", "ibb_linear", "ibb_quadratic", "halfway"):
        assert _rule(rule, 0.5, tau=0.7, **dict(kw)) == 0.123
    assert _rule("zhao_yong", 0.5, **dict(kw)) != 0.123


@pytest.mark.parametrize("q", [0.5, 0.6, 0.9, 1.0])
def test_fh_equals_mls_for_q_ge_half(q):
    """Both use Eq. (10) for q >= 1/2."""
    kw = dict(fa_b=0.123, fab_b=0.456, rho_b=1.1, ubx=0.03, uby=-0.02,
              ufx=0.5, ufy=0.5, dir=5)
    assert _rule("fh", q, tau=0.7, **dict(kw)) == _rule("mls", q, tau=0.7, **dict(kw))


@pytest.mark.parametrize("rule", ["halfway", "fh", "mls", "ibb_linear",
                                  "ibb_quadratic", "zhao_yong"])
@pytest.mark.parametrize("q", [0.1, 0.5, 0.8])
@pytest.mark.parametrize("dir", [2, 7])
def test_rest_state_is_a_fixed_point(rule, q, dir):
    """The coefficients of every rule sum to one, so a fluid at rest with
    f = w rho returns w rho."""
    w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
    rho = 1.37
    v = w[dir] * rho
    got = _rule(rule, q, tau=0.7, dir=dir, fa_b=v, fab_b=v, fa_f=v, fab_f=v,
                fa_ff=v, fpre_a=v, rho_b=rho)
    assert np.isclose(got, v, rtol=2e-15)


def test_mls_chi_limits():
    """chi = (2q-1)/(tau-2) below 1/2 (Eq. 11) and (2q-1)/tau above
    (Eq. 10); FH uses (2q-1)/(tau-1) below 1/2 (Eq. 9)."""
    _, chi, _ = ora.rule_incoming("mls", 1, 0.25, 0.8, rho_b=1.0)
    assert np.isclose(chi, (0.5 - 1) / (0.8 - 2))
    _, chi, _ = ora.rule_incoming("mls", 1, 0.75, 0.8, rho_b=1.0)
    assert np.isclose(chi, 0.5 / 0.8)
    _, chi, _ = ora.rule_incoming("fh", 1, 0.25, 0.8, rho_b=1.0)
    assert np.isclose(chi, -0.5 / -0.2)


def test_moving_wall_halfway_is_ladd():
    """Halfway bounce-back off a wall moving at u_w returns
    f*_a - 2 w_a rho (e_a . u_w) / c_s^2: a fluid in equilibrium moving
    with the wall is reflected into its own equilibrium (the quadratic
    terms of Eq. 4 are even in e)."""
    rho, uw = 1.0, 1e-4
    for d in range(1, 9):
        fa = ora.feq(rho, 0.0, uw)[d]
        got = _rule("halfway", 0.5, dir=d, fa_b=fa, rho_b=rho, uwy=uw)
        want = ora.feq(rho, 0.0, uw)[OPP[d]]
        assert abs(got - want) < 1e-16


# --------------------------------------------- MRT forcing, non-conserved moments
def _ll_basis():
    """Lallemand-Luo rows written out from their polynomials in the lattice
    velocity (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy)."""
    c2 = EX * EX + EY * EY
    return np.array([np.ones(9), -4 + 3 * c2, 4 - 10.5 * c2 + 4.5 * c2 * c2,
                     EX, (-5 + 3 * c2) * EX, EY, (-5 + 3 * c2) * EY,
                     EX * EX - EY * EY, EX * EY])


@pytest.mark.parametrize("rho0", [1.0, 0.37])
def test_mrt_forced_box_fixed_point(rho0):
    """MRT forcing on the non-conserved moments, pinned by a fixed point.

    A spatially uniform, periodic fluid under a constant body force has no
    streaming: each step maps the moments m to
    m - S (m - m_eq) + (I - S/2) M Fbar, while the momentum grows by exactly
    F, so u grows by F/rho and the equilibrium moments grow by
    dm_eq = (0, 6u.F, -6u.F, F_x, -F_x, F_y, -F_y, 2(u_x F_x - u_y F_y),
    u_x F_y + u_y F_x) + O(F^2) per step -- which is the Guo source M Fbar
    itself.  The non-equilibrium part n = m - m_eq therefore settles where
    s n = (1 - s/2) M Fbar - dm_eq, i.e. n = -M Fbar / 2 whatever the rate
    s of the moment.  A prefactor (1 - 1/(2 tau)) in place of (1 - s/2)
    would settle at -M Fbar / (2 tau s) instead, which the rates below keep
    at least 10 % away."""
    tau = 0.8
    s = (1.0, 1.1, 1.6, 1.0, 1.4, 1.0, 1.45, 1 / tau, 1 / tau)
    for i in (1, 2, 4, 6):
        assert abs(1.0 / (2 * tau * s[i]) - 0.5) > 0.05
    n = 4
    g = (1.0e-6, -0.7e-6)
    u0 = (0.05, -0.03)
    p = Problem(nx=n, ny=n, solid=np.zeros((n, n), np.uint8),
                links=np.zeros(0, dtype=LINK_DTYPE), rho0=np.full((n, n), rho0),
                rho_wall=np.ones((n, n)), eos="none", tau=tau, gravity=g,
                collision="mrt", mrt_s=s, ux0=np.full((n, n), u0[0]),
                uy0=np.full((n, n), u0[1]), name="forced_box")
    o = ora.Oracle(p)
    o.step(300)   # the start f_eq(rho0, u0) has n = 0; |1 - s| <= 0.6 per step
    f = o.get_f()[:, 1, 2]
    rho = f.sum()
    Fx, Fy = rho * g[0], rho * g[1]
    ux = (f @ EX + 0.5 * Fx) / rho           # Eq. (5)
    uy = (f @ EY + 0.5 * Fy) / rho
    usq = ux * ux + uy * uy
    m_eq = np.array([rho, -2 * rho + 3 * rho * usq, rho - 3 * rho * usq,
                     rho * ux, -rho * ux, rho * uy, -rho * uy,
                     rho * (ux * ux - uy * uy), rho * ux * uy])
    src = np.array([0.0, 6 * (ux * Fx + uy * Fy), -6 * (ux * Fx + uy * Fy),
                    Fx, -Fx, Fy, -Fy, 2 * (ux * Fx - uy * Fy), ux * Fy + uy * Fx])
    neq = _ll_basis() @ f - m_eq
    for i in (1, 2, 4, 6, 7, 8):
        # O(F^2) and rounding are ~1e-12 against |src| >= 7e-8
        assert abs(neq[i] + 0.5 * src[i]) <= 1e-4 * abs(src[i]), (i, neq[i], -0.5 * src[i])
