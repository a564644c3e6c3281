"""Two steps per pass (k_main2) against single steps: the fields are
bit-identical after any number of steps (odd counts end with a single
step), for every rule, fix, EOS, collision and storage form the two-step
kernel takes, every two-step tile height and lattices narrower than a
strip; masses agree to rounding (the per-tile partial sums are grouped
differently), and so do the wall force, the negative-rest count and
checkpoints."""
import sys

import numpy as np
import pytest

from lbm_inputs import configs as cfg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    from paper_1908_09235_amd import lbm
    lbm.lib()
    return lbm


def _cases():
    return {
        "cfg1_mls_B": lambda: cfg.cfg1("mls", "B"),
        "cfg1_mls_A": lambda: cfg.cfg1("mls", "A"),
        "cfg1_ibbl_none": lambda: cfg.cfg1("ibb_linear", "none"),
        "cfg1_halfway": lambda: cfg.cfg1("halfway", "none"),
        "cfg1_mls_bao": lambda: cfg.cfg1("mls", "bao"),
        "drop_fh_B_mrt": lambda: cfg.droplet_on_cylinder(rule="fh", fix="B", tau=0.8,
                                                         collision="mrt", rho_wall=0.05,
                                                         name="drop_fh_mrt"),
        "drop256_mrt": lambda: cfg.cfg2a(scale=2.0),
        "gravity_q03": lambda: cfg.static_gravity(0.3, rule="mls", fix="A", nx=40, ny=30),
        "sloped16_B": lambda: cfg.sloped_channel(16, fix="B", g0=1e-3),
        "cylarr8_A": lambda: cfg.cylinder_array(8.0, fix="A", g0=1e-3),
        "exp_droplet": lambda: cfg.free_droplet(64, 12.0, eos="exp"),
        "couette10_mls_A": lambda: cfg.couette(10, rule="mls", fix="A"),
    }


def _pair(L, p, storage, tile_h=0):
    a = L.Domain(p, storage=storage, history_capacity=4096)
    b = L.Domain(p, storage=storage, history_capacity=4096)
    L.lbm_set_steps_per_pass(a.h, 2, tile_h)
    L.lbm_set_steps_per_pass(b.h, 1)
    return a, b


def _fluid_state(L, d, p, storage):
    """f*(t) of the fluid nodes from a checkpoint (the buffer holding the
    current state comes first, after a 32-byte header)."""
    st = L.lbm_get_state(d.h)
    es = {"f32": 4, "f32_arith32": 4, "f32dev": 4, "f16dev": 2}[storage]
    dt = {4: np.uint32, 2: np.uint16}[es]
    pitch = (p.nx + 63) // 64 * 64
    plane = pitch * p.ny + 256
    f = np.frombuffer(st[32:32 + 9 * plane * es].tobytes(), dtype=dt).reshape(9, plane)
    f = f[:, :pitch * p.ny].reshape(9, p.ny, pitch)[:, :, :p.nx]
    return f[:, ~p.solid.astype(bool)]


def _same(a, b, tag):
    for x, y in zip(a.moments(), b.moments()):
        assert np.array_equal(x, y, equal_nan=True), tag
    ha, hb = a.mass_history(), b.mass_history()
    assert len(ha) == len(hb)
    ok = np.isfinite(hb)
    assert np.array_equal(np.isfinite(ha), ok), tag
    assert np.all(np.abs(ha[ok] - hb[ok]) <= 1e-13 * np.abs(hb[ok])), tag


@pytest.mark.parametrize("case", sorted(_cases()))
@pytest.mark.parametrize("storage", ["f32", "f32_arith32", "f32dev", "f16dev"])
def test_two_steps_per_pass_equal_single_steps(L, case, storage):
    p = _cases()[case]()
    say(f"[gpu] two-step vs single-step passes: {case} {storage} {p.nx}x{p.ny}")
    a, b = _pair(L, p, storage)
    try:
        for n in (2, 1, 6, 51, 140):
            for d in (a, b):
                try:
                    d.step(n)
                except L.LbmError as e:
                    assert e.code == L.LBM_EUNSTABLE
            assert a.t == b.t
            if a.t % 2 == 0:  # a's last pass made two steps
                fa, fb = _fluid_state(L, a, p, storage), _fluid_state(L, b, p, storage)
                bad = np.nonzero(fa != fb)
                assert bad[0].size == 0, (case, storage, a.t, bad[0][:5], bad[1][:5])
            _same(a, b, (case, storage, a.t))
            fa, fb = a.wall_force(), b.wall_force()
            assert np.array_equal(fa, fb, equal_nan=True), (fa, fb)
        assert a.negative_rest() == b.negative_rest()
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("tile_h", [4, 7, 24, 64])
def test_two_step_tile_heights(L, tile_h):
    p = cfg.cfg1("mls", "B")
    say(f"[gpu] two-step tile height {tile_h}")
    a, b = _pair(L, p, "f32", tile_h)
    try:
        a.step(100)
        b.step(100)
        assert L.lbm_get_steps_per_pass(a.h) == (2, tile_h)
        _same(a, b, tile_h)
    finally:
        a.close()
        b.close()


def test_two_step_checkpoint_resumes(L):
    p = cfg.cfg1("mls", "A")
    say("[gpu] checkpoint after a two-step pass, restored into a new domain")
    with L.Domain(p, storage="f32", history_capacity=256) as a:
        L.lbm_set_steps_per_pass(a.h, 2)
        a.step(20)
        st = L.lbm_get_state(a.h)
        m20 = a.moments()
        a.step(30)
        want = a.moments()
        with L.Domain(p, storage="f32", history_capacity=256) as c:
            L.lbm_set_steps_per_pass(c.h, 2)
            L.lbm_set_state(c.h, st)
            for x, y in zip(c.moments(), m20):
                assert np.array_equal(x, y)
            c.step(30)
            for x, y in zip(c.moments(), want):
                assert np.array_equal(x, y)


def test_two_steps_refused_where_not_available(L):
    for p, st in ((cfg.cfg1("zhao_yong", "A"), "f32"), (cfg.cfg1("ibb_quadratic", "A"), "f32"),
                  (cfg.cfg1("mls", "B"), "f64"),
                  (cfg.cfg1("mls", "B"), "f16node")):
        with L.Domain(p, storage=st) as d:
            assert L.lbm_get_steps_per_pass(d.h)[0] == 1
            assert L.lib().lbm_set_steps_per_pass(d.h, 2, 0) == L.LBM_EINVAL
            assert L.lbm_get_steps_per_pass(d.h)[0] == 1


@pytest.mark.parametrize("storage", ["f32", "f32_arith32", "f64"])
def test_tuner_keeps_results(L, storage):
    """lbm_tune_steps_per_pass times every setting on real steps and keeps
    the fastest; the steps it runs are steps of the domain and give the
    same fields as single steps (FP64 storage has only one setting)."""
    p = cfg.cfg1("mls", "B")
    with L.Domain(p, storage=storage, history_capacity=4096) as a, \
            L.Domain(p, storage=storage, history_capacity=4096) as b:
        best = a.tune_steps_per_pass(4)
        say(f"[gpu] tuned {storage}: {best}")
        assert best["steps_per_pass"] in (1, 2) and best["tile_h"] > 0 and best["us_per_step"] > 0
        if storage == "f64":
            assert best["steps_per_pass"] == 1
        assert L.lbm_get_steps_per_pass(a.h) == (best["steps_per_pass"], best["tile_h"])
        a.step(7)
        b.step(a.t)
        _same(a, b, f"tuned {storage}")
        with pytest.raises(L.LbmError):
            L.lbm_tune_steps_per_pass(a.h, 1)
