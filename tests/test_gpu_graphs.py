"""Captured step graphs: lbm_step replays captured runs of 1, 2, 4, ..., 32
steps; with kernel timing on it launches every kernel itself.  Both must
give the same fields and mass history bit for bit, for run lengths of
either parity and across a checkpoint."""
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


RUNS = (1, 2, 5, 37, 64, 3, 100)


@pytest.mark.parametrize("storage,steps_per_pass", [("f64", 1), ("f32", 1), ("f32", 2)])
def test_graph_replay_equals_plain_launches(L, storage, steps_per_pass):
    p = cfg.cfg1("mls", "B")
    say(f"[gpu] graphs vs plain launches, cfg1 MLS+B {storage}, {steps_per_pass} step(s) "
        f"per pass, runs {RUNS}")
    with L.Domain(p, storage=storage, history_capacity=512) as g, \
            L.Domain(p, storage=storage, history_capacity=512) as e:
        if steps_per_pass == 2:
            L.lbm_set_steps_per_pass(g.h, 2, 0)
            L.lbm_set_steps_per_pass(e.h, 2, 0)
        L.lbm_set_profiling(e.h, 1)  # timed steps launch every kernel
        for n in RUNS:
            g.step(n)
            e.step(n)
            assert g.t == e.t
            for a, b in zip(g.moments(), e.moments()):
                assert np.array_equal(a, b), n
            assert g.total_mass() == e.total_mass()
        # one main launch per pass: two steps each where the domain fuses
        # them, a single step to finish an odd count
        steps, _ = L.lbm_get_steps_per_pass(e.h)
        passes = sum(n if steps == 1 else (n + 1) // 2 for n in RUNS)
        main_ms, cnt, bnd_ms, bcnt = L.lbm_kernel_times(e.h)
        assert cnt == passes and bcnt == passes
        # each launch recorded its own start and end: positive durations,
        # far below a millisecond on a 128 x 128 lattice
        say(f"    main {main_ms / cnt * 1e3:.2f} us, boundary {bnd_ms / bcnt * 1e3:.2f} us")
        assert 0.0 < main_ms / cnt < 1.0 and 0.0 < bnd_ms / bcnt < 1.0
        assert np.array_equal(g.mass_history(), e.mass_history())


def test_graph_replay_resumes_from_a_checkpoint(L):
    p = cfg.cfg1("mls", "A")
    say("[gpu] checkpoint at step 7, restored, 33 more steps by graph replay")
    with L.Domain(p, storage="f64", history_capacity=64) as a:
        a.step(7)
        st = L.lbm_get_state(a.h)
        a.step(33)
        want = a.moments()
        hw = a.mass_history()
        a.step(5)
        L.lbm_set_state(a.h, st)
        assert a.t == 7
        a.step(33)
        for x, y in zip(a.moments(), want):
            assert np.array_equal(x, y)
        assert np.array_equal(a.mass_history(), hw)
