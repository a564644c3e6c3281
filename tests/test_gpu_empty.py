"""Degenerate calls through the C ABI: zero steps, a negative step count, an
empty batch (run and autotuned), an instance that runs no steps beside one
that does, and a server that never receives a request."""
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


def _same(a, b):
    return all(np.array_equal(a[i], b[i]) for i in range(3))


def test_zero_steps_change_nothing(L):
    p = cfg.cfg1("mls", "B")
    say("[gpu] zero and negative step counts, cfg1 mls/B f64")
    with L.Domain(p, storage="f64", history_capacity=16) as d:
        m0, h0 = d.moments(), d.mass_history()
        d.step(0)
        assert d.t == 0 and _same(d.moments(), m0)
        assert np.array_equal(d.mass_history(), h0)
        with pytest.raises(L.LbmError) as e:
            L.lbm_step(d.h, -1)
        assert e.value.code == L.LBM_EINVAL
        d.step(3)
        m3 = d.moments()
        d.step(0)
        assert d.t == 3 and _same(d.moments(), m3)


def test_empty_batch_runs_and_tunes(L):
    say("[gpu] empty batch")
    with L.Batch(storage="f32", eos="cs", max_instances=4, arena_bytes=1 << 26) as b:
        b.run(0)
        b.run(10)
        b.sync()
        assert b.info()["instances"] == 0 and b.info()["tiles"] == 0
        t = b.tune(2)
        assert t["tile_w"] in (64, 128, 256)
        b.run(5)
        b.sync()
        with pytest.raises(L.LbmError) as e:
            b.run(-1)
        assert e.value.code == L.LBM_EINVAL


def test_instance_with_no_steps_beside_one_that_runs(L):
    """An instance added with 0 steps stays at t = 0 with the moments of a
    fresh domain; its neighbour in the batch runs its 5 steps and matches
    the domain run alone (the fields do not depend on the launch shape)."""
    p = cfg.cfg1("mls", "B")
    say("[gpu] batch: instance with 0 steps beside one with 5")
    with L.Domain(p, storage="f64") as d:
        fresh = d.moments()
        d.step(5)
        five = d.moments()
    with L.Batch(storage="f64", eos="cs", max_instances=4, arena_bytes=1 << 28) as b:
        s0 = b.add(p, 0)
        s1 = b.add(p, 5)
        b.run(10)
        b.sync()
        assert b.status(s0) == (0, 0, -1)
        assert b.status(s1) == (5, 0, -1)
        assert _same(b.moments(s0), fresh)
        assert _same(b.moments(s1), five)


def test_server_without_requests(L):
    say("[gpu] server with no requests")
    p = cfg.cfg1("mls", "B")
    with L.Server(chunk_steps=10, storage="f32", eos="cs", max_instances=4,
                  arena_bytes=1 << 26) as s:
        assert s.progress() == [] and s.progress() == []
        info = s.info()
        assert info["queued"] == info["running"] == info["finished"] == 0
        assert info["arena_used"] == 0
        with pytest.raises(L.LbmError) as e:
            s.submit(p, 0)
        assert e.value.code == L.LBM_EINVAL
        assert s.progress() == [] and s.info()["queued"] == 0
