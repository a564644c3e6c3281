"""Checkpoints and the mass-history ring through the C ABI: states that do
not belong to the domain are refused and leave it untouched, and a ring
smaller than the run keeps the last masses in time order."""
import ctypes
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


def _set(L, h, buf):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    return L.lib().lbm_set_state(h, buf.ctypes.data_as(ctypes.c_void_p), ctypes.c_size_t(buf.nbytes))


def test_foreign_or_damaged_states_are_refused(L):
    p = cfg.cfg1("mls", "B")
    say("[gpu] foreign and damaged checkpoints")
    with L.Domain(p, storage="f64", history_capacity=64) as a:
        a.step(7)
        st = L.lbm_get_state(a.h)
        m7 = a.moments()
        n = ctypes.c_size_t(st.size - 1)
        small = np.zeros(st.size, np.uint8)
        assert L.lib().lbm_get_state(a.h, small.ctypes.data_as(ctypes.c_void_p),
                                     ctypes.byref(n)) == L.LBM_EINVAL
        for bad in (st[:-1], np.concatenate([st, st[:1]])):
            assert _set(L, a.h, bad) == L.LBM_EINVAL
        # header: magic, step, nx << 32 | ny, storage (four 64-bit words)
        for word, value in ((0, 0x1234), (2, (64 << 32) | 256), (3, 1)):
            broken = st.copy()
            broken[8 * word:8 * word + 8] = np.frombuffer(np.uint64(value).tobytes(), np.uint8)
            assert _set(L, a.h, broken) == L.LBM_EINVAL, word
        # the refusals left the domain as it was
        assert a.t == 7
        assert all(np.array_equal(x, y) for x, y in zip(a.moments(), m7))
    with L.Domain(p, storage="f32", history_capacity=64) as c:
        assert _set(L, c.h, st) == L.LBM_EINVAL


def test_short_mass_history_keeps_the_last_masses(L):
    p = cfg.cfg1("mls", "A")
    say("[gpu] mass-history ring of 8 over 20 steps")
    with L.Domain(p, storage="f64", history_capacity=64) as a:
        a.step(20)
        full = a.mass_history()
        m = a.total_mass()
    with L.Domain(p, storage="f64", history_capacity=8) as b:
        b.step(20)
        last = b.mass_history()
        assert b.total_mass() == m
    assert full.size == 21 and last.size == 8
    assert np.array_equal(last, full[-8:])
    assert full[-1] == m
