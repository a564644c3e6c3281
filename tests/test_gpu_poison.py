"""Every slot a pull reads across a wall (a ghost slot of a solid node) or
across the cut seam of open x boundaries is written by the boundary pass
of that step: with those slots set to NaN before the step, the step gives
the same fields and mass, bit for bit.  A missing cut link, a ghost
written to the wrong slot or an open row left out would let a NaN in.

This reads the checkpoint layout of the library: a 32-byte header, then
the buffer holding f*(t) -- nine planes of pitch * ny + 256 elements
(pitch = nx rounded up to 64; node (x, y) at y * pitch + x), plus, for the
FP16 per-node form, an FP32 plane of node densities of the same length --
then the other buffer and the rest."""
import sys

import numpy as np
import pytest

from lbm_inputs import configs as cfg

pytestmark = pytest.mark.gpu

DTYPE = {"f64": np.float64, "f32": np.float32, "f32dev": np.float32,
         "f16dev": np.float16, "f16node": np.float16}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    from paper_1908_09235_amd import lbm
    lbm.lib()
    return lbm


def _poison(state, p, storage, seam):
    pitch = (p.nx + 63) // 64 * 64
    plane = pitch * p.ny + 256
    dt = DTYPE[storage]
    st = state.copy()
    f = st[32:32 + 9 * plane * np.dtype(dt).itemsize].view(dt).reshape(9, plane)
    ys, xs = np.nonzero(p.solid)
    idx = ys * pitch + xs
    f[1:, idx] = np.nan  # plane 0 of a solid node holds psi_w
    if storage == "f16node":
        off = 32 + 9 * plane * 2
        rpl = st[off:off + 4 * plane].view(np.float32)
        rpl[idx] = np.nan
    if seam:
        rows = np.arange(p.ny) * pitch
        for a in (1, 5, 8):
            f[a, rows + p.nx - 1] = np.nan
        for a in (3, 6, 7):
            f[a, rows] = np.nan
    return st


CASES = [("f64", cfg.cfg1, ("mls", "B")), ("f32", cfg.cfg1, ("ibb_quadratic", "A")),
         ("f64", cfg.cfg1, ("zhao_yong", "none")), ("f32dev", cfg.cfg1, ("ibb_linear", "none")),
         ("f16node", cfg.cfg1, ("mls", "A")), ("f16dev", cfg.cfg1, ("halfway", "none"))]


@pytest.mark.parametrize("storage,make,args", CASES)
def test_walls_fill_every_ghost_they_expose(L, storage, make, args):
    p = make(*args)
    _check(L, p, storage, seam=False)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_open_boundaries_fill_the_seam(L, storage):
    p = cfg.cylinder_flow(20.0, fix="A", d=8.0)
    _check(L, p, storage, seam=True)


def _check(L, p, storage, seam):
    say(f"[gpu] poison {p.name} {p.rule}/{p.fix} {storage} seam={seam}")
    with L.Domain(p, storage=storage, history_capacity=64) as d:
        d.step(3)
        st = L.lbm_get_state(d.h)
        d.step(1)
        ref = d.moments()
        href = d.mass_history()
    with L.Domain(p, storage=storage, history_capacity=64) as d:
        L.lbm_set_state(d.h, _poison(st, p, storage, seam))
        d.step(1)
        got = d.moments()
        hgot = d.mass_history()
    for i in range(3):
        assert np.array_equal(got[i], ref[i]), i
    assert np.array_equal(hgot, href)
    # control: one poisoned slot that is pulled and not rewritten shows up
    st2 = _poison(st, p, storage, seam)
    pitch = (p.nx + 63) // 64 * 64
    plane = pitch * p.ny + 256
    f = st2[32:32 + 9 * plane * np.dtype(DTYPE[storage]).itemsize].view(DTYPE[storage])
    ys, xs = np.nonzero(~p.solid.astype(bool))
    k = len(ys) // 2
    f[2 * plane + ys[k] * pitch + xs[k]] = np.nan  # f*_2 at a fluid node
    with L.Domain(p, storage=storage, history_capacity=64) as d:
        L.lbm_set_state(d.h, st2)
        try:
            d.step(1)
        except L.LbmError as e:
            assert e.code == L.LBM_EUNSTABLE
        assert np.isnan(d.moments()[0]).any()
