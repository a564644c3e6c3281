"""lbm_moments_device_noalloc against lbm_moments_device through the C ABI:
the same fields bit for bit, on two calls in a row (the second on a
smaller domain), with some outputs omitted, and the size limit refused.
Device buffers come from the library's own HIP runtime."""
import sys

import numpy as np
import pytest

from lbm_inputs import configs as cfg

from _hip import DeviceArray, hip

pytestmark = pytest.mark.gpu

LIMIT_NODES = 1 << 21


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lbm():
    from paper_1908_09235_amd import lbm
    lbm.lib()
    hip()
    return lbm


def _read(fn, d, n, keep=(True, True, True)):
    bufs = [DeviceArray(np.full(n, np.nan)) if k else None for k in keep]
    try:
        rc = fn(d.h, *[b.ptr if b is not None else None for b in bufs])
        return rc, [b.get() if b is not None else None for b in bufs]
    finally:
        for b in bufs:
            if b is not None:
                b.free()


def test_noalloc_moments_match_the_allocating_read_out(lbm):
    raw = lbm.lib()
    big = cfg.cfg1("mls", "B")                       # 128 x 128
    small = cfg.static_gravity(0.3, rule="mls", fix="A", nx=60, ny=30)
    with lbm.Domain(big, storage="f64") as a, lbm.Domain(small, storage="f32") as b:
        a.step(50)
        b.step(20)
        for d, p, name in ((a, big, "cfg1 128x128 f64"), (b, small, "gravity 60x30 f32")):
            n = p.nx * p.ny
            say(f"[gpu] noalloc moments vs lbm_moments_device: {name}")
            rc0, want = _read(raw.lbm_moments_device, d, n)
            rc1, got = _read(raw.lbm_moments_device_noalloc, d, n)
            assert rc0 == lbm.LBM_OK and rc1 == lbm.LBM_OK
            for g, w in zip(got, want):
                assert np.array_equal(g, w)
            for g, h in zip(got, d.moments()):
                assert np.array_equal(g.reshape(p.ny, p.nx), h)
        # the smaller domain again with only u_y requested
        say("[gpu] noalloc moments, u_y only")
        n = small.nx * small.ny
        rc, got = _read(raw.lbm_moments_device_noalloc, b, n, (False, False, True))
        assert rc == lbm.LBM_OK
        assert np.array_equal(got[2].reshape(small.ny, small.nx), b.moments()[2])


def test_noalloc_moments_refuse_domains_beyond_the_buffer(lbm):
    nx, ny = 2048, LIMIT_NODES // 2048 + 1
    say(f"[gpu] noalloc moments refuse {nx}x{ny} ({nx * ny} nodes > {LIMIT_NODES})")
    p = cfg.shear_wave(ny, nx=nx)
    with lbm.Domain(p, storage="f32") as d:
        out = DeviceArray(np.zeros(nx * ny))
        try:
            rc = lbm.lib().lbm_moments_device_noalloc(d.h, out.ptr, None, None)
            assert rc == lbm.LBM_EINVAL
            assert float(np.abs(out.get()).max()) == 0.0
        finally:
            out.free()
