"""The C-ABI library: it loads, exports every declared symbol, and rejects
invalid descriptors with the same codes as the oracle (validation happens
before any device call, so these run without a GPU)."""
import ctypes

import numpy as np
import pytest

from lbm_inputs import configs as cfg
from oracle import core as ora
from tests._lib import ensure_built, header_symbols


@pytest.fixture(scope="module")
def L():
    ensure_built()
    from paper_1908_09235_amd import lbm
    return lbm


def test_library_exports_every_declared_symbol(L):
    syms = header_symbols()
    assert len(syms) >= 17
    raw = ctypes.CDLL(L.LIB_PATH)
    for s in syms:
        assert hasattr(raw, s), s
    assert set(syms) == set(L.EXPORTS)


def test_status_strings(L):
    for code in range(-5, 1):
        assert L.lbm_status_string(code)
    assert "unknown" in L.lbm_status_string(-99)


def test_null_arguments_are_rejected(L):
    lib = L.lib()
    h = ctypes.c_void_p()
    assert lib.lbm_create_domain(None, ctypes.byref(h)) == L.LBM_EINVAL
    assert lib.lbm_step(None, 1) == L.LBM_EINVAL
    assert lib.lbm_total_mass(None, None) == L.LBM_EINVAL
    assert lib.lbm_moments(None, None, None, None) == L.LBM_EINVAL
    assert lib.lbm_wall_force(None, None) == L.LBM_EINVAL
    assert lib.lbm_negative_rest(None, None) == L.LBM_EINVAL
    out3 = (ctypes.c_int32 * 3)()
    assert lib.lbm_tune_steps_per_pass(None, 4, out3) == L.LBM_EINVAL
    n = ctypes.c_size_t()
    assert lib.lbm_get_state(None, None, ctypes.byref(n)) == L.LBM_EINVAL
    lib.lbm_destroy(None)


def _bad_problem(bad):
    p = cfg.cfg1("mls", "A")
    lk = p.links.copy()
    if bad == "q0":
        lk["q"][3] = 0.0
        return p.with_(links=lk)
    if bad == "q_gt_1":
        lk["q"][3] = 1.0000001
        return p.with_(links=lk)
    if bad == "missing":
        return p.with_(links=lk[1:])
    if bad == "dup":
        return p.with_(links=np.concatenate([lk, lk[:1]]))
    if bad == "fluid_target":
        lk["dir"][0] = 1 if lk["dir"][0] != 1 else 3
        return p.with_(links=lk)
    if bad == "tau":
        return p.with_(tau=0.5)
    if bad == "fh_pole":
        return p.with_(rule="fh", tau=1.0)
    if bad == "fixb_rule":
        return p.with_(rule="ibb_linear", fix="B")
    if bad == "rho0":
        r = p.rho0.copy()
        r[100, 5] = -1.0
        return p.with_(rho0=r)
    if bad == "cs_psi":
        r = p.rho0.copy()
        r[100, 5] = 0.6
        return p.with_(rho0=r)
    if bad == "moving_ibb":
        lk["uwx"][0] = 0.01
        return p.with_(links=lk, rule="ibb_linear")
    if bad == "mrt_rates":
        return p.with_(collision="mrt", mrt_s=(1.0,) * 7 + (1.5, 1.5))
    if bad == "wall_density":
        rw = p.rho_wall.copy()
        rw[:] = -1.0
        return p.with_(rho_wall=rw)
    if bad == "open_eos":  # open boundaries are single phase only
        return p.with_(open_x=True, inlet_u=0.05)
    c = cfg.cylinder_flow(20.0, d=8.0, nx_d=6.0, ny_d=4.0)
    if bad == "open_speed":
        return c.with_(inlet_u=1.0)
    if bad == "open_nan":
        return c.with_(inlet_u=float("nan"))
    if bad == "open_edge":  # a solid node two columns from the inlet
        from lbm_inputs import geometry as geo
        m = c.meta
        solid, _, links = geo.build(c.nx, c.ny, [geo.Circle(m["cx"], m["cy"], 0.5 * m["d"]),
                                                 geo.Circle(2.0, 5.0, 0.5)])
        return c.with_(solid=solid, links=links)
    raise AssertionError(bad)


BAD = ["q0", "q_gt_1", "missing", "dup", "fluid_target", "tau", "fh_pole",
       "fixb_rule", "rho0", "cs_psi", "moving_ibb", "mrt_rates", "wall_density",
       "open_eos", "open_speed", "open_nan", "open_edge"]


@pytest.mark.parametrize("bad", BAD)
def test_invalid_descriptors_match_oracle_codes(L, bad):
    p = _bad_problem(bad)
    with pytest.raises(ora.OracleError) as eo:
        ora.Oracle(p)
    with pytest.raises(L.LbmError) as eg:
        L.lbm_create_domain(p, storage="f64")
    assert eg.value.code == eo.value.code
    assert eg.value.code in (L.LBM_EINVAL, L.LBM_ESINGULAR)


def test_bad_launch_shape_and_storage_are_rejected(L):
    p = cfg.cfg1()
    for kw in (dict(tile_w=96), dict(tile_h=-1)):
        with pytest.raises(L.LbmError) as e:
            L.lbm_create_domain(p, **kw)
        assert e.value.code == L.LBM_EINVAL
    d, keep = L.make_desc(p)
    h = ctypes.c_void_p()
    for st in (-1, 6, 7):
        d.storage = st
        assert L.lib().lbm_create_domain(ctypes.byref(d), ctypes.byref(h)) == L.LBM_EINVAL
    d.storage = L.STORAGE["f16dev"]
    for rr in (-1.0, float("nan"), float("inf")):
        d.rho_ref = rr
        assert L.lib().lbm_create_domain(ctypes.byref(d), ctypes.byref(h)) == L.LBM_EINVAL
    d.rho_ref = 0.0
    d.storage = 0
    for ox in (-1, 2):
        d.open_x = ox
        assert L.lib().lbm_create_domain(ctypes.byref(d), ctypes.byref(h)) == L.LBM_EINVAL


def test_binding_struct_layout_matches_header(L, tmp_path):
    """The ctypes mirrors of the header's structs have its field
    offsets and sizes (a C program built from the header prints them)."""
    import shutil
    import subprocess
    from pathlib import Path
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = Path(__file__).resolve().parents[1] / "include"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbm2p.h"',
             'int main(void) {']
    structs = (("lbm_desc", L.lbm_desc), ("lbm_link", L.lbm_link),
               ("lbm_batch_desc", L.lbm_batch_desc))
    for st, cls in structs:
        lines.append(f'printf("{st} sizeof %zu\\n", sizeof({st}));')
        for name, _ in cls._fields_:
            lines.append(f'printf("{st} {name} %zu\\n", offsetof({st}, {name}));')
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", str(inc), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        st, name, val = line.split()
        got[(st, name)] = int(val)
    for st, cls in structs:
        assert got[(st, "sizeof")] == ctypes.sizeof(cls), st
        for name, _ in cls._fields_:
            assert got[(st, name)] == getattr(cls, name).offset, (st, name)


def test_batch_descriptors_are_validated(L):
    """lbm_batch_create and lbm_server_create reject bad fields before any
    device call."""
    lib = L.lib()
    h = ctypes.c_void_p()
    good = dict(storage="f32", eos="cs", max_instances=4, arena_bytes=1 << 20)
    for bad in (dict(max_instances=0), dict(tile_w=96), dict(tile_h=4), dict(persistent=2),
                dict(arena_bytes=0)):
        bd = L.make_batch_desc(**{**good, **bad})
        assert lib.lbm_batch_create(ctypes.byref(bd), ctypes.byref(h)) == L.LBM_EINVAL, bad
    for field, val in (("storage", 9), ("eos", 3), ("ring", 1), ("ring", 5)):
        bd = L.make_batch_desc(**good)
        setattr(bd, field, val)
        assert lib.lbm_batch_create(ctypes.byref(bd), ctypes.byref(h)) == L.LBM_EINVAL, field
    bd = L.make_batch_desc(**{**good, "storage": "f16node", "ring": 2})
    assert lib.lbm_batch_create(ctypes.byref(bd), ctypes.byref(h)) == L.LBM_EINVAL
    bd = L.make_batch_desc(**good)
    assert lib.lbm_server_create(ctypes.byref(bd), 0, ctypes.byref(h)) == L.LBM_EINVAL
    assert lib.lbm_batch_create(None, ctypes.byref(h)) == L.LBM_EINVAL
    for fn, args in (("lbm_batch_run", (None, 1)), ("lbm_batch_sync", (None,)),
                     ("lbm_batch_remove", (None, 0)), ("lbm_batch_info", (None, None)),
                     ("lbm_batch_add", (None, None, 1, None)),
                     ("lbm_server_progress", (None, None, 0, None)),
                     ("lbm_server_release", (None, 0)), ("lbm_server_info", (None, None))):
        assert getattr(lib, fn)(*args) == L.LBM_EINVAL, fn


@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev", "f16node"])
def test_state_buffer_limit_is_enforced_at_create(L, storage):
    """One row past the largest domain whose state buffer fits in 32-bit
    offsets is rejected before any array is read (so a small problem's
    arrays can stand in); so is nx * ny >= 2^30."""
    from tests._limits import max_rows
    p = cfg.cfg1()
    d, keep = L.make_desc(p, storage=storage)
    h = ctypes.c_void_p()
    nx = 16384
    d.nx, d.ny = nx, max_rows(storage, nx) + 1
    assert L.lib().lbm_create_domain(ctypes.byref(d), ctypes.byref(h)) == L.LBM_EINVAL
    d.nx, d.ny = 1 << 15, 1 << 15
    assert L.lib().lbm_create_domain(ctypes.byref(d), ctypes.byref(h)) == L.LBM_EINVAL
