"""ctypes binding of the lbm2p C ABI (include/lbm2p.h).

Functions carry the C names and only marshal arguments: every step of the
method runs in the HIP kernels of liblbm2p.so.  Loading fails loudly if the
library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBM2P_LIB", os.path.join(HERE, "liblbm2p.so"))

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ESINGULAR, LBM_EUNSTABLE = 0, -1, -2, -3, -4, -5
RULE = {"halfway": 0, "fh": 1, "mls": 2, "ibb_linear": 3, "ibb_quadratic": 4,
        "zhao_yong": 5}
FIX = {"none": 0, "A": 1, "B": 2, "bao": 3}
EOS = {"none": 0, "exp": 1, "cs": 2}
COLL = {"bgk": 0, "mrt": 1}
STORAGE = {"f64": 0, "f32": 1, "f32_arith32": 2, "f32dev": 3, "f16dev": 4, "f16node": 5}

LINK_NP = np.dtype([("x", "<i4"), ("y", "<i4"), ("dir", "<i4"),
                    ("reserved", "<i4"), ("q", "<f8"), ("uwx", "<f8"),
                    ("uwy", "<f8")])


class lbm_link(C.Structure):
    _fields_ = [("x", C.c_int32), ("y", C.c_int32), ("dir", C.c_int32),
                ("reserved", C.c_int32), ("q", C.c_double),
                ("uw", C.c_double * 2)]


class lbm_desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("solid", C.POINTER(C.c_uint8)),
                ("links", C.POINTER(lbm_link)), ("nlinks", C.c_int64),
                ("rho_wall", C.POINTER(C.c_double)),
                ("rho_wall_const", C.c_double),
                ("eos", C.c_int32), ("collision", C.c_int32),
                ("eos_param", C.c_double * 4), ("G", C.c_double),
                ("gravity", C.c_double * 2), ("tau", C.c_double),
                ("mrt_s", C.c_double * 9), ("rule", C.c_int32),
                ("fix", C.c_int32), ("storage", C.c_int32),
                ("open_x", C.c_int32),
                ("rho0", C.POINTER(C.c_double)),
                ("ux0", C.POINTER(C.c_double)),
                ("uy0", C.POINTER(C.c_double)),
                ("history_capacity", C.c_int64), ("stream", C.c_void_p),
                ("tile_w", C.c_int32), ("tile_h", C.c_int32),
                ("rho_ref", C.c_double), ("inlet_u", C.c_double)]


class lbm_batch_desc(C.Structure):
    _fields_ = [("storage", C.c_int32), ("eos", C.c_int32),
                ("max_instances", C.c_int32), ("tile_w", C.c_int32),
                ("tile_h", C.c_int32), ("persistent", C.c_int32),
                ("graph_steps", C.c_int32), ("ring", C.c_int32),
                ("arena_bytes", C.c_int64), ("stream", C.c_void_p)]


assert C.sizeof(lbm_link) == 40 and LINK_NP.itemsize == 40

_D = C.POINTER(C.c_double)
_H = C.c_void_p
_lib = None

EXPORTS = {
    "lbm_create_domain": (C.c_int, [C.POINTER(lbm_desc), C.POINTER(_H)]),
    "lbm_step": (C.c_int, [_H, C.c_int64]),
    "lbm_step_async": (C.c_int, [_H, C.c_int64]),
    "lbm_sync": (C.c_int, [_H]),
    "lbm_moments": (C.c_int, [_H, _D, _D, _D]),
    "lbm_moments_device": (C.c_int, [_H, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lbm_moments_device_noalloc": (C.c_int, [_H, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lbm_total_mass": (C.c_int, [_H, _D]),
    "lbm_time": (C.c_int, [_H, C.POINTER(C.c_int64)]),
    "lbm_wall_force": (C.c_int, [_H, _D]),
    "lbm_mass_history": (C.c_int, [_H, _D, C.c_int64, C.POINTER(C.c_int64)]),
    "lbm_unstable_step": (C.c_int, [_H, C.POINTER(C.c_int64)]),
    "lbm_get_state": (C.c_int, [_H, C.c_void_p, C.POINTER(C.c_size_t)]),
    "lbm_set_state": (C.c_int, [_H, C.c_void_p, C.c_size_t]),
    "lbm_set_profiling": (C.c_int, [_H, C.c_int]),
    "lbm_kernel_times": (C.c_int, [_H, _D, C.POINTER(C.c_int64), _D,
                                   C.POINTER(C.c_int64)]),
    "lbm_info": (C.c_int, [_H, C.POINTER(C.c_int64)]),
    "lbm_set_steps_per_pass": (C.c_int, [_H, C.c_int32, C.c_int32]),
    "lbm_get_steps_per_pass": (C.c_int, [_H, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "lbm_tune_steps_per_pass": (C.c_int, [_H, C.c_int64, C.POINTER(C.c_int32)]),
    "lbm_negative_rest": (C.c_int, [_H, C.POINTER(C.c_int64)]),
    "lbm_degenerate_b": (C.c_int, [_H, C.POINTER(C.c_int64)]),
    "lbm_destroy": (None, [_H]),
    "lbm_status_string": (C.c_char_p, [C.c_int]),
    "lbm_batch_create": (C.c_int, [C.POINTER(lbm_batch_desc), C.POINTER(_H)]),
    "lbm_batch_add": (C.c_int, [_H, C.POINTER(lbm_desc), C.c_int64, C.POINTER(C.c_int32)]),
    "lbm_batch_run": (C.c_int, [_H, C.c_int64]),
    "lbm_batch_sync": (C.c_int, [_H]),
    "lbm_batch_status": (C.c_int, [_H, C.c_int32, C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "lbm_batch_moments": (C.c_int, [_H, C.c_int32, _D, _D, _D]),
    "lbm_batch_mass_history": (C.c_int, [_H, C.c_int32, _D, C.c_int64,
                                         C.POINTER(C.c_int64)]),
    "lbm_batch_remove": (C.c_int, [_H, C.c_int32]),
    "lbm_batch_tune": (C.c_int, [_H, C.c_int64, C.POINTER(C.c_int32)]),
    "lbm_batch_info": (C.c_int, [_H, C.POINTER(C.c_int64)]),
    "lbm_batch_destroy": (None, [_H]),
    "lbm_server_create": (C.c_int, [C.POINTER(lbm_batch_desc), C.c_int64, C.POINTER(_H)]),
    "lbm_server_submit": (C.c_int, [_H, C.POINTER(lbm_desc), C.c_int64,
                                    C.POINTER(C.c_int64)]),
    "lbm_server_progress": (C.c_int, [_H, C.POINTER(C.c_int64), C.c_int64,
                                      C.POINTER(C.c_int64)]),
    "lbm_server_result": (C.c_int, [_H, C.c_int64, _D, _D, _D, _D, C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int64)]),
    "lbm_server_release": (C.c_int, [_H, C.c_int64]),
    "lbm_server_info": (C.c_int, [_H, C.POINTER(C.c_int64)]),
    "lbm_server_destroy": (None, [_H]),
}


class LbmError(RuntimeError):
    def __init__(self, code, what=""):
        msg = lib().lbm_status_string(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})")
        self.code = code


def lib():
    """Load liblbm2p.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_1908_09235_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc, what):
    if rc != LBM_OK:
        raise LbmError(rc, what)


def _dptr(a):
    return None if a is None else a.ctypes.data_as(_D)


def make_desc(problem, storage="f64", tile_w=0, tile_h=0, stream=None,
              history_capacity=0, rho_ref=0.0):
    """Marshal a problem description into an lbm_desc.

    Returns (desc, keepalive); the arrays in keepalive must outlive the
    lbm_create_domain call."""
    p = problem
    keep = {}
    keep["solid"] = np.ascontiguousarray(p.solid, dtype=np.uint8).ravel()
    lk = np.zeros(len(p.links), dtype=LINK_NP)
    for f in ("x", "y", "dir", "q", "uwx", "uwy"):
        lk[f] = p.links[f]
    keep["links"] = lk
    keep["rho_wall"] = np.ascontiguousarray(p.rho_wall, dtype=np.float64).ravel()
    keep["rho0"] = np.ascontiguousarray(p.rho0, dtype=np.float64).ravel()
    keep["ux0"] = None if p.ux0 is None else np.ascontiguousarray(p.ux0, np.float64).ravel()
    keep["uy0"] = None if p.uy0 is None else np.ascontiguousarray(p.uy0, np.float64).ravel()
    d = lbm_desc()
    d.nx, d.ny = p.nx, p.ny
    d.solid = keep["solid"].ctypes.data_as(C.POINTER(C.c_uint8))
    d.links = lk.ctypes.data_as(C.POINTER(lbm_link))
    d.nlinks = len(lk)
    d.rho_wall = _dptr(keep["rho_wall"])
    d.rho_wall_const = 0.0
    d.eos = EOS[p.eos]
    d.collision = COLL[p.collision]
    d.eos_param = (C.c_double * 4)(*p.eos_params)
    d.G = p.G
    d.gravity = (C.c_double * 2)(*p.gravity)
    d.tau = p.tau
    d.mrt_s = (C.c_double * 9)(*p.mrt_s)
    d.rule = RULE[p.rule]
    d.fix = FIX[p.fix]
    d.storage = STORAGE[storage]
    d.open_x = 1 if getattr(p, "open_x", False) else 0
    d.inlet_u = float(getattr(p, "inlet_u", 0.0))
    d.rho0 = _dptr(keep["rho0"])
    d.ux0 = _dptr(keep["ux0"])
    d.uy0 = _dptr(keep["uy0"])
    d.history_capacity = history_capacity
    d.stream = stream
    d.tile_w, d.tile_h = tile_w, tile_h
    d.rho_ref = rho_ref
    return d, keep


def lbm_create_domain(problem, storage="f64", tile_w=0, tile_h=0, stream=None,
                      history_capacity=0, rho_ref=0.0):
    d, keep = make_desc(problem, storage, tile_w, tile_h, stream, history_capacity,
                        rho_ref)
    h = _H()
    _check(lib().lbm_create_domain(C.byref(d), C.byref(h)), "lbm_create_domain")
    del keep
    return h


def lbm_step(h, n):
    _check(lib().lbm_step(h, int(n)), "lbm_step")


def lbm_step_async(h, n):
    _check(lib().lbm_step_async(h, int(n)), "lbm_step_async")


def lbm_sync(h):
    _check(lib().lbm_sync(h), "lbm_sync")


def lbm_moments(h, nx, ny):
    r, ux, uy = (np.zeros((ny, nx)) for _ in range(3))
    _check(lib().lbm_moments(h, _dptr(r), _dptr(ux), _dptr(uy)), "lbm_moments")
    return r, ux, uy


def lbm_moments_device(h, rho_ptr, ux_ptr, uy_ptr):
    _check(lib().lbm_moments_device(h, rho_ptr, ux_ptr, uy_ptr), "lbm_moments_device")


def lbm_moments_device_noalloc(h, rho_ptr, ux_ptr, uy_ptr):
    _check(lib().lbm_moments_device_noalloc(h, rho_ptr, ux_ptr, uy_ptr),
           "lbm_moments_device_noalloc")


def lbm_total_mass(h):
    m = C.c_double()
    _check(lib().lbm_total_mass(h, C.byref(m)), "lbm_total_mass")
    return m.value


def lbm_time(h):
    t = C.c_int64()
    _check(lib().lbm_time(h, C.byref(t)), "lbm_time")
    return t.value


def lbm_mass_history(h, cap):
    out = np.zeros(max(int(cap), 1))
    n = C.c_int64()
    _check(lib().lbm_mass_history(h, _dptr(out), int(cap), C.byref(n)), "lbm_mass_history")
    return out[:n.value]


def lbm_unstable_step(h):
    s = C.c_int64()
    _check(lib().lbm_unstable_step(h, C.byref(s)), "lbm_unstable_step")
    return s.value


def lbm_get_state(h):
    n = C.c_size_t()
    _check(lib().lbm_get_state(h, None, C.byref(n)), "lbm_get_state")
    buf = np.zeros(n.value, dtype=np.uint8)
    _check(lib().lbm_get_state(h, buf.ctypes.data_as(C.c_void_p), C.byref(n)), "lbm_get_state")
    return buf


def lbm_set_state(h, buf):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    _check(lib().lbm_set_state(h, buf.ctypes.data_as(C.c_void_p), buf.nbytes), "lbm_set_state")


def lbm_set_profiling(h, every):
    """Time the launches of every `every`-th step with HIP events (0: off)."""
    _check(lib().lbm_set_profiling(h, int(every)), "lbm_set_profiling")


def lbm_kernel_times(h):
    mm, bm = C.c_double(), C.c_double()
    mn, bn = C.c_int64(), C.c_int64()
    _check(lib().lbm_kernel_times(h, C.byref(mm), C.byref(mn), C.byref(bm), C.byref(bn)),
           "lbm_kernel_times")
    return mm.value, mn.value, bm.value, bn.value


def lbm_negative_rest(h):
    n = C.c_int64()
    _check(lib().lbm_negative_rest(h, C.byref(n)), "lbm_negative_rest")
    return n.value


def lbm_degenerate_b(h):
    n = C.c_int64()
    _check(lib().lbm_degenerate_b(h, C.byref(n)), "lbm_degenerate_b")
    return n.value


def lbm_info(h):
    out = (C.c_int64 * 8)()
    _check(lib().lbm_info(h, out), "lbm_info")
    keys = ("fluid_nodes", "links", "boundary_nodes", "device_bytes", "tile_w",
            "tile_h", "main_workgroups", "fallbacks")
    return dict(zip(keys, list(out)))


def lbm_destroy(h):
    lib().lbm_destroy(h)


def lbm_wall_force(h):
    """Force on the walls during the last step (momentum exchange)."""
    out = np.zeros(2)
    _check(lib().lbm_wall_force(h, out.ctypes.data_as(_D)), "lbm_wall_force")
    return out


def lbm_set_steps_per_pass(h, steps, tile_h=0):
    _check(lib().lbm_set_steps_per_pass(h, int(steps), int(tile_h)), "lbm_set_steps_per_pass")


def lbm_get_steps_per_pass(h):
    s, t = C.c_int32(), C.c_int32()
    _check(lib().lbm_get_steps_per_pass(h, C.byref(s), C.byref(t)), "lbm_get_steps_per_pass")
    return s.value, t.value


def lbm_tune_steps_per_pass(h, steps_per_trial):
    """Times one and two steps per pass (tiles of 4..24 rows) on real steps
    and keeps the fastest; returns {steps_per_pass, tile_h, us_per_step}."""
    out = (C.c_int32 * 3)()
    _check(lib().lbm_tune_steps_per_pass(h, int(steps_per_trial), out), "lbm_tune_steps_per_pass")
    return {"steps_per_pass": out[0], "tile_h": out[1], "us_per_step": out[2]}


def lbm_status_string(code):
    return lib().lbm_status_string(code).decode()


class Domain:
    """Owning wrapper around an lbm_domain handle."""

    def __init__(self, problem, storage="f64", **kw):
        self.nx, self.ny = problem.nx, problem.ny
        self.h = lbm_create_domain(problem, storage=storage, **kw)

    def step(self, n):
        lbm_step(self.h, n)

    def moments(self):
        return lbm_moments(self.h, self.nx, self.ny)

    def total_mass(self):
        return lbm_total_mass(self.h)

    def wall_force(self):
        return lbm_wall_force(self.h)

    def mass_history(self, cap=None):
        return lbm_mass_history(self.h, cap if cap is not None else lbm_time(self.h) + 1)

    @property
    def t(self):
        return lbm_time(self.h)

    def info(self):
        return lbm_info(self.h)

    def negative_rest(self):
        return lbm_negative_rest(self.h)

    def degenerate_b(self):
        return lbm_degenerate_b(self.h)

    def tune_steps_per_pass(self, steps_per_trial=100):
        return lbm_tune_steps_per_pass(self.h, steps_per_trial)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lbm_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- batches
def make_batch_desc(storage="f32", eos="cs", max_instances=1024, tile_w=0, tile_h=0,
                    persistent=1, graph_steps=0, arena_bytes=1 << 30, stream=None, ring=0):
    bd = lbm_batch_desc()
    bd.storage = STORAGE[storage]
    bd.eos = EOS[eos]
    bd.max_instances = max_instances
    bd.tile_w, bd.tile_h = tile_w, tile_h
    bd.persistent = persistent
    bd.graph_steps = graph_steps
    bd.ring = ring
    bd.arena_bytes = int(arena_bytes)
    bd.stream = stream
    return bd


def lbm_batch_create(**kw):
    bd = make_batch_desc(**kw)
    h = _H()
    _check(lib().lbm_batch_create(C.byref(bd), C.byref(h)), "lbm_batch_create")
    return h


def lbm_batch_add(h, problem, steps, storage="f32", history_capacity=0, rho_ref=0.0):
    d, keep = make_desc(problem, storage, 0, 0, None, history_capacity, rho_ref)
    slot = C.c_int32()
    _check(lib().lbm_batch_add(h, C.byref(d), int(steps), C.byref(slot)), "lbm_batch_add")
    del keep
    return slot.value


def lbm_batch_run(h, n):
    _check(lib().lbm_batch_run(h, int(n)), "lbm_batch_run")


def lbm_batch_sync(h):
    _check(lib().lbm_batch_sync(h), "lbm_batch_sync")


def lbm_batch_status(h, slot):
    t, r, u = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().lbm_batch_status(h, int(slot), C.byref(t), C.byref(r), C.byref(u)),
           "lbm_batch_status")
    return t.value, r.value, u.value


def lbm_batch_moments(h, slot, nx, ny):
    r, ux, uy = (np.zeros((ny, nx)) for _ in range(3))
    _check(lib().lbm_batch_moments(h, int(slot), _dptr(r), _dptr(ux), _dptr(uy)),
           "lbm_batch_moments")
    return r, ux, uy


def lbm_batch_mass_history(h, slot, cap):
    out = np.zeros(max(int(cap), 1))
    n = C.c_int64()
    _check(lib().lbm_batch_mass_history(h, int(slot), _dptr(out), int(cap), C.byref(n)),
           "lbm_batch_mass_history")
    return out[:n.value]


def lbm_batch_remove(h, slot):
    _check(lib().lbm_batch_remove(h, int(slot)), "lbm_batch_remove")


def lbm_batch_tune(h, steps_per_trial):
    out = (C.c_int32 * 5)()
    _check(lib().lbm_batch_tune(h, int(steps_per_trial), out), "lbm_batch_tune")
    return {"tile_w": out[0], "tile_h": out[1], "persistent": out[2], "us_per_step": out[3],
            "ring": out[4]}


def lbm_batch_info(h):
    out = (C.c_int64 * 8)()
    _check(lib().lbm_batch_info(h, out), "lbm_batch_info")
    keys = ("instances", "tiles", "link_blocks", "arena_bytes", "arena_used", "tile_w",
            "tile_h", "persistent")
    return dict(zip(keys, list(out)))


def lbm_batch_destroy(h):
    lib().lbm_batch_destroy(h)


class Batch:
    """Owning wrapper around an lbm_batch handle."""

    def __init__(self, storage="f32", eos="cs", **kw):
        self.storage = storage
        self.h = lbm_batch_create(storage=storage, eos=eos, **kw)
        self.shape = {}

    def add(self, problem, steps, history_capacity=0, rho_ref=0.0):
        s = lbm_batch_add(self.h, problem, steps, self.storage, history_capacity, rho_ref)
        self.shape[s] = (problem.nx, problem.ny)
        return s

    def run(self, n):
        lbm_batch_run(self.h, n)

    def sync(self):
        lbm_batch_sync(self.h)

    def status(self, slot):
        return lbm_batch_status(self.h, slot)

    def moments(self, slot):
        nx, ny = self.shape[slot]
        return lbm_batch_moments(self.h, slot, nx, ny)

    def mass_history(self, slot):
        t = self.status(slot)[0]
        return lbm_batch_mass_history(self.h, slot, t + 1)

    def remove(self, slot):
        lbm_batch_remove(self.h, slot)
        self.shape.pop(slot, None)

    def tune(self, steps_per_trial):
        return lbm_batch_tune(self.h, steps_per_trial)

    def info(self):
        return lbm_batch_info(self.h)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lbm_batch_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- server
def lbm_server_create(chunk_steps, **kw):
    bd = make_batch_desc(**kw)
    h = _H()
    _check(lib().lbm_server_create(C.byref(bd), int(chunk_steps), C.byref(h)),
           "lbm_server_create")
    return h


def lbm_server_submit(h, desc, steps):
    i = C.c_int64()
    _check(lib().lbm_server_submit(h, C.byref(desc), int(steps), C.byref(i)),
           "lbm_server_submit")
    return i.value


def lbm_server_progress(h, cap=4096):
    ids = (C.c_int64 * max(int(cap), 1))()
    n = C.c_int64()
    _check(lib().lbm_server_progress(h, ids, int(cap), C.byref(n)), "lbm_server_progress")
    return list(ids[:n.value])


def lbm_server_result(h, rid, nx=None, ny=None, fields=True):
    m = (C.c_double * 2)()
    steps, u = C.c_int64(), C.c_int64()
    if fields:
        r, ux, uy = (np.zeros((ny, nx)) for _ in range(3))
        ptrs = (_dptr(r), _dptr(ux), _dptr(uy))
    else:
        r = ux = uy = None
        ptrs = (None, None, None)
    _check(lib().lbm_server_result(h, int(rid), *ptrs, m, C.byref(steps), C.byref(u)),
           "lbm_server_result")
    return {"rho": r, "ux": ux, "uy": uy, "mass0": m[0], "mass": m[1],
            "steps": steps.value, "unstable_step": u.value}


def lbm_server_release(h, rid):
    _check(lib().lbm_server_release(h, int(rid)), "lbm_server_release")


def lbm_server_info(h):
    out = (C.c_int64 * 8)()
    _check(lib().lbm_server_info(h, out), "lbm_server_info")
    keys = ("queued", "running", "finished", "arena_used", "arena_bytes", "chunks",
            "admitted", "rejected")
    return dict(zip(keys, list(out)))


def lbm_server_destroy(h):
    lib().lbm_server_destroy(h)


class Server:
    """Owning wrapper around an lbm_server handle.  Submitted problems are
    kept alive here until they are admitted."""

    def __init__(self, chunk_steps=64, storage="f32", eos="cs", **kw):
        self.storage = storage
        self.h = lbm_server_create(chunk_steps, storage=storage, eos=eos, **kw)
        self.keep = {}
        self.shape = {}

    def submit(self, problem, steps, history_capacity=0, rho_ref=0.0):
        d, keep = make_desc(problem, self.storage, 0, 0, None, history_capacity, rho_ref)
        rid = lbm_server_submit(self.h, d, steps)
        self.keep[rid] = (d, keep)
        self.shape[rid] = (problem.nx, problem.ny)
        return rid

    def progress(self, cap=4096):
        done = lbm_server_progress(self.h, cap)
        # requests leave the queue in id order: the first admitted + rejected
        # ids no longer need their arrays
        info = self.info()
        gone = info["admitted"] + info["rejected"]
        for rid in [r for r in self.keep if r < gone]:
            del self.keep[rid]
        return done

    def result(self, rid, fields=True):
        nx, ny = self.shape[rid]
        return lbm_server_result(self.h, rid, nx, ny, fields)

    def release(self, rid):
        lbm_server_release(self.h, rid)
        self.shape.pop(rid, None)

    def info(self):
        return lbm_server_info(self.h)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lbm_server_destroy(self.h)
            self.h = None
        self.keep = {}

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
