"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Steps, equations and readings are documented in lbm_oracle.c.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import build as _build

RULE = {"halfway": 0, "fh": 1, "mls": 2, "ibb_linear": 3,
        "ibb_quadratic": 4, "zhao_yong": 5}
FIX = {"none": 0, "A": 1, "B": 2, "bao": 3}
EOS = {"none": 0, "exp": 1, "cs": 2}
COLL = {"bgk": 0, "mrt": 1}

_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int32)


class _Desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("solid", C.POINTER(C.c_uint8)), ("nlinks", C.c_int64),
                ("link_x", _I), ("link_y", _I), ("link_dir", _I),
                ("link_q", _D), ("link_uwx", _D), ("link_uwy", _D),
                ("rho_wall", _D), ("eos", C.c_int32),
                ("eos_p", C.c_double * 4), ("G", C.c_double),
                ("gx", C.c_double), ("gy", C.c_double),
                ("collision", C.c_int32), ("tau", C.c_double),
                ("mrt_s", C.c_double * 9), ("rule", C.c_int32),
                ("fix", C.c_int32), ("rho0", _D), ("ux0", _D), ("uy0", _D),
                ("open_x", C.c_int32), ("inlet_u", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(_build.ensure())
        L.ora_create.argtypes = [C.POINTER(_Desc), C.POINTER(C.c_void_p)]
        L.ora_create.restype = C.c_int
        L.ora_destroy.argtypes = [C.c_void_p]
        L.ora_step.argtypes = [C.c_void_p, C.c_int64, _D]
        L.ora_step.restype = C.c_int
        L.ora_moments.argtypes = [C.c_void_p, _D, _D, _D]
        L.ora_total_mass.argtypes = [C.c_void_p]
        L.ora_total_mass.restype = C.c_double
        L.ora_time.argtypes = [C.c_void_p]
        L.ora_time.restype = C.c_int64
        L.ora_get_f.argtypes = [C.c_void_p, _D]
        L.ora_set_f.argtypes = [C.c_void_p, _D]
        L.ora_last_leaks.argtypes = [C.c_void_p, _D, C.c_int64]
        L.ora_last_leaks.restype = C.c_int64
        L.ora_counters.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        L.ora_wall_force.argtypes = [C.c_void_p, _D]
        L.ora_feq.argtypes = [C.c_double] * 3 + [_D]
        L.ora_guo.argtypes = [C.c_double] * 5 + [_D]
        L.ora_mrt_matrix.argtypes = [_D, _D]
        L.ora_collide.argtypes = [C.c_int32, C.c_double, _D, _D] + [C.c_double] * 5 + [_D]
        L.ora_psi.argtypes = [C.c_int32, _D, C.c_double, C.c_double]
        L.ora_psi.restype = C.c_double
        L.ora_pressure_eos.argtypes = [C.c_int32, _D, C.c_double]
        L.ora_pressure_eos.restype = C.c_double
        L.ora_rule_incoming.argtypes = [C.c_int32, C.c_int32, C.c_double,
                                        C.c_double, _D, C.c_double, _D, _D]
        L.ora_rule_incoming.restype = C.c_double
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D) if a is not None else None


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}")
        self.code = code


class Oracle:
    """One simulation held by the C oracle; arrays are [y, x] numpy arrays."""

    def __init__(self, p):
        L = lib()
        self.p = p
        self.nx, self.ny = p.nx, p.ny
        lk = p.links
        keep = {}
        keep["solid"] = np.ascontiguousarray(p.solid, dtype=np.uint8)
        keep["lx"] = np.ascontiguousarray(lk["x"], dtype=np.int32)
        keep["ly"] = np.ascontiguousarray(lk["y"], dtype=np.int32)
        keep["ld"] = np.ascontiguousarray(lk["dir"], dtype=np.int32)
        keep["lq"] = np.ascontiguousarray(lk["q"], dtype=np.float64)
        keep["luwx"] = np.ascontiguousarray(lk["uwx"], dtype=np.float64)
        keep["luwy"] = np.ascontiguousarray(lk["uwy"], dtype=np.float64)
        keep["rw"] = np.ascontiguousarray(p.rho_wall, dtype=np.float64)
        keep["rho0"] = np.ascontiguousarray(p.rho0, dtype=np.float64)
        keep["ux0"] = None if p.ux0 is None else np.ascontiguousarray(p.ux0, dtype=np.float64)
        keep["uy0"] = None if p.uy0 is None else np.ascontiguousarray(p.uy0, dtype=np.float64)
        d = _Desc()
        d.nx, d.ny = p.nx, p.ny
        d.solid = keep["solid"].ctypes.data_as(C.POINTER(C.c_uint8))
        d.nlinks = len(lk)
        d.link_x = keep["lx"].ctypes.data_as(_I)
        d.link_y = keep["ly"].ctypes.data_as(_I)
        d.link_dir = keep["ld"].ctypes.data_as(_I)
        d.link_q = _dp(keep["lq"])
        d.link_uwx = _dp(keep["luwx"])
        d.link_uwy = _dp(keep["luwy"])
        d.rho_wall = _dp(keep["rw"])
        d.eos = EOS[p.eos]
        d.eos_p = (C.c_double * 4)(*p.eos_params)
        d.G = p.G
        d.gx, d.gy = p.gravity
        d.collision = COLL[p.collision]
        d.tau = p.tau
        d.mrt_s = (C.c_double * 9)(*p.mrt_s)
        d.rule = RULE[p.rule]
        d.fix = FIX[p.fix]
        d.rho0 = _dp(keep["rho0"])
        d.ux0 = _dp(keep["ux0"])
        d.uy0 = _dp(keep["uy0"])
        d.open_x = 1 if getattr(p, "open_x", False) else 0
        d.inlet_u = float(getattr(p, "inlet_u", 0.0))
        h = C.c_void_p()
        rc = L.ora_create(C.byref(d), C.byref(h))
        if rc != 0:
            raise OracleError(rc)
        self._h = h
        self._L = L

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._L.ora_destroy(h)
            self._h = None

    def wall_force(self):
        """Force on the walls during the last step (momentum exchange)."""
        out = np.zeros(2)
        self._L.ora_wall_force(self._h, _dp(out))
        return out

    def step(self, n: int) -> np.ndarray:
        hist = np.zeros(max(n, 1))
        rc = self._L.ora_step(self._h, n, _dp(hist))
        if rc != 0:
            raise OracleError(rc)
        return hist[:n]

    def moments(self):
        shape = (self.ny, self.nx)
        r, ux, uy = np.zeros(shape), np.zeros(shape), np.zeros(shape)
        rc = self._L.ora_moments(self._h, _dp(r), _dp(ux), _dp(uy))
        if rc != 0:
            raise OracleError(rc)
        return r, ux, uy

    def total_mass(self) -> float:
        return self._L.ora_total_mass(self._h)

    @property
    def t(self) -> int:
        return self._L.ora_time(self._h)

    def get_f(self) -> np.ndarray:
        f = np.zeros((9, self.ny, self.nx))
        self._L.ora_get_f(self._h, _dp(f))
        return f

    def set_f(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        self._L.ora_set_f(self._h, _dp(f))

    def last_leaks(self) -> np.ndarray:
        n = len(self.p.links) + 1
        out = np.zeros(n)
        nb = self._L.ora_last_leaks(self._h, _dp(out), n)
        return out[:nb]

    def counters(self) -> np.ndarray:
        out = (C.c_int64 * 5)()
        self._L.ora_counters(self._h, out)
        return np.array(list(out))


# ---- pure functions ----------------------------------------------------
def feq(rho, ux, uy) -> np.ndarray:
    out = np.zeros(9)
    lib().ora_feq(rho, ux, uy, _dp(out))
    return out


def guo(tau, ux, uy, Fx, Fy) -> np.ndarray:
    out = np.zeros(9)
    lib().ora_guo(tau, ux, uy, Fx, Fy, _dp(out))
    return out


def mrt_matrix():
    M, Mi = np.zeros(81), np.zeros(81)
    lib().ora_mrt_matrix(_dp(M), _dp(Mi))
    return M.reshape(9, 9), Mi.reshape(9, 9)


def collide(collision, tau, s, f, rho, ux, uy, Fx, Fy) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(9)
    lib().ora_collide(COLL[collision], tau, _dp(s), _dp(f), rho, ux, uy, Fx,
                      Fy, _dp(out))
    return out


def psi(eos, params, G, rho) -> float:
    p = np.ascontiguousarray(params, dtype=np.float64)
    return lib().ora_psi(EOS[eos], _dp(p), G, rho)


def pressure_eos(eos, params, rho) -> float:
    p = np.ascontiguousarray(params, dtype=np.float64)
    return lib().ora_pressure_eos(EOS[eos], _dp(p), rho)


LINK_INPUTS = ("fa_b", "fab_b", "fa_f", "fab_f", "fa_ff", "fpre_a", "rho_b",
               "ubx", "uby", "ufx", "ufy", "uwx", "uwy", "f_ok", "ff_ok")


def rule_incoming(rule, dir, q, tau, rho_eq=None, **kw):
    """Incoming population of one cut link; keyword inputs as LINK_INPUTS."""
    v = np.array([float(kw.get(k, 1.0 if k in ("f_ok", "ff_ok") else 0.0))
                  for k in LINK_INPUTS])
    chi, br = C.c_double(), C.c_double()
    r = lib().ora_rule_incoming(RULE[rule], dir, q, tau, _dp(v),
                                v[6] if rho_eq is None else rho_eq,
                                C.cast(C.byref(chi), _D), C.cast(C.byref(br), _D))
    return r, chi.value, br.value
