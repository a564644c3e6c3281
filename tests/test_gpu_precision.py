"""Reduced-precision forms: populations stored as FP32 or FP16 deviations
g = f - w rho_ref from the lattice weights (or, f16node, g = f - w r(x)
with r(x) the density of the node holding the slot), with FP32 arithmetic;
the boundary sums and the total mass stay FP64.  The paper computes in double
precision and fixes no tolerance for these forms, so each test states the
error it measures against the FP64 oracle (droplet on a cylinder, 128^2) or
against the FP64 GPU form (many cylinders, CS at 0.86 Tc, BGK tau = 0.8,
MLS + scheme B) and bounds it."""
import sys

import numpy as np
import pytest

from lbm_inputs import configs as cfg
from oracle import core as ora
from tests._lib import rel_err

pytestmark = pytest.mark.gpu

# bounds on the max-norm relative error of rho and of ux, uy (fluid nodes).
# FP16 keeps 11 significant bits.  Against one reference density the stored
# deviations reach 0.2 w_a while the velocities here are 1e-3 or less, so
# that form's velocity field is only a rough copy; against each node's own
# density (f16node) what is stored is O(w rho u) and the error drops 20-100x.
BOUND_RHO = {"f32": 1e-5, "f32_arith32": 1e-5, "f32dev": 1e-5, "f16dev": 2.5e-2,
             "f16node": 1e-3}
BOUND_U = {"f32": 1e-5, "f32_arith32": 3e-5, "f32dev": 3e-5, "f16dev": 0.3, "f16node": 1e-2}
# bound on the total-mass drift |M(t) - M(0)| / M(0) with scheme A or B
DRIFT = {"f32": 1e-6, "f32_arith32": 1e-5, "f32dev": 1e-6, "f16dev": 3e-3, "f16node": 2e-5}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    from paper_1908_09235_amd import lbm
    lbm.lib()
    return lbm


def run(L, p, steps, storage, **kw):
    say(f"[gpu] {p.name} {p.rule}+{p.fix} {storage} steps={steps} {kw}")
    with L.Domain(p, storage=storage, **kw) as d:
        d.step(steps)
        r, ux, uy = d.moments()
        h = d.mass_history()
    return r, ux, uy, h


def errors(p, a, b):
    fl = ~p.solid.astype(bool)
    return [rel_err(a[i], b[i], fl) for i in range(3)]


_REF = {}


def oracle_ref(p, steps):
    key = (p.name, p.rule, p.fix, steps)
    if key not in _REF:
        o = ora.Oracle(p)
        o.step(steps)
        _REF[key] = o.moments()
    return _REF[key]


@pytest.mark.parametrize("storage", ["f32dev", "f16dev", "f16node"])
@pytest.mark.parametrize("fix", ["A", "B"])
def test_deviation_storage_vs_oracle(L, storage, fix):
    p = cfg.cfg1("mls", fix)
    g = run(L, p, 1000, storage)
    e = errors(p, g, oracle_ref(p, 1000))
    h = g[3]
    drift = np.max(np.abs(h - h[0])) / h[0]
    say(f"    {storage} vs oracle: rho {e[0]:.3e} ux {e[1]:.3e} uy {e[2]:.3e}; "
        f"mass drift {drift:.3e}")
    assert e[0] <= BOUND_RHO[storage] and max(e[1:]) <= BOUND_U[storage]
    assert drift <= DRIFT[storage]
    assert np.all(np.isfinite(g[0]))


def test_deviation_reference_density_is_a_free_choice(L):
    """rho_ref changes only what the stored numbers carry, not the step:
    two references give the same fields to FP32 rounding."""
    p = cfg.cfg1("mls", "B")
    a = run(L, p, 200, "f32dev")
    b = run(L, p, 200, "f32dev", rho_ref=0.2)
    e = errors(p, a, b)
    say(f"    rho_ref auto vs 0.2: {e}")
    assert e[0] <= 1e-5 and max(e[1:]) <= 3e-5


def test_deviation_rest_state_is_exact(L):
    """A uniform fluid at rest at rho_ref has zero deviations; it stays at
    rest in both deviation forms up to the FP64 rounding of the wall rules
    (0.125 is exact in every format, so the stored numbers start at 0)."""
    p = cfg.cfg1("mls", "B")
    fl = ~p.solid.astype(bool)
    q = p.with_(rho0=np.full_like(p.rho0, 0.125), rho_wall=np.full_like(p.rho_wall, 0.125),
                eos="none", G=0.0, name="rest")
    for st in ("f32dev", "f16dev", "f16node"):
        r, ux, uy, h = run(L, q, 50, st, rho_ref=0.125)
        dr = np.max(np.abs(r[fl] - 0.125))
        du = max(np.max(np.abs(ux[fl])), np.max(np.abs(uy[fl])))
        say(f"    {st} rest: max |rho - 0.125| {dr:.3e}, max |u| {du:.3e}")
        assert dr <= 1e-12 and du <= 1e-12


@pytest.fixture(scope="module")
def cyl_small():
    return cfg.many_cylinders(nx=1024, ny=512, n=8, rmin=12.0, rmax=32.0)


@pytest.fixture(scope="module")
def cyl_small_f64(L, cyl_small):
    return run(L, cyl_small, 1000, "f64")


# (rho, u) bounds for the many-cylinder comparison.  These droplets are
# still spreading at step 1000, and a perturbation grows several-fold per
# thousand steps whatever its source, so FP32 arithmetic lands above the
# 1e-5 that FP32 storage with FP64 arithmetic keeps.
CYL_BOUND = {"f32": (1e-5, 1e-5), "f32_arith32": (5e-5, 1e-4),
             "f32dev": (5e-5, 1e-4), "f16dev": (5e-2, 0.3), "f16node": (1e-3, 5e-3)}


@pytest.mark.parametrize("storage", ["f32", "f32_arith32", "f32dev", "f16dev", "f16node"])
def test_many_cylinders_vs_fp64_gpu(L, cyl_small, cyl_small_f64, storage):
    """1024 x 512, 8 cylinders with droplets and their own wettability,
    1000 steps, against the FP64 form of the same library (itself held to
    1e-12 of the oracle)."""
    p = cyl_small
    g = run(L, p, 1000, storage)
    e = errors(p, g, cyl_small_f64)
    h = g[3]
    drift = np.max(np.abs(h - h[0])) / h[0]
    say(f"    {storage} vs fp64: rho {e[0]:.3e} ux {e[1]:.3e} uy {e[2]:.3e}; "
        f"mass drift {drift:.3e}")
    br, bu = CYL_BOUND[storage]
    assert e[0] <= br and max(e[1:]) <= bu
    assert drift <= DRIFT[storage]


def test_full_size_many_cylinders(L):
    """8192 x 4096 with 96 cylinders in the benchmark's launch shape: the
    deviation forms track the FP64 form over 300 steps and scheme B keeps
    the FP64 form's mass to round-off."""
    p = cfg.many_cylinders()
    ref = run(L, p, 300, "f64")
    h = ref[3]
    drift = np.max(np.abs(h - h[0])) / h[0]
    say(f"    f64 mass drift {drift:.3e}")
    assert drift < 1e-13
    for st in ("f32dev", "f16dev", "f16node"):
        g = run(L, p, 300, st)
        e = errors(p, g, ref)
        say(f"    {st} vs fp64: {e}")
        assert e[0] <= BOUND_RHO[st] and max(e[1:]) <= BOUND_U[st]
