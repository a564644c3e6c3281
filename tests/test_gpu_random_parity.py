"""Randomized parity sweep: seeded small problems that mix lattice size,
discs (some rotating) and a flat wall with arbitrary wall fractions, every
rule and the fixes it admits, no EOS / exponential / Carnahan-Starling with
a droplet, BGK or MRT, a body force, and the launch shape, against the
oracle after 60 steps (or at the first unstable step): FP64 storage
within 1e-12, FP32 storage (FP64 arithmetic) within 1e-5, the FP32- and
FP16-arithmetic forms within the bounds they are held to elsewhere."""
import sys

import numpy as np
import pytest

from oracle import core as ora
from tests._lib import rel_err
from tests._random_cases import random_case
from tests.test_random_cases import N_CASES, N_OPEN, OPEN_STEPS, STEPS

pytestmark = pytest.mark.gpu

# storage -> (field bound, mass-history bound, velocity floor).  Velocities
# are compared relative to max(max|u|, floor): a case near rest (gravity
# ~1e-5, 2 % density noise) has max|u| ~ 1e-4.  FP64 rounds populations of
# O(0.1) to ~1e-17 absolute; FP32 storage rounds them to ~3e-8 (6e-8
# relative, once per step), so velocities are resolved to ~1e-7 absolute,
# which is the FP32 bound 1e-5 times its floor 1e-2.
# The reduced-precision forms take the bounds they are held to on the
# droplet case (FP32 arithmetic 1e-5 / 3e-5, FP16 per-node 1e-3 / 1e-2),
# with mass-history bounds from their stated drift.
# storage -> (rho bound, u bound, mass-history bound, velocity floor)
TOL = {"f64": (1e-12, 1e-12, 1e-13, 1e-3), "f32": (1e-5, 1e-5, 1e-6, 1e-2),
       "f32_arith32": (1e-5, 3e-5, 1e-5, 1e-2), "f32dev": (1e-5, 3e-5, 1e-6, 1e-2),
       "f16node": (1e-3, 1e-2, 2e-5, 1e-2)}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    from paper_1908_09235_amd import lbm
    lbm.lib()
    return lbm


@pytest.mark.parametrize("storage", ["f64", "f32", "f32_arith32", "f32dev", "f16node"])
@pytest.mark.parametrize("k", range(N_CASES))
def test_random_case_matches_oracle(L, k, storage):
    p, tile_w, tile_h = random_case(k)
    tol_r, tol_u, mass_tol, u_floor = TOL[storage]
    say(f"[gpu] random case {k} {storage}: {p.nx}x{p.ny} {p.rule}/{p.fix} eos={p.eos} "
        f"{p.collision} tau={p.tau:.3f} g={p.gravity} tiles {tile_w}x{tile_h}")
    o = ora.Oracle(p)
    m0 = o.total_mass()
    try:
        hist = o.step(STEPS)
        bad = None
    except ora.OracleError:
        bad = o.t
    with L.Domain(p, storage=storage, tile_w=tile_w, tile_h=tile_h,
                  history_capacity=256) as d:
        if bad is not None:
            with pytest.raises(L.LbmError) as e:
                d.step(STEPS)
            assert e.value.code == L.LBM_EUNSTABLE
            u = L.lbm_unstable_step(d.h)
            say(f"    unstable at step {u} (oracle: {bad})")
            # FP64 storage breaks down at the oracle's step; reduced
            # precision may move the blow-up by a few steps
            assert u == bad if storage == "f64" else abs(u - bad) <= 3
            return
        d.step(STEPS)
        got = d.moments()
        gh = d.mass_history()
    ref = o.moments()
    fl = ~p.solid.astype(bool)
    umax = max(np.max(np.abs(ref[1][fl])), np.max(np.abs(ref[2][fl])))
    scale = max(umax, u_floor)
    e = [rel_err(got[0], ref[0], fl)] + \
        [float(np.max(np.abs(got[i][fl] - ref[i][fl]))) / scale for i in (1, 2)]
    oh = np.concatenate([[m0], hist])
    dm = float(np.max(np.abs(gh - oh) / np.abs(oh)))
    say(f"    rel err rho {e[0]:.2e} ux {e[1]:.2e} uy {e[2]:.2e} (max|u| {umax:.1e}) "
        f"mass {dm:.2e}")
    assert e[0] <= tol_r and max(e[1:]) <= tol_u
    assert np.all(got[0][~fl] == 0)
    assert gh.size == STEPS + 1 and dm <= mass_tol


@pytest.mark.parametrize("persistent,graph", [(1, 8), (0, 0)])
@pytest.mark.parametrize("eos", ["none", "exp", "cs"])
def test_random_cases_batched_equal_alone(L, eos, persistent, graph):
    """The sweep's cases of one EOS as one FP64 batch (a batch holds one
    EOS): every instance ends with the fields, mass history and unstable
    step of the same problem run alone at the batch's launch shape."""
    cases = [random_case(k) for k in range(N_CASES)]
    probs = [c[0] for c in cases if c[0].eos == eos]
    say(f"[gpu] random cases, eos {eos}: {len(probs)} instances, persistent={persistent} "
        f"graph={graph}")
    with L.Batch(storage="f64", eos=eos, max_instances=N_CASES, tile_w=128, tile_h=16,
                 persistent=persistent, graph_steps=graph, arena_bytes=1 << 29) as b:
        slots = [b.add(p, STEPS, history_capacity=256) for p in probs]
        b.run(STEPS + 3)
        b.sync()
        for s, p in zip(slots, probs):
            t, rem, u = b.status(s)
            g, h = b.moments(s), b.mass_history(s)
            # an unstable instance stops at its first non-finite mass: the
            # domain alone runs to that step
            n = STEPS if u < 0 else u
            with L.Domain(p, storage="f64", tile_w=128, tile_h=16, history_capacity=256) as d:
                try:
                    d.step(n)
                except L.LbmError as e:
                    assert e.code == L.LBM_EUNSTABLE
                a_u = L.lbm_unstable_step(d.h)
                a = d.moments()
                ah = d.mass_history()
            assert rem == 0 and u == a_u and t == n, (p.name, t, rem, u, a_u)
            assert all(np.array_equal(g[i], a[i], equal_nan=True) for i in range(3)), p.name
            assert np.array_equal(h, ah, equal_nan=True), p.name


@pytest.mark.parametrize("k", range(N_OPEN))
def test_random_open_case_matches_oracle(L, k):
    """Seeded flows past one or two discs with the open x boundaries:
    fields, mass history and the wall force (momentum exchange) in FP64."""
    from tests._random_cases import random_open_case
    p, tile_w, tile_h = random_open_case(k)
    say(f"[gpu] random open case {k}: {p.nx}x{p.ny} {p.rule}/{p.fix} {p.collision} "
        f"tau={p.tau:.3f} U={p.inlet_u:.3f} tiles {tile_w}x{tile_h}")
    o = ora.Oracle(p)
    m0 = o.total_mass()
    hist = o.step(OPEN_STEPS)
    ref, F_o = o.moments(), o.wall_force()
    with L.Domain(p, storage="f64", tile_w=tile_w, tile_h=tile_h, history_capacity=256) as d:
        d.step(OPEN_STEPS)
        got, F, gh = d.moments(), d.wall_force(), d.mass_history()
    fl = ~p.solid.astype(bool)
    e = [rel_err(got[i], ref[i], fl) for i in range(3)]
    ef = float(np.max(np.abs(F - F_o)) / np.max(np.abs(F_o)))
    oh = np.concatenate([[m0], hist])
    dm = float(np.max(np.abs(gh - oh) / np.abs(oh)))
    say(f"    rel err rho {e[0]:.2e} ux {e[1]:.2e} uy {e[2]:.2e} force {ef:.2e} mass {dm:.2e}")
    assert max(e) <= 1e-12 and ef <= 1e-11 and dm <= 1e-13
