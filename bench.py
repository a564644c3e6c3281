#!/usr/bin/env python3
"""Throughput of the plain two-phase D2Q9 step on one MI355X.

Workload: the droplet resting on a cylinder above a floor, 2048 x 2048,
Carnahan-Starling EOS at 0.86 Tc, MRT with s_nu = 1/tau, tau = 0.8, MLS with
scheme B, synthetic seeded geometry (no dataset).  One step = one pass of the
whole hot path (boundary pass + fused stream/force/collide pass).

Prints one JSON line: MLUPS over fluid nodes (whole job) of the plain form
with FP32 populations (FP64 arithmetic), the roofline of the main kernel
(achieved HBM GB/s from its algorithmic bytes and its mean launch duration,
timed with HIP events on its stream), the FP64-storage and FP32-arithmetic
forms of the same workload, the precision forms on 8192 x 4096, two
time steps per pass against one, the batched form (FP32 storage, and the
same mix in FP64 storage) and the served form, the paper's other
experiments (flow past a cylinder, gravity q-sweep, contact angle), and
the CPU oracle timed on a
bounded sample (one copy, then one independent copy per usable core at
once, before the GPU is touched).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
BYTES_PER_POP = {"f64": 8, "f32": 4, "f32_arith32": 4, "f32dev": 4, "f16dev": 2, "f16node": 2}
# algorithmic bytes per lattice update beyond the 18 populations (the
# FP16 per-node form reads and writes each node's FP32 density)
EXTRA_BYTES = {"f16node": 8}
ARITH = {"f64": "f64", "f32": "f64", "f32_arith32": "f32", "f32dev": "f32", "f16dev": "f32",
         "f16node": "f32"}


def progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1908_09235_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_record(storage, workload):
    """Counter-measured HBM bytes per main-kernel launch, if they were taken
    on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    r = rec.get(f"{workload}:{storage}")
    if not r or r.get("source_hash") != source_hash():
        return None
    return r["bytes_per_launch"]


def run_gpu(p, storage, steps, warmup, stream, tile_w, tile_h, prof_steps,
            moments=False):
    """Warm up, then time `steps` steps (captured step graphs, no events);
    then a separate pass of `prof_steps` steps with HIP events around every
    launch on the library's stream gives the mean kernel durations."""
    import torch

    from paper_1908_09235_amd import lbm

    d = lbm.Domain(p, storage=storage, stream=stream, tile_w=tile_w, tile_h=tile_h,
                   history_capacity=1 << 16)
    info = d.info()
    d.step(warmup)  # also captures the step graphs the timed run replays
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lbm.lbm_step_async(d.h, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lbm.lbm_sync(d.h)  # raises if a step was unstable
    hist = d.mass_history(steps + 1)
    drift = float(abs(hist[-1] - hist[0]) / hist[0])
    mom = d.moments() if moments else None
    main_ms = bnd_ms = 0.0
    main_n = 0
    if prof_steps > 0:
        lbm.lbm_set_profiling(d.h, 1)
        lbm.lbm_step(d.h, prof_steps)
        main_ms, main_n, bnd_ms, bnd_n = lbm.lbm_kernel_times(d.h)
        lbm.lbm_set_profiling(d.h, 0)
        main_ms /= max(main_n, 1)
        bnd_ms /= max(bnd_n, 1)
    d.close()
    return dict(seconds=t1 - t0, info=info, main_ms=main_ms, bnd_ms=bnd_ms, samples=main_n,
                drift=drift, mom=mom)


def copy_bandwidth(torch, mib=1024, reps=20):
    """Read + write rate of a plain device copy of mib MiB (HIP events):
    what this HBM delivers to the simplest streaming kernel."""
    x = torch.empty(mib << 18, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    return round(2 * (mib << 20) / (ms * 1e-3) / 1e9, 1)


def precision_leg(steps, warmup, stream, prof_steps, check_every, time_steps):
    """Many cylinders with droplets, 8192 x 4096, CS at 0.86 Tc, BGK
    tau = 0.8, MLS + B.  Accuracy: every storage form advances in lockstep
    with the FP64 form from the same start, and every check_every steps the
    max-norm relative errors of rho and u over fluid nodes are taken on the
    GPU; a form's steps_within_<tol> is the last checked step up to which
    every check stayed within tol (null if none failed within the run).
    Rate: each form then times time_steps further steps, and a separate
    pass of prof_steps gives its mean main-kernel duration."""
    import numpy as np
    import torch

    from lbm_inputs import configs as cfg
    from paper_1908_09235_amd import lbm

    p = cfg.many_cylinders()
    forms = ("f64", "f32", "f32dev", "f16dev", "f16node")
    n = p.nx * p.ny
    fl = torch.from_numpy(~p.solid.astype(bool).reshape(-1)).cuda()
    doms = {st: lbm.Domain(p, storage=st, stream=stream, history_capacity=1 << 16)
            for st in forms}
    fluid = doms["f64"].info()["fluid_nodes"]
    bufs = {st: torch.empty((3, n), dtype=torch.float64, device="cuda") for st in forms}

    def moments(st):
        b = bufs[st]
        lbm.lbm_moments_device(doms[st].h, b[0].data_ptr(), b[1].data_ptr(), b[2].data_ptr())

    tols = (1e-5, 1e-4, 1e-3, 1e-2)
    within = {st: {t: None for t in tols} for st in forms[1:]}
    history = {st: [] for st in forms[1:]}
    m0 = {st: doms[st].total_mass() for st in forms}
    done = 0
    while done < steps:
        k = min(check_every, steps - done)
        progress(f"  precision forms at step {done}")
        for st in forms:
            try:
                doms[st].step(k)
            except lbm.LbmError:
                pass  # an unstable form keeps its non-finite fields
        done += k
        moments("f64")
        torch.cuda.synchronize()
        ref = bufs["f64"][:, fl]
        den = ref.abs().amax(dim=1)
        for st in forms[1:]:
            moments(st)
            torch.cuda.synchronize()
            e = ((bufs[st][:, fl] - ref).abs().amax(dim=1) / den).cpu().numpy()
            e = np.where(np.isfinite(e), e, np.inf)
            history[st].append((done, float(e[0]), float(e[1]), float(e[2])))
            for t in tols:
                if within[st][t] is None and e.max() > t:
                    within[st][t] = done - k  # the last check that held
    out = {"workload": f"{p.name}_bgk_mls_B", "steps": steps, "check_every": check_every,
           "fluid_nodes": fluid, "wettability": cfg.REALISED_WETTABILITY}
    for st in forms:
        d = doms[st]
        drift = abs(d.total_mass() - m0[st]) / m0[st]
        d.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lbm.lbm_step_async(d.h, time_steps)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        main_ms = 0.0
        if prof_steps > 0:
            lbm.lbm_set_profiling(d.h, 1)
            lbm.lbm_step(d.h, prof_steps)
            mm, mn, _, _ = lbm.lbm_kernel_times(d.h)
            lbm.lbm_set_profiling(d.h, 0)
            main_ms = mm / max(mn, 1)
        rec = {"arith": ARITH[st], "mlups": round(fluid * time_steps / sec / 1e6, 1),
               "main_kernel_ms": round(main_ms, 5),
               "main_kernel_gbs": (round((18 * BYTES_PER_POP[st] + EXTRA_BYTES.get(st, 0)) *
                                         fluid / (main_ms * 1e-3) / 1e9, 1)
                                   if main_ms > 0 else None),
               "mass_drift": float(drift)}
        if st != "f64":
            last = history[st][-1]
            rec.update(err_rho=last[1], err_ux=last[2], err_uy=last[3])
            for t in tols:
                rec[f"steps_within_{t:g}"] = within[st][t]
            rec["errors_by_step"] = [[h[0], round(max(h[1:]), 9)] for h in history[st]]
        out[st] = rec
        d.close()
    return out


def workloads_leg(stream, cyl_steps=40000, grav_steps=60000, ca_steps=30000):
    """The paper's other experiments on the same library, timed (the run
    only, not the set-up): flow past a cylinder (Sec. 4.2, Table 1; Re = 20,
    scheme A, D = 40, FP64, a fixed number of steps), the static flow under
    gravity over q (Sec. 3.1; 36 instances in one batch) and the contact
    angle against the virtual wall density (ten sessile droplets in one
    batch)."""
    import numpy as np
    import torch

    from lbm_inputs import configs as cfg
    from paper_1908_09235_amd import lbm
    from paper_1908_09235_amd import observables as obs

    with open(os.path.join(ROOT, "tests", "golden", "paper_values.json")) as f:
        table1 = json.load(f)["table1"]["Re20"]["A"]
    out = {}

    p = cfg.cylinder_flow(20.0, fix="A")
    m = p.meta
    with lbm.Domain(p, storage="f64", stream=stream, history_capacity=1024) as d:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d.step(cyl_steps)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        F = d.wall_force()
        rho, ux, uy = d.moments()
    r = 0.5 * m["d"]
    out["cylinder"] = {
        "workload": f"cylinder_re20_A_{p.nx}x{p.ny}", "storage": "f64", "steps": cyl_steps,
        "seconds": round(sec, 2), "mlups": round(p.fluid_nodes * cyl_steps / sec / 1e6, 1),
        "Cd": round(float(obs.drag_coefficient(F[0], m["u0"], m["d"])), 4),
        "2L/D": round(float(obs.wake_length(ux, m["cx"], m["cy"], r)), 3),
        "theta_s": round(float(obs.separation_angle(ux, uy, p.solid, m["cx"], m["cy"], r)), 2),
        "paper": table1}

    rules = ("mls", "ibb_linear", "ibb_quadratic", "zhao_yong")
    qs = tuple(n / 10 for n in range(1, 10))
    probs = {(ru, q): cfg.static_gravity(q, rule=ru) for ru in rules for q in qs}
    with lbm.Batch(storage="f64", eos="none", max_instances=len(probs), tile_w=128,
                   tile_h=16, arena_bytes=1 << 28, graph_steps=32, stream=stream) as b:
        slots = {k: b.add(pp, grav_steps, history_capacity=grav_steps + 1)
                 for k, pp in probs.items()}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run(grav_steps)
        b.sync()
        sec = time.perf_counter() - t0
        eps = {}
        for (ru, q), sl in slots.items():
            h = b.mass_history(sl)
            eps.setdefault(ru, {})[f"{q:.1f}"] = float(f"{100 * abs(h[-1] - h[0]) / h[0]:.4g}")
    nodes = sum(pp.fluid_nodes for pp in probs.values())
    out["gravity_q_sweep"] = {
        "workload": "static_gravity_100x50_q0.1..0.9_x4rules", "storage": "f64",
        "instances": len(probs), "steps": grav_steps, "seconds": round(sec, 2),
        "mlups": round(nodes * grav_steps / sec / 1e6, 1), "eps_percent": eps}

    rws = (0.10, 0.12, 0.13, 0.147, 0.18, 0.22)
    probs = [cfg.sessile_droplet(rw, nx=400, ny=200, r0=60.0) for rw in rws]
    with lbm.Batch(storage="f64", eos="cs", max_instances=len(probs), arena_bytes=1 << 30,
                   graph_steps=32, stream=stream) as b:
        slots = [b.add(pp, ca_steps, history_capacity=64) for pp in probs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run(ca_steps)
        b.sync()
        sec = time.perf_counter() - t0
        th = {}
        for rw, pp, sl in zip(rws, probs, slots):
            lvl = 0.5 * (pp.meta["rho_l"] + pp.meta["rho_v"])
            th[f"{rw:g}"] = round(obs.contact_angle(b.moments(sl)[0], pp.solid, pp.meta["wall_y"],
                                                    lvl, y_max=pp.ny - 3.5)[0], 2)
    nodes = sum(pp.fluid_nodes for pp in probs)
    out["contact_angle"] = {
        "workload": "sessile_droplet_400x200_r60_cs0.86", "storage": "f64",
        "instances": len(probs), "steps": ca_steps, "seconds": round(sec, 2),
        "mlups": round(nodes * ca_steps / sec / 1e6, 1), "theta_deg_by_rho_wall": th}
    return out


def rel_err_fields(p, g, ref):
    """max |g - ref| / max |ref| of rho, ux, uy over fluid nodes."""
    import numpy as np

    fl = ~p.solid.astype(bool)
    out = {}
    for i, nm in enumerate(("rho", "ux", "uy")):
        den = float(np.max(np.abs(ref[i][fl])))
        out[f"err_{nm}"] = float(np.max(np.abs(g[i][fl] - ref[i][fl])) / den) if den else None
    return out


def _batch_run(probs, storage, steps, stream, tune_steps):
    """One batch of the whole mix: build, tune, run `steps` steps (timed).
    The batch is returned alive for the read-out."""
    import numpy as np
    import torch

    from paper_1908_09235_amd import lbm

    cap = 1 << int(np.ceil(np.log2(steps + 2)))
    b = lbm.Batch(storage=storage, eos="cs", max_instances=len(probs), arena_bytes=48 << 30)
    t0 = time.perf_counter()
    slots = [b.add(p, steps, history_capacity=cap) for p in probs]
    t_build = time.perf_counter() - t0
    tuned = b.tune(tune_steps)
    b.sync()
    done0 = np.array([b.status(s)[0] for s in slots], dtype=np.float64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(steps)
    b.sync()
    secs = time.perf_counter() - t0
    st = [b.status(s) for s in slots]
    done = np.array([x[0] for x in st], dtype=np.float64) - done0
    fluid = np.array([p.fluid_nodes for p in probs], dtype=np.float64)
    stable = [k for k, x in enumerate(st) if x[2] < 0]
    rec = {"storage": storage, "arith": ARITH[storage], "seconds": round(secs, 3),
           "solves_per_s": round(len(stable) / secs, 2),
           "stable": len(stable), "unstable": len(probs) - len(stable),
           "mlups": round(float((fluid * done).sum()) / secs / 1e6, 1),
           "tuned": tuned, "build_seconds": round(t_build, 2), "info": b.info()}
    return b, slots, st, rec


def batch_leg(steps, n_inst, stream, tune_steps, alone_steps, gate=1e-5):
    """The batched mix: n_inst droplet-on-cylinder instances (sides
    64..768, T/Tc, tau drawn per instance), one batch each in FP32 and FP64
    storage, autotuned, each instance run `steps` steps.  A solve is an
    instance that stays stable for all its steps (the unstable ones stop at
    their first non-finite mass and are counted apart).  Every instance
    stable in both is compared with its FP64 run (bit-identical to the
    plain FP64 form, which the GPU tests check), max-norm relative over
    fluid nodes; the gated rate is that of the FP64 batch unless every
    FP32 instance is within the gate.  A sample run one by one gives the
    unbatched rate (alone_steps 0: not measured)."""
    import numpy as np
    import torch

    from lbm_inputs import configs as cfg
    from paper_1908_09235_amd import lbm

    probs = [cfg.batch_instance(k) for k in range(n_inst)]
    fluid = np.array([p.fluid_nodes for p in probs], dtype=np.float64)
    b32, s32, st32, r32 = _batch_run(probs, "f32", steps, stream, tune_steps)
    progress("  FP32 batch done")
    b64, s64, st64, r64 = _batch_run(probs, "f64", steps, stream, tune_steps)
    progress("  FP64 batch done; comparing every stable instance")
    errs = []
    for k in range(n_inst):
        if st32[k][2] >= 0 or st64[k][2] >= 0:
            continue
        e = rel_err_fields(probs[k], b32.moments(s32[k]), b64.moments(s64[k]))
        errs.append((max(e.values()), k, e))
    b32.close()
    b64.close()
    within = sum(1 for m, _, _ in errs if m <= gate)
    worst = sorted(errs, reverse=True)[:5]
    both_unstable = sum(1 for k in range(n_inst) if st32[k][2] >= 0 and st64[k][2] >= 0)
    all_in = within == len(errs)
    out = {"workload": f"droplet_cylinder_mix_{n_inst}", "instances": n_inst, "steps": steps,
           "nodes": int(sum(p.nx * p.ny for p in probs)), "fluid_nodes": int(fluid.sum()),
           "graph_steps": 32, "fp32": r32, "fp64": r64,
           "vs_fp64": {"gate": gate, "compared": len(errs), "within_gate": within,
                       "unstable_in_both": both_unstable,
                       "max_err": max((m for m, _, _ in errs), default=None),
                       "worst": [{"instance": k, "side": probs[k].nx, **e}
                                 for _, k, e in worst]},
           "solves_per_s_at_gate": r32["solves_per_s"] if all_in else r64["solves_per_s"],
           "storage_at_gate": "f32" if all_in else "f64"}
    if alone_steps <= 0:
        return out
    # the unbatched rate: a sample of instances one after another, one
    # domain and two launches per step each
    k_alone = list(range(0, n_inst, max(1, n_inst // 16)))
    lu_a, t_a = 0.0, 0.0
    for k in k_alone:
        with lbm.Domain(probs[k], storage="f32", stream=stream) as d:
            d.step(5)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            try:
                d.step(alone_steps)
            except lbm.LbmError:
                pass
            torch.cuda.synchronize()
            t_a += time.perf_counter() - ta
            lu_a += fluid[k] * alone_steps
    out["one_by_one_mlups"] = round(lu_a / t_a / 1e6, 1)
    out["one_by_one_sample"] = f"{len(k_alone)} instances x {alone_steps} steps, FP32"
    return out


def serve_leg(storage, n_requests, rates, chunk, pool, n_check, gate=1e-5,
              gate_storage="f64"):
    """The served workload: Poisson arrivals of droplet-on-cylinder
    requests (95 % the batched mix, 5 % 2048^2; 2000..20000 steps each) into
    one server.  First a saturated run (every request present at t = 0)
    measures the sustainable completion rate of stable solves, then about
    n_requests arrive at each rate in `rates` (fractions of it) for
    time-to-solution percentiles.  The first n_check stable requests of the
    first rate (and its first 2048^2 one) are run again alone in FP64
    storage and compared (max-norm relative over fluid nodes).  The same
    saturated run in `gate_storage` gives the rate at the accuracy gate:
    its results are those of the FP64 plain form, bit for bit."""
    import numpy as np

    from lbm_inputs import configs as cfg
    from paper_1908_09235_amd import lbm

    probs = {k: cfg.batch_instance(k) for k in range(pool)}
    probs["big"] = cfg.cfg2a()
    nodes = {k: p.nx * p.ny for k, p in probs.items()}
    e_nodes = 0.95 * np.mean([nodes[k] for k in range(pool)]) + 0.05 * nodes["big"]
    e_steps = 11000.0

    def run(reqs, horizon, check=0, storage=storage):
        # one workgroup per tile, 256 x 8 tiles, rings of four rows: the
        # shape the autotuner picks for the FP32 batched mix, and the
        # fastest of those measured on the saturated request mix
        srv = lbm.Server(chunk_steps=chunk, storage=storage, eos="cs", max_instances=4096,
                         arena_bytes=96 << 30, persistent=0, tile_w=256, tile_h=8, ring=4)
        arrive, done_t, info, fields = {}, {}, {}, {}
        i = 0
        t0 = time.perf_counter()
        lu = 0.0
        last_note = 0.0
        while True:
            now = time.perf_counter() - t0
            if now - last_note > 20.0:
                progress(f"  served {len(done_t)} of {len(reqs)} requests, {now:.0f} s")
                last_note = now
            while i < len(reqs) and reqs[i][0] <= now:
                _, key, steps = reqs[i]
                rid = srv.submit(probs[key], steps, history_capacity=1 << 15)
                arrive[rid] = (reqs[i][0], key, steps)
                i += 1
            fin = srv.progress()
            now = time.perf_counter() - t0
            for rid in fin:
                done_t[rid] = now
                key = arrive[rid][1]
                keys = [v[0] for v in fields.values()]
                want = check > 0 and (("big" not in keys) if key == "big"
                                      else (len(keys) - keys.count("big") < check))
                r = srv.result(rid, fields=want)
                info[rid] = r
                if want and r["unstable_step"] < 0:
                    fields[rid] = (key, r["steps"], (r["rho"], r["ux"], r["uy"]))
                lu += probs[key].fluid_nodes * r["steps"]
                srv.release(rid)
            if (i == len(reqs) and len(done_t) == len(reqs)) or now > horizon:
                break
            if not fin and srv.info()["running"] == 0 and i < len(reqs):
                time.sleep(min(0.002, max(0.0, reqs[i][0] - now)))
        wall = time.perf_counter() - t0
        st = srv.info()
        srv.close()
        ok = [r for r in done_t if info[r]["unstable_step"] < 0]
        lat = np.array([done_t[r] - arrive[r][0] for r in ok])
        drift = [abs(info[r]["mass"] - info[r]["mass0"]) / info[r]["mass0"]
                 for r in ok if np.isfinite(info[r]["mass0"])]
        out = {"requests": len(reqs), "completed": len(done_t), "stable": len(ok),
               "unstable": len(done_t) - len(ok), "wall_s": round(wall, 2),
               "solves_per_s": round(len(ok) / wall, 2),
               "mlups": round(lu / wall / 1e6, 1),
               "p50_s": round(float(np.percentile(lat, 50)), 3) if len(lat) else None,
               "p99_s": round(float(np.percentile(lat, 99)), 3) if len(lat) else None,
               "max_s": round(float(lat.max()), 3) if len(lat) else None,
               "max_mass_drift": float(max(drift)) if drift else None,
               "chunks": st["chunks"], "unfinished": len(reqs) - len(done_t)}
        return out, fields

    # saturated: every request present at once
    sat_reqs = [(0.0, k, s) for (_, k, s) in cfg.request_stream(1000.0, 0.12, pool=pool)]
    sat, _ = run(sat_reqs, 120.0)
    lam_max = sat["solves_per_s"]
    progress(f"  saturated {storage}: {lam_max} stable solves/s; the same in {gate_storage}")
    sat_gate, _ = run(sat_reqs, 180.0, storage=gate_storage)
    sweep = []
    for j, f in enumerate(rates):
        lam = max(lam_max * f, 0.1)
        reqs = cfg.request_stream(lam, n_requests / lam, pool=pool)
        r, fields = run(reqs, 3 * n_requests / lam + 60, n_check if j == 0 else 0)
        r["rate"] = round(lam, 2)
        r["rate_fraction"] = f
        if fields:
            chk = []
            for rid, (key, steps, g) in fields.items():
                with lbm.Domain(probs[key], storage="f64") as d:
                    d.step(steps)
                    ref = d.moments()
                chk.append({"request": rid, "instance": key, "steps": steps,
                            **rel_err_fields(probs[key], g, ref)})
            r["vs_fp64"] = {"gate": gate, "checked": len(chk),
                            "within_gate": sum(1 for c in chk if max(
                                c["err_rho"], c["err_ux"], c["err_uy"]) <= gate),
                            "requests": chk}
        sweep.append(r)
    offered = 200.0 * e_nodes * e_steps
    return {"workload": "droplet_cylinder_requests", "storage": storage,
            "chunk_steps": chunk, "pool": pool,
            "launch": {"persistent": 0, "tile_w": 256, "tile_h": 8, "ring": 4},
            "mean_nodes_per_request": round(float(e_nodes)),
            "mean_steps_per_request": e_steps,
            "offered_lups_at_200_per_s": offered,
            "offered_vs_fp32_hbm_roofline": round(offered / (PEAK_HBM_GBS * 1e9 / 72.0), 2),
            "saturated": sat, "sustainable_rate_per_s": lam_max, "sweep": sweep,
            "at_gate": {"storage": gate_storage, "gate": gate,
                        "note": "every result equals the FP64 plain form's, bit for bit",
                        "saturated": sat_gate},
            "solves_per_s_at_gate": sat_gate["solves_per_s"],
            "p99_s_at_gate_saturated": sat_gate["p99_s"]}


def two_step_leg(steps, warmup, stream, prof_steps):
    """Two time steps per pass against one.  Cases: the wall-free shear wave
    (2048 x 2048, BGK, no interaction force) in FP32 storage with FP32 and
    with FP64 arithmetic, the benchmark's workload, and the 96 cylinders of
    the precision forms (8192 x 4096) with FP32 arithmetic, in FP32 storage
    and as FP32 deviations.  Per case and
    setting: the step rate over `steps` timed steps (graph replays), and the
    mean duration of the main launch over a separate pass of `prof_steps`
    steps (each launch records its own start and end).  The effective rate
    counts the algorithmic bytes of the steps one launch advances, 18
    populations per fluid node per step, against the HBM peak.  `tuned` is
    the setting lbm_tune_steps_per_pass picks on a fresh domain."""
    import torch

    from lbm_inputs import configs as cfg
    from paper_1908_09235_amd import lbm

    # (name, problem, storage forms, rows per two-step tile: 0 for the
    # library's default; the droplet's walls run along whole strips, where
    # shorter tiles pay)
    cases = [("shear_wave_2048x2048_bgk", lambda: cfg.shear_wave(2048, nx=2048, collision="bgk"),
              ("f32_arith32", "f32"), 0),
             ("droplet_cylinder_2048x2048_mrt_mls_B", cfg.cfg2a, ("f32",), 8),
             ("droplet_cylinder_2048x2048_mrt_mls_B", cfg.cfg2a, ("f32_arith32",), 5),
             ("cylinders96_8192x4096_bgk_mls_B", cfg.many_cylinders, ("f32_arith32", "f32dev"), 0)]
    out = {}
    for name, make, storages, tile_h in cases:
        p = make()
        fluid = int((~p.solid.astype(bool)).sum())
        for st in storages:
            rec = {}
            for spp in (1, 2):
                d = lbm.Domain(p, storage=st, stream=stream, history_capacity=1 << 12)
                if spp == 2:
                    lbm.lbm_set_steps_per_pass(d.h, 2, tile_h)
                    th_used = lbm.lbm_get_steps_per_pass(d.h)[1]
                d.step(warmup)  # also captures the step graphs
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                lbm.lbm_step_async(d.h, steps)
                torch.cuda.synchronize()
                sec = time.perf_counter() - t0
                lbm.lbm_sync(d.h)
                lbm.lbm_set_profiling(d.h, 1)
                lbm.lbm_step(d.h, prof_steps)
                mm, mn, bm, bn = lbm.lbm_kernel_times(d.h)
                lbm.lbm_set_profiling(d.h, 0)
                d.close()
                main_ms = mm / max(mn, 1)
                alg = spp * 18 * BYTES_PER_POP[st] * fluid
                gbs = alg / (main_ms * 1e-3) / 1e9 if main_ms > 0 else None
                rec[f"steps_per_pass_{spp}"] = {
                    "us_per_step": round(sec / steps * 1e6, 2),
                    "mlups": round(fluid * steps / sec / 1e6, 1),
                    "main_launch_us": round(main_ms * 1e3, 2),
                    "boundary_launch_us": round(bm / max(bn, 1) * 1e3, 2),
                    "algorithmic_bytes_per_launch": alg,
                    "effective_gbs": gbs and round(gbs, 1),
                    "frac": gbs and round(gbs / PEAK_HBM_GBS, 4)}
            rec["two_step_tile_h"] = th_used
            # what the library's own tuner picks for this case
            with lbm.Domain(p, storage=st, stream=stream, history_capacity=1 << 12) as d:
                rec["tuned"] = d.tune_steps_per_pass(max(50, steps // 20))
            out[f"{name}:{st}" + (f":tile_h{tile_h}" if tile_h else "")] = rec
    return out


def cpu_baseline(p, seconds):
    from oracle import core as ora

    o = ora.Oracle(p)
    o.step(1)  # first step outside the timing
    n, t = 0, 0.0
    t0 = time.perf_counter()
    while t < seconds:
        o.step(1)
        n += 1
        t = time.perf_counter() - t0
    return n, t


def host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


def cpu_leg(scale, seconds, procs):
    """The oracle on the benchmark's workload: one copy in this process,
    then `procs` independent copies at once in child processes (the
    oracle is single-threaded; their summed rate is what the host's cores
    give).  Runs before anything touches the GPU."""
    import subprocess

    from lbm_inputs import configs as cfg

    p = cfg.cfg2a(scale=scale)
    fluid = int((~p.solid.astype(bool)).sum())
    n, t = cpu_baseline(p, seconds)
    del p
    out = {"value": round(fluid * n / t / 1e6, 3), "unit": "MLUPS", "cores": 1,
           "kind": "oracle",
           "sample": f"{n} steps of the same workload (FP64 C oracle, single thread, "
                     f"{t:.1f} s)",
           "host": host_cpu()}
    if procs > 1:
        # a secondary figure: a failed or late copy is reported, not fatal
        cmd = [sys.executable, os.path.abspath(__file__), "--oracle-worker",
               str(seconds), "--scale", str(scale)]
        kids = [subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True) for _ in range(procs)]
        res, err = [], None
        for k in kids:
            try:
                o, _ = k.communicate(timeout=seconds + 120)
            except subprocess.TimeoutExpired:
                k.kill()
                k.communicate()
                err = "an oracle copy did not finish in time"
                continue
            if k.returncode != 0:
                err = f"an oracle copy failed ({k.returncode})"
                continue
            res.append(json.loads(o.strip().splitlines()[-1]))
        if err is None:
            rate = sum(fluid * r["n"] / r["t"] for r in res)
            out["all_cores"] = {"value": round(rate / 1e6, 3), "unit": "MLUPS", "procs": procs,
                                "sample": f"{procs} independent copies at once, "
                                          f"{sum(r['n'] for r in res)} steps in all"}
        else:
            out["all_cores"] = {"value": None, "procs": procs, "error": err}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--storage", default="f32", choices=sorted(BYTES_PER_POP))
    ap.add_argument("--other-steps", type=int, default=5000,
                    help="steps of the other storage forms reported beside (0: skip)")
    ap.add_argument("--scale", type=float, default=16.0,
                    help="droplet geometry scale (16 = 2048 x 2048)")
    ap.add_argument("--tile-w", type=int, default=0)
    ap.add_argument("--tile-h", type=int, default=0)
    ap.add_argument("--prof-steps", type=int, default=100,
                    help="steps of the separate pass that times every launch "
                         "with HIP events, after the timed region (events "
                         "between launches would add their own cost to the "
                         "timed steps)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="oracle copies run at once for the all-cores rate "
                         "(0: the usable cores, at most 16; 1: skip)")
    ap.add_argument("--oracle-worker", type=float, default=0.0, help=argparse.SUPPRESS)
    ap.add_argument("--precision-steps", type=int, default=2000,
                    help="steps of the 8192 x 4096 precision-form comparison (0: skip)")
    ap.add_argument("--precision-check", type=int, default=250,
                    help="steps between the precision forms' error checks")
    ap.add_argument("--precision-time-steps", type=int, default=500,
                    help="steps each precision form is timed over")
    ap.add_argument("--two-step-steps", type=int, default=2000,
                    help="steps of each two-steps-per-pass comparison (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=5000,
                    help="steps of each instance of the batched mix (0: skip)")
    ap.add_argument("--batch-instances", type=int, default=512)
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests of each served run at a fixed arrival rate (0: skip; "
                         "1000 puts the 99th percentile at the tenth-longest)")
    ap.add_argument("--serve-check", type=int, default=6,
                    help="served requests compared with an FP64 run of their own")
    ap.add_argument("--serve-chunk", type=int, default=100)
    ap.add_argument("--workloads", type=int, default=1,
                    help="also time the paper's other experiments (0: skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter "
                         "calibration under rocprofv3)")
    a = ap.parse_args()

    if a.oracle_worker > 0:
        # a child of the CPU leg: time one oracle copy, print (steps, seconds)
        from lbm_inputs import configs as cfg

        n, t = cpu_baseline(cfg.cfg2a(scale=a.scale), a.oracle_worker)
        print(json.dumps({"n": n, "t": t}), flush=True)
        return

    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (the domain is not "
              "sharded); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    # the CPU leg first, before anything touches the GPU
    cpu = None
    if a.cpu_seconds > 0:
        procs = a.cpu_procs or min(len(os.sched_getaffinity(0)), 16)
        progress(f"CPU oracle leg ({procs} copies)")
        cpu = cpu_leg(a.scale, a.cpu_seconds, procs)

    import torch

    from lbm_inputs import configs as cfg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    p = cfg.cfg2a(scale=a.scale)
    workload = f"droplet_cylinder_{p.nx}x{p.ny}_mrt_mls_B"
    n_dense = p.nx * p.ny

    if a.copy_probe_mib:
        x = torch.empty(a.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()

    copy_gbs = copy_bandwidth(torch)
    progress(f"headline: {workload}, {a.storage}, {a.steps} steps")
    r = run_gpu(p, a.storage, a.steps, a.warmup, stream, a.tile_w, a.tile_h, a.prof_steps)
    fluid = r["info"]["fluid_nodes"]
    s = BYTES_PER_POP[a.storage]
    mlups = fluid * a.steps / r["seconds"] / 1e6
    alg_bytes = 18 * s * fluid  # 9 reads + 9 writes per fluid node
    achieved = alg_bytes / (r["main_ms"] * 1e-3) / 1e9 if r["main_ms"] > 0 else None
    traffic = traffic_record(a.storage, workload)

    also = {}
    for st in ("f64", "f32_arith32"):
        if st == a.storage or a.other_steps <= 0:
            continue
        ro = run_gpu(p, st, a.other_steps, a.warmup, stream, a.tile_w, a.tile_h,
                     a.prof_steps)
        so = BYTES_PER_POP[st]
        also[st] = {
            "storage": st, "arith": ARITH[st],
            "mlups": round(fluid * a.other_steps / ro["seconds"] / 1e6, 1),
            "ms_per_step": round(ro["seconds"] / a.other_steps * 1e3, 5),
            "main_kernel_ms": round(ro["main_ms"], 5),
            "main_kernel_gbs": (round(18 * so * fluid / (ro["main_ms"] * 1e-3) / 1e9, 1)
                                if ro["main_ms"] > 0 else None),
            "mass_drift": ro["drift"], "steps": a.other_steps}

    prec = None
    if a.precision_steps > 0:
        progress("precision forms, 8192 x 4096")
        prec = precision_leg(a.precision_steps, a.warmup, stream, a.prof_steps,
                             a.precision_check, a.precision_time_steps)

    two = None
    if a.two_step_steps > 0:
        progress("two steps per pass against one")
        two = two_step_leg(a.two_step_steps, a.warmup, stream, a.prof_steps)

    batch = None
    if a.batch_steps > 0:
        progress(f"batched mix, {a.batch_instances} instances")
        batch = batch_leg(a.batch_steps, a.batch_instances, stream, 3, 500)
    serve = None
    if a.serve_requests > 0:
        progress(f"served form, {a.serve_requests} requests per rate")
        serve = serve_leg("f32", a.serve_requests, [0.5, 0.8], a.serve_chunk, 128,
                          a.serve_check)

    if a.workloads:
        progress("the paper's other experiments")
    other = workloads_leg(stream) if a.workloads else None


    out = {
        "metric": "MLUPS (fluid-node lattice updates per second), plain step",
        "value": round(mlups, 1), "unit": "MLUPS",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(r["seconds"] / a.steps * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": ARITH[a.storage], "data": "synthetic",
        "config": {"workload": workload, "storage": a.storage, "nx": p.nx, "ny": p.ny,
                   "fluid_nodes": fluid, "dense_mlups": round(n_dense * a.steps / r["seconds"] / 1e6, 1),
                   "collision": "mrt", "rule": "mls", "fix": "B", "eos": "cs@0.86Tc",
                   "tile_w": r["info"]["tile_w"], "tile_h": r["info"]["tile_h"],
                   "mass_drift": r["drift"]},
        "roofline": {"bound": "hbm", "achieved": achieved and round(achieved, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved and round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic,
                     "kernel": "k_main", "kernel_ms": round(r["main_ms"], 5),
                     "kernel_samples": r["samples"],
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "copy_gbs": copy_gbs,
                     "boundary_kernel_ms": round(r["bnd_ms"], 5)},
        "cpu_baseline": cpu,
        "also": also,
        "precision": prec,
        "two_step": two,
        "batched": batch,
        "served": serve,
        "paper_experiments": other,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
