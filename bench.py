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
forms of the same workload, and the CPU oracle timed on a bounded sample.
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
BYTES_PER_POP = {"f64": 8, "f32": 4, "f32_arith32": 4, "f32dev": 4, "f16dev": 2}
ARITH = {"f64": "f64", "f32": "f64", "f32_arith32": "f32", "f32dev": "f32", "f16dev": "f32"}


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


def run_gpu(p, storage, steps, warmup, stream, tile_w, tile_h, prof_every,
            moments=False):
    import torch

    from paper_1908_09235_amd import lbm

    d = lbm.Domain(p, storage=storage, stream=stream, tile_w=tile_w, tile_h=tile_h,
                   history_capacity=1 << 16)
    info = d.info()
    d.step(warmup)
    torch.cuda.synchronize()
    lbm.lbm_set_profiling(d.h, prof_every)
    t0 = time.perf_counter()
    lbm.lbm_step(d.h, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    main_ms, main_n, bnd_ms, bnd_n = lbm.lbm_kernel_times(d.h)
    lbm.lbm_set_profiling(d.h, 0)
    hist = d.mass_history(steps + 1)
    drift = float(abs(hist[-1] - hist[0]) / hist[0])
    mom = d.moments() if moments else None
    d.close()
    return dict(seconds=t1 - t0, info=info, main_ms=main_ms / max(main_n, 1),
                bnd_ms=bnd_ms / max(bnd_n, 1), samples=main_n, drift=drift, mom=mom)


def precision_leg(steps, warmup, stream, prof_every):
    """Many cylinders with droplets, 8192 x 4096, CS at 0.86 Tc, BGK
    tau = 0.8, MLS + B: each storage form run from the same start for the
    same steps; errors of rho and u (max-norm relative, fluid nodes)
    against the FP64 form."""
    import numpy as np

    from lbm_inputs import configs as cfg

    p = cfg.many_cylinders()
    fl = ~p.solid.astype(bool)
    out = {"workload": f"{p.name}_bgk_mls_B", "steps": steps}
    ref = None
    for st in ("f64", "f32", "f32dev", "f16dev"):
        r = run_gpu(p, st, steps, warmup, stream, 0, 0, prof_every, moments=True)
        fluid = r["info"]["fluid_nodes"]
        rec = {"arith": ARITH[st],
               "mlups": round(fluid * steps / r["seconds"] / 1e6, 1),
               "main_kernel_ms": round(r["main_ms"], 5),
               "main_kernel_gbs": (round(18 * BYTES_PER_POP[st] * fluid /
                                         (r["main_ms"] * 1e-3) / 1e9, 1)
                                   if r["main_ms"] > 0 else None),
               "mass_drift": r["drift"]}
        if st == "f64":
            ref = r["mom"]
        else:
            for i, nm in enumerate(("rho", "ux", "uy")):
                den = np.max(np.abs(ref[i][fl]))
                rec[f"err_{nm}"] = float(np.max(np.abs(r["mom"][i][fl] - ref[i][fl])) / den)
        out[st] = rec
    out["fluid_nodes"] = fluid
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
    ap.add_argument("--prof-every", type=int, default=1,
                    help="time the kernels of every n-th step with HIP events")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--precision-steps", type=int, default=2000,
                    help="steps of the 8192 x 4096 precision-form comparison (0: skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter "
                         "calibration under rocprofv3)")
    a = ap.parse_args()

    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (the domain is not "
              "sharded); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

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

    r = run_gpu(p, a.storage, a.steps, a.warmup, stream, a.tile_w, a.tile_h, a.prof_every)
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
                     a.prof_every)
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
        prec = precision_leg(a.precision_steps, a.warmup, stream, a.prof_every)

    cpu = None
    if a.cpu_seconds > 0:
        n, t = cpu_baseline(p, a.cpu_seconds)
        cpu = {"value": round(fluid * n / t / 1e6, 3), "unit": "MLUPS", "cores": 1,
               "kind": "oracle",
               "sample": f"{n} steps of the same {p.nx}x{p.ny} workload (FP64 C oracle, "
                         f"single thread, {t:.1f} s)"}

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
                     "boundary_kernel_ms": round(r["bnd_ms"], 5)},
        "cpu_baseline": cpu,
        "also": also,
        "precision": prec,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
