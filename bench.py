#!/usr/bin/env python3
"""Benchmark of the PIC particle-grid coupling loop on one MI355X.

Workload: 2D2V thermal plasma, 512 x 512 cells, dx = lambda_D = 1, 64
electrons per cell (16,777,216), Maxwellian v_th = 1, uniform positions,
immobile ion background, CIC, dt = 0.1 (seeded synthetic input).

One step = one full PIC cycle through apic_step: gather + Boris + move,
deposit (CIC), counting sort by tile bucket, periodic Poisson solve and E.
The headline value is the mixed-precision path (binary32 push, cell + binary32
offset positions, int64 fixed-point deposit, FP64 field); the FP64 path is
measured the same way and reported beside it.

Prints one JSON line. Roofline of the dominant kernel (the push pass:
gather + Boris + move + deposit + scatter into the next bucket order) uses
its average launch duration measured with HIP events on the stream the
kernel runs on, inside the timed region.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per particle and pass (particle state read/written
# once per pass; grid terms are O(cells) and excluded):
#   mixed 2D2V state: cell int32 + 2 offsets f32 + 2 velocities f32 = 20 B
#   fp64  2D2V state: 2 positions f64 + 2 velocities f64          = 32 B
# count pass reads the state; push pass reads it and writes it once.
STATE_BYTES = {"mixed": 20, "fp64": 32}


def kernel_source_sha():
    p = os.path.join(ROOT, "paper_2608_15249_amd", "csrc", "apic_kernels.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def load_traffic(precision):
    """HBM bytes per push-pass launch from committed rocprofv3 counter runs,
    if they were taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "step_push_thermal_2d_512_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        e = d.get(precision)
        if not e or d.get("kernel_src_sha") != kernel_source_sha():
            return None
        return float(e["hbm_bytes_per_launch"])
    except Exception:
        return None


def run_path(precision, w, state, steps, warmup, torch):
    from paper_2608_15249_amd.sim import Simulation
    sim = Simulation(w, precision, state=state, tile=(8, 8))
    sim.initialise()
    sim.ctx.sync()
    if warmup:
        sim.run(warmup, diag=False)
    sim.ctx.sync()
    n = sim.n
    diag = torch.zeros(steps * 4, dtype=torch.float64, device="cuda")
    sim.ctx.profile_enable(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.ctx.step(sim.p, sim.E, sim.E32, steps, diag)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.ctx.sync()
    ms, nprof = sim.ctx.profile_read()
    sim.ctx.profile_enable(0)
    elapsed = t1 - t0
    sb = STATE_BYTES[precision]
    push_ms = ms[2] / max(nprof, 1)
    push_bytes = 2 * sb * n
    achieved = push_bytes / (push_ms * 1e-3) / 1e9
    traffic = load_traffic(precision)
    d = diag.cpu().numpy().reshape(steps, 4)
    out = {
        "value": n * steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "hbm_gbs_step": (3 * sb * n * steps) / elapsed / 1e9,
        "phase_ms_per_step": {"count": ms[0] / nprof, "scan": ms[1] / nprof, "push": push_ms,
                              "field": ms[3] / nprof},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if traffic is None else traffic / (push_ms * 1e-3) / 1e9,
                     "kernel": "k_step_push (gather+Boris+move+deposit+scatter)",
                     "bytes_per_launch": push_bytes},
        "final_WE": float(d[-1, 1]),
        "charge": float(d[-1, 0]),
    }
    del sim
    torch.cuda.empty_cache()
    return out


def cpu_baseline(w, state, nsteps):
    """Serial FP64 oracle on the same plasma (host, one core)."""
    import oracle as O
    x, y, vx, vy, vz = state
    s = O.Setup(2, 2, w.nx, w.Lx, len(x), w.dt, ny=w.ny, Ly=w.Ly)
    st = O.State.from_arrays(x, vx, y, vy)
    E, _ = O.initialise(s, st)
    t0 = time.perf_counter()
    for _ in range(nsteps):
        E, _, _ = O.step(s, st, E)
    t1 = time.perf_counter()
    return {"value": len(x) * nsteps / (t1 - t0), "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": "full 512x512 / 16,777,216-particle plasma, %d oracle steps (serial C particle loops + "
                      "numpy FFT, FP64), %.1f s" % (nsteps, t1 - t0)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--paths", default="mixed,fp64")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (N=%d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2608_15249_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = W.thermal_2d()
    state = W.sample(w)
    res = {}
    for path in args.paths.split(","):
        print("bench: %s path, %d warmup + %d timed steps" % (path, args.warmup, args.steps), file=sys.stderr,
              flush=True)
        res[path] = run_path(path, w, state, args.steps, args.warmup, torch)
    head = res.get("mixed") or res[list(res)[0]]
    line = {
        "metric": "particle-steps/s (sort+deposit+gather+push), HBM GB/s; mixed vs FP64 path",
        "value": head["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+i64" if "mixed" in res else "f64",
        "data": "synthetic",
        "config": {"workload": "thermal_2d: 2D2V Maxwellian plasma, 512x512 cells, 64/cell, 16,777,216 electrons, "
                               "dt=0.1, CIC, periodic FFT Poisson",
                   "grid": [512, 512], "particles": w.n_particles, "tile": [8, 8],
                   "precision": "mixed" if "mixed" in res else "fp64"},
        "hbm_gbs_step": head["hbm_gbs_step"],
        "roofline": head["roofline"],
        "phase_ms_per_step": head["phase_ms_per_step"],
    }
    if "fp64" in res and "mixed" in res:
        f = res["fp64"]
        line["fp64"] = {"value": f["value"], "ms_per_step": f["ms_per_step"], "hbm_gbs_step": f["hbm_gbs_step"],
                        "roofline": f["roofline"], "phase_ms_per_step": f["phase_ms_per_step"]}
        line["mixed_over_fp64"] = head["value"] / f["value"]
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (%d oracle steps)" % args.cpu_steps, file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w, state, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
