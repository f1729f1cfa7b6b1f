#!/usr/bin/env python3
"""Benchmark of the PIC particle-grid coupling loop on one MI355X.

Default workload (magnetized_2d3v, the largest single-plasma configuration):
2D3V Maxwellian plasma in a uniform B_z (omega_c/omega_p = 2), 1024 x 1024
cells, dx = lambda_D = 1, 32 electrons per cell (33,554,432), v_th = 1 in all
three components, 1% density perturbation at k = (2 pi/64, 0), Boris push,
CIC, dt = 0.05 (seeded synthetic input); the default run also measures
thermal_2d (2D2V, 512 x 512 cells, 64 per cell, 16,777,216 electrons,
dt = 0.1) and reports it under "thermal_2d". Other workloads (--workload):
thermal_2d alone, thermal_3d (3D3V, 128 x 128 x 128 cells, 8 per cell,
16,777,216 electrons, dt = 0.1: the Cartesian 3D form of the coupling loop)
and landau_batch (256 uneven 1D1V Landau-damping replicas advanced by the
batched path, one graph-replayed persistent launch per step).

One step = one full PIC cycle: gather + Boris + move, deposit (CIC),
counting sort by tile bucket, periodic Poisson solve and E. The headline value
is the mixed-precision path (binary32 push, cell + binary32 offset positions,
int64 fixed-point deposit, FP64 field); the FP64 path is measured the same
way and reported beside it. The sort-bucket tile (single plasma) and the
work-item size (batch) are picked by the library's autotuner unless given.

Prints one JSON line. Roofline of the dominant kernel (the push pass:
gather + Boris + move + deposit + scatter into the next bucket order; the
whole persistent launch for the batch) uses its average launch duration
measured with HIP events on the stream the kernel runs on, inside the timed
region.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# the timed run times the push pass with HIP events on one step in this many
PROF_EVERY = 10

# Algorithmic HBM bytes per particle and pass: the particle state is read
# once (count pass) or read and written once (push pass); grid terms are
# O(cells) and excluded.
#   mixed: cell int32 + dim binary32 offsets + vdim binary32 velocities
#   fp64 : dim FP64 positions + vdim FP64 velocities
def state_bytes(precision, dim, vdim):
    return 4 + 4 * dim + 4 * vdim if precision == "mixed" else 8 * dim + 8 * vdim


PHASE_NOTE = ("from a separate run of %%d steps after the timed one, with HIP events between all phases (each "
              "event drains the queue, so these sum to more than ms_per_step); the timed run records only the two "
              "events around the push, on one step in %d, whose average duration gives roofline.achieved" % PROF_EVERY)


def phase_breakdown(ctx, run, steps):
    """Summed per-phase milliseconds (count, scan, push, field) of a short run
    with events around every phase, and its step count."""
    import torch
    k = min(steps, 20)
    dg = torch.zeros(4 * k, dtype=torch.float64, device="cuda")
    ctx.profile_phases(True)
    ctx.profile_enable(k)
    run(k, dg)
    ctx.sync()
    ms, nprof = ctx.profile_read()
    ctx.profile_enable(0)
    return ms, max(nprof, 1)


def load_traffic(precision, workload, tile):
    """HBM bytes per push-pass launch from committed rocprofv3 counter runs,
    if they were taken on the current kernel source, workload and tile;
    else None."""
    p = os.path.join(ROOT, "profiles", "step_push_%s_traffic.json" % workload)
    if not os.path.exists(p):
        return None
    from paper_2608_15249_amd.rocprof_summary import kernel_source_sha
    try:
        d = json.load(open(p))
        e = d.get(precision)
        if not e or d.get("kernel_src_sha") != kernel_source_sha() or list(e.get("tile", [])) != list(tile):
            return None
        return float(e["hbm_bytes_per_launch"])
    except Exception:
        return None


# Atomic-throughput peaks, derived from unit counts and clock (256 CUs,
# 2.4 GHz): LDS 128 bytes per clock per CU, of which a 64-bit atomic lane
# operation uses 8; L2 one atomic per channel per clock, 16 channels in each of
# the 8 XCDs.
LDS_ATOMIC_PEAK_OPS = 256 * 2.4e9 * 128 / 8
L2_ATOMIC_PEAK_OPS = 8 * 16 * 2.4e9


def load_counters(precision, workload, tile):
    """Per-launch counter values of the push from the committed rocprofv3
    counter runs, if taken on the current kernel source, workload and tile."""
    p = os.path.join(ROOT, "profiles", "step_push_%s_counters.json" % workload)
    if not os.path.exists(p):
        return None
    from paper_2608_15249_amd.rocprof_summary import kernel_source_sha
    try:
        d = json.load(open(p))
        e = d.get(precision)
        if not e or d.get("kernel_src_sha") != kernel_source_sha() or list(e.get("tile", [])) != list(tile):
            return None
        return e["per_launch"]
    except Exception:
        return None


def atomics_of(counters, n, push_ms):
    """Atomic counts per launch of the push (LDS deposit atomics as active
    64-bit lane operations from SQ_INSTS_LDS_ATOMIC_BANDWIDTH, 64-byte units;
    L2 atomics of the tile flushes and far movers from TCC_ATOMIC_sum), per
    particle, and their rates over the measured launch time against the
    derived peaks."""
    if not counters:
        return None
    lds_ops = counters.get("SQ_INSTS_LDS_ATOMIC_BANDWIDTH", 0.0) * 64 / 8
    l2 = counters.get("TCC_ATOMIC_sum", 0.0)
    t = push_ms * 1e-3
    return {"lds_atomic_ops": lds_ops, "lds_atomic_ops_per_particle": lds_ops / n,
            "lds_atomic_rate": lds_ops / t, "lds_atomic_peak": LDS_ATOMIC_PEAK_OPS,
            "lds_atomic_frac": lds_ops / t / LDS_ATOMIC_PEAK_OPS,
            "l2_atomics": l2, "l2_atomics_per_particle": l2 / n, "l2_atomic_rate": l2 / t,
            "l2_atomic_peak": L2_ATOMIC_PEAK_OPS, "l2_atomic_frac": l2 / t / L2_ATOMIC_PEAK_OPS,
            "unit": "operations/s",
            "source": "rocprofv3 counters of the same kernel source and tile (profiles/), rates over this run's "
                      "push time"}


def measure_copy_gbs(torch, nbytes=512 << 20, reps=20):
    """Device-to-device copy rate (bytes read + bytes written per second) of
    the runtime's plain copy on a buffer larger than the last-level cache:
    the practical HBM ceiling the roofline is also compared against."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def with_copy(roof, copy_gbs):
    roof = dict(roof)
    roof["copy_gbs"] = copy_gbs
    roof["frac_of_copy"] = roof["achieved"] / copy_gbs
    return roof


def run_path(precision, w, state, steps, warmup, tile, torch, pusher="boris", c_light=0.0, walls=False):
    from paper_2608_15249_amd.sim import Simulation
    sim = Simulation(w, precision, state=state, tile=tile, pusher=pusher, c_light=c_light, walls=walls)
    sim.initialise()
    sim.ctx.sync()
    # the warm-up steps start from the seeded state: their field energies are
    # compared with the oracle's (cpu_baseline leg) for the field-energy error
    warm_we = []
    if warmup:
        dw = sim.run(warmup, diag=True)
        warm_we = [float(v) for v in dw.cpu().numpy().reshape(warmup, 4)[:, 1]]
    sim.ctx.sync()
    n = sim.n
    n_start = int(sim.p.bucket_start[-1].item()) if walls else n
    diag = torch.zeros(steps * 4, dtype=torch.float64, device="cuda")
    # the timed run records HIP events around the push pass only, on one step
    # in PROF_EVERY (each event makes the queue drain between kernels, about
    # 6 us a side at 1024^2)
    sim.ctx.profile_phases(False)
    sim.ctx.profile_every(PROF_EVERY)
    sim.ctx.profile_enable(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.ctx.step(sim.p, sim.E, sim.E32, steps, diag)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.ctx.sync()
    ms_t, nprof_t = sim.ctx.profile_read()
    sim.ctx.profile_enable(0)
    sim.ctx.profile_every(1)
    elapsed = t1 - t0
    sb = state_bytes(precision, w.dim, w.vdim)
    push_ms = ms_t[2] / max(nprof_t, 1)
    d = diag.cpu().numpy().reshape(steps, 4)
    ms, nprof = phase_breakdown(sim.ctx, lambda k, dg: sim.ctx.step(sim.p, sim.E, sim.E32, k, dg), steps)
    push_bytes = 2 * sb * n
    achieved = push_bytes / (push_ms * 1e-3) / 1e9
    # counters were taken for the Boris kernels only
    traffic = load_traffic(precision, "%s_%d" % (w.name, w.nx), list(sim.tile)) \
        if pusher == "boris" and not walls else None
    counters = load_counters(precision, "%s_%d" % (w.name, w.nx), list(sim.tile)) \
        if pusher == "boris" and not walls else None
    # particle pushes of the timed steps: with absorbing walls the count falls
    # (diag charge = q_macro * live count after each step)
    pushes = n * steps
    if walls:
        live = [int(round(v)) for v in d[:, 0] / sim.ctx.q_macro]
        pushes = n_start + sum(live[:-1])
    out = {
        "value": pushes / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        # the fused step's algorithmic bytes (state read + written once) over the step time
        "hbm_gbs_step": (2 * sb * n * steps) / elapsed / 1e9,
        "tile": list(sim.tile),
        "tune_ms_per_step": sim.tune_ms,
        "phase_ms_per_step": {"count": ms[0] / nprof, "scan": ms[1] / nprof, "push": ms[2] / nprof,
                              "field": ms[3] / nprof, "note": PHASE_NOTE % nprof},
        # particle-steps/s of the fused push kernel alone and of the whole
        # particle part of the step (tallies + scan + push), field excluded
        "particle_steps_s_by_phase": {"push": n / (push_ms * 1e-3),
                                      "count+scan+push": n / ((ms[0] + ms[1] + ms[2]) / nprof * 1e-3)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if traffic is None else traffic / (push_ms * 1e-3) / 1e9,
                     "kernel": "k_step_push (gather+%s+move+deposit+scatter)" % ("Higuera-Cary" if pusher == "hc" else "Boris"),
                     "bytes_per_launch": push_bytes,
                     "atomics": atomics_of(counters, n, push_ms)},
        "final_WE": float(d[-1, 1]),
        "charge": float(d[-1, 0]),
        "warmup_WE": warm_we,
        "push_ms": push_ms,
        "n": n,
        "exact_charge": list(sim.ctx.charge_exact()) if sim.mixed else None,
    }
    if walls:
        out["live_particles"] = {"start": n_start, "end": live[-1]}
    del sim
    torch.cuda.empty_cache()
    return out


def run_em(precision, w, state, steps, warmup, tile, c_light, torch):
    """Electromagnetic cycle (2D3V, Yee grid) on the plasma of w."""
    from paper_2608_15249_amd import workloads as W
    from paper_2608_15249_amd.apic import Context, Particles
    x, y, vx, vy, vz = state
    n = len(x)
    ctx = Context(dim=2, vdim=3, nx=w.nx, ny=w.ny, lx=w.Lx, ly=w.Ly, dt=w.dt, n=n, bz=w.bz, precision=precision,
                  tile=(0, 0) if tile in (None, "auto") else tile, c_light=c_light, model="em")
    p = Particles(ctx)
    if ctx.mixed:
        ix, ox = W.to_cell_offset(x, w.dx, w.nx)
        iy, oy = W.to_cell_offset(y, w.dy, w.ny)
        p.upload(cell=W.pack_cell(ix, iy), ox=ox, oy=oy, vx=vx, vy=vy, vz=vz)
    else:
        p.upload(x=x, y=y, vx=vx, vy=vy, vz=vz)
    ctx.sort_by_cell(p)
    F = torch.zeros(6 * ctx.G, dtype=torch.float64, device="cuda")
    ctx.em_init_fields(p, F)
    ctx.em_gather_push(p, F, dt_scale=-0.5, move=False)
    if warmup:
        ctx.em_step(p, F, warmup)
    ctx.sync()
    diag = torch.zeros(steps * 4, dtype=torch.float64, device="cuda")
    ctx.profile_phases(False)
    ctx.profile_every(PROF_EVERY)
    ctx.profile_enable(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.em_step(p, F, steps, diag=diag)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.sync()
    ms_t, nprof_t = ctx.profile_read()
    ctx.profile_enable(0)
    ctx.profile_every(1)
    elapsed = t1 - t0
    sb = state_bytes(precision, 2, 3)
    push_ms = ms_t[2] / max(nprof_t, 1)
    push_bytes = 2 * sb * n
    achieved = push_bytes / (push_ms * 1e-3) / 1e9
    d = diag.cpu().numpy().reshape(steps, 4)
    ms, nprof = phase_breakdown(ctx, lambda k, dg: ctx.em_step(p, F, k, diag=dg), steps)
    out = {
        "value": n * steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "hbm_gbs_step": (2 * sb * n * steps) / elapsed / 1e9,
        "tile": list(ctx.tile),
        "phase_ms_per_step": {"count": ms[0] / nprof, "scan": ms[1] / nprof, "push": ms[2] / nprof,
                              "field": ms[3] / nprof, "note": PHASE_NOTE % nprof},
        "particle_steps_s_by_phase": {"push": n / (push_ms * 1e-3),
                                      "count+scan+push": n / ((ms[0] + ms[1] + ms[2]) / nprof * 1e-3)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_step_push, electromagnetic form (staggered gather+Boris+move+Esirkepov "
                               "current+scatter)",
                     "bytes_per_launch": push_bytes},
        "final_W_B": float(d[-1, 0]),
        "final_W_E": float(d[-1, 1]),
        "final_KE": float(d[-1, 2]),
    }
    del ctx, p, F
    torch.cuda.empty_cache()
    return out


def cpu_baseline_em(w, state, nsteps, c_light, max_particles=1 << 22):
    """Serial FP64 electromagnetic oracle (host, one core) on a bounded sample
    of the same plasma: the first max_particles particles of the state on the
    full grid (the rate per particle-step is what is reported)."""
    import oracle as O
    from oracle import em as M
    x, y, vx, vy, vz = (a[:max_particles] for a in state)
    s = O.Setup(2, 3, w.nx, w.Lx, len(x), w.dt, ny=w.ny, Ly=w.Ly, bz=w.bz, c=c_light)
    st = O.State.from_arrays(x, vx, y, vy, vz)
    F = M.initialise(s, st)
    t0 = time.perf_counter()
    for _ in range(nsteps):
        M.step(s, st, F)
    t1 = time.perf_counter()
    return {"value": len(x) * nsteps / (t1 - t0), "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": "first %d of the %d particles on the full %s grid, %d electromagnetic oracle steps (serial C "
                      "particle loops + numpy Yee update, FP64), %.1f s" % (len(x), len(state[0]),
                                                                             "x".join(str(v) for v in _grid(w)),
                                                                             nsteps, t1 - t0)}


def cpu_baseline_walls(w, state, nsteps, max_particles=1 << 24):
    """Serial FP64 oracle of the plasma between absorbing walls (host, numpy)
    on a bounded sample: the first max_particles particles on the full grid."""
    from oracle import bounded as B
    x, y, vx, vy = (a[:max_particles] for a in state[:4])
    b = B.Box(w.nx, w.Lx, w.ny, w.Ly, len(x), w.dt, bz=w.bz, vdim=2)
    p = B.Plasma(x.copy(), y.copy(), [vx.copy(), vy.copy()])
    E = B.initialise(b, p)
    t0 = time.perf_counter()
    pushes = 0
    for _ in range(nsteps):
        pushes += len(p.x)
        E, _, _ = B.step(b, p, E)
    t1 = time.perf_counter()
    return {"value": pushes / (t1 - t0), "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": "first %d of the %d particles on the full %s grid between the walls, %d oracle steps "
                      "(numpy, FP64), %.1f s" % (len(x), len(state[0]), "x".join(str(v) for v in _grid(w)), nsteps,
                                                 t1 - t0)}


def run_batch(reps, steps, warmup, chunk, torch):
    """The batched replicas: one graph-replayed persistent launch per step on
    torch's current stream, timed with HIP events on that stream."""
    from paper_2608_15249_amd.sim import BatchSimulation
    bs = BatchSimulation(reps, chunk=chunk)
    bs.initialise()
    if warmup:
        bs.run(warmup, diag=False)
    bs.batch.sync()
    n = bs.batch.n_total
    diag = torch.zeros(steps * len(reps) * 4, dtype=torch.float64, device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    bs.batch.step(steps, diag, use_graph=True)
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    bs.batch.sync()
    kern_ms = ev0.elapsed_time(ev1) / steps
    elapsed = t1 - t0
    sb = state_bytes("mixed", 1, 1)
    launch_bytes = 2 * sb * n
    achieved = launch_bytes / (kern_ms * 1e-3) / 1e9
    out = {
        "value": n * steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "hbm_gbs_step": launch_bytes * steps / elapsed / 1e9,
        "chunk": bs.chunk,
        "tune_ms_per_step": bs.tune_ms,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_batch<step> (gather+Boris+move+deposit+field, all replicas)",
                     "bytes_per_launch": launch_bytes},
        "particles": n,
    }
    del bs
    torch.cuda.empty_cache()
    return out


def cpu_model():
    """Model name of the host CPU, from /proc/cpuinfo."""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.lower().startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores():
    """Cores this process may run on, at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_steps(w, state, nsteps, pusher, c_light, record_we=False):
    """The serial FP64 oracle from the seeded state: initialise, then nsteps
    steps; returns (seconds of the steps, W_E after each step)."""
    import oracle as O
    if w.dim == 3:
        x, y, z, vx, vy, vz = state
    else:
        (x, y, vx, vy, vz), z = state, None
    s = O.Setup(w.dim, w.vdim, w.nx, w.Lx, len(x), w.dt, ny=w.ny, Ly=w.Ly, bz=w.bz, nz=w.nz, Lz=w.Lz, pusher=pusher,
                c=c_light)
    st = O.State.from_arrays(x, vx, y, vy, vz, z)
    E, _ = O.initialise(s, st)
    we = []
    t0 = time.perf_counter()
    for _ in range(nsteps):
        E, _, _ = O.step(s, st, E)
        if record_we:
            we.append(O.field_energy(s, E))
    return time.perf_counter() - t0, we


_FORK_JOB = None   # (workload, state, steps, pusher, c) handed to forked workers by inheritance


def _oracle_worker(_):
    w, state, nsteps, pusher, c_light = _FORK_JOB
    sec, _ = _oracle_steps(w, state, nsteps, pusher, c_light)
    return sec


def cpu_baseline(w, state, nsteps, pusher="boris", c_light=float("inf"), record_we=False, all_cores=True):
    """Serial FP64 oracle on the same plasma (host, one core), then the same
    oracle in one process per host core, each advancing its own copy of the
    plasma (the aggregate host throughput). With record_we, the oracle's
    field energy after each step goes to "_we" (for field_energy_errors)."""
    sec, we = _oracle_steps(w, state, nsteps, pusher, c_light, record_we=record_we)
    n = len(state[0])
    out = {"value": n * nsteps / sec, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": "full %s / %d-particle plasma, %d oracle steps (serial C particle loops + numpy FFT, "
                     "FP64), %.1f s" % ("x".join(str(v) for v in _grid(w)), n, nsteps, sec)}
    if all_cores:
        import multiprocessing as mp
        P = host_cores()
        k = max(1, nsteps // 3)
        global _FORK_JOB
        _FORK_JOB = (w, state, k, pusher, c_light)
        ctx = mp.get_context("fork")
        t0 = time.perf_counter()
        with ctx.Pool(P) as pool:
            secs = pool.map(_oracle_worker, range(P), chunksize=1)
        wall = time.perf_counter() - t0
        _FORK_JOB = None
        out["all_cores"] = {"value": P * n * k / max(secs), "unit": "particle-steps/s", "cores": P,
                            "kind": "oracle, one process per core",
                            "sample": "%d processes, each the full plasma for %d oracle steps (slowest %.1f s, "
                                      "%.1f s wall with set-up)" % (P, k, max(secs), wall)}
    if record_we:
        out["_we"] = we
    return out


def field_energy_errors(gpu_we, we):
    """Relative field-energy difference of each GPU path from the FP64 oracle,
    both started from the same seeded state (the GPU's warm-up steps): after
    the first step (the local error of one step) and the largest over the
    steps both ran (the trajectories then separate at the rate the plasma's
    noise grows)."""
    fe = {}
    for path, g in gpu_we.items():
        m = min(len(g), len(we))
        if m == 0:
            continue
        rel = [abs(g[i] - we[i]) / we[i] for i in range(m)]
        fe[path] = {"first_step": rel[0], "max": max(rel), "steps": m}
    return fe


def _grid(w):
    return [w.nx, w.ny, w.nz] if w.dim == 3 else [w.nx, w.ny]


def cpu_baseline_batch(reps, nsteps, target_particles=3_000_000):
    """Serial FP64 oracle on the first replicas of the ensemble (about
    target_particles particles in all), each advanced nsteps steps."""
    import oracle as O
    from paper_2608_15249_amd import workloads as W
    done, tot, used = 0, 0.0, 0
    for rep in reps:
        if done >= target_particles:
            break
        w = W.replica_workload(rep)
        x, _, vx, _, _ = W.sample(w)
        s = O.Setup(1, 1, w.nx, w.Lx, len(x), w.dt)
        st = O.State.from_arrays(x, vx)
        E, _ = O.initialise(s, st)
        t0 = time.perf_counter()
        for _ in range(nsteps):
            E, _, _ = O.step(s, st, E)
        tot += time.perf_counter() - t0
        done += len(x)
        used += 1
    return {"value": done * nsteps / tot, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": "first %d replicas (%d particles), %d oracle steps each (serial C particle loops + numpy "
                      "FFT, FP64), %.1f s" % (used, done, nsteps, tot)}


def parse_tile(t):
    if t == "auto":
        return "auto"
    return tuple(int(v) for v in t.lower().split("x"))


WORKLOADS = {
    "thermal_2d": "thermal_2d: 2D2V Maxwellian plasma, 512x512 cells, 64/cell, 16,777,216 electrons, dt=0.1, CIC, "
                  "periodic FFT Poisson",
    "magnetized_2d3v": "magnetized_2d3v: 2D3V Maxwellian plasma in uniform B_z (omega_c/omega_p=2), 1024x1024 cells, "
                       "32/cell, 33,554,432 electrons, 1% density perturbation at k=(2pi/64,0), dt=0.05, CIC, "
                       "periodic FFT Poisson",
    "thermal_3d": "thermal_3d: 3D3V Maxwellian plasma, 128x128x128 cells, 8/cell, 16,777,216 electrons, dt=0.1, "
                  "CIC (8 nodes), periodic FFT Poisson (7-point)",
    "landau_batch": "landau_batch: 256 independent 1D1V Landau-damping replicas, Nx log-uniform in [32,512], "
                    "particles log-uniform in [1e4,1e6], Maxwellian v_th=1, k=0.5 perturbation, dt=0.1, CIC",
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--paths", default="mixed,fp64")
    ap.add_argument("--workload", default="magnetized_2d3v", choices=sorted(WORKLOADS))
    ap.add_argument("--also", default=None,
                    help="comma-separated extra single-plasma workloads measured the same way (both paths) and "
                         "reported under their names; default thermal_2d with the default workload, none otherwise")
    ap.add_argument("--tile", default="auto", help="sort-bucket tile TXxTY (TXxTYxTZ in 3D), or auto (autotuner; the default tile in 3D)")
    ap.add_argument("--chunk", default="auto", help="batch work-item size, or auto (autotuner)")
    ap.add_argument("--pusher", default="boris", choices=("boris", "hc"),
                    help="velocity advance: Boris, or Higuera-Cary (relativistic, u = gamma v; 3V workloads)")
    ap.add_argument("--c-light", type=float, default=None,
                    help="speed of light in v_th units (--pusher hc: default 8; --model em: default 10)")
    ap.add_argument("--walls", action="store_true",
                    help="grounded absorbing walls at x = 0 and x = Lx (2D electrostatic workloads)")
    ap.add_argument("--model", default="es", choices=("es", "em"),
                    help="field model: electrostatic (Poisson), or electromagnetic (Yee FDTD with Esirkepov "
                         "current; FP64 2D3V, magnetized_2d3v)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (N=%d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2608_15249_amd import workloads as W
    common = {"metric": "particle-steps/s (sort+deposit+gather+push), HBM GB/s; mixed vs FP64 path",
              "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "data": "synthetic"}
    if args.workload == "landau_batch":
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        reps = W.landau_batch()
        chunk = args.chunk if args.chunk == "auto" else int(args.chunk)
        print("bench: landau_batch, %d replicas, %d warmup + %d timed steps" % (len(reps), args.warmup, args.steps),
              file=sys.stderr, flush=True)
        b = run_batch(reps, args.steps, args.warmup, chunk, torch)
        copy_gbs = measure_copy_gbs(torch)
        line = dict(common)
        line.update({"value": b["value"], "ms_per_step": b["ms_per_step"], "dtype": "f32+i64",
                     "config": {"workload": WORKLOADS["landau_batch"], "replicas": len(reps),
                                "particles": b["particles"], "chunk": b["chunk"], "precision": "mixed"},
                     "hbm_gbs_step": b["hbm_gbs_step"], "roofline": with_copy(b["roofline"], copy_gbs),
                     "tune_ms_per_step": b["tune_ms_per_step"]})
        if not args.no_cpu_baseline:
            print("bench: cpu baseline (%d oracle steps per replica)" % args.cpu_steps, file=sys.stderr, flush=True)
            line["cpu_baseline"] = cpu_baseline_batch(reps, args.cpu_steps)
        print(json.dumps(line), flush=True)
        return
    w = getattr(W, args.workload)()
    state = W.sample3(w) if w.dim == 3 else W.sample(w)
    tile = parse_tile(args.tile)
    if args.model == "em":
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        if w.dim != 2 or w.vdim != 3:
            print("--model em needs a 2D3V workload (magnetized_2d3v)", file=sys.stderr)
            sys.exit(2)
        c_light = 10.0 if args.c_light is None else args.c_light
        res = {}
        for path in args.paths.split(","):
            print("bench: %s, electromagnetic %s path, %d warmup + %d timed steps" % (args.workload, path,
                                                                                     args.warmup, args.steps),
                  file=sys.stderr, flush=True)
            res[path] = run_em(path, w, state, args.steps, args.warmup, tile, c_light, torch)
        copy_gbs = measure_copy_gbs(torch)
        r = res.get("mixed") or res[list(res)[0]]
        line = dict(common)
        line.update({"value": r["value"], "ms_per_step": r["ms_per_step"],
                     "dtype": "f32+f64" if "mixed" in res else "f64",
                     "config": {"workload": WORKLOADS[args.workload] + "; electromagnetic (Yee FDTD, c=%g)" % c_light,
                                "grid": _grid(w), "particles": w.n_particles, "tile": r["tile"],
                                "precision": "mixed" if "mixed" in res else "fp64", "model": "electromagnetic"},
                     "hbm_gbs_step": r["hbm_gbs_step"], "roofline": with_copy(r["roofline"], copy_gbs),
                     "phase_ms_per_step": r["phase_ms_per_step"],
                     "particle_steps_s_by_phase": r["particle_steps_s_by_phase"],
                     "final_energies": {"W_B": r["final_W_B"], "W_E": r["final_W_E"], "KE": r["final_KE"]}})
        if "fp64" in res and "mixed" in res:
            f = res["fp64"]
            line["fp64"] = {"value": f["value"], "ms_per_step": f["ms_per_step"], "tile": f["tile"],
                            "roofline": with_copy(f["roofline"], copy_gbs), "phase_ms_per_step": f["phase_ms_per_step"],
                            "final_energies": {"W_B": f["final_W_B"], "W_E": f["final_W_E"], "KE": f["final_KE"]}}
            line["mixed_over_fp64"] = r["value"] / f["value"]
        if not args.no_cpu_baseline:
            print("bench: cpu baseline (%d oracle steps)" % args.cpu_steps, file=sys.stderr, flush=True)
            line["cpu_baseline"] = cpu_baseline_em(w, state, min(args.cpu_steps, 3), c_light)
        print(json.dumps(line), flush=True)
        return
    if args.walls and (w.dim != 2 or args.pusher != "boris"):
        print("--walls needs a 2D workload with the Boris advance", file=sys.stderr)
        sys.exit(2)
    if args.pusher == "hc" and w.vdim != 3:
        print("--pusher hc needs a 3V workload (magnetized_2d3v or thermal_3d)", file=sys.stderr)
        sys.exit(2)
    c_light = (8.0 if args.c_light is None else args.c_light) if args.pusher == "hc" else 0.0
    # the oracle legs run first, on the host, before this process touches the
    # GPU (the all-core leg forks one process per core)
    cpu = None
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (%d oracle steps, then all host cores)" % args.cpu_steps, file=sys.stderr,
              flush=True)
        if args.walls:
            cpu = cpu_baseline_walls(w, state, min(args.cpu_steps, 6))
        else:
            cpu = cpu_baseline(w, state, args.cpu_steps, args.pusher,
                               c_light if args.pusher == "hc" else float("inf"), record_we=args.warmup > 0)
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    res = {}
    for path in args.paths.split(","):
        print("bench: %s, %s path, %d warmup + %d timed steps" % (args.workload, path, args.warmup, args.steps),
              file=sys.stderr, flush=True)
        res[path] = run_path(path, w, state, args.steps, args.warmup, tile, torch, args.pusher, c_light, args.walls)
    copy_gbs = measure_copy_gbs(torch)
    head = res.get("mixed") or res[list(res)[0]]
    line = dict(common)
    line.update({
        "value": head["value"],
        "ms_per_step": head["ms_per_step"],
        "dtype": "f32+i64" if "mixed" in res else "f64",
        "config": {"workload": WORKLOADS[args.workload], "grid": _grid(w), "particles": w.n_particles,
                   "tile": head["tile"], "precision": "mixed" if "mixed" in res else "fp64",
                   "pusher": "higuera-cary" if args.pusher == "hc" else "boris",
                   "boundaries": "grounded absorbing walls in x" if args.walls else "periodic"},
        "hbm_gbs_step": head["hbm_gbs_step"],
        "roofline": with_copy(head["roofline"], copy_gbs),
        "phase_ms_per_step": head["phase_ms_per_step"],
        "particle_steps_s_by_phase": head["particle_steps_s_by_phase"],
        "tune_ms_per_step": head["tune_ms_per_step"],
    })
    if head.get("exact_charge") is not None:
        line["exact_charge"] = {"whole": head["exact_charge"][0], "frac": head["exact_charge"][1],
                                "particles": head["n"],
                                "note": "the last step's fixed-point node sums, totalled exactly on the device"}
    if "live_particles" in head:
        line["live_particles"] = head["live_particles"]
    if "fp64" in res and "mixed" in res:
        f = res["fp64"]
        line["fp64"] = {"value": f["value"], "ms_per_step": f["ms_per_step"], "hbm_gbs_step": f["hbm_gbs_step"],
                        "tile": f["tile"], "roofline": with_copy(f["roofline"], copy_gbs),
                        "phase_ms_per_step": f["phase_ms_per_step"],
                        "particle_steps_s_by_phase": f["particle_steps_s_by_phase"]}
        line["mixed_over_fp64"] = head["value"] / f["value"]
    if cpu is not None:
        we = cpu.pop("_we", None)
        if we:
            cpu["field_energy_err"] = field_energy_errors({p: r["warmup_WE"] for p, r in res.items()}, we)
            line["field_energy_err"] = cpu["field_energy_err"]
        line["cpu_baseline"] = cpu
    del res
    # the other workloads of the default run, measured the same way (both paths)
    also = args.also if args.also is not None else ("thermal_2d" if args.workload == "magnetized_2d3v" and
                                                      not args.walls and args.pusher == "boris" else "")
    for name in [a for a in also.split(",") if a]:
        w2 = getattr(W, name)()
        st2 = W.sample3(w2) if w2.dim == 3 else W.sample(w2)
        ex = {"config": {"workload": WORKLOADS[name], "grid": _grid(w2), "particles": w2.n_particles}}
        for path in args.paths.split(","):
            print("bench: %s, %s path, %d warmup + %d timed steps" % (name, path, args.warmup, args.steps),
                  file=sys.stderr, flush=True)
            r = run_path(path, w2, st2, args.steps, args.warmup, "auto", torch)
            ex[path] = {"value": r["value"], "ms_per_step": r["ms_per_step"], "tile": r["tile"],
                        "hbm_gbs_step": r["hbm_gbs_step"], "roofline": with_copy(r["roofline"], copy_gbs),
                        "phase_ms_per_step": r["phase_ms_per_step"],
                        "particle_steps_s_by_phase": r["particle_steps_s_by_phase"]}
        line[name] = ex
        del st2
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
