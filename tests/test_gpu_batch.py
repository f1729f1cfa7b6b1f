"""Batched replicas (apic_batch_*): parity with the single-plasma path and the
oracle, graph replay, determinism and Landau damping of the ensemble."""
import numpy as np
import pytest

import oracle as O
from oracle import dispersion as D
from oracle import mixed as OM
from paper_2608_15249_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return t


# uneven replicas: grid sizes not powers of two, particle counts with ragged chunks
REPS = [W.Replica(32, 3001, 0.03, 500), W.Replica(61, 20011, 0.05, 501), W.Replica(173, 50003, 0.02, 502),
        W.Replica(512, 10007, 0.04, 503), W.Replica(100, 257, 0.01, 504)]


def _sorted_rows(c, o, v):
    idx = np.lexsort((v.view(np.uint32), o.view(np.uint32), c))
    return c[idx], o[idx], v[idx]


def test_batch_replica_equals_single_run(torch):
    """Each replica advanced in the batch gives the bits the same plasma gives
    through the single-plasma entry points (sorted there, unsorted here, so
    the particle sets are compared)."""
    from paper_2608_15249_amd.sim import BatchSimulation, Simulation
    nsteps = 6
    bs = BatchSimulation(REPS, chunk=2048)
    bs.initialise()
    dg = bs.run(nsteps)
    bs.batch.sync()
    dg = dg.cpu().numpy().reshape(nsteps, len(REPS), 4)
    for r, rep in enumerate(REPS):
        w = W.replica_workload(rep)
        sim = Simulation(w, "mixed")
        sim.initialise()
        d1 = sim.run(nsteps)
        sim.ctx.sync()
        assert np.array_equal(bs.replica_field(r), sim.field()[0]), r
        c, o, v = bs.replica_state(r)
        st = sim.state()
        a = _sorted_rows(c, o, v)
        b = _sorted_rows(st["cell"], st["ox"], st["vx"])
        for x, y in zip(a, b):
            assert np.array_equal(x, y), r
        d1 = d1.cpu().numpy().reshape(nsteps, 4)
        assert np.array_equal(dg[:, r, :2], d1[:, :2]), r         # charge, field energy: same order
        assert np.allclose(dg[:, r, 2:], d1[:, 2:], rtol=1e-12, atol=1e-14), r


def test_batch_init_and_step_match_oracle(torch):
    """E^0 of every replica against the oracle's field of the fixed-point
    deposit; the half push and one step bit-exact against the oracle's
    binary32 push driven by the binary32 rounding of the oracle's own field."""
    from paper_2608_15249_amd.sim import BatchSimulation
    states = []
    for rep in REPS:
        w = W.replica_workload(rep)
        x, _, vx, _, _ = W.sample(w)
        states.append((x, vx))
    bs = BatchSimulation(REPS, chunk=4096, states=states)
    # reference inputs (oracle side): the same seeded state
    ref = []
    for rep, (x, vx) in zip(REPS, states):
        w = W.replica_workload(rep)
        s = O.Setup(1, 1, w.nx, w.Lx, w.n_particles, w.dt)
        ix, ox = W.to_cell_offset(x, w.dx, w.nx)
        I = O.deposit_quantised(s, ix, ox, 32)
        (E0,) = O.solve_field(s, O.rho_from_quantised(s, I, 32))
        st = {"ix": ix, "iy": None, "ox": ox, "oy": None, "vx": vx.astype(np.float32), "vy": None, "vz": None}
        ref.append((w, s, E0, st))
    bs.initialise()
    bs.batch.sync()
    for r, (w, s, E0, st) in enumerate(ref):
        Eg = bs.replica_field(r)
        assert np.max(np.abs(Eg - E0)) <= 1e-12 * np.max(np.abs(E0)), r
        assert np.array_equal(Eg.astype(np.float32), E0.astype(np.float32)), r
        half = OM.push(st, (E0.astype(np.float32),), dim=1, vdim=1, nx=w.nx, ny=1, dx=w.dx, dy=1.0, qm=-1.0,
                       dt=w.dt, bz=0.0, dt_scale=-0.5, move=False)
        c, o, v = bs.replica_state(r)
        assert np.array_equal(v, half["vx"]), r
        assert np.array_equal(c, st["ix"]) and np.array_equal(o, st["ox"]), r
        ref[r] = (w, s, E0, half)
    rho = torch.zeros(bs.batch.g_total, dtype=torch.int64, device="cuda")
    bs.run(1, rho=rho)
    bs.batch.sync()
    rho = rho.cpu().numpy()
    for r, (w, s, E0, half) in enumerate(ref):
        new = OM.push(half, (E0.astype(np.float32),), dim=1, vdim=1, nx=w.nx, ny=1, dx=w.dx, dy=1.0, qm=-1.0,
                      dt=w.dt, bz=0.0)
        c, o, v = bs.replica_state(r)
        assert np.array_equal(c, new["ix"]) and np.array_equal(o, new["ox"]) and np.array_equal(v, new["vx"]), r
        I1 = O.deposit_quantised(s, new["ix"], new["ox"], 32)
        g0, g1 = bs.batch.grid_off[r], bs.batch.grid_off[r + 1]
        assert np.array_equal(rho[g0:g1], I1), r
        (E1,) = O.solve_field(s, O.rho_from_quantised(s, I1, 32))
        assert np.max(np.abs(bs.replica_field(r) - E1)) <= 1e-12 * np.max(np.abs(E1)), r


def test_batch_graph_replay_equals_direct_launches(torch):
    from paper_2608_15249_amd.sim import BatchSimulation
    out = []
    for use_graph in (True, False):
        bs = BatchSimulation(REPS, chunk=2048)
        bs.initialise()
        d = bs.run(8, use_graph=use_graph)
        d2 = bs.run(3, use_graph=use_graph)   # a second call replays the captured graph
        bs.batch.sync()
        out.append((bs.batch.E.cpu().numpy(), bs.batch.vx.cpu().numpy(), bs.batch.ox.cpu().numpy(),
                    d.cpu().numpy(), d2.cpu().numpy()))
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_batch_landau_damping(torch):
    """Seeded k = 0.5 mode in 1D Maxwellian replicas damps at the Landau rate
    and oscillates at the Bohm-Gross/Landau frequency of the kinetic root."""
    from paper_2608_15249_amd.sim import BatchSimulation
    reps = [W.Replica(64, 1_000_000, 0.05, 600 + r) for r in range(3)]
    bs = BatchSimulation(reps, chunk=8192)
    bs.initialise()
    amps = [[] for _ in reps]
    nsteps = 160
    for n in range(nsteps):
        E = bs.batch.E.cpu().numpy()
        for r in range(len(reps)):
            e = E[bs.batch.grid_off[r]:bs.batch.grid_off[r + 1]]
            amps[r].append(2 * abs(np.fft.fft(e)[1]) / len(e))
        bs.run(1, diag=False)
    bs.batch.sync()
    th = D.two_stream_root(0.5, 0.5, 0.0, 1.0, 1.4 - 0.15j)
    t = np.arange(nsteps) * 0.1
    for r in range(len(reps)):
        a = np.array(amps[r])
        pk = [i for i in range(1, nsteps - 1) if a[i] > a[i - 1] and a[i] >= a[i + 1] and t[i] < 15]
        gam = np.polyfit(t[pk], np.log(a[pk]), 1)[0]
        om = np.pi / np.mean(np.diff(t[pk]))
        assert abs(gam / th.imag - 1) < 0.12, (r, gam, th)
        assert abs(om / th.real - 1) < 0.03, (r, om, th)


def test_batch_autotune_chunk_picks_a_candidate_and_keeps_results(torch):
    """The tuner returns one of its candidates, caches it, and the batch built
    with the pick gives the same particle and field bits as any other chunk."""
    from paper_2608_15249_amd.sim import BatchSimulation
    a = BatchSimulation(REPS, chunk="auto")
    assert a.chunk in (1024, 2048, 4096, 8192, 16384, 32768, 65535)
    assert a.tune_ms is not None and a.tune_ms > 0
    again = BatchSimulation(REPS, chunk="auto")
    assert again.chunk == a.chunk and again.tune_ms == -1.0   # process cache
    b = BatchSimulation(REPS, chunk=1024 if a.chunk != 1024 else 4096)
    for s in (a, b):
        s.initialise()
        s.run(5)
        s.batch.sync()
    for f in ("E", "cell", "ox", "vx"):
        assert torch.equal(getattr(a.batch, f), getattr(b.batch, f)), f


def test_batch_empty_replica(torch):
    """A replica with no particles (q_macro = 0: the ion background alone)
    between others: its field stays zero to rounding and its diagnostics are
    zero, and every other replica gives the bits it gives without it."""
    from paper_2608_15249_amd.sim import BatchSimulation
    nsteps = 4
    empty = W.Replica(48, 0, 0.03, 505)
    with_empty = [REPS[0], REPS[1], empty, REPS[2]]
    runs = []
    for reps in (with_empty, [REPS[0], REPS[1], REPS[2]]):
        bs = BatchSimulation(reps, chunk=2048)
        bs.initialise()
        dg = bs.run(nsteps)
        bs.batch.sync()
        runs.append((bs, dg.cpu().numpy().reshape(nsteps, len(reps), 4)))
    (a, da), (b, db) = runs
    assert np.max(np.abs(a.replica_field(2))) <= 1e-12
    assert np.array_equal(da[:, 2, [0, 2, 3]], np.zeros((nsteps, 3)))
    assert np.all(np.abs(da[:, 2, 1]) <= 1e-20)
    for ra, rb in ((0, 0), (1, 1), (3, 2)):
        assert np.array_equal(a.replica_field(ra), b.replica_field(rb)), ra
        for x, y in zip(a.replica_state(ra), b.replica_state(rb)):
            assert np.array_equal(x, y), ra
        assert np.array_equal(da[:, ra], db[:, rb]), ra
