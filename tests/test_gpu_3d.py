"""GPU parity of the 3D3V path (through the C ABI) against the CPU oracle.

Same bars as the 1D/2D parity tests: the sort order, the bucket table, the
int64 fixed-point deposit and the binary32 push of the mixed state bit-exact;
FP64 work within 1e-12 relative (double rounding of a few dozen operations
per element). Shapes cut a partial tile on every axis."""
import numpy as np
import pytest

import oracle as O
from oracle import mixed as OM
from paper_2608_15249_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2608_15249_amd import apic
    apic.load_library()
    return t


CASES = [
    # nx, ny, nz, lx, ly, lz, n, tile
    (20, 12, 9, 10.0, 6.0, 4.5, 30011, (8, 4, 4)),
    (16, 16, 16, 16.0, 16.0, 16.0, 40009, (4, 4, 4)),
]


def _ctx(torch, case, precision="fp64", bz=0.0, dt=0.1):
    from paper_2608_15249_amd.apic import Context, Particles
    nx, ny, nz, lx, ly, lz, n, tile = case
    c = Context(dim=3, vdim=3, nx=nx, ny=ny, lx=lx, ly=ly, dt=dt, n=n, bz=bz, precision=precision, tile=tile,
                nz=nz, lz=lz)
    return c, Particles(c)


def _setup(case, bz=0.0, dt=0.1):
    nx, ny, nz, lx, ly, lz, n, tile = case
    return O.Setup(3, 3, nx, lx, n, dt, ny=ny, Ly=ly, nz=nz, Lz=lz, bz=bz)


def _state(rng, case, vth=1.0):
    nx, ny, nz, lx, ly, lz, n, tile = case
    return (rng.uniform(0, lx, n), rng.uniform(0, ly, n), rng.uniform(0, lz, n),
            rng.normal(0, vth, n), rng.normal(0, vth, n), rng.normal(0, vth, n))


def _upload(p, s, st, mixed):
    x, y, z, vx, vy, vz = st
    if not mixed:
        p.upload(x=x, y=y, z=z, vx=vx, vy=vy, vz=vz)
        return None
    c = [W.to_cell_offset(a, d, n) for a, d, n in ((x, s.dx, s.nx), (y, s.dy, s.ny), (z, s.dz, s.nz))]
    p.upload(cell=W.pack_cell(c[0][0], c[1][0], c[2][0]), ox=c[0][1], oy=c[1][1], oz=c[2][1], vx=vx, vy=vy, vz=vz)
    return c


def _ostate(d):
    return O.State.from_arrays(d["x"], d["vx"], d["y"], d["vy"], d["vz"], d["z"])


def _field(E, s):
    return np.concatenate([e.ravel() for e in E])


def _mstate(d):
    ix, iy, iz = W.unpack_cell(d["cell"], 3)
    return {"ix": ix, "iy": iy, "iz": iz, "ox": d["ox"], "oy": d["oy"], "oz": d["oz"],
            "vx": d["vx"], "vy": d["vy"], "vz": d["vz"]}


def _key(case, ix, iy, iz):
    nx, ny, nz, lx, ly, lz, n, tile = case
    return O.bucket_key(ix, iy, tile[0], tile[1], nx, iz=iz, tile_z=tile[2], ny=ny)


# ------------------------------------------------------------------ sort

@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sort_by_cell_3d(torch, case, precision):
    rng = np.random.default_rng(31)
    s = _setup(case)
    st = _state(rng, case)
    c, p = _ctx(torch, case, precision)
    cells = _upload(p, s, st, precision == "mixed")
    if cells is None:
        cells = [(np.floor(a / d).astype(np.int64) % n,) for a, d, n in
                 ((st[0], s.dx, s.nx), (st[1], s.dy, s.ny), (st[2], s.dz, s.nz))]
    before = p.download()
    n = case[6]
    perm = torch.zeros(n, dtype=torch.int32, device="cuda")
    c.sort_by_cell(p, perm=perm)
    c.sync()
    after = p.download()
    pm = perm.cpu().numpy().astype(np.int64)
    for k in ("x", "y", "z", "cell", "ox", "oy", "oz", "vx", "vy", "vz"):
        if before[k] is not None:
            assert np.array_equal(after[k], before[k][pm]), k
    key = _key(case, cells[0][0], cells[1][0], cells[2][0])
    perm_ref, start = O.counting_sort(key, c.nbuckets)
    assert c.nbuckets == int(np.prod([-(-a // t) for a, t in zip(case[:3], case[7])]))
    assert np.array_equal(after["bucket_start"].astype(np.int64), start)
    assert np.array_equal(pm, perm_ref)


# --------------------------------------------------------------- deposit

@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("tiled", [False, True])
def test_deposit_fp64_3d(torch, case, tiled):
    rng = np.random.default_rng(32)
    s = _setup(case)
    c, p = _ctx(torch, case)
    _upload(p, s, _state(rng, case), False)
    if tiled:
        c.sort_by_cell(p)
    rho = torch.zeros(c.G, dtype=torch.float64, device="cuda")
    c.deposit(p, rho, tiled=tiled)
    c.sync()
    ref = O.deposit(s, _ostate(p.download()))
    got = rho.cpu().numpy().reshape(ref.shape)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("tiled", [False, True])
def test_deposit_mixed_bit_exact_3d(torch, case, tiled):
    rng = np.random.default_rng(33)
    s = _setup(case)
    st = _state(rng, case)
    c, p = _ctx(torch, case, "mixed")
    S = c.frac_bits
    assert S == 15
    cells = [W.to_cell_offset(a, d, n) for a, d, n in ((st[0], s.dx, s.nx), (st[1], s.dy, s.ny), (st[2], s.dz, s.nz))]
    # offsets at the edges of [0,1) and exact half-way rounding points on every axis
    edge = np.array([0.0, np.nextafter(np.float32(1), np.float32(0)), 0.5, 1.5 * 2.0 ** -S, 2.5 * 2.0 ** -S],
                    dtype=np.float32)
    for k in range(3):
        cells[k][1][:5] = np.roll(edge, k)
    p.upload(cell=W.pack_cell(cells[0][0], cells[1][0], cells[2][0]), ox=cells[0][1], oy=cells[1][1],
             oz=cells[2][1], vx=st[3], vy=st[4], vz=st[5])
    if tiled:
        c.sort_by_cell(p)
    I = torch.zeros(c.G, dtype=torch.int64, device="cuda")
    c.deposit(p, I, tiled=tiled)
    c.sync()
    m = _mstate(p.download())
    ref = O.deposit_quantised(s, m["ix"], m["ox"], S, m["iy"], m["oy"], m["iz"], m["oz"])
    got = I.cpu().numpy().reshape(ref.shape)
    assert np.array_equal(got, ref)
    assert sum(int(v) for v in got.ravel()) == case[6] << (3 * S)


# ----------------------------------------------------------------- field

@pytest.mark.parametrize("case", CASES)
def test_field_solve_3d(torch, case):
    rng = np.random.default_rng(34)
    s = _setup(case)
    rho = rng.normal(size=s.grid_shape)
    c, p = _ctx(torch, case)
    E = torch.zeros(3 * c.G, dtype=torch.float64, device="cuda")
    E32 = torch.zeros(3 * c.G, dtype=torch.float32, device="cuda")
    we = torch.zeros(1, dtype=torch.float64, device="cuda")
    c.field_solve(torch.from_numpy(rho.ravel().copy()).cuda(), E, E32, we)
    c.sync()
    ref = O.solve_field(s, rho)
    got = E.cpu().numpy().reshape((3,) + s.grid_shape)
    scale = max(np.max(np.abs(e)) for e in ref)
    for d_ in range(3):
        assert np.max(np.abs(got[d_] - ref[d_])) <= 1e-12 * scale, d_
    assert np.array_equal(E32.cpu().numpy(), E.cpu().numpy().astype(np.float32))
    assert abs(we.item() / O.field_energy(s, ref) - 1) < 1e-12


@pytest.mark.parametrize("case", CASES)
def test_field_solve_mixed_from_fixed_point_3d(torch, case):
    rng = np.random.default_rng(35)
    s = _setup(case)
    c, p = _ctx(torch, case, "mixed")
    cells = _upload(p, s, _state(rng, case), True)
    S = c.frac_bits
    I = O.deposit_quantised(s, cells[0][0], cells[0][1], S, cells[1][0], cells[1][1], cells[2][0], cells[2][1])
    E = torch.zeros(3 * c.G, dtype=torch.float64, device="cuda")
    c.field_solve(torch.from_numpy(I.ravel().copy()).cuda(), E)
    c.sync()
    ref = O.solve_field(s, O.rho_from_quantised(s, I, S))
    got = E.cpu().numpy().reshape((3,) + s.grid_shape)
    scale = max(np.max(np.abs(e)) for e in ref)
    for d_ in range(3):
        assert np.max(np.abs(got[d_] - ref[d_])) <= 1e-12 * scale


# ------------------------------------------------------------- gather/push

@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("tiled", [False, True])
def test_gather_push_fp64_3d(torch, case, tiled):
    rng = np.random.default_rng(36)
    s = _setup(case, bz=2.0)
    E = tuple(rng.normal(size=s.grid_shape) for _ in range(3))
    c, p = _ctx(torch, case, bz=2.0)
    _upload(p, s, _state(rng, case), False)
    if tiled:
        c.sort_by_cell(p)
    d0 = p.download()
    c.gather_push(p, torch.from_numpy(_field(E, s)).cuda(), dt_scale=1.0, move=True, tiled=tiled)
    c.sync()
    d1 = p.download()
    st = _ostate(d0)
    O.boris(s, st, O.gather(s, st, E), s.dt)
    O.move(s, st)
    for k, ref in (("vx", st.vx), ("vy", st.vy), ("vz", st.vz)):
        assert np.max(np.abs(d1[k] - ref)) <= 1e-13, k
    for k, ref, L in (("x", st.x, s.Lx), ("y", st.y, s.Ly), ("z", st.z, s.Lz)):
        dd = np.abs(d1[k] - ref)
        assert np.max(np.minimum(dd, L - dd)) <= 1e-12 * L, k


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("dt_scale", [1.0, -0.5])
def test_gather_push_mixed_bit_exact_3d(torch, case, dt_scale):
    rng = np.random.default_rng(37)
    s = _setup(case, bz=2.0)
    E32 = tuple(rng.normal(size=s.grid_shape).astype(np.float32) for _ in range(3))
    c, p = _ctx(torch, case, "mixed", bz=2.0)
    _upload(p, s, _state(rng, case, vth=3.0), True)
    c.sort_by_cell(p)
    m0 = _mstate(p.download())
    move = dt_scale == 1.0
    c.gather_push(p, torch.from_numpy(_field(E32, s)).cuda(), dt_scale=dt_scale, move=move)
    c.sync()
    m1 = _mstate(p.download())
    ref = OM.push(m0, E32, dim=3, vdim=3, nx=s.nx, ny=s.ny, dx=s.dx, dy=s.dy, qm=s.qm, dt=s.dt, bz=s.bz,
                  dt_scale=dt_scale, move=move, nz=s.nz, dz=s.dz)
    for k in ("ix", "iy", "iz", "ox", "oy", "oz", "vx", "vy", "vz"):
        assert np.array_equal(m1[k], ref[k]), k


# ------------------------------------------------------------ full steps

def _compose(ids, perm):
    return ids[perm.cpu().numpy().astype(np.int64)]


@pytest.mark.parametrize("case", CASES)
def test_step_fp64_matches_oracle_3d(torch, case):
    rng = np.random.default_rng(38)
    s = _setup(case, bz=2.0)
    st0 = _state(rng, case)
    n = case[6]
    c, p = _ctx(torch, case, bz=2.0)
    _upload(p, s, st0, False)
    perm = torch.zeros(n, dtype=torch.int32, device="cuda")
    c.sort_by_cell(p, perm=perm)
    ids = _compose(np.arange(n), perm)
    rho = torch.zeros(c.G, dtype=torch.float64, device="cuda")
    E = torch.zeros(3 * c.G, dtype=torch.float64, device="cuda")
    c.deposit(p, rho)
    c.field_solve(rho, E)
    c.gather_push(p, E, dt_scale=-0.5, move=False)
    x, y, z, vx, vy, vz = st0
    st = O.State.from_arrays(x, vx, y, vy, vz, z)
    Eo, _ = O.initialise(s, st)
    nsteps = 8
    diag = torch.zeros(nsteps * 4, dtype=torch.float64, device="cuda")
    ref_we, ref_ke = [], []
    for k in range(nsteps):
        c.step(p, E, None, 1, diag[4 * k:4 * k + 4], perm=perm)
        ids = _compose(ids, perm)
        Eo, _, ke = O.step(s, st, Eo)
        ref_we.append(O.field_energy(s, Eo))
        ref_ke.append(ke)
    c.sync()
    d = p.download()
    for k, ref in (("vx", st.vx), ("vy", st.vy), ("vz", st.vz)):
        assert np.max(np.abs(d[k] - ref[ids])) <= 1e-11, k
    for k, ref, L in (("x", st.x, s.Lx), ("y", st.y, s.Ly), ("z", st.z, s.Lz)):
        dd = np.abs(d[k] - ref[ids])
        assert np.max(np.minimum(dd, L - dd)) <= 1e-11 * L, k
    Eg = E.cpu().numpy().reshape((3,) + s.grid_shape)
    scale = max(np.max(np.abs(e)) for e in Eo)
    for d_ in range(3):
        assert np.max(np.abs(Eg[d_] - Eo[d_])) <= 1e-10 * scale
    dg = diag.cpu().numpy().reshape(nsteps, 4)
    assert np.allclose(dg[:, 1], ref_we, rtol=1e-10, atol=0)
    assert np.allclose(dg[:, 2], ref_ke, rtol=1e-12, atol=0)
    assert np.allclose(dg[:, 0], n * s.Q, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("case", CASES)
def test_step_mixed_one_step_bit_exact_3d(torch, case):
    """One mixed 3D step from a seeded state and a binary32 field: particle
    state, int64 deposit of rho^{n+1} and bucket table bit-exact against the
    oracle's binary32 push and quantised deposit; E^{n+1} within 1e-12."""
    rng = np.random.default_rng(39)
    s = _setup(case, bz=2.0)
    n = case[6]
    c, p = _ctx(torch, case, "mixed", bz=2.0)
    cells = _upload(p, s, _state(rng, case), True)
    S = c.frac_bits
    I0 = O.deposit_quantised(s, cells[0][0], cells[0][1], S, cells[1][0], cells[1][1], cells[2][0], cells[2][1])
    E0 = O.solve_field(s, O.rho_from_quantised(s, I0, S))
    E32 = tuple(e.astype(np.float32) for e in E0)
    perm = torch.zeros(n, dtype=torch.int32, device="cuda")
    c.sort_by_cell(p, perm=perm)
    ids = _compose(np.arange(n), perm)
    m0 = _mstate(p.download())
    Ed = torch.from_numpy(_field(E0, s)).cuda()
    E32d = torch.from_numpy(_field(E32, s)).cuda()
    Iout = torch.zeros(c.G, dtype=torch.int64, device="cuda")
    c.step(p, Ed, E32d, 1, None, rho=Iout, perm=perm)
    c.sync()
    ref = OM.push(m0, E32, dim=3, vdim=3, nx=s.nx, ny=s.ny, dx=s.dx, dy=s.dy, qm=s.qm, dt=s.dt, bz=s.bz,
                  nz=s.nz, dz=s.dz)
    pm = perm.cpu().numpy().astype(np.int64)
    m1 = _mstate(p.download())
    for k in ("ix", "iy", "iz", "ox", "oy", "oz", "vx", "vy", "vz"):
        assert np.array_equal(m1[k], ref[k][pm]), k
    I1 = O.deposit_quantised(s, ref["ix"], ref["ox"], S, ref["iy"], ref["oy"], ref["iz"], ref["oz"])
    assert np.array_equal(Iout.cpu().numpy().reshape(I1.shape), I1)
    _, start = O.counting_sort(_key(case, ref["ix"], ref["iy"], ref["iz"]), c.nbuckets)
    assert np.array_equal(p.download()["bucket_start"].astype(np.int64), start)
    E1 = O.solve_field(s, O.rho_from_quantised(s, I1, S))
    Eg = Ed.cpu().numpy().reshape((3,) + s.grid_shape)
    scale = max(np.max(np.abs(e)) for e in E1)
    for d_ in range(3):
        assert np.max(np.abs(Eg[d_] - E1[d_])) <= 1e-12 * scale
    del ids


def test_step_deterministic_3d(torch):
    """Two mixed 3D runs from the same input: identical bits everywhere."""
    from paper_2608_15249_amd.sim import Simulation
    w = W.thermal_3d(seed=8, nx=24, ppc=16)
    outs = []
    for _ in range(2):
        sim = Simulation(w, "mixed", tile=(8, 8, 4))
        sim.initialise()
        d = sim.run(8)
        sim.ctx.sync()
        outs.append((sim.E.cpu().numpy(), d.cpu().numpy(), sim.state()))
    (E1, d1, s1), (E2, d2, s2) = outs
    assert np.array_equal(E1, E2) and np.array_equal(d1, d2)
    for k in ("cell", "ox", "oy", "oz", "vx", "vy", "vz", "bucket_start"):
        assert np.array_equal(s1[k], s2[k]), k


def test_autotuned_tile_3d_gives_the_same_plasma(torch):
    """apic_autotune_tiles in 3D picks one of its candidate tiles (or the
    default), caches the pick, and eight mixed steps with that tile give the
    same field and, as a set, the same particles as a fixed 8 x 4 x 4 tile."""
    from paper_2608_15249_amd.sim import Simulation
    w = W.thermal_3d(seed=9, nx=24, ppc=16)
    state = W.sample3(w)
    a = Simulation(w, "mixed", state=state, tile="auto")
    assert a.tune_ms > 0
    assert len(a.tile) == 3 and all(t in (2, 4, 8, 16) for t in a.tile), a.tile
    again = Simulation(w, "mixed", state=state, tile="auto")
    assert again.tile == a.tile and again.tune_ms == -1.0
    b = Simulation(w, "mixed", state=state, tile=(8, 4, 4))
    for s in (a, b):
        s.initialise()
        s.run(8)
        s.ctx.sync()
    for ea, eb in zip(a.field(), b.field()):
        assert np.array_equal(ea, eb)
    sa, sb = a.state(), b.state()
    keys = ("vz", "vy", "vx", "oz", "oy", "ox")
    ka = np.lexsort(tuple(sa[k].view(np.uint32) for k in keys) + (sa["cell"],))
    kb = np.lexsort(tuple(sb[k].view(np.uint32) for k in keys) + (sb["cell"],))
    for f in ("cell", "ox", "oy", "oz", "vx", "vy", "vz"):
        assert np.array_equal(sa[f][ka], sb[f][kb]), f


def test_mixed_local_field_energy_error_3d(torch):
    """From identical states along an FP64 oracle trajectory, one mixed 3D step
    and one FP64 step give field energies within 1e-5 relative."""
    w = W.thermal_3d(seed=2025, nx=16, ppc=32)
    x, y, z, vx, vy, vz = W.sample3(w)
    s = O.Setup(3, 3, w.nx, w.Lx, w.n_particles, w.dt, ny=w.ny, Ly=w.Ly, nz=w.nz, Lz=w.Lz)
    st = O.State.from_arrays(x, vx, y, vy, vz, z)
    Eo, _ = O.initialise(s, st)
    from paper_2608_15249_amd.sim import Simulation
    worst = 0.0
    for k in range(9):
        if k % 3 == 0:
            sim = Simulation(w, "mixed", state=(st.x, st.y, st.z, st.vx, st.vy, st.vz))
            c = sim.ctx
            c.sort_by_cell(sim.p)
            c.deposit(sim.p, sim.rho)
            c.field_solve(sim.rho, sim.E, sim.E32)
            d = sim.run(1)
            c.sync()
            st_next = st.copy()
            E_next, _, _ = O.step(s, st_next, Eo)
            worst = max(worst, abs(d[1].item() / O.field_energy(s, E_next) - 1))
        Eo, _, _ = O.step(s, st, Eo)
    assert worst <= 1e-5, worst


def test_full_size_3d_sampled(torch):
    """The benchmarked 3D plasma at full size (128^3 cells, 16,777,216
    electrons, the default tile), from the seeded host state: the GPU runs
    the field of the initial charge, the backward half push and one step with
    the permutations recorded; sampled particles equal the oracle's binary32
    half push and push of their initial state in the oracle's field of the
    initial charge (its own quantised deposit and FFT solve), every particle
    sits in the bucket the table says, and the deposited charge is exact."""
    from paper_2608_15249_amd.sim import Simulation
    w = W.thermal_3d()
    x, y, z, vx, vy, vz = W.sample3(w)
    n = len(x)
    sim = Simulation(w, "mixed", state=(x, y, z, vx, vy, vz))
    c, p = sim.ctx, sim.p
    perm0 = torch.zeros(n, dtype=torch.int32, device="cuda")
    c.sort_by_cell(p, perm=perm0)
    c.deposit(p, sim.rho)
    c.field_solve(sim.rho, sim.E, sim.E32, sim.we0)
    c.gather_push(p, sim.E32, dt_scale=-0.5, move=False)
    perm1 = torch.zeros(n, dtype=torch.int32, device="cuda")
    Iout = torch.zeros(c.G, dtype=torch.int64, device="cuda")
    c.step(p, sim.E, sim.E32, 1, None, rho=Iout, perm=perm1)
    c.sync()
    ids = perm0.cpu().numpy().astype(np.int64)[perm1.cpu().numpy().astype(np.int64)]
    after = p.download()
    S = c.frac_bits
    s = O.Setup(3, 3, w.nx, w.Lx, n, w.dt, ny=w.ny, Ly=w.Ly, nz=w.nz, Lz=w.Lz)
    cx, ox = W.to_cell_offset(x, w.dx, w.nx)
    cy, oy = W.to_cell_offset(y, w.dy, w.ny)
    cz, oz = W.to_cell_offset(z, w.dz, w.nz)
    I0 = O.deposit_quantised(s, cx, ox, S, cy, oy, cz, oz)
    E32 = tuple(e.astype(np.float32) for e in O.solve_field(s, O.rho_from_quantised(s, I0, S)))
    rng = np.random.default_rng(5)
    idx = rng.choice(n, 4096, replace=False)
    src = ids[idx]
    m0 = {"ix": cx[src], "iy": cy[src], "iz": cz[src], "ox": ox[src], "oy": oy[src], "oz": oz[src],
          "vx": vx[src].astype(np.float32), "vy": vy[src].astype(np.float32), "vz": vz[src].astype(np.float32)}
    kw = dict(dim=3, vdim=3, nx=w.nx, ny=w.ny, dx=w.dx, dy=w.dy, qm=-1.0, dt=w.dt, bz=0.0, nz=w.nz, dz=w.dz)
    ref = OM.push(OM.push(m0, E32, dt_scale=-0.5, move=False, **kw), E32, **kw)
    m1 = _mstate({k: (v[idx] if v is not None and k != "bucket_start" else v) for k, v in after.items()})
    for k in ("ix", "iy", "iz", "ox", "oy", "oz", "vx", "vy", "vz"):
        assert np.array_equal(m1[k], ref[k]), k
    ix, iy, iz = W.unpack_cell(after["cell"], 3)
    tx, ty, tz = c.tile
    key = O.bucket_key(ix, iy, tx, ty, w.nx, iz=iz, tile_z=tz, ny=w.ny)
    bs = after["bucket_start"].astype(np.int64)
    assert bs[0] == 0 and bs[-1] == n and np.all(np.diff(bs) >= 0)
    assert np.array_equal(np.repeat(np.arange(len(bs) - 1), np.diff(bs)), key)
    # the total (N 2^(3S) = 2^69 here) exceeds int64: sum the high and low
    # 32-bit halves of the node sums separately, then combine exactly
    I = Iout.cpu().numpy()
    total = (int((I >> 32).sum()) << 32) + int((I & 0xFFFFFFFF).sum())
    assert total == n << (3 * S)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_empty_plasma(torch, precision):
    """No particles in 3D: an empty bucket table, the ion background alone as
    the charge (zero field), and steps whose diagnostics are all zero."""
    c, p = _ctx(torch, (16, 8, 12, 16.0, 8.0, 12.0, 0, (8, 4, 4)), precision)
    e = np.zeros(0)
    if precision == "mixed":
        f = e.astype(np.float32)
        p.upload(cell=np.zeros(0, np.int32), ox=f, oy=f, oz=f, vx=f, vy=f, vz=f)
    else:
        p.upload(x=e, y=e, z=e, vx=e, vy=e, vz=e)
    c.sort_by_cell(p)
    E = torch.ones(3 * c.G, dtype=torch.float64, device="cuda")
    E32 = torch.ones(3 * c.G, dtype=torch.float32, device="cuda")
    diag = torch.ones(4 * 3, dtype=torch.float64, device="cuda")
    c.step(p, E, E32, 3, diag)
    c.sync()
    assert np.all(p.bucket_start.cpu().numpy() == 0)
    # a uniform charge has no field; the transform's rounding may leave
    # residues of order 1e-16
    assert np.max(np.abs(E.cpu().numpy())) <= 1e-12 and np.max(np.abs(E32.cpu().numpy())) <= 1e-12
    assert np.max(np.abs(diag.cpu().numpy())) <= 1e-12
