"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Bars: integer/index work bit-exact (sort order table, permutation, int64
fixed-point deposit, binary32 push of the mixed state); FP64 work within a
tolerance derived from double rounding of the few operations per element
(1e-12 relative, well above the 1e-16 rounding noise and far below any
algorithmic error such as a dropped term or wrong index)."""
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


def _ctx(torch, *, dim, vdim, nx, ny, lx, ly, n, dt=0.1, bz=0.0, precision="fp64", tile=(0, 0)):
    from paper_2608_15249_amd.apic import Context, Particles
    c = Context(dim=dim, vdim=vdim, nx=nx, ny=ny, lx=lx, ly=ly, dt=dt, n=n, bz=bz, precision=precision, tile=tile)
    return c, Particles(c)


def _setup(dim, vdim, nx, ny, lx, ly, n, dt=0.1, bz=0.0):
    return O.Setup(dim, vdim, nx, lx, n, dt, ny=ny if dim == 2 else 1, Ly=ly, bz=bz)


def _random_state(rng, dim, vdim, lx, ly, n, vth=1.0):
    x = rng.uniform(0, lx, n)
    y = rng.uniform(0, ly, n) if dim == 2 else None
    vx = rng.normal(0, vth, n)
    vy = rng.normal(0, vth, n) if vdim >= 2 else None
    vz = rng.normal(0, vth, n) if vdim >= 3 else None
    return x, y, vx, vy, vz


CASES = [
    # dim, vdim, nx, ny, lx, ly, n, tile
    (1, 1, 61, 1, 4 * np.pi, 1.0, 20011, (8, 0)),
    (2, 2, 40, 24, 13.0, 7.5, 30011, (8, 8)),
    (2, 3, 37, 29, 37.0, 29.0, 25013, (4, 8)),
]


def _upload_mixed(p, x, y, vx, vy, vz, dx, dy, nx, ny):
    ix, ox = W.to_cell_offset(x, dx, nx)
    iy = oy = None
    if y is not None:
        iy, oy = W.to_cell_offset(y, dy, ny)
    p.upload(cell=W.pack_cell(ix, iy), ox=ox, oy=oy, vx=vx, vy=vy, vz=vz)
    return ix, iy, ox, oy


# ------------------------------------------------------------------ sort

@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sort_by_cell(torch, case, precision):
    dim, vdim, nx, ny, lx, ly, n, tile = case
    rng = np.random.default_rng(11)
    x, y, vx, vy, vz = _random_state(rng, dim, vdim, lx, ly, n)
    c, p = _ctx(torch, dim=dim, vdim=vdim, nx=nx, ny=ny, lx=lx, ly=ly, n=n, precision=precision, tile=tile)
    dx, dy = lx / nx, (ly / ny if dim == 2 else 1.0)
    if precision == "mixed":
        ix, iy, ox, oy = _upload_mixed(p, x, y, vx, vy, vz, dx, dy, nx, ny)
    else:
        p.upload(x=x, y=y, vx=vx, vy=vy, vz=vz)
        ix = np.floor(x / dx).astype(np.int64) % nx
        iy = (np.floor(y / dy).astype(np.int64) % ny) if dim == 2 else None
    before = p.download()
    perm = torch.zeros(n, dtype=torch.int32, device="cuda")
    c.sort_by_cell(p, perm=perm)
    c.sync()
    after = p.download()
    pm = perm.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(pm), np.arange(n))                 # a permutation
    for k in ("x", "y", "cell", "ox", "oy", "vx", "vy", "vz"):
        if before[k] is not None:
            assert np.array_equal(after[k], before[k][pm]), k        # sorted = input[perm]
    key = O.bucket_key(ix, iy, tile[0], max(tile[1], 1), nx)
    nb = c.nbuckets
    perm_ref, start = O.counting_sort(key, nb)
    assert np.array_equal(after["bucket_start"].astype(np.int64), start)
    assert np.all(np.diff(key[pm]) >= 0)                              # ascending buckets
    assert np.array_equal(pm, perm_ref)                               # the stable order, exactly


# --------------------------------------------------------------- deposit

@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("tiled", [False, True])
def test_deposit_fp64(torch, case, tiled):
    dim, vdim, nx, ny, lx, ly, n, tile = case
    rng = np.random.default_rng(12)
    x, y, vx, vy, vz = _random_state(rng, dim, vdim, lx, ly, n)
    c, p = _ctx(torch, dim=dim, vdim=vdim, nx=nx, ny=ny, lx=lx, ly=ly, n=n, tile=tile)
    p.upload(x=x, y=y, vx=vx, vy=vy, vz=vz)
    if tiled:
        c.sort_by_cell(p)
    rho = torch.zeros(c.G, dtype=torch.float64, device="cuda")
    c.deposit(p, rho, tiled=tiled)
    c.sync()
    d = p.download()
    s = _setup(dim, vdim, nx, ny, lx, ly, n)
    ref = O.deposit(s, O.State.from_arrays(d["x"], d["vx"], d["y"], d["vy"], d["vz"]))
    got = rho.cpu().numpy().reshape(ref.shape)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("tiled", [False, True])
def test_deposit_mixed_bit_exact(torch, case, tiled):
    dim, vdim, nx, ny, lx, ly, n, tile = case
    rng = np.random.default_rng(13)
    x, y, vx, vy, vz = _random_state(rng, dim, vdim, lx, ly, n)
    # a few offsets at the edges of [0,1) and exact half-way rounding points
    c, p = _ctx(torch, dim=dim, vdim=vdim, nx=nx, ny=ny, lx=lx, ly=ly, n=n, precision="mixed", tile=tile)
    dx, dy = lx / nx, (ly / ny if dim == 2 else 1.0)
    ix, ox = W.to_cell_offset(x, dx, nx)
    iy = oy = None
    if dim == 2:
        iy, oy = W.to_cell_offset(y, dy, ny)
    S = c.frac_bits
    ox[:5] = np.array([0.0, np.nextafter(np.float32(1), np.float32(0)), 0.5, 1.5 * 2.0 ** -S, 2.5 * 2.0 ** -S],
                      dtype=np.float32)
    p.upload(cell=W.pack_cell(ix, iy), ox=ox, oy=oy, vx=vx, vy=vy, vz=vz)
    if tiled:
        c.sort_by_cell(p)
    I = torch.zeros(c.G, dtype=torch.int64, device="cuda")
    c.deposit(p, I, tiled=tiled)
    c.sync()
    d = p.download()
    jx, jy = W.unpack_cell(d["cell"], dim)
    s = _setup(dim, vdim, nx, ny, lx, ly, n)
    ref = O.deposit_quantised(s, jx, d["ox"], S, jy, d["oy"])
    got = I.cpu().numpy().reshape(ref.shape)
    assert np.array_equal(got, ref)
    assert sum(int(v) for v in got.ravel()) == n << (S * dim)


# ----------------------------------------------------------------- field

@pytest.mark.parametrize("case", CASES)
def test_field_solve(torch, case):
    dim, vdim, nx, ny, lx, ly, n, tile = case
    rng = np.random.default_rng(14)
    s = _setup(dim, vdim, nx, ny, lx, ly, n)
    rho = rng.normal(size=s.grid_shape)
    c, p = _ctx(torch, dim=dim, vdim=vdim, nx=nx, ny=ny, lx=lx, ly=ly, n=n, tile=tile)
    r = torch.from_numpy(rho.ravel().copy()).cuda()
    E = torch.zeros(dim * c.G, dtype=torch.float64, device="cuda")
    E32 = torch.zeros(dim * c.G, dtype=torch.float32, device="cuda")
    we = torch.zeros(1, dtype=torch.float64, device="cuda")
    c.field_solve(r, E, E32, we)
    c.sync()
    ref = O.solve_field(s, rho)
    got = E.cpu().numpy().reshape((dim,) + s.grid_shape)
    scale = max(np.max(np.abs(e)) for e in ref)
    for d_ in range(dim):
        assert np.max(np.abs(got[d_] - ref[d_])) <= 1e-12 * scale
    assert np.array_equal(E32.cpu().numpy(), E.cpu().numpy().astype(np.float32))
    assert abs(we.item() / O.field_energy(s, ref) - 1) < 1e-12


@pytest.mark.parametrize("case", CASES)
def test_field_solve_mixed_from_fixed_point(torch, case):
    dim, vdim, nx, ny, lx, ly, n, tile = case
    rng = np.random.default_rng(15)
    x, y, vx, vy, vz = _random_state(rng, dim, vdim, lx, ly, n)
    s = _setup(dim, vdim, nx, ny, lx, ly, n)
    c, p = _ctx(torch, dim=dim, vdim=vdim, nx=nx, ny=ny, lx=lx, ly=ly, n=n, precision="mixed", tile=tile)
    ix, iy, ox, oy = _upload_mixed(p, x, y, vx, vy, vz, s.dx, s.dy, nx, ny)
    S = c.frac_bits
    I = O.deposit_quantised(s, ix, ox, S, iy, oy)
    Id = torch.from_numpy(I.ravel().copy()).cuda()
    E = torch.zeros(dim * c.G, dtype=torch.float64, device="cuda")
    c.field_solve(Id, E)
    c.sync()
    ref = O.solve_field(s, O.rho_from_quantised(s, I, S))
    got = E.cpu().numpy().reshape((dim,) + s.grid_shape)
    scale = max(np.max(np.abs(e)) for e in ref)
    for d_ in range(dim):
        assert np.max(np.abs(got[d_] - ref[d_])) <= 1e-12 * scale


# ------------------------------------------------------------- gather/push

@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("tiled", [False, True])
def test_gather_push_fp64(torch, case, tiled):
    dim, vdim, nx, ny, lx, ly, n, tile = case
    bz = 2.0 if vdim == 3 else 0.0
    rng = np.random.default_rng(16)
    x, y, vx, vy, vz = _random_state(rng, dim, vdim, lx, ly, n)
    s = _setup(dim, vdim, nx, ny, lx, ly, n, bz=bz)
    E = tuple(rng.normal(size=s.grid_shape) for _ in range(dim))
    c, p = _ctx(torch, dim=dim, vdim=vdim, nx=nx, ny=ny, lx=lx, ly=ly, n=n, bz=bz, tile=tile)
    p.upload(x=x, y=y, vx=vx, vy=vy, vz=vz)
    if tiled:
        c.sort_by_cell(p)
    d0 = p.download()
    Ed = torch.from_numpy(np.concatenate([e.ravel() for e in E])).cuda()
    c.gather_push(p, Ed, dt_scale=1.0, move=True, tiled=tiled)
    c.sync()
    d1 = p.download()
    st = O.State.from_arrays(d0["x"], d0["vx"], d0["y"], d0["vy"], d0["vz"])
    O.boris(s, st, O.gather(s, st, E), s.dt)
    O.move(s, st)
    for k, ref in (("vx", st.vx), ("vy", st.vy), ("vz", st.vz)):
        if ref is not None:
            assert np.max(np.abs(d1[k] - ref)) <= 1e-13, k
    # positions: compare on the circle (wrap-safe)
    dxp = np.abs(d1["x"] - st.x)
    dxp = np.minimum(dxp, lx - dxp)
    assert np.max(dxp) <= 1e-12 * lx
    if dim == 2:
        dyp = np.abs(d1["y"] - st.y)
        dyp = np.minimum(dyp, ly - dyp)
        assert np.max(dyp) <= 1e-12 * ly


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("dt_scale", [1.0, -0.5])
def test_gather_push_mixed_bit_exact(torch, case, dt_scale):
    dim, vdim, nx, ny, lx, ly, n, tile = case
    bz = 2.0 if vdim == 3 else 0.0
    rng = np.random.default_rng(17)
    x, y, vx, vy, vz = _random_state(rng, dim, vdim, lx, ly, n, vth=3.0)
    s = _setup(dim, vdim, nx, ny, lx, ly, n, bz=bz)
    E32 = tuple(rng.normal(size=s.grid_shape).astype(np.float32) for _ in range(dim))
    c, p = _ctx(torch, dim=dim, vdim=vdim, nx=nx, ny=ny, lx=lx, ly=ly, n=n, bz=bz, precision="mixed", tile=tile)
    _upload_mixed(p, x, y, vx, vy, vz, s.dx, s.dy, nx, ny)
    c.sort_by_cell(p)
    d0 = p.download()
    jx, jy = W.unpack_cell(d0["cell"], dim)
    Ed = torch.from_numpy(np.concatenate([e.ravel() for e in E32])).cuda()
    move = dt_scale == 1.0
    c.gather_push(p, Ed, dt_scale=dt_scale, move=move)
    c.sync()
    d1 = p.download()
    st = {"ix": jx, "iy": jy, "ox": d0["ox"], "oy": d0["oy"], "vx": d0["vx"], "vy": d0["vy"], "vz": d0["vz"]}
    ref = OM.push(st, E32, dim=dim, vdim=vdim, nx=nx, ny=ny, dx=s.dx, dy=s.dy, qm=s.qm, dt=s.dt, bz=bz,
                  dt_scale=dt_scale, move=move)
    kx, ky = W.unpack_cell(d1["cell"], dim)
    assert np.array_equal(kx, ref["ix"])
    assert np.array_equal(d1["ox"], ref["ox"])
    if dim == 2:
        assert np.array_equal(ky, ref["iy"])
        assert np.array_equal(d1["oy"], ref["oy"])
    for k in ("vx", "vy", "vz"):
        if ref[k] is not None:
            assert np.array_equal(d1[k], ref[k]), k


# ------------------------------------------------------------ full steps

def _compose(ids, perm):
    return ids[perm.cpu().numpy().astype(np.int64)]


@pytest.mark.parametrize("case", CASES)
def test_step_fp64_matches_oracle(torch, case):
    dim, vdim, nx, ny, lx, ly, n, tile = case
    bz = 2.0 if vdim == 3 else 0.0
    rng = np.random.default_rng(18)
    x, y, vx, vy, vz = _random_state(rng, dim, vdim, lx, ly, n)
    s = _setup(dim, vdim, nx, ny, lx, ly, n, bz=bz)
    c, p = _ctx(torch, dim=dim, vdim=vdim, nx=nx, ny=ny, lx=lx, ly=ly, n=n, bz=bz, tile=tile)
    p.upload(x=x, y=y, vx=vx, vy=vy, vz=vz)
    perm = torch.zeros(n, dtype=torch.int32, device="cuda")
    c.sort_by_cell(p, perm=perm)
    ids = _compose(np.arange(n), perm)
    rho = torch.zeros(c.G, dtype=torch.float64, device="cuda")
    E = torch.zeros(dim * c.G, dtype=torch.float64, device="cuda")
    c.deposit(p, rho)
    c.field_solve(rho, E)
    c.gather_push(p, E, dt_scale=-0.5, move=False)
    st = O.State.from_arrays(x, vx, y, vy, vz)
    Eo, _ = O.initialise(s, st)
    nsteps = 8
    diag = torch.zeros(nsteps * 4, dtype=torch.float64, device="cuda")
    ref_we = []
    ref_ke = []
    for k in range(nsteps):
        c.step(p, E, None, 1, diag[4 * k:4 * k + 4], perm=perm)
        ids = _compose(ids, perm)
        Eo, _, ke = O.step(s, st, Eo)
        ref_we.append(O.field_energy(s, Eo))
        ref_ke.append(ke)
    c.sync()
    d = p.download()
    for k, ref in (("vx", st.vx), ("vy", st.vy), ("vz", st.vz)):
        if ref is not None:
            assert np.max(np.abs(d[k] - ref[ids])) <= 1e-11, k
    dxp = np.abs(d["x"] - st.x[ids])
    assert np.max(np.minimum(dxp, lx - dxp)) <= 1e-11 * lx
    Eg = E.cpu().numpy().reshape((dim,) + s.grid_shape)
    scale = max(np.max(np.abs(e)) for e in Eo)
    for d_ in range(dim):
        assert np.max(np.abs(Eg[d_] - Eo[d_])) <= 1e-10 * scale
    dg = diag.cpu().numpy().reshape(nsteps, 4)
    assert np.allclose(dg[:, 1], ref_we, rtol=1e-10, atol=0)
    assert np.allclose(dg[:, 2], ref_ke, rtol=1e-12, atol=0)
    assert np.allclose(dg[:, 0], n * s.Q, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("case", CASES)
def test_step_mixed_one_step_bit_exact(torch, case):
    """One mixed step from a seeded state and a binary32 field E^n: the new
    particle state, the int64 deposit of rho^{n+1} and the bucket table are
    bit-exact against the oracle's binary32 push and quantised deposit."""
    dim, vdim, nx, ny, lx, ly, n, tile = case
    bz = 2.0 if vdim == 3 else 0.0
    rng = np.random.default_rng(19)
    x, y, vx, vy, vz = _random_state(rng, dim, vdim, lx, ly, n)
    s = _setup(dim, vdim, nx, ny, lx, ly, n, bz=bz)
    c, p = _ctx(torch, dim=dim, vdim=vdim, nx=nx, ny=ny, lx=lx, ly=ly, n=n, bz=bz, precision="mixed", tile=tile)
    ix, iy, ox, oy = _upload_mixed(p, x, y, vx, vy, vz, s.dx, s.dy, nx, ny)
    S = c.frac_bits
    I0 = O.deposit_quantised(s, ix, ox, S, iy, oy)
    E0 = O.solve_field(s, O.rho_from_quantised(s, I0, S))
    E32 = tuple(e.astype(np.float32) for e in E0)
    perm = torch.zeros(n, dtype=torch.int32, device="cuda")
    c.sort_by_cell(p, perm=perm)
    ids = _compose(np.arange(n), perm)
    Ed = torch.from_numpy(np.concatenate([e.ravel() for e in E0])).cuda()
    E32d = torch.from_numpy(np.concatenate([e.ravel() for e in E32])).cuda()
    Iout = torch.zeros(c.G, dtype=torch.int64, device="cuda")
    c.step(p, Ed, E32d, 1, None, rho=Iout, perm=perm)
    c.sync()
    ids = _compose(ids, perm)
    st = {"ix": ix, "iy": iy, "ox": ox, "oy": oy,
          "vx": vx.astype(np.float32), "vy": None if vy is None else vy.astype(np.float32),
          "vz": None if vz is None else vz.astype(np.float32)}
    ref = OM.push(st, E32, dim=dim, vdim=vdim, nx=nx, ny=ny, dx=s.dx, dy=s.dy, qm=s.qm, dt=s.dt, bz=bz)
    d = p.download()
    kx, ky = W.unpack_cell(d["cell"], dim)
    assert np.array_equal(kx, ref["ix"][ids])
    assert np.array_equal(d["ox"], ref["ox"][ids])
    for k in ("vx", "vy", "vz"):
        if ref[k] is not None:
            assert np.array_equal(d[k], ref[k][ids]), k
    if dim == 2:
        assert np.array_equal(ky, ref["iy"][ids])
        assert np.array_equal(d["oy"], ref["oy"][ids])
    I1 = O.deposit_quantised(s, ref["ix"], ref["ox"], S, ref["iy"], ref["oy"])
    assert np.array_equal(Iout.cpu().numpy().reshape(I1.shape), I1)
    key = O.bucket_key(ref["ix"], ref["iy"], tile[0], max(tile[1], 1), nx)
    _, start = O.counting_sort(key, c.nbuckets)
    assert np.array_equal(d["bucket_start"].astype(np.int64), start)
    E1 = O.solve_field(s, O.rho_from_quantised(s, I1, S))
    Eg = Ed.cpu().numpy().reshape((dim,) + s.grid_shape)
    scale = max(np.max(np.abs(e)) for e in E1)
    for d_ in range(dim):
        assert np.max(np.abs(Eg[d_] - E1[d_])) <= 1e-12 * scale


def test_mixed_local_field_energy_error(torch):
    """From identical states along an FP64 oracle trajectory, one mixed step
    and one FP64 step give field energies within 1e-5 relative."""
    w = W.thermal_2d(seed=2024, nx=64, ppc=64)
    x, y, vx, vy, vz = W.sample(w)
    s = O.Setup(2, 2, w.nx, w.Lx, w.n_particles, w.dt, ny=w.ny, Ly=w.Ly)
    st = O.State.from_arrays(x, vx, y, vy)
    Eo, _ = O.initialise(s, st)
    from paper_2608_15249_amd.sim import Simulation
    worst = 0.0
    for k in range(12):
        if k % 4 == 0:
            # mixed state = binary32 rounding of the oracle state (x^n, v^{n-1/2})
            sim = Simulation(w, "mixed", state=(st.x, st.y, st.vx, st.vy, None))
            c = sim.ctx
            c.sort_by_cell(sim.p)
            c.deposit(sim.p, sim.rho)
            c.field_solve(sim.rho, sim.E, sim.E32)
            d = sim.run(1)
            c.sync()
            st_next = st.copy()
            E_next, _, _ = O.step(s, st_next, Eo)
            we_o = O.field_energy(s, E_next)
            we_g = d[1].item()
            worst = max(worst, abs(we_g / we_o - 1))
        Eo, _, _ = O.step(s, st, Eo)
    assert worst <= 1e-5, worst


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_step_deterministic(torch, precision):
    """Mixed path: two runs from the same input give identical bits: particle
    order and values, fields and every diagnostic. Slots come from the
    per-bucket tallies, the int64 deposit is order-free and summed over tiles
    in a fixed order, and every reduction has a fixed tree (no particle here
    jumps more than a tile, the one case that takes a slot from an atomic
    counter)."""
    from paper_2608_15249_amd.sim import Simulation
    w = W.thermal_2d(seed=7, nx=64, ppc=32)
    outs = []
    for _ in range(2):
        sim = Simulation(w, precision, tile=(8, 8))
        sim.initialise()
        d = sim.run(10)
        sim.ctx.sync()
        outs.append((sim.E.cpu().numpy(), d.cpu().numpy(), sim.state()))
    (E1, d1, s1), (E2, d2, s2) = outs
    if precision == "fp64":
        # FP64 sums inside a tile use LDS atomics, whose order varies between
        # runs: equal to rounding, and the bucket tables agree
        assert np.allclose(E1, E2, rtol=0, atol=1e-12 * np.abs(E1).max())
        assert np.array_equal(s1["bucket_start"], s2["bucket_start"])
        return
    assert np.array_equal(E1, E2)
    assert np.array_equal(d1, d2)
    for k in ("cell", "ox", "oy", "vx", "vy", "bucket_start"):
        assert np.array_equal(s1[k], s2[k]), k


def test_nan_particle_reports_domain_error(torch):
    from paper_2608_15249_amd.apic import ApicError
    n = 4096
    rng = np.random.default_rng(3)
    c, p = _ctx(torch, dim=2, vdim=2, nx=16, ny=16, lx=16.0, ly=16.0, n=n, tile=(4, 4))
    x, y, vx, vy, _ = _random_state(rng, 2, 2, 16.0, 16.0, n)
    x[17] = np.nan
    p.upload(x=x, y=y, vx=vx, vy=vy)
    rho = torch.zeros(c.G, dtype=torch.float64, device="cuda")
    c.deposit(p, rho, tiled=False)
    with pytest.raises(ApicError) as ei:
        c.sync()
    assert ei.value.status == -5
    c.sync()  # flag cleared


def test_autotuned_tile_gives_the_same_plasma(torch):
    """apic_autotune_tiles picks one of its candidate tiles (or the default),
    caches the pick, and the mixed step with that tile advances the particle
    set and the field to the same bits as a fixed 8x8 tile."""
    from paper_2608_15249_amd.sim import Simulation
    w = W.thermal_2d(nx=64, ppc=16)
    state = W.sample(w)
    a = Simulation(w, "mixed", state=state, tile="auto")
    assert a.tile in [(4, 4), (8, 4), (8, 8), (16, 8), (16, 16), (32, 16), (32, 32), (0, 0)]
    assert a.tune_ms > 0
    again = Simulation(w, "mixed", state=state, tile="auto")
    assert again.tile == a.tile and again.tune_ms == -1.0
    b = Simulation(w, "mixed", state=state, tile=(8, 8))
    for s in (a, b):
        s.initialise()
        s.run(4)
        s.ctx.sync()
    assert np.array_equal(a.field()[0], b.field()[0]) and np.array_equal(a.field()[1], b.field()[1])
    sa, sb = a.state(), b.state()
    ka = np.lexsort((sa["vy"].view(np.uint32), sa["vx"].view(np.uint32), sa["oy"].view(np.uint32),
                     sa["ox"].view(np.uint32), sa["cell"]))
    kb = np.lexsort((sb["vy"].view(np.uint32), sb["vx"].view(np.uint32), sb["oy"].view(np.uint32),
                     sb["ox"].view(np.uint32), sb["cell"]))
    for f in ("cell", "ox", "oy", "vx", "vy"):
        assert np.array_equal(sa[f][ka], sb[f][kb]), f


def test_profile_phases_modes(torch):
    """Per-phase timing: with every phase profiled all four sums are positive;
    with the push only, the other three read zero and the push is timed."""
    dim, vdim, nx, ny, lx, ly, n, tile = CASES[1]
    rng = np.random.default_rng(23)
    x, y, vx, vy, vz = _random_state(rng, dim, vdim, lx, ly, n)
    c, p = _ctx(torch, dim=dim, vdim=vdim, nx=nx, ny=ny, lx=lx, ly=ly, n=n, precision="mixed", tile=tile)
    s = _setup(dim, vdim, nx, ny, lx, ly, n)
    _upload_mixed(p, x, y, vx, vy, vz, s.dx, s.dy, nx, ny)
    c.sort_by_cell(p)
    I = torch.zeros(c.G, dtype=torch.int64, device="cuda")
    c.deposit(p, I)
    E = torch.zeros(2 * c.G, dtype=torch.float64, device="cuda")
    E32 = torch.zeros(2 * c.G, dtype=torch.float32, device="cuda")
    c.field_solve(I, E, E32)
    for all_phases in (True, False):
        c.profile_phases(all_phases)
        c.profile_enable(4)
        c.step(p, E, E32, 6)
        c.sync()
        ms, steps = c.profile_read()
        c.profile_enable(0)
        assert steps == 4
        assert ms[2] > 0
        if all_phases:
            assert all(m > 0 for m in ms)
        else:
            assert ms[0] == 0 and ms[1] == 0 and ms[3] == 0
    # one step in three: steps 0, 3 and 6 of seven (then 0 of a second call)
    c.profile_phases(False)
    c.profile_every(3)
    c.profile_enable(8)
    c.step(p, E, E32, 7)
    c.sync()
    ms, steps = c.profile_read()
    assert steps == 3 and ms[2] > 0
    c.step(p, E, E32, 2)
    c.sync()
    assert c.profile_read()[1] == 1
    c.profile_enable(0)
    c.profile_every(1)
    from paper_2608_15249_amd.apic import ApicError
    with pytest.raises(ApicError):
        c.profile_every(0)
    c.profile_phases(True)
