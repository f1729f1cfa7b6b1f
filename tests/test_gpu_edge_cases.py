"""GPU edge cases of the electrostatic path against the oracle, through the C
ABI: an empty plasma, a single particle (whose own field must not push it:
the momentum-conserving scheme has no self-force), a clustered plasma that
leaves most buckets empty, and mixed-path particles on cell, tile and domain
edges (offsets 0 and the largest binary32 below 1, wraps across the domain
end in both directions, moves of several tiles in one step)."""

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


def _ctx(n, precision, nx=64, ny=32, lx=64 * 0.7, ly=32 * 0.9, tile=(8, 8), q_macro=None, vdim=2):
    from paper_2608_15249_amd.apic import Context, Particles
    c = Context(dim=2, vdim=vdim, nx=nx, ny=ny, lx=lx, ly=ly, dt=0.1, n=n, precision=precision, tile=tile,
                q_macro=q_macro)
    return c, Particles(c)


def _compose(ids, perm):
    return ids[perm.cpu().numpy().astype(np.int64)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_empty_plasma(torch, precision):
    """No particles: an empty bucket table, the ion background alone as the
    charge (zero field), and steps whose diagnostics are all zero."""
    c, p = _ctx(0, precision)
    e = np.zeros(0)
    if precision == "mixed":
        p.upload(cell=np.zeros(0, np.int32), ox=e.astype(np.float32), oy=e.astype(np.float32),
                 vx=e.astype(np.float32), vy=e.astype(np.float32))
    else:
        p.upload(x=e, y=e, vx=e, vy=e)
    c.sort_by_cell(p)
    acc = torch.zeros(c.G, dtype=torch.int64 if precision == "mixed" else torch.float64, device="cuda")
    c.deposit(p, acc)
    E = torch.ones(2 * c.G, dtype=torch.float64, device="cuda")
    E32 = torch.ones(2 * c.G, dtype=torch.float32, device="cuda")
    we = torch.ones(1, dtype=torch.float64, device="cuda")
    c.field_solve(acc, E, E32, we)
    diag = torch.ones(4 * 3, dtype=torch.float64, device="cuda")
    c.step(p, E, E32, 3, diag)
    c.sync()
    assert np.all(p.bucket_start.cpu().numpy() == 0)
    a = acc.cpu().numpy()
    if precision == "mixed":
        assert np.all(a == 0)
    else:
        assert np.all(a == 1.0)            # rho_ion
    assert np.all(E.cpu().numpy() == 0.0) and np.all(E32.cpu().numpy() == 0.0)
    assert we.item() == 0.0
    assert np.all(diag.cpu().numpy() == 0.0)


def test_single_particle_feels_no_self_force(torch):
    """One electron at rest in an otherwise neutral box: the CIC deposit, the
    centred-difference field and the CIC gather give it no force, so it stays
    at rest; five FP64 steps match the oracle's."""
    nx, ny, lx, ly = 16, 16, 16 * 0.8, 16 * 1.1
    s = O.Setup(2, 2, nx, lx, 1, 0.1, ny=ny, Ly=ly)
    c, p = _ctx(1, "fp64", nx=nx, ny=ny, lx=lx, ly=ly, tile=(8, 8), q_macro=s.Q)
    x, y, vx, vy = np.array([5.3712]), np.array([11.0417]), np.zeros(1), np.zeros(1)
    p.upload(x=x, y=y, vx=vx, vy=vy)
    c.sort_by_cell(p)
    rho = torch.zeros(c.G, dtype=torch.float64, device="cuda")
    c.deposit(p, rho)
    E = torch.zeros(2 * c.G, dtype=torch.float64, device="cuda")
    c.field_solve(rho, E)
    c.gather_push(p, E, dt_scale=-0.5, move=False)
    c.step(p, E, None, 5)
    c.sync()
    d = p.download()
    st = O.State.from_arrays(x, vx, y, vy)
    Eo, _ = O.initialise(s, st)
    for _ in range(5):
        Eo, _, _ = O.step(s, st, Eo)
    scale = np.max(np.abs(Eo[0])) * s.dt
    assert abs(d["vx"][0]) <= 1e-13 * scale and abs(d["vy"][0]) <= 1e-13 * scale
    assert abs(d["vx"][0] - st.vx[0]) <= 1e-13 * scale
    assert abs(d["x"][0] - st.x[0]) <= 1e-12 and abs(d["y"][0] - st.y[0]) <= 1e-12


def _clustered(rng, n, lx, ly):
    """A blob of particles inside three by two cells near the domain corner
    (so the blob straddles the periodic edge), thermal spread 0.5."""
    x = np.mod(lx - 1.5 * (lx / 64) + rng.uniform(0, 3, n) * (lx / 64), lx)
    y = np.mod(ly - 1.0 * (ly / 32) + rng.uniform(0, 2, n) * (ly / 32), ly)
    return x, y, rng.normal(0, 0.5, n), rng.normal(0, 0.5, n)


def test_clustered_plasma_fp64_steps(torch):
    """5001 particles in six cells of a 64 x 32 grid with 8 x 8 tiles: most
    buckets stay empty, the occupied ones hold thousands; five FP64 steps and
    the bucket table against the oracle."""
    n = 5001
    lx, ly = 64 * 0.7, 32 * 0.9
    rng = np.random.default_rng(301)
    x, y, vx, vy = _clustered(rng, n, lx, ly)
    s = O.Setup(2, 2, 64, lx, n, 0.1, ny=32, Ly=ly)
    c, p = _ctx(n, "fp64")
    p.upload(x=x, y=y, vx=vx, vy=vy)
    perm = torch.zeros(n, dtype=torch.int32, device="cuda")
    c.sort_by_cell(p, perm=perm)
    ids = _compose(np.arange(n), perm)
    rho = torch.zeros(c.G, dtype=torch.float64, device="cuda")
    c.deposit(p, rho)
    E = torch.zeros(2 * c.G, dtype=torch.float64, device="cuda")
    c.field_solve(rho, E)
    c.gather_push(p, E, dt_scale=-0.5, move=False)
    for _ in range(5):
        c.step(p, E, None, 1, perm=perm)
        ids = _compose(ids, perm)
    c.sync()
    st = O.State.from_arrays(x, vx, y, vy)
    Eo, _ = O.initialise(s, st)
    for _ in range(5):
        Eo, _, _ = O.step(s, st, Eo)
    d = p.download()
    for k, r in (("vx", st.vx), ("vy", st.vy)):
        assert np.max(np.abs(d[k] - r[ids])) <= 1e-10 * max(1.0, np.max(np.abs(r))), k
    for k, r, L in (("x", st.x, s.Lx), ("y", st.y, s.Ly)):
        dd = np.abs(d[k] - r[ids])
        assert np.max(np.minimum(dd, L - dd)) <= 1e-10 * L, k
    # the table of the GPU's own positions (a position within rounding of a
    # cell edge may sit on either side in the oracle's)
    key = O.bucket_key(np.floor(d["x"] / s.dx).astype(np.int64) % 64, np.floor(d["y"] / s.dy).astype(np.int64) % 32,
                       8, 8, 64)
    _, start = O.counting_sort(key, c.nbuckets)
    bs = d["bucket_start"].astype(np.int64)
    assert np.array_equal(bs, start)
    assert np.sum(np.diff(bs) == 0) >= c.nbuckets // 2


def _edge_state(nx, ny):
    """Mixed states on the edges: offsets 0 and the largest binary32 below 1
    on the first and last cells of each axis and on tile edges, with
    velocities that cross the domain end either way, stop exactly, or jump
    several tiles."""
    top = np.nextafter(np.float32(1), np.float32(0))
    cells_x = [0, 0, nx - 1, nx - 1, 7, 8, 15, 16, 31, 33]
    cells_y = [0, ny - 1, 0, ny - 1, 8, 7, 16, 15, 0, ny - 1]
    offs = [np.float32(0), top]
    vels = [0.0, 1e-7, -1e-7, 3.0, -3.0, 27.5, -41.0, 9.999, 100.0, -123.4]
    ix, iy, ox, oy, vx, vy = [], [], [], [], [], []
    for cx, cy in zip(cells_x, cells_y):
        for fx in offs:
            for fy in offs:
                for v in vels:
                    ix.append(cx); iy.append(cy); ox.append(fx); oy.append(fy)
                    vx.append(v); vy.append(-0.5 * v)
    f32 = np.float32
    return (np.array(ix, np.int64), np.array(iy, np.int64), np.array(ox, f32), np.array(oy, f32),
            np.array(vx, f32), np.array(vy, f32))


def test_mixed_step_on_cell_tile_and_domain_edges(torch):
    """One mixed step of edge states (plus a uniform background so the field
    is not trivial) is bit-exact against the oracle's binary32 push and
    quantised deposit, and the bucket table holds the new positions."""
    nx, ny, lx, ly = 64, 32, 64 * 0.7, 32 * 0.9
    ex_ = _edge_state(nx, ny)
    rng = np.random.default_rng(302)
    nb_ = 3000
    bx, by = rng.uniform(0, lx, nb_), rng.uniform(0, ly, nb_)
    bix, box_ = W.to_cell_offset(bx, lx / nx, nx)
    biy, boy = W.to_cell_offset(by, ly / ny, ny)
    ix = np.concatenate([ex_[0], bix]); iy = np.concatenate([ex_[1], biy])
    ox = np.concatenate([ex_[2], box_]); oy = np.concatenate([ex_[3], boy])
    vx = np.concatenate([ex_[4], rng.normal(0, 1, nb_).astype(np.float32)])
    vy = np.concatenate([ex_[5], rng.normal(0, 1, nb_).astype(np.float32)])
    n = len(ix)
    s = O.Setup(2, 2, nx, lx, n, 0.1, ny=ny, Ly=ly)
    c, p = _ctx(n, "mixed", nx=nx, ny=ny, lx=lx, ly=ly)
    p.upload(cell=W.pack_cell(ix, iy), ox=ox, oy=oy, vx=vx, vy=vy)
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
    st = {"ix": ix, "iy": iy, "ox": ox, "oy": oy, "vx": vx, "vy": vy, "vz": None}
    ref = OM.push(st, E32, dim=2, vdim=2, nx=nx, ny=ny, dx=s.dx, dy=s.dy, qm=s.qm, dt=s.dt, bz=0.0)
    d = p.download()
    kx, ky = W.unpack_cell(d["cell"], 2)
    for got, k in ((kx, "ix"), (ky, "iy"), (d["ox"], "ox"), (d["oy"], "oy"), (d["vx"], "vx"), (d["vy"], "vy")):
        assert np.array_equal(got, ref[k][ids]), k
    assert np.all((d["ox"] >= 0) & (d["ox"] < 1) & (d["oy"] >= 0) & (d["oy"] < 1))
    I1 = O.deposit_quantised(s, ref["ix"], ref["ox"], S, ref["iy"], ref["oy"])
    assert np.array_equal(Iout.cpu().numpy().reshape(I1.shape), I1)
    key = O.bucket_key(ref["ix"], ref["iy"], 8, 8, nx)
    _, start = O.counting_sort(key, c.nbuckets)
    assert np.array_equal(d["bucket_start"].astype(np.int64), start)


def test_more_buckets_than_the_one_launch_scan_covers(torch):
    """256 x 256 cells in 4 x 2 tiles (8192 buckets, above the 4096 that the
    one-launch scan of bucket totals serves): the separate scan and offsets
    launches with the alternating totals buffers; one mixed step bit-exact
    against the oracle's binary32 push and quantised deposit, then three
    FP64 steps of the same plasma against the oracle."""
    nx, ny, lx, ly, n, tile = 256, 256, 256.0, 256.0 * 0.75, 60011, (4, 2)
    rng = np.random.default_rng(303)
    x, y = rng.uniform(0, lx, n), rng.uniform(0, ly, n)
    vx, vy = rng.normal(0, 1, n), rng.normal(0, 1, n)
    s = O.Setup(2, 2, nx, lx, n, 0.1, ny=ny, Ly=ly)
    # mixed: one step from the oracle's field of the quantised charge
    c, p = _ctx(n, "mixed", nx=nx, ny=ny, lx=lx, ly=ly, tile=tile)
    assert c.nbuckets == 8192
    ix, ox = W.to_cell_offset(x, s.dx, nx)
    iy, oy = W.to_cell_offset(y, s.dy, ny)
    p.upload(cell=W.pack_cell(ix, iy), ox=ox, oy=oy, vx=vx.astype(np.float32), vy=vy.astype(np.float32))
    S = c.frac_bits
    E0 = O.solve_field(s, O.rho_from_quantised(s, O.deposit_quantised(s, ix, ox, S, iy, oy), S))
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
    st = {"ix": ix, "iy": iy, "ox": ox, "oy": oy, "vx": vx.astype(np.float32), "vy": vy.astype(np.float32),
          "vz": None}
    ref = OM.push(st, E32, dim=2, vdim=2, nx=nx, ny=ny, dx=s.dx, dy=s.dy, qm=s.qm, dt=s.dt, bz=0.0)
    d = p.download()
    kx, ky = W.unpack_cell(d["cell"], 2)
    for got, k in ((kx, "ix"), (ky, "iy"), (d["ox"], "ox"), (d["oy"], "oy"), (d["vx"], "vx"), (d["vy"], "vy")):
        assert np.array_equal(got, ref[k][ids]), k
    I1 = O.deposit_quantised(s, ref["ix"], ref["ox"], S, ref["iy"], ref["oy"])
    assert np.array_equal(Iout.cpu().numpy().reshape(I1.shape), I1)
    _, start = O.counting_sort(O.bucket_key(ref["ix"], ref["iy"], 4, 2, nx), c.nbuckets)
    assert np.array_equal(d["bucket_start"].astype(np.int64), start)
    # FP64: three steps in calls of two and one (both totals buffers are used)
    c, p = _ctx(n, "fp64", nx=nx, ny=ny, lx=lx, ly=ly, tile=tile)
    p.upload(x=x, y=y, vx=vx, vy=vy)
    c.sort_by_cell(p)
    rho = torch.zeros(c.G, dtype=torch.float64, device="cuda")
    c.deposit(p, rho)
    E = torch.zeros(2 * c.G, dtype=torch.float64, device="cuda")
    c.field_solve(rho, E)
    c.gather_push(p, E, dt_scale=-0.5, move=False)
    c.step(p, E, None, 2)
    c.step(p, E, None, 1)
    c.sync()
    sto = O.State.from_arrays(x, vx, y, vy)
    Eo, _ = O.initialise(s, sto)
    for _ in range(3):
        Eo, _, _ = O.step(s, sto, Eo)
    d = p.download()
    # the permutation of a multi-step call is not recorded: match each GPU
    # particle to the oracle's nearest in (x, y, vx, vy); the match must be
    # one to one and close
    from scipy.spatial import cKDTree
    tree = cKDTree(np.stack([sto.x, sto.y, sto.vx, sto.vy], axis=1))
    dist, idx = tree.query(np.stack([d["x"], d["y"], d["vx"], d["vy"]], axis=1))
    assert len(np.unique(idx)) == n
    assert np.max(dist) <= 1e-9


def test_binding_rejects_mismatched_caller_tensors(torch):
    """The binding checks dtype, device, contiguity and length of every
    caller tensor before the C call: a binary32 E on the FP64 path, a short
    diag, a host tensor or a strided view raise ApicError and launch
    nothing."""
    from paper_2608_15249_amd.apic import ApicError
    c, p = _ctx(100, "fp64")
    E = torch.zeros(2 * c.G, dtype=torch.float64, device="cuda")
    bad = [
        lambda: c.step(p, E.float(), None, 1),
        lambda: c.step(p, E, None, 3, torch.zeros(8, dtype=torch.float64, device="cuda")),
        lambda: c.step(p, E.cpu(), None, 1),
        lambda: c.step(p, torch.zeros(4 * c.G, dtype=torch.float64, device="cuda")[::2], None, 1),
        lambda: c.field_solve(torch.zeros(c.G - 1, dtype=torch.float64, device="cuda"), E),
        lambda: c.gather_push(p, E[: c.G]),
    ]
    for f in bad:
        with pytest.raises(ApicError):
            f()
