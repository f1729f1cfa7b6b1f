"""GPU parity of the plasma between grounded absorbing walls (2D, walls at
x = 0 and x = Lx, periodic in y) against the oracle, through the C ABI: the
Dirichlet field solve, FP64 steps with absorption (live set, states, fields,
diagnostics), and one mixed step bit-exact (binary32 push, fixed-point
deposit)."""
import numpy as np
import pytest

import oracle as O
from oracle import bounded as B
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
    # nx, ny, lx, ly, n, tile, vdim, bz
    (48, 20, 48.0 * 0.5, 20.0 * 0.75, 30011, (8, 4), 2, 0.0),
    (32, 16, 32.0, 16.0, 20011, (16, 8), 3, 1.5),
]


def _box(case):
    nx, ny, lx, ly, n, tile, vdim, bz = case
    return B.Box(nx, lx, ny, ly, n, 0.1, bz=bz, vdim=vdim)


def _ctx(torch, case, precision="fp64"):
    from paper_2608_15249_amd.apic import Context, Particles
    nx, ny, lx, ly, n, tile, vdim, bz = case
    c = Context(dim=2, vdim=vdim, nx=nx, ny=ny, lx=lx, ly=ly, dt=0.1, n=n, bz=bz, precision=precision, tile=tile,
                walls=True)
    return c, Particles(c)


def _state(rng, case, vth=1.5):
    nx, ny, lx, ly, n, tile, vdim, bz = case
    return (rng.uniform(0, lx, n), rng.uniform(0, ly, n)) + tuple(rng.normal(0, vth, n) for _ in range(vdim))


def _ext(b, a):
    """A physical [ny][nx+1] grid array placed in the [ny][2nx] layout."""
    out = np.zeros((b.ny, 2 * b.nx))
    out[:, :b.nx + 1] = a
    return out


def _phys(b, flat):
    return flat.reshape(b.ny, 2 * b.nx)[:, :b.nx + 1]


def _compose(ids, perm, nlive):
    return ids[perm.cpu().numpy().astype(np.int64)[:nlive]]


@pytest.mark.parametrize("case", CASES)
def test_dirichlet_field_solve_matches_oracle(torch, case):
    rng = np.random.default_rng(91)
    b = _box(case)
    rho = rng.normal(size=(b.ny, b.nx + 1))
    c, p = _ctx(torch, case)
    E = torch.zeros(2 * c.G, dtype=torch.float64, device="cuda")
    we = torch.zeros(1, dtype=torch.float64, device="cuda")
    c.field_solve(torch.from_numpy(_ext(b, rho).ravel()).cuda(), E, we=we)
    c.sync()
    Eo = B.solve_field(b, rho)
    Eg = E.cpu().numpy().reshape(2, -1)
    scale = max(np.max(np.abs(e)) for e in Eo)
    for d in range(2):
        assert np.max(np.abs(_phys(b, Eg[d]) - Eo[d])) <= 1e-12 * scale, d
    assert abs(we.item() / B.field_energy(b, Eo) - 1) < 1e-11


@pytest.mark.parametrize("case", CASES)
def test_fp64_steps_with_absorption_match_oracle(torch, case):
    rng = np.random.default_rng(92)
    b = _box(case)
    st0 = _state(rng, case)
    n = case[4]
    vdim = case[6]
    c, p = _ctx(torch, case)
    x, y = st0[0], st0[1]
    v = list(st0[2:])
    p.upload(x=x, y=y, vx=v[0], vy=v[1], vz=v[2] if vdim == 3 else None)
    perm = torch.zeros(n, dtype=torch.int32, device="cuda")
    c.sort_by_cell(p, perm=perm)
    ids = _compose(np.arange(n), perm, n)
    rho = torch.zeros(c.G, dtype=torch.float64, device="cuda")
    E = torch.zeros(2 * c.G, dtype=torch.float64, device="cuda")
    c.deposit(p, rho)
    c.field_solve(rho, E)
    c.gather_push(p, E, dt_scale=-0.5, move=False)
    po = B.Plasma(x.copy(), y.copy(), [a.copy() for a in v], ids=np.arange(n))
    Eo = B.initialise(b, po)
    nsteps = 8
    diag = torch.zeros(4 * nsteps, dtype=torch.float64, device="cuda")
    ref = []
    nlive = n
    for k in range(nsteps):
        c.step(p, E, None, 1, diag[4 * k:4 * k + 4], perm=perm)
        nlive = int(p.bucket_start[-1].item())
        ids = _compose(ids, perm, nlive)
        Eo, _, ke = B.step(b, po, Eo)
        ref.append((b.Q * len(po.x), B.field_energy(b, Eo), ke))
    c.sync()
    assert nlive == len(po.x) < n
    assert np.array_equal(np.sort(ids), np.sort(po.ids))
    order = np.argsort(po.ids)
    where = order[np.searchsorted(po.ids[order], ids)]      # oracle index of each GPU slot
    d = p.download()
    for k, r in (("x", po.x), ("y", po.y), ("vx", po.v[0]), ("vy", po.v[1])) + \
            ((("vz", po.v[2]),) if vdim == 3 else ()):
        assert np.max(np.abs(d[k][:nlive] - r[where])) <= 1e-10 * max(1.0, b.Lx), k
    Eg = E.cpu().numpy().reshape(2, -1)
    scale = max(np.max(np.abs(e)) for e in Eo)
    for dd in range(2):
        assert np.max(np.abs(_phys(b, Eg[dd]) - Eo[dd])) <= 1e-10 * scale
    dg = diag.cpu().numpy().reshape(nsteps, 4)
    ref = np.array(ref)
    assert np.allclose(dg[:, 0], ref[:, 0], rtol=1e-12, atol=0)     # charge of the live particles
    assert np.allclose(dg[:, 1], ref[:, 1], rtol=1e-9, atol=0)      # W_E
    assert np.allclose(dg[:, 2], ref[:, 2], rtol=1e-12, atol=0)     # kinetic (pushed particles)


@pytest.mark.parametrize("case", CASES)
def test_mixed_step_with_absorption_bit_exact(torch, case):
    rng = np.random.default_rng(93)
    b = _box(case)
    nx, ny, lx, ly, n, tile, vdim, bz = case
    st0 = _state(rng, case, vth=4.0)
    c, p = _ctx(torch, case, "mixed")
    cx, ox = W.to_cell_offset(st0[0], b.dx, b.nx)
    cy, oy = W.to_cell_offset(st0[1], b.dy, b.ny)
    v = st0[2:]
    p.upload(cell=W.pack_cell(cx, cy), ox=ox, oy=oy, vx=v[0], vy=v[1], vz=v[2] if vdim == 3 else None)
    perm = torch.zeros(n, dtype=torch.int32, device="cuda")
    c.sort_by_cell(p, perm=perm)
    d0 = p.download()
    u = W.unpack_cell(d0["cell"], 2)
    m0 = {"ix": u[0], "iy": u[1], "ox": d0["ox"], "oy": d0["oy"], "vx": d0["vx"], "vy": d0["vy"]}
    if vdim == 3:
        m0["vz"] = d0["vz"]
    # a field on the whole extended grid (host generated; both sides read it)
    E0 = tuple(rng.normal(size=(ny, 2 * nx)) * 0.5 for _ in range(2))
    E32 = tuple(e.astype(np.float32) for e in E0)
    Ed = torch.from_numpy(np.concatenate([e.ravel() for e in E0])).cuda()
    Iout = torch.zeros(c.G, dtype=torch.int64, device="cuda")
    c.step(p, Ed, None, 1, None, rho=Iout, perm=perm)
    c.sync()
    S = c.frac_bits
    se = O.Setup(2, vdim, 2 * nx, 2 * lx, n, 0.1, ny=ny, Ly=ly, bz=bz)
    ref = OM.push(m0, E32, dim=2, vdim=vdim, nx=2 * nx, ny=ny, dx=b.dx, dy=b.dy, qm=-1.0, dt=0.1, bz=bz)
    live = ref["ix"] < nx
    nlive = int(p.bucket_start[-1].item())
    assert nlive == int(live.sum()) < n
    pm = perm.cpu().numpy().astype(np.int64)[:nlive]
    assert np.all(live[pm])
    d1 = p.download()
    u1 = W.unpack_cell(d1["cell"][:nlive], 2)
    got = {"ix": u1[0], "iy": u1[1], "ox": d1["ox"][:nlive], "oy": d1["oy"][:nlive], "vx": d1["vx"][:nlive],
           "vy": d1["vy"][:nlive]}
    if vdim == 3:
        got["vz"] = d1["vz"][:nlive]
    for k in got:
        assert np.array_equal(got[k], ref[k][pm]), k
    I1 = O.deposit_quantised(se, ref["ix"][live], ref["ox"][live], S, ref["iy"][live], ref["oy"][live])
    assert np.array_equal(Iout.cpu().numpy().reshape(I1.shape), I1)
    # every particle slot of the new order holds a distinct live particle
    assert len(np.unique(pm)) == nlive


def test_walls_context_checks(torch):
    from paper_2608_15249_amd.apic import ApicError, Context
    with pytest.raises(ApicError):
        Context(dim=3, vdim=3, nx=8, ny=8, nz=8, lx=8.0, ly=8.0, lz=8.0, dt=0.1, n=100, precision="fp64",
                walls=True)
    with pytest.raises(ApicError):
        Context(dim=2, vdim=3, nx=16, ny=16, lx=16.0, ly=16.0, dt=0.05, n=100, precision="fp64", c_light=5.0,
                model="em", walls=True)
    c = Context(dim=2, vdim=2, nx=24, ny=8, lx=24.0, ly=8.0, dt=0.1, n=100, precision="fp64", tile=(16, 8),
                walls=True)
    assert 24 % c.tile[0] == 0          # the wall is a tile edge
    with pytest.raises(ApicError):
        c.adjoint_sizes(4, 2)
