"""GPU parity of the Higuera-Cary velocity advance (pusher "hc", state
u = gamma v) against the oracle, in 2D3V and 3D3V, through the C ABI.

Bars as elsewhere: the mixed path (binary32 Higuera-Cary, integer cell and
offset, fixed-point deposit) bit-exact against the oracle's binary32 reading;
the FP64 path within 1e-12 (a few dozen double operations per particle)."""
import numpy as np
import pytest

import oracle as O
from oracle import mixed as OM
from paper_2608_15249_amd import workloads as W

pytestmark = pytest.mark.gpu

C_LIGHT = 3.0      # thermal speed 1 (3 per component at the tails): mildly relativistic


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2608_15249_amd import apic
    apic.load_library()
    return t


CASES = [
    # dim, nx, ny, nz, lx, ly, lz, n, tile
    (2, 37, 29, 1, 37.0, 29.0, 1.0, 25013, (4, 8)),
    (3, 20, 12, 9, 10.0, 6.0, 4.5, 30011, (8, 4, 4)),
]


def _ctx(torch, case, precision, bz=2.0, c=C_LIGHT, pusher="hc"):
    from paper_2608_15249_amd.apic import Context, Particles
    dim, nx, ny, nz, lx, ly, lz, n, tile = case
    ctx = Context(dim=dim, vdim=3, nx=nx, ny=ny, lx=lx, ly=ly, dt=0.1, n=n, bz=bz, precision=precision, tile=tile,
                  nz=nz, lz=lz, pusher=pusher, c_light=c)
    return ctx, Particles(ctx)


def _setup(case, bz=2.0, c=C_LIGHT):
    dim, nx, ny, nz, lx, ly, lz, n, tile = case
    return O.Setup(dim, 3, nx, lx, n, 0.1, ny=ny, Ly=ly, nz=nz, Lz=lz, bz=bz, pusher="hc", c=c)


def _state(rng, case, uth=1.5):
    dim, nx, ny, nz, lx, ly, lz, n, tile = case
    x, y = rng.uniform(0, lx, n), rng.uniform(0, ly, n)
    z = rng.uniform(0, lz, n) if dim == 3 else None
    return x, y, z, rng.normal(0, uth, n), rng.normal(0, uth, n), rng.normal(0, uth, n)


def _upload(p, s, st, mixed):
    x, y, z, ux, uy, uz = st
    if not mixed:
        p.upload(x=x, y=y, z=z, vx=ux, vy=uy, vz=uz)
        return
    cx, ox = W.to_cell_offset(x, s.dx, s.nx)
    cy, oy = W.to_cell_offset(y, s.dy, s.ny)
    if s.dim == 3:
        cz, oz = W.to_cell_offset(z, s.dz, s.nz)
        p.upload(cell=W.pack_cell(cx, cy, cz), ox=ox, oy=oy, oz=oz, vx=ux, vy=uy, vz=uz)
    else:
        p.upload(cell=W.pack_cell(cx, cy), ox=ox, oy=oy, vx=ux, vy=uy, vz=uz)


def _mstate(d, dim):
    u = W.unpack_cell(d["cell"], dim)
    m = {"ix": u[0], "iy": u[1], "ox": d["ox"], "oy": d["oy"], "vx": d["vx"], "vy": d["vy"], "vz": d["vz"]}
    if dim == 3:
        m.update(iz=u[2], oz=d["oz"])
    return m


def _keys(dim):
    return ("ix", "iy", "ox", "oy", "vx", "vy", "vz") + (("iz", "oz") if dim == 3 else ())


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("tiled", [False, True])
def test_gather_push_fp64_hc(torch, case, tiled):
    rng = np.random.default_rng(41)
    s = _setup(case)
    E = tuple(rng.normal(size=s.grid_shape) for _ in range(s.dim))
    c, p = _ctx(torch, case, "fp64")
    _upload(p, s, _state(rng, case), False)
    if tiled:
        c.sort_by_cell(p)
    d0 = p.download()
    c.gather_push(p, torch.from_numpy(np.concatenate([e.ravel() for e in E])).cuda(), tiled=tiled)
    c.sync()
    d1 = p.download()
    st = O.State.from_arrays(d0["x"], d0["vx"], d0["y"], d0["vy"], d0["vz"], d0["z"])
    O.boris(s, st, O.gather(s, st, E), s.dt)
    O.move(s, st)
    for k, ref in (("vx", st.vx), ("vy", st.vy), ("vz", st.vz)):
        assert np.max(np.abs(d1[k] - ref)) <= 1e-12, k
    for k, ref, L in (("x", st.x, s.Lx), ("y", st.y, s.Ly), ("z", st.z, s.Lz)):
        if ref is not None:
            dd = np.abs(d1[k] - ref)
            assert np.max(np.minimum(dd, L - dd)) <= 1e-12 * L, k


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("dt_scale", [1.0, -0.5])
def test_gather_push_mixed_bit_exact_hc(torch, case, dt_scale):
    rng = np.random.default_rng(42)
    s = _setup(case)
    E32 = tuple(rng.normal(size=s.grid_shape).astype(np.float32) for _ in range(s.dim))
    c, p = _ctx(torch, case, "mixed")
    _upload(p, s, _state(rng, case), True)
    c.sort_by_cell(p)
    m0 = _mstate(p.download(), s.dim)
    move = dt_scale == 1.0
    c.gather_push(p, torch.from_numpy(np.concatenate([e.ravel() for e in E32])).cuda(), dt_scale=dt_scale,
                  move=move)
    c.sync()
    m1 = _mstate(p.download(), s.dim)
    ref = OM.push(m0, E32, dim=s.dim, vdim=3, nx=s.nx, ny=s.ny, dx=s.dx, dy=s.dy, qm=s.qm, dt=s.dt, bz=s.bz,
                  dt_scale=dt_scale, move=move, nz=s.nz, dz=s.dz, pusher="hc", c=s.c)
    for k in _keys(s.dim):
        assert np.array_equal(m1[k], ref[k]), k


def _compose(ids, perm):
    return ids[perm.cpu().numpy().astype(np.int64)]


@pytest.mark.parametrize("case", CASES)
def test_step_fp64_hc_matches_oracle(torch, case):
    rng = np.random.default_rng(43)
    s = _setup(case)
    st0 = _state(rng, case)
    n = case[7]
    c, p = _ctx(torch, case, "fp64")
    _upload(p, s, st0, False)
    perm = torch.zeros(n, dtype=torch.int32, device="cuda")
    c.sort_by_cell(p, perm=perm)
    ids = _compose(np.arange(n), perm)
    rho = torch.zeros(c.G, dtype=torch.float64, device="cuda")
    E = torch.zeros(s.dim * c.G, dtype=torch.float64, device="cuda")
    c.deposit(p, rho)
    c.field_solve(rho, E)
    c.gather_push(p, E, dt_scale=-0.5, move=False)
    x, y, z, ux, uy, uz = st0
    st = O.State.from_arrays(x, ux, y, uy, uz, z)
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
        assert np.max(np.abs(d[k] - ref[ids])) <= 1e-10, k
    dg = diag.cpu().numpy().reshape(nsteps, 4)
    assert np.allclose(dg[:, 1], ref_we, rtol=1e-9, atol=0)
    assert np.allclose(dg[:, 2], ref_ke, rtol=1e-12, atol=0)


@pytest.mark.parametrize("case", CASES)
def test_step_mixed_hc_one_step_bit_exact(torch, case):
    rng = np.random.default_rng(44)
    s = _setup(case)
    n = case[7]
    c, p = _ctx(torch, case, "mixed")
    _upload(p, s, _state(rng, case), True)
    S = c.frac_bits
    perm = torch.zeros(n, dtype=torch.int32, device="cuda")
    c.sort_by_cell(p, perm=perm)
    m0 = _mstate(p.download(), s.dim)
    E0 = tuple(rng.normal(size=s.grid_shape) for _ in range(s.dim))
    E32 = tuple(e.astype(np.float32) for e in E0)
    Ed = torch.from_numpy(np.concatenate([e.ravel() for e in E0])).cuda()
    E32d = torch.from_numpy(np.concatenate([e.ravel() for e in E32])).cuda()
    Iout = torch.zeros(c.G, dtype=torch.int64, device="cuda")
    c.step(p, Ed, E32d, 1, None, rho=Iout, perm=perm)
    c.sync()
    ref = OM.push(m0, E32, dim=s.dim, vdim=3, nx=s.nx, ny=s.ny, dx=s.dx, dy=s.dy, qm=s.qm, dt=s.dt, bz=s.bz,
                  nz=s.nz, dz=s.dz, pusher="hc", c=s.c)
    pm = perm.cpu().numpy().astype(np.int64)
    m1 = _mstate(p.download(), s.dim)
    for k in _keys(s.dim):
        assert np.array_equal(m1[k], ref[k][pm]), k
    if s.dim == 3:
        I1 = O.deposit_quantised(s, ref["ix"], ref["ox"], S, ref["iy"], ref["oy"], ref["iz"], ref["oz"])
    else:
        I1 = O.deposit_quantised(s, ref["ix"], ref["ox"], S, ref["iy"], ref["oy"])
    assert np.array_equal(Iout.cpu().numpy().reshape(I1.shape), I1)


@pytest.mark.parametrize("case", CASES)
def test_hc_at_large_c_is_the_boris_path(torch, case):
    """FP64: with c = 1e30 the Higuera-Cary steps equal the Boris steps to
    rounding (the two rotations are the same map when gamma = 1)."""
    rng = np.random.default_rng(45)
    s = _setup(case)
    st0 = _state(rng, case)
    outs = []
    for pusher in ("hc", "boris"):
        c, p = _ctx(torch, case, "fp64", c=1e30 if pusher == "hc" else 0.0, pusher=pusher)
        _upload(p, s, st0, False)
        c.sort_by_cell(p)
        rho = torch.zeros(c.G, dtype=torch.float64, device="cuda")
        E = torch.zeros(s.dim * c.G, dtype=torch.float64, device="cuda")
        c.deposit(p, rho)
        c.field_solve(rho, E)
        c.gather_push(p, E, dt_scale=-0.5, move=False)
        c.step(p, E, None, 5)
        c.sync()
        outs.append(p.download())
    for k in ("vx", "vy", "vz"):
        assert np.max(np.abs(outs[0][k] - outs[1][k])) <= 1e-11, k
    for k, L in (("x", s.Lx), ("y", s.Ly), ("z", s.Lz)):
        if outs[0][k] is not None:
            dd = np.abs(outs[0][k] - outs[1][k])
            assert np.max(np.minimum(dd, L - dd)) <= 1e-11 * L, k


def _adj_case():
    import dataclasses
    w = dataclasses.replace(W.magnetized_2d3v(nx=16, ppc=32), mode=(1, 0))
    return w, W.sample(w)


def _gpu_grad(torch, w, state, nsteps, stride, precision, c=C_LIGHT):
    from paper_2608_15249_amd.adjoint import FieldEnergyRun
    x, y, vx, vy, vz = state
    run = FieldEnergyRun(dim=2, vdim=3, nx=w.nx, ny=w.ny, lx=w.Lx, ly=w.Ly, dt=w.dt, n=len(x), nsteps=nsteps,
                         stride=stride, bz=w.bz, precision=precision, pusher="hc", c_light=c)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    Wv = run.forward(*[dev(a) for a in (x, y, vx, vy, vz)])
    g = run.backward()
    run.sync()
    return float(Wv.item()), [a.cpu().numpy() for a in g[:5]]


def _oracle_grad(w, state, nsteps, c=C_LIGHT):
    from oracle import adjoint as OA
    x, y, vx, vy, vz = state
    s = O.Setup(2, 3, w.nx, w.Lx, len(x), w.dt, ny=w.ny, Ly=w.Ly, bz=w.bz, pusher="hc", c=c)
    Wv, lx, lv = OA.adjoint(s, O.State.from_arrays(x, vx, y, vy, vz), nsteps)
    return Wv, lx + lv


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_hc_fp64_adjoint_matches_oracle_gradient(torch):
    w, state = _adj_case()
    Wg, gg = _gpu_grad(torch, w, state, 20, 6, "fp64")
    Wo, go = _oracle_grad(w, state, 20)
    assert abs(Wg / Wo - 1.0) < 1e-11, (Wg, Wo)
    for k, (a, b) in enumerate(zip(gg, go)):
        assert _rel(a, b) < 1e-9, (k, _rel(a, b))


def test_hc_mixed_adjoint_matches_oracle_gradient(torch):
    """binary32 forward and adjoint against the FP64 reference gradient (the
    trajectories differ by binary32 rounding, as for Boris)."""
    w, state = _adj_case()
    Wg, gg = _gpu_grad(torch, w, state, 20, 6, "mixed")
    Wo, go = _oracle_grad(w, state, 20)
    assert abs(Wg / Wo - 1.0) < 1e-5, (Wg, Wo)
    for k, (a, b) in enumerate(zip(gg, go)):
        assert _rel(a, b) < 5e-5, (k, _rel(a, b))


def test_hc_adjoint_does_not_depend_on_checkpoint_stride(torch):
    w, state = _adj_case()
    ref = None
    for stride in (1, 7, 40):
        _, g = _gpu_grad(torch, w, state, 15, stride, "fp64")
        if ref is None:
            ref = g
            continue
        for a, b in zip(g, ref):
            assert _rel(a, b) < 1e-10, stride


def test_hc_zero_and_one_step_adjoint(torch):
    """0 steps: only the initial charge and the backward half push (whose
    gradient in u is zero: E^0 does not depend on u^0); 1 step: the half push
    inversion by time symmetry enters."""
    w, state = _adj_case()
    for nsteps in (0, 1):
        Wg, gg = _gpu_grad(torch, w, state, nsteps, 3, "fp64")
        Wo, go = _oracle_grad(w, state, nsteps)
        assert abs(Wg / Wo - 1.0) < 1e-12
        for a, b in zip(gg, go):
            if np.any(b):
                assert _rel(a, b) < 1e-10, nsteps
            else:
                assert np.max(np.abs(a)) == 0.0, nsteps


def test_hc_adjoint_strongly_relativistic(torch):
    """c = 0.8 v_th: gamma up to about 5 in the tails."""
    w, state = _adj_case()
    Wg, gg = _gpu_grad(torch, w, state, 10, 4, "fp64", c=0.8)
    Wo, go = _oracle_grad(w, state, 10, c=0.8)
    assert abs(Wg / Wo - 1.0) < 1e-11
    for k, (a, b) in enumerate(zip(gg, go)):
        assert _rel(a, b) < 1e-9, (k, _rel(a, b))
