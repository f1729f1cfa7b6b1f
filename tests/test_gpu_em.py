"""GPU parity of the electromagnetic step (FP64 2D3V, periodic Yee grid)
against the oracle, through the C ABI: initial field, gather + Boris, the
current of one step (Esirkepov), the field update, several steps with the
energy diagnostics, and the discrete Gauss law kept on the GPU."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from oracle import em as M
from paper_2608_15249_amd import workloads as W

pytestmark = pytest.mark.gpu

C_LIGHT = 5.0


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2608_15249_amd import apic
    apic.load_library()
    return t


CASES = [
    # nx, ny, lx, ly, n, tile, dt, bz
    (37, 29, 37.0, 29.0 * 0.9, 30011, (8, 8), 0.1, 1.5),
    (40, 24, 40.0 * 1.1, 24.0, 40003, (16, 16), 0.1, 0.0),
    # narrower than a field-update tile and its halo along both axes
    (16, 12, 16.0, 12.0 * 1.1, 8011, (8, 4), 0.1, 0.7),
    # the mixed path's default tile shape
    (64, 48, 64.0, 48.0, 60013, (32, 16), 0.1, 1.0),
]


def _setup(case):
    nx, ny, lx, ly, n, tile, dt, bz = case
    return O.Setup(2, 3, nx, lx, n, dt, ny=ny, Ly=ly, bz=bz, c=C_LIGHT)


def _ctx(torch, case):
    from paper_2608_15249_amd.apic import Context, Particles
    nx, ny, lx, ly, n, tile, dt, bz = case
    c = Context(dim=2, vdim=3, nx=nx, ny=ny, lx=lx, ly=ly, dt=dt, n=n, bz=bz, precision="fp64", tile=tile,
                c_light=C_LIGHT, model="em")
    return c, Particles(c)


def _state(rng, case):
    nx, ny, lx, ly, n, tile, dt, bz = case
    return (rng.uniform(0, lx, n), rng.uniform(0, ly, n), rng.normal(0, 1, n), rng.normal(0, 1, n),
            rng.normal(0, 1, n))


def _upload(p, st):
    x, y, vx, vy, vz = st
    p.upload(x=x, y=y, vx=vx, vy=vy, vz=vz)


def _compose(ids, perm):
    return ids[perm.cpu().numpy().astype(np.int64)]


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()


def _pdist(a, b, L):
    d = np.abs(a - b)
    return np.minimum(d, L - d)


@pytest.mark.parametrize("case", CASES)
def test_initial_fields_match_oracle(torch, case):
    rng = np.random.default_rng(71)
    s = _setup(case)
    st0 = _state(rng, case)
    c, p = _ctx(torch, case)
    _upload(p, st0)
    F = torch.zeros(6 * c.G, dtype=torch.float64, device="cuda")
    c.em_init_fields(p, F)
    c.sync()
    x, y, vx, vy, vz = st0
    Fo = M.initial_fields(s, O.State.from_arrays(x, vx, y, vy, vz))
    Fg = F.cpu().numpy().reshape(6, s.ny, s.nx)
    scale = np.max(np.abs(Fo[:2]))
    assert np.max(np.abs(Fg - Fo)) <= 1e-12 * scale


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("dt_scale,move", [(1.0, True), (-0.5, False)])
def test_gather_push_matches_oracle(torch, case, dt_scale, move):
    rng = np.random.default_rng(72)
    s = _setup(case)
    st0 = _state(rng, case)
    F = rng.normal(size=(6, s.ny, s.nx))
    F[5] += s.bz
    c, p = _ctx(torch, case)
    _upload(p, st0)
    c.em_gather_push(p, _dev(torch, F), dt_scale=dt_scale, move=move)
    c.sync()
    d = p.download()
    x, y, vx, vy, vz = st0
    st = O.State.from_arrays(x, vx, y, vy, vz)
    Ep, Bp = M.gather(s, st, F)
    M.boris(s, st, Ep, Bp, dt_scale * s.dt)
    if move:
        O.move(s, st)
    for k, ref in (("vx", st.vx), ("vy", st.vy), ("vz", st.vz)):
        assert np.max(np.abs(d[k] - ref)) <= 1e-12, k
    for k, ref, L in (("x", st.x, s.Lx), ("y", st.y, s.Ly)):
        assert np.max(_pdist(d[k], ref, L)) <= 1e-12 * L, k


def _start(torch, case, rng):
    """Sorted GPU plasma with F^0 and the backward half push, and the oracle's
    copy in the input order (ids maps GPU slots to input indices)."""
    s = _setup(case)
    st0 = _state(rng, case)
    n = case[4]
    c, p = _ctx(torch, case)
    _upload(p, st0)
    perm = torch.zeros(n, dtype=torch.int32, device="cuda")
    c.sort_by_cell(p, perm=perm)
    ids = _compose(np.arange(n), perm)
    F = torch.zeros(6 * c.G, dtype=torch.float64, device="cuda")
    c.em_init_fields(p, F)
    c.em_gather_push(p, F, dt_scale=-0.5, move=False)
    x, y, vx, vy, vz = st0
    st = O.State.from_arrays(x, vx, y, vy, vz)
    Fo = M.initialise(s, st)
    return s, c, p, perm, ids, F, st, Fo


@pytest.mark.parametrize("case", CASES)
def test_one_step_current_fields_and_particles(torch, case):
    rng = np.random.default_rng(73)
    s, c, p, perm, ids, F, st, Fo = _start(torch, case, rng)
    J = torch.zeros(3 * c.G, dtype=torch.float64, device="cuda")
    c.em_step(p, F, 1, J=J, perm=perm)
    ids = _compose(ids, perm)
    c.sync()
    Jo, _ = M.step(s, st, Fo)
    Jg = J.cpu().numpy().reshape(3, s.ny, s.nx)
    assert np.max(np.abs(Jg - Jo)) <= 1e-12 * np.max(np.abs(Jo))
    Fg = F.cpu().numpy().reshape(6, s.ny, s.nx)
    assert np.max(np.abs(Fg[:3] - Fo[:3])) <= 1e-12 * np.max(np.abs(Fo[:3]))
    assert np.max(np.abs(Fg[3:] - Fo[3:])) <= 1e-12 * max(1.0, np.max(np.abs(Fo[3:])))
    d = p.download()
    for k, ref in (("vx", st.vx), ("vy", st.vy), ("vz", st.vz)):
        assert np.max(np.abs(d[k] - ref[ids])) <= 1e-12, k
    for k, ref, L in (("x", st.x, s.Lx), ("y", st.y, s.Ly)):
        assert np.max(_pdist(d[k], ref[ids], L)) <= 1e-12 * L, k
    # the new order is the stable bucket order of the new positions
    key = O.bucket_key(np.floor(d["x"] / s.dx).astype(np.int64) % s.nx, np.floor(d["y"] / s.dy).astype(np.int64) % s.ny,
                       c.tile[0], c.tile[1], s.nx)
    assert np.all(np.diff(key) >= 0)


@pytest.mark.parametrize("case", CASES)
def test_eight_steps_and_diagnostics_match_oracle(torch, case):
    rng = np.random.default_rng(74)
    s, c, p, perm, ids, F, st, Fo = _start(torch, case, rng)
    nsteps = 8
    diag = torch.zeros(4 * nsteps, dtype=torch.float64, device="cuda")
    ref = []
    for k in range(nsteps):
        c.em_step(p, F, 1, diag=diag[4 * k:4 * k + 4], perm=perm)
        ids = _compose(ids, perm)
        _, ke = M.step(s, st, Fo)
        ref.append(M.field_energies(s, Fo) + (ke,))
    c.sync()
    d = p.download()
    for k, r in (("vx", st.vx), ("vy", st.vy), ("vz", st.vz)):
        assert np.max(np.abs(d[k] - r[ids])) <= 1e-10, k
    for k, r, L in (("x", st.x, s.Lx), ("y", st.y, s.Ly)):
        assert np.max(_pdist(d[k], r[ids], L)) <= 1e-10 * L, k
    Fg = F.cpu().numpy().reshape(6, s.ny, s.nx)
    assert np.max(np.abs(Fg - Fo)) <= 1e-10 * max(1.0, np.max(np.abs(Fo)))
    dg = diag.cpu().numpy().reshape(nsteps, 4)
    ref = np.array(ref)
    assert np.allclose(dg[:, 1], ref[:, 0], rtol=1e-9, atol=0)          # W_E
    assert np.allclose(dg[:, 0], ref[:, 1], rtol=1e-8, atol=1e-300)     # W_B (starts at zero)
    assert np.allclose(dg[:, 2], ref[:, 2], rtol=1e-12, atol=0)         # kinetic


def test_gauss_law_and_div_b_are_kept_on_the_gpu(torch):
    case = CASES[0]
    rng = np.random.default_rng(75)
    s, c, p, perm, ids, F, st, Fo = _start(torch, case, rng)
    c.em_step(p, F, 20)
    rho = torch.zeros(c.G, dtype=torch.float64, device="cuda")
    c.deposit(p, rho, tiled=False)
    c.sync()
    Fg = F.cpu().numpy().reshape(6, s.ny, s.nx)
    r = rho.cpu().numpy().reshape(s.ny, s.nx)
    assert np.max(np.abs(M.divergence_e(s, Fg) - r)) <= 1e-11 * np.max(np.abs(r))
    assert np.max(np.abs(M.divergence_b(s, Fg))) <= 1e-11 * max(1.0, np.max(np.abs(Fg[3:])))
    assert np.max(np.abs(Fg[3:5])) > 1e-6


def test_electromagnetic_context_checks(torch):
    from paper_2608_15249_amd.apic import ApicError, Context
    nx, ny = 16, 16
    with pytest.raises(ApicError):       # Courant condition: 8 * 0.1 * sqrt(2) > 1
        Context(dim=2, vdim=3, nx=nx, ny=ny, lx=16.0, ly=16.0, dt=0.1, n=100, precision="fp64", c_light=8.0,
                model="em")
    with pytest.raises(ApicError):       # 2D3V only
        Context(dim=2, vdim=2, nx=nx, ny=ny, lx=16.0, ly=16.0, dt=0.1, n=100, precision="fp64", c_light=5.0,
                model="em")
    c, p = _ctx(torch, CASES[0])
    E = torch.zeros(2 * c.G, dtype=torch.float64, device="cuda")
    with pytest.raises(ApicError):
        c.gather_push(p, E)
    with pytest.raises(ApicError):
        c.step(p, E, None, 1)


def test_a_move_of_a_cell_is_reported(torch):
    """A particle displaced a cell or more in one step is outside the current
    deposit's window: the step flags APIC_EDOMAIN (the host forces the
    condition with one fast particle; every kernel exits normally)."""
    from paper_2608_15249_amd.apic import ApicError
    case = CASES[0]
    rng = np.random.default_rng(76)
    s = _setup(case)
    x, y, vx, vy, vz = _state(rng, case)
    vx[17] = 15.0                       # 1.5 cells per step
    c, p = _ctx(torch, case)
    _upload(p, (x, y, vx, vy, vz))
    c.sort_by_cell(p)
    F = torch.zeros(6 * c.G, dtype=torch.float64, device="cuda")
    c.em_init_fields(p, F)
    c.em_step(p, F, 1)
    with pytest.raises(ApicError):
        c.sync()


def test_full_size_magnetized_plasma_sampled(torch):
    """magnetized_2d3v at its full size (1024^2 cells, 33,554,432 electrons,
    c = 10, the default tile the benchmark uses): one step after the initial
    field and half push. 4096 sampled particles against the oracle's
    per-particle gather, Boris and move in the oracle's F^0; Gauss's law of the
    step's output field and charge, and the total-current sum rule, on the
    whole grid."""
    from paper_2608_15249_amd.apic import Context, Particles
    w = W.magnetized_2d3v()
    x, y, vx, vy, vz = W.sample(w)
    n = len(x)
    cl = 10.0
    s = O.Setup(2, 3, w.nx, w.Lx, n, w.dt, ny=w.ny, Ly=w.Ly, bz=w.bz, c=cl)
    c = Context(dim=2, vdim=3, nx=w.nx, ny=w.ny, lx=w.Lx, ly=w.Ly, dt=w.dt, n=n, bz=w.bz, precision="fp64",
                c_light=cl, model="em")
    p = Particles(c)
    p.upload(x=x, y=y, vx=vx, vy=vy, vz=vz)
    perm = torch.zeros(n, dtype=torch.int32, device="cuda")
    c.sort_by_cell(p, perm=perm)
    ids = _compose(np.arange(n), perm)
    F = torch.zeros(6 * c.G, dtype=torch.float64, device="cuda")
    c.em_init_fields(p, F)
    c.em_gather_push(p, F, dt_scale=-0.5, move=False)
    J = torch.zeros(3 * c.G, dtype=torch.float64, device="cuda")
    c.em_step(p, F, 1, J=J, perm=perm)
    ids = _compose(ids, perm)
    rho = torch.zeros(c.G, dtype=torch.float64, device="cuda")
    c.deposit(p, rho, tiled=False)
    c.sync()
    d = p.download()
    F0 = M.initial_fields(s, O.State.from_arrays(x, vx, y, vy, vz))
    rng = np.random.default_rng(77)
    slots = rng.choice(n, 4096, replace=False)
    src = ids[slots]
    st = O.State.from_arrays(x[src], vx[src], y[src], vy[src], vz[src])
    sub = dataclasses.replace(s, n_particles=len(src))
    Ep, Bp = M.gather(sub, st, F0)
    M.boris(sub, st, Ep, Bp, -0.5 * s.dt)
    Ep, Bp = M.gather(sub, st, F0)
    M.boris(sub, st, Ep, Bp, s.dt)
    O.move(sub, st)
    for k, ref in (("vx", st.vx), ("vy", st.vy), ("vz", st.vz)):
        assert np.max(np.abs(d[k][slots] - ref)) <= 1e-12, k
    for k, ref, L in (("x", st.x, s.Lx), ("y", st.y, s.Ly)):
        assert np.max(_pdist(d[k][slots], ref, L)) <= 1e-12 * L, k
    Fg = F.cpu().numpy().reshape(6, s.ny, s.nx)
    r = rho.cpu().numpy().reshape(s.ny, s.nx)
    assert np.max(np.abs(M.divergence_e(s, Fg) - r)) <= 1e-11 * np.max(np.abs(r))
    Jg = J.cpu().numpy().reshape(3, -1)
    tot = Jg.sum(axis=1) * s.dV
    ref = s.Q * np.array([d["vx"].sum(), d["vy"].sum(), d["vz"].sum()])
    assert np.max(np.abs(tot - ref)) <= 1e-9 * np.sum(np.abs(s.Q * d["vx"]))


# ------------------------------------------------------------------ mixed form
# binary32 field tile, gather, Boris and current weights; FP64 current sums
# and field update. Compared with the FP64 oracle at binary32 tolerances, and
# held to the local field-energy criterion of the mixed path.

def _mctx(torch, case):
    from paper_2608_15249_amd.apic import Context, Particles
    nx, ny, lx, ly, n, tile, dt, bz = case
    c = Context(dim=2, vdim=3, nx=nx, ny=ny, lx=lx, ly=ly, dt=dt, n=n, bz=bz, precision="mixed", tile=tile,
                c_light=C_LIGHT, model="em")
    return c, Particles(c)


def _mixed_state(rng, case, s):
    """A mixed-representation state and its exact FP64 positions."""
    x, y, vx, vy, vz = _state(rng, case)
    cx, ox = W.to_cell_offset(x, s.dx, s.nx)
    cy, oy = W.to_cell_offset(y, s.dy, s.ny)
    xe = (cx + ox.astype(np.float64)) * s.dx
    ye = (cy + oy.astype(np.float64)) * s.dy
    v32 = [a.astype(np.float32) for a in (vx, vy, vz)]
    return (cx, ox, cy, oy), (xe, ye), v32


@pytest.mark.parametrize("case", CASES)
def test_mixed_gather_push_tracks_oracle(torch, case):
    rng = np.random.default_rng(78)
    s = _setup(case)
    (cx, ox, cy, oy), (xe, ye), v32 = _mixed_state(rng, case, s)
    F = rng.normal(size=(6, s.ny, s.nx))
    F[5] += s.bz
    c, p = _mctx(torch, case)
    p.upload(cell=W.pack_cell(cx, cy), ox=ox, oy=oy, vx=v32[0], vy=v32[1], vz=v32[2])
    c.em_gather_push(p, _dev(torch, F), dt_scale=1.0, move=True)
    c.sync()
    d = p.download()
    st = O.State.from_arrays(xe, v32[0].astype(np.float64), ye, v32[1].astype(np.float64), v32[2].astype(np.float64))
    Ep, Bp = M.gather(s, st, F)
    M.boris(s, st, Ep, Bp, s.dt)
    O.move(s, st)
    for k, ref in (("vx", st.vx), ("vy", st.vy), ("vz", st.vz)):
        assert np.max(np.abs(d[k] - ref)) <= 2e-5 * (1 + np.max(np.abs(ref))), k
    ix, iy = W.unpack_cell(d["cell"], 2)
    for pos, ref, dd, L in (((ix + d["ox"].astype(np.float64)) * s.dx, st.x, s.dx, s.Lx),
                            ((iy + d["oy"].astype(np.float64)) * s.dy, st.y, s.dy, s.Ly)):
        assert np.max(_pdist(pos, ref, L)) <= 2e-6 * dd * 10


@pytest.mark.parametrize("case", CASES)
def test_mixed_step_current_and_local_field_energy(torch, case):
    """From the same state: the mixed step's J and fields agree with the FP64
    oracle step in the oracle's field of the same quantised charge to binary32
    accuracy, and its field energy W_E + W_B within 1e-5 (relative)."""
    rng = np.random.default_rng(79)
    s = _setup(case)
    n = case[4]
    (cx, ox, cy, oy), (xe, ye), v32 = _mixed_state(rng, case, s)
    c, p = _mctx(torch, case)
    p.upload(cell=W.pack_cell(cx, cy), ox=ox, oy=oy, vx=v32[0], vy=v32[1], vz=v32[2])
    perm = torch.zeros(n, dtype=torch.int32, device="cuda")
    c.sort_by_cell(p, perm=perm)
    ids = _compose(np.arange(n), perm)
    F = torch.zeros(6 * c.G, dtype=torch.float64, device="cuda")
    c.em_init_fields(p, F)
    S = c.frac_bits
    I0 = O.deposit_quantised(s, cx, ox, S, cy, oy)
    Fo = np.zeros((6, s.ny, s.nx))
    Fo[0], Fo[1] = M.staggered_e(s, O.solve_potential(s, O.rho_from_quantised(s, I0, S)))
    Fo[5] = s.bz
    c.sync()
    Fg0 = F.cpu().numpy().reshape(6, s.ny, s.nx)
    assert np.max(np.abs(Fg0 - Fo)) <= 1e-12 * np.max(np.abs(Fo[:2])) + 1e-15
    J = torch.zeros(3 * c.G, dtype=torch.float64, device="cuda")
    diag = torch.zeros(4, dtype=torch.float64, device="cuda")
    c.em_step(p, F, 1, diag=diag, J=J, perm=perm)
    c.sync()
    st = O.State.from_arrays(xe, v32[0].astype(np.float64), ye, v32[1].astype(np.float64), v32[2].astype(np.float64))
    Jo, _ = M.step(s, st, Fo)
    Jg = J.cpu().numpy().reshape(3, s.ny, s.nx)
    assert np.max(np.abs(Jg - Jo)) <= 1e-5 * np.max(np.abs(Jo))
    Fg = F.cpu().numpy().reshape(6, s.ny, s.nx)
    assert np.max(np.abs(Fg[:3] - Fo[:3])) <= 1e-5 * np.max(np.abs(Fo[:3]))
    we, wb = M.field_energies(s, Fo)
    dg = diag.cpu().numpy()
    assert abs((dg[0] + dg[1]) / (we + wb) - 1) <= 1e-5
    ids = _compose(ids, perm)
    d = p.download()
    for k, ref in (("vx", st.vx), ("vy", st.vy), ("vz", st.vz)):
        assert np.max(np.abs(d[k] - ref[ids])) <= 2e-5 * (1 + np.max(np.abs(ref))), k


def test_mixed_gauss_law_is_kept_to_binary32_accuracy(torch):
    case = CASES[0]
    rng = np.random.default_rng(80)
    s = _setup(case)
    (cx, ox, cy, oy), _, v32 = _mixed_state(rng, case, s)
    c, p = _mctx(torch, case)
    p.upload(cell=W.pack_cell(cx, cy), ox=ox, oy=oy, vx=v32[0], vy=v32[1], vz=v32[2])
    c.sort_by_cell(p)
    F = torch.zeros(6 * c.G, dtype=torch.float64, device="cuda")
    c.em_init_fields(p, F)
    c.em_gather_push(p, F, dt_scale=-0.5, move=False)
    c.em_step(p, F, 20)
    I = torch.zeros(c.G, dtype=torch.int64, device="cuda")
    c.deposit(p, I)
    c.sync()
    r = O.rho_from_quantised(s, I.cpu().numpy().reshape(s.ny, s.nx), c.frac_bits)
    Fg = F.cpu().numpy().reshape(6, s.ny, s.nx)
    assert np.max(np.abs(M.divergence_e(s, Fg) - r)) <= 1e-4 * np.max(np.abs(r))
    assert np.max(np.abs(M.divergence_b(s, Fg))) <= 1e-11 * max(1.0, np.max(np.abs(Fg[3:])))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_empty_plasma_evolves_the_vacuum_field(torch, precision):
    """No particles: an empty bucket table, zero current, and the field update
    alone, against the oracle's steps of the same field with an empty state."""
    from paper_2608_15249_amd.apic import Context, Particles
    nx, ny, lx, ly, dt, bz = 16, 12, 16.0, 13.2, 0.1, 0.7
    c = Context(dim=2, vdim=3, nx=nx, ny=ny, lx=lx, ly=ly, dt=dt, n=0, bz=bz, precision=precision, tile=(8, 4),
                c_light=C_LIGHT, model="em")
    p = Particles(c)
    e = np.zeros(0)
    if precision == "mixed":
        f = e.astype(np.float32)
        p.upload(cell=np.zeros(0, np.int32), ox=f, oy=f, vx=f, vy=f, vz=f)
    else:
        p.upload(x=e, y=e, vx=e, vy=e, vz=e)
    c.sort_by_cell(p)
    rng = np.random.default_rng(91)
    Fo = rng.normal(size=(6, ny, nx))
    F = _dev(torch, Fo)
    J = torch.ones(3 * c.G, dtype=torch.float64, device="cuda")
    c.em_step(p, F, 5, J=J)
    c.sync()
    # the oracle's setup takes one nominal particle for its macro-charge,
    # which no particle carries
    s = O.Setup(2, 3, nx, lx, 1, dt, ny=ny, Ly=ly, bz=bz, c=C_LIGHT)
    st = O.State.from_arrays(e, e, e, e, e)
    for _ in range(5):
        M.step(s, st, Fo)
    assert np.all(p.bucket_start.cpu().numpy() == 0)
    assert np.all(J.cpu().numpy() == 0.0)
    Fg = F.cpu().numpy().reshape(6, ny, nx)
    assert np.max(np.abs(Fg - Fo)) <= 1e-12 * np.max(np.abs(Fo))


def test_steps_near_the_count_skip_threshold(torch):
    """A field near the count pass's skip threshold with the peaks of Ex and
    Ey on different Yee indices (so no single index carries the largest
    |E| a particle can gather), a B_z that turns the kick, and particles a
    quarter cell or more inside the tiles' edges: eight steps in one call
    match the oracle particle for particle, and the step reports no error
    (every (wave, direction) range of the scatter filled exactly)."""
    nx = ny = 32
    T = 8
    n = 20000
    bz, E0 = -2.47, 24.85
    s = O.Setup(2, 3, nx, float(nx), n, 0.1, ny=ny, Ly=float(ny), bz=bz, c=C_LIGHT)
    rng = np.random.default_rng(77)
    k = rng.integers(0, nx // T, n)
    x = k * T + rng.uniform(0.2505, 0.6, n)
    y = rng.uniform(0, ny, n)
    vx, vy, vz = (rng.normal(0, 0.3, n) for _ in range(3))
    F0 = np.zeros((6, ny, nx))
    i = np.arange(nx)
    F0[0][:, (i % 4 == 3) | (i % 4 == 0)] = E0
    F0[1][:, i % 4 == 1] = E0
    F0[5] += bz
    # the largest |E| at one index is E0, below the threshold the count pass
    # uses with that bound; a particle between the columns gathers more
    assert np.max(np.sqrt(F0[0] ** 2 + F0[1] ** 2 + F0[2] ** 2)) == E0
    assert 2 * 0.05 * 1.0009765625 * E0 * 0.1 + 0.0009765625 <= 0.25
    from paper_2608_15249_amd.apic import Context, Particles
    c = Context(dim=2, vdim=3, nx=nx, ny=ny, lx=float(nx), ly=float(ny), dt=0.1, n=n, bz=bz, precision="fp64",
                tile=(T, T), c_light=C_LIGHT, model="em")
    p = Particles(c)
    p.upload(x=x, y=y, vx=vx, vy=vy, vz=vz)
    c.sort_by_cell(p)
    F = _dev(torch, F0)
    nsteps = 6
    c.em_step(p, F, nsteps)
    c.sync()
    st = O.State.from_arrays(x, vx, y, vy, vz)
    Fo = F0.copy()
    for _ in range(nsteps):
        M.step(s, st, Fo)
    # compare as sets of particles, matched through their velocities
    d = p.download()
    key_g = np.lexsort((d["vz"], d["vy"], d["vx"]))
    key_o = np.lexsort((st.vz, st.vy, st.vx))
    for k_, ref in (("vx", st.vx), ("vy", st.vy), ("vz", st.vz)):
        assert np.max(np.abs(d[k_][key_g] - ref[key_o])) <= 1e-9, k_
    for k_, ref, L in (("x", st.x, s.Lx), ("y", st.y, s.Ly)):
        assert np.max(_pdist(d[k_][key_g], ref[key_o], L)) <= 1e-9 * L, k_
    Fg = F.cpu().numpy().reshape(6, ny, nx)
    assert np.max(np.abs(Fg - Fo)) <= 1e-9 * np.max(np.abs(Fo))
