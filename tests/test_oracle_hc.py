"""Pins of the Higuera-Cary velocity advance of the oracle (CPU only).

The paper lists the Higuera-Cary pusher beside Boris in A_Pusher and cites
Higuera & Cary (2017) for it. The pins are the properties that method is
built to have, each fixed by the mathematics rather than by the oracle: the
non-relativistic limit is the Boris map; every step satisfies the implicit
midpoint relation that defines the method (the magnetic rotation uses the
Lorentz factor of the mean of the old and new u); a pure magnetic field keeps
|u| and u_z; the relativistic E x B drift velocity is an exact fixed point; an
electric field along B changes only u_z, by (q/m) E dt per step; and the move
advances x by (u / gamma) dt."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from oracle import mixed as OM
from paper_2608_15249_amd import workloads as W


def _s(dim=2, bz=2.0, c=3.0, dt=0.05, n=1):
    if dim == 3:
        return O.Setup(3, 3, 8, 100.0, n, dt, ny=8, Ly=100.0, nz=8, Lz=100.0, bz=bz, pusher="hc", c=c)
    return O.Setup(2, 3, 8, 100.0, n, dt, ny=8, Ly=100.0, bz=bz, pusher="hc", c=c)


def _st(u, n=1):
    u = np.atleast_2d(u)
    return O.State.from_arrays(np.full(n, 50.0), u[:, 0].copy(), np.full(n, 50.0), u[:, 1].copy(), u[:, 2].copy(),
                               np.full(n, 50.0))


@pytest.mark.parametrize("dim", [2, 3])
def test_nonrelativistic_limit_is_boris(dim):
    rng = np.random.default_rng(21)
    n = 500
    sh = _s(dim, bz=1.7, c=1e30, n=n)
    sb = O.Setup(sh.dim, 3, 8, 100.0, n, 0.05, ny=8, Ly=100.0, nz=sh.nz, Lz=sh.Lz, bz=1.7)
    st = _st(rng.normal(size=(n, 3)), n)
    sr = st.copy()
    Ep = tuple(rng.normal(size=n) for _ in range(dim))
    for _ in range(10):
        O.boris(sh, st, Ep, sh.dt)
        O.boris(sb, sr, Ep, sb.dt)
    for a, b in ((st.vx, sr.vx), (st.vy, sr.vy), (st.vz, sr.vz)):
        assert np.max(np.abs(a - b)) < 1e-13


def test_step_satisfies_the_implicit_midpoint_relation():
    """The method's defining relation: u1 - u0 = 2 a E + (u1 + u0) x (tau /
    gamma_bar) z^ with gamma_bar the Lorentz factor of the mean (u0 + u1) / 2
    (the closed form is the solution of this implicit equation)."""
    rng = np.random.default_rng(24)
    for c in (0.9, 1.7, 6.0):
        for _ in range(20):
            bz, dt = rng.uniform(-3, 3), rng.uniform(0.01, 0.3)
            s = _s(3, bz=bz, c=c, dt=dt)
            a = s.qm * dt / 2
            u0 = rng.normal(size=3) * 2.0
            E = rng.normal(size=3)
            st = _st(u0)
            O.boris(s, st, tuple(np.array([e]) for e in E), dt)
            u1 = np.array([st.vx[0], st.vy[0], st.vz[0]])
            ub = 0.5 * (u0 + u1)
            gb = np.sqrt(1 + ub @ ub / c ** 2)
            r = u1 - u0 - 2 * a * E - np.cross(u0 + u1, np.array([0.0, 0.0, a * bz / gb]))
            assert np.max(np.abs(r)) < 1e-14 * (1 + np.abs(u1).max()), (c, r)


def test_pure_b_keeps_u():
    """E = 0: the step is a rotation about z (|u| and u_z kept to rounding)."""
    s = _s(2, bz=2.0, c=1.5, dt=0.05)
    u0 = np.array([2.4, -1.1, 0.7])
    st = _st(u0)
    zero = (np.zeros(1), np.zeros(1))
    for n in range(1, 201):
        O.boris(s, st, zero, s.dt)
        u = np.array([st.vx[0], st.vy[0], st.vz[0]])
        assert abs(np.linalg.norm(u) / np.linalg.norm(u0) - 1) < 2e-16 * n + 1e-15
        assert abs(u[2] - u0[2]) < 2e-16 * n + 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_relativistic_exb_drift_is_a_fixed_point(dim):
    """E = (0, Ey, 0), B = bz z^: v_d = E x B / B^2 = (Ey / bz, 0, 0) makes
    E + v x B = 0; the particle with u = gamma_d v_d is not accelerated."""
    c, bz, Ey = 2.0, 1.3, 1.9          # v_d = 1.46 = 0.73 c
    s = _s(dim, bz=bz, c=c, dt=0.1)
    vd = Ey / bz
    gd = 1 / np.sqrt(1 - (vd / c) ** 2)
    st = _st(np.array([gd * vd, 0.0, 0.0]))
    Ep = (np.zeros(1), np.array([Ey])) + ((np.zeros(1),) if dim == 3 else ())
    for _ in range(200):
        O.boris(s, st, Ep, s.dt)
    assert abs(st.vx[0] / (gd * vd) - 1) < 1e-13 and abs(st.vy[0]) < 1e-13 * gd * vd
    # Boris does not keep this state once the drift is relativistic (it drifts
    # at E/B in v while its u is that of the drift, so it is accelerated)
    sb = O.Setup(dim, 3, 8, 100.0, 1, 0.1, ny=8, Ly=100.0, nz=8 if dim == 3 else 1, Lz=100.0, bz=bz)
    stb = _st(np.array([gd * vd, 0.0, 0.0]))
    for _ in range(20):
        O.boris(sb, stb, Ep, sb.dt)
    assert abs(stb.vx[0] / (gd * vd) - 1) > 1e-3


def test_field_along_b_changes_only_uz():
    c, Ez, dt = 2.0, 0.4, 0.05
    s = _s(3, bz=2.0, c=c, dt=dt)
    u0 = np.array([0.3, 0.2, -0.5])
    st = _st(u0)
    z = np.zeros(1)
    for n in range(1, 41):
        O.boris(s, st, (z, z, np.array([Ez])), dt)
        assert abs(st.vz[0] - (u0[2] + n * s.qm * Ez * dt)) < 1e-13
        assert abs(np.hypot(st.vx[0], st.vy[0]) / np.hypot(u0[0], u0[1]) - 1) < 1e-14 * n


def test_move_uses_u_over_gamma():
    c = 2.0
    for dim in (2, 3):
        s = _s(dim, bz=0.0, c=c, dt=0.25)
        u = np.array([1.5, -2.0, 0.5])
        st = _st(u)
        x0, y0, z0 = st.x[0], st.y[0], st.z[0]
        O.move(s, st)
        g = np.sqrt(1 + u @ u / c ** 2)
        assert abs(st.x[0] - (x0 + u[0] / g * 0.25)) < 1e-13
        assert abs(st.y[0] - (y0 + u[1] / g * 0.25)) < 1e-13
        if dim == 3:
            assert abs(st.z[0] - (z0 + u[2] / g * 0.25)) < 1e-13
        else:
            assert st.z[0] == z0


def test_relativistic_kinetic_energy():
    c = 1.7
    s = _s(2, c=c, n=3)
    u = np.array([[1.0, 0.0, 0.0], [0.3, -2.0, 0.4], [0.0, 0.0, 5.0]])
    st = _st(u, 3)
    g = np.sqrt(1 + np.sum(u * u, axis=1) / c ** 2)
    assert abs(O.kinetic_sum(s, st) / np.sum(2 * (g - 1) * c ** 2) - 1) < 1e-13


def test_mixed_hc_tracks_fp64_hc():
    """The binary32 Higuera-Cary push agrees with the FP64 one to binary32
    precision, in 2D3V and 3D3V, with a mildly relativistic plasma."""
    rng = np.random.default_rng(22)
    for dim in (2, 3):
        w = (W.thermal_3d(seed=23, nx=8, ppc=16) if dim == 3
             else dataclasses.replace(W.magnetized_2d3v(seed=23, nx=16, ppc=16), mode=(1, 0)))
        if dim == 3:
            x, y, z, vx, vy, vz = W.sample3(w)
        else:
            (x, y, vx, vy, vz), z = W.sample(w), None
        n = len(x)
        s = O.Setup(dim, 3, w.nx, w.Lx, n, w.dt, ny=w.ny, Ly=w.Ly, nz=w.nz, Lz=w.Lz, bz=1.5, pusher="hc", c=4.0)
        E = tuple(rng.normal(size=s.grid_shape) for _ in range(dim))
        st = O.State.from_arrays(x, vx, y, vy, vz, z)
        O.boris(s, st, O.gather(s, st, E), s.dt)
        O.move(s, st)
        c_ = [W.to_cell_offset(a, d, m) for a, d, m in ((x, s.dx, s.nx), (y, s.dy, s.ny))]
        ms = {"ix": c_[0][0], "ox": c_[0][1], "iy": c_[1][0], "oy": c_[1][1],
              "vx": vx.astype(np.float32), "vy": vy.astype(np.float32), "vz": vz.astype(np.float32)}
        if dim == 3:
            iz, oz = W.to_cell_offset(z, s.dz, s.nz)
            ms.update(iz=iz, oz=oz)
        out = OM.push(ms, tuple(e.astype(np.float32) for e in E), dim=dim, vdim=3, nx=s.nx, ny=s.ny, dx=s.dx,
                      dy=s.dy, qm=s.qm, dt=s.dt, bz=s.bz, nz=s.nz, dz=s.dz, pusher="hc", c=s.c)
        for k, ref in (("vx", st.vx), ("vy", st.vy), ("vz", st.vz)):
            assert np.max(np.abs(out[k] - ref)) < 3e-5, (dim, k)
        pos = OM.positions(out, s.dx, s.dy, dim, s.dz)
        for p_, ref, L in zip(pos, (st.x, st.y, st.z), (s.Lx, s.Ly, s.Lz)):
            d = np.abs(p_ - ref)
            assert np.max(np.minimum(d, L - d)) < 3e-5


# ---------------------------------------------------------------------------
# The oracle's reference gradient through the Higuera-Cary advance
# ---------------------------------------------------------------------------

from oracle import adjoint as A   # noqa: E402


@pytest.mark.parametrize("c", [0.7, 2.0, 50.0])
def test_hc_adjoint_matches_central_differences_of_the_advance(c):
    """lam^T J of one advance (in u_old and in E_p, full and backward half
    step) against central differences of the forward advance itself."""
    rng = np.random.default_rng(31)
    n = 64
    for dim, dt in ((2, 0.1), (2, -0.05), (3, 0.1)):
        s = _s(dim, bz=1.9, c=c, dt=abs(dt), n=n)
        u0 = [rng.normal(size=n) * 1.5 for _ in range(3)]
        Ep = [rng.normal(size=n) for _ in range(dim)]
        lam = [rng.normal(size=n) for _ in range(3)]

        def f(uu, ee):
            st = _st(np.stack(uu, axis=1), n)
            O.boris(s, st, tuple(ee), dt)
            return st.vx * lam[0] + st.vy * lam[1] + st.vz * lam[2]

        lv = [l.copy() for l in lam]
        lE = A.adj_hc(s, u0, Ep, lv, dt)
        h = 1e-6
        for k in range(3):
            up = [a.copy() for a in u0]
            um = [a.copy() for a in u0]
            up[k] += h
            um[k] -= h
            fd = (f(up, Ep) - f(um, Ep)) / (2 * h)
            assert np.max(np.abs(fd - lv[k])) < 1e-8 * (1 + np.max(np.abs(fd))), (dim, dt, k)
        for k in range(dim):
            ep = [a.copy() for a in Ep]
            em = [a.copy() for a in Ep]
            ep[k] += h
            em[k] -= h
            fd = (f(u0, ep) - f(u0, em)) / (2 * h)
            assert np.max(np.abs(fd - lE[k])) < 1e-8 * (1 + np.max(np.abs(fd))), (dim, dt, "E", k)


def test_hc_adjoint_reduces_to_boris_at_large_c():
    rng = np.random.default_rng(32)
    n = 40
    sh = _s(2, bz=1.3, c=1e30, n=n)
    sb = O.Setup(2, 3, 8, 100.0, n, 0.05, ny=8, Ly=100.0, bz=1.3)
    u0 = [rng.normal(size=n) for _ in range(3)]
    Ep = [rng.normal(size=n) for _ in range(2)]
    lam = [rng.normal(size=n) for _ in range(3)]
    lh = [l.copy() for l in lam]
    lb = [l.copy() for l in lam]
    eh = A.adj_hc(sh, u0, Ep, lh, sh.dt)
    eb = A.adj_boris(sb, lb, sb.dt)
    for a, b in zip(lh + eh, lb + eb):
        assert np.max(np.abs(a - b)) < 1e-13


def test_move_u_adjoint_matches_central_differences():
    rng = np.random.default_rng(33)
    n = 50
    for dim in (2, 3):
        s = _s(dim, bz=0.0, c=1.3, dt=0.2, n=n)
        u = [rng.normal(size=n) * 2 for _ in range(3)]
        lx = [rng.normal(size=n) for _ in range(dim)]
        lv = [np.zeros(n) for _ in range(3)]
        A.adj_move_u(s, u, lx, lv)

        def f(uu):
            st = _st(np.stack(uu, axis=1), n)
            O.move(s, st)
            out = (st.x - 50.0) * lx[0] + (st.y - 50.0) * lx[1]
            return out + ((st.z - 50.0) * lx[2] if dim == 3 else 0.0)

        h = 1e-6
        for k in range(3):
            up = [a.copy() for a in u]
            um = [a.copy() for a in u]
            up[k] += h
            um[k] -= h
            fd = (f(up) - f(um)) / (2 * h)
            # positions near 50 carry rounding of 1e-14, i.e. 1e-8 after the 2h division
            assert np.max(np.abs(fd - lv[k])) < 1e-7, (dim, k)


def _hc_plasma(c=2.5, nx=16, ppc=16):
    w = dataclasses.replace(W.magnetized_2d3v(nx=nx, ppc=ppc), mode=(1, 0))
    x, y, vx, vy, vz = W.sample(w)
    s = O.Setup(2, 3, w.nx, w.Lx, len(x), w.dt, ny=w.ny, Ly=w.Ly, bz=w.bz, pusher="hc", c=c)
    return w, s, (x, y, vx, vy, vz)


def test_hc_adjoint_matches_independent_torch_autograd():
    torch = pytest.importorskip("torch")
    from tests.torch_pic import Plasma
    w, s, (x, y, vx, vy, vz) = _hc_plasma()
    nsteps = 20
    Wo, lx, lv = A.adjoint(s, O.State.from_arrays(x, vx, y, vy, vz), nsteps)
    P = Plasma(2, 3, w.nx, w.Lx, len(x), w.dt, ny=w.ny, Ly=w.Ly, bz=w.bz, pusher="hc", c=s.c)
    tx = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    ty = torch.tensor(y, dtype=torch.float64, requires_grad=True)
    tv = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in (vx, vy, vz)]
    Wt = P.run(tx, ty, tv, nsteps)
    grads = torch.autograd.grad(Wt, [tx, ty] + tv)
    assert abs(Wt.item() / Wo - 1.0) < 1e-11
    for a, b in zip(lx + lv, grads):
        b = b.numpy()
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-9
    # u_z now reaches the field (gamma couples it to the in-plane motion)
    assert np.linalg.norm(lv[2]) > 1e-3 * np.linalg.norm(lv[0])


def test_hc_adjoint_matches_central_differences_in_single_velocities():
    w, s, (x, y, vx, vy, vz) = _hc_plasma(c=2.0, nx=8, ppc=16)
    nsteps = 12
    _, lx, lv = A.adjoint(s, O.State.from_arrays(x, vx, y, vy, vz), nsteps)
    for p in (3, 400, 1000):
        for k in range(3):
            def Wv(dv):
                st = O.State.from_arrays(x, vx, y, vy, vz)
                (st.vx, st.vy, st.vz)[k][p] += dv
                return A.forward_trajectory(s, st, nsteps)[0]
            fd = (Wv(1e-5) - Wv(-1e-5)) / 2e-5
            assert abs(fd - lv[k][p]) <= 2e-5 * abs(lv[k][p]) + 1e-12 * abs(lv[0]).max(), (p, k, fd, lv[k][p])
