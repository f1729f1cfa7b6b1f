"""Pins of the oracle's reference gradient in 3D (the Cartesian three-
dimensional cycle: trilinear weights, the 7-point solve, E_z kicks), each
against something other than the adjoint itself: dot-product identities of
the linear operators with the forward code, central differences of the
forward deposit, gather and Higuera-Cary advance, and central differences of
whole forward runs (Boris and Higuera-Cary) in single velocities, where the
run is smooth, and in the seeded amplitude, where the differences converge
as the step shrinks."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from oracle import adjoint as A
from paper_2608_15249_amd import workloads as W


def _s3(nx=6, ny=5, nz=4, L=(6.0, 5.5, 4.4), n=200, dt=0.1, bz=0.0, pusher="boris", c=float("inf")):
    return O.Setup(3, 3, nx, L[0], n, dt, ny=ny, Ly=L[1], nz=nz, Lz=L[2], bz=bz, pusher=pusher, c=c)


def test_field_adjoint_dot_product_3d():
    rng = np.random.default_rng(31)
    s = _s3()
    rho = rng.normal(size=s.grid_shape)
    lam = [rng.normal(size=s.grid_shape) for _ in range(3)]
    E = O.solve_field(s, rho)
    lhs = sum(float(np.sum(e * l)) for e, l in zip(E, lam))
    rhs = float(np.sum(rho * A.solve_field_adjoint(s, lam)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_gather_adjoint_dot_product_3d():
    rng = np.random.default_rng(32)
    s = _s3(n=300)
    x, y, z = (rng.uniform(0, L, s.n_particles) for L in (s.Lx, s.Ly, s.Lz))
    E = tuple(rng.normal(size=s.grid_shape) for _ in range(3))
    lEp = [rng.normal(size=s.n_particles) for _ in range(3)]
    Ep = O.gather(s, O.State(x, np.zeros_like(x), y, None, None, z), E)
    lhs = sum(float(np.dot(a, b)) for a, b in zip(Ep, lEp))
    lE = [np.zeros(s.grid_shape) for _ in range(3)]
    lx = [np.zeros(s.n_particles) for _ in range(3)]
    A.adj_gather(s, (x, y, z), E, lEp, lE, lx)
    rhs = sum(float(np.sum(a * b)) for a, b in zip(E, lE))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("bz", [0.0, 1.7])
def test_boris_adjoint_dot_product_3d(bz):
    """The 3D Boris map is linear in (v, E_p) with E_z kicking v_z twice."""
    rng = np.random.default_rng(33)
    n = 50
    s = _s3(n=n, dt=0.07, bz=bz)
    v = [rng.normal(size=n) for _ in range(3)]
    Ep = [rng.normal(size=n) for _ in range(3)]
    lam = [rng.normal(size=n) for _ in range(3)]
    for dt in (s.dt, -0.5 * s.dt):
        st = O.State(np.zeros(n), v[0].copy(), np.zeros(n), v[1].copy(), v[2].copy(), np.zeros(n))
        O.boris(s, st, tuple(Ep), dt)
        lhs = sum(float(np.dot(a, b)) for a, b in zip((st.vx, st.vy, st.vz), lam))
        lv = [l.copy() for l in lam]
        lEp = A.adj_boris(s, lv, dt)
        assert len(lEp) == 3
        rhs = sum(float(np.dot(a, b)) for a, b in zip(v, lv)) + sum(float(np.dot(a, b)) for a, b in zip(Ep, lEp))
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0), (dt, lhs, rhs)


def test_deposit_and_gather_position_derivatives_3d():
    rng = np.random.default_rng(34)
    n = 30
    s = _s3(n=n)
    pos = [(rng.integers(0, m, n) + rng.uniform(0.15, 0.85, n)) * d
           for m, d in ((s.nx, s.dx), (s.ny, s.dy), (s.nz, s.dz))]
    lrho = rng.normal(size=s.grid_shape)
    E = tuple(rng.normal(size=s.grid_shape) for _ in range(3))
    lEp = [rng.normal(size=n) for _ in range(3)]
    lx_dep = [np.zeros(n) for _ in range(3)]
    A.adj_deposit(s, tuple(pos), lrho, lx_dep)
    lx_gat = [np.zeros(n) for _ in range(3)]
    A.adj_gather(s, tuple(pos), E, lEp, [np.zeros(s.grid_shape) for _ in range(3)], lx_gat)
    h = 1e-6

    def st_of(p):
        return O.State(p[0], np.zeros(n), p[1], None, None, p[2])

    def f_dep(p):
        return float(np.sum(lrho * O.deposit(s, st_of(p))))

    def f_gat(p):
        return sum(float(np.dot(a, b)) for a, b in zip(O.gather(s, st_of(p), E), lEp))

    for q in range(n):
        for ax in range(3):
            for f, lx in ((f_dep, lx_dep), (f_gat, lx_gat)):
                pp = [a.copy() for a in pos]
                pm = [a.copy() for a in pos]
                pp[ax][q] += h
                pm[ax][q] -= h
                fd = (f(pp) - f(pm)) / (2 * h)
                assert abs(fd - lx[ax][q]) <= 1e-6 * max(1.0, abs(fd)), (q, ax, fd, lx[ax][q])


def test_higuera_cary_adjoint_3d_matches_central_differences():
    """One 3D Higuera-Cary advance with E_z: the adjoint's lam_u0 and lam_E
    against central differences of the advance in every input."""
    rng = np.random.default_rng(35)
    n = 20
    s = _s3(n=n, dt=0.1, bz=1.3, pusher="hc", c=2.5)
    u0 = [rng.normal(0, 1.5, n) for _ in range(3)]
    Ep = [rng.normal(size=n) for _ in range(3)]
    lam = [rng.normal(size=n) for _ in range(3)]

    def adv(u, E):
        st = O.State(np.zeros(n), u[0].copy(), np.zeros(n), u[1].copy(), u[2].copy(), np.zeros(n))
        O.boris(s, st, tuple(E), s.dt)
        return sum(float(np.dot(a, b)) for a, b in zip((st.vx, st.vy, st.vz), lam))

    lv = [l.copy() for l in lam]
    lE = A.adj_hc(s, [a.copy() for a in u0], Ep, lv, s.dt)
    h = 1e-6
    for k in range(3):
        for q in (0, 7, 19):
            up = [a.copy() for a in u0]
            um = [a.copy() for a in u0]
            up[k][q] += h
            um[k][q] -= h
            fd = (adv(up, Ep) - adv(um, Ep)) / (2 * h)
            assert abs(fd - lv[k][q]) <= 1e-7 * max(1.0, abs(fd)), ("u", k, q)
            Epp = [a.copy() for a in Ep]
            Epm = [a.copy() for a in Ep]
            Epp[k][q] += h
            Epm[k][q] -= h
            fd = (adv(u0, Epp) - adv(u0, Epm)) / (2 * h)
            assert abs(fd - lE[k][q]) <= 1e-7 * max(1.0, abs(fd)), ("E", k, q)


def _plasma3(pusher, seed=41):
    w = dataclasses.replace(W.thermal_3d(seed=seed, nx=8, ppc=8), mode=(1, 0), delta0=0.05)
    x, y, z, vx, vy, vz = W.sample3(w)
    c = 3.0 if pusher == "hc" else float("inf")
    s = O.Setup(3, 3, w.nx, w.Lx, len(x), w.dt, ny=w.ny, Ly=w.Ly, nz=w.nz, Lz=w.Lz, bz=0.8, pusher=pusher, c=c)
    return w, s, (x, y, z, vx, vy, vz)


@pytest.mark.parametrize("pusher", ["boris", "hc"])
def test_whole_run_velocity_derivatives_3d(pusher):
    """Eight 3D steps: the adjoint's derivative with respect to single
    velocities (all three components, v_z now reaches the field through E_z
    and the z motion) against central differences of the forward run."""
    w, s, (x, y, z, vx, vy, vz) = _plasma3(pusher)
    nsteps = 8
    _, lx, lv = A.adjoint(s, O.State.from_arrays(x, vx, y, vy, vz, z), nsteps)
    for p in (3, 1500, 4000):
        for k, base in enumerate((vx, vy, vz)):
            def Wv(dv):
                vs = [vx.copy(), vy.copy(), vz.copy()]
                vs[k][p] += dv
                return A.forward_trajectory(s, O.State.from_arrays(x, vs[0], y, vs[1], vs[2], z), nsteps)[0]
            fd = (Wv(1e-5) - Wv(-1e-5)) / 2e-5
            assert abs(fd - lv[k][p]) <= 1e-5 * max(abs(lv[k][p]), 1e-3 * np.max(np.abs(lv[k]))), (p, k)


def test_whole_run_delta0_derivative_3d_converges():
    """The seeded amplitude (mode (1, 0, 0)): central differences of the 3D
    forward run approach the adjoint's dW/d delta0 as the step shrinks."""
    w, s, (x, y, z, vx, vy, vz) = _plasma3("boris", seed=42)
    nsteps = 8
    _, lx, _ = A.adjoint(s, O.State.from_arrays(x, vx, y, vy, vz, z), nsteps)
    xu, yu, *_ = W.sample3(dataclasses.replace(w, delta0=0.0))
    dirn = A.delta0_direction(s, xu, yu, w.mode)
    g = A.grad_delta0(lx, dirn)

    def Wof(d0):
        x2, y2, z2, a, b, c = W.sample3(dataclasses.replace(w, delta0=d0))
        return A.forward_trajectory(s, O.State.from_arrays(x2, a, y2, b, c, z2), nsteps)[0]

    errs = []
    for h in (1e-3, 1e-5, 1e-7):
        fd = (Wof(w.delta0 + h) - Wof(w.delta0 - h)) / (2 * h)
        errs.append(abs(fd / g - 1.0))
    assert errs[-1] < 1e-6 and errs[-1] <= errs[0], errs
