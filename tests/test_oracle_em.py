"""Pins of the electromagnetic step of the oracle (2D3V, periodic Yee grid),
each against something other than the oracle itself:

  * the current deposit satisfies the discrete continuity equation with the
    CIC charge deposit of the electrostatic oracle, for displacements that
    cross cells; closed forms for a particle moving along x inside its cell
    and for a particle at rest with v_z; the total-current sum rule
    sum J dV = q (displacement) / dt;
  * the staggered gather reproduces linear fields given on each component's
    own staggered lattice (pins the half-cell offsets);
  * Boris in a general B: the z-only electrostatic Boris when B = bz z, |v|
    kept in any pure B, the E x B drift as an exact fixed point, E parallel to
    B accelerating only along B;
  * the field update advances discrete plane waves (both polarisations,
    oblique k) exactly along the Yee dispersion relation;
  * the whole cycle keeps the discrete Gauss law div E = rho and div B = 0.
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
from oracle import em as M
from paper_2608_15249_amd import workloads as W


def _s(nx=13, ny=9, Lx=13 * 0.7, Ly=9 * 1.1, n=1, dt=0.1, c=5.0, bz=0.0):
    return O.Setup(2, 3, nx, Lx, n, dt, ny=ny, Ly=Ly, bz=bz, c=c)


def _div_j(s, J):
    return (J[0] - np.roll(J[0], 1, axis=1)) / s.dx + (J[1] - np.roll(J[1], 1, axis=0)) / s.dy


def test_current_satisfies_discrete_continuity():
    rng = np.random.default_rng(61)
    n = 2000
    s = _s(n=n)
    x0 = rng.uniform(0, s.Lx, n)
    y0 = rng.uniform(0, s.Ly, n)
    ddx = rng.uniform(-0.95, 0.95, n) * s.dx
    ddy = rng.uniform(-0.95, 0.95, n) * s.dy
    vz = rng.normal(size=n)
    J = M.current(s, x0, y0, ddx, ddy, vz)
    r0 = O.deposit(s, O.State.from_arrays(x0, np.zeros(n), y0, np.zeros(n)))
    x1 = np.mod(x0 + ddx, s.Lx)
    y1 = np.mod(y0 + ddy, s.Ly)
    r1 = O.deposit(s, O.State.from_arrays(x1, np.zeros(n), y1, np.zeros(n)))
    res = (r1 - r0) / s.dt + _div_j(s, J)
    assert np.max(np.abs(res)) < 1e-12 * np.max(np.abs(r1 - r0)) / s.dt


def test_current_closed_forms():
    s = _s(n=1)
    q = s.Q
    dV = s.dx * s.dy
    # along x inside the cell (i, j) = (4, 3): Jx = q vx W_y / dV on the two rows
    fx, fy, d = 0.2, 0.35, 0.5
    x0 = np.array([(4 + fx) * s.dx])
    y0 = np.array([(3 + fy) * s.dy])
    vx = d * s.dx / s.dt
    J = M.current(s, x0, y0, np.array([d * s.dx]), np.zeros(1), np.zeros(1))
    ref = np.zeros((3, s.ny, s.nx))
    ref[0, 3, 4] = q * vx * (1 - fy) / dV
    ref[0, 4, 4] = q * vx * fy / dV
    assert np.max(np.abs(J - ref)) < 1e-13 * abs(ref).max()
    # at rest with v_z: Jz = q vz W / dV (the CIC charge weights)
    vz = 1.7
    J = M.current(s, x0, y0, np.zeros(1), np.zeros(1), np.array([vz]))
    ref = np.zeros((3, s.ny, s.nx))
    for (j, i, w) in ((3, 4, (1 - fx) * (1 - fy)), (3, 5, fx * (1 - fy)), (4, 4, (1 - fx) * fy), (4, 5, fx * fy)):
        ref[2, j, i] = q * vz * w / dV
    assert np.max(np.abs(J - ref)) < 1e-13 * abs(ref).max()


def test_total_current_sum_rule():
    """sum_j J_j dV = q (displacement) / dt per particle, for any displacement
    within a cell (including crossings and the periodic seam)."""
    rng = np.random.default_rng(62)
    s = _s(n=1)
    for _ in range(200):
        x0 = rng.uniform(0, s.Lx, 1)
        y0 = rng.uniform(0, s.Ly, 1)
        ddx = rng.uniform(-0.99, 0.99, 1) * s.dx
        ddy = rng.uniform(-0.99, 0.99, 1) * s.dy
        vz = rng.normal(size=1)
        J = M.current(s, x0, y0, ddx, ddy, vz)
        dV = s.dx * s.dy
        tot = J.reshape(3, -1).sum(axis=1) * dV
        ref = s.Q * np.array([ddx[0] / s.dt, ddy[0] / s.dt, vz[0]])
        assert np.max(np.abs(tot - ref)) < 1e-13 * (1 + np.max(np.abs(ref)))


def test_current_rejects_moves_of_a_cell():
    s = _s(n=1)
    with pytest.raises(ValueError):
        M.current(s, np.array([1.0]), np.array([1.0]), np.array([1.0 * s.dx]), np.zeros(1), np.zeros(1))


def test_staggered_gather_reproduces_linear_fields():
    rng = np.random.default_rng(63)
    n = 500
    s = _s(n=n, nx=16, ny=12, Lx=16 * 0.8, Ly=12 * 1.3)
    offs = [(0.5, 0.0), (0.0, 0.5), (0.0, 0.0), (0.0, 0.5), (0.5, 0.0), (0.5, 0.5)]
    a = rng.normal(size=6)
    b = rng.normal(size=6)
    F = np.zeros((6, s.ny, s.nx))
    i = np.arange(s.nx)[None, :]
    j = np.arange(s.ny)[:, None]
    for c, (ox, oy) in enumerate(offs):
        F[c] = a[c] * (i + ox) * s.dx + b[c] * (j + oy) * s.dy
    # away from the periodic seam, where the linear field wraps
    x = rng.uniform(2 * s.dx, s.Lx - 3 * s.dx, n)
    y = rng.uniform(2 * s.dy, s.Ly - 3 * s.dy, n)
    Ep, Bp = M.gather(s, O.State.from_arrays(x, np.zeros(n), y, np.zeros(n), np.zeros(n)), F)
    got = np.concatenate([Ep, Bp])
    for c in range(6):
        assert np.max(np.abs(got[c] - (a[c] * x + b[c] * y))) < 1e-12, c


def _st(v, n):
    v = np.atleast_2d(v)
    return O.State.from_arrays(np.full(n, 1.0), v[:, 0].copy(), np.full(n, 1.0), v[:, 1].copy(), v[:, 2].copy())


def test_boris3_with_b_along_z_is_the_electrostatic_boris():
    rng = np.random.default_rng(64)
    n = 300
    s = _s(n=n, bz=1.7)
    v = rng.normal(size=(n, 3))
    Exy = rng.normal(size=(2, n))
    a = _st(v, n)
    b = _st(v, n)
    for _ in range(5):
        M.boris(s, a, np.vstack([Exy, np.zeros(n)]), np.vstack([np.zeros((2, n)), np.full(n, s.bz)]), s.dt)
        O.boris(s, b, (Exy[0], Exy[1]), s.dt)
    for u, w in ((a.vx, b.vx), (a.vy, b.vy), (a.vz, b.vz)):
        assert np.max(np.abs(u - w)) < 1e-13


def test_boris3_general_b():
    rng = np.random.default_rng(65)
    n = 100
    s = _s(n=n)
    B = rng.normal(size=(3, n)) * 2
    v = rng.normal(size=(n, 3))
    st = _st(v, n)
    for k in range(1, 101):
        M.boris(s, st, np.zeros((3, n)), B, s.dt)
    sp = np.sqrt(st.vx ** 2 + st.vy ** 2 + st.vz ** 2)
    assert np.max(np.abs(sp / np.linalg.norm(v, axis=1) - 1)) < 1e-13
    # E x B drift: E perpendicular to B, v = E x B / |B|^2 is not accelerated
    E = rng.normal(size=(3, n))
    E -= B * (np.sum(E * B, axis=0) / np.sum(B * B, axis=0))
    vd = np.cross(E.T, B.T) / np.sum(B * B, axis=0)[:, None]
    st = _st(vd, n)
    for _ in range(50):
        M.boris(s, st, E, B, s.dt)
    got = np.stack([st.vx, st.vy, st.vz], axis=1)
    assert np.max(np.abs(got - vd)) < 1e-12 * (1 + np.abs(vd).max())
    # E parallel to B: the parallel velocity gains (q/m) |E| dt per step, |v_perp| kept
    bh = B / np.linalg.norm(B, axis=0)
    E = 0.3 * bh
    st = _st(v, n)
    for _ in range(20):
        M.boris(s, st, E, B, s.dt)
    got = np.stack([st.vx, st.vy, st.vz], axis=1)
    par0 = np.sum(v * bh.T, axis=1)
    par = np.sum(got * bh.T, axis=1)
    assert np.max(np.abs(par - (par0 + 20 * s.qm * 0.3 * s.dt))) < 1e-12
    perp0 = np.linalg.norm(v - par0[:, None] * bh.T, axis=1)
    perp = np.linalg.norm(got - par[:, None] * bh.T, axis=1)
    assert np.max(np.abs(perp - perp0)) < 1e-12


@pytest.mark.parametrize("pol", ["TM", "TE"])
def test_field_update_follows_the_yee_dispersion_relation(pol):
    """A discrete plane wave of wavevector (3, 2) on a 24 x 16 grid with the
    frequency from sin^2(w dt/2) / (c dt/2)^2 = kappa_x^2 + kappa_y^2,
    kappa = 2 sin(k d / 2) / d, is advanced exactly by the Yee update."""
    nx, ny = 24, 16
    s = O.Setup(2, 3, nx, nx * 1.0, 1, 0.5, ny=ny, Ly=ny * 1.25, c=1.0)
    kx, ky = 2 * np.pi * 3 / s.Lx, 2 * np.pi * 2 / s.Ly
    kapx, kapy = 2 * np.sin(kx * s.dx / 2) / s.dx, 2 * np.sin(ky * s.dy / 2) / s.dy
    w = 2 / s.dt * np.arcsin(0.5 * s.c * s.dt * np.hypot(kapx, kapy))
    Om = 2 * np.sin(w * s.dt / 2) / s.dt
    i = np.arange(nx)[None, :] * 1.0
    j = np.arange(ny)[:, None] * 1.0
    c2 = s.c * s.c

    def wave(t, ox, oy, amp):
        return amp * np.cos(kx * (i + ox) * s.dx + ky * (j + oy) * s.dy - w * t)

    def exact(n_e, n_b):
        F = np.zeros((6, ny, nx))
        if pol == "TM":
            F[2] = wave(n_e * s.dt, 0, 0, 1.0)
            F[3] = wave(n_b * s.dt, 0, 0.5, kapy / Om)
            F[4] = wave(n_b * s.dt, 0.5, 0, -kapx / Om)
        else:
            F[5] = wave(n_b * s.dt, 0.5, 0.5, 1.0)
            F[0] = wave(n_e * s.dt, 0.5, 0, -c2 * kapy / Om)
            F[1] = wave(n_e * s.dt, 0, 0.5, c2 * kapx / Om)
        return F

    F = exact(0, 0.5)
    # B held at integer time: B^0 = B^{1/2} + dt/2 curl E^0
    M.advance_b(s, F, -0.5 * s.dt)
    J = np.zeros((3, ny, nx))
    N = 60
    for _ in range(N):
        M.maxwell(s, F, J)
    ref = exact(N, N + 0.5)
    assert np.max(np.abs(F[:3] - ref[:3])) < 1e-11
    M.advance_b(s, F, 0.5 * s.dt)
    assert np.max(np.abs(F[3:] - ref[3:])) < 1e-11


def test_cycle_keeps_gauss_law_and_div_b():
    w = dataclasses.replace(W.magnetized_2d3v(seed=66, nx=16, ppc=16), mode=(1, 0))
    x, y, vx, vy, vz = W.sample(w)
    n = len(x)
    s = O.Setup(2, 3, w.nx, w.Lx, n, 0.1, ny=w.ny, Ly=w.Ly, bz=w.bz, c=5.0)
    st = O.State.from_arrays(x, vx, y, vy, vz)
    F = M.initialise(s, st)
    scale = np.max(np.abs(O.deposit(s, st)))
    assert np.max(np.abs(M.divergence_e(s, F) - O.deposit(s, st))) < 1e-12 * scale
    for _ in range(20):
        M.step(s, st, F)
    assert np.max(np.abs(M.divergence_e(s, F) - O.deposit(s, st))) < 1e-11 * scale
    assert np.max(np.abs(M.divergence_b(s, F))) < 1e-11 * (1 + np.max(np.abs(F[3:])))
    # the fields did evolve (the check above is not vacuous)
    assert np.max(np.abs(F[3:5])) > 1e-6


def _cold_lattice(nx, ny, Lx, Ly, per):
    """Electrons on a regular lattice (per x per in every cell), at rest."""
    gx = (np.arange(nx * per) + 0.5) * (Lx / (nx * per))
    gy = (np.arange(ny * per) + 0.5) * (Ly / (ny * per))
    X, Y = np.meshgrid(gx, gy)
    return X.ravel(), Y.ravel()


def _frequency(t, a):
    """Angular frequency of a ~cos(w t) record from its zero crossings."""
    s = np.sign(a)
    idx = np.where(s[:-1] * s[1:] < 0)[0]
    tz = t[idx] - a[idx] * (t[idx + 1] - t[idx]) / (a[idx + 1] - a[idx])
    return np.pi / np.mean(np.diff(tz))


def test_cold_plasma_transverse_wave_frequency():
    """A transverse standing wave E_z = E0 cos(k x) in a cold uniform plasma
    oscillates at w^2 = w_p^2 + c^2 k^2 (w_p = 1): the plasma's current and the
    curl terms of the update together."""
    nx, ny, Lx, c = 64, 2, 20.0, 5.0
    Ly = 2 * Lx / nx
    x, y = _cold_lattice(nx, ny, Lx, Ly, 8)
    n = len(x)
    s = O.Setup(2, 3, nx, Lx, n, 0.03, ny=ny, Ly=Ly, c=c)
    st = O.State.from_arrays(x, np.zeros(n), y, np.zeros(n), np.zeros(n))
    F = M.initialise(s, st)
    k = 2 * np.pi / Lx
    xi = np.arange(nx) * s.dx
    F[2] += 1e-3 * np.cos(k * xi)[None, :]
    ts, amp = [], []
    for step in range(300):
        M.step(s, st, F)
        ts.append((step + 1) * s.dt)
        amp.append(np.mean(F[2] * np.cos(k * xi)[None, :]))
    w = _frequency(np.array(ts), np.array(amp))
    assert abs(w / np.sqrt(1 + (c * k) ** 2) - 1) < 0.01, w


def test_cold_plasma_langmuir_oscillation():
    """A longitudinal displacement of a cold lattice plasma oscillates at the
    plasma frequency (w_p = 1) in the electromagnetic step too, with no
    magnetic field generated."""
    nx, ny, Lx, c = 32, 2, 16.0, 5.0
    Ly = 2 * Lx / nx
    x, y = _cold_lattice(nx, ny, Lx, Ly, 8)
    n = len(x)
    k = 2 * np.pi / Lx
    x = np.mod(x + 1e-3 / k * np.sin(k * x), Lx)
    s = O.Setup(2, 3, nx, Lx, n, 0.05, ny=ny, Ly=Ly, c=c)
    st = O.State.from_arrays(x, np.zeros(n), y, np.zeros(n), np.zeros(n))
    F = M.initialise(s, st)
    xi = (np.arange(nx) + 0.5) * s.dx
    ts, amp = [], []
    for step in range(300):
        M.step(s, st, F)
        ts.append((step + 1) * s.dt)
        amp.append(np.mean(F[0] * np.sin(k * xi)[None, :]))
    w = _frequency(np.array(ts), np.array(amp))
    assert abs(w - 1.0) < 0.01, w
    assert np.max(np.abs(F[3:])) < 1e-12


# ---------------------------------------------------------------------------
# Higuera-Cary in the electromagnetic step (general field, state u = gamma v)
# ---------------------------------------------------------------------------

def _hc_setup(n, c=2.0, dt=0.1, bz=0.0):
    return O.Setup(2, 3, 8, 8.0, n, dt, ny=8, Ly=8.0, bz=bz, pusher="hc", c=c)


def test_hc3_with_b_along_z_is_the_electrostatic_higuera_cary():
    rng = np.random.default_rng(111)
    n = 300
    s = _hc_setup(n, bz=1.7)
    u = rng.normal(size=(n, 3)) * 2
    E = rng.normal(size=(3, n))
    a = _st(u, n)
    b = _st(u, n)
    M.boris(s, a, E, np.vstack([np.zeros((2, n)), np.full(n, s.bz)]), s.dt)
    O.boris(s, b, (E[0], E[1], E[2]), s.dt)
    for x, y in ((a.vx, b.vx), (a.vy, b.vy), (a.vz, b.vz)):
        assert np.max(np.abs(x - y)) < 1e-13


def test_hc3_satisfies_the_implicit_midpoint_relation_in_a_general_field():
    """u1 - u0 = 2 a E + (u0 + u1) x (a B / gamma(ubar)), ubar = (u0 + u1)/2."""
    rng = np.random.default_rng(112)
    n = 400
    for c in (0.8, 2.0, 9.0):
        s = _hc_setup(n, c=c)
        a = s.qm * s.dt / 2
        u0 = rng.normal(size=(n, 3)) * 2
        E = rng.normal(size=(3, n))
        B = rng.normal(size=(3, n)) * 2
        st = _st(u0, n)
        M.boris(s, st, E, B, s.dt)
        u1 = np.stack([st.vx, st.vy, st.vz], axis=1)
        ub = 0.5 * (u0 + u1)
        gb = np.sqrt(1 + np.sum(ub * ub, axis=1) / c ** 2)
        r = u1 - u0 - 2 * a * E.T - np.cross(u0 + u1, (a * B / gb).T)
        assert np.max(np.abs(r)) < 1e-13 * (1 + np.abs(u1).max()), c


def test_hc3_limits_and_exb_drift():
    rng = np.random.default_rng(113)
    n = 200
    E = rng.normal(size=(3, n))
    B = rng.normal(size=(3, n)) * 2
    u = rng.normal(size=(n, 3))
    # c -> infinity: the general-field Boris advance
    sh = _hc_setup(n, c=1e30)
    sb = O.Setup(2, 3, 8, 8.0, n, 0.1, ny=8, Ly=8.0, c=5.0)
    a, b = _st(u, n), _st(u, n)
    for _ in range(5):
        M.boris(sh, a, E, B, sh.dt)
        M.boris(sb, b, E, B, sb.dt)
    for x, y in ((a.vx, b.vx), (a.vy, b.vy), (a.vz, b.vz)):
        assert np.max(np.abs(x - y)) < 1e-12
    # E perpendicular to B with |E x B| / B^2 < c: u = gamma_d v_d is a fixed point
    c = 3.0
    s = _hc_setup(n, c=c)
    E = E - B * (np.sum(E * B, axis=0) / np.sum(B * B, axis=0))
    E *= 0.5 * c * np.linalg.norm(B, axis=0) / np.linalg.norm(E, axis=0)       # |v_d| = c / 2
    vd = np.cross(E.T, B.T) / np.sum(B * B, axis=0)[:, None]
    ud = vd / np.sqrt(1 - np.sum(vd * vd, axis=1) / c ** 2)[:, None]
    st = _st(ud, n)
    for _ in range(50):
        M.boris(s, st, E, B, s.dt)
    got = np.stack([st.vx, st.vy, st.vz], axis=1)
    assert np.max(np.abs(got - ud)) < 1e-12 * (1 + np.abs(ud).max())


def test_hc_cycle_keeps_gauss_law():
    """The current of the move by u / gamma keeps div E = rho over 20 steps of a
    mildly relativistic magnetized plasma."""
    w = dataclasses.replace(W.magnetized_2d3v(seed=114, nx=16, ppc=16), mode=(1, 0))
    x, y, vx, vy, vz = W.sample(w)
    n = len(x)
    s = O.Setup(2, 3, w.nx, w.Lx, n, 0.1, ny=w.ny, Ly=w.Ly, bz=w.bz, c=5.0, pusher="hc")
    st = O.State.from_arrays(x, 1.5 * vx, y, 1.5 * vy, 1.5 * vz)
    F = M.initialise(s, st)
    scale = np.max(np.abs(O.deposit(s, st)))
    for _ in range(20):
        M.step(s, st, F)
    assert np.max(np.abs(M.divergence_e(s, F) - O.deposit(s, st))) < 1e-11 * scale
    assert np.max(np.abs(M.divergence_b(s, F))) < 1e-11 * (1 + np.max(np.abs(F[3:])))
