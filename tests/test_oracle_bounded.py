"""Pins of the oracle's cycle between grounded, absorbing walls (2D, walls
at x = 0 and x = Lx, periodic in y), each against something other than the
oracle itself:

  * the sine-transform solve equals a dense solve of the Dirichlet FD system;
  * a charge sheet between grounded plates has the piecewise-linear potential
    of the discrete Green's function, j (nx - k) dx / nx on its left;
  * the wall fields carry the enclosed charge: sum of interior rho dx over
    the box equals the sum over y of (E at the right wall - E at the left wall);
  * absorption: particles leaving through either wall are removed and
    counted, the others move by v dt; the deposit of the live particles
    carries exactly Q N_live.
"""
import numpy as np
import pytest

from oracle import bounded as B


def _box(nx=7, ny=5, Lx=7 * 0.6, Ly=5 * 0.9, n=1000, dt=0.1, **kw):
    return B.Box(nx, Lx, ny, Ly, n, dt, **kw)


def _dense_dirichlet(b, rho):
    nx, ny = b.nx, b.ny
    m = nx - 1
    idx = lambda i, j: j * m + (i - 1)
    A = np.zeros((m * ny, m * ny))
    for j in range(ny):
        for i in range(1, nx):
            r = idx(i, j)
            A[r, r] = 2 / b.dx ** 2 + 2 / b.dy ** 2
            if i > 1:
                A[r, idx(i - 1, j)] -= 1 / b.dx ** 2
            if i < nx - 1:
                A[r, idx(i + 1, j)] -= 1 / b.dx ** 2
            A[r, idx(i, (j + 1) % ny)] -= 1 / b.dy ** 2
            A[r, idx(i, (j - 1) % ny)] -= 1 / b.dy ** 2
    sol = np.linalg.solve(A, rho[:, 1:nx].ravel())
    phi = np.zeros((ny, nx + 1))
    phi[:, 1:nx] = sol.reshape(ny, m)
    return phi


@pytest.mark.parametrize("nx,ny", [(7, 5), (8, 6), (2, 3)])
def test_sine_transform_solve_equals_dense_solve(nx, ny):
    rng = np.random.default_rng(81)
    b = _box(nx=nx, ny=ny, Lx=nx * 0.6, Ly=ny * 0.9)
    rho = rng.normal(size=(ny, nx + 1))
    phi = B.solve_potential(b, rho)
    ref = _dense_dirichlet(b, rho)
    assert np.max(np.abs(phi - ref)) < 1e-12 * np.max(np.abs(ref))
    assert np.all(phi[:, 0] == 0) and np.all(phi[:, -1] == 0)


def test_charge_sheet_between_grounded_plates():
    b = _box(nx=12, ny=4, Lx=12 * 0.5, Ly=4.0)
    for k in (1, 5, 11):
        rho = np.zeros((b.ny, b.nx + 1))
        rho[:, k] = 1.0 / b.dx
        phi = B.solve_potential(b, rho)
        i = np.arange(b.nx + 1)
        ref = np.where(i <= k, b.dx * i * (b.nx - k) / b.nx, b.dx * k * (b.nx - i) / b.nx)
        assert np.max(np.abs(phi - ref[None, :])) < 1e-13
        Ex, Ey = B.field(b, phi)
        assert np.allclose(Ex[:, 0], -(b.nx - k) / b.nx, atol=1e-13, rtol=0)
        assert np.allclose(Ex[:, -1], k / b.nx, atol=1e-13, rtol=0)
        assert np.max(np.abs(Ey)) < 1e-13


def test_wall_fields_carry_the_enclosed_charge():
    rng = np.random.default_rng(82)
    b = _box(nx=10, ny=6)
    rho = rng.normal(size=(b.ny, b.nx + 1))
    Ex, _ = B.solve_field(b, rho)
    inside = float(np.sum(rho[:, 1:b.nx])) * b.dx
    walls = float(np.sum(Ex[:, -1] - Ex[:, 0]))
    assert abs(inside - walls) < 1e-12 * np.sum(np.abs(rho)) * b.dx


def test_absorption_and_charge_bookkeeping():
    rng = np.random.default_rng(83)
    n = 4000
    b = _box(nx=16, ny=8, Lx=16.0, Ly=8.0, n=n, dt=0.2, qm=-1e-12)
    x = rng.uniform(0, b.Lx, n)
    y = rng.uniform(0, b.Ly, n)
    vx = rng.normal(size=n) * 2
    vy = rng.normal(size=n)
    p = B.Plasma(x.copy(), y.copy(), [vx.copy(), vy.copy()])
    E = B.solve_field(b, B.deposit(b, p.x, p.y))
    p0 = p.copy()
    E, rho, _ = B.step(b, p, E)
    x1 = x + vx * b.dt                 # the field is negligible at this q/m
    left, right = x1 < 0, x1 >= b.Lx
    assert p.lost_left == left.sum() > 0 and p.lost_right == right.sum() > 0
    keep = ~(left | right)
    assert np.max(np.abs(p.x - x1[keep])) < 1e-12
    assert np.all((p.x >= 0) & (p.x < b.Lx))
    assert len(p.x) + p.lost_left + p.lost_right == n
    # the deposit of the live particles carries exactly Q N_live
    assert abs(float(np.sum(rho - b.n0)) * b.dV - b.Q * len(p.x)) < 1e-10 * abs(b.Q) * n
    assert p0.lost_left == 0


def test_thermal_plasma_between_walls_loses_charge_only_through_them():
    rng = np.random.default_rng(84)
    n = 8192
    b = _box(nx=32, ny=8, Lx=32.0, Ly=8.0, n=n, dt=0.1)
    p = B.Plasma(rng.uniform(0, b.Lx, n), rng.uniform(0, b.Ly, n), [rng.normal(size=n), rng.normal(size=n)])
    E = B.initialise(b, p)
    for _ in range(40):
        E, rho, _ = B.step(b, p, E)
    assert len(p.x) + p.lost_left + p.lost_right == n
    assert p.lost_left > 0 and p.lost_right > 0
    # electrons leave faster than the (immobile) ions: the plasma charges up
    # positively and the potential peaks inside (a sheath forms at each wall)
    phi = B.solve_potential(b, rho)
    assert phi[:, b.nx // 2].mean() > 0
    assert np.all(phi[:, 0] == 0) and np.all(phi[:, -1] == 0)
