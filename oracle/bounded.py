"""Serial FP64 reference for the electrostatic PIC cycle between two grounded
walls: the non-periodic Poisson problem (the paper's D_Poisson solves
Poisson with HYPRE under general boundary conditions) with particles absorbed
at the walls. 2D: walls at x = 0 and x = Lx, periodic in y.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the test-suite, the
smoke check and the CPU-baseline leg of the benchmark use it; the product
never imports it.

Readings (each listed in the design notes of the repository):
  * nodes X_i = i dx, i = 0..nx along x (nx cells; nodes 0 and nx on the
    walls), periodic nodes j = 0..ny-1 along y; grid arrays [ny][nx+1];
  * CIC deposit and gather on these nodes without wrap along x:
    rho_ij = rho_ion + (Q/dV) sum_p W_ij(x_p) at every node (the wall nodes
    included; their value does not enter the solve);
  * grounded walls: phi = 0 on nodes i = 0 and i = nx; on the interior nodes
    the 5-point FD Laplacian -lap(phi) = rho (no mean condition: the Dirichlet
    problem is non-singular). Solved exactly by a type-I discrete sine
    transform along x and an FFT along y: the eigenvalues of the Dirichlet
    3-point operator are (2/dx)^2 sin^2(pi m / (2 nx)), m = 1..nx-1;
  * E = -(centred difference of phi) on interior nodes; on the wall nodes the
    one-sided difference E_0 = -(phi_1 - phi_0)/dx, E_nx = -(phi_nx -
    phi_{nx-1})/dx (the field of the wall's surface charge); E_y centred and
    periodic;
  * absorbing walls: after the move, a particle with x < 0 or x >= Lx is
    removed (its charge leaves the plasma); the kinetic energy of the step
    counts every particle that was pushed;
  * W_E = 1/2 dV sum_ij w_i |E_ij|^2 with w = 1/2 on the wall nodes (their
    cells are half inside the box) and 1 elsewhere.
Written with numpy (np.add.at for the deposit) and scipy.fft's DST-I and
FFT as library primitives.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.fft as sfft


@dataclass
class Box:
    """2D plasma between grounded walls at x = 0 and x = Lx, periodic in y.
    Macro-electron charge Q = -n0 Lx Ly / N0 (N0 the initial count), mass
    -Q (q/m = qm = -1 by default); uniform immobile ions of density n0."""
    nx: int
    Lx: float
    ny: int
    Ly: float
    n0_particles: int
    dt: float
    qm: float = -1.0
    bz: float = 0.0
    n0: float = 1.0
    vdim: int = 2

    @property
    def dx(self):
        return self.Lx / self.nx

    @property
    def dy(self):
        return self.Ly / self.ny

    @property
    def dV(self):
        return self.dx * self.dy

    @property
    def Q(self):
        return -self.n0 * self.Lx * self.Ly / self.n0_particles

    @property
    def M(self):
        return self.Q / self.qm


def _weights(b: Box, x, y):
    gx = x / b.dx
    i = np.floor(gx).astype(np.int64)
    fx = gx - i
    gy = y / b.dy
    j = np.floor(gy).astype(np.int64)
    fy = gy - j
    j = np.mod(j, b.ny)
    return i, fx, j, fy


def deposit(b: Box, x, y) -> np.ndarray:
    """rho [ny][nx+1] of the particles at (x, y), x in [0, Lx)."""
    i, fx, j, fy = _weights(b, x, y)
    jp = np.mod(j + 1, b.ny)
    acc = np.zeros((b.ny, b.nx + 1))
    np.add.at(acc, (j, i), (1 - fx) * (1 - fy))
    np.add.at(acc, (j, i + 1), fx * (1 - fy))
    np.add.at(acc, (jp, i), (1 - fx) * fy)
    np.add.at(acc, (jp, i + 1), fx * fy)
    return b.n0 + b.Q / b.dV * acc


def dirichlet_eigenvalues(b: Box) -> np.ndarray:
    m = np.arange(1, b.nx)
    return (2.0 / b.dx * np.sin(np.pi * m / (2 * b.nx))) ** 2


def solve_potential(b: Box, rho: np.ndarray) -> np.ndarray:
    """phi [ny][nx+1] with phi = 0 on the walls and -lap(phi) = rho inside."""
    ky = 2.0 * np.pi * np.fft.fftfreq(b.ny, d=b.dy)
    K2y = (2.0 / b.dy * np.sin(ky * b.dy / 2)) ** 2
    inner = rho[:, 1:b.nx]
    h = sfft.dst(np.fft.fft(inner, axis=0), type=1, axis=1)
    h = h / (dirichlet_eigenvalues(b)[None, :] + K2y[:, None])
    phi_in = np.real(np.fft.ifft(sfft.idst(h, type=1, axis=1), axis=0))
    phi = np.zeros((b.ny, b.nx + 1))
    phi[:, 1:b.nx] = phi_in
    return phi


def field(b: Box, phi: np.ndarray):
    """(Ex, Ey) [ny][nx+1] from phi (module header)."""
    Ex = np.empty_like(phi)
    Ex[:, 1:-1] = -(phi[:, 2:] - phi[:, :-2]) / (2 * b.dx)
    Ex[:, 0] = -(phi[:, 1] - phi[:, 0]) / b.dx
    Ex[:, -1] = -(phi[:, -1] - phi[:, -2]) / b.dx
    Ey = -(np.roll(phi, -1, axis=0) - np.roll(phi, 1, axis=0)) / (2 * b.dy)
    return Ex, Ey


def solve_field(b: Box, rho: np.ndarray):
    return field(b, solve_potential(b, rho))


def gather(b: Box, x, y, E):
    i, fx, j, fy = _weights(b, x, y)
    jp = np.mod(j + 1, b.ny)
    out = []
    for e in E:
        out.append((1 - fx) * (1 - fy) * e[j, i] + fx * (1 - fy) * e[j, i + 1] + (1 - fx) * fy * e[jp, i]
                   + fx * fy * e[jp, i + 1])
    return tuple(out)


def _setup(b: Box, n: int):
    from . import Setup
    return Setup(2, b.vdim, b.nx, b.Lx, max(n, 1), b.dt, ny=b.ny, Ly=b.Ly, qm=b.qm, bz=b.bz)


def boris(b: Box, v, Ep, dt: float):
    """Boris advance of v (list of vdim arrays) under (Ex, Ey) and uniform bz
    (the electrostatic oracle's advance)."""
    from . import State, boris as boris_es
    n = v[0].shape[0]
    st = State.from_arrays(np.zeros(n), v[0], np.zeros(n), v[1], v[2] if b.vdim == 3 else None)
    boris_es(_setup(b, n), st, Ep, dt)
    return [st.vx, st.vy] + ([st.vz] if b.vdim == 3 else [])


def field_energy(b: Box, E) -> float:
    w = np.ones(b.nx + 1)
    w[0] = w[-1] = 0.5
    return 0.5 * b.dV * float(sum(np.sum(w[None, :] * e * e) for e in E))


@dataclass
class Plasma:
    """Live particles (structure of arrays) and the count absorbed per wall."""
    x: np.ndarray
    y: np.ndarray
    v: list
    lost_left: int = 0
    lost_right: int = 0
    ids: np.ndarray = None      # optional labels carried with the particles

    def copy(self):
        return Plasma(self.x.copy(), self.y.copy(), [a.copy() for a in self.v], self.lost_left, self.lost_right,
                      None if self.ids is None else self.ids.copy())


def initialise(b: Box, p: Plasma):
    """E^0 of the initial charge, then the backward half push."""
    E = solve_field(b, deposit(b, p.x, p.y))
    p.v = boris(b, p.v, gather(b, p.x, p.y, E), -0.5 * b.dt)
    return E


def step(b: Box, p: Plasma, E):
    """One cycle: push under E^n, move, absorb at the walls, deposit, solve.
    Returns (E^{n+1}, rho^{n+1}, KE^n) and updates p in place."""
    v2 = lambda v: float(sum(np.dot(a, a) for a in v))
    v2_old = v2(p.v)
    p.v = boris(b, p.v, gather(b, p.x, p.y, E), b.dt)
    v2_new = v2(p.v)
    x = p.x + p.v[0] * b.dt
    y = np.mod(p.y + p.v[1] * b.dt, b.Ly)
    y = np.where(y >= b.Ly, y - b.Ly, y)
    left, right = x < 0.0, x >= b.Lx
    keep = ~(left | right)
    p.lost_left += int(left.sum())
    p.lost_right += int(right.sum())
    p.x, p.y = x[keep], y[keep]
    p.v = [a[keep] for a in p.v]
    if p.ids is not None:
        p.ids = p.ids[keep]
    rho = deposit(b, p.x, p.y)
    return solve_field(b, rho), rho, 0.5 * b.M * 0.5 * (v2_old + v2_new)
