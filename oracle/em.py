"""Serial FP64 reference for the electromagnetic PIC step in 2D3V on a
periodic Yee grid: charge-conserving current deposit (B_Scatter of current
densities), staggered gather (C_Gather), Boris in the gathered E and B
(A_Pusher) and the finite-difference time-domain update of Maxwell's
equations (E_Maxwell, Yee 1966).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the test-suite, the
smoke check and the CPU-baseline leg of the benchmark use it; the product
never imports it.

The paper names these modules without writing them out. The readings taken
here (each listed in the design notes of the repository):
  * normalised units eps0 = 1, mu0 = 1/c^2 (c in units of v_th / omega_pe
    lengths per plasma time), electrons q/m = -1, immobile uniform ions;
  * Yee staggering in the x-y plane (``em_oracle.c`` header); all six
    components are kept (2D3V: both polarisations);
  * a uniform external B0 = bz z is part of the grid's Bz from the start (a
    uniform field has no curl, so the update keeps it);
  * E^0 from the electrostatic solve of the initial charge, taken as the
    staggered difference of phi (so the discrete Gauss law holds exactly);
  * one step: gather E^n, B^n at x^n; Boris v^{n-1/2} -> v^{n+1/2}; move
    x^{n+1} = x^n + v^{n+1/2} dt; current J^{n+1/2} by Esirkepov from x^n to
    x^{n+1}; then B^{n+1/2} = B^n - dt/2 curl E^n,
    E^{n+1} = E^n + dt (c^2 curl B^{n+1/2} - J^{n+1/2}),
    B^{n+1} = B^{n+1/2} - dt/2 curl E^{n+1} (the Yee leapfrog with B also
    held at integer times for the push);
  * the initial half push is backward, v^{-1/2} = Boris(v^0, E^0, B^0, -dt/2);
  * with pusher "hc" the velocity advance is Higuera & Cary (2017) in its
    general-field form, the state holds u = gamma v, the move and the current
    use u / gamma;
  * energies: W_E = 1/2 sum |E|^2 dV, W_B = c^2/2 sum |B - B0|^2 dV (the
    self-consistent part), KE as in the electrostatic cycle.
The particle loops are serial C (``em_oracle.c``); the field update is
written with numpy array shifts.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import Setup, State, _c64, deposit, kinetic_sum, move, solve_potential

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "em_oracle.c")
_SO = os.path.join(_HERE, "_em_oracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double


def build(force: bool = True) -> str:
    """Compile the C part with gcc (serial, FP64, no FMA contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build(force=True)
    L = ctypes.CDLL(_SO)
    L.or_em_gather_2d.argtypes = [_i64, _D, _D, _int, _int, _dbl, _dbl, _D, _D]
    L.or_em_gather_2d.restype = None
    L.or_boris3.argtypes = [_i64, _D, _D, _D, _D, _D, _dbl, _dbl]
    L.or_boris3.restype = None
    L.or_hc3.argtypes = [_i64, _D, _D, _D, _D, _D, _dbl, _dbl, _dbl]
    L.or_hc3.restype = None
    L.or_esirkepov_2d.argtypes = [_i64, _D, _D, _D, _D, _D, _int, _int, _dbl, _dbl, _dbl, _dbl, _D]
    L.or_esirkepov_2d.restype = _i64
    _lib = L
    return L


def _p(a):
    return a.ctypes.data_as(_D)


def check_setup(s: Setup) -> None:
    if s.dim != 2 or s.vdim != 3 or not np.isfinite(s.c) or s.c <= 0:
        raise ValueError("the electromagnetic step is 2D3V with a finite c > 0")


def gather(s: Setup, st: State, F: np.ndarray):
    """(E_p, B_p), each [3][n], at the particle positions; F is [6][ny][nx]."""
    n = st.x.shape[0]
    out = np.empty((6, n))
    _load().or_em_gather_2d(n, _p(_c64(st.x)), _p(_c64(st.y)), s.nx, s.ny, s.dx, s.dy, _p(_c64(F)), _p(out))
    return out[:3], out[3:]


def boris(s: Setup, st: State, Ep: np.ndarray, Bp: np.ndarray, dt: float) -> None:
    """In-place velocity advance by dt in the gathered E and B ([3][n] each):
    Boris, or Higuera-Cary in its general-field form when s.pusher == "hc"
    (the state then holds u = gamma v)."""
    n = st.x.shape[0]
    if s.pusher == "hc":
        _load().or_hc3(n, _p(st.vx), _p(st.vy), _p(st.vz), _p(_c64(Ep)), _p(_c64(Bp)), s.qm, dt, s.c)
        return
    _load().or_boris3(n, _p(st.vx), _p(st.vy), _p(st.vz), _p(_c64(Ep)), _p(_c64(Bp)), s.qm, dt)


def velocity(s: Setup, st: State):
    """dx/dt of the state: v, or u / gamma with gamma = sqrt(1 + |u|^2/c^2)."""
    if s.pusher != "hc":
        return st.vx, st.vy, st.vz
    g = np.sqrt(1.0 + (st.vx * st.vx + st.vy * st.vy + st.vz * st.vz) * (1.0 / (s.c * s.c)))
    return st.vx / g, st.vy / g, st.vz / g


def current(s: Setup, x0, y0, ddx, ddy, vz, q: float = None) -> np.ndarray:
    """J [3][ny][nx] of particles moving from (x0, y0) by (ddx, ddy) in one
    step (Esirkepov). Raises if a particle moves a cell or more along an axis."""
    n = x0.shape[0]
    J = np.zeros((3, s.ny, s.nx))
    q = s.Q if q is None else q
    skipped = _load().or_esirkepov_2d(n, _p(_c64(x0)), _p(_c64(y0)), _p(_c64(ddx)), _p(_c64(ddy)), _p(_c64(vz)),
                                      s.nx, s.ny, s.dx, s.dy, q, s.dt, _p(J))
    if skipped:
        raise ValueError("%d particles moved a cell or more in one step" % skipped)
    return J


def curl_e(s: Setup, F: np.ndarray):
    """curl E at the B locations: (dEz/dy, -dEz/dx, dEy/dx - dEx/dy)."""
    Ex, Ey, Ez = F[0], F[1], F[2]
    fwd_x = lambda a: (np.roll(a, -1, axis=1) - a) / s.dx
    fwd_y = lambda a: (np.roll(a, -1, axis=0) - a) / s.dy
    return fwd_y(Ez), -fwd_x(Ez), fwd_x(Ey) - fwd_y(Ex)


def curl_b(s: Setup, F: np.ndarray):
    """curl B at the E locations: (dBz/dy, -dBz/dx, dBy/dx - dBx/dy)."""
    Bx, By, Bz = F[3], F[4], F[5]
    bwd_x = lambda a: (a - np.roll(a, 1, axis=1)) / s.dx
    bwd_y = lambda a: (a - np.roll(a, 1, axis=0)) / s.dy
    return bwd_y(Bz), -bwd_x(Bz), bwd_x(By) - bwd_y(Bx)


def advance_b(s: Setup, F: np.ndarray, h: float) -> None:
    """Faraday: B -= h curl E (in place)."""
    cx, cy, cz = curl_e(s, F)
    F[3] -= h * cx
    F[4] -= h * cy
    F[5] -= h * cz


def advance_e(s: Setup, F: np.ndarray, J: np.ndarray, h: float) -> None:
    """Ampere: E += h (c^2 curl B - J) (in place)."""
    cx, cy, cz = curl_b(s, F)
    c2 = s.c * s.c
    F[0] += h * (c2 * cx - J[0])
    F[1] += h * (c2 * cy - J[1])
    F[2] += h * (c2 * cz - J[2])


def maxwell(s: Setup, F: np.ndarray, J: np.ndarray) -> None:
    """One field step: B half, E full, B half."""
    advance_b(s, F, 0.5 * s.dt)
    advance_e(s, F, J, s.dt)
    advance_b(s, F, 0.5 * s.dt)


def staggered_e(s: Setup, phi: np.ndarray):
    """(Ex, Ey) = -(forward differences of phi) at the Ex and Ey locations."""
    return (-(np.roll(phi, -1, axis=1) - phi) / s.dx, -(np.roll(phi, -1, axis=0) - phi) / s.dy)


def divergence_e(s: Setup, F: np.ndarray) -> np.ndarray:
    """div E at the nodes."""
    return (F[0] - np.roll(F[0], 1, axis=1)) / s.dx + (F[1] - np.roll(F[1], 1, axis=0)) / s.dy


def divergence_b(s: Setup, F: np.ndarray) -> np.ndarray:
    """div B at the cell centres."""
    return (np.roll(F[3], -1, axis=1) - F[3]) / s.dx + (np.roll(F[4], -1, axis=0) - F[4]) / s.dy


def initial_fields(s: Setup, st: State) -> np.ndarray:
    """F^0: E from the electrostatic solve of the initial charge, B = B0."""
    check_setup(s)
    F = np.zeros((6, s.ny, s.nx))
    Ex, Ey = staggered_e(s, solve_potential(s, deposit(s, st)))
    F[0], F[1] = Ex, Ey
    F[5] = s.bz
    return F


def initialise(s: Setup, st: State):
    """F^0, then the backward half push v^0 -> v^{-1/2}."""
    F = initial_fields(s, st)
    Ep, Bp = gather(s, st, F)
    boris(s, st, Ep, Bp, -0.5 * s.dt)
    return F


def step(s: Setup, st: State, F: np.ndarray):
    """One electromagnetic cycle in place on st and F; returns (J^{n+1/2}, KE^n)."""
    Ep, Bp = gather(s, st, F)
    v2_old = kinetic_sum(s, st)
    boris(s, st, Ep, Bp, s.dt)
    v2_new = kinetic_sum(s, st)
    x0, y0 = st.x.copy(), st.y.copy()
    vx, vy, vz = velocity(s, st)
    J = current(s, x0, y0, vx * s.dt, vy * s.dt, vz)
    move(s, st)
    maxwell(s, F, J)
    return J, 0.5 * s.M * 0.5 * (v2_old + v2_new)


def field_energies(s: Setup, F: np.ndarray):
    """(W_E, W_B) with W_B of B - B0."""
    dV = s.dV
    we = 0.5 * dV * float(np.sum(F[0] ** 2) + np.sum(F[1] ** 2) + np.sum(F[2] ** 2))
    wb = 0.5 * s.c * s.c * dV * float(np.sum(F[3] ** 2) + np.sum(F[4] ** 2) + np.sum((F[5] - s.bz) ** 2))
    return we, wb
