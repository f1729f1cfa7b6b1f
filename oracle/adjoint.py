"""FP64 reference gradient of the PIC cycle (discrete adjoint), serial CPU.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the test-suite and
the smoke check use it to check the HIP adjoint; the product never imports it.

The paper has no adjoint; this is the reverse-mode derivative of the exact
discrete map the oracle's forward cycle computes (``oracle.step`` order:
gather E^n -> Boris -> move -> deposit -> Poisson -> E^{n+1}, after the field
of the initial charge and the backward half push of "Example setup and
implementation"). The objective is the final field energy
W = 1/2 sum_j |E_j^T|^2 dV, and the gradients are taken with respect to the
initial positions x^0 and velocities v^0 of every particle. Plasmas in 1D,
2D and 3D (the Cartesian three-dimensional form: trilinear weights, the
7-point solve, E_z kicks).

Adjoint of each module (lam_* is the derivative of W with respect to *):
  field      E = A rho, with A the FFT solve of the FD Poisson problem and the
             centred gradient; A is real and circulant with the odd symbol
             -i kappa_d / K^2, so A^T has the conjugate symbol +i kappa_d / K^2:
             lam_rho = sum_d A_d^T lam_E_d.
  deposit    rho_j = rho_ion + (Q/dV) sum_p W_j(x_p):
             lam_x_p += (Q/dV) sum_j lam_rho_j dW_j/dx(x_p).
  gather     E_p = sum_j W_j(x_p) E_j: lam_E_j += sum_p W_j(x_p) lam_Ep_p and
             lam_x_p += sum_j dW_j/dx(x_p) E_j . lam_Ep_p.
  Boris      v_new = R v + a (R + I) E_p (linear for fixed B):
             lam_v_old = R^T lam_v_new, lam_Ep = a (R + I)^T lam_v_new.
  move       x^{n+1} = wrap(x^n + v^{n+1/2} dt): lam_x^n = lam_x^{n+1},
             lam_v^{n+1/2} += dt lam_x^{n+1} (the periodic wrap has slope one).
With the Higuera-Cary advance (pusher "hc", state u = gamma v) two modules
are nonlinear in u and take the trajectory's velocities:
  advance    u1 solves the implicit midpoint relation that defines the method,
             F(u0, u1, E) = u1 - u0 - 2aE - (u0 + u1) x (tau / gamma(ubar)) z = 0
             with ubar = (u0 + u1) / 2; by the implicit function theorem
             lam_u0 = -J0^T J1^-T lam_u1 and lam_E = 2a J1^-T lam_u1, with
             J0 = dF/du0 and J1 = dF/du1 (one 3 x 3 solve per particle);
  move       x += (u / gamma(u)) dt: lam_u += dt M lam_x with the symmetric
             M = (I - u u^T / (c^2 gamma^2)) / gamma.
The CIC hat is piecewise linear, so dW/dx is its slope inside the particle's
cell: the derivative almost everywhere, which is what central differences of
the forward map see at steps small against a cell.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from . import (Setup, State, _c64, _D, _load, _p, boris, centred_kappa, deposit, field_energy, gather,
               modified_k2, move, solve_field)


def solve_field_adjoint(s: Setup, lam_E) -> np.ndarray:
    """lam_rho = A^T lam_E for the field operator A of ``solve_field``.

    In Fourier space lam_rho_hat = sum_d (+i kappa_d / K^2) lam_E_d_hat, with
    the k = 0 mode zero (A drops the mean of rho)."""
    if s.dim == 1:
        K2 = modified_k2(s.nx, s.dx).copy()
        K2[0] = 1.0
        h = 1j * centred_kappa(s.nx, s.dx) * np.fft.fft(lam_E[0]) / K2
        h[0] = 0.0
        return np.real(np.fft.ifft(h))
    if s.dim == 3:
        kz2, ky2, kx2 = modified_k2(s.nz, s.dz), modified_k2(s.ny, s.dy), modified_k2(s.nx, s.dx)
        K2 = kz2[:, None, None] + ky2[None, :, None] + kx2[None, None, :]
        K2[0, 0, 0] = 1.0
        h = (1j * centred_kappa(s.nx, s.dx)[None, None, :] * np.fft.fftn(lam_E[0])
             + 1j * centred_kappa(s.ny, s.dy)[None, :, None] * np.fft.fftn(lam_E[1])
             + 1j * centred_kappa(s.nz, s.dz)[:, None, None] * np.fft.fftn(lam_E[2])) / K2
        h[0, 0, 0] = 0.0
        return np.real(np.fft.ifftn(h))
    K2 = modified_k2(s.ny, s.dy)[:, None] + modified_k2(s.nx, s.dx)[None, :]
    K2[0, 0] = 1.0
    h = (1j * centred_kappa(s.nx, s.dx)[None, :] * np.fft.fft2(lam_E[0])
         + 1j * centred_kappa(s.ny, s.dy)[:, None] * np.fft.fft2(lam_E[1])) / K2
    h[0, 0] = 0.0
    return np.real(np.fft.ifft2(h))


def _positions(st: State):
    return (st.x.copy(), None if st.y is None else st.y.copy(), None if st.z is None else st.z.copy())


def _velocities(st: State):
    return [None if a is None else a.copy() for a in (st.vx, st.vy, st.vz)]


def trajectory(s: Setup, st0: State, nsteps: int):
    """Run the cycle from (x^0, v^0) and keep what the reverse sweep needs.

    Returns (W, xs, vs, Es): W = W_E(T); xs[n] = positions at time level n
    (n = 0..T); vs[n] = velocities held at level n, v^{n-1/2} (vs[0] is the
    result of the backward half push); Es[n] = node field E^n. st0 is not
    modified."""
    st = st0.copy()
    E = solve_field(s, deposit(s, st))
    xs = [_positions(st)]
    Es = [E]
    boris(s, st, gather(s, st, E), -0.5 * s.dt)
    vs = [_velocities(st)]
    for _ in range(nsteps):
        boris(s, st, gather(s, st, E), s.dt)
        move(s, st)
        E = solve_field(s, deposit(s, st))
        xs.append(_positions(st))
        vs.append(_velocities(st))
        Es.append(E)
    return field_energy(s, E), xs, vs, Es


def forward_trajectory(s: Setup, st0: State, nsteps: int):
    """(W, xs, Es) of ``trajectory``."""
    W, xs, _, Es = trajectory(s, st0, nsteps)
    return W, xs, Es


def _pos_state(s: Setup, pos) -> State:
    return State(pos[0], np.zeros_like(pos[0]), pos[1], None, None, pos[2])


def adj_deposit(s: Setup, pos, lam_rho, lam_x) -> None:
    """lam_x += (Q/dV) sum_j lam_rho_j dW_j/dx at the positions pos (in place)."""
    L = _load()
    x, y, z = (tuple(pos) + (None, None))[:3]
    n = x.shape[0]
    c = s.Q / s.dV
    lr = _c64(lam_rho)
    if s.dim == 3:
        L.or_adj_deposit_3d(n, _p(x, _D), _p(y, _D), _p(z, _D), s.nx, s.ny, s.nz, s.dx, s.dy, s.dz, c, _p(lr, _D),
                            _p(lam_x[0], _D), _p(lam_x[1], _D), _p(lam_x[2], _D))
    elif s.dim == 1:
        L.or_adj_deposit_1d(n, _p(x, _D), s.nx, s.dx, c, _p(lr, _D), _p(lam_x[0], _D))
    else:
        L.or_adj_deposit_2d(n, _p(x, _D), _p(y, _D), s.nx, s.ny, s.dx, s.dy, c, _p(lr, _D),
                            _p(lam_x[0], _D), _p(lam_x[1], _D))


def adj_gather(s: Setup, pos, E, lam_Ep, lam_E, lam_x) -> None:
    """Scatter lam_Ep into lam_E and add the field-gradient term to lam_x."""
    L = _load()
    x, y, z = (tuple(pos) + (None, None))[:3]
    n = x.shape[0]
    if s.dim == 3:
        Ex, Ey, Ez = (_c64(e) for e in E)
        L.or_adj_gather_3d(n, _p(x, _D), _p(y, _D), _p(z, _D), s.nx, s.ny, s.nz, s.dx, s.dy, s.dz, _p(Ex, _D),
                           _p(Ey, _D), _p(Ez, _D), _p(lam_Ep[0], _D), _p(lam_Ep[1], _D), _p(lam_Ep[2], _D),
                           _p(lam_E[0], _D), _p(lam_E[1], _D), _p(lam_E[2], _D), _p(lam_x[0], _D), _p(lam_x[1], _D),
                           _p(lam_x[2], _D))
    elif s.dim == 1:
        L.or_adj_gather_1d(n, _p(x, _D), s.nx, s.dx, _p(_c64(E[0]), _D), _p(lam_Ep[0], _D), _p(lam_E[0], _D),
                           _p(lam_x[0], _D))
    else:
        L.or_adj_gather_2d(n, _p(x, _D), _p(y, _D), s.nx, s.ny, s.dx, s.dy, _p(_c64(E[0]), _D),
                           _p(_c64(E[1]), _D), _p(lam_Ep[0], _D), _p(lam_Ep[1], _D), _p(lam_E[0], _D),
                           _p(lam_E[1], _D), _p(lam_x[0], _D), _p(lam_x[1], _D))


def adj_boris(s: Setup, lam_v, dt: float):
    """Boris adjoint for a velocity advance by dt: lam_v (list of vdim arrays,
    lam of v_new) becomes lam of v_old in place; returns lam_Ep (dim arrays)."""
    L = _load()
    n = lam_v[0].shape[0]
    lEx = np.zeros(n)
    lEy = np.zeros(n) if s.dim >= 2 else None
    lvy = lam_v[1] if s.vdim >= 2 else None
    L.or_adj_boris(n, s.vdim, _p(lam_v[0], _D), _p(lvy, _D), _p(lEx, _D), _p(lEy, _D), s.qm, dt, s.bz)
    # the pusher's electric field has dim components; with vdim > dim (2D3V
    # has no E_z) the extra velocity components take no kick
    if s.dim == 3:
        # the rotation about z leaves v_z alone: v_z gains the two half kicks
        # a E_z, so lam_Ez = 2a lam_vz and lam_vz passes through
        return [lEx, lEy, 2.0 * (s.qm * dt * 0.5) * lam_v[2]]
    return [lEx] if s.dim == 1 else [lEx, lEy]


def adj_hc(s: Setup, u_old, Ep, lam_v, dt: float):
    """Higuera-Cary adjoint for one advance by dt from u_old (3 arrays) under
    Ep (dim arrays): lam_v (3 arrays, lam of u_new) becomes lam of u_old in
    place; returns lam_Ep (one array per component of Ep).

    From the defining relation F(u0, u1, E) = 0 (module header), with
    w = u0 + u1, beta = tau / gamma(w / 2) and K the matrix of w -> w x z:
      dF/du1 = I - beta K - (w x z) dbeta^T,
      dF/du0 = -I - beta K - (w x z) dbeta^T,
      dbeta/du0 = dbeta/du1 = -beta ubar / (2 c^2 gamma(ubar)^2),
      dF/dE = -2a I."""
    n = u_old[0].shape[0]
    st = State(np.zeros(n), u_old[0].copy(), np.zeros(n), u_old[1].copy(), u_old[2].copy())
    boris(s, st, Ep, dt)
    u0 = np.stack(u_old, axis=1)
    u1 = np.stack([st.vx, st.vy, st.vz], axis=1)
    a = s.qm * dt / 2.0
    tau = a * s.bz
    ic2 = 1.0 / (s.c * s.c)
    w = u0 + u1
    ub = 0.5 * w
    gb2 = 1.0 + ic2 * np.sum(ub * ub, axis=1)
    beta = tau / np.sqrt(gb2)
    wxz = np.stack([w[:, 1], -w[:, 0], np.zeros(n)], axis=1)
    dbeta = (-beta * ic2 / (2.0 * gb2))[:, None] * ub
    K = np.array([[0.0, 1.0, 0.0], [-1.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    common = beta[:, None, None] * K + wxz[:, :, None] * dbeta[:, None, :]
    J1 = np.eye(3) - common
    J0 = -np.eye(3) - common
    lam = np.stack(lam_v, axis=1)
    mu = np.linalg.solve(np.transpose(J1, (0, 2, 1)), lam[:, :, None])[:, :, 0]
    lam_u0 = -np.einsum("pji,pj->pi", J0, mu)
    for k in range(3):
        lam_v[k][:] = lam_u0[:, k]
    return [2.0 * a * mu[:, k] for k in range(len(Ep))]


def adj_move_u(s: Setup, u, lam_x, lam_v) -> None:
    """Move x += (u / gamma) dt (each of the dim position axes):
    lam_v += dt M lam_x with M = (I - u u^T / (c^2 gamma^2)) / gamma."""
    ic2 = 1.0 / (s.c * s.c)
    u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    g = np.sqrt(1.0 + ic2 * u2)
    lx = [lam_x[k] if k < s.dim else np.zeros_like(u[0]) for k in range(3)]
    dot = u[0] * lx[0] + u[1] * lx[1] + u[2] * lx[2]
    for k in range(3):
        lam_v[k] += s.dt / g * (lx[k] - ic2 * u[k] * dot / (g * g))


def adjoint(s: Setup, st0: State, nsteps: int, seed: float = 1.0):
    """Reverse sweep of the cycle from (x^0, v^0) over nsteps steps.

    Returns (W, lam_x, lam_v): W = W_E(T), lam_x = [dW/dx^0 (, dW/dy^0)],
    lam_v = [dW/dv_x^0, ...] (vdim arrays), all multiplied by seed."""
    W, xs, vs, Es = trajectory(s, st0, nsteps)
    hc = s.pusher == "hc"
    n = st0.x.shape[0]
    lam_x = [np.zeros(n) for _ in range(s.dim)]
    lam_v = [np.zeros(n) for _ in range(s.vdim)]
    # level T: only the objective depends on E^T
    lam_E = [seed * s.dV * _c64(e).copy() for e in Es[nsteps]]
    for lev in range(nsteps, -1, -1):
        # complete level lev: E^lev = A rho(x^lev)
        adj_deposit(s, xs[lev], solve_field_adjoint(s, lam_E), lam_x)
        if lev == 0:
            break
        # reverse step lev-1: x^lev = x^{lev-1} + v^{lev-1/2} dt, v^{lev-1/2} = Boris(v^{lev-3/2}, E_p^{lev-1})
        if hc:
            Ep = gather(s, _pos_state(s, xs[lev - 1]), Es[lev - 1])
            adj_move_u(s, vs[lev], lam_x, lam_v)
            lam_Ep = adj_hc(s, vs[lev - 1], Ep, lam_v, s.dt)
            if lev - 1 == 0:
                u0 = [st0.vx, st0.vy, st0.vz]
                lam_h = adj_hc(s, u0, Ep, lam_v, -0.5 * s.dt)
                lam_Ep = [a + b for a, b in zip(lam_Ep, lam_h)]
        else:
            for d in range(s.dim):
                lam_v[d] += s.dt * lam_x[d]
            lam_Ep = adj_boris(s, lam_v, s.dt)
            if lev - 1 == 0:
                # the backward half push v^{-1/2} = Boris(v^0, E_p^0, -dt/2) uses the same E_p^0
                lam_h = adj_boris(s, lam_v, -0.5 * s.dt)
                lam_Ep = [a + b for a, b in zip(lam_Ep, lam_h)]
        lam_E = [np.zeros(s.grid_shape) for _ in range(s.dim)]
        adj_gather(s, xs[lev - 1], Es[lev - 1], lam_Ep, lam_E, lam_x)
    return W, lam_x, lam_v


def delta0_direction(s: Setup, x_u, y_u, mode) -> List[np.ndarray]:
    """d x^0 / d delta0 for the mode seeding x = x_u + delta0 k/|k|^2 sin(k.x_u)
    (per axis; the periodic wrap has slope one). In 3D the mode is
    (mx, my, 0): z is not displaced."""
    kx = 2.0 * np.pi * mode[0] / s.Lx
    ky = 2.0 * np.pi * mode[1] / s.Ly if s.dim >= 2 else 0.0
    k2 = kx * kx + ky * ky
    ph = kx * x_u + (ky * y_u if s.dim >= 2 else 0.0)
    sn = np.sin(ph)
    out = [kx / k2 * sn]
    if s.dim >= 2:
        out.append(ky / k2 * sn)
    if s.dim == 3:
        out.append(np.zeros_like(sn))
    return out


def grad_delta0(lam_x, direction) -> float:
    """dW/d delta0 = sum_p lam_x_p . d x_p^0 / d delta0."""
    return float(sum(np.dot(a, b) for a, b in zip(lam_x, direction)))
