"""An independent vectorised re-implementation of the oracle's PIC cycle in
plain torch (CPU, float64), differentiated by torch.autograd.

Used only as a cross-check of the oracle's hand-written adjoint: it shares no
code with it (no C operators, its own CIC, Poisson and Boris written from the
same textbook definitions), so agreement of the two gradients pins both the
forward map and its adjoint.
"""
from __future__ import annotations

import math

import torch

DT = torch.float64


def _cic(x, n, d):
    g = x / d
    i = torch.floor(g.detach())
    f = g - i                               # slope 1/d inside the cell
    i = i.long()
    edge = i >= n                           # a coordinate rounding onto L belongs to node 0
    i = torch.where(edge, torch.zeros_like(i), i)
    f = torch.where(edge, f - n, f)
    return i, (i + 1) % n, f


def _kmod(n, d):
    k = 2.0 * math.pi * torch.fft.fftfreq(n, d=d, dtype=DT)
    return (2.0 / d * torch.sin(k * d / 2.0)) ** 2, torch.sin(k * d) / d


class Plasma:
    def __init__(self, dim, vdim, nx, Lx, n, dt, ny=1, Ly=1.0, qm=-1.0, bz=0.0, n0=1.0, pusher="boris", c=math.inf):
        self.pusher, self.c = pusher, c
        self.dim, self.vdim, self.nx, self.ny = dim, vdim, nx, (ny if dim == 2 else 1)
        self.Lx, self.Ly = Lx, (Ly if dim == 2 else 1.0)
        self.dx, self.dy = Lx / nx, (self.Ly / self.ny if dim == 2 else 1.0)
        self.dV = self.dx * self.dy
        self.n, self.dt, self.qm, self.bz, self.n0 = n, dt, qm, bz, n0
        vol = self.Lx * self.Ly
        self.Q = -n0 * vol / n

    def deposit(self, x, y):
        if self.dim == 1:
            i, ip, f = _cic(x, self.nx, self.dx)
            rho = torch.zeros(self.nx, dtype=DT)
            rho = rho.index_add(0, i, 1.0 - f).index_add(0, ip, f)
        else:
            i, ip, fx = _cic(x, self.nx, self.dx)
            j, jp, fy = _cic(y, self.ny, self.dy)
            rho = torch.zeros(self.nx * self.ny, dtype=DT)
            for a, b, w in ((i, j, (1 - fx) * (1 - fy)), (ip, j, fx * (1 - fy)), (i, jp, (1 - fx) * fy),
                            (ip, jp, fx * fy)):
                rho = rho.index_add(0, b * self.nx + a, w)
            rho = rho.reshape(self.ny, self.nx)
        return self.n0 + self.Q / self.dV * rho

    def field(self, rho):
        if self.dim == 1:
            K2, kap = _kmod(self.nx, self.dx)
            K2 = torch.where(K2 == 0, torch.ones_like(K2), K2)
            ph = torch.fft.fft(rho.to(torch.complex128)) / K2
            ph = torch.cat([ph[:1] * 0, ph[1:]])
            return (torch.fft.ifft(-1j * kap * ph).real,)
        K2x, kapx = _kmod(self.nx, self.dx)
        K2y, kapy = _kmod(self.ny, self.dy)
        K2 = K2y[:, None] + K2x[None, :]
        mask = torch.ones_like(K2)
        mask[0, 0] = 0.0
        K2 = torch.where(mask == 0, torch.ones_like(K2), K2)
        ph = torch.fft.fft2(rho.to(torch.complex128)) / K2 * mask
        return (torch.fft.ifft2(-1j * kapx[None, :] * ph).real, torch.fft.ifft2(-1j * kapy[:, None] * ph).real)

    def gather(self, x, y, E):
        if self.dim == 1:
            i, ip, f = _cic(x, self.nx, self.dx)
            return (E[0][i] * (1 - f) + E[0][ip] * f,)
        i, ip, fx = _cic(x, self.nx, self.dx)
        j, jp, fy = _cic(y, self.ny, self.dy)
        out = []
        for e in E:
            out.append(e[j, i] * (1 - fx) * (1 - fy) + e[j, ip] * fx * (1 - fy) + e[jp, i] * (1 - fx) * fy
                       + e[jp, ip] * fx * fy)
        return tuple(out)

    def higuera_cary(self, u, Ep, dt):
        """Higuera & Cary (2017) in its vector form, u = gamma v, B = bz z:
        u- = u + a E; gamma_new^2 = (sigma + sqrt(sigma^2 + 4 (|tau|^2 + (u-.tau)^2/c^2))) / 2
        with sigma = gamma(u-)^2 - |tau|^2; t = tau / gamma_new; s = 1/(1+|t|^2);
        u+ = s (u- + (u-.t) t + u- x t); u_new = u+ + a E + u+ x t."""
        a = self.qm * dt / 2.0
        n = u[0].shape[0]
        E3 = torch.stack(list(Ep) + [torch.zeros(n, dtype=DT)] * (3 - len(Ep)), dim=1)
        um = torch.stack(u, dim=1) + a * E3
        tau = torch.tensor([0.0, 0.0, a * self.bz], dtype=DT).expand(n, 3)
        ic2 = 1.0 / (self.c * self.c)
        sig = 1.0 + ic2 * (um * um).sum(1) - (tau * tau).sum(1)
        ust = (um * tau).sum(1)
        gnew = torch.sqrt(0.5 * (sig + torch.sqrt(sig * sig + 4.0 * ((tau * tau).sum(1) + ic2 * ust * ust))))
        t = tau / gnew[:, None]
        sfac = 1.0 / (1.0 + (t * t).sum(1))
        up = sfac[:, None] * (um + (um * t).sum(1, keepdim=True) * t + torch.linalg.cross(um, t, dim=1))
        out = up + a * E3 + torch.linalg.cross(up, t, dim=1)
        return [out[:, 0], out[:, 1], out[:, 2]]

    def velocity(self, u):
        """dx/dt of the state: v, or u / gamma for the relativistic state."""
        if self.pusher != "hc":
            return u
        g = torch.sqrt(1.0 + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / (self.c * self.c))
        return [a / g for a in u]

    def boris(self, v, Ep, dt):
        if self.pusher == "hc":
            return self.higuera_cary(v, Ep, dt)
        a = self.qm * dt / 2.0
        if self.vdim == 1:
            return [v[0] + 2.0 * a * Ep[0]]
        t = a * self.bz
        s = 2.0 * t / (1.0 + t * t)
        mx, my = v[0] + a * Ep[0], v[1] + a * Ep[1]
        px, py = mx + my * t, my - mx * t            # v- + v- x t (t along z)
        qx, qy = mx + py * s, my - px * s            # v- + v' x s
        out = [qx + a * Ep[0], qy + a * Ep[1]]
        if self.vdim == 3:
            out.append(v[2])                          # no E_z, rotation about z
        return out

    def run(self, x, y, v, nsteps):
        """Field energy W_E(T) of the cycle started from (x^0, v^0)."""
        E = self.field(self.deposit(x, y))
        v = self.boris(v, self.gather(x, y, E), -0.5 * self.dt)
        for _ in range(nsteps):
            v = self.boris(v, self.gather(x, y, E), self.dt)
            vel = self.velocity(v)
            x = torch.remainder(x + vel[0] * self.dt, self.Lx)
            if self.dim == 2:
                y = torch.remainder(y + vel[1] * self.dt, self.Ly)
            E = self.field(self.deposit(x, y))
        return 0.5 * sum((e * e).sum() for e in E) * self.dV
