"""Driver of one plasma on the GPU: uploads a seeded initial state, runs the
paper's PIC cycle through libapic and hands diagnostics back.

The cycle is the two-stream example's driver order: field of the initial
charge (sort -> deposit -> Poisson), the initial backward half push of the
velocities, then apic_step for the time loop. Host code here only marshals
arguments and converts the seeded FP64 input to the caller's representation.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import workloads as W
from .apic import Batch, Context, Particles


class Simulation:
    def __init__(self, w: W.Workload, precision: str = "mixed", n: Optional[int] = None, state=None,
                 tile=(0, 0), frac_bits: int = 0, device="cuda", pusher: str = "boris", c_light: float = 0.0,
                 walls: bool = False):
        import torch
        self.torch = torch
        self.w = w
        if state is None:
            state = W.sample3(w, n) if w.dim == 3 else W.sample(w, n)
        self.n = len(state[0])
        mk = lambda t: Context(dim=w.dim, vdim=w.vdim, nx=w.nx, ny=w.ny, lx=w.Lx, ly=w.Ly, dt=w.dt, n=self.n,
                               bz=w.bz, precision=precision, frac_bits=frac_bits, tile=t, device=device,
                               nz=w.nz, lz=w.Lz, pusher=pusher, c_light=c_light, walls=walls)
        self.tune_ms = None
        if tile == "auto" and walls:
            # the tile autotuner covers periodic plasmas; between walls the default tile is kept
            tile = (0, 0)
        if tile == "auto":
            # time the candidate tiles on this very state, then build the context with the pick
            ctx = mk((0, 0, 0) if w.dim == 3 else (0, 0))
            p = Particles(ctx)
            self._upload(p, ctx.mixed, state)
            tile, self.tune_ms = ctx.autotune_tiles(p)
            del p, ctx
        self.ctx = mk(tuple(tile))
        self.tile = self.ctx.tile      # the tile the context uses (defaults resolved)
        self.mixed = self.ctx.mixed
        self.p = Particles(self.ctx)
        self._upload(self.p, self.mixed, state)
        dev = self.ctx.device
        G = self.ctx.G
        self.E = torch.zeros(w.dim * G, dtype=torch.float64, device=dev)
        self.E32 = torch.zeros(w.dim * G, dtype=torch.float32, device=dev) if self.mixed else None
        self.rho = torch.zeros(G, dtype=torch.int64 if self.mixed else torch.float64, device=dev)
        self.we0 = torch.zeros(1, dtype=torch.float64, device=dev)

    def _upload(self, p, mixed, state):
        w = self.w
        if w.dim == 3:
            x, y, z, vx, vy, vz = state
            if mixed:
                c = [W.to_cell_offset(a, d, n) for a, d, n in ((x, w.dx, w.nx), (y, w.dy, w.ny), (z, w.dz, w.nz))]
                p.upload(cell=W.pack_cell(c[0][0], c[1][0], c[2][0]), ox=c[0][1], oy=c[1][1], oz=c[2][1],
                         vx=vx, vy=vy, vz=vz)
            else:
                p.upload(x=x, y=y, z=z, vx=vx, vy=vy, vz=vz)
            return
        x, y, vx, vy, vz = state
        if mixed:
            ix, ox = W.to_cell_offset(x, w.dx, w.nx)
            iy = oy = None
            if w.dim == 2:
                iy, oy = W.to_cell_offset(y, w.dy, w.ny)
            p.upload(cell=W.pack_cell(ix, iy), ox=ox, oy=oy, vx=vx, vy=vy, vz=vz)
        else:
            p.upload(x=x, y=y, vx=vx, vy=vy, vz=vz)

    def initialise(self):
        c = self.ctx
        c.sort_by_cell(self.p)
        c.deposit(self.p, self.rho)
        c.field_solve(self.rho, self.E, self.E32, self.we0)
        c.gather_push(self.p, self.E32 if self.mixed else self.E, dt_scale=-0.5, move=False)

    def run(self, nsteps: int, diag: bool = True, rho_out=None, perm=None):
        d = None
        if diag:
            d = self.torch.zeros(nsteps * 4, dtype=self.torch.float64, device=self.ctx.device)
        self.ctx.step(self.p, self.E, self.E32, nsteps, d, rho=rho_out, perm=perm)
        return d

    def field(self):
        G = self.ctx.G
        e = self.E.cpu().numpy()
        if self.w.dim == 1:
            return (e[:G].copy(),)
        sh = (self.w.nz, self.w.ny, self.w.nx) if self.w.dim == 3 else (self.w.ny, self.ctx.nx_grid)
        out = tuple(e[k * G:(k + 1) * G].reshape(sh).copy() for k in range(self.w.dim))
        if self.ctx.walls:
            # the physical nodes 0..nx of the odd extension
            out = tuple(a[:, :self.w.nx + 1].copy() for a in out)
        return out

    def state(self):
        """Host copy: dict of arrays in the device order (positions in FP64
        for the FP64 path; cell/offset for the mixed path)."""
        d = self.p.download()
        if self.mixed:
            u = W.unpack_cell(d["cell"], self.w.dim)
            d["ix"], d["iy"] = u[0], u[1]
            if self.w.dim == 3:
                d["iz"] = u[2]
        return d


class BatchSimulation:
    """Replicas of 1D1V plasmas (e.g. the Landau-damping ensemble) advanced
    together by the batched path. Inputs are the seeded replica workloads."""

    def __init__(self, replicas, dt=0.1, chunk=0, states=None, device="cuda"):
        self.replicas = list(replicas)
        ws = [W.replica_workload(r) for r in self.replicas]
        self.workloads = ws
        reps = [(w.nx, w.n_particles, w.Lx) for w in ws]
        cells, offs, vels = [], [], []
        for i, w in enumerate(ws):
            if states is not None:
                x, vx = states[i]
            else:
                x, _, vx, _, _ = W.sample(w)
            c, o = W.to_cell_offset(x, w.dx, w.nx)
            cells.append(c)
            offs.append(o)
            vels.append(vx)
        packed = (np.concatenate(cells), np.concatenate(offs), np.concatenate(vels))
        self.tune_ms = None
        if chunk == "auto":
            b = Batch(reps, dt, chunk=0, device=device)
            b.upload(*packed)
            chunk, self.tune_ms = b.autotune_chunk()
            del b
        self.chunk = int(chunk)
        self.batch = Batch(reps, dt, chunk=self.chunk, device=device)
        self.batch.upload(*packed)

    def initialise(self):
        self.batch.init()

    def run(self, nsteps, diag=True, use_graph=True, rho=None):
        d = None
        if diag:
            d = self.batch.torch.zeros(nsteps * self.batch.nrep * 4, dtype=self.batch.torch.float64,
                                       device=self.batch.device)
        self.batch.step(nsteps, d, rho=rho, use_graph=use_graph)
        return d

    def replica_field(self, r):
        g0, g1 = self.batch.grid_off[r], self.batch.grid_off[r + 1]
        return self.batch.E[g0:g1].cpu().numpy()

    def replica_state(self, r):
        p0, p1 = self.batch.part_off[r], self.batch.part_off[r + 1]
        return (self.batch.cell[p0:p1].cpu().numpy(), self.batch.ox[p0:p1].cpu().numpy(),
                self.batch.vx[p0:p1].cpu().numpy())
