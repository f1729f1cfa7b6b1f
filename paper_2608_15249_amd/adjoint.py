"""Differentiable PIC run: torch.autograd.Function over apic_adjoint_forward /
apic_step_adjoint.

``FieldEnergyRun`` owns one libapic context, its particle buffers, the
checkpoint buffer and the adjoint workspace for a fixed plasma shape, step
count and checkpoint stride. ``field_energy(run, x, y, vx, vy, vz, z)``
returns W_E(T) of the run started from the given initial state (FP64 device
tensors in physical units, any particle order; z only in 3D) and propagates
gradients to every input. Every step of the forward run and of the reverse sweep runs in
libapic's kernels; this module only marshals arguments and applies the
upstream gradient factor (chain rule) to the library's output.
"""
from __future__ import annotations

from typing import Optional

from .apic import Context, Particles


class FieldEnergyRun:
    def __init__(self, *, dim, vdim, nx, ny, lx, ly, dt, n, nsteps, stride=20, bz=0.0, qm=-1.0, rho_ion=1.0,
                 precision="mixed", tile=(0, 0), device="cuda", pusher="boris", c_light=0.0, nz=1, lz=1.0):
        import torch
        self.torch = torch
        self.ctx = Context(dim=dim, vdim=vdim, nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz, dt=dt, n=n, qm=qm,
                           rho_ion=rho_ion, bz=bz, precision=precision, tile=tile, device=device, pusher=pusher,
                           c_light=c_light)
        self.parts = Particles(self.ctx)
        self.nsteps, self.stride = int(nsteps), int(stride)
        ck, ws = self.ctx.adjoint_sizes(self.nsteps, self.stride)
        dev = self.ctx.device
        self.ckpt = torch.empty(max(ck, 256), dtype=torch.uint8, device=dev)
        self.ws = torch.empty(max(ws, 256), dtype=torch.uint8, device=dev)
        self.W = torch.zeros(1, dtype=torch.float64, device=dev)
        self.dim, self.vdim, self.n = dim, vdim, int(n)
        # forward() runs so far: the checkpoints belong to the latest one only
        self.generation = 0

    @classmethod
    def for_workload(cls, w, stride=20, precision="mixed", nsteps: Optional[int] = None, **kw):
        if w.dim == 3:
            kw = dict(nz=w.nz, lz=w.Lz, **kw)
        return cls(dim=w.dim, vdim=w.vdim, nx=w.nx, ny=w.ny, lx=w.Lx, ly=w.Ly, dt=w.dt, n=w.n_particles,
                   nsteps=w.steps if nsteps is None else nsteps, stride=stride, bz=w.bz, precision=precision, **kw)

    def forward(self, x, y, vx, vy=None, vz=None, E_out=None, z=None):
        """W_E(T) (a 1-element FP64 device tensor) from the FP64 initial state."""
        self.ctx.import_state(self.parts, x, y, vx, vy, vz, z=z)
        self.ctx.adjoint_forward(self.parts, self.nsteps, self.stride, self.ckpt, self.ws, W=self.W, E_out=E_out)
        self.generation += 1
        return self.W.clone()

    def backward(self, seed: float = 1.0, dx_ddelta0=None, dy_ddelta0=None):
        """seed * dW/d(x, y, vx, vy, vz, z) after forward(); None for absent
        components. With dx_ddelta0 (and dy_ddelta0 from 2D on), the
        derivative of each initial position with respect to the mode
        amplitude delta0, a seventh entry holds seed * dW/d delta0 (a
        1-element device tensor)."""
        t = self.torch
        mk = lambda on: t.empty(self.n, dtype=t.float64, device=self.ctx.device) if on else None
        out = [mk(True), mk(self.dim >= 2), mk(True), mk(self.vdim >= 2), mk(self.vdim >= 3), mk(self.dim == 3)]
        gd = t.zeros(1, dtype=t.float64, device=self.ctx.device) if dx_ddelta0 is not None else None
        self.ctx.step_adjoint(self.ckpt, self.nsteps, self.stride, self.ws, out[0], out[1], out[2], out[3], out[4],
                              seed=seed, dx_ddelta0=dx_ddelta0, dy_ddelta0=dy_ddelta0, grad_delta0=gd,
                              lam_z=out[5])
        return out + [gd] if gd is not None else out

    def sync(self):
        self.ctx.sync()


def _function():
    import torch

    class FieldEnergy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, run: FieldEnergyRun, x, y, vx, vy, vz, z):
            ctx.run = run
            ctx.inputs = (x, y, vx, vy, vz, z)
            W = run.forward(x, y, vx, vy, vz, z=z)
            ctx.generation = run.generation
            return W

        @staticmethod
        def backward(ctx, gW):
            run = ctx.run
            if run.generation != ctx.generation:
                # a later forward of the same run overwrote the checkpoints:
                # recompute them from this graph's own inputs
                with torch.no_grad():
                    a = [None if a is None else a.detach() for a in ctx.inputs]
                    run.forward(*a[:5], z=a[5])
            grads = run.backward(1.0)
            return (None,) + tuple(None if g is None else g * gW for g in grads)

    return FieldEnergy


_FE = None


def field_energy(run: FieldEnergyRun, x, y, vx, vy=None, vz=None, z=None):
    """Differentiable W_E(T) of `run` from the initial state (torch autograd)."""
    global _FE
    if _FE is None:
        _FE = _function()
    return _FE.apply(run, x, y, vx, vy, vz, z)
