"""Seeded synthetic initial plasmas shared by the HIP path, the oracle and tests.

This module holds no arithmetic of the PIC method itself: it only draws
particle positions and velocities (numpy PCG64 streams), applies the mode
seeding of the paper's two-stream example ("Example setup and implementation":
each particle is displaced by xi = delta0 k/|k|^2 sin(k.x), which gives a
first-order density perturbation -delta0 cos(k.x)), and converts positions to
the (cell index, binary32 in-cell offset) representation used by the
mixed-precision path. Every result is FP64 numpy unless stated.

Workloads (lengths in Debye lengths of the stated v_th; omega_pe = 1):
  two_stream_1d    1D1V, L = 4 pi (k = 0.5), 64 cells, 16,384 electrons in two
                   beams at +-1 with Gaussian spread 0.01, delta0 = 1e-3 at k = 0.5,
                   dt = 0.1, 200 steps.
  thermal_2d       2D2V, 512 x 512 cells, dx = 1, 64 per cell (16,777,216),
                   Maxwellian v_th = 1, uniform positions, dt = 0.1, 500 steps.
  magnetized_2d3v  2D3V, 1024 x 1024 cells, dx = 1, 32 per cell (33,554,432),
                   Maxwellian v_th = 1 (3 components), delta0 = 0.01 at
                   k = (2 pi/64, 0), B_z = 2 (omega_c = 2), dt = 0.05, 300 steps.
  landau_batch     256 1D1V replicas, L = 4 pi, Nx and N log-uniform in [32, 512]
                   and [1e4, 1e6], Maxwellian v_th = 1, delta0 ~ U[0.01, 0.05] at
                   k = 0.5, dt = 0.1, 400 steps.
  two_stream_2d    2D2V, 256 x 256 cells, L = 4 pi, 16 per cell (1,048,576),
                   beams v_x = +-1 with spread 0.05, delta0 = 1e-3 at mode (1, 0),
                   dt = 0.1, 200 steps (checkpoint stride 20 for the adjoint).
  paper_two_stream 2D3V, 64 x 64 cells, L = 64, 64 per cell per beam (524,288),
                   beams N(+-3, 1) in v_x, N(0, 1) in v_y, v_z, delta0 = 0.005 at
                   mode (2, 1), dt = 0.05, 800 steps.
  thermal_3d       3D3V, 128 x 128 x 128 cells, dx = 1, 8 per cell (16,777,216),
                   Maxwellian v_th = 1 (3 components), uniform positions,
                   dt = 0.1, 500 steps (the 3D Cartesian form of thermal_2d).
Beam and thermal positions are iid uniform (no quiet start).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

TWO_PI = 2.0 * np.pi


@dataclass
class Workload:
    name: str
    dim: int
    vdim: int
    nx: int
    ny: int
    Lx: float
    Ly: float
    n_particles: int
    dt: float
    steps: int
    bz: float = 0.0
    seed: int = 0
    # seeded mode (integer mode numbers) and displacement amplitude
    mode: tuple = (1, 0)
    delta0: float = 0.0
    # beams: list of (drift_x, spread); thermal plasmas use a single (0, v_th)
    beams: list = field(default_factory=lambda: [(0.0, 1.0)])
    spread_perp: Optional[float] = None  # spread of v_y, v_z (default: beam spread)
    nz: int = 1
    Lz: float = 1.0

    @property
    def dx(self):
        return self.Lx / self.nx

    @property
    def dy(self):
        return self.Ly / self.ny if self.dim >= 2 else 1.0

    @property
    def dz(self):
        return self.Lz / self.nz if self.dim == 3 else 1.0


def two_stream_1d(seed: int = 1000) -> Workload:
    return Workload("two_stream_1d", 1, 1, 64, 1, TWO_PI / 0.5, 1.0, 16384, 0.1, 200,
                    seed=seed, mode=(1, 0), delta0=1e-3, beams=[(1.0, 0.01), (-1.0, 0.01)])


def thermal_2d(seed: int = 1001, nx: int = 512, ppc: int = 64) -> Workload:
    return Workload("thermal_2d", 2, 2, nx, nx, float(nx), float(nx), nx * nx * ppc, 0.1, 500,
                    seed=seed, delta0=0.0, beams=[(0.0, 1.0)])


def magnetized_2d3v(seed: int = 1002, nx: int = 1024, ppc: int = 32) -> Workload:
    L = float(nx)
    mx = int(round(L / 64.0))
    return Workload("magnetized_2d3v", 2, 3, nx, nx, L, L, nx * nx * ppc, 0.05, 300, bz=2.0,
                    seed=seed, mode=(mx, 0), delta0=0.01, beams=[(0.0, 1.0)])


def two_stream_2d(seed: int = 1004, nx: int = 256, ppc: int = 16) -> Workload:
    L = TWO_PI / 0.5
    return Workload("two_stream_2d", 2, 2, nx, nx, L, L, nx * nx * ppc, 0.1, 200,
                    seed=seed, mode=(1, 0), delta0=1e-3, beams=[(1.0, 0.05), (-1.0, 0.05)])


def paper_two_stream(seed: int = 1005, nx: int = 64, ppc_per_beam: int = 64) -> Workload:
    return Workload("paper_two_stream", 2, 3, nx, nx, 64.0, 64.0, 2 * nx * nx * ppc_per_beam, 0.05, 800,
                    seed=seed, mode=(2, 1), delta0=0.005, beams=[(3.0, 1.0), (-3.0, 1.0)])


def thermal_3d(seed: int = 1006, nx: int = 128, ppc: int = 8, ny: Optional[int] = None,
               nz: Optional[int] = None) -> Workload:
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return Workload("thermal_3d", 3, 3, nx, ny, float(nx), float(ny), nx * ny * nz * ppc, 0.1, 500,
                    seed=seed, delta0=0.0, beams=[(0.0, 1.0)], nz=nz, Lz=float(nz))


@dataclass
class Replica:
    nx: int
    n_particles: int
    delta0: float
    seed: int
    L: float = TWO_PI / 0.5


def landau_batch(n_replicas: int = 256, seed: int = 1003, nx_range=(32, 512),
                 n_range=(1e4, 1e6)) -> List[Replica]:
    """Replica shapes of the batched Landau-damping ensemble (log-uniform)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for r in range(n_replicas):
        nx = int(round(np.exp(rng.uniform(np.log(nx_range[0]), np.log(nx_range[1])))))
        n = int(round(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1])))))
        d0 = float(rng.uniform(0.01, 0.05))
        out.append(Replica(nx, n, d0, 40000 + r))
    return out


def replica_workload(rep: Replica) -> Workload:
    return Workload("landau_replica", 1, 1, rep.nx, 1, rep.L, 1.0, rep.n_particles, 0.1, 400,
                    seed=rep.seed, mode=(1, 0), delta0=rep.delta0, beams=[(0.0, 1.0)])


def _wrap(a, L):
    a = np.mod(a, L)
    a[a >= L] -= L
    return a


def sample(w: Workload, n: Optional[int] = None):
    """Draw the FP64 initial state (x, y, vx, vy, vz); absent components are None.

    Beams split the particles evenly; each beam draws uniform positions and
    N(drift, spread^2) v_x, N(0, spread_perp^2) in the other components."""
    n = w.n_particles if n is None else n
    rng = np.random.Generator(np.random.PCG64(w.seed))
    nb = len(w.beams)
    counts = [n // nb + (1 if b < n % nb else 0) for b in range(nb)]
    xs, ys, vxs, vys, vzs = [], [], [], [], []
    for (drift, spread), c in zip(w.beams, counts):
        sp = spread if w.spread_perp is None else w.spread_perp
        xs.append(rng.uniform(0.0, w.Lx, c))
        if w.dim == 2:
            ys.append(rng.uniform(0.0, w.Ly, c))
        vxs.append(rng.normal(drift, spread, c))
        if w.vdim >= 2:
            vys.append(rng.normal(0.0, sp, c))
        if w.vdim >= 3:
            vzs.append(rng.normal(0.0, sp, c))
    x = np.concatenate(xs)
    y = np.concatenate(ys) if w.dim == 2 else None
    vx = np.concatenate(vxs)
    vy = np.concatenate(vys) if w.vdim >= 2 else None
    vz = np.concatenate(vzs) if w.vdim >= 3 else None
    if w.delta0 != 0.0:
        kx = TWO_PI * w.mode[0] / w.Lx
        ky = TWO_PI * w.mode[1] / w.Ly if w.dim == 2 else 0.0
        k2 = kx * kx + ky * ky
        phase = kx * x + (ky * y if w.dim == 2 else 0.0)
        sn = np.sin(phase)
        x = x + w.delta0 * kx / k2 * sn
        if w.dim == 2:
            y = y + w.delta0 * ky / k2 * sn
    x = _wrap(x, w.Lx)
    if y is not None:
        y = _wrap(y, w.Ly)
    return x, y, vx, vy, vz


def sample3(w: Workload, n: Optional[int] = None):
    """3D initial state (x, y, z, vx, vy, vz), FP64: per beam uniform
    positions in the box, N(drift, spread^2) v_x and N(0, spread_perp^2) v_y,
    v_z; the seeded mode (mode[0], mode[1], 0) displaces x and y as in
    sample()."""
    assert w.dim == 3 and w.vdim == 3
    n = w.n_particles if n is None else n
    rng = np.random.Generator(np.random.PCG64(w.seed))
    nb = len(w.beams)
    counts = [n // nb + (1 if b < n % nb else 0) for b in range(nb)]
    cols = [[] for _ in range(6)]
    for (drift, spread), c in zip(w.beams, counts):
        sp = spread if w.spread_perp is None else w.spread_perp
        cols[0].append(rng.uniform(0.0, w.Lx, c))
        cols[1].append(rng.uniform(0.0, w.Ly, c))
        cols[2].append(rng.uniform(0.0, w.Lz, c))
        cols[3].append(rng.normal(drift, spread, c))
        cols[4].append(rng.normal(0.0, sp, c))
        cols[5].append(rng.normal(0.0, sp, c))
    x, y, z, vx, vy, vz = (np.concatenate(c) for c in cols)
    if w.delta0 != 0.0:
        kx = TWO_PI * w.mode[0] / w.Lx
        ky = TWO_PI * w.mode[1] / w.Ly
        k2 = kx * kx + ky * ky
        sn = np.sin(kx * x + ky * y)
        x = x + w.delta0 * kx / k2 * sn
        y = y + w.delta0 * ky / k2 * sn
    return _wrap(x, w.Lx), _wrap(y, w.Ly), _wrap(z, w.Lz), vx, vy, vz


def to_cell_offset(x: np.ndarray, d: float, n: int):
    """Position -> (int32 cell, float32 offset in [0,1)) on a periodic axis.

    cell = floor(x/d); offset = binary32(x/d - cell); an offset that rounds to
    1.0 moves to the next cell with offset 0."""
    g = x / d
    c = np.floor(g).astype(np.int64)
    o = (g - c).astype(np.float32)
    up = o >= np.float32(1.0)
    o[up] = np.float32(0.0)
    c[up] += 1
    c = np.mod(c, n).astype(np.int32)
    return c, o


def pack_cell(ix: np.ndarray, iy: Optional[np.ndarray], iz: Optional[np.ndarray] = None) -> np.ndarray:
    """Mixed-path cell word, int32: ix (1D), iy << 16 | ix (2D),
    iz << 20 | iy << 10 | ix (3D, 10 bits per axis)."""
    if iy is None:
        return ix.astype(np.int32)
    if iz is not None:
        return ((iz.astype(np.int64) << 20) | (iy.astype(np.int64) << 10) | ix.astype(np.int64)).astype(np.int32)
    return ((iy.astype(np.int64) << 16) | ix.astype(np.int64)).astype(np.int32)


def unpack_cell(c: np.ndarray, dim: int):
    """Inverse of pack_cell: (ix, iy) for dim <= 2 (iy None in 1D), (ix, iy, iz)
    in 3D."""
    c = np.asarray(c).astype(np.int64)
    if dim == 1:
        return c.astype(np.int32), None
    if dim == 3:
        return (c & 0x3FF).astype(np.int32), ((c >> 10) & 0x3FF).astype(np.int32), (c >> 20).astype(np.int32)
    return (c & 0xFFFF).astype(np.int32), (c >> 16).astype(np.int32)
