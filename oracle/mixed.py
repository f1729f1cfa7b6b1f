"""Binary32 reading of the particle push for the mixed-precision state.

TEST INFRASTRUCTURE ONLY.

The mixed representation (not in the paper; it is the fixed-point/binary32
form of the same CIC-Boris-leapfrog step) holds a particle as an integer cell
(ix[, iy]), a binary32 in-cell offset o in [0,1) (cell units) and binary32
velocities. The push reads the grid field rounded to binary32. Every
operation below is one IEEE-754 binary32 operation (numpy float32, no fused
multiply-add), in the order of the textbook formulas of the FP64 oracle:

  gather : w00 = (1-fx)(1-fy), w10 = fx(1-fy), w01 = (1-fx)fy, w11 = fx fy,
           E_p = ((w00 E00 + w10 E10) + w01 E01) + w11 E11   (1D: (1-f)E0 + f E1)
  Boris  : a = (q/m) dt/2, t = a bz, s = 2t/(1+t^2) computed in FP64 and
           rounded to binary32; v- = v + aE; v' = v- + v- x t;
           v+ = v- + v' x s; v = v+ + aE
  move   : o' = o + v * fl32(dt/dx); k = floor(o'); o' = o' - k;
           if o' >= 1 then o' = o' - 1, k = k + 1; cell = (cell + k) mod n.
The deposit of the result is oracle.deposit_quantised (exact integers).
"""
from __future__ import annotations

import numpy as np

f32 = np.float32


def _gather(ix, iy, fx, fy, E32, nx, ny, dim):
    one = f32(1.0)
    if dim == 1:
        e = E32[0]
        ip = (ix + 1) % nx
        return ((one - fx) * e[ix] + fx * e[ip]).astype(f32), None
    Ex, Ey = E32[0], E32[1]
    ip = (ix + 1) % nx
    jp = (iy + 1) % ny
    w00 = (one - fx) * (one - fy)
    w10 = fx * (one - fy)
    w01 = (one - fx) * fy
    w11 = fx * fy
    ex = ((w00 * Ex[iy, ix] + w10 * Ex[iy, ip]) + w01 * Ex[jp, ix]) + w11 * Ex[jp, ip]
    ey = ((w00 * Ey[iy, ix] + w10 * Ey[iy, ip]) + w01 * Ey[jp, ix]) + w11 * Ey[jp, ip]
    return ex.astype(f32), ey.astype(f32)


def boris_coeffs(qm: float, dt: float, bz: float):
    a = qm * dt * 0.5
    t = a * bz
    s = 2.0 * t / (1.0 + t * t)
    return f32(a), f32(t), f32(s)


def push(st: dict, E32, *, dim, vdim, nx, ny, dx, dy, qm, dt, bz, dt_scale=1.0, move=True) -> dict:
    """One binary32 gather + Boris (+ move) of a mixed state.

    st: dict with ix, iy (int32 or None), ox, oy, vx, vy, vz (float32 or None).
    E32: tuple of float32 node fields shaped like the grid. Returns a new dict."""
    ix = st["ix"].astype(np.int64)
    iy = st["iy"].astype(np.int64) if dim == 2 else None
    fx = st["ox"].astype(f32)
    fy = st["oy"].astype(f32) if dim == 2 else None
    vx = st["vx"].astype(f32).copy()
    vy = st["vy"].astype(f32).copy() if vdim >= 2 else None
    vz = st["vz"].astype(f32).copy() if vdim >= 3 else None
    ex, ey = _gather(ix, iy, fx, fy, E32, nx, ny, dim)
    a, t, s = boris_coeffs(qm, dt * dt_scale, bz)
    if vdim == 1:
        m1 = vx + a * ex
        vx = (m1 + a * ex).astype(f32)
    else:
        mx = vx + a * ex
        my = vy + a * ey
        px = mx + my * t
        py = my - mx * t
        qx = mx + py * s
        qy = my - px * s
        vx = (qx + a * ex).astype(f32)
        vy = (qy + a * ey).astype(f32)
    out = dict(st)
    out["vx"], out["vy"], out["vz"] = vx, vy, vz
    if move:
        def mv(c, o, v, d, n):
            o2 = o + v * f32(dt / d)
            k = np.floor(o2)
            o2 = (o2 - k).astype(f32)
            k = k.astype(np.int64)
            up = o2 >= f32(1.0)
            o2[up] = o2[up] - f32(1.0)
            k[up] += 1
            return np.mod(c + k, n).astype(np.int32), o2.astype(f32)

        out["ix"], out["ox"] = mv(ix, fx, vx, dx, nx)
        if dim == 2:
            out["iy"], out["oy"] = mv(iy, fy, vy, dy, ny)
    return out


def positions(st: dict, dx: float, dy: float, dim: int):
    """FP64 positions (ix + ox) dx of a mixed state (for comparisons)."""
    x = (st["ix"].astype(np.float64) + st["ox"].astype(np.float64)) * dx
    y = None
    if dim == 2:
        y = (st["iy"].astype(np.float64) + st["oy"].astype(np.float64)) * dy
    return x, y
