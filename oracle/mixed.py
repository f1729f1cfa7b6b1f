"""Binary32 reading of the particle push for the mixed-precision state.

TEST INFRASTRUCTURE ONLY.

The mixed representation (not in the paper; it is the fixed-point/binary32
form of the same CIC-Boris-leapfrog step) holds a particle as an integer cell
(ix[, iy[, iz]]), a binary32 in-cell offset o in [0,1) (cell units) and binary32
velocities. The push reads the grid field rounded to binary32. Every
operation below is one IEEE-754 binary32 operation (numpy float32, no fused
multiply-add), in the order of the textbook formulas of the FP64 oracle:

  gather : w00 = (1-fx)(1-fy), w10 = fx(1-fy), w01 = (1-fx)fy, w11 = fx fy,
           E_p = ((w00 E00 + w10 E10) + w01 E01) + w11 E11   (1D: (1-f)E0 + f E1);
           3D: w_abc = (wx_a wy_b) wz_c, the eight terms added left to right
           with a (x) fastest, then b (y), then c (z)
  Boris  : a = (q/m) dt/2, t = a bz, s = 2t/(1+t^2) computed in FP64 and
           rounded to binary32; v- = v + aE; v' = v- + v- x t;
           v+ = v- + v' x s; v = v+ + aE (in 3D vz takes the two kicks of Ez)
  Higuera-Cary (pusher "hc", state u = gamma v, ic2 = fl32(1/c^2)):
           m = u + aE; g2 = 1 + ((mx mx + my my) + mz mz) ic2;
           sig = g2 - tau tau; us = mz tau;
           gp = sqrt(0.5 (sig + sqrt(sig sig + 4 (tau tau + (us us) ic2))));
           t = tau / gp; s = 1 / (1 + t t);
           p = s (mx + my t, my - mx t, mz + (mz t) t);
           u = (px + aEx + py t, py + aEy - px t, pz + aEz); the move uses
           v = u r with r = 1 / sqrt(1 + ((ux ux + uy uy) + uz uz) ic2)
           (one binary32 division for r, then three products)
  move   : o' = o + v * fl32(dt/dx); k = floor(o'); o' = o' - k;
           if o' >= 1 then o' = o' - 1, k = k + 1; cell = (cell + k) mod n.
The deposit of the result is oracle.deposit_quantised (exact integers).
"""
from __future__ import annotations

import numpy as np

f32 = np.float32


def _gather3(ix, iy, iz, fx, fy, fz, E32, nx, ny, nz):
    one = f32(1.0)
    i = (ix, (ix + 1) % nx)
    j = (iy, (iy + 1) % ny)
    k = (iz, (iz + 1) % nz)
    wx = (one - fx, fx)
    wy = (one - fy, fy)
    wz = (one - fz, fz)
    out = []
    for E in E32:
        acc = None
        for c in range(2):
            for b in range(2):
                for a in range(2):
                    w = (wx[a] * wy[b]) * wz[c]
                    term = w * E[k[c], j[b], i[a]]
                    acc = term if acc is None else (acc + term).astype(f32)
        out.append(acc.astype(f32))
    return out


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


def push(st: dict, E32, *, dim, vdim, nx, ny, dx, dy, qm, dt, bz, dt_scale=1.0, move=True,
         nz=1, dz=1.0, pusher="boris", c=float("inf")) -> dict:
    """One binary32 gather + Boris or Higuera-Cary (+ move) of a mixed state.

    st: dict with ix, iy, iz (int32 or None), ox, oy, oz, vx, vy, vz (float32
    or None). E32: tuple of float32 node fields shaped like the grid. Returns
    a new dict."""
    ix = st["ix"].astype(np.int64)
    iy = st["iy"].astype(np.int64) if dim >= 2 else None
    iz = st["iz"].astype(np.int64) if dim == 3 else None
    fx = st["ox"].astype(f32)
    fy = st["oy"].astype(f32) if dim >= 2 else None
    fz = st["oz"].astype(f32) if dim == 3 else None
    vx = st["vx"].astype(f32).copy()
    vy = st["vy"].astype(f32).copy() if vdim >= 2 else None
    vz = st["vz"].astype(f32).copy() if vdim >= 3 else None
    ez = None
    if dim == 3:
        ex, ey, ez = _gather3(ix, iy, iz, fx, fy, fz, E32, nx, ny, nz)
    else:
        ex, ey = _gather(ix, iy, fx, fy, E32, nx, ny, dim)
    a, t, s = boris_coeffs(qm, dt * dt_scale, bz)
    ic2 = f32(1.0 / (c * c))
    if pusher == "hc":
        ezz = ez if ez is not None else np.zeros_like(ex)
        mx = (vx + a * ex).astype(f32)
        my = (vy + a * ey).astype(f32)
        mz = (vz + a * ezz).astype(f32)
        g2 = f32(1.0) + (mx * mx + my * my + mz * mz) * ic2
        sig = g2 - t * t
        us = mz * t
        gp = np.sqrt(f32(0.5) * (sig + np.sqrt(sig * sig + f32(4.0) * (t * t + (us * us) * ic2))))
        tt = (t / gp).astype(f32)
        ss = (f32(1.0) / (f32(1.0) + tt * tt)).astype(f32)
        px = ss * (mx + my * tt)
        py = ss * (my - mx * tt)
        pz = ss * (mz + (mz * tt) * tt)
        vx = (px + a * ex + py * tt).astype(f32)
        vy = (py + a * ey - px * tt).astype(f32)
        vz = (pz + a * ezz).astype(f32)
    else:
        if ez is not None:
            mz = vz + a * ez
            vz = (mz + a * ez).astype(f32)
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

        wx, wy, wz = vx, vy, vz
        if pusher == "hc":
            g = np.sqrt(f32(1.0) + (vx * vx + vy * vy + vz * vz) * ic2).astype(f32)
            r = (f32(1.0) / g).astype(f32)
            wx, wy, wz = (vx * r).astype(f32), (vy * r).astype(f32), (vz * r).astype(f32)
        out["ix"], out["ox"] = mv(ix, fx, wx, dx, nx)
        if dim >= 2:
            out["iy"], out["oy"] = mv(iy, fy, wy, dy, ny)
        if dim == 3:
            out["iz"], out["oz"] = mv(iz, fz, wz, dz, nz)
    return out


def positions(st: dict, dx: float, dy: float, dim: int, dz: float = 1.0):
    """FP64 positions (ix + ox) dx of a mixed state (for comparisons); a
    third array (z) is returned in 3D."""
    x = (st["ix"].astype(np.float64) + st["ox"].astype(np.float64)) * dx
    y = None
    if dim >= 2:
        y = (st["iy"].astype(np.float64) + st["oy"].astype(np.float64)) * dy
    if dim == 3:
        z = (st["iz"].astype(np.float64) + st["oz"].astype(np.float64)) * dz
        return x, y, z
    return x, y
