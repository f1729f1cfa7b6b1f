// Device helpers of the electromagnetic 2D3V step on a periodic Yee grid:
// the six-component field tile and its staggered gather, the Boris advance in
// a general magnetic field, and the charge-conserving current deposit of
// Esirkepov (2001) for the linear shape into an LDS tile. R is the push
// precision (double, or float for the mixed path: field tile, gather, Boris
// and the current weights in binary32); the current accumulates in FP64.
//
// Yee staggering: element [j][i] of each component sits at
//   Ex, Jx: ((i+1/2) dx, j dy)      Bx: (i dx, (j+1/2) dy)
//   Ey, Jy: (i dx, (j+1/2) dy)      By: ((i+1/2) dx, j dy)
//   Ez, Jz: (i dx, j dy)            Bz: ((i+1/2) dx, (j+1/2) dy)
// Fields are [6][ny][nx] (Ex, Ey, Ez, Bx, By, Bz), currents [3][ny][nx].
#pragma once

#include "apic_device.h"

namespace apic {
namespace {

// Field tile: the six components on nodes [x0-1, x0+T] x [y0-1, y0+T]
// (fw x fh = (T+2)^2 entries each, periodic), component-major, converted to
// the push precision R on the way into LDS.
template <typename R>
__device__ void load_f_tile(R *sF, const double *F, const Geo &g, int x0, int y0, int fw, int fh) {
    const int64_t G = (int64_t)g.nx * g.ny;
    const int tot = fw * fh;
    for (int t = threadIdx.x; t < tot; t += blockDim.x) {
        const int lx = t % fw, ly = t / fw;
        int gx = x0 - 1 + lx;
        gx = gx < 0 ? gx + g.nx : (gx >= g.nx ? gx - g.nx : gx);
        int gy = y0 - 1 + ly;
        gy = gy < 0 ? gy + g.ny : (gy >= g.ny ? gy - g.ny : gy);
        const int64_t gi = (int64_t)gy * g.nx + gx;
#pragma unroll
        for (int c = 0; c < 6; ++c) sF[c * tot + t] = (R)F[c * G + gi];
    }
}

// Linear interpolation of one staggered component from the tile: (bx, by)
// the tile index of the lower node, (fx, fy) the fractions.
template <typename R>
__device__ __forceinline__ R lerp_tile(const R *f, int fw, int bx, int by, R fx, R fy) {
    const int a = by * fw + bx;
    return (R(1) - fx) * (R(1) - fy) * f[a] + fx * (R(1) - fy) * f[a + 1] + (R(1) - fx) * fy * f[a + fw] +
           fx * fy * f[a + fw + 1];
}

// E and B at a particle in local cell (lx, ly) of the tile at fractions
// (fx, fy). A component offset by half a cell along an axis uses the lower
// node and fraction of the coordinate shifted back by half a cell.
template <typename R>
__device__ __forceinline__ void gather_em(const R *sF, int fw, int tot, int lx, int ly, R fx, R fy, R e[3],
                                          R b[3]) {
    const int ax0 = lx + 1, ay0 = ly + 1;                 // unshifted lattice
    const bool hx = fx >= R(0.5), hy = fy >= R(0.5);
    const int ax1 = hx ? lx + 1 : lx, ay1 = hy ? ly + 1 : ly;  // half-shifted lattice
    const R fx1 = hx ? fx - R(0.5) : fx + R(0.5), fy1 = hy ? fy - R(0.5) : fy + R(0.5);
    e[0] = lerp_tile(sF + 0 * tot, fw, ax1, ay0, fx1, fy);
    e[1] = lerp_tile(sF + 1 * tot, fw, ax0, ay1, fx, fy1);
    e[2] = lerp_tile(sF + 2 * tot, fw, ax0, ay0, fx, fy);
    b[0] = lerp_tile(sF + 3 * tot, fw, ax0, ay1, fx, fy1);
    b[1] = lerp_tile(sF + 4 * tot, fw, ax1, ay0, fx1, fy);
    b[2] = lerp_tile(sF + 5 * tot, fw, ax1, ay1, fx1, fy1);
}

// Boris (1970) in a general B: a = (q/m) dt_eff / 2, t = a B,
// s = 2 t / (1 + |t|^2), v- = v + a E, v' = v- + v- x t, v+ = v- + v' x s,
// v = v+ + a E.
template <typename R>
__device__ __forceinline__ void boris3(R &vx, R &vy, R &vz, const R e[3], const R b[3], R a) {
    const R tx = a * b[0], ty = a * b[1], tz = a * b[2];
    const R t2 = tx * tx + ty * ty + tz * tz;
    const R sx = R(2) * tx / (R(1) + t2), sy = R(2) * ty / (R(1) + t2), sz = R(2) * tz / (R(1) + t2);
    const R mx = vx + a * e[0], my = vy + a * e[1], mz = vz + a * e[2];
    const R qx = mx + (my * tz - mz * ty);
    const R qy = my + (mz * tx - mx * tz);
    const R qz = mz + (mx * ty - my * tx);
    const R px = mx + (qy * sz - qz * sy);
    const R py = my + (qz * sx - qx * sz);
    const R pz = mz + (qx * sy - qy * sx);
    vx = px + a * e[0];
    vy = py + a * e[1];
    vz = pz + a * e[2];
}

// Higuera & Cary (2017) in a general field, state u = gamma v (a = (q/m)
// dt_eff / 2, ic2 = 1/c^2): u- = u + a E, tau = a B,
// sigma = 1 + |u-|^2/c^2 - |tau|^2,
// gamma+ = sqrt((sigma + sqrt(sigma^2 + 4 (|tau|^2 + (u- . tau)^2/c^2))) / 2),
// t = tau / gamma+, s = 1 / (1 + |t|^2), u+ = s (u- + (u- . t) t + u- x t),
// u = u+ + a E + u+ x t.
template <typename R>
__device__ __forceinline__ void hc3(R &ux, R &uy, R &uz, const R e[3], const R b[3], R a, R ic2) {
    const R tx = a * b[0], ty = a * b[1], tz = a * b[2];
    const R mx = ux + a * e[0], my = uy + a * e[1], mz = uz + a * e[2];
    const R tau2 = tx * tx + ty * ty + tz * tz;
    const R sig = R(1) + (mx * mx + my * my + mz * mz) * ic2 - tau2;
    const R us = mx * tx + my * ty + mz * tz;
    const R gp = sqrt(R(0.5) * (sig + sqrt(sig * sig + R(4) * (tau2 + us * us * ic2))));
    const R wx = tx / gp, wy = ty / gp, wz = tz / gp;
    const R s = R(1) / (R(1) + (wx * wx + wy * wy + wz * wz));
    const R mw = mx * wx + my * wy + mz * wz;
    const R px = s * (mx + mw * wx + (my * wz - mz * wy));
    const R py = s * (my + mw * wy + (mz * wx - mx * wz));
    const R pz = s * (mz + mw * wz + (mx * wy - my * wx));
    ux = px + a * e[0] + (py * wz - pz * wy);
    uy = py + a * e[1] + (pz * wx - px * wz);
    uz = pz + a * e[2] + (px * wy - py * wx);
}

// Hat weights of one axis on a three-node window starting at node s0 of the
// old cell (s0 = min(0, c1)): S0 of the old fraction f0, S1 after a move by d
// cells (new cell c1 = floor(f0 + d) in {-1, 0, 1}). False when |d| >= 1.
// nn: the window nodes that carry weight (2 without a cell crossing, else 3).
// With R = float, g1 = f0 + d is the same binary32 sum the mixed move forms,
// so S1 is the hat of the particle's new offset.
template <typename R>
__device__ __forceinline__ bool hat3(R f0, R d, R S0[3], R DS[3], int &s0, int &nn) {
    const bool ok = fabs(d) < R(1);
    const R g1 = f0 + (ok ? d : R(0));
    const R fl = floor(g1);
    const int c1 = (int)fl;
    const R f1 = g1 - fl;
    s0 = c1 < 0 ? -1 : 0;
    nn = c1 == 0 ? 2 : 3;
    R S1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int node = s0 + k;   // relative to the old cell
        S0[k] = node == 0 ? R(1) - f0 : (node == 1 ? f0 : R(0));
        S1[k] = node == c1 ? R(1) - f1 : (node == c1 + 1 ? f1 : R(0));
        DS[k] = S1[k] - S0[k];
    }
    return ok;
}

// Esirkepov current of one particle into the LDS tile sJ (three components of
// jw x jh entries, node (x0-1, y0-1) at index 0). (lx, ly): old local cell in
// [0, T); (fx, fy): old fractions; (dx, dy): displacement in cells; cj:
// (-Q/(dy dt), -Q/(dx dt), Q vz/(dx dy)). Returns false (and deposits
// nothing) for a displacement of a cell or more.
// Only the part of the window that carries current is added: without a cell
// crossing along x the second half-node of Jx is the sum of the hat changes
// over the old cell's two nodes, zero in exact arithmetic (its rounding
// residue is not deposited), and the third node row/column has no weight;
// a particle that stays in its cell adds 8 entries instead of 21.
template <typename R>
__device__ __forceinline__ bool esirkepov_lds(double *sJ, int jw, int jtot, int lx, int ly, R fx, R fy, R dx, R dy,
                                              double cx, double cy, double cz) {
    R S0x[3], DSx[3], S0y[3], DSy[3];
    int sx, sy, nx, ny;
    const bool okx = hat3(fx, dx, S0x, DSx, sx, nx);
    const bool oky = hat3(fy, dy, S0y, DSy, sy, ny);
    const bool ok = okx && oky;
    if (!ok) return false;
    const int bx = lx + 1 + sx, by = ly + 1 + sy;   // tile index of window node (0, 0)
    double *jx = sJ, *jy = sJ + jtot, *jz = sJ + 2 * jtot;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const R wy = S0y[l] + R(0.5) * DSy[l];
        R run = R(0);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            run += DSx[k] * wy;
            if (l < ny && k < nx - 1) atomicAdd(&jx[(by + l) * jw + bx + k], cx * (double)run);
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const R wx = S0x[k] + R(0.5) * DSx[k];
        R run = R(0);
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            run += DSy[l] * wx;
            if (k < nx && l < ny - 1) atomicAdd(&jy[(by + l) * jw + bx + k], cy * (double)run);
        }
    }
#pragma unroll
    for (int l = 0; l < 3; ++l) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const R wz = S0x[k] * S0y[l] + R(0.5) * DSx[k] * S0y[l] + R(0.5) * S0x[k] * DSy[l] +
                         DSx[k] * DSy[l] / R(3);
            if (k < nx && l < ny) atomicAdd(&jz[(by + l) * jw + bx + k], cz * (double)wz);
        }
    }
    return true;
}

// Add the current tile to the global J (one atomic per non-zero entry).
__device__ void flush_j(double *J, const double *sJ, const Geo &g, int x0, int y0, int jw, int jh) {
    const int64_t G = (int64_t)g.nx * g.ny;
    const int tot = jw * jh;
    for (int t = threadIdx.x; t < 3 * tot; t += blockDim.x) {
        const double v = sJ[t];
        if (v == 0.0) continue;
        const int c = t / tot, r = t % tot;
        int gx = x0 - 1 + r % jw;
        gx = gx < 0 ? gx + g.nx : (gx >= g.nx ? gx - g.nx : gx);
        int gy = y0 - 1 + r / jw;
        gy = gy < 0 ? gy + g.ny : (gy >= g.ny ? gy - g.ny : gy);
        atomicAdd(&J[c * G + (int64_t)gy * g.nx + gx], v);
    }
}

}  // namespace
}  // namespace apic
