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
// the tile index of the lower node, (fx, fy) the fractions; along x on the
// two node rows, then along y, each as one fused multiply-add.
template <typename R>
__device__ __forceinline__ R lerp_tile(const R *f, int fw, int bx, int by, R fx, R fy) {
    const int a = by * fw + bx;
    const R lo = fma(fx, f[a + 1] - f[a], f[a]);
    const R hi = fma(fx, f[a + fw + 1] - f[a + fw], f[a + fw]);
    return fma(fy, hi - lo, lo);
}

// 1 / x in the push precision: the hardware reciprocal on the mixed path
// (within 1 ulp of binary32), a correctly rounded division in FP64.
template <typename R> __device__ __forceinline__ R recip(R x);
template <> __device__ __forceinline__ float recip<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double recip<double>(double x) { return 1.0 / x; }

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
    const R k = R(2) * recip<R>(R(1) + t2);
    const R sx = k * tx, sy = k * ty, sz = k * tz;
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
    const R ig = recip<R>(gp);
    const R wx = tx * ig, wy = ty * ig, wz = tz * ig;
    const R s = recip<R>(R(1) + (wx * wx + wy * wy + wz * wz));
    const R mw = mx * wx + my * wy + mz * wz;
    const R px = s * (mx + mw * wx + (my * wz - mz * wy));
    const R py = s * (my + mw * wy + (mz * wx - mx * wz));
    const R pz = s * (mz + mw * wz + (mx * wy - my * wx));
    ux = px + a * e[0] + (py * wz - pz * wy);
    uy = py + a * e[1] + (pz * wx - px * wz);
    uz = pz + a * e[2] + (px * wy - py * wx);
}

// Hat weights of one axis on a three-node window starting at node s0 of the
// old cell (s0 = -1 when the particle moves down a cell, else 0): S0 of the
// old fraction f0 and the change DS = S1 - S0 after a move by d cells (new
// cell c1 = floor(f0 + d) in {-1, 0, 1}). False when |d| >= 1. cross: the
// move leaves the cell (the window's third node carries weight). With
// R = float, f0 + d is the same binary32 sum the mixed move forms, so S1 is
// the hat of the particle's new offset.
template <typename R>
__device__ __forceinline__ bool hat3(R f0, R d, R S0[3], R DS[3], int &s0, bool &cross) {
    const bool ok = fabs(d) < R(1);
    const R g1 = f0 + (ok ? d : R(0));
    const R fl = floor(g1);
    const R f1 = g1 - fl;
    const bool dn = fl < R(0), up = fl > R(0);
    s0 = dn ? -1 : 0;
    cross = dn || up;
    const R a0 = R(1) - f0, a1 = R(1) - f1;
    // the old cell's two nodes sit at window index -s0 and 1 - s0, the new
    // cell's at c1 - s0 and c1 - s0 + 1 (1 and 2 after a move up, else 0 and 1)
    S0[0] = dn ? R(0) : a0;
    S0[1] = dn ? a0 : f0;
    S0[2] = dn ? f0 : R(0);
    DS[0] = (up ? R(0) : a1) - S0[0];
    DS[1] = (up ? a1 : f1) - S0[1];
    DS[2] = (up ? f1 : R(0)) - S0[2];
    return ok;
}

// Esirkepov current of one particle into the LDS tile sJ (three components of
// jw x jh entries, node (x0-1, y0-1) at index 0). (lx, ly): old local cell in
// [0, T); (fx, fy): old fractions; (dx, dy): displacement in cells; cz:
// Q vz/(dx dy). Returns false (and deposits nothing) for a displacement of a
// cell or more.
// Jx and Jy are kept without their constant factors -Q/(dy dt) and
// -Q/(dx dt), which flush_j applies to the tile sums. With the hat weights
// W^x_kl = DSx_k (S0y_l + DSy_l / 2) the current at half node k + 1/2 of row
// l is minus the running sum over k' <= k; the hat changes of a row sum to
// zero, so the second half node holds -DSx_2 (S0y_l + DSy_l / 2), zero unless
// the particle leaves its cell along x, and the third none. Likewise for Jy.
// Jz's weight S0x S0y + (DSx S0y + S0x DSy) / 2 + DSx DSy / 3 is taken as
// S0x_k (S0y_l + DSy_l / 2) + DSx_k (S0y_l / 2 + DSy_l / 3). Only entries that
// can carry current are added: a particle that stays in its cell adds 8
// entries, one that crosses up to 21.
template <typename R>
__device__ __forceinline__ bool esirkepov_lds(double *sJ, int jw, int jtot, int lx, int ly, R fx, R fy, R dx, R dy,
                                              R cz) {
    R S0x[3], DSx[3], S0y[3], DSy[3];
    int sx, sy;
    bool cx3, cy3;
    const bool okx = hat3(fx, dx, S0x, DSx, sx, cx3);
    const bool oky = hat3(fy, dy, S0y, DSy, sy, cy3);
    if (!(okx && oky)) return false;
    const int a0 = (ly + 1 + sy) * jw + lx + 1 + sx;   // tile index of window node (0, 0)
    double *jx = sJ + a0, *jy = sJ + jtot + a0, *jz = sJ + 2 * jtot + a0;
    R wx[3], wy[3], vy[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        wx[k] = fma(R(0.5), DSx[k], S0x[k]);
        wy[k] = fma(R(0.5), DSy[k], S0y[k]);
        vy[k] = fma(R(1) / R(3), DSy[k], R(0.5) * S0y[k]) * cz;
    }
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        if (l < 2 || cy3) {
            atomicAdd(&jx[l * jw], (double)(DSx[0] * wy[l]));
            if (cx3) atomicAdd(&jx[l * jw + 1], (double)(-DSx[2] * wy[l]));
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (k < 2 || cx3) {
            atomicAdd(&jy[k], (double)(DSy[0] * wx[k]));
            if (cy3) atomicAdd(&jy[jw + k], (double)(-DSy[2] * wx[k]));
        }
    }
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const R wyz = wy[l] * cz;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if ((k < 2 || cx3) && (l < 2 || cy3))
                atomicAdd(&jz[l * jw + k], (double)fma(DSx[k], vy[l], S0x[k] * wyz));
        }
    }
    return true;
}

// Add the current tile to the global J (one atomic per non-zero entry),
// applying the factors cx and cy that the tile's Jx and Jy sums leave out.
__device__ void flush_j(double *J, const double *sJ, const Geo &g, int x0, int y0, int jw, int jh, double cx,
                        double cy) {
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
        atomicAdd(&J[c * G + (int64_t)gy * g.nx + gx], c == 0 ? cx * v : (c == 1 ? cy * v : v));
    }
}

}  // namespace
}  // namespace apic
