// Reverse-mode derivative (adjoint) of the PIC cycle: the gradient of the
// final field energy W = 1/2 sum_j |E_j^T|^2 dV with respect to every
// particle's initial position and velocity, with step checkpointing.
//
// The forward map is the cycle the library runs: field of the initial charge,
// backward half push, then per step gather -> Boris -> move -> deposit ->
// sort -> Poisson. Adjoint of each module (lam_* = dW/d*):
//   field    E = A rho with A circulant and odd (symbol -i kappa/K^2):
//            lam_rho = A^T lam_E = -sum_d A_d lam_E_d (symbol +i kappa/K^2);
//   deposit  lam_x += (Q/dV) sum_j lam_rho_j dW_j/dx  (a gradient gather);
//   gather   lam_E += scatter of W_j lam_Ep, lam_x += sum_j dW_j/dx E_j.lam_Ep;
//   Boris    linear for fixed B: lam_v_old = R^T lam_v, lam_Ep = a (R+I)^T lam_v;
//   move     lam_v^{n+1/2} += dt lam_x^{n+1} (the wrap has slope one);
//   Higuera-Cary (state u = gamma v): the advance is u1 = R(t(m)) m + aE with
//            m = u0 + aE, R the rotation of the method's closed form and
//            t = tau / gamma+(m); its adjoint adds to R^T lam the term
//            (lam . dR/dt m) dt/dm from the dependence of gamma+ on m. The
//            move x += (u / gamma) dt gives lam_u += dt M lam_x with
//            M = (I - u u^T / (c^2 gamma^2)) / gamma. Both need the velocity
//            before the advance, so the recomputed segment also keeps the
//            velocities of every level; the advance is then re-run from them.
//            The backward half push needs u^0, which the checkpoints do not
//            hold: the method solves a time-symmetric implicit relation, so
//            u^0 is the advance of v^{-1/2} by +dt/2 under the same E_p^0;
//   sort     a permutation: each reverse step sends lam back to the order the
//            particles had before that step (perm from the forward step).
// dW/dx of the CIC hat is its slope inside the particle's cell.
//
// Checkpointing: the forward run stores the state every `stride` steps
// (positions, v^{n-1/2}, bucket table, E^n, and each particle's index in the
// caller's input order). The reverse sweep recomputes one segment at a time
// from its checkpoint, keeping per-step positions, E^n and the sort
// permutation of the segment, and walks it backwards. Particle order at a
// segment's end may differ between the recomputation and the stored next
// checkpoint (far movers take slots in arrival order; FP64 rounding), so the
// step that crosses a checkpoint maps particles through their input indices.
//
// Arithmetic: the per-particle adjoint runs in the path's precision (binary32
// for the mixed path, FP64 otherwise); grid adjoints accumulate in FP64 with
// global atomics (their summation order is not fixed, so FP64 gradients
// reproduce to rounding, not bitwise); the adjoint field solve is FP64.
#include "apic.h"
#include "apic_ctx.h"
#include "apic_device.h"

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <utility>

using namespace apic;
using namespace apic_host;

namespace apic {
namespace {

inline int nblocks(int64_t n, int cap = 8192) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    return (int)(b > cap ? cap : b);
}

// Positions of one time level (structure of arrays of the path's layout).
struct PosP {
    const int32_t *cell;
    const float *ox, *oy, *oz;
    const double *x, *y, *z;
};

template <typename R>
struct AdjP {
    Geo g;
    int64_t n;
    // level n: positions, field, lam_rho; lam arrays in the level-n order
    PosP pos;
    const double *E;        // [dim][G]
    const double *lrho;     // [G]
    const R *lxp_in;        // [dim][n]  lam_x carried from level n+1
    const R *lep_in;        // [dim][n]  lam_Ep of the push at level n
    const R *lv_in;         // [vdim][n] lam of v^{n-1/2}
    int terminal;           // the three inputs above are zero
    // reverse step n-1 (back != 0): lam in the level-(n-1) order
    int back;
    const int32_t *perm;    // level-n slot i came from level-(n-1) slot perm[i]
    const int32_t *bs;      // bucket table of the level-n order (NULL: no LDS tiling)
    PosP prev;
    double *lE_prev;        // [dim][G] accumulated with atomics
    R *lxp_out, *lep_out, *lv_out;
    int init;               // level n-1 is 0: add the backward half push
    // final output (level 0): out[id0[i]] = lam of particle i
    int final_out;
    const int32_t *id0;
    double *out_x, *out_y, *out_z, *out_vx, *out_vy, *out_vz;
    // coefficients
    R dt, cq;               // dt; Q/dV
    R a, t, s;              // Boris of a full step (t = tau = a bz for Higuera-Cary)
    R ah, th, sh;           // Boris of the backward half step
    // Higuera-Cary: level-(n-1) velocities (before the advance, level-(n-1)
    // order), E^{n-1}, and 1/c^2
    const R *vprev;         // [3][n]
    const double *Eprev;    // [dim][G]
    R ic2;
    int *err;
};

template <bool MIX, int DIM>
__device__ __forceinline__ bool load_pos(const PosP &p, int64_t i, const Geo &g, int &ix, int &iy, int &iz,
                                         typename RealOf<MIX>::T &fx, typename RealOf<MIX>::T &fy,
                                         typename RealOf<MIX>::T &fz) {
    using R = typename RealOf<MIX>::T;
    bool ok = true;
    iz = 0;
    fz = R(0);
    if constexpr (MIX) {
        const int32_t c = p.cell[i];
        if constexpr (DIM == 3) {
            ix = c & 0x3FF;
            iy = (c >> 10) & 0x3FF;
            iz = (c >> 20) & 0x3FF;
            fz = p.oz[i];
        } else {
            ix = (DIM == 2) ? (c & 0xFFFF) : c;
            iy = (DIM == 2) ? (c >> 16) : 0;
        }
        fx = p.ox[i];
        fy = (DIM >= 2) ? p.oy[i] : 0.0f;
        ok = ix >= 0 && ix < g.nx && iy >= 0 && iy < g.ny && iz >= 0 && iz < g.nz && fx >= 0.0f && fx < 1.0f &&
             fy >= 0.0f && fy < 1.0f && fz >= 0.0f && fz < 1.0f;
    } else {
        double f;
        ok = cell_f64(p.x[i], g.inv_dx, g.nx, ix, f);
        fx = (R)f;
        iy = 0;
        fy = R(0);
        if constexpr (DIM >= 2) {
            ok = cell_f64(p.y[i], g.inv_dy, g.ny, iy, f) && ok;
            fy = (R)f;
        }
        if constexpr (DIM == 3) {
            ok = cell_f64(p.z[i], g.inv_dz, g.nz, iz, f) && ok;
            fz = (R)f;
        }
    }
    if (!ok) {
        ix = iy = iz = 0;
        fx = fy = fz = R(0);
    }
    return ok;
}

// lam^T (R + I)-type Boris adjoint for one velocity advance:
// g (lam of v_new, x/y) -> lam of v_old; returns lam_Ep in ex, ey.
template <typename R, int VDIM>
__device__ __forceinline__ void boris_adj(R &gx, R &gy, R a, R t, R s, R &ex, R &ey) {
    if constexpr (VDIM == 1) {
        ex = R(2) * a * gx;
        ey = R(0);
    } else {
        const R r = R(1) - s * t;
        const R ox = r * gx - s * gy;   // R^T g, R = [[r, s], [-s, r]]
        const R oy = s * gx + r * gy;
        ex = a * (ox + gx);
        ey = a * (oy + gy);
        gx = ox;
        gy = oy;
    }
}

// Higuera-Cary adjoint of one advance u1 = R(t) m + aE, m = u0 + aE:
// l (lam of u1) -> lam of u0 in place; returns lam_Ep in ex, ey, ez (ez is
// unused in 2D, where E_z = 0).
//   R = [[C, S], [-S, C]] on (x, y), identity on z, C = (1-t^2)/(1+t^2),
//   S = 2t/(1+t^2); t = tau / gamma+, gamma+^2 = (sigma + D)/2,
//   sigma = 1 + |m|^2/c^2 - tau^2, D = sqrt(sigma^2 + 4 tau^2 (1 + mz^2/c^2));
//   dt/dm = -t/(2 gamma+^2) d(gamma+^2)/dm,
//   d(gamma+^2)/dm = (m (1 + sigma/D) + 2 tau^2 mz z / D) / c^2.
template <typename R>
__device__ __forceinline__ void hc_adj(R mx, R my, R mz, R a, R tau, R ic2, R &lx, R &ly, R &lz, R &ex, R &ey,
                                       R &ez) {
    const R g2 = R(1) + ((mx * mx + my * my) + mz * mz) * ic2;
    const R sig = g2 - tau * tau;
    const R us = mz * tau;
    const R D = sqrt(sig * sig + R(4) * (tau * tau + (us * us) * ic2));
    const R gp2 = R(0.5) * (sig + D);
    const R t = tau / sqrt(gp2);
    const R q = R(1) / (R(1) + t * t);
    const R C = (R(1) - t * t) * q, S = R(2) * t * q;
    const R dC = R(-4) * t * q * q, dS = R(2) * (R(1) - t * t) * q * q;
    const R w = lx * (dC * mx + dS * my) + ly * (dC * my - dS * mx);
    const R f = -t / (R(2) * gp2) * ic2 * w;
    const R k = R(1) + sig / D;
    const R ox = (C * lx - S * ly) + f * k * mx;
    const R oy = (S * lx + C * ly) + f * k * my;
    const R oz = lz + f * (k * mz + R(2) * tau * tau * mz / D);
    ex = a * (ox + lx);
    ey = a * (oy + ly);
    ez = a * (oz + lz);
    lx = ox;
    ly = oy;
    lz = oz;
}

// Tile coordinates of bucket b of a 1D or 2D plasma (tiles x fastest).
template <int DIM>
__device__ __forceinline__ void tile_coords2(const Geo &g, int b, int &bx, int &by) {
    bx = DIM == 2 ? b % g.nbx : b;
    by = DIM == 2 ? b / g.nbx : 0;
}

template <bool MIX, int DIM, int VDIM, bool HC>
__global__ void __launch_bounds__(kBlock) k_adj_level(AdjP<typename RealOf<MIX>::T> P) {
    using R = typename RealOf<MIX>::T;
    const Geo &g = P.g;
    const int64_t n = P.n;
    const int G = g.nx * g.ny * g.nz;
    const R idx = (R)g.inv_dx, idy = (R)g.inv_dy, idz = (R)g.inv_dz;
    // lam_Ep scattered at x^{n-1}: into the block's LDS tile when the level's
    // bucket table is given and the node lies in the tile's window, else
    // straight to global memory
    extern __shared__ __align__(16) unsigned char smem[];
    double *sT = (double *)smem;
    const bool tiled = P.bs != nullptr;
    constexpr int H = 2;
    const int tw = (1 << g.tsx) + 1 + 2 * H, th = (DIM == 2) ? (1 << g.tsy) + 1 + 2 * H : 1;
    int wx0 = 0, wy0 = 0;
    auto scat = [&](int comp, int gx, int gy, double v) {
        if (tiled) {
            int dx = gx - wx0, dy = gy - wy0;
            if (dx < 0) dx += g.nx;
            if (dy < 0) dy += g.ny;
            if (dx < tw && dy < th) {
                // through an LDS-typed pointer: ds_add_f64 with no flat
                // address-space test (the generic form of this add has
                // crashed instruction selection for gfx950)
                __hip_atomic_fetch_add((__attribute__((address_space(3))) double *)&sT[(comp * th + dy) * tw + dx], v,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                return;
            }
        }
        unsafeAtomicAdd(&P.lE_prev[comp * G + gy * g.nx + gx], v);
    };
    // 3D: the cycle with trilinear weights, E_z and the z motion; lam_Ep is
    // scattered with global atomics (no LDS tile)
    auto body3 = [&](int64_t i) {
        int ix, iy, iz;
        R fx, fy, fz;
        if (!load_pos<MIX, 3>(P.pos, i, g, ix, iy, iz, fx, fy, fz)) raise_err(P.err, ERR_DOMAIN);
        R lx = R(0), ly = R(0), lz = R(0), lex = R(0), ley = R(0), lez = R(0), lvx = R(0), lvy = R(0), lvz = R(0);
        if (!P.terminal) {
            lx = P.lxp_in[i];
            ly = P.lxp_in[n + i];
            lz = P.lxp_in[2 * n + i];
            lex = P.lep_in[i];
            ley = P.lep_in[n + i];
            lez = P.lep_in[2 * n + i];
            lvx = P.lv_in[i];
            lvy = P.lv_in[n + i];
            lvz = P.lv_in[2 * n + i];
        }
        // deposit and gather adjoints at level n: the slope of the trilinear
        // hat applied to g = E . lam_Ep + (Q/dV) lam_rho over the cell
        {
            const int xs[2] = {ix, ix + 1 >= g.nx ? 0 : ix + 1};
            const int ys[2] = {iy, iy + 1 >= g.ny ? 0 : iy + 1};
            const int zs[2] = {iz, iz + 1 >= g.nz ? 0 : iz + 1};
            R gv[2][2][2];
#pragma unroll
            for (int c2 = 0; c2 < 2; ++c2)
#pragma unroll
                for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
                    for (int a2 = 0; a2 < 2; ++a2) {
                        const int m = (zs[c2] * g.ny + ys[b2]) * g.nx + xs[a2];
                        gv[c2][b2][a2] = (R)P.E[m] * lex + (R)P.E[G + m] * ley + (R)P.E[2 * G + m] * lez +
                                         P.cq * (R)P.lrho[m];
                    }
            const R wx[2] = {R(1) - fx, fx}, wy[2] = {R(1) - fy, fy}, wz[2] = {R(1) - fz, fz};
            R gx = R(0), gy = R(0), gz = R(0);
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v) {
                    gx += wy[u] * wz[v] * (gv[v][u][1] - gv[v][u][0]);
                    gy += wx[u] * wz[v] * (gv[v][1][u] - gv[v][0][u]);
                    gz += wx[u] * wy[v] * (gv[1][v][u] - gv[0][v][u]);
                }
            lx += gx * idx;
            ly += gy * idy;
            lz += gz * idz;
        }
        if (P.final_out) {
            const int32_t o = P.id0[i];
            if ((uint32_t)o >= (uint32_t)n) {
                raise_err(P.err, ERR_ORDER);
                return;
            }
            P.out_x[o] = (double)lx;
            P.out_y[o] = (double)ly;
            P.out_z[o] = (double)lz;
            P.out_vx[o] = (double)lvx;
            P.out_vy[o] = (double)lvy;
            P.out_vz[o] = (double)lvz;
            return;
        }
        if (!P.back) return;
        const int32_t j = P.perm[i];
        if ((uint32_t)j >= (uint32_t)n) {
            raise_err(P.err, ERR_ORDER);
            return;
        }
        int jx, jy, jz;
        R qx, qy, qz;
        if (!load_pos<MIX, 3>(P.prev, j, g, jx, jy, jz, qx, qy, qz)) raise_err(P.err, ERR_DOMAIN);
        const int pxs[2] = {jx, jx + 1 >= g.nx ? 0 : jx + 1};
        const int pys[2] = {jy, jy + 1 >= g.ny ? 0 : jy + 1};
        const int pzs[2] = {jz, jz + 1 >= g.nz ? 0 : jz + 1};
        const R vx2[2] = {R(1) - qx, qx}, vy2[2] = {R(1) - qy, qy}, vz2[2] = {R(1) - qz, qz};
        R gx, gy, gz, ex, ey, ez;
        if constexpr (HC) {
            // re-run the advance from the level-(n-1) velocity in E_p^{n-1}
            R epx = R(0), epy = R(0), epz = R(0);
#pragma unroll
            for (int c2 = 0; c2 < 2; ++c2)
#pragma unroll
                for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
                    for (int a2 = 0; a2 < 2; ++a2) {
                        const int m = (pzs[c2] * g.ny + pys[b2]) * g.nx + pxs[a2];
                        const R w = (vx2[a2] * vy2[b2]) * vz2[c2];
                        epx += w * (R)P.Eprev[m];
                        epy += w * (R)P.Eprev[G + m];
                        epz += w * (R)P.Eprev[2 * G + m];
                    }
            const R u0x = P.vprev[j], u0y = P.vprev[n + j], u0z = P.vprev[2 * n + j];
            R ux = u0x, uy = u0y, uz = u0z;
            higuera_cary<R>(ux, uy, uz, epx, epy, epz, P.a, P.t, P.ic2);
            // move x += (u / gamma) dt on all three axes: lam_u1 = lam_v + dt M(u1) lam_x
            const R ig = R(1) / lorentz<R>(ux, uy, uz, P.ic2);
            const R cf = P.ic2 * ((ux * lx + uy * ly) + uz * lz) * ig * ig;
            gx = lvx + P.dt * ig * (lx - ux * cf);
            gy = lvy + P.dt * ig * (ly - uy * cf);
            gz = lvz + P.dt * ig * (lz - uz * cf);
            hc_adj<R>(u0x + P.a * epx, u0y + P.a * epy, u0z + P.a * epz, P.a, P.t, P.ic2, gx, gy, gz, ex, ey, ez);
            if (P.init) {
                R hx = u0x, hy = u0y, hz = u0z;
                higuera_cary<R>(hx, hy, hz, epx, epy, epz, -P.ah, -P.th, P.ic2);
                R fx2, fy2, fz2;
                hc_adj<R>(hx + P.ah * epx, hy + P.ah * epy, hz + P.ah * epz, P.ah, P.th, P.ic2, gx, gy, gz, fx2, fy2,
                          fz2);
                ex += fx2;
                ey += fy2;
                ez += fz2;
            }
        } else {
            // move, then Boris: the rotation about z acts on (x, y); v_z takes
            // the two half kicks a E_z, so lam_Ez = 2a lam_vz
            gx = lvx + P.dt * lx;
            gy = lvy + P.dt * ly;
            gz = lvz + P.dt * lz;
            boris_adj<R, 3>(gx, gy, P.a, P.t, P.s, ex, ey);
            ez = R(2) * P.a * gz;
            if (P.init) {
                R hx, hy;
                boris_adj<R, 3>(gx, gy, P.ah, P.th, P.sh, hx, hy);
                ex += hx;
                ey += hy;
                ez += R(2) * P.ah * gz;
            }
        }
        // gather adjoint at level n-1: W_j(x^{n-1}) lam_Ep into lam_E
#pragma unroll
        for (int c2 = 0; c2 < 2; ++c2)
#pragma unroll
            for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
                for (int a2 = 0; a2 < 2; ++a2) {
                    const int m = (pzs[c2] * g.ny + pys[b2]) * g.nx + pxs[a2];
                    const R w = (vx2[a2] * vy2[b2]) * vz2[c2];
                    unsafeAtomicAdd(&P.lE_prev[m], (double)(w * ex));
                    unsafeAtomicAdd(&P.lE_prev[G + m], (double)(w * ey));
                    unsafeAtomicAdd(&P.lE_prev[2 * G + m], (double)(w * ez));
                }
        P.lxp_out[j] = lx;
        P.lxp_out[n + j] = ly;
        P.lxp_out[2 * n + j] = lz;
        P.lep_out[j] = ex;
        P.lep_out[n + j] = ey;
        P.lep_out[2 * n + j] = ez;
        P.lv_out[j] = gx;
        P.lv_out[n + j] = gy;
        P.lv_out[2 * n + j] = gz;
    };
    auto body = [&](int64_t i) {
        int ix, iy, iz_;
        R fx, fy, fz_;
        if (!load_pos<MIX, DIM>(P.pos, i, g, ix, iy, iz_, fx, fy, fz_)) raise_err(P.err, ERR_DOMAIN);
        R lx = R(0), ly = R(0), lex = R(0), ley = R(0), lvx = R(0), lvy = R(0), lvz = R(0);
        if (!P.terminal) {
            lx = P.lxp_in[i];
            lex = P.lep_in[i];
            lvx = P.lv_in[i];
            if constexpr (DIM == 2) {
                ly = P.lxp_in[n + i];
                ley = P.lep_in[n + i];
            }
            if constexpr (VDIM >= 2) lvy = P.lv_in[n + i];
            if constexpr (VDIM >= 3) lvz = P.lv_in[2 * n + i];
        }
        // deposit and gather adjoints at level n: slope of the hat applied to
        // g_j = E_j . lam_Ep + (Q/dV) lam_rho_j over the particle's cell
        int ip = ix + 1;
        if (ip >= g.nx) ip = 0;
        if constexpr (DIM == 1) {
            const R g0 = (R)P.E[ix] * lex + P.cq * (R)P.lrho[ix];
            const R g1 = (R)P.E[ip] * lex + P.cq * (R)P.lrho[ip];
            lx += (g1 - g0) * idx;
        } else {
            int jp = iy + 1;
            if (jp >= g.ny) jp = 0;
            const int a00 = iy * g.nx + ix, a10 = iy * g.nx + ip, a01 = jp * g.nx + ix, a11 = jp * g.nx + ip;
            const R g00 = (R)P.E[a00] * lex + (R)P.E[G + a00] * ley + P.cq * (R)P.lrho[a00];
            const R g10 = (R)P.E[a10] * lex + (R)P.E[G + a10] * ley + P.cq * (R)P.lrho[a10];
            const R g01 = (R)P.E[a01] * lex + (R)P.E[G + a01] * ley + P.cq * (R)P.lrho[a01];
            const R g11 = (R)P.E[a11] * lex + (R)P.E[G + a11] * ley + P.cq * (R)P.lrho[a11];
            lx += ((R(1) - fy) * (g10 - g00) + fy * (g11 - g01)) * idx;
            ly += ((R(1) - fx) * (g01 - g00) + fx * (g11 - g10)) * idy;
        }
        if (P.final_out) {
            const int32_t o = P.id0[i];
            if ((uint32_t)o >= (uint32_t)n) {
                raise_err(P.err, ERR_ORDER);
                return;
            }
            P.out_x[o] = (double)lx;
            if constexpr (DIM == 2) P.out_y[o] = (double)ly;
            P.out_vx[o] = (double)lvx;
            if constexpr (VDIM >= 2) P.out_vy[o] = (double)lvy;
            if constexpr (VDIM >= 3) P.out_vz[o] = (double)lvz;
            return;
        }
        if (!P.back) return;
        if constexpr (HC) {
            static_assert(VDIM == 3, "the Higuera-Cary adjoint needs three velocity components");
            // reverse of the step n-1 -> n: re-run the advance from the
            // level-(n-1) velocity, then the move and advance adjoints
            const int32_t j = P.perm[i];
            if ((uint32_t)j >= (uint32_t)n) {
                raise_err(P.err, ERR_ORDER);
                return;
            }
            int jx, jy, jz_;
            R qx, qy, qz_;
            if (!load_pos<MIX, DIM>(P.prev, j, g, jx, jy, jz_, qx, qy, qz_)) raise_err(P.err, ERR_DOMAIN);
            int jxp = jx + 1, jyp = jy + 1;
            if (jxp >= g.nx) jxp = 0;
            if (jyp >= g.ny) jyp = 0;
            const R w00 = (R(1) - qx) * (R(1) - qy), w10 = qx * (R(1) - qy);
            const R w01 = (R(1) - qx) * qy, w11 = qx * qy;
            const int b00 = jy * g.nx + jx, b10 = jy * g.nx + jxp, b01 = jyp * g.nx + jx, b11 = jyp * g.nx + jxp;
            const R epx = w00 * (R)P.Eprev[b00] + w10 * (R)P.Eprev[b10] + w01 * (R)P.Eprev[b01] +
                          w11 * (R)P.Eprev[b11];
            const R epy = w00 * (R)P.Eprev[G + b00] + w10 * (R)P.Eprev[G + b10] + w01 * (R)P.Eprev[G + b01] +
                          w11 * (R)P.Eprev[G + b11];
            const R u0x = P.vprev[j], u0y = P.vprev[n + j], u0z = P.vprev[2 * n + j];
            R ux = u0x, uy = u0y, uz = u0z;
            higuera_cary<R>(ux, uy, uz, epx, epy, R(0), P.a, P.t, P.ic2);
            // move: lam_u1 = lam_v + dt M(u1) lam_x
            const R ig = R(1) / lorentz<R>(ux, uy, uz, P.ic2);
            const R cf = P.ic2 * (ux * lx + uy * ly) * ig * ig;
            R gx = lvx + P.dt * ig * (lx - ux * cf);
            R gy = lvy + P.dt * ig * (ly - uy * cf);
            R gz = lvz - P.dt * ig * (uz * cf);
            R ex, ey, ez_unused;
            hc_adj<R>(u0x + P.a * epx, u0y + P.a * epy, u0z, P.a, P.t, P.ic2, gx, gy, gz, ex, ey, ez_unused);
            if (P.init) {
                // v^{-1/2} = advance(u^0, E_p^0, -dt/2); u^0 = advance(v^{-1/2}, E_p^0, +dt/2)
                R hx = u0x, hy = u0y, hz = u0z;
                higuera_cary<R>(hx, hy, hz, epx, epy, R(0), -P.ah, -P.th, P.ic2);
                R fx, fy, fz_unused;
                hc_adj<R>(hx + P.ah * epx, hy + P.ah * epy, hz, P.ah, P.th, P.ic2, gx, gy, gz, fx, fy, fz_unused);
                ex += fx;
                ey += fy;
            }
            scat(0, jx, jy, (double)(w00 * ex));
            scat(0, jxp, jy, (double)(w10 * ex));
            scat(0, jx, jyp, (double)(w01 * ex));
            scat(0, jxp, jyp, (double)(w11 * ex));
            scat(1, jx, jy, (double)(w00 * ey));
            scat(1, jxp, jy, (double)(w10 * ey));
            scat(1, jx, jyp, (double)(w01 * ey));
            scat(1, jxp, jyp, (double)(w11 * ey));
            P.lxp_out[j] = lx;
            P.lxp_out[n + j] = ly;
            P.lep_out[j] = ex;
            P.lep_out[n + j] = ey;
            P.lv_out[j] = gx;
            P.lv_out[n + j] = gy;
            P.lv_out[2 * n + j] = gz;
            return;
        }
        // reverse of the step n-1 -> n: move, then Boris
        R gx = lvx + P.dt * lx;
        R gy = (DIM == 2) ? lvy + P.dt * ly : lvy;
        R ex, ey;
        boris_adj<R, VDIM>(gx, gy, P.a, P.t, P.s, ex, ey);
        if (P.init) {
            // v^{-1/2} = Boris(v^0, E_p^0, -dt/2) uses the same E_p^0
            R hx, hy;
            boris_adj<R, VDIM>(gx, gy, P.ah, P.th, P.sh, hx, hy);
            ex += hx;
            ey += hy;
        }
        const int32_t j = P.perm[i];
        if ((uint32_t)j >= (uint32_t)n) {
            raise_err(P.err, ERR_ORDER);
            return;
        }
        int jx, jy, jz_;
        R qx, qy, qz_;
        if (!load_pos<MIX, DIM>(P.prev, j, g, jx, jy, jz_, qx, qy, qz_)) raise_err(P.err, ERR_DOMAIN);
        // gather adjoint at level n-1: scatter W_j(x^{n-1}) lam_Ep into lam_E
        int jxp = jx + 1;
        if (jxp >= g.nx) jxp = 0;
        if constexpr (DIM == 1) {
            scat(0, jx, 0, (double)((R(1) - qx) * ex));
            scat(0, jxp, 0, (double)(qx * ex));
        } else {
            int jyp = jy + 1;
            if (jyp >= g.ny) jyp = 0;
            const R w00 = (R(1) - qx) * (R(1) - qy), w10 = qx * (R(1) - qy);
            const R w01 = (R(1) - qx) * qy, w11 = qx * qy;
            scat(0, jx, jy, (double)(w00 * ex));
            scat(0, jxp, jy, (double)(w10 * ex));
            scat(0, jx, jyp, (double)(w01 * ex));
            scat(0, jxp, jyp, (double)(w11 * ex));
            scat(1, jx, jy, (double)(w00 * ey));
            scat(1, jxp, jy, (double)(w10 * ey));
            scat(1, jx, jyp, (double)(w01 * ey));
            scat(1, jxp, jyp, (double)(w11 * ey));
        }
        P.lxp_out[j] = lx;
        P.lep_out[j] = ex;
        P.lv_out[j] = gx;
        if constexpr (DIM == 2) {
            P.lxp_out[n + j] = ly;
            P.lep_out[n + j] = ey;
        }
        if constexpr (VDIM >= 2) P.lv_out[n + j] = gy;
        if constexpr (VDIM >= 3) P.lv_out[2 * n + j] = lvz;   // no E_z and no z motion
    };
    if constexpr (DIM == 3) {
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
            body3(i);
        return;
    } else {
    if (!tiled) {
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
            body(i);
        return;
    }
    // level-n buckets: the particles of one tile, their old positions within
    // a couple of cells of it
    int first, end, stride;
    bucket_walk(g.nbuckets, first, end, stride);
    const int nt = (DIM == 2 ? 2 : 1) * tw * th;
    for (int b = first; b < end; b += stride) {
        int bx, by;
        tile_coords2<DIM>(g, b, bx, by);
        wx0 = (bx << g.tsx) - H;
        wx0 = wx0 < 0 ? wx0 + g.nx : wx0;
        wy0 = 0;
        if constexpr (DIM == 2) {
            wy0 = (by << g.tsy) - H;
            wy0 = wy0 < 0 ? wy0 + g.ny : wy0;
        }
        for (int t = threadIdx.x; t < nt; t += blockDim.x) sT[t] = 0.0;
        __syncthreads();
        const int64_t i0 = min(max((int64_t)P.bs[b], (int64_t)0), n);
        const int64_t i1 = min(max((int64_t)P.bs[b + 1], i0), n);
        for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) body(i);
        __syncthreads();
        for (int t = threadIdx.x; t < nt; t += blockDim.x) {
            const double v = sT[t];
            if (v == 0.0) continue;
            const int comp = t / (tw * th), r = t % (tw * th);
            int gx = wx0 + r % tw, gy = wy0 + r / tw;
            gx = gx >= g.nx ? gx - g.nx : gx;
            gy = gy >= g.ny ? gy - g.ny : gy;
            unsafeAtomicAdd(&P.lE_prev[comp * G + gy * g.nx + gx], v);
        }
        __syncthreads();
    }
    }
}

// Physical FP64 state -> the path's representation (see apic_import_state).
template <bool MIX, int DIM, int VDIM>
__global__ void k_import(Geo g, int64_t n, double dx, double dy, double dz, const double *x, const double *y,
                         const double *z, const double *vx, const double *vy, const double *vz, Parts out, int *err) {
    using R = typename RealOf<MIX>::T;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double xi = x[i];
        const double yi = (DIM >= 2) ? y[i] : 0.0;
        const double zi = (DIM == 3) ? z[i] : 0.0;
        // x = L (a wrap that rounded up) is the same node as x = 0
        if (!(xi >= 0.0 && xi <= g.lx) || (DIM >= 2 && !(yi >= 0.0 && yi <= g.ly)) ||
            (DIM == 3 && !(zi >= 0.0 && zi <= g.lz)))
            raise_err(err, ERR_DOMAIN);
        if constexpr (MIX) {
            auto split = [](double v, double d, int nn, int &c, float &o) {
                const double q = v / d;
                double fl = floor(q);
                o = (float)(q - fl);
                if (o >= 1.0f) {
                    o = 0.0f;
                    fl += 1.0;
                }
                long long ci = (long long)fl % nn;
                if (ci < 0) ci += nn;
                c = (int)ci;
            };
            int cx, cy = 0, cz = 0;
            float ox, oy = 0.0f, oz = 0.0f;
            split(isfinite(xi) ? xi : 0.0, dx, g.nx, cx, ox);
            if constexpr (DIM >= 2) split(isfinite(yi) ? yi : 0.0, dy, g.ny, cy, oy);
            if constexpr (DIM == 3) split(isfinite(zi) ? zi : 0.0, dz, g.nz, cz, oz);
            out.cell[i] = (DIM == 3) ? ((cz << 20) | (cy << 10) | cx) : (DIM == 2) ? ((cy << 16) | cx) : cx;
            out.ox[i] = ox;
            if constexpr (DIM >= 2) out.oy[i] = oy;
            if constexpr (DIM == 3) out.oz[i] = oz;
        } else {
            out.x[i] = xi;
            if constexpr (DIM >= 2) out.y[i] = yi;
            if constexpr (DIM == 3) out.z[i] = zi;
        }
        ((R *)out.vx)[i] = (R)vx[i];
        if constexpr (VDIM >= 2) ((R *)out.vy)[i] = (R)vy[i];
        if constexpr (VDIM >= 3) ((R *)out.vz)[i] = (R)vz[i];
    }
}

// out[i] = src[perm[i]] (input index carried through one forward step)
__global__ void k_adj_compose_ids(int64_t n, const int32_t *src, const int32_t *perm, int32_t *out, int *err) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p = perm[i];
        if ((uint32_t)p >= (uint32_t)n) {
            raise_err(err, ERR_ORDER);
            out[i] = 0;
            continue;
        }
        out[i] = src[p];
    }
}

// inv[id[k]] = k
__global__ void k_adj_invert(int64_t n, const int32_t *id, int32_t *inv, int *err) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t o = id[k];
        if ((uint32_t)o >= (uint32_t)n) {
            raise_err(err, ERR_ORDER);
            continue;
        }
        inv[o] = (int32_t)k;
    }
}

// out[i] = perm_last[inv[id_next[i]]]: the level-(e-1) slot of the particle
// that sits in slot i of the stored level-e order
__global__ void k_adj_cross_perm(int64_t n, const int32_t *id_next, const int32_t *inv, const int32_t *perm_last,
                                 int32_t *out, int *err) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t o = id_next[i];
        int32_t r = 0;
        if ((uint32_t)o < (uint32_t)n) {
            const int32_t k = inv[o];
            if ((uint32_t)k < (uint32_t)n) r = perm_last[k];
            else raise_err(err, ERR_ORDER);
        } else {
            raise_err(err, ERR_ORDER);
        }
        out[i] = r;
    }
}

__global__ void k_adj_scale(int64_t m, const double *src, double *dst, double scale) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = scale * src[i];
}

__global__ void k_adj_fill(int64_t m, double *dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = 0.0;
}

// lam_rho_hat = norm * (i kappa_x lam_Ex_hat + i kappa_y lam_Ey_hat
// [+ i kappa_z lam_Ez_hat]) / K^2, 0 at k = 0; lzh NULL below 3D. lrh may be
// lxh (each entry is read before it is written).
__global__ void k_adj_spectral(Geo g, const double2 *lxh, const double2 *lyh, const double2 *lzh, double2 *lrh,
                               CtxDev c) {
    const int hx = g.nx / 2 + 1;
    const int64_t tot = (int64_t)hx * g.ny * g.nz;
    const double norm = 1.0 / ((double)g.nx * (double)g.ny * (double)g.nz);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        const int kx = (int)(i % hx);
        const int64_t r = i / hx;
        const int ky = (int)(r % g.ny), kz = (int)(r / g.ny);
        const double K2 = c.kx2[kx] + c.ky2[ky] + c.kz2[kz];
        const double inv = (i == 0) ? 0.0 : norm / K2;
        const double2 a = lxh[i], b = lyh[i];
        const double2 z = lzh ? lzh[i] : make_double2(0.0, 0.0);
        const double kax = c.kapx[kx], kay = c.kapy[ky], kaz = c.kapz[kz];
        // i * kappa * (re + i im) = -kappa * im + i kappa * re
        lrh[i] = make_double2(-((kax * a.y + kay * b.y) + kaz * z.y) * inv, ((kax * a.x + kay * b.x) + kaz * z.x) * inv);
    }
}

// 1D: lam_rho = -A lam_E with A the same Gauss-law solve as the forward field
__global__ void __launch_bounds__(kBlock) k_adj_field1d(int nx, const double *lE, double dx, double *lrho) {
    extern __shared__ __align__(16) unsigned char smem[];
    double *sr = (double *)smem;
    __shared__ double sRed[kWaves];
    __shared__ double sScan[kBlock];
    for (int i = threadIdx.x; i < nx; i += blockDim.x) sr[i] = lE[i];
    __syncthreads();
    (void)field1d_block(sr, nx, dx, lrho, nullptr, sRed, sScan);
    for (int i = threadIdx.x; i < nx; i += blockDim.x) lrho[i] = -lrho[i];
}

// dW/d delta0 = sum_p (lam_x[p] dx[p] + lam_y[p] dy[p]): the chain rule through
// the seeded displacement x_p^0 = x_p,u + delta0 d_p; one workgroup, fixed order
// (ly, dy NULL in 1D)
__global__ void __launch_bounds__(1024) k_adj_delta0(int64_t n, const double *lx, const double *dx, const double *ly,
                                                    const double *dy, double *out) {
    __shared__ double sRed[16];
    double p = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        p += lx[i] * dx[i];
        if (ly) p += ly[i] * dy[i];
    }
    p = block_sum(p, sRed);
    if (threadIdx.x == 0) *out = p;
}

// W = 1/2 dV sum_i E_i^2 in a fixed order (one workgroup)
__global__ void __launch_bounds__(1024) k_adj_energy(int64_t m, const double *E, double dV, double *W) {
    __shared__ double sRed[16];
    double p = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) p += E[i] * E[i];
    p = block_sum(p, sRed);
    if (threadIdx.x == 0) *W = 0.5 * dV * p;
}

}  // namespace
}  // namespace apic

namespace {

// ---- layout of the checkpoint buffer and of the adjoint workspace ---------

struct CkLayout {
    size_t pos[4];      // mixed: cell, ox, oy, oz; FP64: x, y, z (-1 = absent)
    size_t vel[3];
    size_t bstart, E, id;
    size_t bytes;       // one checkpoint
};

CkLayout ck_layout(const apic_ctx *c) {
    CkLayout L;
    const int64_t n = c->n;
    const size_t r = c->mixed ? 4 : 8;
    const int64_t G = (int64_t)c->d.nx * c->d.ny * c->d.nz;
    size_t off = 0;
    auto take = [&](size_t b) { size_t o = off; off = align256(off + b); return o; };
    for (auto &v : L.pos) v = (size_t)-1;
    for (auto &v : L.vel) v = (size_t)-1;
    if (c->mixed) {
        L.pos[0] = take(4 * n);
        for (int k = 0; k < c->d.dim; ++k) L.pos[1 + k] = take(4 * n);
    } else {
        for (int k = 0; k < c->d.dim; ++k) L.pos[k] = take(8 * n);
    }
    for (int k = 0; k < c->d.vdim; ++k) L.vel[k] = take(r * n);
    L.bstart = take(4 * (c->g.nbuckets + 1));
    L.E = take(8 * (size_t)c->d.dim * G);
    L.id = take(4 * n);
    L.bytes = off;
    return L;
}

struct AdjWs {
    size_t ctx;                 // the context workspace (sort, step, field solve)
    size_t pw_pos[4], pw_vel[3], bstart, E, E32, rho;
    size_t id_a, id_b, inv, cross;
    size_t snap_pos;            // stride entries of positions
    size_t snap_pos_bytes;
    size_t snap_perm, snap_E;   // stride entries
    size_t snap_vel;            // stride entries of [3][n] velocities (Higuera-Cary)
    size_t snap_bs;             // stride entries of the bucket table (nb + 1)
    size_t lam[2][3];           // ping-pong: lam_x carried, lam_Ep, lam_v
    size_t lE, lrho, W;
    size_t bytes;
};

size_t pos_bytes(const apic_ctx *c) {
    const int64_t n = c->n;
    if (c->mixed) return align256(4 * n) * (c->d.dim + 1);
    return align256(8 * n) * c->d.dim;
}

AdjWs adj_layout(const apic_ctx *c, int stride) {
    AdjWs L;
    const int64_t n = c->n;
    const size_t r = c->mixed ? 4 : 8;
    const int64_t G = (int64_t)c->d.nx * c->d.ny * c->d.nz;
    const int dim = c->d.dim, vdim = c->d.vdim;
    size_t off = 0;
    auto take = [&](size_t b) { size_t o = off; off = align256(off + b); return o; };
    L.ctx = take(c->ws_bytes);
    for (auto &v : L.pw_pos) v = (size_t)-1;
    for (auto &v : L.pw_vel) v = (size_t)-1;
    if (c->mixed) {
        L.pw_pos[0] = take(4 * n);
        for (int k = 0; k < dim; ++k) L.pw_pos[1 + k] = take(4 * n);
    } else {
        for (int k = 0; k < dim; ++k) L.pw_pos[k] = take(8 * n);
    }
    for (int k = 0; k < vdim; ++k) L.pw_vel[k] = take(r * n);
    L.bstart = take(4 * (c->g.nbuckets + 1));
    L.E = take(8 * (size_t)dim * G);
    L.E32 = take(4 * (size_t)dim * G);
    L.rho = take(8 * (size_t)G);
    L.id_a = take(4 * n);
    L.id_b = take(4 * n);
    L.inv = take(4 * n);
    L.cross = take(4 * n);
    L.snap_pos_bytes = pos_bytes(c);
    L.snap_pos = take(L.snap_pos_bytes * (size_t)stride);
    L.snap_perm = take(align256(4 * n) * (size_t)stride);
    L.snap_E = take(align256(8 * (size_t)dim * G) * (size_t)stride);
    L.snap_vel = c->g.hc ? take(align256(r * 3 * n) * (size_t)stride) : (size_t)-1;
    L.snap_bs = take(align256(4 * (size_t)(c->g.nbuckets + 1)) * (size_t)stride);
    for (int b = 0; b < 2; ++b) {
        L.lam[b][0] = take(r * dim * n);
        L.lam[b][1] = take(r * dim * n);
        L.lam[b][2] = take(r * vdim * n);
    }
    L.lE = take(8 * (size_t)dim * G);
    L.lrho = take(8 * (size_t)G);
    L.W = take(8);
    L.bytes = off;
    return L;
}

// Position arrays of a position block laid out like pos_bytes() describes.
PosP pos_block(const apic_ctx *c, char *base) {
    PosP p{};
    const int64_t n = c->n;
    if (c->mixed) {
        const size_t a = align256(4 * n);
        p.cell = (const int32_t *)base;
        p.ox = (const float *)(base + a);
        p.oy = c->d.dim >= 2 ? (const float *)(base + 2 * a) : nullptr;
        p.oz = c->d.dim == 3 ? (const float *)(base + 3 * a) : nullptr;
    } else {
        const size_t a = align256(8 * n);
        p.x = (const double *)base;
        p.y = c->d.dim >= 2 ? (const double *)(base + a) : nullptr;
        p.z = c->d.dim == 3 ? (const double *)(base + 2 * a) : nullptr;
    }
    return p;
}

PosP pos_ck(const apic_ctx *c, const CkLayout &L, char *ck) {
    PosP p{};
    if (c->mixed) {
        p.cell = wsp<const int32_t>(ck, L.pos[0]);
        p.ox = wsp<const float>(ck, L.pos[1]);
        p.oy = wsp<const float>(ck, L.pos[2]);
        p.oz = wsp<const float>(ck, L.pos[3]);
    } else {
        p.x = wsp<const double>(ck, L.pos[0]);
        p.y = wsp<const double>(ck, L.pos[1]);
        p.z = wsp<const double>(ck, L.pos[2]);
    }
    return p;
}

apic_particles work_parts(const apic_ctx *c, const AdjWs &L, char *ws) {
    apic_particles p{};
    p.n = c->n;
    if (c->mixed) {
        p.cell = wsp<int32_t>(ws, L.pw_pos[0]);
        p.ox = wsp<float>(ws, L.pw_pos[1]);
        p.oy = wsp<float>(ws, L.pw_pos[2]);
        p.oz = wsp<float>(ws, L.pw_pos[3]);
    } else {
        p.x = wsp<double>(ws, L.pw_pos[0]);
        p.y = wsp<double>(ws, L.pw_pos[1]);
        p.z = wsp<double>(ws, L.pw_pos[2]);
    }
    p.vx = wsp<void>(ws, L.pw_vel[0]);
    p.vy = wsp<void>(ws, L.pw_vel[1]);
    p.vz = wsp<void>(ws, L.pw_vel[2]);
    p.bucket_start = wsp<int32_t>(ws, L.bstart);
    p.perm = nullptr;
    return p;
}

// Copy the positions of p into a position block (pos_bytes layout).
apic_status save_pos(apic_ctx *c, const apic_particles &p, char *dst, hipStream_t s) {
    const int64_t n = c->n;
    if (c->mixed) {
        const size_t a = align256(4 * n);
        HIPCHK(c, launch_copy_bytes(dst, p.cell, 4 * n, s));
        HIPCHK(c, launch_copy_bytes(dst + a, p.ox, 4 * n, s));
        if (c->d.dim >= 2) HIPCHK(c, launch_copy_bytes(dst + 2 * a, p.oy, 4 * n, s));
        if (c->d.dim == 3) HIPCHK(c, launch_copy_bytes(dst + 3 * a, p.oz, 4 * n, s));
    } else {
        const size_t a = align256(8 * n);
        HIPCHK(c, launch_copy_bytes(dst, p.x, 8 * n, s));
        if (c->d.dim >= 2) HIPCHK(c, launch_copy_bytes(dst + a, p.y, 8 * n, s));
        if (c->d.dim == 3) HIPCHK(c, launch_copy_bytes(dst + 2 * a, p.z, 8 * n, s));
    }
    return APIC_OK;
}

// state <-> checkpoint (dir = +1: save, -1: load)
apic_status ck_transfer(apic_ctx *c, const CkLayout &L, char *ck, apic_particles &p, double *E, int32_t *id,
                        int dir, hipStream_t s) {
    const int64_t n = c->n;
    const size_t r = c->mixed ? 4 : 8;
    const int64_t G = (int64_t)c->d.nx * c->d.ny * c->d.nz;
    auto mv = [&](void *state, size_t off, size_t bytes) -> hipError_t {
        if (!state || off == (size_t)-1) return hipSuccess;
        return dir > 0 ? launch_copy_bytes(ck + off, state, (int64_t)bytes, s)
                       : launch_copy_bytes(state, ck + off, (int64_t)bytes, s);
    };
    if (c->mixed) {
        HIPCHK(c, mv(p.cell, L.pos[0], 4 * n));
        HIPCHK(c, mv(p.ox, L.pos[1], 4 * n));
        HIPCHK(c, mv(p.oy, L.pos[2], 4 * n));
        HIPCHK(c, mv(p.oz, L.pos[3], 4 * n));
    } else {
        HIPCHK(c, mv(p.x, L.pos[0], 8 * n));
        HIPCHK(c, mv(p.y, L.pos[1], 8 * n));
        HIPCHK(c, mv(p.z, L.pos[2], 8 * n));
    }
    HIPCHK(c, mv(p.vx, L.vel[0], r * n));
    HIPCHK(c, mv(p.vy, L.vel[1], r * n));
    HIPCHK(c, mv(p.vz, L.vel[2], r * n));
    HIPCHK(c, mv(p.bucket_start, L.bstart, 4 * (size_t)(c->g.nbuckets + 1)));
    HIPCHK(c, mv(E, L.E, 8 * (size_t)c->d.dim * G));
    HIPCHK(c, mv(id, L.id, 4 * n));
    return APIC_OK;
}

int n_checkpoints(int nsteps, int stride) { return (nsteps + stride - 1) / stride; }

// lam_rho = A^T lam_E (FP64)
apic_status adj_solve(apic_ctx *c, double *lE, double *lrho, char *ws_ctx, hipStream_t s) {
    const int64_t G = (int64_t)c->d.nx * c->d.ny * c->d.nz;
    if (c->d.dim == 1) {
        hipLaunchKernelGGL(k_adj_field1d, dim3(1), dim3(kBlock), (size_t)c->d.nx * sizeof(double), s, c->d.nx, lE,
                           c->d.lx / c->d.nx, lrho);
        HIPCHK(c, hipGetLastError());
        return APIC_OK;
    }
    // half spectra of the dim components (the context's one rho spectrum and
    // its dim phi spectra hold them), combined in place into the first
    const size_t H = (size_t)(c->d.nx / 2 + 1) * c->d.ny * c->d.nz;
    char *rhat = wsp<char>(ws_ctx, c->o_rhat);
    char *ehat = wsp<char>(ws_ctx, c->o_ehat);
    FFTCHK(c, hipfftSetStream(c->fwd, s));
    FFTCHK(c, hipfftExecD2Z(c->fwd, (hipfftDoubleReal *)lE, (hipfftDoubleComplex *)rhat));
    FFTCHK(c, hipfftExecD2Z(c->fwd, (hipfftDoubleReal *)(lE + G), (hipfftDoubleComplex *)ehat));
    if (c->d.dim == 3)
        FFTCHK(c, hipfftExecD2Z(c->fwd, (hipfftDoubleReal *)(lE + 2 * G), (hipfftDoubleComplex *)(ehat + 16 * H)));
    hipLaunchKernelGGL(k_adj_spectral, dim3(nblocks((int64_t)H, 1024)), dim3(kBlock), 0, s, c->g,
                       (const double2 *)rhat, (const double2 *)ehat,
                       c->d.dim == 3 ? (const double2 *)(ehat + 16 * H) : nullptr, (double2 *)rhat, c->dev);
    HIPCHK(c, hipGetLastError());
    FFTCHK(c, hipfftSetStream(c->inv, s));
    FFTCHK(c, hipfftExecZ2D(c->inv, (hipfftDoubleComplex *)rhat, (hipfftDoubleReal *)lrho));
    return APIC_OK;
}

// Velocities of p into a [3][n] block (Higuera-Cary snapshots).
apic_status save_vel(apic_ctx *c, const apic_particles &p, char *dst, hipStream_t s) {
    const int64_t n = c->n;
    const size_t r = c->mixed ? 4 : 8;
    HIPCHK(c, launch_copy_bytes(dst, p.vx, (int64_t)(r * n), s));
    HIPCHK(c, launch_copy_bytes(dst + r * n, p.vy, (int64_t)(r * n), s));
    HIPCHK(c, launch_copy_bytes(dst + 2 * r * n, p.vz, (int64_t)(r * n), s));
    return APIC_OK;
}

template <typename R>
void boris_consts(const apic_ctx *c, double dt_scale, R &a, R &t, R &s) {
    const PushC pc = push_coeffs(c, dt_scale, 1);
    if (c->mixed) {
        a = (R)pc.af;
        t = (R)pc.tf;
        s = (R)pc.sf;
    } else {
        a = (R)pc.a;
        t = (R)pc.t;
        s = (R)pc.s;
    }
}

template <typename R>
apic_status launch_level(apic_ctx *c, AdjP<R> &P, hipStream_t s) {
    P.g = c->g;
    P.n = c->n;
    P.err = c->dev.err;
    P.dt = (R)c->d.dt;
    P.cq = (R)(c->d.q_macro / c->dV);
    boris_consts<R>(c, 1.0, P.a, P.t, P.s);
    boris_consts<R>(c, -0.5, P.ah, P.th, P.sh);
    const PushC pc = push_coeffs(c, 1.0, 1);
    P.ic2 = c->mixed ? (R)pc.ic2f : (R)pc.ic2;
    // with the level's bucket table: one workgroup per bucket and the lam_Ep
    // scatter into an LDS tile (tile + 2-cell halo per scattered component)
    dim3 grid(nblocks(c->n));
    size_t sh = 0;
    if (c->d.dim == 3) P.bs = nullptr;   // 3D scatters lam_Ep with global atomics
    if (P.bs) {
        const int tw = (1 << c->g.tsx) + 5, th = c->d.dim == 2 ? (1 << c->g.tsy) + 5 : 1;
        sh = (size_t)c->d.dim * tw * th * sizeof(double);
        grid = dim3(grid_for_buckets(c->g.nbuckets));
        if (sh > 65536) {
            P.bs = nullptr;
            sh = 0;
            grid = dim3(nblocks(c->n));
        }
    }
    if (c->d.dim == 3) {
        if (c->mixed) {
            if constexpr (std::is_same<R, float>::value) {
                if (c->g.hc) hipLaunchKernelGGL((k_adj_level<true, 3, 3, true>), grid, dim3(kBlock), 0, s, P);
                else hipLaunchKernelGGL((k_adj_level<true, 3, 3, false>), grid, dim3(kBlock), 0, s, P);
            }
        } else {
            if constexpr (std::is_same<R, double>::value) {
                if (c->g.hc) hipLaunchKernelGGL((k_adj_level<false, 3, 3, true>), grid, dim3(kBlock), 0, s, P);
                else hipLaunchKernelGGL((k_adj_level<false, 3, 3, false>), grid, dim3(kBlock), 0, s, P);
            }
        }
    } else if (c->g.hc) {
        if (c->mixed) {
            if constexpr (std::is_same<R, float>::value)
                hipLaunchKernelGGL((k_adj_level<true, 2, 3, true>), grid, dim3(kBlock), sh, s, P);
        } else {
            if constexpr (std::is_same<R, double>::value)
                hipLaunchKernelGGL((k_adj_level<false, 2, 3, true>), grid, dim3(kBlock), sh, s, P);
        }
    } else {
        APIC_DISPATCH_2D(c->g, c->mixed, {
            if constexpr (std::is_same<R, typename RealOf<MIX>::T>::value)
                hipLaunchKernelGGL((k_adj_level<MIX, DIM, VDIM, false>), grid, dim3(kBlock), sh, s, P);
        });
    }
    HIPCHK(c, hipGetLastError());
    return APIC_OK;
}

apic_status check_adj_args(apic_ctx *c, int nsteps, int stride) {
    if (c->g.em) return fail(c, APIC_EUNSUPPORTED, "the adjoint covers the electrostatic step");
    if (c->g.walls) return fail(c, APIC_EUNSUPPORTED, "the adjoint covers periodic plasmas (no absorbing walls)");
    if (nsteps < 0) return fail(c, APIC_EINVAL, "nsteps must be >= 0");
    if (stride < 1) return fail(c, APIC_EINVAL, "checkpoint stride must be >= 1");
    if (c->n < 1) return fail(c, APIC_EINVAL, "the adjoint needs at least one particle");
    return APIC_OK;
}

template <typename R>
apic_status step_adjoint_impl(apic_ctx *c, char *ck, int nsteps, int stride, double seed, double *out_x,
                              double *out_y, double *out_z, double *out_vx, double *out_vy, double *out_vz, char *ws,
                              hipStream_t s) {
    const CkLayout CL = ck_layout(c);
    const AdjWs L = adj_layout(c, stride);
    const int64_t n = c->n;
    const int64_t G = (int64_t)c->d.nx * c->d.ny * c->d.nz;
    const int dim = c->d.dim;
    char *ws_ctx = ws + L.ctx;
    double *lE = wsp<double>(ws, L.lE);
    double *lrho = wsp<double>(ws, L.lrho);
    double *E_w = wsp<double>(ws, L.E);
    int32_t *id_w = wsp<int32_t>(ws, L.id_a), *id_t = wsp<int32_t>(ws, L.id_b);
    int32_t *inv = wsp<int32_t>(ws, L.inv), *cross = wsp<int32_t>(ws, L.cross);
    const int C = n_checkpoints(nsteps, stride);
    auto ckp = [&](int k) { return ck + (size_t)k * CL.bytes; };
    auto snap_pos = [&](int k) { return ws + L.snap_pos + (size_t)k * L.snap_pos_bytes; };
    auto snap_perm = [&](int k) { return (int32_t *)(ws + L.snap_perm + (size_t)k * align256(4 * n)); };
    auto snap_E = [&](int k) { return (double *)(ws + L.snap_E + (size_t)k * align256(8 * (size_t)dim * G)); };
    const size_t r = c->mixed ? 4 : 8;
    auto snap_vel = [&](int k) { return ws + L.snap_vel + (size_t)k * align256(r * 3 * n); };
    const size_t bs_bytes = 4 * (size_t)(c->g.nbuckets + 1);
    auto snap_bs = [&](int k) { return (int32_t *)(ws + L.snap_bs + (size_t)k * align256(bs_bytes)); };
    // level T: only the objective depends on E^T
    hipLaunchKernelGGL(k_adj_scale, dim3(nblocks(dim * G)), dim3(kBlock), 0, s, (int64_t)dim * G,
                       (const double *)(ckp(C) + CL.E), lE, seed * c->dV);
    HIPCHK(c, hipGetLastError());
    apic_status st = adj_solve(c, lE, lrho, ws_ctx, s);
    if (st != APIC_OK) return st;
    int cur = 0;
    bool terminal = true;
    apic_particles pw = work_parts(c, L, ws);
    for (int seg = C - 1; seg >= 0; --seg) {
        const int s0 = seg * stride, e = std::min(s0 + stride, nsteps), m = e - s0;
        // recompute the segment from its checkpoint
        st = ck_transfer(c, CL, ckp(seg), pw, E_w, id_w, -1, s);
        if (st != APIC_OK) return st;
        for (int k = 0; k < m; ++k) {
            st = save_pos(c, pw, snap_pos(k), s);
            if (st != APIC_OK) return st;
            if (c->g.hc) {
                st = save_vel(c, pw, snap_vel(k), s);
                if (st != APIC_OK) return st;
            }
            HIPCHK(c, launch_copy_bytes(snap_bs(k), pw.bucket_start, (int64_t)bs_bytes, s));
            HIPCHK(c, launch_copy_bytes(snap_E(k), E_w, 8 * (int64_t)dim * G, s));
            pw.perm = snap_perm(k);
            st = apic_step(c, &pw, nullptr, E_w, nullptr, 1, nullptr, ws_ctx, s);
            pw.perm = nullptr;
            if (st != APIC_OK) return st;
            hipLaunchKernelGGL(k_adj_compose_ids, dim3(nblocks(n)), dim3(kBlock), 0, s, n, id_w, snap_perm(k), id_t,
                               c->dev.err);
            HIPCHK(c, hipGetLastError());
            std::swap(id_w, id_t);
        }
        // the step that ends at the stored checkpoint maps through input indices
        hipLaunchKernelGGL(k_adj_invert, dim3(nblocks(n)), dim3(kBlock), 0, s, n, id_w, inv, c->dev.err);
        HIPCHK(c, hipGetLastError());
        hipLaunchKernelGGL(k_adj_cross_perm, dim3(nblocks(n)), dim3(kBlock), 0, s, n,
                           (const int32_t *)(ckp(seg + 1) + CL.id), inv, snap_perm(m - 1), cross, c->dev.err);
        HIPCHK(c, hipGetLastError());
        for (int lvl = e; lvl > s0; --lvl) {
            const int k = lvl - s0;
            AdjP<R> P{};
            P.pos = (lvl == e) ? pos_ck(c, CL, ckp(seg + 1)) : pos_block(c, snap_pos(k));
            P.E = (lvl == e) ? (const double *)(ckp(seg + 1) + CL.E) : snap_E(k);
            P.bs = (lvl == e) ? (const int32_t *)(ckp(seg + 1) + CL.bstart) : snap_bs(k);
            P.lrho = lrho;
            P.lxp_in = wsp<R>(ws, L.lam[cur][0]);
            P.lep_in = wsp<R>(ws, L.lam[cur][1]);
            P.lv_in = wsp<R>(ws, L.lam[cur][2]);
            P.terminal = terminal ? 1 : 0;
            P.back = 1;
            P.perm = (lvl == e) ? cross : snap_perm(k - 1);
            P.prev = pos_block(c, snap_pos(k - 1));
            P.lE_prev = lE;
            P.lxp_out = wsp<R>(ws, L.lam[cur ^ 1][0]);
            P.lep_out = wsp<R>(ws, L.lam[cur ^ 1][1]);
            P.lv_out = wsp<R>(ws, L.lam[cur ^ 1][2]);
            P.init = (lvl - 1 == 0) ? 1 : 0;
            if (c->g.hc) {
                P.vprev = (const R *)snap_vel(k - 1);
                P.Eprev = snap_E(k - 1);
            }
            hipLaunchKernelGGL(k_adj_fill, dim3(nblocks(dim * G)), dim3(kBlock), 0, s, (int64_t)dim * G, lE);
            HIPCHK(c, hipGetLastError());
            st = launch_level<R>(c, P, s);
            if (st != APIC_OK) return st;
            cur ^= 1;
            terminal = false;
            st = adj_solve(c, lE, lrho, ws_ctx, s);
            if (st != APIC_OK) return st;
        }
    }
    // level 0: deposit and gather adjoints at x^0, then the outputs in input order
    AdjP<R> P{};
    P.pos = pos_ck(c, CL, ckp(0));
    P.E = (const double *)(ckp(0) + CL.E);
    P.lrho = lrho;
    P.lxp_in = wsp<R>(ws, L.lam[cur][0]);
    P.lep_in = wsp<R>(ws, L.lam[cur][1]);
    P.lv_in = wsp<R>(ws, L.lam[cur][2]);
    P.terminal = terminal ? 1 : 0;
    P.final_out = 1;
    P.id0 = (const int32_t *)(ckp(0) + CL.id);
    P.out_x = out_x;
    P.out_y = out_y;
    P.out_z = out_z;
    P.out_vx = out_vx;
    P.out_vy = out_vy;
    P.out_vz = out_vz;
    return launch_level<R>(c, P, s);
}

}  // namespace

extern "C" {

apic_status apic_import_state(apic_ctx *c, const double *x, const double *y, const double *z, const double *vx,
                              const double *vy, const double *vz, apic_particles *p, void *stream) {
    if (!c) return APIC_EINVAL;
    if (c->g.walls) return fail(c, APIC_EUNSUPPORTED, "state import covers periodic plasmas");
    apic_status st = check_parts(c, p, false);
    if (st != APIC_OK) return st;
    if (!x || (c->d.dim >= 2 && !y) || (c->d.dim == 3 && !z) || !vx || (c->d.vdim >= 2 && !vy) ||
        (c->d.vdim >= 3 && !vz))
        return fail(c, APIC_EINVAL, "a state array is NULL");
    hipStream_t s = (hipStream_t)stream;
    const double dx = c->d.lx / c->d.nx, dy = c->d.dim >= 2 ? c->d.ly / c->d.ny : 1.0;
    const double dz = c->d.dim == 3 ? c->d.lz / c->d.nz : 1.0;
    const Parts out = parts_of(p);
    APIC_DISPATCH(c->g, c->mixed,
                  hipLaunchKernelGGL((k_import<MIX, DIM, VDIM>), dim3(nblocks(c->n)), dim3(kBlock), 0, s, c->g, c->n,
                                     dx, dy, dz, x, y, z, vx, vy, vz, out, c->dev.err));
    HIPCHK(c, hipGetLastError());
    return APIC_OK;
}

apic_status apic_adjoint_sizes(const apic_ctx *c, int nsteps, int stride, size_t *ckpt_bytes, size_t *ws_bytes) {
    if (!c || nsteps < 0 || stride < 1) return APIC_EINVAL;
    if (c->g.em || c->g.walls) return APIC_EUNSUPPORTED;
    const CkLayout CL = ck_layout(c);
    if (ckpt_bytes) *ckpt_bytes = CL.bytes * (size_t)(n_checkpoints(nsteps, stride) + 1);
    if (ws_bytes) *ws_bytes = adj_layout(c, stride).bytes;
    return APIC_OK;
}

apic_status apic_adjoint_forward(apic_ctx *c, const apic_particles *p0, int nsteps, int stride, void *ckpt,
                                 double *W, double *E_out, void *ws, void *stream) {
    if (!c) return APIC_EINVAL;
    apic_status st = check_parts(c, p0, false);
    if (st != APIC_OK) return st;
    st = check_adj_args(c, nsteps, stride);
    if (st != APIC_OK) return st;
    if (!ckpt || !ws) return fail(c, APIC_EINVAL, "checkpoint buffer and workspace are required");
    hipStream_t s = (hipStream_t)stream;
    const CkLayout CL = ck_layout(c);
    const AdjWs L = adj_layout(c, stride);
    char *w = (char *)ws, *ck = (char *)ckpt;
    char *ws_ctx = w + L.ctx;
    const int64_t n = c->n;
    const int64_t G = (int64_t)c->d.nx * c->d.ny * c->d.nz;
    const int dim = c->d.dim;
    double *E_w = wsp<double>(w, L.E);
    float *E32_w = wsp<float>(w, L.E32);
    int32_t *id_w = wsp<int32_t>(w, L.id_a), *id_t = wsp<int32_t>(w, L.id_b);
    int32_t *perm = wsp<int32_t>(w, L.inv);
    apic_particles pw = work_parts(c, L, w);
    // x^0, v^0 in the caller's order -> sorted copy; id = input index
    st = copy_parts(c, parts_of(&pw), parts_of(p0), s);
    if (st != APIC_OK) return st;
    pw.perm = id_w;
    st = apic_sort_by_cell(c, &pw, ws_ctx, s);
    pw.perm = nullptr;
    if (st != APIC_OK) return st;
    // E^0, then the backward half push
    st = apic_deposit(c, &pw, wsp<void>(w, L.rho), s);
    if (st != APIC_OK) return st;
    st = apic_field_solve(c, wsp<void>(w, L.rho), E_w, c->mixed ? E32_w : nullptr, nullptr, ws_ctx, s);
    if (st != APIC_OK) return st;
    st = apic_gather_push(c, &pw, c->mixed ? (const void *)E32_w : (const void *)E_w, -0.5, 0, s);
    if (st != APIC_OK) return st;
    st = ck_transfer(c, CL, ck, pw, E_w, id_w, +1, s);
    if (st != APIC_OK) return st;
    for (int k = 0; k < nsteps; ++k) {
        pw.perm = perm;
        st = apic_step(c, &pw, nullptr, E_w, nullptr, 1, nullptr, ws_ctx, s);
        pw.perm = nullptr;
        if (st != APIC_OK) return st;
        hipLaunchKernelGGL(k_adj_compose_ids, dim3(nblocks(n)), dim3(kBlock), 0, s, n, id_w, perm, id_t, c->dev.err);
        HIPCHK(c, hipGetLastError());
        std::swap(id_w, id_t);
        if ((k + 1) % stride == 0 || k + 1 == nsteps) {
            const int idx = (k + 1 + stride - 1) / stride;
            st = ck_transfer(c, CL, ck + (size_t)idx * CL.bytes, pw, E_w, id_w, +1, s);
            if (st != APIC_OK) return st;
        }
    }
    if (W) {
        hipLaunchKernelGGL(k_adj_energy, dim3(1), dim3(1024), 0, s, (int64_t)dim * G, E_w, c->dV, W);
        HIPCHK(c, hipGetLastError());
    }
    if (E_out) HIPCHK(c, launch_copy_bytes(E_out, E_w, 8 * (int64_t)dim * G, s));
    return APIC_OK;
}

apic_status apic_step_adjoint(apic_ctx *c, const void *ckpt, int nsteps, int stride, double seed, double *lam_x,
                              double *lam_y, double *lam_z, double *lam_vx, double *lam_vy, double *lam_vz,
                              const double *dx_ddelta0, const double *dy_ddelta0, double *grad_delta0, void *ws,
                              void *stream) {
    if (!c) return APIC_EINVAL;
    apic_status st = check_adj_args(c, nsteps, stride);
    if (st != APIC_OK) return st;
    if (!ckpt || !ws) return fail(c, APIC_EINVAL, "checkpoint buffer and workspace are required");
    if (!lam_x || (c->d.dim >= 2 && !lam_y) || (c->d.dim == 3 && !lam_z) || !lam_vx || (c->d.vdim >= 2 && !lam_vy) ||
        (c->d.vdim >= 3 && !lam_vz))
        return fail(c, APIC_EINVAL, "a gradient output array is NULL");
    if (!std::isfinite(seed)) return fail(c, APIC_EINVAL, "seed is not finite");
    if (grad_delta0 && (!dx_ddelta0 || (c->d.dim >= 2 && !dy_ddelta0)))
        return fail(c, APIC_EINVAL, "grad_delta0 needs the displacement direction of every particle (dx, dy in 2D)");
    hipStream_t s = (hipStream_t)stream;
    if (c->mixed)
        st = step_adjoint_impl<float>(c, (char *)const_cast<void *>(ckpt), nsteps, stride, seed, lam_x, lam_y, lam_z,
                                      lam_vx, lam_vy, lam_vz, (char *)ws, s);
    else
        st = step_adjoint_impl<double>(c, (char *)const_cast<void *>(ckpt), nsteps, stride, seed, lam_x, lam_y,
                                       lam_z, lam_vx, lam_vy, lam_vz, (char *)ws, s);
    if (st != APIC_OK || !grad_delta0) return st;
    hipLaunchKernelGGL(apic::k_adj_delta0, dim3(1), dim3(1024), 0, s, c->n, lam_x, dx_ddelta0,
                       c->d.dim >= 2 ? lam_y : nullptr, c->d.dim >= 2 ? dy_ddelta0 : nullptr, grad_delta0);
    HIPCHK(c, hipGetLastError());
    return APIC_OK;
}

}  // extern "C"
