// Device helpers shared by the HIP translation units of libapic: the particle
// model (cell + offset or FP64 position), the CIC weights, the Boris advance,
// the move with periodic wrap, LDS tile helpers and fixed-order reductions.
// Every kernel that advances or deposits particles uses these, so the fused
// step, the standalone entry points and the batched replicas compute the same
// bits for the same particle.
#pragma once

#include "apic_internal.h"

#include <math.h>

namespace apic {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ void raise_err(int *err, int bit) { atomicOr(err, bit); }

// s_waitcnt immediate (gfx9 layout) for vmcnt(0) with expcnt and lgkmcnt left
// at their maximum: waits for every vector-memory load and store in flight.
constexpr int kWaitVmem = 0x0F70;

__device__ __forceinline__ uint64_t lanemask_lt() {
    const unsigned lane = __lane_id();
    return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

// XCD-aware bucket for this workgroup: workgroups are dispatched round-robin
// over the 8 XCDs, so block i runs on XCD i % 8; give XCD k the contiguous
// bucket range [k*per, (k+1)*per).
__device__ __forceinline__ int bucket_of_block(int nbuckets) {
    const int per = (nbuckets + 7) >> 3;
    const int b = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    return b;
}

inline int grid_for_buckets(int nbuckets) { return ((nbuckets + 7) >> 3) << 3; }

// Persistent launches: gridDim.x (a multiple of 8) blocks walk the buckets.
// Block i runs on XCD i % 8 and takes every (gridDim.x/8)-th bucket of that
// XCD's contiguous bucket range, so neighbouring tiles share an L2.
__device__ __forceinline__ void bucket_walk(int nbuckets, int &first, int &end, int &stride) {
    const int per = (nbuckets + 7) >> 3;
    const int x = (int)(blockIdx.x & 7);
    first = x * per + (int)(blockIdx.x >> 3);
    end = min((x + 1) * per, nbuckets);
    stride = (int)(gridDim.x >> 3);
}

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Block-wide sum, deterministic (fixed tree); result valid in every thread.
__device__ double block_sum(double v, double *sh /* [waves] */) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    __syncthreads();
    return t;
}

__device__ __forceinline__ double *step_slot(double *base, const CtxDev &c) {
    return base ? base + 4 * (*c.step) : nullptr;
}

// ------------------------------------------------------------ particle model

template <bool MIX> struct RealOf { using T = double; };
template <> struct RealOf<true> { using T = float; };

template <bool MIX>
struct Pt {
    using R = typename RealOf<MIX>::T;
    int ix, iy;       // cell indices
    R fx, fy;         // fractional position inside the cell
    double x, y;      // absolute position (FP64 path only)
    R vx, vy, vz;
};

// FP64 cell of a coordinate: i = floor(x/d), f = x/d - i, computed with
// x * (1/d). A coordinate that rounds onto the right edge wraps to node 0.
__device__ __forceinline__ bool cell_f64(double x, double inv_d, int n, int &i, double &f) {
    double gx = x * inv_d;
    double fl = floor(gx);
    f = gx - fl;
    bool ok = (gx >= 0.0) && (gx <= (double)n);
    i = ok ? (int)fl : 0;
    if (i >= n) i -= n;
    if (!ok) f = 0.0;
    return ok;
}

template <bool MIX, int DIM, int VDIM>
__device__ __forceinline__ bool load_pt(const Parts &s, int64_t i, const Geo &g, Pt<MIX> &p) {
    using R = typename Pt<MIX>::R;
    bool ok = true;
    if constexpr (MIX) {
        int32_t c = s.cell[i];
        if constexpr (DIM == 2) {
            p.ix = c & 0xFFFF;
            p.iy = c >> 16;
            p.fy = s.oy[i];
            ok = (p.iy >= 0) && (p.iy < g.ny) && (p.fy >= 0.0f) && (p.fy < 1.0f);
        } else {
            p.ix = c;
            p.iy = 0;
            p.fy = 0.0f;
        }
        p.fx = s.ox[i];
        ok = ok && (p.ix >= 0) && (p.ix < g.nx) && (p.fx >= 0.0f) && (p.fx < 1.0f);
        if (!ok) { p.ix = 0; p.iy = 0; p.fx = 0.0f; p.fy = 0.0f; }
    } else {
        p.x = s.x[i];
        double f;
        ok = cell_f64(p.x, g.inv_dx, g.nx, p.ix, f);
        p.fx = f;
        if constexpr (DIM == 2) {
            p.y = s.y[i];
            ok = cell_f64(p.y, g.inv_dy, g.ny, p.iy, f) && ok;
            p.fy = f;
        } else {
            p.y = 0.0;
            p.iy = 0;
            p.fy = 0.0;
        }
    }
    p.vx = ((const R *)s.vx)[i];
    p.vy = (VDIM >= 2) ? ((const R *)s.vy)[i] : R(0);
    p.vz = (VDIM >= 3) ? ((const R *)s.vz)[i] : R(0);
    return ok;
}

template <bool MIX, int DIM, int VDIM>
__device__ __forceinline__ void store_pt(const Parts &d, int64_t j, const Pt<MIX> &p) {
    using R = typename Pt<MIX>::R;
    if constexpr (MIX) {
        d.cell[j] = (DIM == 2) ? ((p.iy << 16) | p.ix) : p.ix;
        d.ox[j] = p.fx;
        if constexpr (DIM == 2) d.oy[j] = p.fy;
    } else {
        d.x[j] = p.x;
        if constexpr (DIM == 2) d.y[j] = p.y;
    }
    ((R *)d.vx)[j] = p.vx;
    if constexpr (VDIM >= 2) ((R *)d.vy)[j] = p.vy;
    if constexpr (VDIM >= 3) ((R *)d.vz)[j] = p.vz;
}

template <bool MIX, int DIM>
__device__ __forceinline__ int bucket_of(const Geo &g, int ix, int iy) {
    int bx = ix >> g.tsx;
    if constexpr (DIM == 2) return (iy >> g.tsy) * g.nbx + bx;
    return bx;
}

// Boris advance: half kick, rotation about z, half kick (Boris 1970).
// With t = 0 (no magnetic field) the rotation terms are exact zeros, so the
// uniform branch that skips them gives the same bits as the full formula.
template <typename R, int VDIM>
__device__ __forceinline__ void boris(R &vx, R &vy, R ex, R ey, R a, R t, R s) {
    if constexpr (VDIM == 1) {
        R m1 = vx + a * ex;
        vx = m1 + a * ex;
    } else {
        R mx = vx + a * ex;
        R my = vy + a * ey;
        if (t != R(0)) {
            R px = mx + my * t;
            R py = my - mx * t;
            R qx = mx + py * s;
            R qy = my - px * s;
            mx = qx;
            my = qy;
        }
        vx = mx + a * ex;
        vy = my + a * ey;
    }
}

// Position update with periodic wrap. Returns the unwrapped cell shift
// (new cell - old cell) per axis in sx, sy, and false for a non-finite or
// runaway coordinate.
template <bool MIX, int DIM>
__device__ __forceinline__ bool move_pt(Pt<MIX> &p, const Geo &g, const PushC &pc, int &sx, int &sy) {
    if constexpr (MIX) {
        bool ok = true;
        float o = p.fx + p.vx * pc.dtdx;
        float fl = floorf(o);
        o = o - fl;
        ok = ok && (fabsf(fl) < 1.0e8f);
        int sh = ok ? (int)fl : 0;
        if (o >= 1.0f) { o = o - 1.0f; sh += 1; }
        int ix = p.ix + sh;
        if (ix >= g.nx || ix < 0) { ix %= g.nx; if (ix < 0) ix += g.nx; }
        p.ix = ix;
        p.fx = ok ? o : 0.0f;
        sx = sh;
        sy = 0;
        if constexpr (DIM == 2) {
            float q = p.fy + p.vy * pc.dtdy;
            float fq = floorf(q);
            q = q - fq;
            bool oky = fabsf(fq) < 1.0e8f;
            int shy = oky ? (int)fq : 0;
            if (q >= 1.0f) { q = q - 1.0f; shy += 1; }
            int iy = p.iy + shy;
            if (iy >= g.ny || iy < 0) { iy %= g.ny; if (iy < 0) iy += g.ny; }
            p.iy = iy;
            p.fy = oky ? q : 0.0f;
            sy = shy;
            ok = ok && oky;
        }
        return ok;
    } else {
        const int ix0 = p.ix, iy0 = p.iy;
        double x = p.x + p.vx * pc.dt;
        if (x < 0.0) x += g.lx;
        if (x >= g.lx) x -= g.lx;
        if (!(x >= 0.0 && x < g.lx)) {
            x = x - g.lx * floor(x / g.lx);
            if (!(x >= 0.0 && x < g.lx)) x = 0.0;
        }
        p.x = x;
        double f;
        bool ok = cell_f64(x, g.inv_dx, g.nx, p.ix, f);
        p.fx = f;
        int d = p.ix - ix0;
        if (d > g.nx / 2) d -= g.nx;
        if (d < -(g.nx / 2)) d += g.nx;
        sx = d;
        sy = 0;
        if constexpr (DIM == 2) {
            double y = p.y + p.vy * pc.dt;
            if (y < 0.0) y += g.ly;
            if (y >= g.ly) y -= g.ly;
            if (!(y >= 0.0 && y < g.ly)) {
                y = y - g.ly * floor(y / g.ly);
                if (!(y >= 0.0 && y < g.ly)) y = 0.0;
            }
            p.y = y;
            ok = cell_f64(y, g.inv_dy, g.ny, p.iy, f) && ok;
            p.fy = f;
            int e = p.iy - iy0;
            if (e > g.ny / 2) e -= g.ny;
            if (e < -(g.ny / 2)) e += g.ny;
            sy = e;
        }
        return ok;
    }
}

// Fixed-point CIC weight along one axis: round-half-even(o * 2^S).
__device__ __forceinline__ int64_t qw1(float o, float scale) {
    return (int64_t)rintf(o * scale);
}

// ------------------------------------------------------- LDS tile helpers

// E tile: nodes [x0, x0+TX] x [y0, y0+TY] (periodic), comps [DIM], converted
// to the push precision R on the way into LDS.
template <typename R, typename ET, int DIM>
__device__ void load_e_tile(R *sE, const ET *E, const Geo &g, int x0, int y0, int wx, int wy) {
    const int G = g.nx * g.ny;
    const int tot = wx * wy;
    for (int t = threadIdx.x; t < tot; t += blockDim.x) {
        int lx = t % wx, ly = t / wx;
        int gx = x0 + lx;
        if (gx >= g.nx) gx -= g.nx;
        int gy = y0 + ly;
        if (gy >= g.ny) gy -= g.ny;
        int gi = gy * g.nx + gx;
        sE[t] = (R)E[gi];
        if constexpr (DIM == 2) sE[tot + t] = (R)E[G + gi];
    }
}

template <typename R, int DIM>
__device__ __forceinline__ void gather_lds(const R *sE, int wx, int tot, int lx, int ly, R fx, R fy,
                                           R &ex, R &ey) {
    if constexpr (DIM == 1) {
        ex = (R(1) - fx) * sE[lx] + fx * sE[lx + 1];
        ey = R(0);
    } else {
        R w00 = (R(1) - fx) * (R(1) - fy), w10 = fx * (R(1) - fy);
        R w01 = (R(1) - fx) * fy, w11 = fx * fy;
        int a00 = ly * wx + lx;
        ex = w00 * sE[a00] + w10 * sE[a00 + 1] + w01 * sE[a00 + wx] + w11 * sE[a00 + wx + 1];
        ey = w00 * sE[tot + a00] + w10 * sE[tot + a00 + 1] + w01 * sE[tot + a00 + wx] +
             w11 * sE[tot + a00 + wx + 1];
    }
}

// Same interpolation from the global field (node values converted to R first,
// exactly as the LDS tile holds them).
template <typename R, typename ET, int DIM>
__device__ __forceinline__ void gather_global(const ET *E, const Geo &g, int ix, int iy, R fx, R fy,
                                              R &ex, R &ey) {
    int ip = ix + 1;
    if (ip >= g.nx) ip = 0;
    if constexpr (DIM == 1) {
        ex = (R(1) - fx) * (R)E[ix] + fx * (R)E[ip];
        ey = R(0);
    } else {
        const int G = g.nx * g.ny;
        int jp = iy + 1;
        if (jp >= g.ny) jp = 0;
        R w00 = (R(1) - fx) * (R(1) - fy), w10 = fx * (R(1) - fy);
        R w01 = (R(1) - fx) * fy, w11 = fx * fy;
        int a00 = iy * g.nx + ix, a10 = iy * g.nx + ip, a01 = jp * g.nx + ix, a11 = jp * g.nx + ip;
        ex = w00 * (R)E[a00] + w10 * (R)E[a10] + w01 * (R)E[a01] + w11 * (R)E[a11];
        ey = w00 * (R)E[G + a00] + w10 * (R)E[G + a10] + w01 * (R)E[G + a01] + w11 * (R)E[G + a11];
    }
}

// Accumulator element: double weights (FP64 path) or int64 fixed-point sums.
template <bool MIX> struct AccOf { using T = double; };
template <> struct AccOf<true> { using T = unsigned long long; };

template <bool MIX>
__device__ __forceinline__ void acc_add(typename AccOf<MIX>::T *a, typename AccOf<MIX>::T v) {
    atomicAdd(a, v);
}

// CIC weights of a particle at (fx, fy) as accumulator values. Fixed point:
// w1 = round-half-even(o 2^S) (o 2^S is exact in binary32), w0 = 2^S - w1;
// in 2D (S <= 23) both fit 24 bits and the node weight is their exact 48-bit
// product (24-bit multiplies).
template <bool MIX, int DIM>
__device__ __forceinline__ void dep_weights(const Pt<MIX> &p, const Geo &g,
                                            typename AccOf<MIX>::T w[4]) {
    if constexpr (MIX) {
        const float scale = (float)(1ull << g.S);
        if constexpr (DIM == 1) {
            const unsigned long long w1 = (uint32_t)rintf(p.fx * scale);
            w[0] = (1ull << g.S) - w1;
            w[1] = w1;
        } else {
            const uint32_t one = 1u << g.S;
            const uint32_t w1x = (uint32_t)rintf(p.fx * scale) & 0xFFFFFFu;
            const uint32_t w0x = (one - w1x) & 0xFFFFFFu;
            const uint32_t w1y = (uint32_t)rintf(p.fy * scale) & 0xFFFFFFu;
            const uint32_t w0y = (one - w1y) & 0xFFFFFFu;
            w[0] = (unsigned long long)w0x * w0y;
            w[1] = (unsigned long long)w1x * w0y;
            w[2] = (unsigned long long)w0x * w1y;
            w[3] = (unsigned long long)w1x * w1y;
        }
    } else {
        double fx = p.fx, fy = p.fy;
        if constexpr (DIM == 1) {
            w[0] = 1.0 - fx;
            w[1] = fx;
        } else {
            w[0] = (1.0 - fx) * (1.0 - fy);
            w[1] = fx * (1.0 - fy);
            w[2] = (1.0 - fx) * fy;
            w[3] = fx * fy;
        }
    }
}

template <bool MIX, int DIM>
__device__ __forceinline__ void deposit_global(typename AccOf<MIX>::T *acc, const Geo &g, int ix, int iy,
                                               const typename AccOf<MIX>::T w[4]) {
    int ip = ix + 1;
    if (ip >= g.nx) ip = 0;
    if constexpr (DIM == 1) {
        acc_add<MIX>(&acc[ix], w[0]);
        acc_add<MIX>(&acc[ip], w[1]);
    } else {
        int jp = iy + 1;
        if (jp >= g.ny) jp = 0;
        acc_add<MIX>(&acc[iy * g.nx + ix], w[0]);
        acc_add<MIX>(&acc[iy * g.nx + ip], w[1]);
        acc_add<MIX>(&acc[jp * g.nx + ix], w[2]);
        acc_add<MIX>(&acc[jp * g.nx + ip], w[3]);
    }
}

// Flush an LDS deposit region (nodes [x0-H, x0+TX+H] x [y0-H, y0+TY+H]) to
// global memory with one atomic per non-zero node.
template <bool MIX, int DIM>
__device__ void flush_region(typename AccOf<MIX>::T *acc, const typename AccOf<MIX>::T *sA, const Geo &g,
                             int x0, int y0, int wx, int wy, int halo) {
    const int tot = wx * wy;
    for (int t = threadIdx.x; t < tot; t += blockDim.x) {
        typename AccOf<MIX>::T v = sA[t];
        if (v == (typename AccOf<MIX>::T)0) continue;
        int lx = t % wx, ly = t / wx;
        int gx = x0 - halo + lx;
        gx %= g.nx;
        if (gx < 0) gx += g.nx;
        int gy = 0;
        if constexpr (DIM == 2) {
            gy = y0 - halo + ly;
            gy %= g.ny;
            if (gy < 0) gy += g.ny;
        }
        acc_add<MIX>(&acc[gy * g.nx + gx], v);
    }
}

// 1D periodic field by Gauss's law on the half nodes (identical to the FFT
// solve of the 3-point Laplacian with centred gradient):
//   E_{j+1/2} = E_{j-1/2} + (rho_j - <rho>) dx,  sum_j E_{j+1/2} = 0,
//   E_j = (E_{j-1/2} + E_{j+1/2}) / 2.
// Whole workgroup (blockDim.x threads, multiple of 64); sr[nx] in LDS holds
// rho on entry and is overwritten. Returns sum_j E_j^2 and writes E (and E32
// when non-NULL). The association order of every sum depends only on nx and
// blockDim.x.
__device__ double field1d_block(double *sr, int nx, double dx, double *E, float *E32, double *sRed,
                                double *sScan) {
    const int T = blockDim.x;
    double ps = 0.0;
    for (int i = threadIdx.x; i < nx; i += T) ps += sr[i];
    const double mean = block_sum(ps, sRed) / (double)nx;
    const int per = (nx + T - 1) / T;
    const int lo = threadIdx.x * per, hi = min(nx, lo + per);
    double loc = 0.0;
    for (int i = lo; i < hi; ++i) loc += (sr[i] - mean) * dx;
    sScan[threadIdx.x] = loc;
    __syncthreads();
    for (int off = 1; off < T; off <<= 1) {
        double addv = (threadIdx.x >= (unsigned)off) ? sScan[threadIdx.x - off] : 0.0;
        __syncthreads();
        sScan[threadIdx.x] += addv;
        __syncthreads();
    }
    double run = sScan[threadIdx.x] - loc;
    __syncthreads();
    for (int i = lo; i < hi; ++i) {
        run += (sr[i] - mean) * dx;
        sr[i] = run;                       // E_{i+1/2} up to a constant
    }
    __syncthreads();
    double hs = 0.0;
    for (int i = threadIdx.x; i < nx; i += T) hs += sr[i];
    const double hmean = block_sum(hs, sRed) / (double)nx;
    double wpart = 0.0;
    for (int i = threadIdx.x; i < nx; i += T) {
        const int im = (i == 0) ? nx - 1 : i - 1;
        const double e = 0.5 * ((sr[im] - hmean) + (sr[i] - hmean));
        E[i] = e;
        if (E32) E32[i] = (float)e;
        wpart += e * e;
    }
    const double wsum = block_sum(wpart, sRed);
    __syncthreads();
    return wsum;
}

}  // namespace
}  // namespace apic

// Particles per thread and pipeline stage in the fused step kernels.
#ifndef APIC_STEP_U
#define APIC_STEP_U 1
#endif

// Instantiates a statement for the precision / dimension combination of a
// launch: MIX, DIM, VDIM (and the unroll factor U) are constexpr inside.
#define APIC_DISPATCH(g, mixed, ...)                                                    \
    do {                                                                                \
        if (mixed) {                                                                    \
            constexpr bool MIX = true;                                                  \
            [[maybe_unused]] constexpr int U = APIC_STEP_U;                                       \
            if ((g).dim == 1) { [[maybe_unused]] constexpr int DIM = 1, VDIM = 1; __VA_ARGS__; }         \
            else if ((g).vdim == 2) { [[maybe_unused]] constexpr int DIM = 2, VDIM = 2; __VA_ARGS__; }   \
            else { [[maybe_unused]] constexpr int DIM = 2, VDIM = 3; __VA_ARGS__; }                      \
        } else {                                                                        \
            constexpr bool MIX = false;                                                 \
            [[maybe_unused]] constexpr int U = APIC_STEP_U;                                       \
            if ((g).dim == 1) { [[maybe_unused]] constexpr int DIM = 1, VDIM = 1; __VA_ARGS__; }         \
            else if ((g).vdim == 2) { [[maybe_unused]] constexpr int DIM = 2, VDIM = 2; __VA_ARGS__; }   \
            else { [[maybe_unused]] constexpr int DIM = 2, VDIM = 3; __VA_ARGS__; }                      \
        }                                                                               \
    } while (0)
