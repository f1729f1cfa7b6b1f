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

// ---- exact charge of fixed-point node sums ------------------------------------
// A node sum I of the mixed deposit counts weight units of 2^-sd particle
// (sd = S * dim). It splits exactly into whole particles, I >> sd, and a
// remainder, I & (2^sd - 1). Both parts are summed in 64-bit integers, each
// remainder carried into the whole part once it reaches 2^sd, so no sum can
// overflow (the total of a grid, N 2^sd units, would overflow int64 for
// N 2^sd >= 2^63) and the result is exact and independent of the order of
// the additions. A correct deposit of N particles sums to N whole particles
// and a zero remainder.
struct QSum {
    int64_t whole;
    uint64_t rem;
};

__device__ __forceinline__ void qsum_add(QSum &q, int64_t I, int sd) {
    const uint64_t mask = (1ull << sd) - 1;
    q.whole += I >> sd;
    q.rem += (uint64_t)I & mask;
    q.whole += (int64_t)(q.rem >> sd);
    q.rem &= mask;
}

// Wave sums (64 remainders below 2^sd stay below 2^(sd+6) <= 2^54), then the
// block's waves in order: the normalised block total, valid in thread 0.
__device__ QSum qsum_block(QSum q, int sd) {
    __shared__ int64_t sQw[16];
    __shared__ uint64_t sQr[16];
    for (int off = 32; off > 0; off >>= 1) {
        q.whole += __shfl_xor(q.whole, off);
        q.rem += __shfl_xor(q.rem, off);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sQw[w] = q.whole;
        sQr[w] = q.rem;
    }
    __syncthreads();
    QSum t{0, 0};
    if (threadIdx.x == 0) {
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            t.whole += sQw[i];
            t.rem += sQr[i];
            t.whole += (int64_t)(t.rem >> sd);
            t.rem &= (1ull << sd) - 1;
        }
    }
    __syncthreads();
    return t;
}

// The block total added with one integer atomic each for the whole part and
// the remainder, into one of kQSlots counter pairs (one 128-byte line each,
// picked by the block index: hundreds of blocks adding to a single pair
// serialise on it) read by a later launch. Integer sums: exact in any order.
__device__ void qsum_flush(QSum q, int sd, unsigned long long *acc) {
    const QSum t = qsum_block(q, sd);
    if (threadIdx.x == 0) {
        unsigned long long *a = acc + (size_t)(blockIdx.x % kQSlots) * kQStride;
        if (t.whole) atomicAdd(&a[0], (unsigned long long)t.whole);
        if (t.rem) atomicAdd(&a[1], (unsigned long long)t.rem);
    }
}

// The normalised total of every slot, which are then cleared for the next
// solve (the whole workgroup of a launch after every launch that added to
// them; valid in thread 0).
__device__ QSum qsum_take(unsigned long long *acc, int sd) {
    QSum t{0, 0};
    for (int i = threadIdx.x; i < kQSlots; i += blockDim.x) {
        unsigned long long *a = acc + (size_t)i * kQStride;
        t.whole += (int64_t)a[0];
        t.rem += a[1];
        t.whole += (int64_t)(t.rem >> sd);
        t.rem &= (1ull << sd) - 1;
        a[0] = 0ull;
        a[1] = 0ull;
    }
    return qsum_block(t, sd);
}

// Charge of an exact particle count whole + rem 2^-sd.
__device__ __forceinline__ double qsum_charge(const QSum &t, int sd, double q_macro) {
    return q_macro * ((double)t.whole + ldexp((double)t.rem, -sd));
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
    int ix, iy, iz;   // cell indices
    R fx, fy, fz;     // fractional position inside the cell
    double x, y, z;   // absolute position (FP64 path only)
    R vx, vy, vz;
};

// Mixed-path cell word: ix (1D), iy << 16 | ix (2D), iz << 20 | iy << 10 | ix
// (3D, at most 1024 nodes per axis).
template <int DIM>
__device__ __forceinline__ void unpack_cell(int32_t c, int &ix, int &iy, int &iz) {
    if constexpr (DIM == 1) {
        ix = c; iy = 0; iz = 0;
    } else if constexpr (DIM == 2) {
        ix = c & 0xFFFF; iy = c >> 16; iz = 0;
    } else {
        ix = c & 0x3FF; iy = (c >> 10) & 0x3FF; iz = c >> 20;
    }
}

template <int DIM>
__device__ __forceinline__ int32_t pack_cell(int ix, int iy, int iz) {
    if constexpr (DIM == 1) return ix;
    if constexpr (DIM == 2) return (iy << 16) | ix;
    return (iz << 20) | (iy << 10) | ix;
}

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
        unpack_cell<DIM>(s.cell[i], p.ix, p.iy, p.iz);
        p.fx = s.ox[i];
        p.fy = (DIM >= 2) ? s.oy[i] : 0.0f;
        p.fz = (DIM == 3) ? s.oz[i] : 0.0f;
        ok = (p.ix >= 0) && (p.ix < g.nx) && (p.fx >= 0.0f) && (p.fx < 1.0f);
        if constexpr (DIM >= 2) ok = ok && (p.iy >= 0) && (p.iy < g.ny) && (p.fy >= 0.0f) && (p.fy < 1.0f);
        if constexpr (DIM == 3) ok = ok && (p.iz >= 0) && (p.iz < g.nz) && (p.fz >= 0.0f) && (p.fz < 1.0f);
        if (!ok) { p.ix = 0; p.iy = 0; p.iz = 0; p.fx = 0.0f; p.fy = 0.0f; p.fz = 0.0f; }
    } else {
        p.x = s.x[i];
        double f;
        ok = cell_f64(p.x, g.inv_dx, g.nx, p.ix, f);
        p.fx = f;
        p.y = 0.0; p.iy = 0; p.fy = 0.0;
        p.z = 0.0; p.iz = 0; p.fz = 0.0;
        if constexpr (DIM >= 2) {
            p.y = s.y[i];
            ok = cell_f64(p.y, g.inv_dy, g.ny, p.iy, f) && ok;
            p.fy = f;
        }
        if constexpr (DIM == 3) {
            p.z = s.z[i];
            ok = cell_f64(p.z, g.inv_dz, g.nz, p.iz, f) && ok;
            p.fz = f;
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
        d.cell[j] = pack_cell<DIM>(p.ix, p.iy, p.iz);
        d.ox[j] = p.fx;
        if constexpr (DIM >= 2) d.oy[j] = p.fy;
        if constexpr (DIM == 3) d.oz[j] = p.fz;
    } else {
        d.x[j] = p.x;
        if constexpr (DIM >= 2) d.y[j] = p.y;
        if constexpr (DIM == 3) d.z[j] = p.z;
    }
    ((R *)d.vx)[j] = p.vx;
    if constexpr (VDIM >= 2) ((R *)d.vy)[j] = p.vy;
    if constexpr (VDIM >= 3) ((R *)d.vz)[j] = p.vz;
}

// Bucket of a cell: tiles numbered x fastest, then y, then z.
template <bool MIX, int DIM>
__device__ __forceinline__ int bucket_of(const Geo &g, int ix, int iy, int iz = 0) {
    int bx = ix >> g.tsx;
    if constexpr (DIM == 2) return (iy >> g.tsy) * g.nbx + bx;
    if constexpr (DIM == 3) return ((iz >> g.tsz) * g.nby + (iy >> g.tsy)) * g.nbx + bx;
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

// The z part of the Boris advance in 3D: the rotation about z leaves vz
// alone, so vz takes the two half kicks of Ez.
template <typename R>
__device__ __forceinline__ void boris_z(R &vz, R ez, R a) {
    R mz = vz + a * ez;
    vz = mz + a * ez;
}

// Higuera-Cary advance (Higuera & Cary 2017) of u = gamma v under E and a
// uniform B along z, tau = a bz, ic2 = 1/c^2: the half kick u- = u + a E;
// gamma+ solves the method's implicit relation (the Lorentz factor of the
// mean of u- and u+); t = tau / gamma+, s = 1 / (1 + t^2);
// u+ = s (u- + (u-.t) t + u- x t); u = u+ + a E + u+ x t. The operations and
// their order are the ones the binary32 reading of the oracle uses.
template <typename R>
__device__ __forceinline__ void higuera_cary(R &ux, R &uy, R &uz, R ex, R ey, R ez, R a, R tau, R ic2) {
    const R mx = ux + a * ex, my = uy + a * ey, mz = uz + a * ez;
    const R g2 = R(1) + ((mx * mx + my * my) + mz * mz) * ic2;
    const R sig = g2 - tau * tau;
    const R us = mz * tau;
    const R gp = sqrt(R(0.5) * (sig + sqrt(sig * sig + R(4) * (tau * tau + (us * us) * ic2))));
    const R t = tau / gp;
    const R s = R(1) / (R(1) + t * t);
    const R px = s * (mx + my * t);
    const R py = s * (my - mx * t);
    const R pz = s * (mz + (mz * t) * t);
    ux = (px + a * ex) + py * t;
    uy = (py + a * ey) - px * t;
    uz = pz + a * ez;
}

// gamma of u = gamma v: sqrt(1 + |u|^2 / c^2); the move divides u by it
// (FP64) or multiplies u by its correctly rounded reciprocal (binary32).
template <typename R>
__device__ __forceinline__ R lorentz(R ux, R uy, R uz, R ic2) {
    return sqrt(R(1) + ((ux * ux + uy * uy) + uz * uz) * ic2);
}

// Position update with periodic wrap. Returns the unwrapped cell shift
// (new cell - old cell) per axis in sx, sy, sz, and false for a non-finite or
// runaway coordinate.
//
// Mixed path, one axis: offset o += v dt/d (binary32), k = floor(o),
// o -= k (and o >= 1 after rounding moves one more cell), cell += k modulo n.
__device__ __forceinline__ bool move_axis_mixed(int &ic, float &f, float v, float dtd, int n, int &shift) {
    float o = f + v * dtd;
    float fl = floorf(o);
    o = o - fl;
    const bool ok = fabsf(fl) < 1.0e8f;
    int sh = ok ? (int)fl : 0;
    if (o >= 1.0f) { o = o - 1.0f; sh += 1; }
    int i = ic + sh;
    if (i >= n || i < 0) { i %= n; if (i < 0) i += n; }
    ic = i;
    f = ok ? o : 0.0f;
    shift = sh;
    return ok;
}

// FP64 path, one axis: x += v dt wrapped into [0, L), then the new cell; the
// shift is the cell difference taken modulo n into (-n/2, n/2].
__device__ __forceinline__ bool move_axis_f64(double &xc, int &ic, double &f, double v, double dt, double L,
                                              double inv_d, int n, int &shift) {
    const int i0 = ic;
    double x = xc + v * dt;
    if (x < 0.0) x += L;
    if (x >= L) x -= L;
    if (!(x >= 0.0 && x < L)) {
        x = x - L * floor(x / L);
        if (!(x >= 0.0 && x < L)) x = 0.0;
    }
    xc = x;
    const bool ok = cell_f64(x, inv_d, n, ic, f);
    int d = ic - i0;
    if (d > n / 2) d -= n;
    if (d < -(n / 2)) d += n;
    shift = d;
    return ok;
}

// Move by the velocity (vx, vy, vz) (the particle's v, or u / gamma).
template <bool MIX, int DIM>
__device__ __forceinline__ bool move_pt_v(Pt<MIX> &p, const Geo &g, const PushC &pc, typename Pt<MIX>::R vx,
                                          typename Pt<MIX>::R vy, typename Pt<MIX>::R vz, int &sx, int &sy,
                                          int &sz) {
    sy = 0;
    sz = 0;
    if constexpr (MIX) {
        bool ok = move_axis_mixed(p.ix, p.fx, vx, pc.dtdx, g.nx, sx);
        if constexpr (DIM >= 2) ok = move_axis_mixed(p.iy, p.fy, vy, pc.dtdy, g.ny, sy) && ok;
        if constexpr (DIM == 3) ok = move_axis_mixed(p.iz, p.fz, vz, pc.dtdz, g.nz, sz) && ok;
        return ok;
    } else {
        double f;
        bool ok = move_axis_f64(p.x, p.ix, f, vx, pc.dt, g.lx, g.inv_dx, g.nx, sx);
        p.fx = f;
        if constexpr (DIM >= 2) {
            ok = move_axis_f64(p.y, p.iy, f, vy, pc.dt, g.ly, g.inv_dy, g.ny, sy) && ok;
            p.fy = f;
        }
        if constexpr (DIM == 3) {
            ok = move_axis_f64(p.z, p.iz, f, vz, pc.dt, g.lz, g.inv_dz, g.nz, sz) && ok;
            p.fz = f;
        }
        return ok;
    }
}

template <bool MIX, int DIM>
__device__ __forceinline__ bool move_pt(Pt<MIX> &p, const Geo &g, const PushC &pc, int &sx, int &sy, int &sz) {
    return move_pt_v<MIX, DIM>(p, g, pc, p.vx, p.vy, p.vz, sx, sy, sz);
}

// Velocity advance (Boris, or Higuera-Cary when HC) and move of a particle
// whose E has been gathered (ez = 0 below 3D).
template <bool MIX, int DIM, int VDIM, bool HC>
__device__ __forceinline__ bool push_move(Pt<MIX> &p, const Geo &g, const PushC &pc, typename Pt<MIX>::R ex,
                                          typename Pt<MIX>::R ey, typename Pt<MIX>::R ez, bool move, int &sx,
                                          int &sy, int &sz) {
    using R = typename Pt<MIX>::R;
    const R a = MIX ? (R)pc.af : (R)pc.a, t = MIX ? (R)pc.tf : (R)pc.t, s = MIX ? (R)pc.sf : (R)pc.s;
    if constexpr (HC) {
        static_assert(VDIM == 3, "the Higuera-Cary state has three components");
        const R ic2 = MIX ? (R)pc.ic2f : (R)pc.ic2;
        higuera_cary<R>(p.vx, p.vy, p.vz, ex, ey, ez, a, t, ic2);
        if (!move) {
            sx = sy = sz = 0;
            return true;
        }
        const R gm = lorentz<R>(p.vx, p.vy, p.vz, ic2);
        if constexpr (MIX) {
            // binary32: one correctly rounded 1 / gamma, then three products
            const R ig = R(1) / gm;
            return move_pt_v<MIX, DIM>(p, g, pc, p.vx * ig, p.vy * ig, p.vz * ig, sx, sy, sz);
        } else {
            return move_pt_v<MIX, DIM>(p, g, pc, p.vx / gm, p.vy / gm, p.vz / gm, sx, sy, sz);
        }
    } else {
        if constexpr (DIM == 3) boris_z<R>(p.vz, ez, a);
        boris<R, VDIM>(p.vx, p.vy, ex, ey, a, t, s);
        if (!move) {
            sx = sy = sz = 0;
            return true;
        }
        return move_pt<MIX, DIM>(p, g, pc, sx, sy, sz);
    }
}

template <bool MIX, int DIM>
__device__ __forceinline__ bool move_pt(Pt<MIX> &p, const Geo &g, const PushC &pc, int &sx, int &sy) {
    int sz;
    return move_pt<MIX, DIM>(p, g, pc, sx, sy, sz);
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

// E tile in 3D: nodes [x0, x0+TX] x [y0, y0+TY] x [z0, z0+TZ] (periodic),
// three components, converted to R on the way into LDS.
template <typename R, typename ET>
__device__ void load_e_tile3(R *sE, const ET *E, const Geo &g, int x0, int y0, int z0, int wx, int wy, int wz) {
    const int G = g.nx * g.ny * g.nz;
    const int tot = wx * wy * wz;
    for (int t = threadIdx.x; t < tot; t += blockDim.x) {
        const int lx = t % wx, r = t / wx, ly = r % wy, lz = r / wy;
        int gx = x0 + lx;
        if (gx >= g.nx) gx -= g.nx;
        int gy = y0 + ly;
        if (gy >= g.ny) gy -= g.ny;
        int gz = z0 + lz;
        if (gz >= g.nz) gz -= g.nz;
        const int gi = (gz * g.ny + gy) * g.nx + gx;
        sE[t] = (R)E[gi];
        sE[tot + t] = (R)E[G + gi];
        sE[2 * tot + t] = (R)E[2 * G + gi];
    }
}

// The E tile of a 1D, 2D or 3D step from a field of element type ET.
template <typename R, typename ET, int DIM>
__device__ __forceinline__ void load_tile_any(R *sE, const ET *E, const Geo &g, int x0, int y0, int z0, int wx,
                                              int wy, int wz) {
    if constexpr (DIM == 3)
        load_e_tile3<R, ET>(sE, E, g, x0, y0, z0, wx, wy, wz);
    else
        load_e_tile<R, ET, DIM>(sE, E, g, x0, y0, wx, wy);
}

// 3D CIC interpolation: node weight (wx_a wy_b) wz_c; the eight terms are
// added left to right with a (x) fastest, then b (y), then c (z). e(k) gives
// the value of component comp at corner k = c*4 + b*2 + a.
template <typename R, typename F>
__device__ __forceinline__ R cic3_sum(R fx, R fy, R fz, F e) {
    const R wx0 = R(1) - fx, wy0 = R(1) - fy, wz0 = R(1) - fz;
    const R w00 = wx0 * wy0, w10 = fx * wy0, w01 = wx0 * fy, w11 = fx * fy;
    R acc = (w00 * wz0) * e(0);
    acc = acc + (w10 * wz0) * e(1);
    acc = acc + (w01 * wz0) * e(2);
    acc = acc + (w11 * wz0) * e(3);
    acc = acc + (w00 * fz) * e(4);
    acc = acc + (w10 * fz) * e(5);
    acc = acc + (w01 * fz) * e(6);
    acc = acc + (w11 * fz) * e(7);
    return acc;
}

template <typename R>
__device__ __forceinline__ void gather_lds3(const R *sE, int wx, int wxy, int tot, int lx, int ly, int lz, R fx,
                                            R fy, R fz, R &ex, R &ey, R &ez) {
    const int a = (lz * wxy + ly * wx) + lx;
    const int off[8] = {0, 1, wx, wx + 1, wxy, wxy + 1, wxy + wx, wxy + wx + 1};
    ex = cic3_sum<R>(fx, fy, fz, [&](int k) { return sE[a + off[k]]; });
    ey = cic3_sum<R>(fx, fy, fz, [&](int k) { return sE[tot + a + off[k]]; });
    ez = cic3_sum<R>(fx, fy, fz, [&](int k) { return sE[2 * tot + a + off[k]]; });
}

// Node indices of the eight corners of cell (ix, iy, iz), periodic.
__device__ __forceinline__ void corners3(const Geo &g, int ix, int iy, int iz, int m[8]) {
    const int ip = (ix + 1 >= g.nx) ? 0 : ix + 1;
    const int jp = (iy + 1 >= g.ny) ? 0 : iy + 1;
    const int kp = (iz + 1 >= g.nz) ? 0 : iz + 1;
    const int r0 = (iz * g.ny + iy) * g.nx, r1 = (iz * g.ny + jp) * g.nx;
    const int r2 = (kp * g.ny + iy) * g.nx, r3 = (kp * g.ny + jp) * g.nx;
    m[0] = r0 + ix; m[1] = r0 + ip; m[2] = r1 + ix; m[3] = r1 + ip;
    m[4] = r2 + ix; m[5] = r2 + ip; m[6] = r3 + ix; m[7] = r3 + ip;
}

template <typename R, typename ET>
__device__ __forceinline__ void gather_global3(const ET *E, const Geo &g, int ix, int iy, int iz, R fx, R fy, R fz,
                                               R &ex, R &ey, R &ez) {
    int m[8];
    corners3(g, ix, iy, iz, m);
    const int G = g.nx * g.ny * g.nz;
    ex = cic3_sum<R>(fx, fy, fz, [&](int k) { return (R)E[m[k]]; });
    ey = cic3_sum<R>(fx, fy, fz, [&](int k) { return (R)E[G + m[k]]; });
    ez = cic3_sum<R>(fx, fy, fz, [&](int k) { return (R)E[2 * G + m[k]]; });
}

// Accumulator element: double weights (FP64 path) or int64 fixed-point sums.
template <bool MIX> struct AccOf { using T = double; };
template <> struct AccOf<true> { using T = unsigned long long; };

// Accumulator adds with the address space stated: a device-memory atomic
// (acc_add) and an LDS atomic (acc_add_lds, ds_add_u64 / ds_add_f64). Left
// generic, the compiler may merge an LDS and a global add into one flat
// atomic, which tests the address space per lane and holds the vector-memory
// wait counter, so that the next wait for a particle load also waits for it.
template <bool MIX>
__device__ __forceinline__ void acc_add(typename AccOf<MIX>::T *a, typename AccOf<MIX>::T v) {
    using T = typename AccOf<MIX>::T;
    __hip_atomic_fetch_add((__attribute__((address_space(1))) T *)a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool MIX>
__device__ __forceinline__ void acc_add_lds(typename AccOf<MIX>::T *a, typename AccOf<MIX>::T v) {
    using T = typename AccOf<MIX>::T;
    __hip_atomic_fetch_add((__attribute__((address_space(3))) T *)a, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

// CIC weights of a particle at (fx, fy) as accumulator values. Fixed point:
// w1 = round-half-even(o 2^S) (o 2^S is exact in binary32), w0 = 2^S - w1;
// in 2D (S <= 23) both fit 24 bits and the node weight is their exact 48-bit
// product (24-bit multiplies).
// In 3D (S <= 16) the node weight is (w_a w_b) w_c, exact in 64 bits; the
// eight weights are ordered k = c*4 + b*2 + a.
template <bool MIX, int DIM>
__device__ __forceinline__ void dep_weights(const Pt<MIX> &p, const Geo &g,
                                            typename AccOf<MIX>::T *w) {
    if constexpr (MIX && DIM == 3) {
        const float scale = (float)(1ull << g.S);
        const uint32_t one = 1u << g.S;
        const uint32_t w1x = (uint32_t)rintf(p.fx * scale), w0x = one - w1x;
        const uint32_t w1y = (uint32_t)rintf(p.fy * scale), w0y = one - w1y;
        const uint32_t w1z = (uint32_t)rintf(p.fz * scale), w0z = one - w1z;
        const unsigned long long a00 = (unsigned long long)w0x * w0y, a10 = (unsigned long long)w1x * w0y;
        const unsigned long long a01 = (unsigned long long)w0x * w1y, a11 = (unsigned long long)w1x * w1y;
        w[0] = a00 * w0z; w[1] = a10 * w0z; w[2] = a01 * w0z; w[3] = a11 * w0z;
        w[4] = a00 * w1z; w[5] = a10 * w1z; w[6] = a01 * w1z; w[7] = a11 * w1z;
    } else if constexpr (!MIX && DIM == 3) {
        const double fx = p.fx, fy = p.fy, fz = p.fz;
        const double wx0 = 1.0 - fx, wy0 = 1.0 - fy, wz0 = 1.0 - fz;
        const double a00 = wx0 * wy0, a10 = fx * wy0, a01 = wx0 * fy, a11 = fx * fy;
        w[0] = a00 * wz0; w[1] = a10 * wz0; w[2] = a01 * wz0; w[3] = a11 * wz0;
        w[4] = a00 * fz; w[5] = a10 * fz; w[6] = a01 * fz; w[7] = a11 * fz;
    } else if constexpr (MIX) {
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

template <bool MIX>
__device__ __forceinline__ void deposit_global3(typename AccOf<MIX>::T *acc, const Geo &g, int ix, int iy, int iz,
                                                const typename AccOf<MIX>::T *w) {
    int m[8];
    corners3(g, ix, iy, iz, m);
#pragma unroll
    for (int k = 0; k < 8; ++k) acc_add<MIX>(&acc[m[k]], w[k]);
}

template <bool MIX, int DIM>
__device__ __forceinline__ void deposit_global(typename AccOf<MIX>::T *acc, const Geo &g, int ix, int iy,
                                               const typename AccOf<MIX>::T *w) {
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

// 3D region (nodes [x0-H, x0+TX+H] x [y0-H, ..] x [z0-H, ..]).
template <bool MIX>
__device__ void flush_region3(typename AccOf<MIX>::T *acc, const typename AccOf<MIX>::T *sA, const Geo &g,
                              int x0, int y0, int z0, int wx, int wy, int wz, int halo) {
    const int tot = wx * wy * wz;
    for (int t = threadIdx.x; t < tot; t += blockDim.x) {
        typename AccOf<MIX>::T v = sA[t];
        if (v == (typename AccOf<MIX>::T)0) continue;
        const int lx = t % wx, r = t / wx, ly = r % wy, lz = r / wy;
        int gx = (x0 - halo + lx) % g.nx;
        if (gx < 0) gx += g.nx;
        int gy = (y0 - halo + ly) % g.ny;
        if (gy < 0) gy += g.ny;
        int gz = (z0 - halo + lz) % g.nz;
        if (gz < 0) gz += g.nz;
        acc_add<MIX>(&acc[(gz * g.ny + gy) * g.nx + gx], v);
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

// Field diagnostics of one solve (one workgroup): fixed-order sums of the
// spectral and push partials into diag[step] or we/charge.
__device__ void finalize_block(const FinArgs &f, const CtxDev &c) {
    __shared__ double sRed[16];
    double k = 0.0, p = 0.0, e = 0.0;
    for (int i = threadIdx.x; i < f.npush; i += blockDim.x) {
        k += c.part_push[2 * i];
        p += c.part_push[2 * i + 1];
    }
    for (int i = threadIdx.x; i < f.nspec; i += blockDim.x) e += c.part_spec[i];
    k = block_sum(k, sRed);
    p = block_sum(p, sRed);
    e = block_sum(e, sRed);
    // fixed-point node sums: the exact integer total (whole workgroup)
    QSum qt{0, 0};
    if (f.nspec && f.sd) {
        qt = qsum_take(c.qacc, f.sd);
        if (threadIdx.x == 0) {
            c.qexact[0] = qt.whole;
            c.qexact[1] = (int64_t)qt.rem;
        }
    }
    if (threadIdx.x == 0) {
        double *d = f.diag ? step_slot(f.diag, c) : nullptr;
        if (f.npush && d) {
            d[2] = 0.5 * f.mass * k;
            d[3] = f.mass * p;
        }
        if (f.nspec) {
            double wE = 0.5 * f.dV / f.G * e;
            double q = f.dV * (*c.rho0 - f.G * f.rho_ion);
            if (f.sd) {
                // fixed-point node sums: the exact integer total
                q = qsum_charge(qt, f.sd, f.q_macro);
            }
            if (f.walls) {
                // the physical half of the odd extension, wall nodes at half weight
                wE = 0.5 * wE;
                q = f.nlive ? f.q_macro * (double)*f.nlive : 0.0;
            }
            if (d) {
                d[0] = q;
                d[1] = wE;
            }
            if (f.we) *f.we = wE;
            if (f.charge) *f.charge = q;
        }
    }
}


}  // namespace
}  // namespace apic

// Particles per thread and pipeline stage in the fused step kernels.
#ifndef APIC_STEP_U
#define APIC_STEP_U 1
#endif

// Instantiates a statement for the precision / dimension combination of a
// launch: MIX, DIM, VDIM (and the unroll factor U) are constexpr inside.
#define APIC_DISPATCH_2D(g, mixed, ...)                                                 \
    do {                                                                                \
        [[maybe_unused]] constexpr bool HC = false;                                     \
        if (mixed) {                                                                    \
            constexpr bool MIX = true;                                                  \
            [[maybe_unused]] constexpr int U = APIC_STEP_U;                             \
            if ((g).dim == 1) { [[maybe_unused]] constexpr int DIM = 1, VDIM = 1; __VA_ARGS__; }         \
            else if ((g).vdim == 2) { [[maybe_unused]] constexpr int DIM = 2, VDIM = 2; __VA_ARGS__; }   \
            else { [[maybe_unused]] constexpr int DIM = 2, VDIM = 3; __VA_ARGS__; }                      \
        } else {                                                                        \
            constexpr bool MIX = false;                                                 \
            [[maybe_unused]] constexpr int U = APIC_STEP_U;                             \
            if ((g).dim == 1) { [[maybe_unused]] constexpr int DIM = 1, VDIM = 1; __VA_ARGS__; }         \
            else if ((g).vdim == 2) { [[maybe_unused]] constexpr int DIM = 2, VDIM = 2; __VA_ARGS__; }   \
            else { [[maybe_unused]] constexpr int DIM = 2, VDIM = 3; __VA_ARGS__; }                      \
        }                                                                               \
    } while (0)

// Both precisions, one velocity advance (HCV), a given (DIM, VDIM).
#define APIC_DISPATCH_MIX(mixed, HCV, D, V, ...)                                       \
    do {                                                                                \
        [[maybe_unused]] constexpr bool HC = HCV;                                       \
        [[maybe_unused]] constexpr int U = APIC_STEP_U;                                 \
        [[maybe_unused]] constexpr int DIM = D, VDIM = V;                               \
        if (mixed) { constexpr bool MIX = true; __VA_ARGS__; }                          \
        else { constexpr bool MIX = false; __VA_ARGS__; }                               \
    } while (0)

// Every case, with the 3D3V one and the velocity advance (Higuera-Cary, g.hc,
// only with three velocity components).
#define APIC_DISPATCH(g, mixed, ...)                                                    \
    do {                                                                                \
        if ((g).vdim == 3 && (g).hc) {                                                  \
            if ((g).dim == 3) APIC_DISPATCH_MIX(mixed, true, 3, 3, __VA_ARGS__);        \
            else APIC_DISPATCH_MIX(mixed, true, 2, 3, __VA_ARGS__);                     \
        } else if ((g).dim == 3) {                                                      \
            APIC_DISPATCH_MIX(mixed, false, 3, 3, __VA_ARGS__);                         \
        } else {                                                                        \
            APIC_DISPATCH_2D(g, mixed, __VA_ARGS__);                                    \
        }                                                                               \
    } while (0)
