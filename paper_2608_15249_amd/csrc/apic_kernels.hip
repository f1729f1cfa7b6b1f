// HIP kernels of the PIC coupling loop for CDNA4 (gfx950, wave64).
//
// The loop is the electrostatic particle-in-cell cycle described in the
// AlgoPlasma paper ("Core functionality": B_Scatter, C_Gather, A_Pusher with
// the Boris pusher, D_Poisson; the two-stream example's driver fixes the
// order push -> move -> deposit -> field). Shape functions are linear
// (cloud-in-cell) on a periodic node-centred grid.
//
// Design (one GPU):
//  * Particles live in HBM as structure-of-arrays; every kernel reads them
//    with unit-stride (coalesced) loads.
//  * Particles are kept ordered by bucket = tile of 2^tsx x 2^tsy cells. A
//    workgroup owns one bucket: it stages the tile's E nodes in LDS for the
//    gather and accumulates the deposit of its particles into an LDS copy of
//    the tile plus a halo, then flushes each touched node with one global
//    atomic. Workgroup -> bucket mapping is XCD-aware: consecutive buckets
//    (neighbouring tiles, which share halo nodes and E tiles) run on the same
//    XCD, so their traffic stays in that XCD's L2.
//  * Per step the fused path runs two particle passes: a count pass (gather,
//    push and move computed, only the new bucket histogram kept) and a push
//    pass that recomputes the same update bit for bit, deposits rho^{n+1} and
//    writes each particle straight to its slot of the next bucket order
//    (counting sort: histogram -> exclusive scan -> scatter). State traffic is
//    read + read + write per particle-step instead of read/write for the push
//    plus read/write for a separate sort.
//  * The mixed path holds positions as an integer cell plus a binary32
//    in-cell offset and deposits with int64 fixed-point weights, so the charge
//    density is exact and independent of summation order.
//  * This file is compiled with -ffp-contract=off: the count pass and the push
//    pass must produce identical bits for the same particle.
#include "apic_internal.h"

#include <math.h>

namespace apic {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ void raise_err(int *err, int bit) { atomicOr(err, bit); }

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

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Block-wide sum, deterministic (fixed tree); result valid in every thread.
__device__ double block_sum(double v, double *sh /* [kWaves] */) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    __syncthreads();
    return t;
}

// Deterministic grid-wide sum: each block stores its partial, the last block
// to arrive adds the partials in block order and writes out = scale * sum.
__device__ void grid_sum_store(double v, double *out, double scale, const CtxDev &c, double *sh) {
    double b = block_sum(v, sh);
    __shared__ int is_last;
    if (threadIdx.x == 0) {
        c.partials[blockIdx.x] = b;
        __threadfence();
        unsigned prev = atomicAdd(c.counter, 1u);
        is_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (is_last) {
        __threadfence();
        double t = 0.0;
        for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x)
            t += ((volatile double *)c.partials)[i];
        t = block_sum(t, sh);
        if (threadIdx.x == 0) {
            if (out) *out = t * scale;
            *c.counter = 0u;
        }
    }
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
template <typename R, int VDIM>
__device__ __forceinline__ void boris(R &vx, R &vy, R ex, R ey, R a, R t, R s) {
    if constexpr (VDIM == 1) {
        R m1 = vx + a * ex;
        vx = m1 + a * ex;
    } else {
        R mx = vx + a * ex;
        R my = vy + a * ey;
        R px = mx + my * t;
        R py = my - mx * t;
        R qx = mx + py * s;
        R qy = my - px * s;
        vx = qx + a * ex;
        vy = qy + a * ey;
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

// E tile: nodes [x0, x0+TX] x [y0, y0+TY] (periodic), comps [DIM].
template <typename R, int DIM>
__device__ void load_e_tile(R *sE, const R *E, const Geo &g, int x0, int y0, int wx, int wy) {
    const int G = g.nx * g.ny;
    const int tot = wx * wy;
    for (int t = threadIdx.x; t < tot; t += blockDim.x) {
        int lx = t % wx, ly = t / wx;
        int gx = x0 + lx;
        if (gx >= g.nx) gx -= g.nx;
        int gy = y0 + ly;
        if (gy >= g.ny) gy -= g.ny;
        int gi = gy * g.nx + gx;
        sE[t] = E[gi];
        if constexpr (DIM == 2) sE[tot + t] = E[G + gi];
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

template <typename R, int DIM>
__device__ __forceinline__ void gather_global(const R *E, const Geo &g, int ix, int iy, R fx, R fy,
                                              R &ex, R &ey) {
    int ip = ix + 1;
    if (ip >= g.nx) ip = 0;
    if constexpr (DIM == 1) {
        ex = (R(1) - fx) * E[ix] + fx * E[ip];
        ey = R(0);
    } else {
        const int G = g.nx * g.ny;
        int jp = iy + 1;
        if (jp >= g.ny) jp = 0;
        R w00 = (R(1) - fx) * (R(1) - fy), w10 = fx * (R(1) - fy);
        R w01 = (R(1) - fx) * fy, w11 = fx * fy;
        int a00 = iy * g.nx + ix, a10 = iy * g.nx + ip, a01 = jp * g.nx + ix, a11 = jp * g.nx + ip;
        ex = w00 * E[a00] + w10 * E[a10] + w01 * E[a01] + w11 * E[a11];
        ey = w00 * E[G + a00] + w10 * E[G + a10] + w01 * E[G + a01] + w11 * E[G + a11];
    }
}

// Accumulator element: double weights (FP64 path) or int64 fixed-point sums.
template <bool MIX> struct AccOf { using T = double; };
template <> struct AccOf<true> { using T = unsigned long long; };

template <bool MIX>
__device__ __forceinline__ void acc_add(typename AccOf<MIX>::T *a, typename AccOf<MIX>::T v) {
    atomicAdd(a, v);
}

// CIC weights of a particle at (fx, fy) as accumulator values.
template <bool MIX, int DIM>
__device__ __forceinline__ void dep_weights(const Pt<MIX> &p, const Geo &g,
                                            typename AccOf<MIX>::T w[4]) {
    if constexpr (MIX) {
        const float scale = (float)(1ull << g.S);
        const int64_t one = (int64_t)1 << g.S;
        int64_t w1x = qw1(p.fx, scale), w0x = one - w1x;
        if constexpr (DIM == 1) {
            w[0] = (unsigned long long)w0x;
            w[1] = (unsigned long long)w1x;
        } else {
            int64_t w1y = qw1(p.fy, scale), w0y = one - w1y;
            w[0] = (unsigned long long)(w0x * w0y);
            w[1] = (unsigned long long)(w1x * w0y);
            w[2] = (unsigned long long)(w0x * w1y);
            w[3] = (unsigned long long)(w1x * w1y);
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
                             int x0, int y0, int wx, int wy) {
    const int tot = wx * wy;
    for (int t = threadIdx.x; t < tot; t += blockDim.x) {
        typename AccOf<MIX>::T v = sA[t];
        if (v == (typename AccOf<MIX>::T)0) continue;
        int lx = t % wx, ly = t / wx;
        int gx = x0 - g.halo + lx;
        gx %= g.nx;
        if (gx < 0) gx += g.nx;
        int gy = 0;
        if constexpr (DIM == 2) {
            gy = y0 - g.halo + ly;
            gy %= g.ny;
            if (gy < 0) gy += g.ny;
        }
        acc_add<MIX>(&acc[gy * g.nx + gx], v);
    }
}

// Wave-aggregated reservation of slots in per-key counters: lanes with equal
// key get consecutive slots (in lane order) from one atomicAdd per key.
__device__ __forceinline__ int reserve_slot(int32_t *cursor, int key, bool active) {
    uint64_t rem = __ballot(active);
    int slot = -1;
    const uint64_t lt = lanemask_lt();
    while (rem) {
        const int leader = __ffsll((unsigned long long)rem) - 1;
        const int k = __shfl(key, leader);
        const uint64_t grp = __ballot(active && key == k);
        int base = 0;
        if ((int)__lane_id() == leader) base = atomicAdd(&cursor[k], (int)__popcll(grp));
        base = __shfl(base, leader);
        if (active && key == k) slot = base + (int)__popcll(grp & lt);
        rem &= ~grp;
    }
    return slot;
}

// Wave-aggregated increment of per-key counters.
__device__ __forceinline__ void count_keys(int32_t *count, int key, bool active) {
    uint64_t rem = __ballot(active);
    while (rem) {
        const int leader = __ffsll((unsigned long long)rem) - 1;
        const int k = __shfl(key, leader);
        const uint64_t grp = __ballot(active && key == k);
        if ((int)__lane_id() == leader) atomicAdd(&count[k], (int)__popcll(grp));
        rem &= ~grp;
    }
}

// ================================================================= kernels

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_set_step(int *step, int v) { *step = v; }

__global__ void k_copy_bytes(uint4 *dst, const uint4 *src, int64_t n16, char *dtail, const char *stail,
                             int tail) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
    if (blockIdx.x == 0 && (int)threadIdx.x < tail) dtail[threadIdx.x] = stail[threadIdx.x];
}

// ---- general counting sort: keys + histogram --------------------------------
template <bool MIX, int DIM, int VDIM>
__global__ void __launch_bounds__(kBlock) k_keys_hist(Geo g, Parts p, int64_t n, int32_t *keys,
                                                      int32_t *count, CtxDev c) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t n_up = ((n + 63) / 64) * 64;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_up; i += stride) {
        bool act = i < n;
        int key = 0;
        if (act) {
            Pt<MIX> q;
            bool ok = load_pt<MIX, DIM, VDIM>(p, i, g, q);
            if (!ok) raise_err(c.err, ERR_DOMAIN);
            key = bucket_of<MIX, DIM>(g, q.ix, q.iy);
            keys[i] = key;
        }
        count_keys(count, key, act);
    }
}

// ---- exclusive scan over buckets (one workgroup) ------------------------------
// start[b] = sum_{b'<b} count[b'], start[nb] = total; cursor = start;
// count_zero (if non-null) is cleared for the next histogram. Also clears the
// per-step diag accumulators and advances the device step index.
__global__ void __launch_bounds__(1024) k_scan(const int32_t *count, int32_t *start, int32_t *cursor,
                                               int32_t *count_zero, int nb, int64_t n, int64_t max_per,
                                               double *diag, CtxDev c) {
    __shared__ int64_t sh[1024];
    __shared__ int64_t carry;
    __shared__ int step_now;
    if (threadIdx.x == 0) {
        carry = 0;
        if (diag) {
            int st = *c.step + 1;
            *c.step = st;
            step_now = st;
        }
    }
    __syncthreads();
    const int T = blockDim.x;
    const int per = 16;
    int bad = 0;
    for (int base = 0; base < nb; base += T * per) {
        int64_t loc[per];
        int64_t s = 0;
        for (int k = 0; k < per; ++k) {
            int b = base + threadIdx.x * per + k;
            int64_t v = (b < nb) ? count[b] : 0;
            if (v > max_per) bad = 1;
            loc[k] = v;
            s += v;
        }
        sh[threadIdx.x] = s;
        __syncthreads();
        // Hillis-Steele inclusive scan over thread sums
        for (int off = 1; off < T; off <<= 1) {
            int64_t add = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        int64_t run = carry + sh[threadIdx.x] - s;
        for (int k = 0; k < per; ++k) {
            int b = base + threadIdx.x * per + k;
            if (b < nb) {
                start[b] = (int32_t)run;
                cursor[b] = (int32_t)run;
                if (count_zero) count_zero[b] = 0;
            }
            run += loc[k];
        }
        __syncthreads();
        if (threadIdx.x == T - 1) carry += sh[T - 1];
        __syncthreads();
    }
    if (bad) raise_err(c.err, ERR_OVERFLOW);
    if (threadIdx.x == 0) {
        start[nb] = (int32_t)carry;
        if (carry != n) raise_err(c.err, ERR_COUNT);
        if (diag) {
            double *d = diag + 4 * step_now;
            d[2] = 0.0;
            d[3] = 0.0;
        }
    }
}

// ---- general counting sort: scatter -----------------------------------------
template <bool MIX, int DIM, int VDIM>
__global__ void __launch_bounds__(kBlock) k_scatter(Geo g, Parts src, Parts dst, int64_t n, const int32_t *keys,
                                                    int32_t *cursor, const int32_t *start, int32_t *perm,
                                                    CtxDev c) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t n_up = ((n + 63) / 64) * 64;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_up; i += stride) {
        bool act = i < n;
        int key = act ? keys[i] : 0;
        int slot = reserve_slot(cursor, key, act);
        if (act) {
            if (slot >= start[key + 1]) {
                raise_err(c.err, ERR_ORDER);
                continue;
            }
            Pt<MIX> q;
            load_pt<MIX, DIM, VDIM>(src, i, g, q);
            // copy the raw stored values (no re-normalisation)
            if constexpr (MIX) {
                dst.cell[slot] = src.cell[i];
                dst.ox[slot] = src.ox[i];
                if constexpr (DIM == 2) dst.oy[slot] = src.oy[i];
            } else {
                dst.x[slot] = src.x[i];
                if constexpr (DIM == 2) dst.y[slot] = src.y[i];
            }
            using R = typename Pt<MIX>::R;
            ((R *)dst.vx)[slot] = q.vx;
            if constexpr (VDIM >= 2) ((R *)dst.vy)[slot] = q.vy;
            if constexpr (VDIM >= 3) ((R *)dst.vz)[slot] = q.vz;
            if (perm) perm[slot] = (int32_t)i;
        }
    }
}

// ---- deposit of current positions ---------------------------------------------
template <bool MIX, int DIM, int VDIM>
__global__ void __launch_bounds__(kBlock) k_deposit_direct(Geo g, Parts p, int64_t n,
                                                           typename AccOf<MIX>::T *acc, CtxDev c) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
        Pt<MIX> q;
        if (!load_pt<MIX, DIM, VDIM>(p, i, g, q)) {
            raise_err(c.err, ERR_DOMAIN);
            continue;
        }
        typename AccOf<MIX>::T w[4];
        dep_weights<MIX, DIM>(q, g, w);
        deposit_global<MIX, DIM>(acc, g, q.ix, q.iy, w);
    }
}

template <bool MIX, int DIM, int VDIM>
__global__ void __launch_bounds__(kBlock) k_deposit_tiled(Geo g, Parts p, const int32_t *bstart,
                                                          typename AccOf<MIX>::T *acc, CtxDev c) {
    using A = typename AccOf<MIX>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    A *sA = (A *)smem;
    const int b = bucket_of_block(g.nbuckets);
    if (b >= g.nbuckets) return;
    const int bx = (DIM == 2) ? (b % g.nbx) : b;
    const int by = (DIM == 2) ? (b / g.nbx) : 0;
    const int x0 = bx << g.tsx, y0 = (DIM == 2) ? (by << g.tsy) : 0;
    const int wx = (1 << g.tsx) + 1 + 2 * g.halo;
    const int wy = (DIM == 2) ? (1 << g.tsy) + 1 + 2 * g.halo : 1;
    for (int t = threadIdx.x; t < wx * wy; t += blockDim.x) sA[t] = (A)0;
    __syncthreads();
    const int i0 = min(max(bstart[b], 0), g.np), i1 = min(max(bstart[b + 1], i0), g.np);
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        Pt<MIX> q;
        if (!load_pt<MIX, DIM, VDIM>(p, i, g, q)) {
            raise_err(c.err, ERR_DOMAIN);
            continue;
        }
        A w[4];
        dep_weights<MIX, DIM>(q, g, w);
        int lx = q.ix - x0 + g.halo;
        int ly = (DIM == 2) ? q.iy - y0 + g.halo : 0;
        bool inl = (lx >= 0) && (lx <= wx - 2) && ((DIM == 1) || (ly >= 0 && ly <= wy - 2));
        if (inl) {
            int a = ly * wx + lx;
            acc_add<MIX>(&sA[a], w[0]);
            acc_add<MIX>(&sA[a + 1], w[1]);
            if constexpr (DIM == 2) {
                acc_add<MIX>(&sA[a + wx], w[2]);
                acc_add<MIX>(&sA[a + wx + 1], w[3]);
            }
        } else {
            raise_err(c.err, ERR_ORDER);
            deposit_global<MIX, DIM>(acc, g, q.ix, q.iy, w);
        }
    }
    __syncthreads();
    flush_region<MIX, DIM>(acc, sA, g, x0, y0, wx, wy);
}

// ---- gather + push (+ move), in place -------------------------------------------
template <bool MIX, int DIM, int VDIM>
__global__ void __launch_bounds__(kBlock) k_gather_push_direct(Geo g, Parts p, int64_t n,
                                                               const typename Pt<MIX>::R *E, PushC pc,
                                                               CtxDev c) {
    using R = typename Pt<MIX>::R;
    const R a = MIX ? (R)pc.af : (R)pc.a, t = MIX ? (R)pc.tf : (R)pc.t, s = MIX ? (R)pc.sf : (R)pc.s;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
        Pt<MIX> q;
        if (!load_pt<MIX, DIM, VDIM>(p, i, g, q)) {
            raise_err(c.err, ERR_DOMAIN);
            continue;
        }
        R ex, ey;
        gather_global<R, DIM>(E, g, q.ix, q.iy, q.fx, q.fy, ex, ey);
        boris<R, VDIM>(q.vx, q.vy, ex, ey, a, t, s);
        if (pc.move) {
            int sx, sy;
            if (!move_pt<MIX, DIM>(q, g, pc, sx, sy)) raise_err(c.err, ERR_DOMAIN);
        }
        store_pt<MIX, DIM, VDIM>(p, i, q);
    }
}

template <bool MIX, int DIM, int VDIM>
__global__ void __launch_bounds__(kBlock) k_gather_push_tiled(Geo g, Parts p, const int32_t *bstart,
                                                              const typename Pt<MIX>::R *E, PushC pc,
                                                              CtxDev c) {
    using R = typename Pt<MIX>::R;
    extern __shared__ __align__(16) unsigned char smem[];
    R *sE = (R *)smem;
    const int b = bucket_of_block(g.nbuckets);
    if (b >= g.nbuckets) return;
    const int bx = (DIM == 2) ? (b % g.nbx) : b;
    const int by = (DIM == 2) ? (b / g.nbx) : 0;
    const int x0 = bx << g.tsx, y0 = (DIM == 2) ? (by << g.tsy) : 0;
    const int ex_w = (1 << g.tsx) + 1, ey_w = (DIM == 2) ? (1 << g.tsy) + 1 : 1;
    load_e_tile<R, DIM>(sE, E, g, x0, y0, ex_w, ey_w);
    __syncthreads();
    const R a = MIX ? (R)pc.af : (R)pc.a, t = MIX ? (R)pc.tf : (R)pc.t, s = MIX ? (R)pc.sf : (R)pc.s;
    const int i0 = min(max(bstart[b], 0), g.np), i1 = min(max(bstart[b + 1], i0), g.np);
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        Pt<MIX> q;
        if (!load_pt<MIX, DIM, VDIM>(p, i, g, q)) {
            raise_err(c.err, ERR_DOMAIN);
            continue;
        }
        int lx = q.ix - x0, ly = (DIM == 2) ? q.iy - y0 : 0;
        R ex, ey;
        if (lx >= 0 && lx < ex_w - 1 && ly >= 0 && (DIM == 1 || ly < ey_w - 1)) {
            gather_lds<R, DIM>(sE, ex_w, ex_w * ey_w, lx, ly, q.fx, q.fy, ex, ey);
        } else {
            raise_err(c.err, ERR_ORDER);
            gather_global<R, DIM>(E, g, q.ix, q.iy, q.fx, q.fy, ex, ey);
        }
        boris<R, VDIM>(q.vx, q.vy, ex, ey, a, t, s);
        if (pc.move) {
            int sx, sy;
            if (!move_pt<MIX, DIM>(q, g, pc, sx, sy)) raise_err(c.err, ERR_DOMAIN);
        }
        store_pt<MIX, DIM, VDIM>(p, i, q);
    }
}

// ---- fused step, pass 1: new-bucket histogram ---------------------------------
// Same arithmetic as k_step_push up to the new cell; keeps only the counts.
template <bool MIX, int DIM, int VDIM>
__global__ void __launch_bounds__(kBlock) k_step_count(Geo g, Parts p, const int32_t *bstart,
                                                       const typename Pt<MIX>::R *E, PushC pc,
                                                       int32_t *count, CtxDev c) {
    using R = typename Pt<MIX>::R;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t sCnt[9];
    R *sE = (R *)smem;
    const int b = bucket_of_block(g.nbuckets);
    if (b >= g.nbuckets) return;
    const int bx = (DIM == 2) ? (b % g.nbx) : b;
    const int by = (DIM == 2) ? (b / g.nbx) : 0;
    const int x0 = bx << g.tsx, y0 = (DIM == 2) ? (by << g.tsy) : 0;
    const int ex_w = (1 << g.tsx) + 1, ey_w = (DIM == 2) ? (1 << g.tsy) + 1 : 1;
    if (threadIdx.x < 9) sCnt[threadIdx.x] = 0;
    load_e_tile<R, DIM>(sE, E, g, x0, y0, ex_w, ey_w);
    __syncthreads();
    const R a = MIX ? (R)pc.af : (R)pc.a, t = MIX ? (R)pc.tf : (R)pc.t, s = MIX ? (R)pc.sf : (R)pc.s;
    const int i0 = min(max(bstart[b], 0), g.np), i1 = min(max(bstart[b + 1], i0), g.np);
    // whole waves iterate together so the wave-aggregated counters see all lanes
    const int span = i1 - i0;
    const int span_up = ((span + 63) / 64) * 64;
    for (int k = threadIdx.x; k < span_up; k += blockDim.x) {
        const bool act = k < span;
        int slot_code = 0;   // neighbour index 0..8, or 9 = far
        int nbk = 0;
        if (act) {
            Pt<MIX> q;
            bool ok = load_pt<MIX, DIM, VDIM>(p, i0 + k, g, q);
            int lx = q.ix - x0, ly = (DIM == 2) ? q.iy - y0 : 0;
            R ex, ey;
            if (lx >= 0 && lx < ex_w - 1 && ly >= 0 && (DIM == 1 || ly < ey_w - 1)) {
                gather_lds<R, DIM>(sE, ex_w, ex_w * ey_w, lx, ly, q.fx, q.fy, ex, ey);
            } else {
                ok = false;
                gather_global<R, DIM>(E, g, q.ix, q.iy, q.fx, q.fy, ex, ey);
            }
            boris<R, VDIM>(q.vx, q.vy, ex, ey, a, t, s);
            int sx, sy;
            ok = move_pt<MIX, DIM>(q, g, pc, sx, sy) && ok;
            if (!ok) raise_err(c.err, ERR_DOMAIN);
            nbk = bucket_of<MIX, DIM>(g, q.ix, q.iy);
            int nbx_ = (DIM == 2) ? nbk % g.nbx : nbk;
            int nby_ = (DIM == 2) ? nbk / g.nbx : 0;
            int dbx = nbx_ - bx, dby = nby_ - by;
            if (dbx > g.nbx / 2) dbx -= g.nbx;
            if (dbx < -(g.nbx / 2)) dbx += g.nbx;
            if (dby > g.nby / 2) dby -= g.nby;
            if (dby < -(g.nby / 2)) dby += g.nby;
            slot_code = (dbx >= -1 && dbx <= 1 && dby >= -1 && dby <= 1) ? (dby + 1) * 3 + (dbx + 1) : 9;
        }
        // near buckets: wave-aggregated LDS counters; far buckets: global atomics
        uint64_t rem = __ballot(act && slot_code < 9);
        while (rem) {
            const int leader = __ffsll((unsigned long long)rem) - 1;
            const int kc = __shfl(slot_code, leader);
            const uint64_t grp = __ballot(act && slot_code == kc);
            if ((int)__lane_id() == leader) atomicAdd(&sCnt[kc], (int)__popcll(grp));
            rem &= ~grp;
        }
        if (act && slot_code == 9) atomicAdd(&count[nbk], 1);
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        int v = sCnt[threadIdx.x];
        if (v) {
            int dbx = (int)(threadIdx.x % 3) - 1, dby = (int)(threadIdx.x / 3) - 1;
            int nbx_ = bx + dbx, nby_ = by + dby;
            if (nbx_ < 0) nbx_ += g.nbx;
            if (nbx_ >= g.nbx) nbx_ -= g.nbx;
            if (nby_ < 0) nby_ += g.nby;
            if (nby_ >= g.nby) nby_ -= g.nby;
            int nb = (DIM == 2) ? nby_ * g.nbx + nbx_ : nbx_;
            atomicAdd(&count[nb], v);
        }
    }
}

// ---- fused step, pass 2: push, deposit, scatter into the next bucket order -----
template <bool MIX, int DIM, int VDIM>
__global__ void __launch_bounds__(kBlock) k_step_push(Geo g, Parts src, Parts dst, const int32_t *bstart,
                                                      const int32_t *bstart_new, int32_t *cursor,
                                                      const typename Pt<MIX>::R *E, PushC pc,
                                                      typename AccOf<MIX>::T *acc, int32_t *perm,
                                                      double *diag, double mass, CtxDev c) {
    using R = typename Pt<MIX>::R;
    using A = typename AccOf<MIX>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double sRed[kWaves];
    const int b = bucket_of_block(g.nbuckets);
    if (b >= g.nbuckets) return;
    const int bx = (DIM == 2) ? (b % g.nbx) : b;
    const int by = (DIM == 2) ? (b / g.nbx) : 0;
    const int x0 = bx << g.tsx, y0 = (DIM == 2) ? (by << g.tsy) : 0;
    const int ex_w = (1 << g.tsx) + 1, ey_w = (DIM == 2) ? (1 << g.tsy) + 1 : 1;
    const int wx = (1 << g.tsx) + 1 + 2 * g.halo;
    const int wy = (DIM == 2) ? (1 << g.tsy) + 1 + 2 * g.halo : 1;
    A *sA = (A *)smem;
    R *sE = (R *)(smem + (((size_t)wx * wy * sizeof(A) + 15) & ~(size_t)15));
    for (int t2 = threadIdx.x; t2 < wx * wy; t2 += blockDim.x) sA[t2] = (A)0;
    load_e_tile<R, DIM>(sE, E, g, x0, y0, ex_w, ey_w);
    __syncthreads();
    const R a = MIX ? (R)pc.af : (R)pc.a, t = MIX ? (R)pc.tf : (R)pc.t, s = MIX ? (R)pc.sf : (R)pc.s;
    const int i0 = min(max(bstart[b], 0), g.np), i1 = min(max(bstart[b + 1], i0), g.np);
    const int span = i1 - i0;
    const int span_up = ((span + 63) / 64) * 64;
    double ke = 0.0, px = 0.0;
    for (int k = threadIdx.x; k < span_up; k += blockDim.x) {
        const bool act = k < span;
        Pt<MIX> q;
        int nbk = 0;
        if (act) {
            bool ok = load_pt<MIX, DIM, VDIM>(src, i0 + k, g, q);
            const double v2o = (double)q.vx * (double)q.vx + (double)q.vy * (double)q.vy +
                               (double)q.vz * (double)q.vz;
            int lx = q.ix - x0, ly = (DIM == 2) ? q.iy - y0 : 0;
            R ex, ey;
            if (lx >= 0 && lx < ex_w - 1 && ly >= 0 && (DIM == 1 || ly < ey_w - 1)) {
                gather_lds<R, DIM>(sE, ex_w, ex_w * ey_w, lx, ly, q.fx, q.fy, ex, ey);
            } else {
                ok = false;
                gather_global<R, DIM>(E, g, q.ix, q.iy, q.fx, q.fy, ex, ey);
            }
            boris<R, VDIM>(q.vx, q.vy, ex, ey, a, t, s);
            const double v2n = (double)q.vx * (double)q.vx + (double)q.vy * (double)q.vy +
                               (double)q.vz * (double)q.vz;
            ke += 0.5 * (v2o + v2n);
            px += (double)q.vx;
            int sx, sy;
            ok = move_pt<MIX, DIM>(q, g, pc, sx, sy) && ok;
            if (!ok) raise_err(c.err, ERR_DOMAIN);
            nbk = bucket_of<MIX, DIM>(g, q.ix, q.iy);
            // deposit rho^{n+1}
            A w[4];
            dep_weights<MIX, DIM>(q, g, w);
            int dlx = lx + sx + g.halo;
            int dly = (DIM == 2) ? ly + sy + g.halo : 0;
            bool inl = (dlx >= 0) && (dlx <= wx - 2) && ((DIM == 1) || (dly >= 0 && dly <= wy - 2));
            if (inl) {
                int a0 = dly * wx + dlx;
                acc_add<MIX>(&sA[a0], w[0]);
                acc_add<MIX>(&sA[a0 + 1], w[1]);
                if constexpr (DIM == 2) {
                    acc_add<MIX>(&sA[a0 + wx], w[2]);
                    acc_add<MIX>(&sA[a0 + wx + 1], w[3]);
                }
            } else {
                deposit_global<MIX, DIM>(acc, g, q.ix, q.iy, w);
            }
        }
        const int slot = reserve_slot(cursor, nbk, act);
        if (act) {
            if (slot >= 0 && slot < bstart_new[nbk + 1]) {
                store_pt<MIX, DIM, VDIM>(dst, slot, q);
                if (perm) perm[slot] = i0 + k;
            } else {
                raise_err(c.err, ERR_ORDER);
            }
        }
    }
    __syncthreads();
    flush_region<MIX, DIM>(acc, sA, g, x0, y0, wx, wy);
    if (diag) {
        double kt = block_sum(ke, sRed);
        double pt = block_sum(px, sRed);
        if (threadIdx.x == 0) {
            double *d = step_slot(diag, c);
            atomicAdd(&d[2], 0.5 * mass * kt);
            atomicAdd(&d[3], mass * pt);
        }
    }
}

// ---- field: accumulation -> rho --------------------------------------------------
// rho_j = add + scale * acc_j (acc: double weights or int64 fixed-point sums);
// charge = dV * sum_j (rho_j - ion); acc is cleared when clear != 0.
template <bool MIX>
__global__ void __launch_bounds__(kBlock) k_rho(int64_t G, typename AccOf<MIX>::T *acc, double *rho,
                                                double scale, double add, double ion, double dV, int clear,
                                                double *charge, int step_mode, CtxDev c) {
    __shared__ double sRed[kWaves];
    double part = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < G; i += (int64_t)gridDim.x * blockDim.x) {
        typename AccOf<MIX>::T v = acc[i];
        double w;
        if constexpr (MIX) w = (double)(int64_t)v;
        else w = v;
        double r = add + scale * w;
        rho[i] = r;
        part += r - ion;
        if (clear) acc[i] = (typename AccOf<MIX>::T)0;
    }
    double *out = charge ? (step_mode ? step_slot(charge, c) : charge) : nullptr;
    grid_sum_store(part, out, dV, c, sRed);
}

// Spectral Poisson + centred gradient on the half-spectrum [ny][nx/2+1]:
//   phi_hat = rho_hat / K^2 (K^2 = modified wavenumber of the FD Laplacian,
//   phi_hat(0) = 0), E_hat_d = -i kappa_d phi_hat with kappa = sin(k d)/d,
//   scaled by 1/(nx ny) for the unnormalised inverse transform.
__global__ void __launch_bounds__(kBlock) k_spectral(Geo g, const double2 *rh, double2 *exh, double2 *eyh,
                                                     CtxDev c) {
    const int hx = g.nx / 2 + 1;
    const int64_t tot = (int64_t)hx * g.ny;
    const double norm = 1.0 / ((double)g.nx * (double)g.ny);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        int kx = (int)(i % hx), ky = (int)(i / hx);
        double K2 = c.kx2[kx] + c.ky2[ky];
        double2 r = rh[i];
        double inv = (kx == 0 && ky == 0) ? 0.0 : norm / K2;
        double pr = r.x * inv, pi = r.y * inv;
        // -i * kappa * (pr + i pi) = kappa * pi - i kappa * pr
        double kax = c.kapx[kx], kay = c.kapy[ky];
        exh[i] = make_double2(kax * pi, -kax * pr);
        eyh[i] = make_double2(kay * pi, -kay * pr);
    }
}

__global__ void __launch_bounds__(kBlock) k_efinish(int64_t G, int dim, const double *E, float *E32, double dV,
                                                    double *we, int step_mode, CtxDev c) {
    __shared__ double sRed[kWaves];
    double part = 0.0;
    const int64_t n = G * dim;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double e = E[i];
        part += e * e;
        if (E32) E32[i] = (float)e;
    }
    double *out = we ? (step_mode ? step_slot(we, c) : we) : nullptr;
    grid_sum_store(part, out, 0.5 * dV, c, sRed);
}

// 1D periodic field by Gauss's law on the half nodes (identical to the FFT
// solve of the 3-point Laplacian with centred gradient):
//   E_{j+1/2} = E_{j-1/2} + (rho_j - <rho>) dx,  sum_j E_{j+1/2} = 0,
//   E_j = (E_{j-1/2} + E_{j+1/2}) / 2.
// One workgroup; nodes held in LDS.
template <bool MIX>
__global__ void __launch_bounds__(1024) k_field1d(int nx, typename AccOf<MIX>::T *acc, double scale,
                                                  double add, double ion, double dx, int clear, double *E,
                                                  float *E32, double *we, double *charge, int step_mode,
                                                  CtxDev c) {
    extern __shared__ __align__(16) unsigned char smem[];
    double *sr = (double *)smem;          // [nx] rho, then half-node field
    __shared__ double sRed[16];
    __shared__ double sScan[1024];
    const int T = blockDim.x;
    double part = 0.0;
    for (int i = threadIdx.x; i < nx; i += T) {
        typename AccOf<MIX>::T v = acc[i];
        double w;
        if constexpr (MIX) w = (double)(int64_t)v;
        else w = v;
        double r = add + scale * w;
        sr[i] = r;
        part += r - ion;
        if (clear) acc[i] = (typename AccOf<MIX>::T)0;
    }
    double qsum = block_sum(part, sRed);
    // mean of rho, computed from the stored values in a fixed order
    double ps = 0.0;
    for (int i = threadIdx.x; i < nx; i += T) ps += sr[i];
    double mean = block_sum(ps, sRed) / (double)nx;
    // inclusive prefix sum of (rho - mean) dx: contiguous chunks per thread
    const int per = (nx + T - 1) / T;
    const int lo = threadIdx.x * per, hi = min(nx, lo + per);
    double loc = 0.0;
    for (int i = lo; i < hi; ++i) loc += (sr[i] - mean) * dx;
    sScan[threadIdx.x] = loc;
    __syncthreads();
    for (int off = 1; off < T; off <<= 1) {
        double add = (threadIdx.x >= (unsigned)off) ? sScan[threadIdx.x - off] : 0.0;
        __syncthreads();
        sScan[threadIdx.x] += add;
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
    double hmean = block_sum(hs, sRed) / (double)nx;
    double wpart = 0.0;
    for (int i = threadIdx.x; i < nx; i += T) {
        int im = (i == 0) ? nx - 1 : i - 1;
        double e = 0.5 * ((sr[im] - hmean) + (sr[i] - hmean));
        E[i] = e;
        if (E32) E32[i] = (float)e;
        wpart += e * e;
    }
    double wsum = block_sum(wpart, sRed);
    if (threadIdx.x == 0) {
        if (we) *(step_mode ? step_slot(we, c) : we) = 0.5 * wsum * dx;
        if (charge) *(step_mode ? step_slot(charge, c) : charge) = qsum * dx;
    }
}

inline int blocks_for(int64_t n, int cap = 4096) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    return (int)(b > cap ? cap : b);
}

inline size_t tile_e_bytes(const Geo &g, bool mixed) {
    const int ex_w = (1 << g.tsx) + 1, ey_w = (g.dim == 2) ? (1 << g.tsy) + 1 : 1;
    return (size_t)ex_w * ey_w * g.dim * (mixed ? 4 : 8);
}

inline size_t tile_acc_bytes(const Geo &g) {
    const int wx = (1 << g.tsx) + 1 + 2 * g.halo;
    const int wy = (g.dim == 2) ? (1 << g.tsy) + 1 + 2 * g.halo : 1;
    return (((size_t)wx * wy * 8) + 15) & ~(size_t)15;
}

}  // namespace

// ================================================================ launchers

#define APIC_DISPATCH(g, mixed, KERNEL_CALL)                                             \
    do {                                                                                 \
        if (mixed) {                                                                     \
            constexpr bool MIX = true;                                                   \
            if ((g).dim == 1) { constexpr int DIM = 1, VDIM = 1; KERNEL_CALL; }          \
            else if ((g).vdim == 2) { constexpr int DIM = 2, VDIM = 2; KERNEL_CALL; }    \
            else { constexpr int DIM = 2, VDIM = 3; KERNEL_CALL; }                       \
        } else {                                                                         \
            constexpr bool MIX = false;                                                  \
            if ((g).dim == 1) { constexpr int DIM = 1, VDIM = 1; KERNEL_CALL; }          \
            else if ((g).vdim == 2) { constexpr int DIM = 2, VDIM = 2; KERNEL_CALL; }    \
            else { constexpr int DIM = 2, VDIM = 3; KERNEL_CALL; }                       \
        }                                                                                \
    } while (0)

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n)), dim3(kBlock), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n)), dim3(kBlock), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_set_step(int *step, int v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, s, step, v);
    return hipGetLastError();
}

hipError_t launch_copy_bytes(void *dst, const void *src, int64_t bytes, hipStream_t s) {
    if (bytes <= 0) return hipSuccess;
    int64_t n16 = bytes / 16;
    int tail = (int)(bytes - n16 * 16);
    hipLaunchKernelGGL(k_copy_bytes, dim3(blocks_for(n16 > 0 ? n16 : 1)), dim3(kBlock), 0, s, (uint4 *)dst,
                       (const uint4 *)src, n16, (char *)dst + n16 * 16, (const char *)src + n16 * 16, tail);
    return hipGetLastError();
}

hipError_t launch_keys_hist(const Geo &g, bool mixed, const Parts &p, int64_t n, int32_t *keys, int32_t *count,
                            const CtxDev &c, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    APIC_DISPATCH(g, mixed,
                  hipLaunchKernelGGL((k_keys_hist<MIX, DIM, VDIM>), dim3(blocks_for(n)), dim3(kBlock), 0, s, g, p, n,
                                     keys, count, c));
    return hipGetLastError();
}

hipError_t launch_scan(const int32_t *count, int32_t *start, int32_t *cursor, int32_t *count_zero, int nb,
                       int64_t n, int64_t max_per_bucket, double *diag, const CtxDev &c, hipStream_t s) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, count, start, cursor, count_zero, nb, n, max_per_bucket,
                       diag, c);
    return hipGetLastError();
}

hipError_t launch_scatter(const Geo &g, bool mixed, const Parts &src, const Parts &dst, int64_t n,
                          const int32_t *keys, int32_t *cursor, const int32_t *start, int32_t *perm,
                          const CtxDev &c, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    APIC_DISPATCH(g, mixed,
                  hipLaunchKernelGGL((k_scatter<MIX, DIM, VDIM>), dim3(blocks_for(n)), dim3(kBlock), 0, s, g, src,
                                     dst, n, keys, cursor, start, perm, c));
    return hipGetLastError();
}

hipError_t launch_deposit(const Geo &g, bool mixed, const Parts &p, int64_t n, const int32_t *bstart, void *acc,
                          const CtxDev &c, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (bstart) {
        Geo g0 = g;
        g0.halo = 0;
        size_t sh = tile_acc_bytes(g0);
        APIC_DISPATCH(g, mixed,
                      hipLaunchKernelGGL((k_deposit_tiled<MIX, DIM, VDIM>), dim3(grid_for_buckets(g.nbuckets)),
                                         dim3(kBlock), sh, s, g0, p, bstart, (typename AccOf<MIX>::T *)acc, c));
    } else {
        APIC_DISPATCH(g, mixed,
                      hipLaunchKernelGGL((k_deposit_direct<MIX, DIM, VDIM>), dim3(blocks_for(n)), dim3(kBlock), 0, s,
                                         g, p, n, (typename AccOf<MIX>::T *)acc, c));
    }
    return hipGetLastError();
}

hipError_t launch_gather_push(const Geo &g, bool mixed, const Parts &p, int64_t n, const int32_t *bstart,
                              const void *E, const PushC &pc, const CtxDev &c, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (bstart) {
        size_t sh = tile_e_bytes(g, mixed);
        APIC_DISPATCH(g, mixed,
                      hipLaunchKernelGGL((k_gather_push_tiled<MIX, DIM, VDIM>), dim3(grid_for_buckets(g.nbuckets)),
                                         dim3(kBlock), sh, s, g, p, bstart, (const typename Pt<MIX>::R *)E, pc, c));
    } else {
        APIC_DISPATCH(g, mixed,
                      hipLaunchKernelGGL((k_gather_push_direct<MIX, DIM, VDIM>), dim3(blocks_for(n)), dim3(kBlock), 0,
                                         s, g, p, n, (const typename Pt<MIX>::R *)E, pc, c));
    }
    return hipGetLastError();
}

hipError_t launch_step_count(const Geo &g, bool mixed, const Parts &p, const int32_t *bstart, const void *E,
                             const PushC &pc, int32_t *count, const CtxDev &c, hipStream_t s) {
    size_t sh = tile_e_bytes(g, mixed);
    APIC_DISPATCH(g, mixed,
                  hipLaunchKernelGGL((k_step_count<MIX, DIM, VDIM>), dim3(grid_for_buckets(g.nbuckets)), dim3(kBlock),
                                     sh, s, g, p, bstart, (const typename Pt<MIX>::R *)E, pc, count, c));
    return hipGetLastError();
}

hipError_t launch_step_push(const Geo &g, bool mixed, const Parts &src, const Parts &dst, const int32_t *bstart,
                            const int32_t *bstart_new, int32_t *cursor, const void *E, const PushC &pc, void *acc,
                            int32_t *perm, double *diag, double mass, const CtxDev &c, hipStream_t s) {
    size_t sh = tile_acc_bytes(g) + tile_e_bytes(g, mixed);
    APIC_DISPATCH(g, mixed,
                  hipLaunchKernelGGL((k_step_push<MIX, DIM, VDIM>), dim3(grid_for_buckets(g.nbuckets)), dim3(kBlock),
                                     sh, s, g, src, dst, bstart, bstart_new, cursor, (const typename Pt<MIX>::R *)E,
                                     pc, (typename AccOf<MIX>::T *)acc, perm, diag, mass, c));
    return hipGetLastError();
}

hipError_t launch_rho(const Geo &g, bool mixed, void *acc, double *rho, double scale, double add, double ion,
                      double dV, int clear, double *charge_out, int step_mode, const CtxDev &c, hipStream_t s) {
    const int64_t G = (int64_t)g.nx * g.ny;
    const int nb = blocks_for(G, 1024);
    if (mixed)
        hipLaunchKernelGGL(k_rho<true>, dim3(nb), dim3(kBlock), 0, s, G, (unsigned long long *)acc, rho, scale, add,
                           ion, dV, clear, charge_out, step_mode, c);
    else
        hipLaunchKernelGGL(k_rho<false>, dim3(nb), dim3(kBlock), 0, s, G, (double *)acc, rho, scale, add, ion, dV,
                           clear, charge_out, step_mode, c);
    return hipGetLastError();
}

hipError_t launch_spectral(const Geo &g, const void *rho_hat, void *ex_hat, void *ey_hat, const CtxDev &c,
                           hipStream_t s) {
    const int64_t tot = (int64_t)(g.nx / 2 + 1) * g.ny;
    hipLaunchKernelGGL(k_spectral, dim3(blocks_for(tot)), dim3(kBlock), 0, s, g, (const double2 *)rho_hat,
                       (double2 *)ex_hat, (double2 *)ey_hat, c);
    return hipGetLastError();
}

hipError_t launch_efinish(const Geo &g, const double *E, float *E32, double dV, double *we_out, int step_mode,
                          const CtxDev &c, hipStream_t s) {
    const int64_t G = (int64_t)g.nx * g.ny;
    const int nb = blocks_for(G * g.dim, 1024);
    hipLaunchKernelGGL(k_efinish, dim3(nb), dim3(kBlock), 0, s, G, g.dim, E, E32, dV, we_out, step_mode, c);
    return hipGetLastError();
}

hipError_t launch_field1d(const Geo &g, bool mixed, void *acc, double scale, double add, double ion, double dx,
                          int clear, double *E, float *E32, double *we_out, double *charge_out, int step_mode,
                          const CtxDev &c, hipStream_t s) {
    size_t sh = (size_t)g.nx * sizeof(double);
    if (mixed)
        hipLaunchKernelGGL(k_field1d<true>, dim3(1), dim3(1024), sh, s, g.nx, (unsigned long long *)acc, scale, add,
                           ion, dx, clear, E, E32, we_out, charge_out, step_mode, c);
    else
        hipLaunchKernelGGL(k_field1d<false>, dim3(1), dim3(1024), sh, s, g.nx, (double *)acc, scale, add, ion, dx,
                           clear, E, E32, we_out, charge_out, step_mode, c);
    return hipGetLastError();
}

}  // namespace apic
