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
//    push and move computed, only the tallies of new buckets kept) and a push
//    pass that recomputes the same update bit for bit, deposits rho^{n+1} and
//    writes each particle straight to its slot of the next bucket order
//    (counting sort: histogram -> exclusive scan -> scatter). State traffic is
//    read + read + write per particle-step instead of read/write for the push
//    plus read/write for a separate sort. Slots come from a per-(bucket,
//    wave, direction) offset table, so the order, the deposit sums and all
//    reductions are reproducible run to run.
//  * The mixed path holds positions as an integer cell plus a binary32
//    in-cell offset and deposits with int64 fixed-point weights, so the charge
//    density is exact and independent of summation order.
//  * This file is compiled with -ffp-contract=off: the count pass and the push
//    pass must produce identical bits for the same particle.
#include <algorithm>

#include "apic_device.h"
#include "apic_em.h"

namespace apic {

namespace {

// ------------------------------------------------- step: bucket directions
//
// A particle of bucket (bx, by[, bz]) lands after the move in bucket
// (bx+dbx, by+dby[, bz+dbz]) (periodic). Moves with every |db| <= 1 get the
// direction code d = (dby+1)*3 + (dbx+1) in 0..8 (1D, 2D), or
// d = ((dbz+1)*3 + (dby+1))*3 + (dbx+1) in 0..26 (3D); larger jumps get the
// far code. The count pass tallies particles per (source bucket, wave, d);
// the scan turns the tallies into start offsets inside the destination
// buckets (ordered by d, then wave); the push pass hands out consecutive
// slots per (wave, d) in the order the wave meets its particles. The order is
// therefore fixed by the previous order alone: no atomics decide where a near
// particle goes. Far movers (rare) take slots from an atomic cursor at the
// end of their bucket.
template <int DIM> struct Dir {
    static constexpr int kN = (DIM == 3) ? 28 : 10;      // direction codes (near + far)
    static constexpr int kFar = kN - 1;
    static constexpr int kStay = (DIM == 3) ? 13 : 4;    // the code of a particle that stays
    static constexpr int kTab = kN;                      // per-bucket table entries (one per direction)
    static constexpr int kCodeBits = (DIM == 3) ? 5 : 4; // bits of a near code
};
static_assert(Dir<3>::kTab <= kStepTab && Dir<2>::kTab <= kStepTab, "direction table size");
static_assert(kDeepTab == 2, "deep table size");

// Tile coordinates of bucket b (tiles numbered x fastest, then y, then z).
template <int DIM>
__device__ __forceinline__ void tile_coords(const Geo &g, int b, int &bx, int &by, int &bz) {
    if constexpr (DIM == 1) {
        bx = b; by = 0; bz = 0;
    } else if constexpr (DIM == 2) {
        bx = b % g.nbx; by = b / g.nbx; bz = 0;
    } else {
        bx = b % g.nbx; const int r = b / g.nbx; by = r % g.nby; bz = r / g.nby;
    }
}

template <int DIM>
__device__ __forceinline__ int bucket_index(const Geo &g, int bx, int by, int bz) {
    if constexpr (DIM == 1) return bx;
    if constexpr (DIM == 2) return by * g.nbx + bx;
    return (bz * g.nby + by) * g.nbx + bx;
}

__device__ __forceinline__ int wrap_tile(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Bucket reached from (bx, by, bz) with near direction d.
template <int DIM>
__device__ __forceinline__ int dir_target(const Geo &g, int bx, int by, int bz, int d) {
    const int tx = wrap_tile(bx + d % 3 - 1, g.nbx);
    const int ty = (DIM >= 2) ? wrap_tile(by + (d / 3) % 3 - 1, g.nby) : 0;
    const int tz = (DIM == 3) ? wrap_tile(bz + d / 9 - 1, g.nbz) : 0;
    return bucket_index<DIM>(g, tx, ty, tz);
}

// Source bucket that reaches bucket nbk with direction d.
template <int DIM>
__device__ __forceinline__ int dir_source(const Geo &g, int nbk, int d) {
    int bx, by, bz;
    tile_coords<DIM>(g, nbk, bx, by, bz);
    const int sx = wrap_tile(bx - (d % 3 - 1), g.nbx);
    const int sy = (DIM >= 2) ? wrap_tile(by - ((d / 3) % 3 - 1), g.nby) : 0;
    const int sz = (DIM == 3) ? wrap_tile(bz - (d / 9 - 1), g.nbz) : 0;
    return bucket_index<DIM>(g, sx, sy, sz);
}

// Direction code from a particle's tile-local cell after the move, (lxn,
// lyn, lzn) = old tile-local cell + unwrapped cell shift: the widths of the
// tile and of its neighbours (the last tile of an axis may be cut by the grid
// edge; neighbours wrap periodically) decide whether it stayed, crossed into
// a neighbour, or jumped farther (the far code), without per-particle wrap
// arithmetic.
struct TileNb {
    int txe, lw, rw;   // widths (cells) of this tile and its left / right neighbour
    int tye, dw, uw;   // same along y
    int tze, bw, fw;   // same along z
};

__device__ __forceinline__ int tile_width(int i, int t, int n) { return min(t, n - i * t); }

// A wave-uniform 32-bit value moved into a vector register (when ON):
// per-lane arithmetic reads it from there, leaving the scalar registers to
// the state the chunk loop itself carries.
template <bool ON, typename T>
__device__ __forceinline__ T vreg(T x) {
    static_assert(sizeof(T) == 4, "a 32-bit value");
    if constexpr (ON) asm("" : "+v"(x));
    return x;
}

template <int DIM>
__device__ __forceinline__ TileNb tile_nb(const Geo &g, int bx, int by, int bz = 0) {
    TileNb t;
    const int T = 1 << g.tsx;
    t.txe = tile_width(bx, T, g.nx);
    t.lw = tile_width(bx == 0 ? g.nbx - 1 : bx - 1, T, g.nx);
    t.rw = tile_width(bx == g.nbx - 1 ? 0 : bx + 1, T, g.nx);
    t.tye = t.dw = t.uw = 1;
    t.tze = t.bw = t.fw = 1;
    if constexpr (DIM >= 2) {
        const int V = 1 << g.tsy;
        t.tye = tile_width(by, V, g.ny);
        t.dw = tile_width(by == 0 ? g.nby - 1 : by - 1, V, g.ny);
        t.uw = tile_width(by == g.nby - 1 ? 0 : by + 1, V, g.ny);
    }
    if constexpr (DIM == 3) {
        const int Z = 1 << g.tsz;
        t.tze = tile_width(bz, Z, g.nz);
        t.bw = tile_width(bz == 0 ? g.nbz - 1 : bz - 1, Z, g.nz);
        t.fw = tile_width(bz == g.nbz - 1 ? 0 : bz + 1, Z, g.nz);
    }
    return t;
}

template <int DIM>
__device__ __forceinline__ int dir_local(const TileNb &t, int lxn, int lyn, int lzn = 0) {
    const int dbx = (lxn < 0) ? -1 : (lxn >= t.txe) ? 1 : 0;
    bool far = lxn < -t.lw || lxn >= t.txe + t.rw;
    int dby = 0, dbz = 0;
    if constexpr (DIM >= 2) {
        dby = (lyn < 0) ? -1 : (lyn >= t.tye) ? 1 : 0;
        far = far || lyn < -t.dw || lyn >= t.tye + t.uw;
    }
    if constexpr (DIM == 3) {
        dbz = (lzn < 0) ? -1 : (lzn >= t.tze) ? 1 : 0;
        far = far || lzn < -t.bw || lzn >= t.tze + t.fw;
        return far ? Dir<3>::kFar : ((dbz + 1) * 3 + (dby + 1)) * 3 + (dbx + 1);
    }
    return far ? Dir<DIM>::kFar : (dby + 1) * 3 + (dbx + 1);
}

// Twice the kinetic energy per unit mass of a particle for the diagnostic:
// |v|^2 (binary32 squares on the mixed path, FP64 on the FP64 path), or for
// the Higuera-Cary state 2 (gamma - 1) c^2 = 2 |u|^2 / (gamma + 1): in FP64
// on the FP64 path, on the mixed path in binary32 with the hardware square
// root and reciprocal (each within 1 ulp; a diagnostic, summed in FP64).
template <bool MIX, int VDIM, bool HC>
__device__ __forceinline__ double vsq(const Pt<MIX> &q, const PushC &pc) {
    if constexpr (HC && MIX) {
        const float u2 = (q.vx * q.vx + q.vy * q.vy) + q.vz * q.vz;
        const float gp1 = __builtin_amdgcn_sqrtf(1.0f + u2 * pc.ic2f) + 1.0f;
        return (double)(2.0f * u2 * __builtin_amdgcn_rcpf(gp1));
    } else if constexpr (HC) {
        const double ux = q.vx, uy = q.vy, uz = q.vz;
        const double u2 = (ux * ux + uy * uy) + uz * uz;
        return 2.0 * u2 / (sqrt(1.0 + u2 * pc.ic2) + 1.0);
    }
    auto v2 = q.vx * q.vx;
    if constexpr (VDIM >= 2) v2 = v2 + q.vy * q.vy;
    if constexpr (VDIM >= 3) v2 = v2 + q.vz * q.vz;
    return (double)v2;
}

// Gather + Boris + move of one loaded particle of the block's tile; shared by
// the count and the push pass so that both compute identical bits. A particle
// outside the tile (the bucket table does not match the order) is flagged
// and clamped into the tile so that every access stays in bounds. The E tile
// spans ex_w x ey_w x ez_w nodes from (x0, y0, z0).
template <bool MIX, int DIM, int VDIM, bool HC>
__device__ __forceinline__ bool advance(Pt<MIX> &q, const Geo &g, const PushC &pc,
                                        const typename Pt<MIX>::R *sE, int ex_w, int ey_w, int ez_w, int x0, int y0,
                                        int z0, int &lx, int &ly, int &lz, int &sx, int &sy, int &sz) {
    using R = typename Pt<MIX>::R;
    lx = q.ix - x0;
    ly = (DIM >= 2) ? q.iy - y0 : 0;
    lz = (DIM == 3) ? q.iz - z0 : 0;
    bool in = (unsigned)lx < (unsigned)(ex_w - 1);
    if constexpr (DIM >= 2) in = in && (unsigned)ly < (unsigned)(ey_w - 1);
    if constexpr (DIM == 3) in = in && (unsigned)lz < (unsigned)(ez_w - 1);
    if (!in) {
        lx = min(max(lx, 0), ex_w - 2);
        ly = (DIM >= 2) ? min(max(ly, 0), ey_w - 2) : 0;
        lz = (DIM == 3) ? min(max(lz, 0), ez_w - 2) : 0;
        q.ix = x0 + lx;
        q.iy = y0 + ly;
        q.iz = z0 + lz;
    }
    R ex, ey, ez = R(0);
    if constexpr (DIM == 3) {
        const int wxy = ex_w * ey_w;
        gather_lds3<R>(sE, ex_w, wxy, wxy * ez_w, lx, ly, lz, q.fx, q.fy, q.fz, ex, ey, ez);
    } else {
        gather_lds<R, DIM>(sE, ex_w, ex_w * ey_w, lx, ly, q.fx, q.fy, ex, ey);
    }
    return push_move<MIX, DIM, VDIM, HC>(q, g, pc, ex, ey, ez, true, sx, sy, sz) && in;
}

// Electromagnetic form (2D3V): E and B gathered from the Yee field tile
// (nodes from (x0-1, y0-1), width fw), Boris (or Higuera-Cary with the state
// u = gamma v) in B, move. (lx, ly) and (fx0, fy0) return the old local cell
// and fractions for the current deposit, ig the factor 1 / gamma the move
// multiplied u by (1 for Boris).
template <bool MIX, bool HC>
__device__ __forceinline__ bool advance_em(Pt<MIX> &q, const Geo &g, const PushC &pc,
                                           const typename Pt<MIX>::R *sF, int fw, int x0, int y0, int &lx, int &ly,
                                           int &sx, int &sy, typename Pt<MIX>::R &fx0, typename Pt<MIX>::R &fy0,
                                           typename Pt<MIX>::R &ig) {
    using R = typename Pt<MIX>::R;
    const int tx = 1 << g.tsx, ty = 1 << g.tsy;
    lx = q.ix - x0;
    ly = q.iy - y0;
    const bool in = (unsigned)lx < (unsigned)tx && (unsigned)ly < (unsigned)ty;
    if (!in) {
        lx = min(max(lx, 0), tx - 1);
        ly = min(max(ly, 0), ty - 1);
        q.ix = x0 + lx;
        q.iy = y0 + ly;
    }
    fx0 = q.fx;
    fy0 = q.fy;
    R e[3], b[3];
    gather_em<R>(sF, fw, fw * (ty + 2), lx, ly, q.fx, q.fy, e, b);
    int sz;
    if constexpr (HC) {
        const R ic2 = MIX ? (R)pc.ic2f : (R)pc.ic2;
        hc3<R>(q.vx, q.vy, q.vz, e, b, MIX ? (R)pc.af : (R)pc.a, ic2);
        ig = recip<R>(lorentz<R>(q.vx, q.vy, q.vz, ic2));
        return move_pt_v<MIX, 2>(q, g, pc, q.vx * ig, q.vy * ig, q.vz * ig, sx, sy, sz) && in;
    } else {
        boris3<R>(q.vx, q.vy, q.vz, e, b, MIX ? (R)pc.af : (R)pc.a);
        ig = R(1);
        return move_pt<MIX, 2>(q, g, pc, sx, sy, sz) && in;
    }
}

// Raw stored words of one particle: loaded unconditionally (the caller clamps
// the index) so that a wave issues all its loads before it needs any data.
template <bool MIX> struct Raw {
    int32_t c;
    float ox, oy, oz, vx, vy, vz;
};
template <> struct Raw<false> {
    double x, y, z, vx, vy, vz;
};

template <bool MIX, int DIM, int VDIM>
__device__ __forceinline__ void load_raw(const Parts &s, int i, Raw<MIX> &r) {
    // each particle is read once per pass, in whole 128-byte lines per wave
    // (the passes align their chunks). The mixed state loads with the
    // nontemporal hint: measured at 512^2 (2D2V), 1024^2 (2D3V) and 128^3,
    // it was faster or equal; the FP64 state loads through the caches (the
    // hint made its push 5% slower). Nontemporal stores of the scattered
    // destination slots made the mixed push 1.6x slower.
    if constexpr (MIX) {
        r.c = __builtin_nontemporal_load(&s.cell[i]);
        r.ox = __builtin_nontemporal_load(&s.ox[i]);
        r.oy = (DIM >= 2) ? __builtin_nontemporal_load(&s.oy[i]) : 0.0f;
        r.oz = (DIM == 3) ? __builtin_nontemporal_load(&s.oz[i]) : 0.0f;
        r.vx = __builtin_nontemporal_load(&((const float *)s.vx)[i]);
        r.vy = (VDIM >= 2) ? __builtin_nontemporal_load(&((const float *)s.vy)[i]) : 0.0f;
        r.vz = (VDIM >= 3) ? __builtin_nontemporal_load(&((const float *)s.vz)[i]) : 0.0f;
    } else {
        r.x = s.x[i];
        r.y = (DIM >= 2) ? s.y[i] : 0.0;
        r.z = (DIM == 3) ? s.z[i] : 0.0;
        r.vx = ((const double *)s.vx)[i];
        r.vy = (VDIM >= 2) ? ((const double *)s.vy)[i] : 0.0;
        r.vz = (VDIM >= 3) ? ((const double *)s.vz)[i] : 0.0;
    }
}

// Decode raw words into the working form (same checks as load_pt).
template <bool MIX, int DIM, int VDIM>
__device__ __forceinline__ bool decode(const Raw<MIX> &r, const Geo &g, Pt<MIX> &p) {
    bool ok;
    if constexpr (MIX) {
        unpack_cell<DIM>(r.c, p.ix, p.iy, p.iz);
        p.fx = r.ox;
        p.fy = (DIM >= 2) ? r.oy : 0.0f;
        p.fz = (DIM == 3) ? r.oz : 0.0f;
        ok = (unsigned)p.ix < (unsigned)g.nx && (p.fx >= 0.0f) && (p.fx < 1.0f);
        if constexpr (DIM >= 2) ok = ok && (unsigned)p.iy < (unsigned)g.ny && (p.fy >= 0.0f) && (p.fy < 1.0f);
        if constexpr (DIM == 3) ok = ok && (unsigned)p.iz < (unsigned)g.nz && (p.fz >= 0.0f) && (p.fz < 1.0f);
        if (!ok) { p.ix = 0; p.iy = 0; p.iz = 0; p.fx = 0.0f; p.fy = 0.0f; p.fz = 0.0f; }
    } else {
        p.x = r.x;
        double f;
        ok = cell_f64(p.x, g.inv_dx, g.nx, p.ix, f);
        p.fx = f;
        p.y = 0.0; p.iy = 0; p.fy = 0.0;
        p.z = 0.0; p.iz = 0; p.fz = 0.0;
        if constexpr (DIM >= 2) {
            p.y = r.y;
            ok = cell_f64(p.y, g.inv_dy, g.ny, p.iy, f) && ok;
            p.fy = f;
        }
        if constexpr (DIM == 3) {
            p.z = r.z;
            ok = cell_f64(p.z, g.inv_dz, g.nz, p.iz, f) && ok;
            p.fz = f;
        }
    }
    p.vx = r.vx;
    p.vy = r.vy;
    p.vz = r.vz;
    return ok;
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

// ---- block-wide exclusive scan helper (1024 threads) ------------------------
// Scans vals[0..nb) into out[0..nb] (out[nb] = total) in chunks of
// 1024*kPer elements; returns the total in every thread.
constexpr int kScanPer = 16;

__device__ int64_t block_exclusive_scan(const int32_t *vals, int32_t *out, int nb, int64_t max_per, int &bad,
                                        int64_t *sh /* [32] */) {
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int base = 0; base < nb; base += blockDim.x * kScanPer) {
        int64_t loc[kScanPer];
        int64_t s = 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            int b = base + threadIdx.x * kScanPer + k;
            int64_t v = (b < nb) ? vals[b] : 0;
            if (v > max_per) bad = 1;
            loc[k] = v;
            s += v;
        }
        // inclusive wave scan of thread sums
        int64_t inc = s;
        for (int off = 1; off < 64; off <<= 1) {
            int64_t y = __shfl_up(inc, off);
            if (lane >= off) inc += y;
        }
        if (lane == 63) sh[w] = inc;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t r = 0;
            for (int i = 0; i < nw; ++i) {
                int64_t t = sh[i];
                sh[i] = r;
                r += t;
            }
            sh[nw] = r;
        }
        __syncthreads();
        int64_t run = carry + sh[w] + inc - s;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            int b = base + threadIdx.x * kScanPer + k;
            if (b < nb) out[b] = (int32_t)run;
            run += loc[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) carry += sh[nw];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[nb] = (int32_t)carry;
    __syncthreads();
    return carry;
}

// ---- step: destination totals -> scan -> per-source offsets -------------------
// tot [nb] (summed by the count pass) is scanned into start (the next bucket
// table) and cleared; the device step index advances when step_mode.
__global__ void __launch_bounds__(1024) k_scan_tot(int32_t *tot, int32_t *start, int nb, int64_t n,
                                                   int64_t max_per, int step_mode, int walls, CtxDev c) {
    __shared__ int64_t sh[32];
    int bad = 0;
    int64_t total = block_exclusive_scan(tot, start, nb, max_per, bad, sh);
    if (bad) raise_err(c.err, ERR_OVERFLOW);
    for (int b = threadIdx.x; b < nb; b += blockDim.x) tot[b] = 0;
    if (threadIdx.x == 0) {
        if (walls ? total > n : total != n) raise_err(c.err, ERR_COUNT);
        if (step_mode) *c.step = *c.step + 1;
    }
}

// ---- general sort: stable LSD radix sort of (bucket key, index) ----------------
// Keys are bucket indices; each pass orders by 8 more key bits, keeping the
// previous order among equal digits (stable), so the result is the stable
// counting sort of the input by bucket. Per pass: tallies per (chunk, wave,
// digit), one exclusive scan in (digit, chunk, wave) order, and a scatter that
// hands out slots per (wave, digit) in the order the wave meets its elements
// (lanes with equal digits are ranked with ballots). Each wave owns a
// contiguous range of its chunk, so (chunk, wave, element) order is input
// order and every pass is stable; no atomic decides an element's slot.
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortPer = 16;                    // elements per thread and chunk
constexpr int kSortChunk = kBlock * kSortPer;   // elements per chunk (block)
constexpr int kSortTab = kWaves * kRadix;       // tallies per chunk

template <bool MIX, int DIM, int VDIM>
__global__ void __launch_bounds__(kBlock) k_keys_init(Geo g, Parts p, int64_t n, int32_t *keys, int32_t *idx,
                                                      CtxDev c) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        Pt<MIX> q;
        bool ok = load_pt<MIX, DIM, VDIM>(p, i, g, q);
        if (g.walls && q.ix >= g.nxp) {
            // outside the box between the walls
            ok = false;
            q.ix = 0;
        }
        if (!ok) raise_err(c.err, ERR_DOMAIN);
        keys[i] = bucket_of<MIX, DIM>(g, q.ix, q.iy, q.iz);
        idx[i] = (int32_t)i;
    }
}

__global__ void __launch_bounds__(kBlock) k_radix_count(const int32_t *keys, int64_t n, int shift, int32_t *cnt) {
    __shared__ int32_t s[kSortTab];
    for (int t = threadIdx.x; t < kSortTab; t += blockDim.x) s[t] = 0;
    __syncthreads();
    const int w = threadIdx.x >> 6;
    // wave w owns the contiguous range [w*64*kSortPer, (w+1)*64*kSortPer) of the chunk
    const int64_t base = (int64_t)blockIdx.x * kSortChunk + (int64_t)w * 64 * kSortPer + __lane_id();
    for (int j = 0; j < kSortPer; ++j) {
        const int64_t i = base + j * 64;
        if (i < n) atomicAdd(&s[w * kRadix + ((keys[i] >> shift) & (kRadix - 1))], 1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kSortTab; t += blockDim.x) cnt[(int64_t)blockIdx.x * kSortTab + t] = s[t];
}

// Exclusive scan of the tallies in (digit, chunk, wave) order, in three
// launches that read the tally table row by row (thread d of a workgroup
// handles digit d, so every load and store is coalesced): per range of R
// chunks the digit totals, then (one workgroup) the first slot of every
// digit in every range, then the offsets inside each range.
static_assert(kRadix == kBlock, "one thread per digit");
constexpr int kRadixParts = 256;  // chunk ranges at most

__device__ __forceinline__ void chunk_range(int nchunks, int R, int &c0, int &c1) {
    c0 = (int)blockIdx.x * R;
    c1 = min(c0 + R, nchunks);
}

__global__ void __launch_bounds__(kBlock) k_radix_part(const int32_t *cnt, int nchunks, int R, int32_t *part) {
    const int d = threadIdx.x;
    int c0, c1;
    chunk_range(nchunks, R, c0, c1);
    int32_t s = 0;
    for (int ch = c0; ch < c1; ++ch) {
        const int32_t *row = cnt + (int64_t)ch * kSortTab + d;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) s += row[w * kRadix];
    }
    part[blockIdx.x * kRadix + d] = s;
}

// part[r][d] (digit d's tally in range r) becomes the slot where range r's
// elements of digit d start: sum of all lower digits plus digit d in ranges
// before r.
__global__ void __launch_bounds__(kBlock) k_radix_base(int32_t *part, int P) {
    __shared__ int32_t sw[kWaves];
    const int d = threadIdx.x, lane = d & 63, w = d >> 6;
    int32_t tot = 0;
#pragma unroll 16
    for (int r = 0; r < P; ++r) tot += part[r * kRadix + d];
    int32_t inc = tot;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) sw[w] = inc;
    __syncthreads();
    int32_t run = inc - tot;
    for (int i = 0; i < w; ++i) run += sw[i];
#pragma unroll 16
    for (int r = 0; r < P; ++r) {
        const int32_t t = part[r * kRadix + d];
        part[r * kRadix + d] = run;
        run += t;
    }
}

__global__ void __launch_bounds__(kBlock) k_radix_off(const int32_t *cnt, const int32_t *part, int nchunks, int R,
                                                      int32_t *off) {
    const int d = threadIdx.x;
    int c0, c1;
    chunk_range(nchunks, R, c0, c1);
    int32_t run = part[blockIdx.x * kRadix + d];
    for (int ch = c0; ch < c1; ++ch) {
        const int64_t a = (int64_t)ch * kSortTab + d;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const int32_t t = cnt[a + w * kRadix];
            off[a + w * kRadix] = run;
            run += t;
        }
    }
}

// Bucket table of the sorted keys: start[b] is the first position whose key
// is at least b (start[nb] = n). Position i (0 <= i <= n) writes the entries of
// the buckets in (key[i-1], key[i]], with key[-1] = -1 and key[n] = nb, so each
// entry has exactly one writer; the clamp keeps keys of out-of-domain
// particles (already reported) inside the table.
__global__ void k_bucket_bounds(const int32_t *key, int64_t n, int nb, int32_t *start) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
        const int lo = max(i == 0 ? 0 : key[i - 1] + 1, 0);
        const int hi = min(i == n ? nb : key[i], nb);
        for (int b = lo; b <= hi; ++b) start[b] = (int32_t)i;
    }
}

// Buckets holding more particles than the fixed-point node sums allow.
__global__ void k_bucket_check(const int32_t *start, int nb, int64_t max_per, CtxDev c) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x)
        if ((int64_t)start[b + 1] - start[b] > max_per) raise_err(c.err, ERR_OVERFLOW);
}

__global__ void __launch_bounds__(kBlock) k_radix_scatter(const int32_t *kin, const int32_t *iin, int32_t *kout,
                                                          int32_t *iout, int64_t n, int shift, const int32_t *off,
                                                          CtxDev c) {
    __shared__ int32_t sRun[kSortTab];
    for (int t = threadIdx.x; t < kSortTab; t += blockDim.x) sRun[t] = off[(int64_t)blockIdx.x * kSortTab + t];
    __syncthreads();
    const int w = threadIdx.x >> 6;
    const uint64_t lt = lanemask_lt();
    // same element -> wave mapping as k_radix_count; wave-major order is input order (stable)
    const int64_t base = (int64_t)blockIdx.x * kSortChunk + (int64_t)w * 64 * kSortPer + __lane_id();
    for (int j = 0; j < kSortPer; ++j) {
        const int64_t i = base + j * 64;
        const bool act = i < n;
        const int key = act ? kin[i] : 0;
        const int d = (key >> shift) & (kRadix - 1);
        // lanes holding the same digit
        uint64_t peers = __ballot(act);
#pragma unroll
        for (int bit = 0; bit < kRadixBits; ++bit) {
            const uint64_t bb = __ballot(act && ((d >> bit) & 1));
            peers &= ((d >> bit) & 1) ? bb : ~bb;
        }
        if (act) {
            const int basek = sRun[w * kRadix + d];
            const int slot = basek + (int)__popcll(peers & lt);
            if ((int)__lane_id() == __ffsll((unsigned long long)peers) - 1)
                sRun[w * kRadix + d] = basek + (int)__popcll(peers);
            if (slot >= 0 && slot < n) {
                kout[slot] = key;
                iout[slot] = iin[i];
            } else {
                raise_err(c.err, ERR_ORDER);
            }
        }
    }
}

// dst[j] = src[idx[j]] for every particle array; perm (optional) = idx.
template <bool MIX, int DIM, int VDIM>
__global__ void __launch_bounds__(kBlock) k_gather_parts(Parts src, Parts dst, int64_t n, const int32_t *idx,
                                                         int32_t *perm, CtxDev c) {
    using R = typename Pt<MIX>::R;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx[j];
        if (i < 0 || i >= n) {
            raise_err(c.err, ERR_ORDER);
            continue;
        }
        if constexpr (MIX) {
            dst.cell[j] = src.cell[i];
            dst.ox[j] = src.ox[i];
            if constexpr (DIM >= 2) dst.oy[j] = src.oy[i];
            if constexpr (DIM == 3) dst.oz[j] = src.oz[i];
        } else {
            dst.x[j] = src.x[i];
            if constexpr (DIM >= 2) dst.y[j] = src.y[i];
            if constexpr (DIM == 3) dst.z[j] = src.z[i];
        }
        ((R *)dst.vx)[j] = ((const R *)src.vx)[i];
        if constexpr (VDIM >= 2) ((R *)dst.vy)[j] = ((const R *)src.vy)[i];
        if constexpr (VDIM >= 3) ((R *)dst.vz)[j] = ((const R *)src.vz)[i];
        if (perm) perm[j] = (int32_t)i;
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
        typename AccOf<MIX>::T w[8];
        dep_weights<MIX, DIM>(q, g, w);
        if constexpr (DIM == 3)
            deposit_global3<MIX>(acc, g, q.ix, q.iy, q.iz, w);
        else
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
    int bx, by, bz;
    tile_coords<DIM>(g, b, bx, by, bz);
    const int x0 = bx << g.tsx, y0 = (DIM >= 2) ? (by << g.tsy) : 0, z0 = (DIM == 3) ? (bz << g.tsz) : 0;
    const int wx = (1 << g.tsx) + 1;
    const int wy = (DIM >= 2) ? (1 << g.tsy) + 1 : 1;
    const int wz = (DIM == 3) ? (1 << g.tsz) + 1 : 1;
    for (int t = threadIdx.x; t < wx * wy * wz; t += blockDim.x) sA[t] = (A)0;
    __syncthreads();
    const int i0 = min(max(bstart[b], 0), g.np), i1 = min(max(bstart[b + 1], i0), g.np);
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        Pt<MIX> q;
        if (!load_pt<MIX, DIM, VDIM>(p, i, g, q)) {
            raise_err(c.err, ERR_DOMAIN);
            continue;
        }
        A w[8];
        dep_weights<MIX, DIM>(q, g, w);
        int lx = q.ix - x0;
        int ly = (DIM >= 2) ? q.iy - y0 : 0;
        int lz = (DIM == 3) ? q.iz - z0 : 0;
        bool inl = (lx >= 0) && (lx <= wx - 2);
        if constexpr (DIM >= 2) inl = inl && ly >= 0 && ly <= wy - 2;
        if constexpr (DIM == 3) inl = inl && lz >= 0 && lz <= wz - 2;
        if (inl) {
            int a = (lz * wy + ly) * wx + lx;
            acc_add_lds<MIX>(&sA[a], w[0]);
            acc_add_lds<MIX>(&sA[a + 1], w[1]);
            if constexpr (DIM >= 2) {
                acc_add_lds<MIX>(&sA[a + wx], w[2]);
                acc_add_lds<MIX>(&sA[a + wx + 1], w[3]);
            }
            if constexpr (DIM == 3) {
                const int wxy = wx * wy;
                acc_add_lds<MIX>(&sA[a + wxy], w[4]);
                acc_add_lds<MIX>(&sA[a + wxy + 1], w[5]);
                acc_add_lds<MIX>(&sA[a + wxy + wx], w[6]);
                acc_add_lds<MIX>(&sA[a + wxy + wx + 1], w[7]);
            }
        } else {
            raise_err(c.err, ERR_ORDER);
            if constexpr (DIM == 3)
                deposit_global3<MIX>(acc, g, q.ix, q.iy, q.iz, w);
            else
                deposit_global<MIX, DIM>(acc, g, q.ix, q.iy, w);
        }
    }
    __syncthreads();
    if constexpr (DIM == 3)
        flush_region3<MIX>(acc, sA, g, x0, y0, z0, wx, wy, wz, 0);
    else
        flush_region<MIX, DIM>(acc, sA, g, x0, y0, wx, wy, 0);
}

// ---- gather + push (+ move), in place -------------------------------------------
template <bool MIX, int DIM, int VDIM, bool HC>
__global__ void __launch_bounds__(kBlock) k_gather_push_direct(Geo g, Parts p, int64_t n,
                                                               const typename Pt<MIX>::R *E, PushC pc,
                                                               CtxDev c) {
    using R = typename Pt<MIX>::R;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
        Pt<MIX> q;
        if (!load_pt<MIX, DIM, VDIM>(p, i, g, q)) {
            raise_err(c.err, ERR_DOMAIN);
            continue;
        }
        R ex, ey, ez = R(0);
        if constexpr (DIM == 3)
            gather_global3<R, R>(E, g, q.ix, q.iy, q.iz, q.fx, q.fy, q.fz, ex, ey, ez);
        else
            gather_global<R, R, DIM>(E, g, q.ix, q.iy, q.fx, q.fy, ex, ey);
        int sx, sy, sz;
        if (!push_move<MIX, DIM, VDIM, HC>(q, g, pc, ex, ey, ez, pc.move != 0, sx, sy, sz))
            raise_err(c.err, ERR_DOMAIN);
        store_pt<MIX, DIM, VDIM>(p, i, q);
    }
}

template <bool MIX, int DIM, int VDIM, bool HC>
__global__ void __launch_bounds__(kBlock) k_gather_push_tiled(Geo g, Parts p, const int32_t *bstart,
                                                              const typename Pt<MIX>::R *E, PushC pc,
                                                              CtxDev c) {
    using R = typename Pt<MIX>::R;
    extern __shared__ __align__(16) unsigned char smem[];
    R *sE = (R *)smem;
    const int b = bucket_of_block(g.nbuckets);
    if (b >= g.nbuckets) return;
    int bx, by, bz;
    tile_coords<DIM>(g, b, bx, by, bz);
    const int x0 = bx << g.tsx, y0 = (DIM >= 2) ? (by << g.tsy) : 0, z0 = (DIM == 3) ? (bz << g.tsz) : 0;
    const int ex_w = (1 << g.tsx) + 1, ey_w = (DIM >= 2) ? (1 << g.tsy) + 1 : 1;
    const int ez_w = (DIM == 3) ? (1 << g.tsz) + 1 : 1;
    if constexpr (DIM == 3)
        load_e_tile3<R, R>(sE, E, g, x0, y0, z0, ex_w, ey_w, ez_w);
    else
        load_e_tile<R, R, DIM>(sE, E, g, x0, y0, ex_w, ey_w);
    __syncthreads();
    const int i0 = min(max(bstart[b], 0), g.np), i1 = min(max(bstart[b + 1], i0), g.np);
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        Pt<MIX> q;
        if (!load_pt<MIX, DIM, VDIM>(p, i, g, q)) {
            raise_err(c.err, ERR_DOMAIN);
            continue;
        }
        const int lx = q.ix - x0, ly = (DIM >= 2) ? q.iy - y0 : 0, lz = (DIM == 3) ? q.iz - z0 : 0;
        bool inl = lx >= 0 && lx < ex_w - 1;
        if constexpr (DIM >= 2) inl = inl && ly >= 0 && ly < ey_w - 1;
        if constexpr (DIM == 3) inl = inl && lz >= 0 && lz < ez_w - 1;
        R ex, ey, ez = R(0);
        if constexpr (DIM == 3) {
            if (inl) {
                const int wxy = ex_w * ey_w;
                gather_lds3<R>(sE, ex_w, wxy, wxy * ez_w, lx, ly, lz, q.fx, q.fy, q.fz, ex, ey, ez);
            } else {
                raise_err(c.err, ERR_ORDER);
                gather_global3<R, R>(E, g, q.ix, q.iy, q.iz, q.fx, q.fy, q.fz, ex, ey, ez);
            }
        } else {
            if (inl) {
                gather_lds<R, DIM>(sE, ex_w, ex_w * ey_w, lx, ly, q.fx, q.fy, ex, ey);
            } else {
                raise_err(c.err, ERR_ORDER);
                gather_global<R, R, DIM>(E, g, q.ix, q.iy, q.fx, q.fy, ex, ey);
            }
        }
        int sx, sy, sz;
        if (!push_move<MIX, DIM, VDIM, HC>(q, g, pc, ex, ey, ez, pc.move != 0, sx, sy, sz))
            raise_err(c.err, ERR_DOMAIN);
        store_pt<MIX, DIM, VDIM>(p, i, q);
    }
}

// ---- fused step, pass 1: direction tallies ------------------------------------
// Same arithmetic as k_step_push up to the new cell; keeps only the tallies
// per (bucket, direction) and counts far movers at their destination.
// U particles per thread are loaded before any is processed (more loads in
// flight per wave).
//
// The deep range (see the push pass) is skipped when the tile's field cannot
// move a deep particle out of the tile: 2|a| max|E| dt/dx, with slack for
// rounding, below pc.deep. Its particles are credited as stays; the remaining
// particles run the full computation and are tallied with LDS atomics.
// EM: the electromagnetic form (FP64 2D3V): E is the [6][G] Yee field.
// E32 (mixed path, may be NULL): E already rounded to binary32, read instead.
template <bool MIX, int DIM, int VDIM, int U, bool HC, bool EM>
__global__ void __launch_bounds__(kSBlock) k_step_count(Geo g, Parts p, const int32_t *bstart, const double *E,
                                                       const float *E32, PushC pc, int32_t *cnt, int32_t *tot, int32_t *farcnt,
                                                       const int32_t *deep, CtxDev c) {
    static_assert(!EM || (DIM == 2 && VDIM == 3), "the electromagnetic step is 2D3V");
    using R = typename Pt<MIX>::R;
    constexpr int kFar = Dir<DIM>::kFar, kStay = Dir<DIM>::kStay, kTab = Dir<DIM>::kTab;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int sErr;
    __shared__ int32_t sCnt[kTab];
    __shared__ float sMax[kSWaves][3];
    R *sE = (R *)smem;
    const int w = threadIdx.x >> 6;
    const uint64_t lt = lanemask_lt();
    const int ex_w = (1 << g.tsx) + 1, ey_w = (DIM >= 2) ? (1 << g.tsy) + 1 : 1;
    const int ez_w = (DIM == 3) ? (1 << g.tsz) + 1 : 1;
    const int fw = EM ? (1 << g.tsx) + 2 : 0, fh = EM ? (1 << g.tsy) + 2 : 0;
    if (threadIdx.x == 0) sErr = 0;
    int first, end, stride;
    bucket_walk(g.nbuckets, first, end, stride);
    for (int b = first; b < end; b += stride) {
        int bx, by, bz;
        tile_coords<DIM>(g, b, bx, by, bz);
        const int x0 = bx << g.tsx, y0 = (DIM >= 2) ? (by << g.tsy) : 0, z0 = (DIM == 3) ? (bz << g.tsz) : 0;
        const TileNb tn = tile_nb<DIM>(g, bx, by, bz);
        if (threadIdx.x < kTab) sCnt[threadIdx.x] = 0;
        // the bucket's range and the previous push's deep ranges, read with the
        // field tile (one memory round trip for all three)
        const int i0 = min(max(bstart[b], 0), g.np), i1 = min(max(bstart[b + 1], i0), g.np);
        const int span = i1 - i0;
        // every wave reads whole 128-byte lines of the particle arrays: chunks
        // start at the line boundary at or below the bucket's first particle
        // (32 binary32 or 16 FP64 elements per line), index k at chunk
        // position k + sh (the push uses the same positions, so the waves'
        // tallies agree)
        const int sh = i0 & (MIX ? 31 : 15);
        const int send = span > 0 ? span + sh : 0;
        const int draw0 = deep[b * kDeepTab], draw1 = deep[b * kDeepTab + 1];
        if constexpr (EM)
            load_f_tile<R>((R *)smem, E, g, x0, y0, fw, fh);
        else if (MIX && E32)
            load_tile_any<R, float, DIM>(sE, E32, g, x0, y0, z0, ex_w, ey_w, ez_w);
        else
            load_tile_any<R, double, DIM>(sE, E, g, x0, y0, z0, ex_w, ey_w, ez_w);
        __syncthreads();
        // field bound of the tile: per axis, or the in-plane |E| when the push
        // rotates v about z (on the node-centred grid the gathered E is a
        // convex combination of node vectors, so its norm is at most the
        // largest node norm), or, on the staggered Yee grid (EM), where each
        // component is interpolated with its own weights,
        // sqrt(max|Ex|^2 + max|Ey|^2 + max|Ez|^2) from per-component maxima
        {
            float e0 = 0.0f, e1 = 0.0f, e2 = 0.0f;
            const int tn = EM ? fw * fh : ex_w * ey_w * ez_w;
            for (int t = threadIdx.x; t < tn; t += blockDim.x) {
                const float ex = fabsf((float)sE[t]);
                const float ey = (DIM >= 2) ? fabsf((float)sE[tn + t]) : 0.0f;
                if constexpr (EM) {
                    e0 = fmaxf(e0, ex);
                    e1 = fmaxf(e1, ey);
                    e2 = fmaxf(e2, fabsf((float)sE[2 * tn + t]));
                } else if (pc.rot) {
                    e0 = fmaxf(e0, sqrtf(ex * ex + ey * ey));
                } else {
                    e0 = fmaxf(e0, ex);
                    e1 = fmaxf(e1, ey);
                }
                if constexpr (DIM == 3) e2 = fmaxf(e2, fabsf((float)sE[2 * tn + t]));
            }
            for (int off = 32; off > 0; off >>= 1) {
                e0 = fmaxf(e0, __shfl_xor(e0, off));
                e1 = fmaxf(e1, __shfl_xor(e1, off));
                e2 = fmaxf(e2, __shfl_xor(e2, off));
            }
            if ((threadIdx.x & 63) == 0) {
                sMax[w][0] = e0;
                sMax[w][1] = (pc.rot && !EM) ? e0 : e1;
                sMax[w][2] = e2;
            }
        }
        __syncthreads();
        float emx = 0.0f, emy = 0.0f, emz = 0.0f;
        for (int w2 = 0; w2 < kSWaves; ++w2) {
            emx = fmaxf(emx, sMax[w2][0]);
            emy = fmaxf(emy, sMax[w2][1]);
            emz = fmaxf(emz, sMax[w2][2]);
        }
        if constexpr (EM) {
            // a general B can turn the whole kick along either axis
            emx = emy = sqrtf(emx * emx + emy * emy + emz * emz);
        }
        const float kick = 2.0f * fabsf(MIX ? pc.af : (float)pc.a) * 1.0009765625f;
        bool skip = kick * emx * pc.dtdx + 0.0009765625f <= pc.deep;
        if constexpr (DIM >= 2) skip = skip && kick * emy * pc.dtdy + 0.0009765625f <= pc.deep;
        if constexpr (DIM == 3) skip = skip && kick * emz * pc.dtdz + 0.0009765625f <= pc.deep;
        // the deep range of this bucket, inside [0, span)
        const int da = skip ? min(max(draw0, 0), span) : 0;
        const int ndeep = skip ? min(max(draw1, 0), span - da) : 0;
        if (ndeep > 0) {
            if (threadIdx.x == 0) atomicAdd(&sCnt[kStay], ndeep);
            // the shallow particles: indices of [0, span) outside the deep
            // range, two register sets with each chunk's loads issued one
            // chunk ahead of its use
            const int nsh = span - ndeep;
            auto kmap = [&](int t) { return t >= da ? t + ndeep : t; };
            auto sfetch = [&](Raw<MIX> &r1, int t) {
                load_raw<MIX, DIM, VDIM>(p, i0 + kmap(min(t, nsh - 1)), r1);
                __builtin_amdgcn_sched_barrier(0);
            };
            auto sprocess = [&](const Raw<MIX> &r1, int t) {
                if (t >= nsh) return;
                Pt<MIX> q;
                bool good = decode<MIX, DIM, VDIM>(r1, g, q);
                int lx, ly, lz = 0, sx, sy, sz = 0;
                if constexpr (EM) {
                    R f0x, f0y, ig;
                    good = advance_em<MIX, HC>(q, g, pc, (const R *)smem, fw, x0, y0, lx, ly, sx, sy, f0x, f0y, ig) &&
                           good;
                } else {
                    good = advance<MIX, DIM, VDIM, HC>(q, g, pc, sE, ex_w, ey_w, ez_w, x0, y0, z0, lx, ly, lz, sx, sy,
                                                       sz) && good;
                }
                if (!good) atomicOr(&sErr, ERR_DOMAIN);
                if (g.walls && q.ix >= g.nxp) return;   // absorbed by a wall: leaves the order
                const int code = dir_local<DIM>(tn, lx + sx, ly + sy, lz + sz);
                if (code < kFar) {
                    atomicAdd(&sCnt[code], 1);
                } else {
                    const int nbk = bucket_of<MIX, DIM>(g, q.ix, q.iy, q.iz);
                    atomicAdd(&farcnt[nbk], 1);
                    atomicAdd(&tot[nbk], 1);
                }
            };
            Raw<MIX> sa, sb;
            if (nsh > 0) sfetch(sa, threadIdx.x);
            for (int t0 = 0; t0 < nsh; t0 += 2 * kSBlock) {
                if (t0 + kSBlock < nsh) sfetch(sb, t0 + kSBlock + threadIdx.x);
                sprocess(sa, t0 + threadIdx.x);
                if (t0 + 2 * kSBlock < nsh) sfetch(sa, t0 + 2 * kSBlock + threadIdx.x);
                if (t0 + kSBlock < nsh) sprocess(sb, t0 + kSBlock + threadIdx.x);
            }
        } else {
        // two register sets, each chunk's loads issued one chunk ahead of its use
        constexpr int CH = kSBlock * U;
        Raw<MIX> ra[U], rb[U];
        auto fetch = [&](Raw<MIX> *r, int base) {
#pragma unroll
            for (int j = 0; j < U; ++j)
                load_raw<MIX, DIM, VDIM>(p, i0 + min(max(base + j * kSBlock + (int)threadIdx.x - sh, 0), span - 1),
                                         r[j]);
            // keep these loads where they are: issued one chunk ahead of their use
            __builtin_amdgcn_sched_barrier(0);
        };
        auto process = [&](Raw<MIX> *r, int base) {
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int k = base + j * kSBlock + (int)threadIdx.x - sh;
                const bool act = k >= 0 && k < span;
                int code = -1, nbk = 0;
                if (act) {
                    Pt<MIX> q;
                    bool good = decode<MIX, DIM, VDIM>(r[j], g, q);
                    int lx, ly, lz = 0, sx, sy, sz = 0;
                    if constexpr (EM) {
                        R f0x, f0y, ig;
                        good = advance_em<MIX, HC>(q, g, pc, (const R *)smem, fw, x0, y0, lx, ly, sx, sy, f0x, f0y,
                                                   ig) && good;
                    } else {
                        good = advance<MIX, DIM, VDIM, HC>(q, g, pc, sE, ex_w, ey_w, ez_w, x0, y0, z0, lx, ly, lz, sx,
                                                           sy, sz) && good;
                    }
                    if (!good) atomicOr(&sErr, ERR_DOMAIN);
                    code = dir_local<DIM>(tn, lx + sx, ly + sy, lz + sz);
                    if (g.walls && q.ix >= g.nxp) code = -1;   // absorbed by a wall: leaves the order
                    if (code == kFar) nbk = bucket_of<MIX, DIM>(g, q.ix, q.iy, q.iz);
                }
                // lanes sharing a near code, from one ballot per code bit; the
                // group's lowest lane adds the group's size
                const bool near = code >= 0 && code < kFar;
                uint64_t peers = __ballot(near);
#pragma unroll
                for (int bit = 0; bit < Dir<DIM>::kCodeBits; ++bit) {
                    const uint64_t bb = __ballot(near && ((code >> bit) & 1));
                    peers &= ((code >> bit) & 1) ? bb : ~bb;
                }
                if (near && (peers & lt) == 0) atomicAdd(&sCnt[code], (int)__popcll(peers));
                if (code == kFar) {
                    atomicAdd(&farcnt[nbk], 1);
                    atomicAdd(&tot[nbk], 1);
                }
            }
        };
        if (span > 0) fetch(ra, 0);
        for (int base = 0; base < send; base += 2 * CH) {
            if (base + CH < send) fetch(rb, base + CH);
            process(ra, base);
            if (base + 2 * CH < send) fetch(ra, base + 2 * CH);
            if (base + CH < send) process(rb, base + CH);
        }
        }
        __syncthreads();
        if (threadIdx.x < kTab) cnt[b * kTab + threadIdx.x] = sCnt[threadIdx.x];
        if (threadIdx.x < kFar) {
            const int v = sCnt[threadIdx.x];
            if (v) atomicAdd(&tot[dir_target<DIM>(g, bx, by, bz, threadIdx.x)], v);
        }
        __syncthreads();
    }
    __syncthreads();
    if (threadIdx.x == 0 && sErr) raise_err(c.err, sErr);
}

// ---- fused step: first slot of every tally inside its destination bucket -----
// One wave per destination bucket nbk: its incoming tallies, in direction
// order, are prefix-summed from the bucket's new start. Every (source bucket,
// near direction) entry has exactly one destination, so each offs entry is
// written once.
template <int DIM>
__device__ __forceinline__ void dest_offsets_wave(const Geo &g, int nbk, int run, const int32_t *cnt, int32_t *offs) {
    constexpr int kFar = Dir<DIM>::kFar, kTab = Dir<DIM>::kTab;
    static_assert(kFar <= 64, "one lane per incoming direction");
    const int lane = threadIdx.x & 63;
    const bool ok = lane < kFar;
    const int d = ok ? lane : 0;
    const int src = ok ? dir_source<DIM>(g, nbk, d) : 0;
    const int v = ok ? cnt[src * kTab + d] : 0;
    int inc = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (ok) offs[src * kTab + d] = run + inc - v;
}

template <int DIM>
__global__ void __launch_bounds__(kSBlock) k_dest_offsets(Geo g, const int32_t *cnt, const int32_t *start,
                                                         int32_t *offs) {
    const int nbk = (int)blockIdx.x * kSWaves + (int)(threadIdx.x >> 6);
    if (nbk >= g.nbuckets) return;      // whole waves leave together; no barrier below
    dest_offsets_wave<DIM>(g, nbk, start[nbk], cnt, offs);
}

// The bucket-total scan and the offsets in one launch, for grids of at most
// kFusedScanMax buckets: every workgroup sums the totals of the buckets before
// its own (a few KiB, cache resident) instead of waiting for a separate scan.
// Also as k_scan_tot: the per-bucket headroom check, the new bucket_start
// (start[nb] by the last workgroup, with the count check), the step counter
// (workgroup 0). The totals of the next step live in tot_next, cleared here
// bucket by bucket; tot itself is read by every workgroup and is cleared by
// the next step's launch (the two buffers alternate).
constexpr int kFusedScanMax = 4096;

__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t *sh /* [kSWaves] */) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    int64_t t = 0;
    for (int i = 0; i < kSWaves; ++i) t += sh[i];
    return t;
}

template <int DIM>
__global__ void __launch_bounds__(kSBlock) k_scan_offsets(Geo g, const int32_t *tot, int32_t *tot_next,
                                                         int32_t *start, int64_t n, int64_t max_per, int step_mode,
                                                         int walls, const int32_t *cnt, int32_t *offs, CtxDev c) {
    __shared__ int64_t sh[kSWaves];
    const int nb = g.nbuckets;
    const int first = (int)blockIdx.x * kSWaves;
    int64_t part = 0;
    for (int b = threadIdx.x; b < first; b += blockDim.x) part += tot[b];
    const int64_t base = block_sum_i64(part, sh);
    const int w = threadIdx.x >> 6;
    const int nbk = first + w;
    int64_t run = base;
    for (int w2 = 0; w2 < w && first + w2 < nb; ++w2) run += tot[first + w2];
    if (nbk >= nb) return;              // whole waves leave together; no barrier below
    const int own = tot[nbk];
    if ((threadIdx.x & 63) == 0) {
        start[nbk] = (int32_t)run;
        tot_next[nbk] = 0;
        if (own > max_per) raise_err(c.err, ERR_OVERFLOW);
        if (nbk == nb - 1) {
            const int64_t total = run + own;
            start[nb] = (int32_t)total;
            if (walls ? total > n : total != n) raise_err(c.err, ERR_COUNT);
        }
        if (nbk == 0 && step_mode) *c.step = *c.step + 1;
    }
    dest_offsets_wave<DIM>(g, nbk, (int)run, cnt, offs);
}

// ---- fused step, pass 2: push, deposit, scatter into the next bucket order -----
// Slots are handed out per workgroup: each direction of the bucket (its stay
// range, and its range inside every neighbour bucket) is filled in the order
// of the bucket's chunks, and within a chunk in wave order, then lane order.
// After each chunk the waves publish their counts in LDS and, past one
// barrier, every wave takes its offsets from the counts of the waves before
// it. The bucket then writes to one advancing run per range instead of one
// per (wave, range): far fewer concurrent write streams into HBM.
// Staying particles are split by how far they sit from their tile's edges
// after the move: a particle whose distance to every edge exceeds its own
// displacement at the current velocity, |v| dt/dx, by at least pc.deep cells
// is "deep" and takes its slot from the front of the bucket's stay range; the
// others fill that range from the back. The deep part of the range goes to
// the deep table, so that the next count pass can credit those particles as
// stays without reading them, as long as the field's share of the next move,
// 2|a| max|E| dt/dx, stays below pc.deep.
// EM: the electromagnetic form (FP64 2D3V): E is the [6][G] Yee field and
// acc the [3][G] current J^{n+1/2} (Esirkepov), accumulated with atomics.
// VR (mixed electrostatic push only): the tile's constants, and in 2D the
// call's, held in vector registers (vreg). This variant spills no scalar
// registers inside the chunk loop but needs more vector registers; the
// launch takes it where that costs no resident workgroup.
// The mixed electromagnetic push (Boris), bound by its vector ALU work, holds
// its tile constants in vector registers too and is compiled for five waves
// per SIMD (96 vector registers), the most its LDS tile allows at 32 x 16.
template <bool MIX, bool HC, bool EM>
constexpr int push_waves() { return (MIX && EM && !HC) ? 5 : 1; }

template <bool MIX, int DIM, int VDIM, int U, bool HC, bool EM, bool VR = false>
__global__ void __launch_bounds__(kSBlock, (push_waves<MIX, HC, EM>())) k_step_push(Geo g, Parts src, Parts dst, const int32_t *bstart,
                                                      const int32_t *bstart_new, const int32_t *cnt,
                                                      const int32_t *offs, int32_t *farcnt, const double *E,
                                                      const float *E32, PushC pc,
                                                      typename AccOf<MIX>::T *acc, int32_t *perm, double *part,
                                                      int32_t *deep_out, CtxDev c) {
    using R = typename Pt<MIX>::R;
    using A = typename AccOf<MIX>::T;
    constexpr int kFar = Dir<DIM>::kFar, kStay = Dir<DIM>::kStay, kTab = Dir<DIM>::kTab;
    constexpr int kCodeBits = Dir<DIM>::kCodeBits;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int sErr;
    __shared__ double sRed[kSWaves];
    __shared__ int32_t sRunEnd[kTab];  // end of each direction's slot range
    __shared__ int32_t sEnd[kFar];     // end of each destination bucket (slot bound)
    __shared__ int32_t sStay[2];       // the stay range [first, end)
    __shared__ int32_t sCur[kSWaves][kTab];  // each wave's copy of the movers' next slots
    // per-chunk counts, double-buffered by chunk parity: each wave's movers per
    // direction (valid when its flag is set) and a packed word with its deep
    // count, shallow count and mover flag
    __shared__ int32_t sMv[2][kSWaves][kTab];
    __shared__ int32_t sPk[2][kSWaves];
    const int ex_w = (1 << g.tsx) + 1, ey_w = (DIM >= 2) ? (1 << g.tsy) + 1 : 1;
    const int ez_w = (DIM == 3) ? (1 << g.tsz) + 1 : 1;
    const int wx = (1 << g.tsx) + 1 + 2 * g.halo;
    const int wy = (DIM >= 2) ? (1 << g.tsy) + 1 + 2 * g.halo : 1;
    const int wz = (DIM == 3) ? (1 << g.tsz) + 1 + 2 * g.halo : 1;
    const int wxy = wx * wy;
    // EM: current tile jw x jh per component from node (x0-1, y0-1), then the
    // six-component field tile fw x fh
    const int jw = EM ? (1 << g.tsx) + 3 : 0, jh = EM ? (1 << g.tsy) + 3 : 0;
    const int fw = EM ? (1 << g.tsx) + 2 : 0, fh = EM ? (1 << g.tsy) + 2 : 0;
    const size_t acc_bytes = EM ? (size_t)3 * jw * jh * sizeof(double) : (size_t)wxy * wz * sizeof(A);
    A *sA = (A *)smem;
    R *sE = (R *)(smem + ((acc_bytes + 15) & ~(size_t)15));
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const uint64_t lt = lanemask_lt();
    const int lane = (int)(threadIdx.x & 63);
    int it = 0;   // chunks processed by this workgroup (the parity picks the count table)
    static_assert(!VR || (MIX && !HC && !EM), "the register-relieved build is the mixed electrostatic push");
    constexpr bool kVt = VR || (MIX && EM && !HC), kVc = VR && DIM == 2;
    // the LDS tiles' strides as the per-particle code reads them (in vector
    // registers in 2D; in 3D they would cost the VR build a wave per SIMD)
    const int pwx = vreg<kVc>(wx), pwy = vreg<kVc>(wy), pwxy = vreg<kVc>(wxy);
    const int pex = vreg<kVc>(ex_w), pey = vreg<kVc>(ey_w), pez = vreg<kVc>(ez_w);
    // all ones for the waves before this one (their counts come first)
    int before[kSWaves];
#pragma unroll
    for (int w2 = 0; w2 < kSWaves; ++w2) before[w2] = vreg<kVt || (MIX && EM)>(w2 < w ? -1 : 0);
    if (threadIdx.x == 0) sErr = 0;
    int first, end, stride;
    bucket_walk(g.nbuckets, first, end, stride);
    for (int b = first; b < end; b += stride) {
        int bx, by, bz;
        tile_coords<DIM>(g, b, bx, by, bz);
        const int x0s = bx << g.tsx, y0s = (DIM >= 2) ? (by << g.tsy) : 0, z0s = (DIM == 3) ? (bz << g.tsz) : 0;
        TileNb tn = tile_nb<DIM>(g, bx, by, bz);
        const int x0 = vreg<kVt>(x0s), y0 = vreg<kVt>(y0s), z0 = vreg<kVt>(z0s);
        tn.txe = vreg<kVt>(tn.txe);
        tn.lw = vreg<kVt>(tn.lw);
        tn.rw = vreg<kVt>(tn.rw);
        if constexpr (DIM >= 2) {
            tn.tye = vreg<kVt>(tn.tye);
            tn.dw = vreg<kVt>(tn.dw);
            tn.uw = vreg<kVt>(tn.uw);
        }
        if constexpr (DIM == 3) {
            tn.tze = vreg<kVt>(tn.tze);
            tn.bw = vreg<kVt>(tn.bw);
            tn.fw = vreg<kVt>(tn.fw);
        }
        PushC pv = pc;
        pv.af = vreg<kVc>(pc.af);
        pv.tf = vreg<kVc>(pc.tf);
        pv.sf = vreg<kVc>(pc.sf);
        pv.dtdx = vreg<kVc>(pc.dtdx);
        pv.dtdy = vreg<kVc>(pc.dtdy);
        pv.dtdz = vreg<kVc>(pc.dtdz);
        pv.dtdx2 = vreg<kVc>(pc.dtdx2);
        pv.dtdy2 = vreg<kVc>(pc.dtdy2);
        pv.deep = vreg<kVc>(pc.deep);
        Geo gv = g;
        gv.nx = vreg<kVc>(g.nx);
        gv.ny = vreg<kVc>(g.ny);
        gv.nz = vreg<kVc>(g.nz);
        gv.nxp = vreg<kVc>(g.nxp);
        // the bucket's range and (mixed path) its first chunk of particles,
        // loaded before the tables and the field tile so that the memory round
        // trips overlap; the FP64 pipeline issues its first chunk below
        const int i0 = min(max(bstart[b], 0), g.np), i1 = min(max(bstart[b + 1], i0), g.np);
        const int span = i1 - i0;
        // whole 128-byte lines per wave, as in the tally pass (index k at
        // chunk position k + sh)
        const int sh = i0 & (MIX ? 31 : 15);
        const int send = span > 0 ? span + sh : 0;
        Raw<MIX> ra[U], rb[U];
        auto fetch = [&](Raw<MIX> *r, int base) {
#pragma unroll
            for (int j = 0; j < U; ++j)
                load_raw<MIX, DIM, VDIM>(src, i0 + min(max(base + j * kSBlock + (int)threadIdx.x - sh, 0), span - 1),
                                         r[j]);
            // keep these loads where they are: issued one chunk ahead of their use
            __builtin_amdgcn_sched_barrier(0);
        };
        if (MIX && span > 0) fetch(ra, 0);
        {
            const int na = EM ? 3 * jw * jh : wxy * wz;
            for (int t2 = threadIdx.x; t2 < na; t2 += blockDim.x) sA[t2] = (A)0;
        }
        // first slot of each direction of this bucket inside its destination
        // bucket (from the offsets pass), and each destination's end
        if (threadIdx.x < kTab) {
            const int d = threadIdx.x;
            int off = 0, ct = 0;
            if (d < kFar) {
                off = offs[b * kTab + d];
                ct = cnt[b * kTab + d];
                sEnd[d] = bstart_new[dir_target<DIM>(g, bx, by, bz, d) + 1];
                if (d == kStay) {
                    sStay[0] = off;
                    sStay[1] = off + ct;
                }
            }
#pragma unroll
            for (int w2 = 0; w2 < kSWaves; ++w2) sCur[w2][d] = off;
            sRunEnd[d] = off + ct;
        }
        if constexpr (EM)
            load_f_tile<R>(sE, E, g, x0, y0, fw, fh);
        else if (MIX && E32)
            load_tile_any<R, float, DIM>(sE, E32, g, x0, y0, z0, ex_w, ey_w, ez_w);
        else
            load_tile_any<R, double, DIM>(sE, E, g, x0, y0, z0, ex_w, ey_w, ez_w);
        __syncthreads();
        // the bucket's stay cursors (front: next deep slot, back: one past the
        // next shallow slot), the same in every wave, and the end of the bucket
        const int front0 = __builtin_amdgcn_readfirstlane(sStay[0]);
        int front = front0;
        int back = __builtin_amdgcn_readfirstlane(sStay[1]);
        const int stayEnd = __builtin_amdgcn_readfirstlane(sEnd[kStay]);
        // cells of this tile (the last tile of an axis may be cut by the grid edge)
        const float txe = (float)tn.txe;
        const float tye = (float)tn.tye;
        const float tze = (float)tn.tze;
        double ke = 0.0, px = 0.0;
        constexpr int CH = kSBlock * U;
        // Two schedules over chunks of CH particles.
        // FP64 (twice the bytes per particle, latency-exposed): a software
        // pipeline whose loads of chunk c+1 and stores of chunk c-1 are both
        // issued right after the wait for chunk c's data, so each has one
        // compute period to complete (one vector-memory counter covers loads
        // and stores, so a wait for a load also waits for every store issued
        // before it). Mixed (measured faster): two register sets, the next
        // chunk's loads issued before the current chunk is processed and its
        // stores made inside the processing.
        constexpr bool kPipe = !MIX;
        Pt<MIX> pq[U];      // results of the previous chunk, stored at the next wait
        int pslot[U], psrc[U];
        bool pact[U];
#pragma unroll
        for (int j = 0; j < U; ++j) pact[j] = false;
        auto commit = [&]() {
#pragma unroll
            for (int j = 0; j < U; ++j) {
                if (pact[j]) {
                    if (pslot[j] >= 0) {
                        store_pt<MIX, DIM, VDIM>(dst, pslot[j], pq[j]);
                        if (perm) perm[pslot[j]] = psrc[j];
                    } else {
                        atomicOr(&sErr, ERR_ORDER);
                    }
                }
            }
        };
        auto process = [&](const Raw<MIX> *r, int base) {
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int k = base + j * kSBlock + (int)threadIdx.x - sh;
                const bool act = k >= 0 && k < span;
                int code = -1, nbk = 0;
                bool deep = false;
                Pt<MIX> q;
                if (act) {
                    bool good = decode<MIX, DIM, VDIM>(r[j], gv, q);
                    const double v2o = vsq<MIX, VDIM, HC>(q, pv);
                    int lx, ly, lz = 0, sx, sy, sz = 0;
                    R f0x = R(0), f0y = R(0), ig = R(1);
                    if constexpr (EM) {
                        good = advance_em<MIX, HC>(q, gv, pv, sE, fw, x0, y0, lx, ly, sx, sy, f0x, f0y, ig) && good;
                    } else {
                        good = advance<MIX, DIM, VDIM, HC>(q, gv, pv, sE, pex, pey, pez, x0, y0, z0, lx, ly, lz, sx,
                                                           sy, sz) && good;
                    }
                    if (!good) atomicOr(&sErr, ERR_DOMAIN);
                    const double v2n = vsq<MIX, VDIM, HC>(q, pv);
                    ke += v2o + v2n;   // halved once per bucket (exact: a power of two)
                    px += (double)q.vx;
                    code = dir_local<DIM>(tn, lx + sx, ly + sy, lz + sz);
                    // absorbed by a wall: no deposit, no slot
                    const bool dead = g.walls && q.ix >= gv.nxp;
                    if (dead) code = -1;
                    if (code == kFar) nbk = bucket_of<MIX, DIM>(gv, q.ix, q.iy, q.iz);
                    if (code == kStay) {
                        const float ux = (float)(q.ix - x0) + (float)q.fx;
                        const float mx = fminf(ux, txe - ux) - pv.deep;
                        const float vx = fabsf((float)q.vx);
                        if constexpr (DIM == 1) {
                            deep = mx >= vx * pv.dtdx;
                        } else {
                            const float uy = (float)(q.iy - y0) + (float)q.fy;
                            const float my = fminf(uy, tye - uy) - pv.deep;
                            const float vy = fabsf((float)q.vy);
                            // with a rotation the speed can turn along either axis:
                            // compared as squares, |v| dt/dx <= m <=> |v|^2 (dt/dx)^2
                            // <= m^2 for m >= 0 (the rounding of either side,
                            // a few ulps, is far inside the margin pv.deep keeps)
                            if constexpr (EM) {
                                // a general B can turn the whole speed along either axis
                                const float vz = (float)q.vz;
                                const float vv2 = vx * vx + vy * vy + vz * vz;
                                deep = mx >= 0.0f && my >= 0.0f && mx * mx >= vv2 * pv.dtdx2 &&
                                       my * my >= vv2 * pv.dtdy2;
                            } else if (!pv.rot) {
                                deep = mx >= vx * pv.dtdx && my >= vy * pv.dtdy;
                            } else {
                                // the rotation about z turns the in-plane speed
                                const float vv2 = vx * vx + vy * vy;
                                deep = mx >= 0.0f && my >= 0.0f && mx * mx >= vv2 * pv.dtdx2 &&
                                       my * my >= vv2 * pv.dtdy2;
                            }
                            if constexpr (DIM == 3) {
                                // vz only takes the kicks of Ez (the rotation is about z)
                                const float uz = (float)(q.iz - z0) + (float)q.fz;
                                const float mz = fminf(uz, tze - uz) - pv.deep;
                                deep = deep && mz >= fabsf((float)q.vz) * pv.dtdz;
                            }
                        }
                    }
                    if (dead) {
                    } else if constexpr (EM) {
                        // current J^{n+1/2} of the move x^n -> x^{n+1} (Esirkepov); the
                        // mixed path's displacement is the binary32 product its move adds
                        // (with Higuera-Cary the velocity is u / gamma, the product the move used)
                        const R wvx = q.vx * ig, wvy = q.vy * ig, wvz = q.vz * ig;
                        R ddx, ddy;
                        if constexpr (MIX) {
                            ddx = wvx * pv.dtdx;
                            ddy = wvy * pv.dtdy;
                        } else {
                            ddx = (wvx * pc.dt) * g.inv_dx;
                            ddy = (wvy * pc.dt) * g.inv_dy;
                        }
                        if (!esirkepov_lds<R>((double *)sA, jw, jw * jh, lx, ly, f0x, f0y, ddx, ddy,
                                              (R)(pc.jz * (double)wvz)))
                            atomicOr(&sErr, ERR_DOMAIN);
                    } else {
                    // deposit rho^{n+1}: LDS tile + halo, global beyond it
                    A wgt[8];
                    dep_weights<MIX, DIM>(q, gv, wgt);
                    const int dlx = lx + sx + g.halo;
                    const int dly = (DIM >= 2) ? ly + sy + g.halo : 0;
                    const int dlz = (DIM == 3) ? lz + sz + g.halo : 0;
                    bool inl = (unsigned)dlx <= (unsigned)(pwx - 2);
                    if constexpr (DIM >= 2) inl = inl && (unsigned)dly <= (unsigned)(pwy - 2);
                    if constexpr (DIM == 3) inl = inl && (unsigned)dlz <= (unsigned)(wz - 2);
                    if (inl) {
                        const int a0 = (dlz * pwy + dly) * pwx + dlx;
                        acc_add_lds<MIX>(&sA[a0], wgt[0]);
                        acc_add_lds<MIX>(&sA[a0 + 1], wgt[1]);
                        if constexpr (DIM >= 2) {
                            acc_add_lds<MIX>(&sA[a0 + pwx], wgt[2]);
                            acc_add_lds<MIX>(&sA[a0 + pwx + 1], wgt[3]);
                        }
                        if constexpr (DIM == 3) {
                            acc_add_lds<MIX>(&sA[a0 + pwxy], wgt[4]);
                            acc_add_lds<MIX>(&sA[a0 + pwxy + 1], wgt[5]);
                            acc_add_lds<MIX>(&sA[a0 + pwxy + pwx], wgt[6]);
                            acc_add_lds<MIX>(&sA[a0 + pwxy + pwx + 1], wgt[7]);
                        }
                    } else if constexpr (DIM == 3) {
                        deposit_global3<MIX>(acc, g, q.ix, q.iy, q.iz, wgt);
                    } else {
                        deposit_global<MIX, DIM>(acc, g, q.ix, q.iy, wgt);
                    }
                    }
                }
                // slot: in chunk order, then wave order, then lane order, per
                // direction; each group's range is checked against its bucket's
                // end (the start is its offset-table entry, from the same scan)
                int slot = -1;
                // this wave's counts: deep and shallow stays, and movers to a
                // neighbour bucket (lanes sharing a code found with one ballot
                // per code bit; the group's lowest lane records its size)
                const uint64_t gst = __ballot(code == kStay);
                const uint64_t gd = __ballot(code == kStay && deep);
                const uint64_t gs = gst & ~gd;
                const int nd = (int)__popcll(gd), ns = (int)__popcll(gs);
                const bool mv = code >= 0 && code < kFar && code != kStay;
                const uint64_t gmv = __ballot(mv);
                const int par = it & 1;
                ++it;
                uint64_t peers = 0;
                if (gmv) {
                    peers = gmv;
#pragma unroll
                    for (int bit = 0; bit < kCodeBits; ++bit) {
                        const uint64_t bb = __ballot(mv && ((code >> bit) & 1));
                        peers &= ((code >> bit) & 1) ? bb : ~bb;
                    }
                    if (lane < kTab) sMv[par][w][lane] = 0;
                    if (mv && (peers & lt) == 0) sMv[par][w][code] = (int)__popcll(peers);
                }
                // packed: deep count in bits 0-9, shallow count in bits 10-19, the
                // mover flag from bit 20 (sums over the waves stay below 1024)
                static_assert(kSBlock < 1024, "a chunk's counts fill ten bits");
                if (lane == 0) sPk[par][w] = nd | (ns << 10) | ((gmv != 0) << 20);
                __syncthreads();
                // the counts of the waves before this one, and of the whole chunk,
                // summed as packed words
                int pk[kSWaves], pre = 0, tot = 0;
#pragma unroll
                for (int w2 = 0; w2 < kSWaves; ++w2) {
                    pk[w2] = sPk[par][w2];
                    tot += pk[w2];
                    pre += pk[w2] & before[w2];
                }
                const int pd = pre & 1023, ps = (pre >> 10) & 1023;
                const int td = tot & 1023, ts = (tot >> 10) & 1023;
                const int anymv = tot >> 20;
                // stays: deep ones from the front of the bucket's stay range,
                // the rest from its back
                const bool sfits = front >= 0 && front + td <= back - ts && back <= stayEnd;
                if (code == kStay)
                    slot = !sfits ? -1
                                  : deep ? front + pd + (int)__popcll(gd & lt)
                                         : back - 1 - ps - (int)__popcll(gs & lt);
                front += td;
                back -= ts;
                if (anymv) {
                    // lane d of every wave: this wave's first slot in direction d,
                    // and the wave's copy of the cursor moved past the chunk
                    int offd = 0;
                    if (lane < kTab) {
                        int mpre = 0, mtot = 0;
#pragma unroll
                        for (int w2 = 0; w2 < kSWaves; ++w2) {
                            const int c2 = (pk[w2] >> 20) ? sMv[par][w2][lane] : 0;
                            mpre += c2 & before[w2];
                            mtot += c2;
                        }
                        offd = sCur[w][lane] + mpre;
                        sCur[w][lane] += mtot;
                    }
                    const int basek = __shfl(offd, mv ? code : 0);
                    if (mv) {
                        const int r = (int)__popcll(peers & lt), cntk = (int)__popcll(peers);
                        // inside this direction's own range (and so inside its bucket)
                        const bool fits =
                            basek >= 0 && basek + cntk <= sRunEnd[code] && sRunEnd[code] <= sEnd[code];
                        slot = fits ? basek + r : -1;
                    }
                }
                if (code == kFar) {
                    // far arrivals fill the end of their bucket; the counter
                    // returns to zero for the next step
                    const int v = atomicSub(&farcnt[nbk], 1);
                    slot = (v > 0) ? bstart_new[nbk + 1] - v : -1;
                }
                if constexpr (kPipe) {
                    pq[j] = q;
                    pslot[j] = slot;
                    psrc[j] = i0 + k;
                    pact[j] = act && code >= 0;
                } else if (act && code >= 0) {
                    if (slot >= 0) {
                        store_pt<MIX, DIM, VDIM>(dst, slot, q);
                        if (perm) perm[slot] = i0 + k;
                    } else {
                        atomicOr(&sErr, ERR_ORDER);
                    }
                }
            }
        };
        if constexpr (kPipe) {
            if (span > 0) fetch(ra, 0);
            for (int base = 0; base < send; base += CH) {
                __builtin_amdgcn_s_waitcnt(kWaitVmem);
                __builtin_amdgcn_sched_barrier(0);
                Raw<MIX> rc[U];
#pragma unroll
                for (int j = 0; j < U; ++j) rc[j] = ra[j];
                commit();
                fetch(ra, base + CH);  // index clamped to the span: harmless re-reads after the last chunk
                process(rc, base);
            }
            commit();
        } else {
            // the fetches are unconditional (indices clamped to the span: at
            // most a chunk of harmless re-reads past the end), so that every
            // path issues the same loads and a wait for one chunk's data
            // never waits for the chunk fetched after it
            for (int base = 0; base < send; base += 2 * CH) {
                fetch(rb, base + CH);
                process(ra, base);
                fetch(ra, base + 2 * CH);
                if (base + CH < send) process(rb, base + CH);
            }
        }
        __syncthreads();
        // every range filled exactly: a count that differs from the push's (a
        // particle the count pass credited as staying that moved, or the
        // reverse) leaves a slot empty or overflows a range
        if (threadIdx.x < kFar) {
            const int d = threadIdx.x;
            const bool full = d == kStay ? front == back : sCur[0][d] == sRunEnd[d];
            if (!full) atomicOr(&sErr, ERR_ORDER);
        }
        if (threadIdx.x == 0) {
            // the deep range of the stays, relative to this bucket's new start
            deep_out[b * kDeepTab] = front0 - bstart_new[b];
            deep_out[b * kDeepTab + 1] = front - front0;
        }
        if constexpr (EM)
            flush_j((double *)acc, (const double *)sA, g, x0, y0, jw, jh, pc.jx, pc.jy);
        else if constexpr (DIM == 3)
            flush_region3<MIX>(acc, sA, g, x0, y0, z0, wx, wy, wz, g.halo);
        else
            flush_region<MIX, DIM>(acc, sA, g, x0, y0, wx, wy, g.halo);
        if (part) {
            double kt = 0.5 * block_sum(ke, sRed);
            double pt = block_sum(px, sRed);
            if (threadIdx.x == 0) {
                part[2 * b] = kt;
                part[2 * b + 1] = pt;
            }
        }
        __syncthreads();
    }
    __syncthreads();
    if (threadIdx.x == 0 && sErr) raise_err(c.err, sErr);
}

// ---- field: accumulation -> rho --------------------------------------------------
// rho_j = add + scale * acc_j (acc: double weights or int64 fixed-point sums);
// acc is cleared when clear != 0. Fixed-point sums with qacc set: their exact
// total (sd = S * dim weight bits per particle) is added to qacc.
template <bool MIX>
__global__ void __launch_bounds__(kBlock) k_rho(int64_t G, typename AccOf<MIX>::T *acc, double *rho,
                                                double scale, double add, int clear, int sd,
                                                unsigned long long *qacc) {
    QSum q{0, 0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < G; i += (int64_t)gridDim.x * blockDim.x) {
        typename AccOf<MIX>::T v = acc[i];
        double w;
        if constexpr (MIX) {
            w = (double)(int64_t)v;
            if (qacc) qsum_add(q, (int64_t)v, sd);
        } else {
            w = v;
        }
        rho[i] = add + scale * w;
        if (clear) acc[i] = (typename AccOf<MIX>::T)0;
    }
    if constexpr (MIX) {
        if (qacc) qsum_flush(q, sd, qacc);
    }
}

// Walls: rho of the odd extension along x (rows of nx = 2 nxp nodes): the
// physical interior node i in (0, nxp) holds add + scale acc_i and its mirror
// nx - i the negated value; the wall nodes 0 and nxp hold zero (phi is zero
// there, so their charge does not enter the solve). One thread per
// (physical node, row) writes both halves, so acc can be cleared in place.
// Fixed-point sums with qacc set: the exact total of the physical nodes
// (walls included) is added to qacc.
template <bool MIX>
__global__ void __launch_bounds__(kBlock) k_rho_odd(Geo g, typename AccOf<MIX>::T *acc, double *rho, double scale,
                                                    double add, int clear, unsigned long long *qacc) {
    const int half = g.nxp + 1;
    const int64_t tot = (int64_t)half * g.ny;
    const int sd = g.S * g.dim;
    QSum q{0, 0};
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int ix = (int)(t % half);
        const int64_t row = (t / half) * g.nx;
        typename AccOf<MIX>::T v = acc[row + ix];
        double w;
        if constexpr (MIX) {
            w = (double)(int64_t)v;
            if (qacc) qsum_add(q, (int64_t)v, sd);
        } else {
            w = v;
        }
        const bool wall = ix == 0 || ix == g.nxp;
        const double r = wall ? 0.0 : add + scale * w;
        rho[row + ix] = r;
        if (!wall) rho[row + g.nx - ix] = -r;
        if (clear) {
            acc[row + ix] = (typename AccOf<MIX>::T)0;
            if (!wall) acc[row + g.nx - ix] = (typename AccOf<MIX>::T)0;
        }
    }
    if constexpr (MIX) {
        if (qacc) qsum_flush(q, sd, qacc);
    }
}

__global__ void __launch_bounds__(1024) k_finalize(FinArgs f, CtxDev c) { finalize_block(f, c); }

// phi_hat = rho_hat / K^2 (K^2 = sum of the per-axis modified wavenumbers,
// phi_hat(0) = 0), scaled by 1/G for the unnormalised inverse transform, and
// the per-block partials of sum |E_hat|^2 = sum kappa^2 |phi_hat|^2 over the
// full spectrum (Parseval; the half spectrum counts every kx other than 0
// and nx/2 twice).
__global__ void __launch_bounds__(kBlock) k_spectral(Geo g, const double2 *rh, double2 *ph, CtxDev c) {
    __shared__ double sRed[kWaves];
    const int hx = g.nx / 2 + 1;
    const int64_t rows = (int64_t)g.ny * g.nz;
    const double norm = 1.0 / ((double)g.nx * (double)g.ny * (double)g.nz);
    double part = 0.0;
    // one (ky, kz) row of the half spectrum per wave at a time
    const int lane = (int)(threadIdx.x & 63);
    const int wv = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const int64_t nwv = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t r = wv; r < rows; r += nwv) {
        const int ky = (int)(r % g.ny), kz = (int)(r / g.ny);
        const double ky2 = c.ky2[ky], kz2 = c.kz2[kz], kay = c.kapy[ky], kaz = c.kapz[kz];
        for (int kx = lane; kx < hx; kx += 64) {
            const int64_t i = r * hx + kx;
            const double K2 = (c.kx2[kx] + ky2) + kz2;
            const double2 rr = rh[i];
            if (i == 0) *c.rho0 = rr.x;
            const double inv = (i == 0) ? 0.0 : 1.0 / K2;
            const double pr = rr.x * inv, pi = rr.y * inv;
            const double kax = c.kapx[kx];
            const double wgt = (kx == 0 || 2 * kx == g.nx) ? 1.0 : 2.0;
            part += wgt * (kax * kax + kay * kay + kaz * kaz) * (pr * pr + pi * pi);
            ph[i] = make_double2(pr * norm, pi * norm);
        }
    }
    double bs = block_sum(part, sRed);
    if (threadIdx.x == 0) c.part_spec[blockIdx.x] = bs;
}

// E = -(centred difference of phi), periodic: E_d[j] = (phi[j - e_d] -
// phi[j + e_d]) / (2 d_d), the real-space form of E_hat = -i sin(k d)/d
// phi_hat. Writes E [dim][G] when E is not NULL and, when E32 is not NULL,
// its binary32 rounding. h = 1 / (2 d) per axis.
// The last workgroup of the launch reduces the field diagnostics instead
// (it reads only what earlier launches wrote).
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_grad(Geo g, const double *__restrict__ phi, double *__restrict__ E,
                                                 float *__restrict__ E32, double hx, double hy, double hz, FinArgs f,
                                                 CtxDev c) {
    if (blockIdx.x == gridDim.x - 1) {
        finalize_block(f, c);
        return;
    }
    const int64_t G = (int64_t)g.nx * g.ny * g.nz;
    const int64_t sxy = (int64_t)g.nx * g.ny;
    const int64_t rows = (int64_t)g.ny * g.nz;
    // one (y, z) row per wave at a time: the neighbour rows' offsets once per row
    const int lane = (int)(threadIdx.x & 63);
    const int wv = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const int64_t nwv = (int64_t)(gridDim.x - 1) * (blockDim.x >> 6);
    constexpr int U = 2;   // nodes per lane and round: their loads all issued before the first wait
    constexpr int NV = 2 * DIM;
    for (int64_t r = wv; r < rows; r += nwv) {
        const int iy = (int)(r % g.ny), iz = (int)(r / g.ny);
        const int64_t row = r * g.nx;
        const int64_t ym = (iy == 0) ? row + sxy - g.nx : row - g.nx;
        const int64_t yp = (iy == g.ny - 1) ? row - (sxy - g.nx) : row + g.nx;
        const int64_t zm = (iz == 0) ? row + G - sxy : row - sxy;
        const int64_t zp = (iz == g.nz - 1) ? row - (G - sxy) : row + sxy;
        for (int ix0 = 0; ix0 < g.nx; ix0 += U * 64) {
            // nodes past the row repeat its last node: the same values to the same addresses
            double v[U][NV];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int ix = min(ix0 + u * 64 + lane, g.nx - 1);
                const int xm = (ix == 0) ? g.nx - 1 : ix - 1, xp = (ix == g.nx - 1) ? 0 : ix + 1;
                v[u][0] = phi[row + xm];
                v[u][1] = phi[row + xp];
                v[u][2] = phi[ym + ix];
                v[u][3] = phi[yp + ix];
                if constexpr (DIM == 3) {
                    v[u][4] = phi[zm + ix];
                    v[u][5] = phi[zp + ix];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = row + min(ix0 + u * 64 + lane, g.nx - 1);
                const double ex = (v[u][0] - v[u][1]) * hx, ey = (v[u][2] - v[u][3]) * hy;
                if (E) {
                    E[i] = ex;
                    E[G + i] = ey;
                }
                if (E32) {
                    E32[i] = (float)ex;
                    E32[G + i] = (float)ey;
                }
                if constexpr (DIM == 3) {
                    const double ez = (v[u][4] - v[u][5]) * hz;
                    if (E) E[2 * G + i] = ez;
                    if (E32) E32[2 * G + i] = (float)ez;
                }
            }
        }
    }
}

// Sums the per-block partials in a fixed order (deterministic) and writes the
// step diagnostics, or the field energy / charge of a standalone solve.
//   kinetic  = 0.5 * mass * sum(part_push[2b]),   momentum = mass * sum(part_push[2b+1])
//   W_E      = 0.5 * dV / G * sum(part_spec)      (Parseval)
//   charge   = dV * (rho0 - G * rho_ion)

// 1D field (one workgroup of kBlock threads; nodes held in LDS).
// Fixed-point sums (MIX): the charge is their exact integer total (sd = S
// weight bits per particle) times q_macro, also stored in c.qexact.
template <bool MIX>
__global__ void __launch_bounds__(kBlock) k_field1d(int nx, typename AccOf<MIX>::T *acc, double scale,
                                                    double add, double ion, double dx, int clear, double *E,
                                                    float *E32, double *we, double *charge, int step_mode,
                                                    int sd, double q_macro, CtxDev c) {
    extern __shared__ __align__(16) unsigned char smem[];
    double *sr = (double *)smem;          // [nx] rho, then half-node field
    __shared__ double sRed[kWaves];
    __shared__ double sScan[kBlock];
    double part = 0.0;
    QSum q{0, 0};
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        typename AccOf<MIX>::T v = acc[i];
        double w;
        if constexpr (MIX) {
            w = (double)(int64_t)v;
            qsum_add(q, (int64_t)v, sd);
        } else {
            w = v;
        }
        double r = add + scale * w;
        sr[i] = r;
        part += r - ion;
        if (clear) acc[i] = (typename AccOf<MIX>::T)0;
    }
    double qtot = block_sum(part, sRed) * dx;
    if constexpr (MIX) {
        const QSum t = qsum_block(q, sd);
        if (threadIdx.x == 0) {
            c.qexact[0] = t.whole;
            c.qexact[1] = (int64_t)t.rem;
            qtot = qsum_charge(t, sd, q_macro);
        }
    }
    const double wsum = field1d_block(sr, nx, dx, E, E32, sRed, sScan);
    if (threadIdx.x == 0) {
        if (we) *(step_mode ? step_slot(we, c) : we) = 0.5 * wsum * dx;
        if (charge) *(step_mode ? step_slot(charge, c) : charge) = qtot;
    }
}

inline int blocks_for(int64_t n, int cap = 4096) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    return (int)(b > cap ? cap : b);
}

inline size_t tile_e_bytes(const Geo &g, bool mixed) {
    const int ex_w = (1 << g.tsx) + 1, ey_w = (g.dim >= 2) ? (1 << g.tsy) + 1 : 1;
    const int ez_w = (g.dim == 3) ? (1 << g.tsz) + 1 : 1;
    return (size_t)ex_w * ey_w * ez_w * g.dim * (mixed ? 4 : 8);
}

// electromagnetic step: six-component field tile ((T+2)^2 each) and the
// three-component current tile ((T+3)^2 each), rounded to 16 bytes
inline size_t em_f_tile_bytes(const Geo &g, bool mixed) {
    return ((size_t)6 * ((1 << g.tsx) + 2) * ((1 << g.tsy) + 2) * (mixed ? 4 : 8) + 15) & ~(size_t)15;
}
inline size_t em_j_tile_bytes(const Geo &g) {
    return ((size_t)3 * ((1 << g.tsx) + 3) * ((1 << g.tsy) + 3) * sizeof(double) + 15) & ~(size_t)15;
}

inline size_t tile_acc_bytes(const Geo &g, int halo) {
    const int wx = (1 << g.tsx) + 1 + 2 * halo;
    const int wy = (g.dim >= 2) ? (1 << g.tsy) + 1 + 2 * halo : 1;
    const int wz = (g.dim == 3) ? (1 << g.tsz) + 1 + 2 * halo : 1;
    return (((size_t)wx * wy * wz * 8) + 15) & ~(size_t)15;
}

}  // namespace

// ================================================================ launchers


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


hipError_t launch_keys_init(const Geo &g, bool mixed, const Parts &p, int64_t n, int32_t *keys, int32_t *idx,
                            const CtxDev &c, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    APIC_DISPATCH(g, mixed,
                  hipLaunchKernelGGL((k_keys_init<MIX, DIM, VDIM>), dim3(blocks_for(n)), dim3(kBlock), 0, s, g, p, n,
                                     keys, idx, c));
    return hipGetLastError();
}

int sort_chunks(int64_t n) { return (int)((n + kSortChunk - 1) / kSortChunk); }
int sort_table_entries() { return kSortTab; }
int sort_part_entries() { return kRadixParts * kRadix; }

hipError_t launch_bucket_table(const int32_t *sorted_keys, int64_t n, int nb, int32_t *start, int64_t max_per_bucket,
                               const CtxDev &c, hipStream_t s) {
    hipLaunchKernelGGL(k_bucket_bounds, dim3(blocks_for(n + 1)), dim3(kBlock), 0, s, sorted_keys, n, nb, start);
    hipLaunchKernelGGL(k_bucket_check, dim3(blocks_for(nb)), dim3(kBlock), 0, s, start, nb, max_per_bucket, c);
    return hipGetLastError();
}

hipError_t launch_radix_pass(const int32_t *kin, const int32_t *iin, int32_t *kout, int32_t *iout, int64_t n,
                             int shift, int32_t *cnt, int32_t *off, int32_t *part, const CtxDev &c, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int C = sort_chunks(n);
    hipLaunchKernelGGL(k_radix_count, dim3(C), dim3(kBlock), 0, s, kin, n, shift, cnt);
    const int R = (C + kRadixParts - 1) / kRadixParts, P = (C + R - 1) / R;
    hipLaunchKernelGGL(k_radix_part, dim3(P), dim3(kBlock), 0, s, cnt, C, R, part);
    hipLaunchKernelGGL(k_radix_base, dim3(1), dim3(kBlock), 0, s, part, P);
    hipLaunchKernelGGL(k_radix_off, dim3(P), dim3(kBlock), 0, s, cnt, part, C, R, off);
    hipLaunchKernelGGL(k_radix_scatter, dim3(C), dim3(kBlock), 0, s, kin, iin, kout, iout, n, shift, off, c);
    return hipGetLastError();
}

hipError_t launch_gather_parts(const Geo &g, bool mixed, const Parts &src, const Parts &dst, int64_t n,
                               const int32_t *idx, int32_t *perm, const CtxDev &c, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    APIC_DISPATCH(g, mixed,
                  hipLaunchKernelGGL((k_gather_parts<MIX, DIM, VDIM>), dim3(blocks_for(n)), dim3(kBlock), 0, s, src,
                                     dst, n, idx, perm, c));
    return hipGetLastError();
}

hipError_t launch_deposit(const Geo &g, bool mixed, const Parts &p, int64_t n, const int32_t *bstart, void *acc,
                          const CtxDev &c, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (bstart) {
        size_t sh = tile_acc_bytes(g, 0);
        APIC_DISPATCH(g, mixed,
                      hipLaunchKernelGGL((k_deposit_tiled<MIX, DIM, VDIM>), dim3(grid_for_buckets(g.nbuckets)),
                                         dim3(kBlock), sh, s, g, p, bstart, (typename AccOf<MIX>::T *)acc, c));
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
                      hipLaunchKernelGGL((k_gather_push_tiled<MIX, DIM, VDIM, HC>), dim3(grid_for_buckets(g.nbuckets)),
                                         dim3(kBlock), sh, s, g, p, bstart, (const typename Pt<MIX>::R *)E, pc, c));
    } else {
        APIC_DISPATCH(g, mixed,
                      hipLaunchKernelGGL((k_gather_push_direct<MIX, DIM, VDIM, HC>), dim3(blocks_for(n)), dim3(kBlock), 0,
                                         s, g, p, n, (const typename Pt<MIX>::R *)E, pc, c));
    }
    return hipGetLastError();
}

int cu_count() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

// Workgroups of a bucket kernel resident on one CU during a launch over
// nbuckets buckets: what its registers and LDS allow, at most the buckets'
// share of a CU.
template <typename K>
int resident_per_cu(K kernel, size_t shmem, int nbuckets, int block) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, shmem) != hipSuccess || per_cu <= 0)
        per_cu = 1;
    const int cus = cu_count();
    const int share = (nbuckets + cus - 1) / cus;
    return per_cu < share ? per_cu : share;
}

// Persistent grid: as many blocks as fit on the device at once (a multiple of
// 8 for the XCD walk), never more than the bucket count needs.
template <typename K>
int persistent_grid(K kernel, size_t shmem, int nbuckets, int block = kBlock) {
    const int cus = cu_count();
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, shmem) != hipSuccess || per_cu <= 0)
        per_cu = 4;
    int g = cus * per_cu;
    const int need = grid_for_buckets(nbuckets);
    if (g > need) g = need;
    return ((g + 7) >> 3) << 3;
}

hipError_t launch_step_count(const Geo &g, bool mixed, const Parts &p, const int32_t *bstart, const double *E,
                             const float *E32, const PushC &pc, int32_t *cnt, int32_t *tot, int32_t *farcnt,
                             const int32_t *deep, const CtxDev &c, hipStream_t s) {
    if (g.em) {
        const size_t sh = em_f_tile_bytes(g, mixed);
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(persistent_grid(kern, sh, g.nbuckets, kSBlock)), dim3(kSBlock), sh, s, g, p, bstart,
                               E, nullptr, pc, cnt, tot, farcnt, deep, c);
        };
        if (mixed && g.hc) go(k_step_count<true, 2, 3, APIC_STEP_U, true, true>);
        else if (mixed) go(k_step_count<true, 2, 3, APIC_STEP_U, false, true>);
        else if (g.hc) go(k_step_count<false, 2, 3, APIC_STEP_U, true, true>);
        else go(k_step_count<false, 2, 3, APIC_STEP_U, false, true>);
        return hipGetLastError();
    }
    size_t sh = tile_e_bytes(g, mixed);
    APIC_DISPATCH(g, mixed, {
        auto kern = k_step_count<MIX, DIM, VDIM, U, HC, false>;
        hipLaunchKernelGGL(kern, dim3(persistent_grid(kern, sh, g.nbuckets, kSBlock)), dim3(kSBlock), sh, s, g, p, bstart, E,
                           MIX ? E32 : nullptr, pc, cnt, tot, farcnt, deep, c);
    });
    return hipGetLastError();
}

hipError_t launch_scan_dir(const Geo &g, int32_t *tot, int32_t *start, int64_t n, int64_t max_per_bucket,
                           int step_mode, const CtxDev &c, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_tot, dim3(1), dim3(1024), 0, s, tot, start, g.nbuckets, n, max_per_bucket, step_mode,
                       g.walls, c);
    return hipGetLastError();
}

bool fused_scan_offsets(const Geo &g) { return g.nbuckets <= kFusedScanMax; }

hipError_t launch_scan_offsets(const Geo &g, const int32_t *tot, int32_t *tot_next, int32_t *start, int64_t n,
                               int64_t max_per_bucket, int step_mode, const int32_t *cnt, int32_t *offs,
                               const CtxDev &c, hipStream_t s) {
    const dim3 grid((g.nbuckets + kSWaves - 1) / kSWaves);
    const int walls = g.walls ? 1 : 0;
    if (g.dim == 3)
        hipLaunchKernelGGL(k_scan_offsets<3>, grid, dim3(kSBlock), 0, s, g, tot, tot_next, start, n, max_per_bucket,
                           step_mode, walls, cnt, offs, c);
    else if (g.dim == 2)
        hipLaunchKernelGGL(k_scan_offsets<2>, grid, dim3(kSBlock), 0, s, g, tot, tot_next, start, n, max_per_bucket,
                           step_mode, walls, cnt, offs, c);
    else
        hipLaunchKernelGGL(k_scan_offsets<1>, grid, dim3(kSBlock), 0, s, g, tot, tot_next, start, n, max_per_bucket,
                           step_mode, walls, cnt, offs, c);
    return hipGetLastError();
}

hipError_t launch_dest_offsets(const Geo &g, const int32_t *cnt, const int32_t *start, int32_t *offs,
                               hipStream_t s) {
    const dim3 grid((g.nbuckets + kSWaves - 1) / kSWaves);
    if (g.dim == 3)
        hipLaunchKernelGGL(k_dest_offsets<3>, grid, dim3(kSBlock), 0, s, g, cnt, start, offs);
    else if (g.dim == 2)
        hipLaunchKernelGGL(k_dest_offsets<2>, grid, dim3(kSBlock), 0, s, g, cnt, start, offs);
    else
        hipLaunchKernelGGL(k_dest_offsets<1>, grid, dim3(kSBlock), 0, s, g, cnt, start, offs);
    return hipGetLastError();
}

hipError_t launch_step_push(const Geo &g, bool mixed, const Parts &src, const Parts &dst, const int32_t *bstart,
                            const int32_t *bstart_new, const int32_t *cnt, const int32_t *offs, int32_t *farcnt,
                            const double *E, const float *E32, const PushC &pc, void *acc, int32_t *perm,
                            double *part, int32_t *deep, const CtxDev &c, hipStream_t s) {
    if (g.em) {
        const size_t sh = em_j_tile_bytes(g) + em_f_tile_bytes(g, mixed);
        auto go = [&](auto kern, auto *accp) {
            hipLaunchKernelGGL(kern, dim3(persistent_grid(kern, sh, g.nbuckets, kSBlock)), dim3(kSBlock), sh, s, g, src, dst,
                               bstart, bstart_new, cnt, offs, farcnt, E, nullptr, pc, accp, perm, part, deep, c);
        };
        unsigned long long *am = (unsigned long long *)acc;
        double *ad = (double *)acc;
        if (mixed && g.hc) go(k_step_push<true, 2, 3, APIC_STEP_U, true, true>, am);
        else if (mixed) go(k_step_push<true, 2, 3, APIC_STEP_U, false, true>, am);
        else if (g.hc) go(k_step_push<false, 2, 3, APIC_STEP_U, true, true>, ad);
        else go(k_step_push<false, 2, 3, APIC_STEP_U, false, true>, ad);
        return hipGetLastError();
    }
    size_t sh = tile_acc_bytes(g, g.halo) + tile_e_bytes(g, mixed);
    APIC_DISPATCH(g, mixed, {
        auto kern = k_step_push<MIX, DIM, VDIM, U, HC, false>;
        auto run = [&](auto k) {
            hipLaunchKernelGGL(k, dim3(persistent_grid(k, sh, g.nbuckets, kSBlock)), dim3(kSBlock), sh, s, g, src,
                               dst, bstart, bstart_new, cnt, offs, farcnt, E, MIX ? E32 : nullptr, pc,
                               (typename AccOf<MIX>::T *)acc, perm, part, deep, c);
        };
        if constexpr (MIX && !HC) {
            auto kvr = k_step_push<MIX, DIM, VDIM, U, HC, false, true>;
            if (g.push_vr == 2 ||
                (g.push_vr == 0 &&
                 resident_per_cu(kvr, sh, g.nbuckets, kSBlock) >= resident_per_cu(kern, sh, g.nbuckets, kSBlock)))
                run(kvr);
            else
                run(kern);
        } else {
            run(kern);
        }
    });
    return hipGetLastError();
}

hipError_t launch_rho(const Geo &g, bool mixed, void *acc, double *rho, double scale, double add, int clear,
                      unsigned long long *qacc, hipStream_t s) {
    const int64_t G = (int64_t)g.nx * g.ny * g.nz;
    const int nb = blocks_for(G, 2048);
    if (mixed)
        hipLaunchKernelGGL(k_rho<true>, dim3(nb), dim3(kBlock), 0, s, G, (unsigned long long *)acc, rho, scale, add,
                           clear, g.S * g.dim, qacc);
    else
        hipLaunchKernelGGL(k_rho<false>, dim3(nb), dim3(kBlock), 0, s, G, (double *)acc, rho, scale, add, clear, 0,
                           nullptr);
    return hipGetLastError();
}

hipError_t launch_rho_odd(const Geo &g, bool mixed, void *acc, double *rho, double scale, double add, int clear,
                          unsigned long long *qacc, hipStream_t s) {
    const int nb = blocks_for((int64_t)(g.nxp + 1) * g.ny, 2048);
    if (mixed)
        hipLaunchKernelGGL(k_rho_odd<true>, dim3(nb), dim3(kBlock), 0, s, g, (unsigned long long *)acc, rho, scale,
                           add, clear, qacc);
    else
        hipLaunchKernelGGL(k_rho_odd<false>, dim3(nb), dim3(kBlock), 0, s, g, (double *)acc, rho, scale, add, clear,
                           nullptr);
    return hipGetLastError();
}

int spectral_blocks(const Geo &g) { return blocks_for((int64_t)(g.nx / 2 + 1) * g.ny * g.nz, 1024); }

hipError_t launch_spectral(const Geo &g, const void *rho_hat, void *phi_hat, const CtxDev &c, hipStream_t s) {
    hipLaunchKernelGGL(k_spectral, dim3(spectral_blocks(g)), dim3(kBlock), 0, s, g, (const double2 *)rho_hat,
                       (double2 *)phi_hat, c);
    return hipGetLastError();
}

hipError_t launch_grad(const Geo &g, const double *phi, double *E, float *E32, const FinArgs &f,
                       const CtxDev &c, hipStream_t s) {
    const double hx = 0.5 * g.inv_dx, hy = 0.5 * g.inv_dy, hz = 0.5 * g.inv_dz;
    // a wave per (y, z) row, up to 8192 workgroups, then the diagnostics block
    const int64_t rows = (int64_t)g.ny * g.nz;
    const int nblk = (int)std::min<int64_t>(std::max<int64_t>((rows + kWaves - 1) / kWaves, 1), 8192);
    if (g.dim == 3)
        hipLaunchKernelGGL(k_grad<3>, dim3(nblk + 1), dim3(kBlock), 0, s, g, phi, E, E32, hx, hy, hz, f, c);
    else
        hipLaunchKernelGGL(k_grad<2>, dim3(nblk + 1), dim3(kBlock), 0, s, g, phi, E, E32, hx, hy, hz, f, c);
    return hipGetLastError();
}

hipError_t launch_finalize(int npush, int nspec, double mass, double dV, double G, double rho_ion, double *diag,
                           double *we, double *charge, const CtxDev &c, hipStream_t s) {
    const FinArgs f{npush, nspec, mass, dV, G, rho_ion, diag, we, charge};
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, f, c);
    return hipGetLastError();
}

hipError_t launch_field1d(const Geo &g, bool mixed, void *acc, double scale, double add, double ion, double dx,
                          int clear, double *E, float *E32, double *we_out, double *charge_out, int step_mode,
                          double q_macro, const CtxDev &c, hipStream_t s) {
    size_t sh = (size_t)g.nx * sizeof(double);
    if (mixed)
        hipLaunchKernelGGL(k_field1d<true>, dim3(1), dim3(kBlock), sh, s, g.nx, (unsigned long long *)acc, scale, add,
                           ion, dx, clear, E, E32, we_out, charge_out, step_mode, g.S * g.dim, q_macro, c);
    else
        hipLaunchKernelGGL(k_field1d<false>, dim3(1), dim3(kBlock), sh, s, g.nx, (double *)acc, scale, add, ion, dx,
                           clear, E, E32, we_out, charge_out, step_mode, 0, q_macro, c);
    return hipGetLastError();
}

}  // namespace apic
