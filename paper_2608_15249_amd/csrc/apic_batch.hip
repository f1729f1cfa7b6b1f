// Batched replicas: many independent 1D1V periodic plasmas of uneven grid and
// particle counts advanced by one persistent kernel launch per step.
//
// Each replica is the same PIC cycle as the single-plasma path (mixed
// precision: binary32 push of cell + offset positions, int64 fixed-point CIC
// deposit, FP64 1D Gauss-law field solve) and uses the same device helpers,
// so a replica run here gives the bits it gives when run alone.
//
// Launch structure (one kernel per step): a persistent grid pulls work items
// (replica, chunk of that replica's particles) from a global counter. A block
// stages the replica's whole grid in LDS (nx <= kBatchMaxNx): the field as
// binary32 for the gather and an int64 charge accumulator for the deposit,
// then flushes the accumulator to the replica's global int64 grid with one
// atomic per touched node. The block that finishes a replica's last chunk
// (per-replica arrival counter, release/acquire fences) solves that
// replica's field for the next step and writes its diagnostics. No block
// ever waits for another, so co-residency is not required. The last block
// to leave resets the counters, so the launch can be replayed from a graph.
#include "apic.h"
#include "apic_device.h"

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

namespace apic {
namespace {

constexpr int kBatchMaxNx = 1024;
#ifndef APIC_BATCH_U
#define APIC_BATCH_U 8
#endif
constexpr int kBatchU = APIC_BATCH_U;   // particles per thread per pipeline stage
// LDS deposit word of cell j: the sum W_j of the right-node weights w1 < 2^32
// of its particles in the low 48 bits, their count in the high 16 bits; a work
// item holds at most kBatchMaxChunk particles, so neither field overflows.
constexpr int kCountShift = 48;
constexpr unsigned long long kCountUnit = 1ull << kCountShift;
constexpr unsigned long long kSumMask = kCountUnit - 1;
constexpr int kBatchMaxChunk = (1 << 16) - 1;

struct RepP {
    int nx, nitems, item0, p0;   // grid nodes, work items, first item, first particle
    int64_t g0;                  // first grid node in the packed grid arrays
    int n;                       // particles
    float dtdx;                  // dt / dx in binary32
    double dx, acc_scale, mass;  // acc_scale = q_macro 2^-S / dx
    double q_macro;              // charge of one particle
};

struct Item {
    int r, p0, cnt, pad;         // replica, first particle (packed index), count
};

struct BatchP {
    const RepP *reps;
    const Item *items;
    int n_items, nrep, S;
    int *head, *done, *rep_done, *step, *err;
    double *part;                // per item (kinetic sum, momentum sum)
    float a, t, s;               // Boris coefficients (q/m dt_eff / 2, no magnetic field)
    double rho_ion;
};

enum { MODE_DEPOSIT = 0, MODE_HALF = 1, MODE_STEP = 2 };

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform_f(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ int64_t uniform_l(int64_t v) {
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ double uniform_d(double v) { return __longlong_as_double(uniform_l(__double_as_longlong(v))); }

template <int MODE>
__global__ void __launch_bounds__(kBlock) k_batch(BatchP bp, int32_t *cell, float *ox, float *vx, double *E,
                                                  unsigned long long *acc, double *diag, int64_t *rho_out) {
    __shared__ float sE[kBatchMaxNx + 1];
    __shared__ unsigned long long sA[kBatchMaxNx];   // charge; reused as rho for the field solve
    double *sR = reinterpret_cast<double *>(sA);
    __shared__ double sRed[kWaves];
    __shared__ double sScan[kBlock];
    __shared__ int sItem, sLast, sErr;
    if (threadIdx.x == 0) sErr = 0;
    Parts ps;
    ps.x = ps.y = nullptr;
    ps.cell = cell;
    ps.ox = ox;
    ps.oy = nullptr;
    ps.vx = vx;
    ps.vy = ps.vz = nullptr;
    for (;;) {
        if (threadIdx.x == 0) sItem = atomicAdd(bp.head, 1);
        __syncthreads();
        // uniform across the block: the item and replica records become scalar
        // loads, so per-item constants never wait behind the particle loads
        const int item = __builtin_amdgcn_readfirstlane(sItem);
        if (item >= bp.n_items) break;
        // per-item constants moved to scalar registers once, before the particle
        // loop (a value still pending from a vector load would make every wait
        // inside the loop also wait for the prefetched particle loads)
        Item it = bp.items[item];
        it.r = uniform_i(it.r);
        it.p0 = uniform_i(it.p0);
        it.cnt = uniform_i(it.cnt);
        RepP rp = bp.reps[it.r];
        rp.nx = uniform_i(rp.nx);
        rp.nitems = uniform_i(rp.nitems);
        rp.item0 = uniform_i(rp.item0);
        rp.n = uniform_i(rp.n);
        rp.g0 = uniform_l(rp.g0);
        rp.dtdx = uniform_f(rp.dtdx);
        rp.dx = uniform_d(rp.dx);
        rp.acc_scale = uniform_d(rp.acc_scale);
        rp.mass = uniform_d(rp.mass);
        Geo g{};
        g.dim = 1;
        g.vdim = 1;
        g.nx = rp.nx;
        g.ny = 1;
        g.S = bp.S;
        PushC pc{};
        pc.af = bp.a;
        pc.tf = bp.t;
        pc.sf = bp.s;
        pc.dtdx = rp.dtdx;
        for (int i = threadIdx.x; i <= rp.nx; i += blockDim.x) {
            if (i < rp.nx) sA[i] = 0ull;
            sE[i] = (float)E[rp.g0 + (i == rp.nx ? 0 : i)];
        }
        __syncthreads();
        double ke = 0.0, px = 0.0;
        // kBatchU particles per thread per stage, each stage's words loaded one
        // stage ahead of their use (indices clamped into the item, so every
        // load is in bounds): enough loads in flight per wave to cover the
        // memory latency with the few waves a replica chunk gives a CU
        struct W3 {
            int32_t c[kBatchU];
            float o[kBatchU], v[kBatchU];
        };
        constexpr int CH = kBlock * kBatchU;
        auto fetch = [&](int base, W3 &r) {
#pragma unroll
            for (int j = 0; j < kBatchU; ++j) {
                const int i = it.p0 + min(base + j * kBlock + (int)threadIdx.x, it.cnt - 1);
                r.c[j] = cell[i];
                r.o[j] = ox[i];
                r.v[j] = vx[i];
            }
            __builtin_amdgcn_sched_barrier(0);
        };
        auto process = [&](int base, const W3 &r) {
#pragma unroll
            for (int j = 0; j < kBatchU; ++j) {
                const int k = base + j * kBlock + threadIdx.x;
                if (k >= it.cnt) continue;
                const int i = it.p0 + k;
                Pt<true> q;
                q.ix = r.c[j];
                q.iy = 0;
                q.fx = r.o[j];
                q.fy = 0.0f;
                q.vx = r.v[j];
                q.vy = q.vz = 0.0f;
                bool ok = (unsigned)q.ix < (unsigned)rp.nx && q.fx >= 0.0f && q.fx < 1.0f;
                if (!ok) {
                    q.ix = 0;
                    q.fx = 0.0f;
                }
                if constexpr (MODE == MODE_DEPOSIT) {
                    unsigned long long w[4];
                    dep_weights<true, 1>(q, g, w);
                    atomicAdd(&sA[q.ix], w[1] + kCountUnit);
                } else {
                    float ex, ey;
                    gather_lds<float, 1>(sE, rp.nx + 1, rp.nx + 1, q.ix, 0, q.fx, q.fy, ex, ey);
                    const double v2o = (double)(q.vx * q.vx);
                    boris<float, 1>(q.vx, q.vy, ex, ey, pc.af, pc.tf, pc.sf);
                    if constexpr (MODE == MODE_STEP) {
                        const double v2n = (double)(q.vx * q.vx);
                        ke += 0.5 * (v2o + v2n);
                        px += (double)q.vx;
                        int sx, sy;
                        ok = move_pt<true, 1>(q, g, pc, sx, sy) && ok;
                        unsigned long long w[4];
                        dep_weights<true, 1>(q, g, w);
                        atomicAdd(&sA[q.ix], w[1] + kCountUnit);
                        cell[i] = q.ix;
                        ox[i] = q.fx;
                    }
                    vx[i] = q.vx;
                }
                if (!ok) atomicOr(&sErr, ERR_DOMAIN);
            }
        };
        W3 ra, rb;
        if (it.cnt > 0) fetch(0, ra);
        for (int base = 0; base < it.cnt; base += 2 * CH) {
            if (base + CH < it.cnt) fetch(base + CH, rb);
            process(base, ra);
            if (base + 2 * CH < it.cnt) fetch(base + 2 * CH, ra);
            if (base + CH < it.cnt) process(base + CH, rb);
        }
        __syncthreads();
        if constexpr (MODE == MODE_HALF) continue;
        // node j receives w0 = 2^S - w1 from each particle of cell j and w1 from
        // each particle of cell j-1: I_j = 2^S count_j - W_j + W_{j-1}
        // (modulo 2^64, exact: the same integers as two atomics per particle)
        for (int i = threadIdx.x; i < rp.nx; i += blockDim.x) {
            const unsigned long long a = sA[i], b = sA[i == 0 ? rp.nx - 1 : i - 1];
            const unsigned long long v = ((a >> kCountShift) << bp.S) - (a & kSumMask) + (b & kSumMask);
            if (v) atomicAdd(&acc[rp.g0 + i], v);
        }
        if constexpr (MODE == MODE_STEP) {
            const double kt = block_sum(ke, sRed);
            const double pt = block_sum(px, sRed);
            if (threadIdx.x == 0) {
                __hip_atomic_store(&bp.part[2 * item], kt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&bp.part[2 * item + 1], pt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        // publish this chunk; the block that completes the replica solves its
        // field. Everything another block reads from it (the deposit in acc,
        // the partial sums) is written and read with device-scope atomics, so
        // completing those writes before the counter is enough: each thread
        // waits for its own memory operations, the barrier for everyone's (no
        // L2 write-back or invalidate)
        __builtin_amdgcn_s_waitcnt(kWaitVmem);
        __syncthreads();
        if (threadIdx.x == 0) sLast = (atomicAdd(&bp.rep_done[it.r], 1) == rp.nitems - 1);
        __syncthreads();
        if (!sLast) continue;
        // the replica's charge: the exact integer total of its node sums
        // (whole particles + remainder in units of 2^-S particle)
        QSum qs{0, 0};
        for (int i = threadIdx.x; i < rp.nx; i += blockDim.x) {
            // read-and-clear at the device coherence point (sA is free again:
            // this block's own flush above has completed)
            const unsigned long long v = atomicExch(&acc[rp.g0 + i], 0ull);
            if (rho_out) rho_out[rp.g0 + i] = (int64_t)v;
            const double rr = bp.rho_ion + rp.acc_scale * (double)(int64_t)v;
            sR[i] = rr;
            qsum_add(qs, (int64_t)v, bp.S);
        }
        // (block-local: this block alone reduces the replica's grid)
        const QSum qt = qsum_block(qs, bp.S);
        const double wsum = field1d_block(sR, rp.nx, rp.dx, E + rp.g0, nullptr, sRed, sScan);
        double kt = 0.0, pt = 0.0;
        if constexpr (MODE == MODE_STEP) {
            for (int j = threadIdx.x; j < rp.nitems; j += blockDim.x) {
                // written by other blocks before their release fence: read at agent scope
                kt += __hip_atomic_load(&bp.part[2 * (rp.item0 + j)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                pt += __hip_atomic_load(&bp.part[2 * (rp.item0 + j) + 1], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
            }
            kt = block_sum(kt, sRed);
            pt = block_sum(pt, sRed);
        }
        if (threadIdx.x == 0) {
            if (diag) {
                double *d = diag + ((size_t)(*bp.step) * bp.nrep + it.r) * 4;
                d[0] = qsum_charge(qt, bp.S, uniform_d(rp.q_macro));
                d[1] = 0.5 * wsum * rp.dx;
                d[2] = 0.5 * rp.mass * kt;
                d[3] = rp.mass * pt;
            }
            bp.rep_done[it.r] = 0;
        }
        __syncthreads();
    }
    // leave: the last block out resets the work counter and advances the step
    __syncthreads();
    if (threadIdx.x == 0) {
        if (sErr) atomicOr(bp.err, sErr);
        // every work-queue atomic of this block has completed before its exit
        // is counted; the resets are read by the next launch
        __builtin_amdgcn_s_waitcnt(kWaitVmem);
        if (atomicAdd(bp.done, 1) == (int)gridDim.x - 1) {
            *bp.head = 0;
            *bp.done = 0;
            if (MODE == MODE_STEP) *bp.step = *bp.step + 1;
        }
    }
}

__global__ void k_batch_set(int *p, int v) { *p = v; }

}  // namespace
}  // namespace apic

using namespace apic;

struct apic_batch {
    int nrep = 0;
    std::vector<apic_replica> reps;
    std::vector<int64_t> poff, goff;
    int64_t n_total = 0, g_total = 0;
    int n_items = 0, chunk = 0, grid = 0;
    double dt = 0, qm = 0, rho_ion = 0;
    void *dev = nullptr;
    RepP *d_reps = nullptr;
    Item *d_items = nullptr;
    int *d_words = nullptr;       // head, done, step, err, rep_done[nrep]
    double *d_part = nullptr;
    std::string err;
    // captured step graph (keyed by the pointers it bakes in)
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    const void *gkey[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
};

namespace {

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

BatchP batch_params(const apic_batch *b, double dt_scale) {
    BatchP p{};
    p.reps = b->d_reps;
    p.items = b->d_items;
    p.n_items = b->n_items;
    p.nrep = b->nrep;
    p.S = 32;
    p.head = b->d_words + 0;
    p.done = b->d_words + 1;
    p.step = b->d_words + 2;
    p.err = b->d_words + 3;
    p.rep_done = b->d_words + 4;
    p.part = b->d_part;
    // same coefficient arithmetic as the single-plasma path
    const double dte = b->dt * dt_scale;
    const double a = b->qm * dte * 0.5;
    const double t = a * 0.0;
    const double s = 2.0 * t / (1.0 + t * t);
    p.a = (float)a;
    p.t = (float)t;
    p.s = (float)s;
    p.rho_ion = b->rho_ion;
    return p;
}

apic_status bfail(apic_batch *b, apic_status st, const std::string &m) {
    if (b) b->err = m;
    return st;
}

#define BCHK(b, expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return bfail(b, APIC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

apic_status check_state(apic_batch *b, const apic_batch_state *st) {
    if (!st || !st->cell || !st->ox || !st->vx || !st->E) return bfail(b, APIC_EINVAL, "state arrays are required");
    return APIC_OK;
}

template <int MODE>
apic_status launch_mode(apic_batch *b, apic_batch_state *st, double dt_scale, double *diag, int64_t *rho_out,
                        void *ws, hipStream_t s) {
    BatchP p = batch_params(b, dt_scale);
    hipLaunchKernelGGL(k_batch<MODE>, dim3(b->grid), dim3(kBlock), 0, s, p, st->cell, st->ox, st->vx, st->E,
                       (unsigned long long *)ws, diag, rho_out);
    BCHK(b, hipGetLastError());
    return APIC_OK;
}

}  // namespace

extern "C" {

apic_status apic_batch_create(const apic_replica *reps, int nrep, double dt, double qm, double rho_ion, int chunk,
                              apic_batch **out) {
    if (!reps || !out || nrep <= 0 || !(dt > 0) || qm == 0.0 || !std::isfinite(qm)) return APIC_EINVAL;
    *out = nullptr;
    if (chunk <= 0) chunk = 8192;
    if (chunk < kBlock) return APIC_EINVAL;
    chunk = std::min(chunk, kBatchMaxChunk);
    apic_batch *b = new (std::nothrow) apic_batch();
    if (!b) return APIC_ENOMEM;
    b->nrep = nrep;
    b->reps.assign(reps, reps + nrep);
    b->dt = dt;
    b->qm = qm;
    b->rho_ion = rho_ion;
    b->chunk = chunk;
    b->poff.assign(nrep + 1, 0);
    b->goff.assign(nrep + 1, 0);
    for (int r = 0; r < nrep; ++r) {
        const apic_replica &R = reps[r];
        if (R.nx < 2 || R.nx > kBatchMaxNx || R.n < 0 || !(R.lx > 0)) {
            delete b;
            return APIC_EINVAL;
        }
        b->poff[r + 1] = b->poff[r] + R.n;
        b->goff[r + 1] = b->goff[r] + R.nx;
    }
    b->n_total = b->poff[nrep];
    b->g_total = b->goff[nrep];
    if (b->n_total > (int64_t)INT32_MAX - 1) {
        delete b;
        return APIC_EINVAL;
    }
    // work items: replicas in descending particle count, each cut in chunks
    std::vector<int> order(nrep);
    for (int r = 0; r < nrep; ++r) order[r] = r;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return reps[a].n > reps[c].n; });
    std::vector<RepP> rp(nrep);
    std::vector<Item> items;
    for (int r : order) {
        const apic_replica &R = reps[r];
        RepP &q = rp[r];
        q.nx = R.nx;
        q.n = (int)R.n;
        q.p0 = (int)b->poff[r];
        q.g0 = b->goff[r];
        q.dx = R.lx / R.nx;
        q.dtdx = (float)(dt / q.dx);
        const double q_macro = R.n > 0 ? -rho_ion * R.lx / (double)R.n : 0.0;
        q.acc_scale = std::ldexp(q_macro / q.dx, -32);
        q.q_macro = q_macro;
        q.mass = q_macro / qm;
        q.item0 = (int)items.size();
        int64_t left = R.n, at = 0;
        do {
            Item it;
            it.r = r;
            it.p0 = (int)(b->poff[r] + at);
            it.cnt = (int)std::min<int64_t>(left, chunk);
            it.pad = 0;
            items.push_back(it);
            at += it.cnt;
            left -= it.cnt;
        } while (left > 0);
        q.nitems = (int)items.size() - q.item0;
    }
    b->n_items = (int)items.size();
    size_t bytes = al256(sizeof(RepP) * nrep) + al256(sizeof(Item) * items.size()) +
                   al256(sizeof(int) * (4 + nrep)) + al256(sizeof(double) * 2 * items.size());
    if (hipMalloc(&b->dev, bytes) != hipSuccess) {
        delete b;
        return APIC_ENOMEM;
    }
    char *p = (char *)b->dev;
    b->d_reps = (RepP *)p;
    p += al256(sizeof(RepP) * nrep);
    b->d_items = (Item *)p;
    p += al256(sizeof(Item) * items.size());
    b->d_words = (int *)p;
    p += al256(sizeof(int) * (4 + nrep));
    b->d_part = (double *)p;
    bool ok = hipMemset(b->dev, 0, bytes) == hipSuccess &&
              hipMemcpy(b->d_reps, rp.data(), sizeof(RepP) * nrep, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(b->d_items, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        (void)hipFree(b->dev);
        delete b;
        return APIC_EHIP;
    }
    // persistent grid: what fits on the device at once
    int dev = 0, cus = 256, per_cu = 0;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<MODE_STEP>, kBlock, 0) != hipSuccess ||
        per_cu <= 0)
        per_cu = 4;
    b->grid = std::max(1, std::min(cus * per_cu, b->n_items));
    *out = b;
    return APIC_OK;
}

void apic_batch_destroy(apic_batch *b) {
    if (!b) return;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->dev) (void)hipFree(b->dev);
    delete b;
}

apic_status apic_batch_sizes(const apic_batch *b, int64_t *n_total, int64_t *g_total, size_t *ws_bytes) {
    if (!b) return APIC_EINVAL;
    if (n_total) *n_total = b->n_total;
    if (g_total) *g_total = b->g_total;
    if (ws_bytes) *ws_bytes = al256(8 * (size_t)b->g_total);
    return APIC_OK;
}

apic_status apic_batch_offsets(const apic_batch *b, int64_t *part_off, int64_t *grid_off) {
    if (!b) return APIC_EINVAL;
    if (part_off) std::copy(b->poff.begin(), b->poff.end(), part_off);
    if (grid_off) std::copy(b->goff.begin(), b->goff.end(), grid_off);
    return APIC_OK;
}

int apic_batch_work_items(const apic_batch *b) { return b ? b->n_items : -1; }

apic_status apic_batch_init(apic_batch *b, apic_batch_state *st, void *ws, void *stream) {
    if (!b) return APIC_EINVAL;
    apic_status r = check_state(b, st);
    if (r != APIC_OK) return r;
    if (!ws) return bfail(b, APIC_EINVAL, "workspace is NULL");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_batch_set, dim3(1), dim3(1), 0, s, b->d_words + 2, 0);
    BCHK(b, hipGetLastError());
    // the accumulator starts at zero; every field solve leaves it at zero
    BCHK(b, launch_fill_u64((uint64_t *)ws, b->g_total, 0, s));
    r = launch_mode<MODE_DEPOSIT>(b, st, 1.0, nullptr, nullptr, ws, s);
    if (r != APIC_OK) return r;
    return launch_mode<MODE_HALF>(b, st, -0.5, nullptr, nullptr, ws, s);
}

apic_status apic_batch_step(apic_batch *b, apic_batch_state *st, int nsteps, double *diag, int64_t *rho, void *ws,
                            void *stream, int use_graph) {
    if (!b) return APIC_EINVAL;
    apic_status r = check_state(b, st);
    if (r != APIC_OK) return r;
    if (!ws || nsteps < 0) return bfail(b, APIC_EINVAL, "workspace and nsteps >= 0 are required");
    if (nsteps == 0) return APIC_OK;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_batch_set, dim3(1), dim3(1), 0, s, b->d_words + 2, 0);
    BCHK(b, hipGetLastError());
    for (int k = 0; k < nsteps; ++k) {
        int64_t *rho_k = (k == nsteps - 1) ? rho : nullptr;
        if (!use_graph || rho_k) {
            r = launch_mode<MODE_STEP>(b, st, 1.0, diag, rho_k, ws, s);
            if (r != APIC_OK) return r;
            continue;
        }
        const void *key[6] = {st->cell, st->ox, st->vx, st->E, ws, diag};
        if (!b->gexec || !std::equal(key, key + 6, b->gkey)) {
            if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
            if (b->graph) (void)hipGraphDestroy(b->graph);
            b->gexec = nullptr;
            b->graph = nullptr;
            hipStream_t cs;
            BCHK(b, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            BCHK(b, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            BatchP p = batch_params(b, 1.0);
            hipLaunchKernelGGL(k_batch<MODE_STEP>, dim3(b->grid), dim3(kBlock), 0, cs, p, st->cell, st->ox, st->vx,
                               st->E, (unsigned long long *)ws, diag, (int64_t *)nullptr);
            hipError_t le = hipGetLastError();
            hipError_t ce = hipStreamEndCapture(cs, &b->graph);
            (void)hipStreamDestroy(cs);
            if (le != hipSuccess || ce != hipSuccess) return bfail(b, APIC_EHIP, "graph capture of the batch step failed");
            BCHK(b, hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
            std::copy(key, key + 6, b->gkey);
        }
        BCHK(b, hipGraphLaunch(b->gexec, s));
    }
    return APIC_OK;
}

apic_status apic_batch_sync_status(apic_batch *b, void *stream) {
    if (!b) return APIC_EINVAL;
    BCHK(b, hipStreamSynchronize((hipStream_t)stream));
    int bits = 0;
    BCHK(b, hipMemcpy(&bits, b->d_words + 3, sizeof(int), hipMemcpyDeviceToHost));
    if (!bits) return APIC_OK;
    int zero = 0;
    BCHK(b, hipMemcpy(b->d_words + 3, &zero, sizeof(int), hipMemcpyHostToDevice));
    return bfail(b, APIC_EDOMAIN, "non-finite or out-of-range particle coordinate in a replica");
}

const char *apic_batch_last_error(const apic_batch *b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
