// Autotuner: picks the sort-bucket tile of the single-plasma step and the
// work-item size of the batched replicas by timing candidates on the caller's
// own particles (the caller's arrays are only read).
//
// A setup call, never part of a timed loop: each trial allocates a scratch
// copy of the particles and a context, runs two warm-up steps and times a few
// more with HIP events on the caller's stream. The winner is kept in a
// process-wide cache keyed by the problem's shape, so a later call with the
// same shape returns at once.
#include "apic.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

namespace {

// dim, vdim, nx, ny, nz, precision, floor(log2(particles per cell)), velocity advance
using TileKey = std::tuple<int, int, int, int, int, int, int, int>;
using Tile = std::tuple<int, int, int>;

std::mutex g_mu;
std::map<TileKey, Tile> g_tiles;
std::map<std::pair<int64_t, int>, int> g_chunks;  // (total particles, replicas) -> chunk

struct DevBuf {
    void *p = nullptr;
    bool ok = true;
    explicit DevBuf(size_t n) {
        if (n) ok = hipMalloc(&p, n) == hipSuccess;
    }
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
};

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    Timer() {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    double ms() {
        (void)hipEventSynchronize(b);
        float t = 0;
        return hipEventElapsedTime(&t, a, b) == hipSuccess ? t : INFINITY;
    }
};

int floor_log2(double v) {
    int r = 0;
    while (v >= 2.0) {
        v *= 0.5;
        ++r;
    }
    return r;
}

hipError_t copy_in(void *dst, const void *src, size_t bytes, hipStream_t s) {
    if (!src || !dst || !bytes) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
}

// One trial of a tile shape: copy the particles, sort, deposit, solve E^0,
// four untimed steps (the first steps after the sort read every particle in
// the tally pass and start from the sort's order), then two timed runs of
// nsteps steps (rounded up to even, so that no run ends with the copy back
// of an odd count), the faster of the two. Returns ms per step or INFINITY.
double trial_tiles(const apic_grid_desc &d, const apic_particles &src, const Tile &t, int nsteps, hipStream_t s) {
    apic_grid_desc dd = d;
    dd.tile_x = std::get<0>(t);
    dd.tile_y = std::get<1>(t);
    dd.tile_z = std::get<2>(t);
    apic_ctx *c = nullptr;
    if (apic_create(&dd, src.n, &c) != APIC_OK) return INFINITY;
    const bool mixed = d.prec == APIC_MIXED;
    const size_t n = (size_t)src.n, r = mixed ? 4 : 8;
    const size_t G = (size_t)d.nx * (d.dim >= 2 ? d.ny : 1) * (d.dim == 3 ? d.nz : 1);
    size_t wsb = 0;
    (void)apic_workspace_size(c, &wsb);
    DevBuf ws(wsb), pa(r * n), pb(d.dim >= 2 ? r * n : 0), pc(d.dim == 3 ? r * n : 0), cell(mixed ? 4 * n : 0),
        vx(r * n), vy(d.vdim >= 2 ? r * n : 0), vz(d.vdim >= 3 ? r * n : 0),
        bs(4 * ((size_t)apic_num_buckets(c) + 1)), rho(8 * G), E(8 * G * d.dim);
    double out = INFINITY;
    if (ws.ok && pa.ok && pb.ok && pc.ok && cell.ok && vx.ok && vy.ok && vz.ok && bs.ok && rho.ok && E.ok) {
        apic_particles p{};
        p.n = src.n;
        hipError_t e = hipSuccess;
        if (mixed) {
            p.cell = (int32_t *)cell.p;
            p.ox = (float *)pa.p;
            p.oy = (float *)pb.p;
            p.oz = (float *)pc.p;
            e = copy_in(p.cell, src.cell, 4 * n, s);
            if (e == hipSuccess) e = copy_in(p.ox, src.ox, 4 * n, s);
            if (e == hipSuccess && d.dim >= 2) e = copy_in(p.oy, src.oy, 4 * n, s);
            if (e == hipSuccess && d.dim == 3) e = copy_in(p.oz, src.oz, 4 * n, s);
        } else {
            p.x = (double *)pa.p;
            p.y = (double *)pb.p;
            p.z = (double *)pc.p;
            e = copy_in(p.x, src.x, 8 * n, s);
            if (e == hipSuccess && d.dim >= 2) e = copy_in(p.y, src.y, 8 * n, s);
            if (e == hipSuccess && d.dim == 3) e = copy_in(p.z, src.z, 8 * n, s);
        }
        p.vx = vx.p;
        p.vy = d.vdim >= 2 ? vy.p : nullptr;
        p.vz = d.vdim >= 3 ? vz.p : nullptr;
        if (e == hipSuccess) e = copy_in(p.vx, src.vx, r * n, s);
        if (e == hipSuccess && d.vdim >= 2) e = copy_in(p.vy, src.vy, r * n, s);
        if (e == hipSuccess && d.vdim >= 3) e = copy_in(p.vz, src.vz, r * n, s);
        p.bucket_start = (int32_t *)bs.p;
        apic_status st = e == hipSuccess ? APIC_OK : APIC_EHIP;
        if (st == APIC_OK) st = apic_sort_by_cell(c, &p, ws.p, s);
        if (st == APIC_OK) st = apic_deposit(c, &p, rho.p, s);
        if (st == APIC_OK) st = apic_field_solve(c, rho.p, (double *)E.p, nullptr, nullptr, ws.p, s);
        if (st == APIC_OK) st = apic_step(c, &p, nullptr, (double *)E.p, nullptr, 4, nullptr, ws.p, s);
        const int ns = nsteps + (nsteps & 1);
        for (int run = 0; run < 2 && st == APIC_OK; ++run) {
            Timer t;
            (void)hipEventRecord(t.a, s);
            st = apic_step(c, &p, nullptr, (double *)E.p, nullptr, ns, nullptr, ws.p, s);
            (void)hipEventRecord(t.b, s);
            if (st == APIC_OK) {
                const double ms = t.ms();
                if (apic_sync_status(c, s) != APIC_OK) st = APIC_EDOMAIN;
                else out = std::min(out, ms / ns);
            }
        }
        if (st != APIC_OK) out = INFINITY;
    }
    (void)hipStreamSynchronize(s);
    apic_destroy(c);
    return out;
}

double trial_chunk(const apic_replica *reps, int nrep, double dt, double qm, double rho_ion,
                   const apic_batch_state &src, int chunk, int nsteps, hipStream_t s) {
    apic_batch *b = nullptr;
    if (apic_batch_create(reps, nrep, dt, qm, rho_ion, chunk, &b) != APIC_OK) return INFINITY;
    int64_t n = 0, g = 0;
    size_t wsb = 0;
    (void)apic_batch_sizes(b, &n, &g, &wsb);
    DevBuf ws(wsb), cell(4 * (size_t)n), ox(4 * (size_t)n), vx(4 * (size_t)n), E(8 * (size_t)g);
    double out = INFINITY;
    if (ws.ok && cell.ok && ox.ok && vx.ok && E.ok) {
        hipError_t e = copy_in(cell.p, src.cell, 4 * (size_t)n, s);
        if (e == hipSuccess) e = copy_in(ox.p, src.ox, 4 * (size_t)n, s);
        if (e == hipSuccess) e = copy_in(vx.p, src.vx, 4 * (size_t)n, s);
        apic_batch_state st{(int32_t *)cell.p, (float *)ox.p, (float *)vx.p, (double *)E.p};
        apic_status r = e == hipSuccess ? APIC_OK : APIC_EHIP;
        if (r == APIC_OK) r = apic_batch_init(b, &st, ws.p, s);
        if (r == APIC_OK) r = apic_batch_step(b, &st, 2, nullptr, nullptr, ws.p, s, 1);
        Timer t;
        if (r == APIC_OK) {
            (void)hipEventRecord(t.a, s);
            r = apic_batch_step(b, &st, nsteps, nullptr, nullptr, ws.p, s, 1);
            (void)hipEventRecord(t.b, s);
        }
        if (r == APIC_OK) {
            const double ms = t.ms();
            if (apic_batch_sync_status(b, s) == APIC_OK) out = ms / nsteps;
        }
    }
    (void)hipStreamSynchronize(s);
    apic_batch_destroy(b);
    return out;
}

}  // namespace

extern "C" {

apic_status apic_autotune_tiles(const apic_grid_desc *desc, const apic_particles *p, int nsteps, int *tile_x,
                                int *tile_y, int *tile_z, double *ms_per_step, void *stream) {
    if (!desc || !p || !tile_x || !tile_y || nsteps <= 0 || p->n <= 0) return APIC_EINVAL;
    const apic_grid_desc &d = *desc;
    if (d.dim == 3 && !tile_z) return APIC_EINVAL;
    if (d.model == APIC_ELECTROMAGNETIC || d.walls_x) return APIC_EUNSUPPORTED;
    if (d.prec == APIC_MIXED ? (!p->cell || !p->ox || (d.dim == 3 && !p->oz)) : (!p->x || (d.dim == 3 && !p->z)))
        return APIC_EINVAL;
    const int ny = d.dim >= 2 ? d.ny : 1, nz = d.dim == 3 ? d.nz : 1;
    const TileKey key{d.dim, d.vdim, d.nx, ny, nz, (int)d.prec,
                      floor_log2((double)p->n / ((double)d.nx * ny * nz)), d.pusher};
    auto put = [&](const Tile &t) {
        *tile_x = std::get<0>(t);
        *tile_y = std::get<1>(t);
        if (tile_z) *tile_z = std::get<2>(t);
    };
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_tiles.find(key);
        if (it != g_tiles.end()) {
            put(it->second);
            if (ms_per_step) *ms_per_step = -1.0;
            return APIC_OK;
        }
    }
    std::vector<Tile> cand;
    if (d.dim == 3) {
        // 4 to 16 cells along x, 4 to 8 along y and z (a candidate whose E
        // tile and deposit region do not fit a workgroup's LDS is rejected by
        // apic_create and skipped)
        const int sizes[][3] = {{4, 4, 4}, {8, 4, 4}, {8, 8, 4}, {8, 8, 8}, {16, 8, 4}, {16, 8, 8}, {16, 16, 8}};
        for (auto &t : sizes)
            if (t[0] <= d.nx && t[1] <= d.ny && t[2] <= d.nz) cand.push_back({t[0], t[1], t[2]});
    } else if (d.dim == 2) {
        const int sizes[][2] = {{4, 4}, {8, 4}, {8, 8}, {16, 8}, {16, 16}, {32, 16}, {32, 32}};
        for (auto &t : sizes)
            if (t[0] <= d.nx && t[1] <= d.ny) cand.push_back({t[0], t[1], 0});
    } else {
        for (int t = 8; t <= 1024 && t <= d.nx; t *= 2) cand.push_back({t, 1, 0});
    }
    cand.push_back({0, 0, 0});  // the library's default
    hipStream_t s = (hipStream_t)stream;
    double best = INFINITY;
    Tile pick{0, 0, 0};
    for (auto &t : cand) {
        const double ms = trial_tiles(d, *p, t, nsteps, s);
        if (ms < best) {
            best = ms;
            pick = t;
        }
    }
    if (!std::isfinite(best)) return APIC_EHIP;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_tiles[key] = pick;
    }
    put(pick);
    if (ms_per_step) *ms_per_step = best;
    return APIC_OK;
}

apic_status apic_batch_autotune_chunk(const apic_replica *reps, int nrep, double dt, double qm, double rho_ion,
                                      const apic_batch_state *st, int nsteps, int *chunk, double *ms_per_step,
                                      void *stream) {
    if (!reps || nrep <= 0 || !st || !st->cell || !st->ox || !st->vx || !chunk || nsteps <= 0)
        return APIC_EINVAL;
    int64_t ntot = 0;
    for (int r = 0; r < nrep; ++r) ntot += reps[r].n;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_chunks.find({ntot, nrep});
        if (it != g_chunks.end()) {
            *chunk = it->second;
            if (ms_per_step) *ms_per_step = -1.0;
            return APIC_OK;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    const int cands[] = {1024, 2048, 4096, 8192, 16384, 32768, 65535};
    double best = INFINITY;
    int pick = 0;
    for (int ch : cands) {
        const double ms = trial_chunk(reps, nrep, dt, qm, rho_ion, *st, ch, nsteps, s);
        if (ms < best) {
            best = ms;
            pick = ch;
        }
    }
    if (!std::isfinite(best)) return APIC_EHIP;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_chunks[{ntot, nrep}] = pick;
    }
    *chunk = pick;
    if (ms_per_step) *ms_per_step = best;
    return APIC_OK;
}

}  // extern "C"
