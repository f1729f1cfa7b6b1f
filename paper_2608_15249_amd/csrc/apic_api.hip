// Host side of libapic: context, workspace layout, argument checks and the
// C-ABI entry points declared in include/apic.h.
#include "apic.h"
#include "apic_ctx.h"

#include <cstdlib>

#include <hipfft/hipfft.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <algorithm>
#include <vector>

using namespace apic;
using namespace apic_host;

// ---- fixed device workspace of apic_step_static -------------------------------
// One array per GPU the library runs on, held until the process ends. In host
// code its name is only a host-side stand-in: every use goes through the
// device address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[APIC_STATIC_WS_BYTES];

namespace {
constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_ok[kMaxDevices] = {};
std::mutex g_scratch_mu;

// The current device's address of scratch (looked up once per device).
hipError_t scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ok[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = ptr;
        g_scratch_ok[dev] = true;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

namespace apic_host {

apic_status fail(apic_ctx *c, apic_status st, const char *msg) {
    if (c) c->err = msg;
    return st;
}

apic_status hip_fail(apic_ctx *c, hipError_t e, const char *where) {
    if (c) c->err = std::string(where) + ": " + hipGetErrorString(e);
    return APIC_EHIP;
}

int ilog2_floor(int64_t v) {
    int r = 0;
    while ((int64_t(1) << (r + 1)) <= v) ++r;
    return r;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Default bucket tile: about 4096 particles per bucket (the workgroup's work
// item), tile side a power of two.
void default_tiles(const apic_grid_desc &d, int64_t n, int &tsx, int &tsy, int &tsz) {
    const double cells = (double)d.nx * (d.dim >= 2 ? d.ny : 1) * (d.dim == 3 ? d.nz : 1);
    const double ppc = n > 0 ? (double)n / cells : 1.0;
    double target = 4096.0 / (ppc > 0 ? ppc : 1.0);
    if (target < 1.0) target = 1.0;
    tsz = 0;
    if (d.dim == 1) {
        tsx = ilog2_floor((int64_t)target);
        if (tsx > 12) tsx = 12;
        tsy = 0;
    } else if (d.dim == 3) {
        // about 8192 particles per tile, cube-like, at most 16 cells along x
        // and 8 along y and z (E tile and deposit region of a workgroup stay
        // within LDS). Measured at 128^3, 8 per cell: 16 x 8 x 8 tiles give
        // 0.537 / 0.664 ms per step (mixed / FP64) against 0.549 / 0.707 with
        // 8^3: fewer particles near a tile face for the count pass.
        const int t = ilog2_floor((int64_t)(2.0 * target));
        tsx = std::min(4, std::max(1, (t + 2) / 3));
        tsy = std::min(3, std::max(1, (t + 1) / 3));
        tsz = std::min(3, std::max(1, t / 3));
    } else {
        // about 16384 particles per tile where the grid still has 1024 tiles
        // or more (the autotuner's picks at 512^2 and 1024^2 hold 16384-32768
        // particles: fewer cross a tile edge), else about 4096 (enough
        // workgroups on small grids)
        const double big = 4.0 * target;
        int t = ilog2_floor((int64_t)(cells / big >= 1024.0 ? big : target));
        tsx = (t + 1) / 2;
        tsy = t / 2;
        if (tsx > 5) tsx = 5;
        if (tsy > 5) tsy = 5;
        if (tsx < 1) tsx = 1;
        if (tsy < 1) tsy = 1;
    }
}

void layout(apic_ctx *c) {
    const int64_t n = c->n;
    const size_t r = c->mixed ? 4 : 8;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    const int dim = c->d.dim, vdim = c->d.vdim;
    c->o_x = c->o_y = c->o_z = c->o_cell = c->o_ox = c->o_oy = c->o_oz = (size_t)-1;
    c->o_vx = c->o_vy = c->o_vz = (size_t)-1;
    if (c->mixed) {
        c->o_cell = take(4 * n);
        c->o_ox = take(4 * n);
        if (dim >= 2) c->o_oy = take(4 * n);
        if (dim == 3) c->o_oz = take(4 * n);
    } else {
        c->o_x = take(8 * n);
        if (dim >= 2) c->o_y = take(8 * n);
        if (dim == 3) c->o_z = take(8 * n);
    }
    c->o_vx = take(r * n);
    if (vdim >= 2) c->o_vy = take(r * n);
    if (vdim >= 3) c->o_vz = take(r * n);
    const int64_t nb = c->g.nbuckets;
    const int64_t G = (int64_t)c->d.nx * c->d.ny * c->d.nz;
    c->o_keys = take(4 * n);
    c->o_keys2 = take(4 * n);
    c->o_idx = take(4 * n);
    c->o_idx2 = take(4 * n);
    c->o_rcnt = take(4 * (int64_t)sort_chunks(n) * sort_table_entries());
    c->o_roff = take(4 * (int64_t)sort_chunks(n) * sort_table_entries());
    c->o_rpart = take(4 * (int64_t)sort_part_entries());
    c->o_bstart = take(4 * (nb + 1));
    c->o_cnt = take(4 * nb * kStepTab);
    c->o_offs = take(4 * nb * kStepTab);
    c->o_farcnt = take(4 * nb);
    c->o_farcur = take(4 * nb);
    c->o_tot = take(4 * 2 * nb);   // two alternating buffers
    c->o_deep = take(4 * nb * kDeepTab);
    c->o_acc = take(8 * G);
    // electromagnetic step: two current buffers and a second field buffer,
    // alternating by step (the one-launch field update reads one, writes the other)
    c->o_jacc = c->d.model == APIC_ELECTROMAGNETIC ? take(2 * 24 * G) : (size_t)-1;
    c->o_f2 = c->d.model == APIC_ELECTROMAGNETIC ? take(48 * G) : (size_t)-1;
    c->o_e32 = (c->mixed && dim >= 2 && c->d.model != APIC_ELECTROMAGNETIC) ? take(4 * dim * G) : (size_t)-1;
    c->o_rho = take(8 * G);
    if (dim >= 2) {
        const int64_t H = (int64_t)(c->d.nx / 2 + 1) * c->d.ny * c->d.nz;
        c->o_rhat = take(16 * H);
        // phi_hat (the field solve); the adjoint uses 2 spectra here in 2D
        c->o_ehat = take(16 * dim * H);
    } else {
        c->o_rhat = c->o_ehat = (size_t)-1;
    }
    c->ws_bytes = off;
}


Parts parts_of(const apic_particles *p) {
    Parts q;
    q.x = p->x;
    q.y = p->y;
    q.z = p->z;
    q.cell = p->cell;
    q.ox = p->ox;
    q.oy = p->oy;
    q.oz = p->oz;
    q.vx = p->vx;
    q.vy = p->vy;
    q.vz = p->vz;
    return q;
}

Parts parts_ws(const apic_ctx *c, void *ws) {
    Parts q;
    q.x = wsp<double>(ws, c->o_x);
    q.y = wsp<double>(ws, c->o_y);
    q.z = wsp<double>(ws, c->o_z);
    q.cell = wsp<int32_t>(ws, c->o_cell);
    q.ox = wsp<float>(ws, c->o_ox);
    q.oy = wsp<float>(ws, c->o_oy);
    q.oz = wsp<float>(ws, c->o_oz);
    q.vx = wsp<void>(ws, c->o_vx);
    q.vy = wsp<void>(ws, c->o_vy);
    q.vz = wsp<void>(ws, c->o_vz);
    return q;
}

apic_status check_parts(apic_ctx *c, const apic_particles *p, bool need_bstart) {
    if (!p) return fail(c, APIC_EINVAL, "particles is NULL");
    if (p->n != c->n) return fail(c, APIC_EINVAL, "particles.n differs from the context's particle count");
    if (need_bstart && !p->bucket_start) return fail(c, APIC_EINVAL, "bucket_start is NULL");
    if (c->n == 0) return APIC_OK;   // an empty plasma: no particle array is read
    const int dim = c->d.dim, vdim = c->d.vdim;
    if (c->mixed) {
        if (!p->cell || !p->ox || (dim >= 2 && !p->oy) || (dim == 3 && !p->oz))
            return fail(c, APIC_EINVAL, "mixed path needs cell, ox (and oy in 2D and 3D, oz in 3D)");
    } else {
        if (!p->x || (dim >= 2 && !p->y) || (dim == 3 && !p->z))
            return fail(c, APIC_EINVAL, "FP64 path needs x (and y in 2D and 3D, z in 3D)");
    }
    if (!p->vx || (vdim >= 2 && !p->vy) || (vdim >= 3 && !p->vz))
        return fail(c, APIC_EINVAL, "missing velocity component");
    if (need_bstart && !p->bucket_start) return fail(c, APIC_EINVAL, "bucket_start is NULL");
    return APIC_OK;
}

PushC push_coeffs(const apic_ctx *c, double dt_scale, int move) {
    PushC pc;
    const double dte = c->d.dt * dt_scale;
    pc.a = c->d.qm * dte * 0.5;
    pc.t = pc.a * c->d.bz;
    pc.s = 2.0 * pc.t / (1.0 + pc.t * pc.t);
    pc.af = (float)pc.a;
    pc.tf = (float)pc.t;
    pc.sf = (float)pc.s;
    pc.dt = c->d.dt;
    const double dx = c->d.lx / c->d.nx;
    const double dy = c->d.dim >= 2 ? c->d.ly / c->d.ny : 1.0;
    const double dz = c->d.dim == 3 ? c->d.lz / c->d.nz : 1.0;
    pc.dtdx = (float)(c->d.dt / dx);
    pc.dtdy = (float)(c->d.dt / dy);
    pc.dtdz = (float)(c->d.dt / dz);
    pc.dtdx2 = pc.dtdx * pc.dtdx;
    pc.dtdy2 = pc.dtdy * pc.dtdy;
    pc.move = move;
    pc.rot = c->d.bz != 0.0;
    // margin of a deep stay (cells): the next tally pass skips the deep range
    // while the field's share of a move, 2|a| max|E| dt/dx (with slack for
    // rounding), stays below it. Measured against 1/4, 1/8 and 1/16 cell: the
    // smaller margin leaves fewer shallow particles to tally (magnetized 2D3V
    // 1024^2: tally pass 30 -> 23 us) and still covers the kicks of these
    // plasmas by a wide factor; a stronger field only makes the pass read the
    // whole bucket
    pc.deep = 0.03125f;
    pc.ic2 = c->g.hc ? 1.0 / (c->d.c_light * c->d.c_light) : 0.0;
    pc.ic2f = (float)pc.ic2;
    pc.jx = -c->d.q_macro / (dy * c->d.dt);
    pc.jy = -c->d.q_macro / (dx * c->d.dt);
    pc.jz = c->d.q_macro / (dx * dy);
    return pc;
}

// Scale of the accumulation buffer to charge density.
double acc_scale(const apic_ctx *c) {
    double s = c->d.q_macro / c->dV;
    if (c->mixed) s = std::ldexp(s, -c->g.S * c->d.dim);
    return s;
}

int64_t max_per_bucket(const apic_ctx *c) {
    if (!c->mixed) return INT32_MAX;
    const int bits = 63 - c->g.S * c->d.dim - c->d.dim;
    if (bits >= 31) return INT32_MAX;
    return (int64_t(1) << bits) - 1;
}

// Field of an accumulation buffer (or of a given FP64 rho): rho -> E (and
// E32 when non-NULL). step_mode: diagnostics go to diag[step] together with
// the push-pass partials (npush buckets); otherwise we/charge are written
// directly when non-NULL.
apic_status field_from_acc(apic_ctx *c, void *acc, bool acc_is_rho, double *E, float *E32, double *diag,
                           double *we, double *charge, int npush, int clear, void *ws, hipStream_t s,
                           const int32_t *nlive) {
    const double scale = acc_is_rho ? 1.0 : acc_scale(c);
    const double add = acc_is_rho ? 0.0 : c->d.rho_ion;
    const bool mixed_acc = c->mixed && !acc_is_rho;
    const double G = (double)c->d.nx * c->d.ny * c->d.nz;
    if (c->d.dim == 1) {
        const int step_mode = diag ? 1 : 0;
        HIPCHK(c, launch_field1d(c->g, mixed_acc, acc, scale, add, c->d.rho_ion, c->d.lx / c->d.nx, clear, E, E32,
                                 diag ? diag + 1 : we, diag ? diag + 0 : charge, step_mode, c->d.q_macro, c->dev, s));
        if (diag && npush)
            HIPCHK(c, launch_finalize(npush, 0, c->mass, c->dV, G, c->d.rho_ion, diag, nullptr, nullptr, c->dev, s));
        return APIC_OK;
    }
    double *rho = wsp<double>(ws, c->o_rho);
    void *rhat = wsp<void>(ws, c->o_rhat);
    char *ehat = wsp<char>(ws, c->o_ehat);
    if (c->fused_fft) {
        // half spectra in rhat, the x-spectrum of Ex + i Ey ([ny][nx] complex) in ehat
        const FinArgs fin{diag ? npush : 0, 0, c->mass, c->dV, G, c->d.rho_ion, diag, we, charge, c->g.walls,
                          c->d.q_macro, nlive, mixed_acc ? c->g.S * c->d.dim : 0};
        HIPCHK(c, launch_fused_field(c->g, mixed_acc, acc, scale, add, clear, rhat, ehat, E, E32, c->dev.tw, fin,
                                     c->dev, s));
        return APIC_OK;
    }
    if (c->fused_fft3) {
        // phi into the rho buffer through the two spectra buffers, then E from phi
        HIPCHK(c, launch_fused_field3(c->g, mixed_acc, acc, scale, add, clear, rhat, ehat, rho, c->dev.tw,
                                      mixed_acc ? c->dev.qacc : nullptr, c->dev, s));
        const FinArgs fin{diag ? npush : 0, fused_fft3_spec_blocks(c->g), c->mass, c->dV, G, c->d.rho_ion, diag,
                          we, charge, c->g.walls, c->d.q_macro, nlive, mixed_acc ? c->g.S * c->d.dim : 0};
        HIPCHK(c, launch_grad(c->g, rho, E, E32, fin, c->dev, s));
        return APIC_OK;
    }
    if (c->g.walls)
        HIPCHK(c, launch_rho_odd(c->g, mixed_acc, acc, rho, scale, add, clear, c->dev.qacc, s));
    else
        HIPCHK(c, launch_rho(c->g, mixed_acc, acc, rho, scale, add, clear, c->dev.qacc, s));
    FFTCHK(c, hipfftSetStream(c->fwd, s));
    FFTCHK(c, hipfftExecD2Z(c->fwd, (hipfftDoubleReal *)rho, (hipfftDoubleComplex *)rhat));
    HIPCHK(c, launch_spectral(c->g, rhat, ehat, c->dev, s));
    const FinArgs fin{diag ? npush : 0, spectral_blocks(c->g), c->mass, c->dV, G, c->d.rho_ion, diag, we, charge,
                      c->g.walls, c->d.q_macro, nlive, mixed_acc ? c->g.S * c->d.dim : 0};
    // phi into the rho buffer (rho is no longer needed), then E from phi
    FFTCHK(c, hipfftSetStream(c->inv, s));
    FFTCHK(c, hipfftExecZ2D(c->inv, (hipfftDoubleComplex *)ehat, (hipfftDoubleReal *)rho));
    HIPCHK(c, launch_grad(c->g, rho, E, E32, fin, c->dev, s));
    return APIC_OK;
}

apic_status copy_parts(apic_ctx *c, const Parts &dst, const Parts &src, hipStream_t s) {
    const int64_t n = c->n;
    const size_t r = c->mixed ? 4 : 8;
    if (c->mixed) {
        HIPCHK(c, launch_copy_bytes(dst.cell, src.cell, 4 * n, s));
        HIPCHK(c, launch_copy_bytes(dst.ox, src.ox, 4 * n, s));
        if (c->d.dim >= 2) HIPCHK(c, launch_copy_bytes(dst.oy, src.oy, 4 * n, s));
        if (c->d.dim == 3) HIPCHK(c, launch_copy_bytes(dst.oz, src.oz, 4 * n, s));
    } else {
        HIPCHK(c, launch_copy_bytes(dst.x, src.x, 8 * n, s));
        if (c->d.dim >= 2) HIPCHK(c, launch_copy_bytes(dst.y, src.y, 8 * n, s));
        if (c->d.dim == 3) HIPCHK(c, launch_copy_bytes(dst.z, src.z, 8 * n, s));
    }
    HIPCHK(c, launch_copy_bytes(dst.vx, src.vx, r * n, s));
    if (c->d.vdim >= 2) HIPCHK(c, launch_copy_bytes(dst.vy, src.vy, r * n, s));
    if (c->d.vdim >= 3) HIPCHK(c, launch_copy_bytes(dst.vz, src.vz, r * n, s));
    return APIC_OK;
}

}  // namespace apic_host

extern "C" {

apic_status apic_create(const apic_grid_desc *desc, int64_t n_particles, apic_ctx **out) {
    if (!desc || !out) return APIC_EINVAL;
    *out = nullptr;
    const apic_grid_desc &d = *desc;
    if (d.dim < 1 || d.dim > 3) return APIC_EINVAL;
    if (d.dim == 1 && (d.vdim != 1 || d.ny != 1)) return APIC_EINVAL;
    if (d.dim == 2 && (d.vdim != 2 && d.vdim != 3)) return APIC_EINVAL;
    if (d.dim == 3 && d.vdim != 3) return APIC_EINVAL;
    if (d.dim < 3 && d.nz != 0 && d.nz != 1) return APIC_EINVAL;
    if (d.nx < 2 || d.ny < 1 || (d.dim == 2 && (d.ny < 2 || d.nx > 32768 || d.ny > 32768))) return APIC_EINVAL;
    if (d.dim == 3 && (d.ny < 2 || d.nz < 2 || d.nx > 1024 || d.ny > 1024 || d.nz > 1024)) return APIC_EINVAL;
    if (d.dim == 1 && d.nx > 8192) return APIC_EUNSUPPORTED;
    if (!(d.lx > 0) || (d.dim >= 2 && !(d.ly > 0)) || (d.dim == 3 && !(d.lz > 0)) || !(d.dt > 0) ||
        !std::isfinite(d.qm) || d.qm == 0.0)
        return APIC_EINVAL;
    if (d.bz != 0.0 && d.vdim < 2) return APIC_EINVAL;
    if (n_particles < 0 || n_particles > (int64_t)INT32_MAX - 1) return APIC_EINVAL;
    if (d.prec != APIC_FP64 && d.prec != APIC_MIXED) return APIC_EINVAL;
    if ((d.tile_x && !is_pow2(d.tile_x)) || (d.tile_y && !is_pow2(d.tile_y)) || (d.tile_z && !is_pow2(d.tile_z)))
        return APIC_EINVAL;
    if (d.pusher != APIC_BORIS && d.pusher != APIC_HIGUERA_CARY) return APIC_EINVAL;
    if (d.pusher == APIC_HIGUERA_CARY && (d.vdim != 3 || !(d.c_light > 0) || !std::isfinite(d.c_light)))
        return APIC_EINVAL;
    if (d.model != APIC_ELECTROSTATIC && d.model != APIC_ELECTROMAGNETIC) return APIC_EINVAL;
    if (d.walls_x != 0 && d.walls_x != 1) return APIC_EINVAL;
    if (d.walls_x) {
        if (d.dim != 2 || d.model != APIC_ELECTROSTATIC) return APIC_EUNSUPPORTED;
        if (d.nx > 16384) return APIC_EINVAL;
    }
    if (d.model == APIC_ELECTROMAGNETIC) {
        if (d.dim != 2 || d.vdim != 3 || !(d.c_light > 0) || !std::isfinite(d.c_light)) return APIC_EINVAL;
        // Courant condition of the Yee update
        const double dx = d.lx / d.nx, dy = d.ly / d.ny;
        if (!(d.c_light * d.dt * std::sqrt(1.0 / (dx * dx) + 1.0 / (dy * dy)) < 1.0)) return APIC_EINVAL;
    }

    apic_ctx *c = new (std::nothrow) apic_ctx();
    if (!c) return APIC_ENOMEM;
    c->d = d;
    c->n = n_particles;
    c->mixed = d.prec == APIC_MIXED;
    Geo &g = c->g;
    g.dim = d.dim;
    g.vdim = d.vdim;
    g.nx = d.nx;
    g.ny = d.dim >= 2 ? d.ny : 1;
    g.nz = d.dim == 3 ? d.nz : 1;
    c->d.ny = g.ny;
    c->d.nz = g.nz;
    // walls: every grid array is the odd extension along x (2 nx nodes over
    // 2 lx); particles live in the first nx cells
    g.walls = d.walls_x;
    g.nxp = d.nx;
    // the push build (APIC_PUSH_VR=0 or 1 forces the plain or the
    // register-relieved one, for comparisons; otherwise by resident workgroups)
    {
        const char *vr_env = std::getenv("APIC_PUSH_VR");
        g.push_vr = !vr_env ? 0 : (std::string(vr_env) == "1" ? 2 : (std::string(vr_env) == "0" ? 1 : 0));
    }
    if (g.walls) {
        g.nx = 2 * d.nx;
        c->d.nx = g.nx;
        c->d.lx = 2.0 * d.lx;
    }
    int tsx, tsy, tsz;
    default_tiles(d, n_particles, tsx, tsy, tsz);
    if (d.model == APIC_ELECTROMAGNETIC) {
        // 32 x 16: the six-component field tile and the current tile stay
        // within LDS, and at 1024^2, 33.5M particles it is 4% faster than
        // 16 x 16 in both precisions (32 x 32 leaves too few workgroups per CU)
        tsx = 5;
        tsy = 4;
    }
    if (d.tile_x) tsx = ilog2_floor(d.tile_x);
    if (d.dim >= 2 && d.tile_y) tsy = ilog2_floor(d.tile_y);
    if (d.dim == 3 && d.tile_z) tsz = ilog2_floor(d.tile_z);
    if (d.dim == 1) tsy = 0;
    if (d.dim < 3) tsz = 0;
    if (tsx > 10 || tsy > 10 || tsz > 10) { delete c; return APIC_EINVAL; }
    // a tile side never exceeds its axis (the tile loads wrap an index once)
    auto fit = [](int ts, int n) {
        while (ts > 0 && (1 << ts) > n) --ts;
        return ts;
    };
    tsx = fit(tsx, g.nxp);
    // walls: the wall is a tile edge (the deep classification measures the
    // distance to the tile edges)
    while (g.walls && tsx > 0 && g.nxp % (1 << tsx) != 0) --tsx;
    tsy = fit(tsy, g.ny);
    tsz = fit(tsz, g.nz);
    {
        // LDS of the fused push: E tile (dim components) + deposit region with
        // a one-cell halo; must fit one workgroup's 64 KiB
        const int64_t ex = (1 << tsx) + 1, ey = d.dim >= 2 ? (1 << tsy) + 1 : 1, ez = d.dim == 3 ? (1 << tsz) + 1 : 1;
        const int64_t e_bytes = ex * ey * ez * d.dim * (c->mixed ? 4 : 8);
        const int64_t a_bytes = (ex + 2) * (d.dim >= 2 ? ey + 2 : 1) * (d.dim == 3 ? ez + 2 : 1) * 8;
        if (e_bytes + a_bytes + 16 > 65536) { delete c; return APIC_EINVAL; }
        if (d.model == APIC_ELECTROMAGNETIC) {
            const int64_t tx = 1 << tsx, ty = 1 << tsy;
            // the field tile in the push precision, the current tile in FP64
            const int64_t em_bytes = 6 * (tx + 2) * (ty + 2) * (c->mixed ? 4 : 8) + 3 * (tx + 3) * (ty + 3) * 8;
            if (em_bytes + 32 > 65536) { delete c; return APIC_EINVAL; }
        }
    }
    g.tsx = tsx;
    g.tsy = tsy;
    g.tsz = tsz;
    g.nbx = g.walls ? g.nxp >> tsx : (g.nx + (1 << tsx) - 1) >> tsx;
    g.nby = d.dim >= 2 ? (g.ny + (1 << tsy) - 1) >> tsy : 1;
    g.nbz = d.dim == 3 ? (g.nz + (1 << tsz) - 1) >> tsz : 1;
    g.nbuckets = g.nbx * g.nby * g.nbz;
    g.halo = 1;
    g.np = (int)n_particles;
    g.hc = d.pusher == APIC_HIGUERA_CARY;
    g.em = d.model == APIC_ELECTROMAGNETIC;
    g.S = d.frac_bits ? d.frac_bits : (d.dim == 1 ? 32 : d.dim == 2 ? 20 : 15);
    if (c->mixed && (g.S < 1 || g.S > 32 || (d.dim == 2 && g.S > 23) || (d.dim == 3 && g.S > 16))) {
        delete c;
        return APIC_EINVAL;
    }
    g.lx = c->d.lx;
    g.ly = d.dim >= 2 ? d.ly : 1.0;
    g.lz = d.dim == 3 ? d.lz : 1.0;
    const double dx = d.lx / d.nx, dy = d.dim >= 2 ? d.ly / d.ny : 1.0, dz = d.dim == 3 ? d.lz / d.nz : 1.0;
    g.inv_dx = 1.0 / dx;
    g.inv_dy = 1.0 / dy;
    g.inv_dz = 1.0 / dz;
    c->dV = dx * dy * dz;
    // the neutralising macro-charge by default: n electrons carry the
    // opposite of the ion charge rho_ion V of the box (V of the physical box,
    // before the odd extension of walls)
    if (c->d.q_macro == 0.0 && n_particles > 0) {
        const double vol = d.lx * (d.dim >= 2 ? d.ly : 1.0) * (d.dim == 3 ? d.lz : 1.0);
        c->d.q_macro = -d.rho_ion * vol / (double)n_particles;
    }
    if (!std::isfinite(c->d.q_macro)) { delete c; return APIC_EINVAL; }
    c->mass = c->d.q_macro / d.qm;
    layout(c);

    // context device words + wavenumber tables
    const int hx = g.nx / 2 + 1;
    // the fused field solve (unless APIC_FIELD_FFT=library asks for the
    // library transforms, for comparison)
    const char *fft_env = std::getenv("APIC_FIELD_FFT");
    const bool lib_fft = fft_env && std::string(fft_env) == "library";
    c->fused_fft = fused_fft_supported(d.dim, g.nx, g.ny, g.nz) && !lib_fft;
    c->fused_fft3 = fused_fft3_supported(d.dim, g.nx, g.ny, g.nz) && !lib_fft;
    const int nmax = std::max(g.nx, std::max(g.ny, d.dim == 3 ? g.nz : 1));
    const size_t tw_bytes = (c->fused_fft || c->fused_fft3) ? 2 * sizeof(double) * nmax : 0;   // nmax complex
    size_t bytes = align256(sizeof(int)) * 2 + align256(sizeof(double) * 2 * g.nbuckets) +
                   align256(sizeof(double) * kMaxSpecBlocks) + align256(sizeof(double)) +
                   align256(sizeof(double) * hx) * 2 + align256(sizeof(double) * g.ny) * 2 +
                   align256(sizeof(double) * g.nz) * 2 + align256(tw_bytes) +
                   align256(((size_t)kQSlots * kQStride + 2) * sizeof(int64_t));
    if (hipMalloc(&c->dev_block, bytes) != hipSuccess) { delete c; return APIC_ENOMEM; }
    if (hipMemset(c->dev_block, 0, bytes) != hipSuccess) { (void)hipFree(c->dev_block); delete c; return APIC_EHIP; }
    char *b = (char *)c->dev_block;
    size_t off = 0;
    auto take = [&](size_t sz) { char *p = b + off; off += align256(sz); return p; };
    c->dev.err = (int *)take(sizeof(int));
    c->dev.step = (int *)take(sizeof(int));
    c->dev.part_push = (double *)take(sizeof(double) * 2 * g.nbuckets);
    c->dev.part_spec = (double *)take(sizeof(double) * kMaxSpecBlocks);
    c->dev.rho0 = (double *)take(sizeof(double));
    c->dev.kx2 = (double *)take(sizeof(double) * hx);
    c->dev.kapx = (double *)take(sizeof(double) * hx);
    c->dev.ky2 = (double *)take(sizeof(double) * g.ny);
    c->dev.kapy = (double *)take(sizeof(double) * g.ny);
    c->dev.kz2 = (double *)take(sizeof(double) * g.nz);
    c->dev.kapz = (double *)take(sizeof(double) * g.nz);
    c->dev.tw = tw_bytes ? (double *)take(tw_bytes) : nullptr;
    {
        int64_t *q = (int64_t *)take(((size_t)kQSlots * kQStride + 2) * sizeof(int64_t));
        c->dev.qacc = (unsigned long long *)q;
        c->dev.qexact = q + (size_t)kQSlots * kQStride;
    }
    // modified wavenumbers of the periodic FD operators:
    //   K^2_d = (2/d sin(k d / 2))^2 (3-point second difference),
    //   kappa_d = sin(k d)/d (centred first difference), k = 2 pi m / L.
    std::vector<double> kx2(hx), kapx(hx), ky2(g.ny), kapy(g.ny), kz2(g.nz), kapz(g.nz);
    for (int m = 0; m < hx; ++m) {
        double h = M_PI * m / g.nx;  // k dx / 2
        kx2[m] = std::pow(2.0 / dx * std::sin(h), 2);
        kapx[m] = std::sin(2.0 * h) / dx;
    }
    for (int m = 0; m < g.ny; ++m) {
        int mm = (m <= g.ny / 2) ? m : m - g.ny;
        double h = M_PI * mm / g.ny;
        ky2[m] = std::pow(2.0 / dy * std::sin(h), 2);
        kapy[m] = std::sin(2.0 * h) / dy;
    }
    for (int m = 0; m < g.nz; ++m) {
        int mm = (m <= g.nz / 2) ? m : m - g.nz;
        double h = M_PI * mm / g.nz;
        kz2[m] = std::pow(2.0 / dz * std::sin(h), 2);
        kapz[m] = std::sin(2.0 * h) / dz;
    }
    if (d.dim == 1) { ky2[0] = 0.0; kapy[0] = 0.0; }
    if (d.dim < 3) { kz2[0] = 0.0; kapz[0] = 0.0; }
    bool copied = hipMemcpy(c->dev.kx2, kx2.data(), sizeof(double) * hx, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(c->dev.kapx, kapx.data(), sizeof(double) * hx, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(c->dev.ky2, ky2.data(), sizeof(double) * g.ny, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(c->dev.kapy, kapy.data(), sizeof(double) * g.ny, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(c->dev.kz2, kz2.data(), sizeof(double) * g.nz, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(c->dev.kapz, kapz.data(), sizeof(double) * g.nz, hipMemcpyHostToDevice) == hipSuccess;
    if (copied && tw_bytes) {
        // exp(-2 pi i k / nmax), k < nmax; the angle 2 pi k / nmax is one rounding of pi times an exact ratio
        std::vector<double> tw(2 * nmax);
        for (int k = 0; k < nmax; ++k) {
            const double ang = M_PI * (2.0 * k / nmax);
            tw[2 * k] = std::cos(ang);
            tw[2 * k + 1] = -std::sin(ang);
        }
        copied = hipMemcpy(c->dev.tw, tw.data(), tw_bytes, hipMemcpyHostToDevice) == hipSuccess;
    }
    if (!copied) {
        (void)hipFree(c->dev_block);
        delete c;
        return APIC_EHIP;
    }
    if (d.dim == 2) {
        if (hipfftPlan2d(&c->fwd, g.ny, g.nx, HIPFFT_D2Z) != HIPFFT_SUCCESS ||
            hipfftPlan2d(&c->inv, g.ny, g.nx, HIPFFT_Z2D) != HIPFFT_SUCCESS) {
            (void)hipFree(c->dev_block);
            delete c;
            return APIC_EHIP;
        }
        c->have_fft = true;
    } else if (d.dim == 3) {
        if (hipfftPlan3d(&c->fwd, g.nz, g.ny, g.nx, HIPFFT_D2Z) != HIPFFT_SUCCESS ||
            hipfftPlan3d(&c->inv, g.nz, g.ny, g.nx, HIPFFT_Z2D) != HIPFFT_SUCCESS) {
            (void)hipFree(c->dev_block);
            delete c;
            return APIC_EHIP;
        }
        c->have_fft = true;
    }
    *out = c;
    return APIC_OK;
}

void apic_destroy(apic_ctx *c) {
    if (!c) return;
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    if (c->have_fft) {
        hipfftDestroy(c->fwd);
        hipfftDestroy(c->inv);
    }
    if (c->dev_block) (void)hipFree(c->dev_block);
    delete c;
}

apic_status apic_workspace_size(const apic_ctx *c, size_t *bytes) {
    if (!c || !bytes) return APIC_EINVAL;
    *bytes = c->ws_bytes;
    return APIC_OK;
}

int64_t apic_num_buckets(const apic_ctx *c) { return c ? c->g.nbuckets : -1; }

int apic_frac_bits(const apic_ctx *c) { return c ? c->g.S : -1; }

double apic_q_macro(const apic_ctx *c) { return c ? c->d.q_macro : NAN; }

int apic_tile_size(const apic_ctx *c, int axis) {
    if (!c || axis < 0 || axis > 2) return -1;
    if (axis >= c->d.dim) return 1;
    return 1 << (axis == 0 ? c->g.tsx : axis == 1 ? c->g.tsy : c->g.tsz);
}

const char *apic_last_error(const apic_ctx *c) { return c ? c->err.c_str() : "null context"; }

apic_status apic_sort_by_cell(apic_ctx *c, apic_particles *p, void *ws, void *stream) {
    if (!c) return APIC_EINVAL;
    apic_status st = check_parts(c, p, true);
    if (st != APIC_OK) return st;
    if (!ws) return fail(c, APIC_EINVAL, "workspace is NULL");
    hipStream_t s = (hipStream_t)stream;
    const int nb = c->g.nbuckets;
    int32_t *k0 = wsp<int32_t>(ws, c->o_keys), *k1 = wsp<int32_t>(ws, c->o_keys2);
    int32_t *i0 = wsp<int32_t>(ws, c->o_idx), *i1 = wsp<int32_t>(ws, c->o_idx2);
    Parts src = parts_of(p), tmp = parts_ws(c, ws);
    // stable order by key
    HIPCHK(c, launch_keys_init(c->g, c->mixed, src, c->n, k0, i0, c->dev, s));
    int bits = 1;
    while ((1ll << bits) < (int64_t)nb) ++bits;
    for (int shift = 0; shift < bits; shift += 8) {
        HIPCHK(c, launch_radix_pass(k0, i0, k1, i1, c->n, shift, wsp<int32_t>(ws, c->o_rcnt),
                                    wsp<int32_t>(ws, c->o_roff), wsp<int32_t>(ws, c->o_rpart), c->dev, s));
        std::swap(k0, k1);
        std::swap(i0, i1);
    }
    // bucket table from the sorted keys
    HIPCHK(c, launch_bucket_table(k0, c->n, nb, p->bucket_start, max_per_bucket(c), c->dev, s));
    HIPCHK(c, launch_gather_parts(c->g, c->mixed, src, tmp, c->n, i0, p->perm, c->dev, s));
    return copy_parts(c, src, tmp, s);
}

apic_status apic_deposit(apic_ctx *c, const apic_particles *p, void *rho, void *stream) {
    if (!c) return APIC_EINVAL;
    apic_status st = check_parts(c, p, false);
    if (st != APIC_OK) return st;
    if (!rho) return fail(c, APIC_EINVAL, "rho is NULL");
    hipStream_t s = (hipStream_t)stream;
    const int64_t G = (int64_t)c->d.nx * c->d.ny * c->d.nz;
    HIPCHK(c, launch_fill_u64((uint64_t *)rho, G, 0, s));
    HIPCHK(c, launch_deposit(c->g, c->mixed, parts_of(p), c->n, p->bucket_start, rho, c->dev, s));
    if (!c->mixed) HIPCHK(c, launch_rho(c->g, false, rho, (double *)rho, acc_scale(c), c->d.rho_ion, 0, nullptr, s));
    return APIC_OK;
}

apic_status apic_field_solve(apic_ctx *c, const void *rho, double *E, float *E32, double *we, void *ws,
                             void *stream) {
    if (!c) return APIC_EINVAL;
    if (c->g.em) return fail(c, APIC_EUNSUPPORTED, "electromagnetic context: use apic_em_init_fields");
    if (!rho || !E || !ws) return fail(c, APIC_EINVAL, "rho, E and workspace are required");
    hipStream_t s = (hipStream_t)stream;
    // FP64 input already is rho; mixed input is the fixed-point node sums.
    return field_from_acc(c, const_cast<void *>(rho), !c->mixed, E, E32, nullptr, we, nullptr, 0, 0, ws, s);
}

apic_status apic_gather_push(apic_ctx *c, apic_particles *p, const void *E, double dt_scale, int move,
                             void *stream) {
    if (!c) return APIC_EINVAL;
    if (c->g.em) return fail(c, APIC_EUNSUPPORTED, "electromagnetic context: use apic_em_gather_push");
    apic_status st = check_parts(c, p, false);
    if (st != APIC_OK) return st;
    if (!E) return fail(c, APIC_EINVAL, "E is NULL");
    if (!std::isfinite(dt_scale)) return fail(c, APIC_EINVAL, "dt_scale is not finite");
    hipStream_t s = (hipStream_t)stream;
    PushC pc = push_coeffs(c, dt_scale, move);
    HIPCHK(c, launch_gather_push(c->g, c->mixed, parts_of(p), c->n, p->bucket_start, E, pc, c->dev, s));
    return APIC_OK;
}

}  // extern "C"

namespace apic_host {

// nsteps cycles alternating between the particle buffers A (p, holding the
// state on entry) and B with its bucket table bsB; after an odd count the
// state is in B, and copy_back moves it to p.
apic_status step_run(apic_ctx *c, apic_particles *p, const Parts &B, int32_t *bsB, bool copy_back, void *rho,
                     double *E, float *E32, int nsteps, double *diag, void *ws, hipStream_t s) {
    apic_status st = APIC_OK;
    const int nb = c->g.nbuckets;
    const int64_t G = (int64_t)c->d.nx * c->d.ny * c->d.nz;
    int32_t *cnt = wsp<int32_t>(ws, c->o_cnt);
    int32_t *offs = wsp<int32_t>(ws, c->o_offs);
    int32_t *farcnt = wsp<int32_t>(ws, c->o_farcnt);
    int32_t *tot = wsp<int32_t>(ws, c->o_tot);
    int32_t *deep = wsp<int32_t>(ws, c->o_deep);
    void *acc = wsp<void>(ws, c->o_acc);
    const Parts A = parts_of(p);
    int32_t *bsA = p->bucket_start;
    const PushC pc = push_coeffs(c, 1.0, 1);
    // binary32 E between the steps of the mixed path (2D and 3D)
    float *e32 = c->o_e32 != (size_t)-1 ? wsp<float>(ws, c->o_e32) : nullptr;
    HIPCHK(c, launch_fill_i32(farcnt, nb, 0, s));
    // the bucket totals: two buffers, alternating by step
    HIPCHK(c, launch_fill_i32(tot, 2 * (int64_t)nb, 0, s));
    // no deep ranges known for the incoming order: the first count reads all
    HIPCHK(c, launch_fill_i32(deep, (int64_t)nb * kDeepTab, 0, s));
    HIPCHK(c, launch_fill_u64((uint64_t *)acc, G, 0, s));
    HIPCHK(c, launch_set_step(c->dev.step, -1, s));
    for (int k = 0; k < nsteps; ++k) {
        const bool even = (k & 1) == 0;
        const Parts &src = even ? A : B;
        const Parts &dst = even ? B : A;
        int32_t *bs_src = even ? bsA : bsB;
        int32_t *bs_dst = even ? bsB : bsA;
        const bool last = k == nsteps - 1;
        hipEvent_t *ev = nullptr;
        if (c->prof_used < c->prof_max && c->prof_step++ % c->prof_every == 0) ev = &c->ev[5 * (size_t)c->prof_used++];
        if (ev && c->prof_all) HIPCHK(c, hipEventRecord(ev[0], s));
        int32_t *tot_k = tot + (even ? 0 : nb), *tot_n = tot + (even ? nb : 0);
        HIPCHK(c, launch_step_count(c->g, c->mixed, src, bs_src, E, k > 0 ? e32 : nullptr, pc, cnt, tot_k, farcnt,
                                    deep, c->dev, s));
        if (ev && c->prof_all) HIPCHK(c, hipEventRecord(ev[1], s));
        if (fused_scan_offsets(c->g)) {
            HIPCHK(c, launch_scan_offsets(c->g, tot_k, tot_n, bs_dst, c->n, max_per_bucket(c), 1, cnt, offs, c->dev,
                                          s));
        } else {
            HIPCHK(c, launch_scan_dir(c->g, tot_k, bs_dst, c->n, max_per_bucket(c), 1, c->dev, s));
            HIPCHK(c, launch_dest_offsets(c->g, cnt, bs_dst, offs, s));
        }
        if (ev) HIPCHK(c, hipEventRecord(ev[2], s));
        HIPCHK(c, launch_step_push(c->g, c->mixed, src, dst, bs_src, bs_dst, cnt, offs, farcnt, E,
                                   k > 0 ? e32 : nullptr, pc, acc, p->perm, diag ? c->dev.part_push : nullptr, deep,
                                   c->dev, s));
        if (ev) HIPCHK(c, hipEventRecord(ev[3], s));
        if (rho && last) {
            if (c->mixed)
                HIPCHK(c, launch_copy_bytes(rho, acc, 8 * G, s));
            else
                HIPCHK(c, launch_rho(c->g, false, acc, (double *)rho, acc_scale(c), c->d.rho_ion, 0, nullptr, s));
        }
        // mixed path: between steps only the binary32 field (the push reads no
        // more); the FP64 E (and the caller's E32) after the last step
        st = field_from_acc(c, acc, false, (last || !e32) ? E : nullptr, last ? E32 : e32, diag, nullptr, nullptr,
                            diag ? nb : 0, 1, ws, s, bs_dst + nb);
        if (st != APIC_OK) return st;
        if (ev && c->prof_all) HIPCHK(c, hipEventRecord(ev[4], s));
    }
    if ((nsteps & 1) && copy_back) {
        st = copy_parts(c, A, B, s);
        if (st != APIC_OK) return st;
        HIPCHK(c, launch_copy_bytes(bsA, bsB, 4 * (int64_t)(nb + 1), s));
    }
    return APIC_OK;
}

}  // namespace apic_host

extern "C" {

apic_status apic_step(apic_ctx *c, apic_particles *p, void *rho, double *E, float *E32, int nsteps, double *diag,
                      void *ws, void *stream) {
    if (!c) return APIC_EINVAL;
    if (c->g.em) return fail(c, APIC_EUNSUPPORTED, "electromagnetic context: use apic_em_step");
    apic_status st = check_parts(c, p, true);
    if (st != APIC_OK) return st;
    if (!E || !ws || nsteps < 0) return fail(c, APIC_EINVAL, "E, workspace and nsteps >= 0 are required");
    if (nsteps == 0) return APIC_OK;
    return step_run(c, p, parts_ws(c, ws), wsp<int32_t>(ws, c->o_bstart), true, rho, E, E32, nsteps, diag, ws,
                    (hipStream_t)stream);
}

apic_status apic_step_pair(apic_ctx *c, apic_particles *p, apic_particles *q, void *rho, double *E, float *E32,
                           int nsteps, double *diag, int *in_q, void *ws, void *stream) {
    if (!c) return APIC_EINVAL;
    if (c->g.em) return fail(c, APIC_EUNSUPPORTED, "electromagnetic context: use apic_em_step");
    apic_status st = check_parts(c, p, true);
    if (st != APIC_OK) return st;
    st = check_parts(c, q, true);
    if (st != APIC_OK) return st;
    if (!E || !ws || !in_q || nsteps < 0)
        return fail(c, APIC_EINVAL, "E, workspace, in_q and nsteps >= 0 are required");
    if (c->n > 0 && (p->vx == q->vx || p->bucket_start == q->bucket_start))
        return fail(c, APIC_EINVAL, "the two particle buffers must not share arrays");
    *in_q = nsteps & 1;
    if (nsteps == 0) return APIC_OK;
    return step_run(c, p, parts_of(q), q->bucket_start, false, rho, E, E32, nsteps, diag, ws, (hipStream_t)stream);
}

apic_status apic_step_static(apic_ctx *c, apic_particles *p, void *rho, double *E, float *E32, int nsteps,
                             double *diag, void *stream) {
    if (!c) return APIC_EINVAL;
    if (c->ws_bytes > APIC_STATIC_WS_BYTES) {
        c->err = "apic_step_static: the context needs " + std::to_string(c->ws_bytes) +
                 " bytes of workspace, above the fixed array's " + std::to_string((size_t)APIC_STATIC_WS_BYTES);
        return APIC_EINVAL;
    }
    if (c->d.dim >= 2 && !c->fused_fft)
        return fail(c, APIC_EUNSUPPORTED,
                    "apic_step_static: the field solve of this grid uses the FFT library (3D, or 2D sides that "
                    "are not powers of two up to 1024)");
    void *ws = nullptr;
    HIPCHK(c, scratch_address(&ws));
    return apic_step(c, p, rho, E, E32, nsteps, diag, ws, stream);
}

apic_status apic_profile_enable(apic_ctx *c, int max_steps) {
    if (!c || max_steps < 0) return APIC_EINVAL;
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    c->ev.clear();
    c->prof_max = c->prof_used = 0;
    c->prof_step = 0;
    if (max_steps == 0) return APIC_OK;
    c->ev.resize(5 * (size_t)max_steps);
    for (auto &e : c->ev) HIPCHK(c, hipEventCreate(&e));
    c->prof_max = max_steps;
    return APIC_OK;
}

apic_status apic_profile_phases(apic_ctx *c, int all) {
    if (!c) return APIC_EINVAL;
    c->prof_all = all != 0;
    c->prof_used = 0;
    c->prof_step = 0;
    return APIC_OK;
}

apic_status apic_profile_every(apic_ctx *c, int every) {
    if (!c || every < 1) return APIC_EINVAL;
    c->prof_every = every;
    c->prof_used = 0;
    c->prof_step = 0;
    return APIC_OK;
}

apic_status apic_profile_read(apic_ctx *c, double ms[4], int *steps) {
    if (!c || !ms || !steps) return APIC_EINVAL;
    for (int k = 0; k < 4; ++k) ms[k] = 0.0;
    *steps = c->prof_used;
    c->prof_step = 0;
    if (c->prof_used == 0) return APIC_OK;
    HIPCHK(c, hipEventSynchronize(c->ev[5 * (size_t)(c->prof_used - 1) + (c->prof_all ? 4 : 3)]));
    for (int st = 0; st < c->prof_used; ++st) {
        for (int k = c->prof_all ? 0 : 2; k < (c->prof_all ? 4 : 3); ++k) {
            float t = 0.0f;
            HIPCHK(c, hipEventElapsedTime(&t, c->ev[5 * (size_t)st + k], c->ev[5 * (size_t)st + k + 1]));
            ms[k] += t;
        }
    }
    c->prof_used = 0;
    return APIC_OK;
}

apic_status apic_charge_exact(apic_ctx *c, int64_t *whole, int64_t *frac, void *stream) {
    if (!c || !whole || !frac) return APIC_EINVAL;
    if (!c->mixed) return fail(c, APIC_EUNSUPPORTED, "the exact charge is a mixed-path (fixed-point) figure");
    HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
    int64_t q[2];
    HIPCHK(c, hipMemcpy(q, c->dev.qexact, sizeof(q), hipMemcpyDeviceToHost));
    *whole = q[0];
    *frac = q[1];
    return APIC_OK;
}

apic_status apic_sync_status(apic_ctx *c, void *stream) {
    if (!c) return APIC_EINVAL;
    HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
    int bits = 0;
    HIPCHK(c, hipMemcpy(&bits, c->dev.err, sizeof(int), hipMemcpyDeviceToHost));
    if (bits == 0) return APIC_OK;
    int zero = 0;
    HIPCHK(c, hipMemcpy(c->dev.err, &zero, sizeof(int), hipMemcpyHostToDevice));
    if (bits & ERR_OVERFLOW)
        return fail(c, APIC_EOVERFLOW, "fixed-point deposit headroom exceeded (too many particles per bucket)");
    if (bits & ERR_COUNT) return fail(c, APIC_EDOMAIN, "bucket totals differ from particle count");
    if (bits & ERR_ORDER)
        return fail(c, APIC_EDOMAIN, "particles not ordered as bucket_start says, or a slot overflowed");
    return fail(c, APIC_EDOMAIN, "non-finite or out-of-range particle coordinate");
}

}  // extern "C"
