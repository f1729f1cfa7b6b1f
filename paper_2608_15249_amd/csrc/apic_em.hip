// Electromagnetic step (2D3V, periodic Yee grid): the field kernels of
// the finite-difference time-domain update (E_Maxwell, Yee 1966), the
// initial field, the standalone gather + Boris, and the C-ABI entry points
// apic_em_init_fields, apic_em_gather_push and apic_em_step. The particle
// pass of the step is the fused count/push pair of apic_kernels.hip in its
// electromagnetic form (staggered gather, Boris in the gathered B,
// Esirkepov current deposit), on the same sorted, tiled particle layout.
//
// Cycle (normalised units eps0 = 1, mu0 = 1/c^2): gather E^n, B^n at x^n;
// Boris v^{n-1/2} -> v^{n+1/2}; move; J^{n+1/2} of the move; then
// B^{n+1/2} = B^n - dt/2 curl E^n, E^{n+1} = E^n + dt (c^2 curl B^{n+1/2} -
// J^{n+1/2}), B^{n+1} = B^{n+1/2} - dt/2 curl E^{n+1}.
#include "apic.h"
#include "apic_ctx.h"
#include "apic_em.h"
#include "apic_fill.h"

#include <cmath>

using namespace apic;
using namespace apic_host;

namespace apic {
namespace {

constexpr int kEmStepBlocks = 2048;  // most workgroups (and partials per energy) of the one-launch field update

__device__ __forceinline__ int wrap_up(int i, int n) { return i + 1 == n ? 0 : i + 1; }
__device__ __forceinline__ int wrap_dn(int i, int n) { return i == 0 ? n - 1 : i - 1; }

__global__ void __launch_bounds__(kBlock) k_em_init(Geo g, const double *phi, double bz, double *F) {
    const int64_t G = (int64_t)g.nx * g.ny;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < G; i += (int64_t)gridDim.x * blockDim.x) {
        const int ix = (int)(i % g.nx), iy = (int)(i / g.nx);
        const double p = phi[i];
        F[i] = -(phi[(int64_t)iy * g.nx + wrap_up(ix, g.nx)] - p) * g.inv_dx;
        F[G + i] = -(phi[(int64_t)wrap_up(iy, g.ny) * g.nx + ix] - p) * g.inv_dy;
        F[2 * G + i] = 0.0;
        F[3 * G + i] = 0.0;
        F[4 * G + i] = 0.0;
        F[5 * G + i] = bz;
    }
}

// The whole field update of one step in one launch, tile by tile (32 x 8
// nodes, one per thread): B^{n+1/2}, E^{n+1} and B^{n+1} with the operations
// of the three kernels above, in the same order, so the results are the same
// bits. A tile stages E^n from one node below its first to two beyond its
// last along each axis and B^n from one below to one beyond (the second B
// half step needs E^{n+1} one node beyond the tile, that needs B^{n+1/2} one
// node below, and that needs E^n one node beyond), computes the intermediate
// values over that halo, and writes its own nodes of E^{n+1} and B^{n+1} to
// Fn. The step reads F and J and writes Fn: neighbouring tiles
// read F while this one writes, so the caller alternates two field buffers,
// and J is only read here; Jnext (the current buffer of the next step) is
// cleared instead. With diag, per-block partials of sum |E^{n+1}|^2 and
// sum |B^{n+1} - B0|^2 over the tiles the block owns.
constexpr int kFTX = 32, kFTY = 8;
static_assert(kFTX * kFTY == kBlock, "one node per thread");

template <bool DIAG>
__global__ void __launch_bounds__(kBlock) k_fdtd_step(Geo g, const double *F, double *Fn, const double *J,
                                                      double *Jnext, double *Jout, double dt, double c2, double bz,
                                                      double *part) {
    __shared__ double sE[3][kFTY + 3][kFTX + 3];   // E^n from node (x0 - 1, y0 - 1)
    __shared__ double sB[3][kFTY + 2][kFTX + 2];   // B^n, then B^{n+1/2}, from (x0 - 1, y0 - 1)
    __shared__ double sN[3][kFTY + 1][kFTX + 1];   // E^{n+1} from (x0, y0)
    static_assert(3 * (kFTY + 1) * (kFTX + 1) >= kBlock, "sN takes the staging entries past sE and sB");
    const int nx = g.nx, ny = g.ny;
    const int64_t G = (int64_t)nx * ny;
    const double h = 0.5 * dt;
    const int ntx = (nx + kFTX - 1) / kFTX, nty = (ny + kFTY - 1) / kFTY;
    const int lx0 = threadIdx.x % kFTX, ly0 = threadIdx.x / kFTX;
    // periodic node index (the halo can reach more than one period on grids
    // narrower than a tile)
    auto wrapx = [nx](int x) {
        const int r = x % nx;
        return r < 0 ? r + nx : r;
    };
    auto wrapy = [ny](int y) {
        const int r = y % ny;
        return r < 0 ? r + ny : r;
    };
    double we = 0.0, wb = 0.0;
    for (int t = blockIdx.x; t < ntx * nty; t += gridDim.x) {
        const int x0 = (t % ntx) * kFTX, y0 = (t / ntx) * kFTY;
        // E^n and B^n staged in one round of loads (entries past both go to
        // sN, which is written only after the next two barriers)
        constexpr int nE = 3 * (kFTY + 3) * (kFTX + 3), nB = 3 * (kFTY + 2) * (kFTX + 2);
        fill_batched<double, (nE + nB + kBlock - 1) / kBlock>(
            nE + nB,
            [&](int k) {
                const bool e = k < nE;
                const int kk = e ? k : k - nE;
                const int ce = kk / ((kFTY + 3) * (kFTX + 3)), re = kk % ((kFTY + 3) * (kFTX + 3));
                const int cb = kk / ((kFTY + 2) * (kFTX + 2)), rb = kk % ((kFTY + 2) * (kFTX + 2));
                const int c = e ? ce : 3 + cb;
                const int ly = e ? re / (kFTX + 3) : rb / (kFTX + 2), lx = e ? re % (kFTX + 3) : rb % (kFTX + 2);
                return F[c * G + (int64_t)wrapy(y0 - 1 + ly) * nx + wrapx(x0 - 1 + lx)];
            },
            [&](int k, double v) {
                *(k < nE ? &sE[0][0][0] + k : (k < nE + nB ? &sB[0][0][0] + (k - nE) : &sN[0][0][0] + threadIdx.x)) = v;
            });
        __syncthreads();
        // B^{n+1/2} over the staged B nodes (forward differences of E^n)
        for (int k = threadIdx.x; k < (kFTY + 2) * (kFTX + 2); k += blockDim.x) {
            const int ly = k / (kFTX + 2), lx = k % (kFTX + 2);
            const double ex = sE[0][ly][lx], ey = sE[1][ly][lx], ez = sE[2][ly][lx];
            const double bx = sB[0][ly][lx] - h * ((sE[2][ly + 1][lx] - ez) * g.inv_dy);
            const double by = sB[1][ly][lx] + h * ((sE[2][ly][lx + 1] - ez) * g.inv_dx);
            const double bzn =
                sB[2][ly][lx] - h * ((sE[1][ly][lx + 1] - ey) * g.inv_dx - (sE[0][ly + 1][lx] - ex) * g.inv_dy);
            sB[0][ly][lx] = bx;
            sB[1][ly][lx] = by;
            sB[2][ly][lx] = bzn;
        }
        __syncthreads();
        // E^{n+1} over the tile and one node beyond (backward differences of B^{n+1/2})
        for (int k = threadIdx.x; k < (kFTY + 1) * (kFTX + 1); k += blockDim.x) {
            const int ey_ = k / (kFTX + 1), ex_ = k % (kFTX + 1);
            const int64_t gi = (int64_t)wrapy(y0 + ey_) * nx + wrapx(x0 + ex_);
            const double jx = J[gi], jy = J[G + gi], jz = J[2 * G + gi];
            const double bzc = sB[2][ey_ + 1][ex_ + 1], byc = sB[1][ey_ + 1][ex_ + 1], bxc = sB[0][ey_ + 1][ex_ + 1];
            sN[0][ey_][ex_] = sE[0][ey_ + 1][ex_ + 1] + dt * (c2 * ((bzc - sB[2][ey_][ex_ + 1]) * g.inv_dy) - jx);
            sN[1][ey_][ex_] = sE[1][ey_ + 1][ex_ + 1] + dt * (-c2 * ((bzc - sB[2][ey_ + 1][ex_]) * g.inv_dx) - jy);
            sN[2][ey_][ex_] = sE[2][ey_ + 1][ex_ + 1] +
                              dt * (c2 * ((byc - sB[1][ey_ + 1][ex_]) * g.inv_dx - (bxc - sB[0][ey_][ex_ + 1]) * g.inv_dy) -
                                    jz);
        }
        __syncthreads();
        // B^{n+1} and the writes of this tile's own nodes
        {
            const int gx = x0 + lx0, gy = y0 + ly0;
            if (gx < nx && gy < ny) {
                const int64_t gi = (int64_t)gy * nx + gx;
                const double ex = sN[0][ly0][lx0], ey = sN[1][ly0][lx0], ez = sN[2][ly0][lx0];
                const double bx = sB[0][ly0 + 1][lx0 + 1] - h * ((sN[2][ly0 + 1][lx0] - ez) * g.inv_dy);
                const double by = sB[1][ly0 + 1][lx0 + 1] + h * ((sN[2][ly0][lx0 + 1] - ez) * g.inv_dx);
                const double bzn = sB[2][ly0 + 1][lx0 + 1] -
                                   h * ((sN[1][ly0][lx0 + 1] - ey) * g.inv_dx - (sN[0][ly0 + 1][lx0] - ex) * g.inv_dy);
                Fn[gi] = ex;
                Fn[G + gi] = ey;
                Fn[2 * G + gi] = ez;
                Fn[3 * G + gi] = bx;
                Fn[4 * G + gi] = by;
                Fn[5 * G + gi] = bzn;
                if (Jout) {
                    Jout[gi] = J[gi];
                    Jout[G + gi] = J[G + gi];
                    Jout[2 * G + gi] = J[2 * G + gi];
                }
                Jnext[gi] = 0.0;
                Jnext[G + gi] = 0.0;
                Jnext[2 * G + gi] = 0.0;
                if constexpr (DIAG) {
                    we += (ex * ex + ey * ey) + ez * ez;
                    wb += (bx * bx + by * by) + (bzn - bz) * (bzn - bz);
                }
            }
        }
        __syncthreads();
    }
    if constexpr (DIAG) {
        __shared__ double sRed[kWaves];
        const double a = block_sum(we, sRed), b = block_sum(wb, sRed);
        if (threadIdx.x == 0) {
            part[blockIdx.x] = a;
            part[kEmStepBlocks + blockIdx.x] = b;
        }
    }
}

// diag[step] = (W_B, W_E, kinetic, momentum) from fixed-order sums of the
// field partials and the push partials.
__global__ void __launch_bounds__(1024) k_em_finalize(int nblk, int half, int npush, double c2, double dV,
                                                      double mass, double *diag, CtxDev c) {
    __shared__ double sRed[16];
    double we = 0.0, wb = 0.0, k = 0.0, p = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
        we += c.part_spec[i];
        wb += c.part_spec[half + i];
    }
    for (int i = threadIdx.x; i < npush; i += blockDim.x) {
        k += c.part_push[2 * i];
        p += c.part_push[2 * i + 1];
    }
    we = block_sum(we, sRed);
    wb = block_sum(wb, sRed);
    k = block_sum(k, sRed);
    p = block_sum(p, sRed);
    if (threadIdx.x == 0) {
        double *d = step_slot(diag, c);
        d[0] = 0.5 * c2 * dV * wb;
        d[1] = 0.5 * dV * we;
        d[2] = 0.5 * mass * k;
        d[3] = mass * p;
    }
}

// E, B at a particle from the global field: the tile gather's arithmetic with
// global (periodic) node indices (node values converted to R first, as the
// tile holds them).
template <typename R>
__device__ __forceinline__ R lerp_glob(const double *f, const Geo &g, int i, int j, R fx, R fy) {
    const int ip = wrap_up(i, g.nx), jp = wrap_up(j, g.ny);
    const int64_t r0 = (int64_t)j * g.nx, r1 = (int64_t)jp * g.nx;
    const R f00 = (R)f[r0 + i], f10 = (R)f[r0 + ip], f01 = (R)f[r1 + i], f11 = (R)f[r1 + ip];
    const R lo = fma(fx, f10 - f00, f00), hi = fma(fx, f11 - f01, f01);
    return fma(fy, hi - lo, lo);
}

template <bool MIX, bool HC>
__global__ void __launch_bounds__(kBlock) k_em_gather_push(Geo g, Parts p, int64_t n, const double *F, PushC pc,
                                                           CtxDev c) {
    using R = typename Pt<MIX>::R;
    const int64_t G = (int64_t)g.nx * g.ny;
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        Pt<MIX> q;
        bool ok = load_pt<MIX, 2, 3>(p, i, g, q);
        const bool hx = q.fx >= R(0.5), hy = q.fy >= R(0.5);
        const int ax1 = hx ? q.ix : wrap_dn(q.ix, g.nx), ay1 = hy ? q.iy : wrap_dn(q.iy, g.ny);
        const R fx1 = hx ? q.fx - R(0.5) : q.fx + R(0.5), fy1 = hy ? q.fy - R(0.5) : q.fy + R(0.5);
        R e[3], b[3];
        e[0] = lerp_glob<R>(F, g, ax1, q.iy, fx1, q.fy);
        e[1] = lerp_glob<R>(F + G, g, q.ix, ay1, q.fx, fy1);
        e[2] = lerp_glob<R>(F + 2 * G, g, q.ix, q.iy, q.fx, q.fy);
        b[0] = lerp_glob<R>(F + 3 * G, g, q.ix, ay1, q.fx, fy1);
        b[1] = lerp_glob<R>(F + 4 * G, g, ax1, q.iy, fx1, q.fy);
        b[2] = lerp_glob<R>(F + 5 * G, g, ax1, ay1, fx1, fy1);
        const R a = MIX ? (R)pc.af : (R)pc.a;
        int sx, sy, sz;
        if constexpr (HC) {
            const R ic2 = MIX ? (R)pc.ic2f : (R)pc.ic2;
            hc3<R>(q.vx, q.vy, q.vz, e, b, a, ic2);
            if (pc.move) {
                const R ig = recip<R>(lorentz<R>(q.vx, q.vy, q.vz, ic2));
                ok = move_pt_v<MIX, 2>(q, g, pc, q.vx * ig, q.vy * ig, q.vz * ig, sx, sy, sz) && ok;
            }
        } else {
            boris3<R>(q.vx, q.vy, q.vz, e, b, a);
            if (pc.move) ok = move_pt<MIX, 2>(q, g, pc, sx, sy, sz) && ok;
        }
        if (!ok) bad = 1;
        store_pt<MIX, 2, 3>(p, i, q);
    }
    if (bad) raise_err(c.err, ERR_DOMAIN);
}

inline int em_blocks(int64_t G, int cap) {
    int64_t b = (G + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    return (int)(b > cap ? cap : b);
}

}  // namespace

hipError_t launch_em_init(const Geo &g, const double *phi, double bz, double *F, hipStream_t s) {
    hipLaunchKernelGGL(k_em_init, dim3(em_blocks((int64_t)g.nx * g.ny, 4096)), dim3(kBlock), 0, s, g, phi, bz, F);
    return hipGetLastError();
}

hipError_t launch_em_gather_push(const Geo &g, bool mixed, const Parts &p, int64_t n, const double *F,
                                 const PushC &pc, const CtxDev &c, hipStream_t s) {
    const dim3 grid(em_blocks(n, 8192));
    if (mixed && g.hc)
        hipLaunchKernelGGL((k_em_gather_push<true, true>), grid, dim3(kBlock), 0, s, g, p, n, F, pc, c);
    else if (mixed)
        hipLaunchKernelGGL((k_em_gather_push<true, false>), grid, dim3(kBlock), 0, s, g, p, n, F, pc, c);
    else if (g.hc)
        hipLaunchKernelGGL((k_em_gather_push<false, true>), grid, dim3(kBlock), 0, s, g, p, n, F, pc, c);
    else
        hipLaunchKernelGGL((k_em_gather_push<false, false>), grid, dim3(kBlock), 0, s, g, p, n, F, pc, c);
    return hipGetLastError();
}

static_assert(2 * kEmStepBlocks <= kMaxSpecBlocks, "field partials fit part_spec");

hipError_t launch_fdtd_step(const Geo &g, const double *F, double *Fn, const double *J, double *Jnext, double *Jout,
                            double dt, double c2, double bz, double dV, double mass, int npush, double *diag,
                            const CtxDev &c, hipStream_t s) {
    // one round of resident workgroups (measured at 1024^2: 53 us with one
    // round, 60 us with 2048 workgroups, 62 us with 1024)
    static int resident = 0;
    if (!resident) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fdtd_step<true>, kBlock, 0) != hipSuccess ||
            per_cu <= 0)
            per_cu = 4;
        resident = cus * per_cu;
    }
    const int nt = ((g.nx + kFTX - 1) / kFTX) * ((g.ny + kFTY - 1) / kFTY);
    int nblk = nt < resident ? nt : resident;
    if (nblk > kEmStepBlocks) nblk = kEmStepBlocks;
    if (diag) {
        hipLaunchKernelGGL(k_fdtd_step<true>, dim3(nblk), dim3(kBlock), 0, s, g, F, Fn, J, Jnext, Jout, dt, c2, bz,
                           c.part_spec);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_em_finalize, dim3(1), dim3(1024), 0, s, nblk, kEmStepBlocks, npush, c2, dV, mass, diag,
                           c);
    } else {
        hipLaunchKernelGGL(k_fdtd_step<false>, dim3(nblk), dim3(kBlock), 0, s, g, F, Fn, J, Jnext, Jout, dt, c2, bz,
                           nullptr);
    }
    return hipGetLastError();
}

}  // namespace apic

extern "C" {

static apic_status check_em(apic_ctx *c) {
    if (!c) return APIC_EINVAL;
    if (!c->g.em) return fail(c, APIC_EINVAL, "the context is electrostatic (model = APIC_ELECTROSTATIC)");
    return APIC_OK;
}

apic_status apic_em_init_fields(apic_ctx *c, const apic_particles *p, double *F, void *ws, void *stream) {
    apic_status st = check_em(c);
    if (st != APIC_OK) return st;
    st = check_parts(c, p, false);
    if (st != APIC_OK) return st;
    if (!F || !ws) return fail(c, APIC_EINVAL, "F and workspace are required");
    hipStream_t s = (hipStream_t)stream;
    // charge (FP64 weights or fixed-point sums) -> rho -> phi -> F
    void *acc = wsp<void>(ws, c->o_acc);
    double *rho = wsp<double>(ws, c->o_rho);
    double *phi = rho;
    void *rhat = wsp<void>(ws, c->o_rhat);
    void *phat = wsp<void>(ws, c->o_ehat);
    st = apic_deposit(c, p, acc, stream);
    if (st != APIC_OK) return st;
    if (c->mixed)
        HIPCHK(c, launch_rho(c->g, true, acc, rho, acc_scale(c), c->d.rho_ion, 1, nullptr, s));
    else
        HIPCHK(c, launch_copy_bytes(rho, acc, 8 * (int64_t)c->d.nx * c->d.ny, s));
    FFTCHK(c, hipfftSetStream(c->fwd, s));
    FFTCHK(c, hipfftExecD2Z(c->fwd, (hipfftDoubleReal *)rho, (hipfftDoubleComplex *)rhat));
    HIPCHK(c, launch_spectral(c->g, rhat, phat, c->dev, s));
    FFTCHK(c, hipfftSetStream(c->inv, s));
    FFTCHK(c, hipfftExecZ2D(c->inv, (hipfftDoubleComplex *)phat, (hipfftDoubleReal *)phi));
    HIPCHK(c, launch_em_init(c->g, phi, c->d.bz, F, s));
    return APIC_OK;
}

apic_status apic_em_gather_push(apic_ctx *c, apic_particles *p, const double *F, double dt_scale, int move,
                                void *stream) {
    apic_status st = check_em(c);
    if (st != APIC_OK) return st;
    st = check_parts(c, p, false);
    if (st != APIC_OK) return st;
    if (!F) return fail(c, APIC_EINVAL, "F is NULL");
    if (!std::isfinite(dt_scale)) return fail(c, APIC_EINVAL, "dt_scale is not finite");
    const PushC pc = push_coeffs(c, dt_scale, move);
    HIPCHK(c, launch_em_gather_push(c->g, c->mixed, parts_of(p), c->n, F, pc, c->dev, (hipStream_t)stream));
    return APIC_OK;
}

apic_status apic_em_step(apic_ctx *c, apic_particles *p, double *F, double *J, int nsteps, double *diag, void *ws,
                         void *stream) {
    apic_status st = check_em(c);
    if (st != APIC_OK) return st;
    st = check_parts(c, p, true);
    if (st != APIC_OK) return st;
    if (!F || !ws || nsteps < 0) return fail(c, APIC_EINVAL, "F, workspace and nsteps >= 0 are required");
    if (nsteps == 0) return APIC_OK;
    hipStream_t s = (hipStream_t)stream;
    const int nb = c->g.nbuckets;
    const int64_t G = (int64_t)c->d.nx * c->d.ny;
    int32_t *cnt = wsp<int32_t>(ws, c->o_cnt);
    int32_t *offs = wsp<int32_t>(ws, c->o_offs);
    int32_t *farcnt = wsp<int32_t>(ws, c->o_farcnt);
    int32_t *tot = wsp<int32_t>(ws, c->o_tot);
    int32_t *deep = wsp<int32_t>(ws, c->o_deep);
    double *jacc = wsp<double>(ws, c->o_jacc);
    Parts A = parts_of(p), B = parts_ws(c, ws);
    int32_t *bsA = p->bucket_start, *bsB = wsp<int32_t>(ws, c->o_bstart);
    const PushC pc = push_coeffs(c, 1.0, 1);
    const double c2 = c->d.c_light * c->d.c_light, dt = c->d.dt;
    HIPCHK(c, launch_fill_i32(farcnt, nb, 0, s));
    // the bucket totals: two buffers, alternating by step
    HIPCHK(c, launch_fill_i32(tot, 2 * (int64_t)nb, 0, s));
    HIPCHK(c, launch_fill_i32(deep, (int64_t)nb * kDeepTab, 0, s));
    double *F2 = wsp<double>(ws, c->o_f2);
    HIPCHK(c, launch_fill_u64((uint64_t *)jacc, 2 * 3 * G, 0, s));
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
        // F^n in F on even steps and in F2 on odd ones; J^{n+1/2} alternates likewise
        double *Fk = even ? F : F2, *Fk1 = even ? F2 : F;
        double *Jk = jacc + (even ? 0 : 3 * G), *Jk1 = jacc + (even ? 3 * G : 0);
        HIPCHK(c, launch_step_count(c->g, c->mixed, src, bs_src, Fk, nullptr, pc, cnt, tot_k, farcnt, deep, c->dev, s));
        if (ev && c->prof_all) HIPCHK(c, hipEventRecord(ev[1], s));
        if (fused_scan_offsets(c->g)) {
            HIPCHK(c, launch_scan_offsets(c->g, tot_k, tot_n, bs_dst, c->n, max_per_bucket(c), 1, cnt, offs, c->dev,
                                          s));
        } else {
            HIPCHK(c, launch_scan_dir(c->g, tot_k, bs_dst, c->n, max_per_bucket(c), 1, c->dev, s));
            HIPCHK(c, launch_dest_offsets(c->g, cnt, bs_dst, offs, s));
        }
        if (ev) HIPCHK(c, hipEventRecord(ev[2], s));
        HIPCHK(c, launch_step_push(c->g, c->mixed, src, dst, bs_src, bs_dst, cnt, offs, farcnt, Fk, nullptr, pc, Jk, p->perm,
                                   diag ? c->dev.part_push : nullptr, deep, c->dev, s));
        if (ev) HIPCHK(c, hipEventRecord(ev[3], s));
        HIPCHK(c, launch_fdtd_step(c->g, Fk, Fk1, Jk, Jk1, (J && last) ? J : nullptr, dt, c2, c->d.bz, c->dV, c->mass,
                                   nb, diag, c->dev, s));
        if (ev && c->prof_all) HIPCHK(c, hipEventRecord(ev[4], s));
    }
    if (nsteps & 1) {
        st = copy_parts(c, A, B, s);
        if (st != APIC_OK) return st;
        HIPCHK(c, launch_copy_bytes(bsA, bsB, 4 * (int64_t)(nb + 1), s));
        HIPCHK(c, launch_copy_bytes(F, F2, 48 * G, s));
    }
    return APIC_OK;
}

}  // extern "C"
