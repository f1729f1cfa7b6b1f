// Periodic 2D Poisson solve on power-of-two grids (up to 1024 nodes per
// axis) in three launches, for the field step of the cycle: charge
// accumulation -> rho -> phi (5-point Laplacian, zero mean) -> E = -(centred
// difference of phi), with the field-energy and charge diagnostics.
//
//   1. k_fft_rows: one workgroup per pair of rows. rho of both rows from the
//      accumulation buffer (cleared behind it), one complex FFT along x of
//      rho_j0 + i rho_j1 in LDS, split into the two rows' half spectra
//      H [ny][nx/2+1] (the layout of a real-to-complex transform). Fixed-point
//      node sums are also reduced exactly (integer sums) for the charge.
//   2. k_fft_cols: one workgroup per column kx of H. FFT along y, then
//      phi_hat = rho_hat / K^2 (K^2 the Laplacian's modified wavenumber,
//      phi_hat(0) = 0), with the per-block Parseval partial of
//      sum |E_hat|^2 (E_hat_d = -i kappa_d phi_hat, kappa_d = sin(k d)/d the
//      symbol of the centred difference). One inverse FFT along y gives the
//      x-spectrum of phi at kx; Ex~ = -i kappa_x of it, and Ey~ its centred
//      difference along y. The x-spectrum Z of the complex field Ex + i Ey
//      follows at columns kx and nx - kx from the Hermitian symmetry of the
//      two real fields. Z is
//      stored column by column ([nx][ny]), so that each workgroup writes its
//      two columns as whole contiguous lines (stores that cover part of a
//      line measured far slower than whole-line stores).
//   3. k_fft_rows_inv: one workgroup per row. Inverse FFT along x of Z (a
//      strided read of the column-major Z; the rows of one XCD are adjacent,
//      so its L2 serves each fetched line to eight rows): Ex = Re, Ey = Im
//      (and their binary32 rounding). The launch's last workgroup reduces
//      the diagnostics.
// The same mathematics as the general path (library real-to-complex
// transforms, spectral division, real-space centred difference); the x
// derivative is taken in spectral form, -i sin(kx dx)/dx, which is the
// transform of the centred difference exactly, the y derivative as the
// centred difference itself, applied to the x-spectrum of phi.
//
// Transforms: Stockham passes between two LDS buffers (the output in natural
// order, one barrier per pass), radix 8 in registers after one radix-2 or
// radix-4 pass; twiddles exp(-2 pi i k / nmax) from a table in global memory
// (16 KiB at most, cache resident), one entry per butterfly and its powers
// by complex products.
#include "apic_fftlds.h"

namespace apic {
namespace {

static_assert(kFusedFftMax <= 8 * kBlock, "one radix-8 butterfly per thread and pass");

// Entries of one line per thread (a line of at most kFusedFftMax): the loads
// of a line are all issued before the first is waited for.
constexpr int kLinePer = kFusedFftMax / kBlock;

// LDS: two buffers of nx complex.
// qacc (fixed-point sums only, may be NULL): the exact total of the two rows'
// node sums (the physical nodes 0..nxp between walls) is added to it.
template <bool MIX, bool WALLS>
__global__ void __launch_bounds__(kBlock) k_fft_rows(Geo g, typename AccOf<MIX>::T *acc, double scale, double add,
                                                     int clear, double2 *H, const double2 *tw, int lgnx,
                                                     int lgmax, unsigned long long *qacc) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nx = g.nx;
    double2 *b0 = (double2 *)smem, *b1 = b0 + nx;
    const int64_t r0 = (int64_t)(2 * blockIdx.x) * nx, r1 = r0 + nx;
    const int sd = g.S * g.dim;
    const FftTw ft = fft_twiddles(lgnx, tw, lgmax);
    QSum q{0, 0};
    if constexpr (WALLS) {
        for (int i = threadIdx.x; i < nx; i += blockDim.x) {
            double v0, v1;
            // odd extension of the physical rows [0, nxp]: zero on the walls
            const int nxp = g.nxp;
            if (i == 0 || i == nxp) {
                v0 = v1 = 0.0;
            } else {
                const int src = i < nxp ? i : nx - i;
                const double sg = i < nxp ? 1.0 : -1.0;
                v0 = sg * acc_value<MIX>(acc, r0 + src, scale, add);
                v1 = sg * acc_value<MIX>(acc, r1 + src, scale, add);
            }
            b0[i] = make_double2(v0, v1);
        }
    }
    if constexpr (!WALLS) {
        typename AccOf<MIX>::T a0[kLinePer], a1[kLinePer];
#pragma unroll
        for (int r = 0; r < kLinePer; ++r) {
            const int i = min((int)threadIdx.x + r * kBlock, nx - 1);   // in bounds, used only below nx
            a0[r] = acc[r0 + i];
            a1[r] = acc[r1 + i];
        }
#pragma unroll
        for (int r = 0; r < kLinePer; ++r) {
            const int i = threadIdx.x + r * kBlock;
            if (i < nx) {
                if constexpr (MIX) {
                    if (qacc) {
                        qsum_add(q, (int64_t)a0[r], sd);
                        qsum_add(q, (int64_t)a1[r], sd);
                    }
                }
                b0[i] = make_double2(acc_to_rho<MIX>(a0[r], scale, add), acc_to_rho<MIX>(a1[r], scale, add));
            }
        }
    }
    if constexpr (MIX) {
        if (qacc) {
            // between walls: the physical nodes 0..nxp, walls included
            if constexpr (WALLS) {
                for (int i = threadIdx.x; i <= g.nxp; i += blockDim.x) {
                    qsum_add(q, (int64_t)acc[r0 + i], sd);
                    qsum_add(q, (int64_t)acc[r1 + i], sd);
                }
            }
            qsum_flush(q, sd, qacc);
        }
    }
    __syncthreads();
    if (clear) {
        // after every read of the two rows (the walls read mirrored entries)
        for (int i = threadIdx.x; i < nx; i += blockDim.x) {
            acc[r0 + i] = (typename AccOf<MIX>::T)0;
            acc[r1 + i] = (typename AccOf<MIX>::T)0;
        }
    }
    const double2 *R = fft_lds_one<-1>(b0, b1, lgnx, tw, lgmax, ft);
    // split: rho_j0_hat(k) = (Z(k) + conj Z(-k)) / 2, rho_j1_hat(k) = (Z(k) - conj Z(-k)) / (2i)
    const int hx = nx / 2 + 1;
    const int64_t h0 = (int64_t)(2 * blockIdx.x) * hx, h1 = h0 + hx;
    for (int k = threadIdx.x; k < hx; k += blockDim.x) {
        const double2 zk = R[k], zm = R[(nx - k) & (nx - 1)];
        H[h0 + k] = make_double2(0.5 * (zk.x + zm.x), 0.5 * (zk.y - zm.y));
        H[h1 + k] = make_double2(0.5 * (zk.y + zm.y), -0.5 * (zk.x - zm.x));
    }
}

// LDS: two buffers of ny complex. Block b handles column (b % 8) * per + b / 8
// (per = ceil(hx / 8)), so that neighbouring columns share an XCD's L2;
// blocks past the last column only write their zero partial.
__global__ void __launch_bounds__(kBlock) k_fft_cols(Geo g, const double2 *H, double2 *Z, const double2 *tw,
                                                     int lgny, int lgmax, int per, CtxDev c) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double sRed[kWaves];
    const int nx = g.nx, ny = g.ny, hx = nx / 2 + 1;
    double2 *A = (double2 *)smem, *B = A + ny;
    const int kx = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    double part = 0.0;
    if (kx < hx) {
        const FftTw ft = fft_twiddles(lgny, tw, lgmax);   // the same for the inverse
        double2 h[kLinePer];
#pragma unroll
        for (int r = 0; r < kLinePer; ++r) {
            const int y = min((int)threadIdx.x + r * kBlock, ny - 1);   // in bounds, used only below ny
            h[r] = H[(int64_t)y * hx + kx];
        }
#pragma unroll
        for (int r = 0; r < kLinePer; ++r) {
            // entries past the line go to B, which the first pass overwrites
            // (a store for every entry keeps the loads ahead of the first wait)
            const int y = threadIdx.x + r * kBlock;
            *(y < ny ? &A[y] : &B[threadIdx.x & (ny - 1)]) = h[r];
        }
        __syncthreads();
        double2 *R = fft_lds_one<-1>(A, B, lgny, tw, lgmax, ft);
        double2 *S = (R == A) ? B : A;
        const double norm = 1.0 / ((double)nx * (double)ny);
        const double kx2 = c.kx2[kx], kax = c.kapx[kx];
        const double wgt = (kx == 0 || 2 * kx == nx) ? 1.0 : 2.0;
        // phi_hat (scaled by 1/G for the unnormalised inverse) into S
        for (int ky = threadIdx.x; ky < ny; ky += blockDim.x) {
            const double2 r = R[ky];
            if (kx == 0 && ky == 0) *c.rho0 = r.x;
            const double inv = (kx == 0 && ky == 0) ? 0.0 : 1.0 / (kx2 + c.ky2[ky]);
            const double pr = r.x * inv, pi = r.y * inv;
            const double kay = c.kapy[ky];
            part += wgt * (kax * kax + kay * kay) * (pr * pr + pi * pi);
            S[ky] = make_double2(pr * norm, pi * norm);
        }
        __syncthreads();
        // P = inverse_y(phi_hat), the x-spectrum of phi at this kx. Ex~ = -i kappa_x P;
        // Ey~ = -(P(y+1) - P(y-1)) / (2 dy), the centred difference along y (whose
        // symbol i sin(ky dy)/dy makes it the inverse of -i kappa_y phi_hat)
        const double2 *P = fft_lds_one<+1>(S, R, lgny, tw, lgmax, ft);
        const double hy = 0.5 * g.inv_dy;
        const bool self = kx == 0 || 2 * kx == nx;
        const int64_t c0 = (int64_t)kx * ny, c1 = (int64_t)(nx - kx) * ny;   // column-major Z
        for (int y = threadIdx.x; y < ny; y += blockDim.x) {
            const double2 p = P[y], pm = P[(y - 1) & (ny - 1)], pp = P[(y + 1) & (ny - 1)];
            const double dx_ = (pp.x - pm.x) * hy, dy_ = (pp.y - pm.y) * hy;   // centred difference of P
            if (self) {
                // a self-conjugate column of two real fields: their real parts
                Z[c0 + y] = make_double2(kax * p.y, -dx_);
            } else {
                Z[c0 + y] = make_double2(kax * p.y + dy_, -kax * p.x - dx_);
                Z[c1 + y] = make_double2(kax * p.y - dy_, kax * p.x - dx_);
            }
        }
    }
    const double bs = block_sum(part, sRed);
    if (threadIdx.x == 0) c.part_spec[blockIdx.x] = bs;
}

// LDS: two buffers of nx complex. Block ny (the last)
// reduces the diagnostics from the partials of the earlier launches.
__global__ void __launch_bounds__(kBlock) k_fft_rows_inv(Geo g, const double2 *Z, double *E, float *E32,
                                                         const double2 *tw, int lgnx, int lgmax, FinArgs f,
                                                         CtxDev c) {
    if (blockIdx.x == gridDim.x - 1) {
        finalize_block(f, c);
        return;
    }
    extern __shared__ __align__(16) unsigned char smem[];
    const int nx = g.nx;
    const int64_t G = (int64_t)nx * g.ny;
    double2 *b0 = (double2 *)smem, *b1 = b0 + nx;
    // rows of one XCD (workgroups b, b + 8, ...) adjacent
    const int ny = g.ny;
    const int y = ny >= 8 ? (int)(blockIdx.x % 8) * (ny / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
    const int64_t row = (int64_t)y * nx;
    const FftTw ft = fft_twiddles(lgnx, tw, lgmax);
    double2 z[kLinePer];
#pragma unroll
    for (int r = 0; r < kLinePer; ++r) {
        const int i = min((int)threadIdx.x + r * kBlock, nx - 1);   // in bounds, used only below nx
        z[r] = Z[(int64_t)i * ny + y];
    }
#pragma unroll
    for (int r = 0; r < kLinePer; ++r) {
        // entries past the line go to b1, which the first pass overwrites
        const int i = threadIdx.x + r * kBlock;
        *(i < nx ? &b0[i] : &b1[threadIdx.x & (nx - 1)]) = z[r];
    }
    __syncthreads();
    const double2 *U = fft_lds_one<+1>(b0, b1, lgnx, tw, lgmax, ft);
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        const double2 e = U[i];
        if (E) {
            E[row + i] = e.x;
            E[G + row + i] = e.y;
        }
        if (E32) {
            E32[row + i] = (float)e.x;
            E32[G + row + i] = (float)e.y;
        }
    }
}

inline int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

}  // namespace

bool fused_fft_supported(int dim, int nx, int ny, int nz) {
    auto pow2 = [](int v) { return v >= 4 && v <= kFusedFftMax && (v & (v - 1)) == 0; };
    return dim == 2 && nz <= 1 && pow2(nx) && pow2(ny);
}

hipError_t launch_fused_field(const Geo &g, bool mixed_acc, void *acc, double scale, double add, int clear,
                              void *H, void *Z, double *E, float *E32, const double *tw_table, const FinArgs &f0,
                              const CtxDev &c, hipStream_t s) {
    const int lgnx = ilog2(g.nx), lgny = ilog2(g.ny);
    const int lgmax = lgnx > lgny ? lgnx : lgny;
    const double2 *tw = (const double2 *)tw_table;
    const size_t sh_rows = 2 * (size_t)g.nx * sizeof(double2);
    const size_t sh_cols = 2 * (size_t)g.ny * sizeof(double2);
    const dim3 rows(g.ny / 2);
    if (mixed_acc) {
        auto *a = (unsigned long long *)acc;
        if (g.walls)
            hipLaunchKernelGGL((k_fft_rows<true, true>), rows, dim3(kBlock), sh_rows, s, g, a, scale, add, clear,
                               (double2 *)H, tw, lgnx, lgmax, f0.sd ? c.qacc : nullptr);
        else
            hipLaunchKernelGGL((k_fft_rows<true, false>), rows, dim3(kBlock), sh_rows, s, g, a, scale, add, clear,
                               (double2 *)H, tw, lgnx, lgmax, f0.sd ? c.qacc : nullptr);
    } else {
        auto *a = (double *)acc;
        if (g.walls)
            hipLaunchKernelGGL((k_fft_rows<false, true>), rows, dim3(kBlock), sh_rows, s, g, a, scale, add, clear,
                               (double2 *)H, tw, lgnx, lgmax, nullptr);
        else
            hipLaunchKernelGGL((k_fft_rows<false, false>), rows, dim3(kBlock), sh_rows, s, g, a, scale, add, clear,
                               (double2 *)H, tw, lgnx, lgmax, nullptr);
    }
    const int hx = g.nx / 2 + 1;
    const int per = (hx + 7) / 8;
    const int ncol = 8 * per;
    hipLaunchKernelGGL(k_fft_cols, dim3(ncol), dim3(kBlock), sh_cols, s, g, (const double2 *)H, (double2 *)Z, tw,
                       lgny, lgmax, per, c);
    FinArgs f = f0;
    f.nspec = ncol;
    hipLaunchKernelGGL(k_fft_rows_inv, dim3(g.ny + 1), dim3(kBlock), sh_rows, s, g, (const double2 *)Z, E, E32, tw,
                       lgnx, lgmax, f, c);
    return hipGetLastError();
}

}  // namespace apic
