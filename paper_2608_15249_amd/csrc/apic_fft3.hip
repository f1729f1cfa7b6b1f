// Periodic 3D Poisson solve on power-of-two grids (4 to 256 nodes per axis)
// for the field step of the 3D cycle: charge accumulation -> rho -> phi
// (7-point Laplacian, zero mean) -> E = -(centred difference of phi), with
// the field-energy and charge diagnostics. Five transform launches and the
// gradient:
//
//   1. k3_xfwd: a workgroup per block of Y rows of one z plane. rho of the
//      rows from the accumulation buffer (cleared behind it; fixed-point node
//      sums also totalled exactly), one complex FFT along x per row pair
//      (rho_a + i rho_b), split into the rows' half spectra, stored as
//      A[z][kx][y] (y fastest) so that the y transforms read whole lines.
//   2. k3_yfwd: a workgroup per (kx, block of ZB planes): FFT along y of the
//      ZB lines, stored as B[kx][ky][z] (z fastest).
//   3. k3_zsolve: a workgroup per (kx, block of KY values of ky): FFT along
//      z, phi_hat = rho_hat / K^2 (K^2 the sum of the three axes' modified
//      wavenumbers, phi_hat(0) = 0) with the Parseval partial of
//      sum |E_hat|^2 = sum (kappa_x^2 + kappa_y^2 + kappa_z^2) |phi_hat|^2,
//      the 1/G of the unnormalised inverses, inverse FFT along z, in place.
//   4. k3_yinv: inverse FFT along y, back to A[z][kx][y].
//   5. k3_xinv: per block of Y rows, the inverse along x of two rows at once
//      (their half spectra combined by Hermitian symmetry into one complex
//      spectrum whose inverse has the rows as real and imaginary parts):
//      phi [nz][ny][nx].
//   then the gradient launch of the general path (k_grad), whose last
//   workgroup reduces the diagnostics.
// The mathematics of the general path (library real-to-complex transforms,
// spectral division, real-space centred difference) with the transforms
// done in LDS; every global read and write covers runs of at least 128
// bytes.
#include "apic_fftlds.h"

namespace apic {
namespace {

// Work split (all powers of two): rows per x workgroup, planes per y
// workgroup, ky values per z workgroup.
struct Split3 {
    int Y, ZB, KY;
};

inline Split3 split3(const Geo &g) {
    Split3 s;
    s.Y = g.nx <= 128 ? 16 : 8;
    if (s.Y > g.ny) s.Y = g.ny;
    s.ZB = g.nz < 8 ? g.nz : 8;
    // (the z workgroup also holds a small reduction array: 2 KY nz complex
    // stay below 64 KiB)
    s.KY = g.nz <= 128 ? 8 : 4;
    if (s.KY > g.ny) s.KY = g.ny;
    return s;
}

// LDS: two buffers of (Y/2) nx complex.
template <bool MIX>
__global__ void __launch_bounds__(kBlock) k3_xfwd(Geo g, typename AccOf<MIX>::T *acc, double scale, double add,
                                                  int clear, double2 *A, const double2 *tw, int lgnx, int lgmax,
                                                  int Y, unsigned long long *qacc) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nx = g.nx, ny = g.ny, hx = nx / 2 + 1, P = Y / 2;
    double2 *b0 = (double2 *)smem, *b1 = b0 + (size_t)P * nx;
    const int nyb = ny / Y;
    const int z = (int)blockIdx.x / nyb, y0 = ((int)blockIdx.x % nyb) * Y;
    const int64_t base = ((int64_t)z * ny + y0) * nx;   // first of the Y rows
    const int sd = g.S * g.dim;
    QSum q{0, 0};
    // row pair p: rows y0 + 2p (real part) and y0 + 2p + 1 (imaginary part);
    // entries past the rows go to b1, which the first pass overwrites
    using T = typename AccOf<MIX>::T;
    struct Two {
        T a, b;
    };
    const int cnt = P * nx;
    fill_batched<Two, 4>(
        cnt,
        [&](int t) {
            const int p = t / nx, i = t - p * nx;
            const int64_t ia = base + (int64_t)(2 * p) * nx + i;
            return Two{acc[ia], acc[ia + nx]};
        },
        [&](int t, const Two &v) {
            const bool in = t < cnt;
            if constexpr (MIX) {
                if (qacc) {
                    qsum_add(q, in ? (int64_t)v.a : 0, sd);
                    qsum_add(q, in ? (int64_t)v.b : 0, sd);
                }
            }
            *(in ? &b0[t] : &b1[threadIdx.x & (cnt - 1)]) =
                make_double2(acc_to_rho<MIX>(v.a, scale, add), acc_to_rho<MIX>(v.b, scale, add));
        });
    if constexpr (MIX) {
        if (qacc) qsum_flush(q, sd, qacc);
    }
    __syncthreads();
    if (clear) {
        for (int t = threadIdx.x; t < Y * nx; t += blockDim.x) acc[base + t] = (typename AccOf<MIX>::T)0;
    }
    const double2 *R = fft_lds<-1>(b0, b1, lgnx, P, tw, lgmax);
    // split: rho_a_hat(k) = (Z(k) + conj Z(-k)) / 2, rho_b_hat(k) = (Z(k) - conj Z(-k)) / (2i);
    // thread t: kx = t / Y, row r = t % Y (consecutive threads, consecutive y)
    for (int t = threadIdx.x; t < hx * Y; t += blockDim.x) {
        const int kx = t / Y, r = t - kx * Y, p = r >> 1;
        const double2 zk = R[p * nx + kx], zm = R[p * nx + ((nx - kx) & (nx - 1))];
        const double2 h = (r & 1) ? make_double2(0.5 * (zk.y + zm.y), -0.5 * (zk.x - zm.x))
                                  : make_double2(0.5 * (zk.x + zm.x), 0.5 * (zk.y - zm.y));
        A[((int64_t)z * hx + kx) * ny + y0 + r] = h;
    }
}

// LDS: two buffers of ZB ny complex.
__global__ void __launch_bounds__(kBlock) k3_yfwd(Geo g, const double2 *A, double2 *B, const double2 *tw,
                                                  int lgny, int lgmax, int ZB) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nx = g.nx, ny = g.ny, nz = g.nz, hx = nx / 2 + 1;
    double2 *b0 = (double2 *)smem, *b1 = b0 + (size_t)ZB * ny;
    const int nzb = nz / ZB;
    const int kx = (int)blockIdx.x / nzb, z0 = ((int)blockIdx.x % nzb) * ZB;
    const int cnt = ZB * ny;
    fill_batched<double2, 4>(
        cnt,
        [&](int t) {
            const int l = t / ny, y = t - l * ny;
            return A[((int64_t)(z0 + l) * hx + kx) * ny + y];
        },
        [&](int t, double2 v) { *(t < cnt ? &b0[t] : &b1[threadIdx.x & (cnt - 1)]) = v; });
    __syncthreads();
    const double2 *R = fft_lds<-1>(b0, b1, lgny, ZB, tw, lgmax);
    for (int t = threadIdx.x; t < ny * ZB; t += blockDim.x) {
        const int ky = t / ZB, l = t - ky * ZB;
        B[((int64_t)kx * ny + ky) * nz + z0 + l] = R[l * ny + ky];
    }
}

// LDS: two buffers of KY nz complex.
__global__ void __launch_bounds__(kBlock) k3_zsolve(Geo g, double2 *B, const double2 *tw, int lgnz, int lgmax,
                                                    int KY, CtxDev c) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double sRed[kWaves];
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    double2 *b0 = (double2 *)smem, *b1 = b0 + (size_t)KY * nz;
    const int nyb = ny / KY;
    const int kx = (int)blockIdx.x / nyb, ky0 = ((int)blockIdx.x % nyb) * KY;
    double2 *line = B + ((int64_t)kx * ny + ky0) * nz;   // KY lines back to back
    const int cnt = KY * nz;
    fill_batched<double2, 4>(
        cnt, [&](int t) { return line[t]; },
        [&](int t, double2 v) { *(t < cnt ? &b0[t] : &b1[threadIdx.x & (cnt - 1)]) = v; });
    __syncthreads();
    double2 *R = fft_lds<-1>(b0, b1, lgnz, KY, tw, lgmax);
    double2 *S = (R == b0) ? b1 : b0;
    const double norm = 1.0 / ((double)nx * (double)ny * (double)nz);
    const double kx2 = c.kx2[kx], kax = c.kapx[kx];
    const double wgt = (kx == 0 || 2 * kx == nx) ? 1.0 : 2.0;
    double part = 0.0;
    for (int t = threadIdx.x; t < KY * nz; t += blockDim.x) {
        const int l = t / nz, kz = t - l * nz, ky = ky0 + l;
        const bool dc = kx == 0 && ky == 0 && kz == 0;
        const double2 r = R[t];
        if (dc) *c.rho0 = r.x;
        const double inv = dc ? 0.0 : 1.0 / ((kx2 + c.ky2[ky]) + c.kz2[kz]);
        const double pr = r.x * inv, pi = r.y * inv;
        const double kay = c.kapy[ky], kaz = c.kapz[kz];
        part += wgt * (kax * kax + kay * kay + kaz * kaz) * (pr * pr + pi * pi);
        S[t] = make_double2(pr * norm, pi * norm);
    }
    __syncthreads();
    const double2 *P = fft_lds<+1>(S, R, lgnz, KY, tw, lgmax);
    for (int t = threadIdx.x; t < KY * nz; t += blockDim.x) line[t] = P[t];
    const double bs = block_sum(part, sRed);
    if (threadIdx.x == 0) c.part_spec[blockIdx.x] = bs;
}

// LDS: two buffers of ZB ny complex.
__global__ void __launch_bounds__(kBlock) k3_yinv(Geo g, const double2 *B, double2 *A, const double2 *tw,
                                                  int lgny, int lgmax, int ZB) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nx = g.nx, ny = g.ny, nz = g.nz, hx = nx / 2 + 1;
    double2 *b0 = (double2 *)smem, *b1 = b0 + (size_t)ZB * ny;
    const int nzb = nz / ZB;
    const int kx = (int)blockIdx.x / nzb, z0 = ((int)blockIdx.x % nzb) * ZB;
    const int cnt = ny * ZB;
    fill_batched<double2, 4>(
        cnt,
        [&](int t) {
            const int ky = t / ZB, l = t - ky * ZB;
            return B[((int64_t)kx * ny + ky) * nz + z0 + l];
        },
        [&](int t, double2 v) {
            const int ky = t / ZB, l = t - ky * ZB;
            *(t < cnt ? &b0[l * ny + ky] : &b1[threadIdx.x & (cnt - 1)]) = v;
        });
    __syncthreads();
    const double2 *R = fft_lds<+1>(b0, b1, lgny, ZB, tw, lgmax);
    for (int t = threadIdx.x; t < ZB * ny; t += blockDim.x) {
        const int l = t / ny, y = t - l * ny;
        A[((int64_t)(z0 + l) * hx + kx) * ny + y] = R[t];
    }
}

// LDS: the Y rows' half spectra (Y hx complex), then two buffers of (Y/2) nx.
__global__ void __launch_bounds__(kBlock) k3_xinv(Geo g, const double2 *A, double *phi, const double2 *tw,
                                                  int lgnx, int lgmax, int Y) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nx = g.nx, ny = g.ny, hx = nx / 2 + 1, P = Y / 2;
    double2 *h = (double2 *)smem;
    double2 *b0 = h + (size_t)Y * hx, *b1 = b0 + (size_t)P * nx;
    const int nyb = ny / Y;
    const int z = (int)blockIdx.x / nyb, y0 = ((int)blockIdx.x % nyb) * Y;
    // entries past the spectra go to b0, written only after the next barrier
    const int cnt = hx * Y;
    fill_batched<double2, 4>(
        cnt,
        [&](int t) {
            const int kx = t / Y, r = t - kx * Y;
            return A[((int64_t)z * hx + kx) * ny + y0 + r];
        },
        [&](int t, double2 v) {
            const int kx = t / Y, r = t - kx * Y;
            *(t < cnt ? &h[r * hx + kx] : &b0[threadIdx.x & (P * nx - 1)]) = v;
        });
    __syncthreads();
    // Z_p(k) = Ha(k) + i Hb(k) over the full range, Ha(k) = conj Ha(nx - k)
    // above nx/2; at k = 0 and nx/2 the half spectra of real rows are real
    // (their rounding residue in the imaginary part is dropped, as a
    // complex-to-real library transform does)
    for (int t = threadIdx.x; t < P * nx; t += blockDim.x) {
        const int p = t / nx, k = t - p * nx;
        const bool up = k > nx / 2;
        const int kk = up ? nx - k : k;
        double2 a = h[(2 * p) * hx + kk], b = h[(2 * p + 1) * hx + kk];
        if (kk == 0 || 2 * kk == nx) a.y = b.y = 0.0;
        b0[t] = up ? make_double2(a.x + b.y, b.x - a.y) : make_double2(a.x - b.y, a.y + b.x);
    }
    __syncthreads();
    const double2 *U = fft_lds<+1>(b0, b1, lgnx, P, tw, lgmax);
    const int64_t base = ((int64_t)z * ny + y0) * nx;
    for (int t = threadIdx.x; t < P * nx; t += blockDim.x) {
        const int p = t / nx, i = t - p * nx;
        const double2 u = U[t];
        phi[base + (int64_t)(2 * p) * nx + i] = u.x;
        phi[base + (int64_t)(2 * p + 1) * nx + i] = u.y;
    }
}

inline int ilog2_3(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

}  // namespace

bool fused_fft3_supported(int dim, int nx, int ny, int nz) {
    auto pow2 = [](int v) { return v >= 4 && v <= kFusedFft3Max && (v & (v - 1)) == 0; };
    return dim == 3 && pow2(nx) && pow2(ny) && pow2(nz);
}

int fused_fft3_spec_blocks(const Geo &g) { return (g.nx / 2 + 1) * (g.ny / split3(g).KY); }

hipError_t launch_fused_field3(const Geo &g, bool mixed_acc, void *acc, double scale, double add, int clear,
                               void *Av, void *Bv, double *phi, const double *tw_table, unsigned long long *qacc,
                               const CtxDev &c, hipStream_t s) {
    const int lgnx = ilog2_3(g.nx), lgny = ilog2_3(g.ny), lgnz = ilog2_3(g.nz);
    int lgmax = lgnx > lgny ? lgnx : lgny;
    if (lgnz > lgmax) lgmax = lgnz;
    const double2 *tw = (const double2 *)tw_table;
    double2 *A = (double2 *)Av, *B = (double2 *)Bv;
    const Split3 sp = split3(g);
    const int hx = g.nx / 2 + 1;
    const dim3 rows((g.ny / sp.Y) * g.nz), cols(hx * (g.nz / sp.ZB)), lines(hx * (g.ny / sp.KY));
    const size_t sh_x = (size_t)sp.Y * g.nx * sizeof(double2);
    const size_t sh_y = 2 * (size_t)sp.ZB * g.ny * sizeof(double2);
    const size_t sh_z = 2 * (size_t)sp.KY * g.nz * sizeof(double2);
    const size_t sh_xi = ((size_t)sp.Y * hx + (size_t)sp.Y * g.nx) * sizeof(double2);
    if (mixed_acc)
        hipLaunchKernelGGL(k3_xfwd<true>, rows, dim3(kBlock), sh_x, s, g, (unsigned long long *)acc, scale, add,
                           clear, A, tw, lgnx, lgmax, sp.Y, qacc);
    else
        hipLaunchKernelGGL(k3_xfwd<false>, rows, dim3(kBlock), sh_x, s, g, (double *)acc, scale, add, clear, A, tw,
                           lgnx, lgmax, sp.Y, nullptr);
    hipLaunchKernelGGL(k3_yfwd, cols, dim3(kBlock), sh_y, s, g, (const double2 *)A, B, tw, lgny, lgmax, sp.ZB);
    hipLaunchKernelGGL(k3_zsolve, lines, dim3(kBlock), sh_z, s, g, B, tw, lgnz, lgmax, sp.KY, c);
    hipLaunchKernelGGL(k3_yinv, cols, dim3(kBlock), sh_y, s, g, (const double2 *)B, A, tw, lgny, lgmax, sp.ZB);
    hipLaunchKernelGGL(k3_xinv, rows, dim3(kBlock), sh_xi, s, g, (const double2 *)A, phi, tw, lgnx, lgmax, sp.Y);
    return hipGetLastError();
}

}  // namespace apic
