// Power-of-two complex FFTs in LDS (Stockham passes, radix 8 in registers)
// and the conversion of an accumulation buffer entry to rho, shared by the
// fused 2D and 3D periodic field solves.
#pragma once

#include "apic_device.h"
#include "apic_fill.h"

namespace apic {
namespace {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// x * (SIGN i)
template <int SIGN>
__device__ __forceinline__ double2 rot_i(double2 x) {
    return SIGN < 0 ? make_double2(x.y, -x.x) : make_double2(-x.y, x.x);
}

// In-register DFTs of 2, 4 and 8 points, kernel exp(SIGN 2 pi i j k / R),
// outputs in natural order. The 8-point one combines the 4-point DFTs of
// the even and odd inputs with the factors w^k, w = exp(SIGN 2 pi i / 8).
__device__ __forceinline__ void dft2(double2 &a, double2 &b) {
    const double2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <int SIGN>
__device__ __forceinline__ void dft4(double2 &v0, double2 &v1, double2 &v2, double2 &v3) {
    const double2 t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), u = rot_i<SIGN>(csub(v1, v3));
    v0 = cadd(t0, t2);
    v2 = csub(t0, t2);
    v1 = cadd(t1, u);
    v3 = csub(t1, u);
}

template <int SIGN>
__device__ __forceinline__ void dft8(double2 *v) {
    double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    double2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<SIGN>(e0, e1, e2, e3);
    dft4<SIGN>(o0, o1, o2, o3);
    const double h = 0.70710678118654752440;  // sqrt(1/2)
    const double sg = (double)SIGN;
    const double2 p1 = make_double2(h * (o1.x - sg * o1.y), h * (o1.y + sg * o1.x));    // w o1
    const double2 p2 = rot_i<SIGN>(o2);                                                 // w^2 o2
    const double2 p3 = make_double2(h * (-o3.x - sg * o3.y), h * (-o3.y + sg * o3.x));  // w^3 o3
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, p1);
    v[5] = csub(e1, p1);
    v[2] = cadd(e2, p2);
    v[6] = csub(e2, p2);
    v[3] = cadd(e3, p3);
    v[7] = csub(e3, p3);
}

// One radix-2^LR Stockham pass over m transforms of length 2^lgn stored back
// to back, sub-transform length ns = 2^lgns so far: butterfly j (of n/R per
// transform) takes the R inputs j + q n/R, twists input q by
// exp(SIGN 2 pi i q k / (R ns)) with k = j mod ns, and writes its R-point DFT
// to (j - k) R + k + q ns. Ends with a barrier.
template <int SIGN, int LR>
__device__ __forceinline__ void fft_pass(const double2 *a, double2 *b, int lgn, int m, int lgns, const double2 *tw,
                                         int lgmax) {
    constexpr int R = 1 << LR;
    const int lgnr = lgn - LR;
    const int nr = 1 << lgnr;
    const int ns = 1 << lgns;
    const int total = nr * m;
    const int tsh = lgmax - lgns - LR;
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
        const int j = t & (nr - 1);
        const int base = (t >> lgnr) << lgn;
        const int k = j & (ns - 1);
        double2 v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) v[q] = a[base + j + q * nr];
        if (lgns > 0) {
            // w^q from w = exp(SIGN 2 pi i k / (R ns)), one table entry: each a
            // product of at most three factors (fewer scattered table reads)
            double2 w[R];
            w[1] = tw[k << tsh];
            if (SIGN > 0) w[1].y = -w[1].y;
#pragma unroll
            for (int q = 2; q < R; ++q) w[q] = cmul(w[q / 2], w[q - q / 2]);
#pragma unroll
            for (int q = 1; q < R; ++q) v[q] = cmul(v[q], w[q]);
        }
        if constexpr (LR == 1) dft2(v[0], v[1]);
        else if constexpr (LR == 2) dft4<SIGN>(v[0], v[1], v[2], v[3]);
        else dft8<SIGN>(v);
        const int d = base + ((j - k) << LR) + k;
#pragma unroll
        for (int q = 0; q < R; ++q) b[d + q * ns] = v[q];
    }
    __syncthreads();
}

// m transforms of length 2^lgn stored back to back in a; SIGN = -1 forward,
// +1 inverse (unnormalised). b is a buffer of the same size. The data must be
// visible to the whole block on entry; the result (in a or b, returned) is
// visible on return. Radix-8 passes after one radix-2 or radix-4 pass for
// the remaining factor. tw[k] = exp(-2 pi i k / 2^lgmax), k < 2^lgmax.
template <int SIGN>
__device__ double2 *fft_lds(double2 *a, double2 *b, int lgn, int m, const double2 *tw, int lgmax) {
    int lgns = lgn % 3;
    if (lgns == 1) fft_pass<SIGN, 1>(a, b, lgn, m, 0, tw, lgmax);
    if (lgns == 2) fft_pass<SIGN, 2>(a, b, lgn, m, 0, tw, lgmax);
    if (lgns) {
        double2 *t = a;
        a = b;
        b = t;
    }
    for (; lgns < lgn; lgns += 3) {
        fft_pass<SIGN, 3>(a, b, lgn, m, lgns, tw, lgmax);
        double2 *t = a;
        a = b;
        b = t;
    }
    return a;
}

// One transform of n = 2^lgn <= 8 blockDim.x points: in each radix-8 pass a
// thread has at most one butterfly, and its twiddle can be read before the
// data. Entry q belongs to the pass with ns = 2^(lgn % 3 + 3 q) (when that is
// below n and not 1).
struct FftTw {
    double2 w[3];
};

__device__ __forceinline__ FftTw fft_twiddles(int lgn, const double2 *tw, int lgmax) {
    FftTw f;
    const int j = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int lgns = lgn % 3 + 3 * q;
        f.w[q] = make_double2(1.0, 0.0);
        if (lgns > 0 && lgns < lgn && j < (1 << (lgn - 3))) f.w[q] = tw[(j & ((1 << lgns) - 1)) << (lgmax - lgns - 3)];
    }
    return f;
}

// fft_pass<SIGN, 3> for one transform with at most one butterfly per thread,
// its twiddle w1 given.
template <int SIGN>
__device__ __forceinline__ void fft_pass8_one(const double2 *a, double2 *b, int lgn, int lgns, double2 w1) {
    const int nr = 1 << (lgn - 3);
    const int ns = 1 << lgns;
    const int j = threadIdx.x;
    if (j < nr) {
        const int k = j & (ns - 1);
        double2 v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = a[j + q * nr];
        if (lgns > 0) {
            double2 w[8];
            w[1] = w1;
            if (SIGN > 0) w[1].y = -w[1].y;
#pragma unroll
            for (int q = 2; q < 8; ++q) w[q] = cmul(w[q / 2], w[q - q / 2]);
#pragma unroll
            for (int q = 1; q < 8; ++q) v[q] = cmul(v[q], w[q]);
        }
        dft8<SIGN>(v);
        const int d = ((j - k) << 3) + k;
#pragma unroll
        for (int q = 0; q < 8; ++q) b[d + q * ns] = v[q];
    }
    __syncthreads();
}

// fft_lds for one transform of n <= 8 blockDim.x points with the twiddles of
// fft_twiddles (the same arithmetic in the same order).
template <int SIGN>
__device__ double2 *fft_lds_one(double2 *a, double2 *b, int lgn, const double2 *tw, int lgmax, const FftTw &f) {
    int lgns = lgn % 3;
    if (lgns == 1) fft_pass<SIGN, 1>(a, b, lgn, 1, 0, tw, lgmax);
    if (lgns == 2) fft_pass<SIGN, 2>(a, b, lgn, 1, 0, tw, lgmax);
    if (lgns) {
        double2 *t = a;
        a = b;
        b = t;
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        if (lgns < lgn) {
            fft_pass8_one<SIGN>(a, b, lgn, lgns, f.w[q]);
            double2 *t = a;
            a = b;
            b = t;
            lgns += 3;
        }
    }
    return a;
}

template <bool MIX>
__device__ __forceinline__ double acc_to_rho(typename AccOf<MIX>::T v, double scale, double add) {
    double w;
    if constexpr (MIX) w = (double)(int64_t)v;
    else w = v;
    return add + scale * w;
}

template <bool MIX>
__device__ __forceinline__ double acc_value(const typename AccOf<MIX>::T *acc, int64_t i, double scale, double add) {
    return acc_to_rho<MIX>(acc[i], scale, add);
}

}  // namespace
}  // namespace apic
