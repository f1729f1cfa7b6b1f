// Host-side context of libapic shared by the host translation units (the
// C-ABI entry points, the adjoint): the context object, its workspace layout
// and the helpers that launch the kernels for it. Not part of the public ABI.
#pragma once

#include "apic.h"
#include "apic_internal.h"

#include <hipfft/hipfft.h>

#include <string>
#include <vector>

struct apic_ctx {
    apic_grid_desc d;
    int64_t n;
    apic::Geo g;
    bool mixed;
    apic::CtxDev dev;
    void *dev_block = nullptr;
    hipfftHandle fwd = 0, inv = 0;
    bool have_fft = false;
    bool fused_fft = false;   // 2D periodic field solve by the fused three-launch path
    bool fused_fft3 = false;  // 3D periodic field solve by the fused transforms in LDS
    std::string err;
    // workspace layout (byte offsets)
    size_t o_x, o_y, o_z, o_cell, o_ox, o_oy, o_oz, o_vx, o_vy, o_vz;
    size_t o_keys, o_bstart, o_acc, o_rho, o_rhat, o_ehat;
    size_t o_jacc;    // electromagnetic step: J [2][3][G] (two buffers)
    size_t o_f2;      // electromagnetic step: the second field buffer [6][G]
    size_t o_e32;     // mixed electrostatic step in 2D and 3D: E between steps, binary32 [dim][G]
    size_t o_cnt, o_offs, o_farcnt, o_farcur, o_tot, o_deep;
    size_t o_keys2, o_idx, o_idx2, o_rcnt, o_roff, o_rpart;
    size_t ws_bytes;
    double dV, mass;
    // per-phase timing (apic_profile_enable)
    std::vector<hipEvent_t> ev;   // 5 events per profiled step
    int prof_max = 0, prof_used = 0;
    bool prof_all = true;          // events around every phase, or only around the push pass
    int prof_every = 1;            // events on one step in prof_every
    int64_t prof_step = 0;         // steps seen since profiling was armed
};

namespace apic_host {

using apic::Parts;
using apic::PushC;

apic_status fail(apic_ctx *c, apic_status st, const char *msg);
apic_status hip_fail(apic_ctx *c, hipError_t e, const char *where);

#define HIPCHK(ctx, expr)                                   \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

#define FFTCHK(ctx, expr)                                                    \
    do {                                                                     \
        hipfftResult r_ = (expr);                                            \
        if (r_ != HIPFFT_SUCCESS) {                                          \
            (ctx)->err = std::string(#expr) + " failed (" + std::to_string((int)r_) + ")"; \
            return APIC_EHIP;                                                \
        }                                                                    \
    } while (0)

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Pointer at a byte offset of the workspace (NULL for an absent array).
template <typename T>
T *wsp(void *ws, size_t off) {
    return off == (size_t)-1 ? nullptr : (T *)((char *)ws + off);
}

Parts parts_of(const apic_particles *p);
Parts parts_ws(const apic_ctx *c, void *ws);
apic_status check_parts(apic_ctx *c, const apic_particles *p, bool need_bstart);
PushC push_coeffs(const apic_ctx *c, double dt_scale, int move);
double acc_scale(const apic_ctx *c);
int64_t max_per_bucket(const apic_ctx *c);
apic_status field_from_acc(apic_ctx *c, void *acc, bool acc_is_rho, double *E, float *E32, double *diag,
                           double *we, double *charge, int npush, int clear, void *ws, hipStream_t s,
                           const int32_t *nlive = nullptr);
apic_status copy_parts(apic_ctx *c, const Parts &dst, const Parts &src, hipStream_t s);

}  // namespace apic_host
