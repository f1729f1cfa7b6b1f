// Internal declarations shared by the kernel and host translation units of
// libapic (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace apic {

// Error bits raised by kernels (OR-ed into a device word of the context).
enum : int {
    ERR_DOMAIN = 1,    // NaN/Inf or out-of-range particle coordinate
    ERR_ORDER = 2,     // particle outside the tile its bucket says / slot overflow
    ERR_OVERFLOW = 4,  // fixed-point node sums may exceed int64
    ERR_COUNT = 8,     // bucket totals differ from the particle count
};

// Grid geometry and bucket (tile) layout, passed to kernels by value.
struct Geo {
    int dim, vdim;
    int nx, ny, nz;       // nodes per axis (ny = 1 in 1D, nz = 1 below 3D)
    int tsx, tsy, tsz;    // log2 of the tile size in cells
    int nbx, nby, nbz;    // tiles per axis
    int nbuckets;
    int halo;             // deposit halo (cells) around a tile held in LDS
    int S;                // fixed-point weight bits per axis (mixed path)
    int np;               // number of particles (bounds for bucket tables)
    int hc;               // velocity advance: 0 Boris, 1 Higuera-Cary (u = gamma v)
    int em;               // field model: 0 electrostatic, 1 electromagnetic (Yee, FP64 2D3V)
    int walls;            // grounded absorbing walls at x = 0 and x = lx/2 (2D): nx, lx are then those of the
                          // odd extension (2 nxp nodes, length 2 Lx) and particles live in cells [0, nxp)
    int nxp;              // physical cells along x (nx without walls)
    double lx, ly, lz;
    double inv_dx, inv_dy, inv_dz;
    int push_vr;          // mixed electrostatic push build: 0 by resident workgroups, 1 plain, 2 VR
};

// Boris / move coefficients for one call (dt_eff = dt * dt_scale).
struct PushC {
    double a, t, s;       // a = (q/m) dt_eff / 2, t = a bz, s = 2t/(1+t^2)
    float af, tf, sf;
    double dt;            // position step (unscaled dt)
    float dtdx, dtdy, dtdz;  // dt/dx, dt/dy, dt/dz in binary32 (mixed path)
    float dtdx2, dtdy2;      // their squares (the deep test of a rotating push)
    int move;
    int rot;              // bz != 0 (the push rotates v in the x-y plane)
    float deep;           // slack (cells) that makes a staying particle "deep"
    double ic2;           // 1/c^2 (Higuera-Cary)
    float ic2f;
    double jx, jy, jz;    // current deposit: -Q/(dy dt), -Q/(dx dt), Q/(dx dy) (electromagnetic step)
};

// One particle buffer set (structure of arrays).
struct Parts {
    double *x, *y, *z;
    int32_t *cell;
    float *ox, *oy, *oz;
    void *vx, *vy, *vz;
};

// Exact-charge counter slots (see CtxDev::qacc).
constexpr int kQSlots = 64;
constexpr int kQStride = 16;   // 64-bit words per slot (a 128-byte line)

// Device scratch owned by the context.
struct CtxDev {
    int *err;             // error bits
    int *step;            // step index inside apic_step (device side)
    double *part_push;    // per-bucket (kinetic, momentum) partials [2 * nbuckets]
    double *part_spec;    // per-block field-energy partials [kMaxSpecBlocks]
    double *rho0;         // rho_hat(0) = sum_j rho_j of the last spectral solve
    double *kx2, *kapx;   // modified wavenumber tables, x: [nx/2+1]
    double *ky2, *kapy;   // y: [ny]
    double *kz2, *kapz;   // z: [nz]
    double *tw;           // fused 2D field solve: exp(-2 pi i k / nmax), k < nmax, interleaved (re, im)
    // exact charge of a fixed-point accumulation (mixed path): the launch that
    // converts the node sums adds (whole particles, remainder in units of
    // 2^-(S dim) particle) to qacc with integer atomics, spread over counter
    // slots; the diagnostics workgroup moves the normalised total to qexact
    // and clears the slots
    unsigned long long *qacc;   // [kQSlots * kQStride] (slot i: words 16 i, 16 i + 1)
    int64_t *qexact;            // [2]
};

// Field diagnostics of one solve: charge and W_E (and, with npush, the
// kinetic energy and momentum partials of the push) into diag[step] or
// we/charge.
struct FinArgs {
    int npush, nspec;
    double mass, dV, G, rho_ion;
    double *diag, *we, *charge;
    // walls: W_E of the physical half of the odd extension (with half weight
    // on the wall nodes) and the charge Q * (live particles) when nlive
    int walls;
    double q_macro;
    const int32_t *nlive;
    // S * dim when the solve converted fixed-point node sums (their exact
    // total is in CtxDev::qacc), 0 for an FP64 accumulation
    int sd;
};

constexpr int kMaxSpecBlocks = 16384;  // per-block partials of the field energies
// Waves per workgroup of the fused step passes (tally, offsets, push): one
// workgroup per bucket, so this sets the waves a tile's particles share.
// Measured at 512^2, 16.8M particles: 6 or 8 waves per bucket were slower
// than 4 at 16 x 16 tiles (push 239 / 219 us against 196 us) and within 1%
// of it at 32 x 16.
#ifndef APIC_STEP_WAVES
#define APIC_STEP_WAVES 4
#endif
constexpr int kSWaves = APIC_STEP_WAVES;
constexpr int kSBlock = 64 * kSWaves;
constexpr int kStepTab = 28;   // per-bucket direction table entries, at most (28 directions in 3D)
constexpr int kDeepTab = 2;    // per-bucket deep-range entries (start, count)

// ---- launchers (apic_kernels.hip) -----------------------------------------
// All return hipSuccess or the launch error.

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s);
hipError_t launch_set_step(int *step, int v, hipStream_t s);
hipError_t launch_copy_bytes(void *dst, const void *src, int64_t bytes, hipStream_t s);

// general sort (arbitrary input order): stable LSD radix sort of
// (bucket key, index), the bucket table of the sorted keys, then a gather of
// the arrays
hipError_t launch_keys_init(const Geo &g, bool mixed, const Parts &p, int64_t n, int32_t *keys,
                            int32_t *idx, const CtxDev &c, hipStream_t s);
int sort_chunks(int64_t n);
int sort_table_entries();
int sort_part_entries();
hipError_t launch_radix_pass(const int32_t *kin, const int32_t *iin, int32_t *kout, int32_t *iout,
                             int64_t n, int shift, int32_t *cnt, int32_t *off, int32_t *part,
                             const CtxDev &c, hipStream_t s);
hipError_t launch_bucket_table(const int32_t *sorted_keys, int64_t n, int nb, int32_t *start,
                               int64_t max_per_bucket, const CtxDev &c, hipStream_t s);
hipError_t launch_gather_parts(const Geo &g, bool mixed, const Parts &src, const Parts &dst, int64_t n,
                               const int32_t *idx, int32_t *perm, const CtxDev &c, hipStream_t s);

// deposit of current positions into acc (double weights or int64 sums)
hipError_t launch_deposit(const Geo &g, bool mixed, const Parts &p, int64_t n, const int32_t *bstart,
                          void *acc, const CtxDev &c, hipStream_t s);

// gather + Boris (+ move), in place; E is double (FP64) or float (mixed)
hipError_t launch_gather_push(const Geo &g, bool mixed, const Parts &p, int64_t n,
                              const int32_t *bstart, const void *E, const PushC &pc, const CtxDev &c,
                              hipStream_t s);

// fused step: direction tallies, scan into offsets, push + deposit + scatter
// deep: per (bucket, wave) the [start, count) range, relative to the bucket,
// of particles the previous push found deep inside their tile (written by
// launch_step_push, all zero when unknown).
// E32 (mixed path, may be NULL): the field already rounded to binary32, read
// in place of E.
hipError_t launch_step_count(const Geo &g, bool mixed, const Parts &p, const int32_t *bstart,
                             const double *E, const float *E32, const PushC &pc, int32_t *cnt, int32_t *tot,
                             int32_t *farcnt, const int32_t *deep, const CtxDev &c, hipStream_t s);
hipError_t launch_scan_dir(const Geo &g, int32_t *tot, int32_t *start, int64_t n, int64_t max_per_bucket,
                           int step_mode, const CtxDev &c, hipStream_t s);
// (with walls the total may fall below n: absorbed particles leave the order)
// first slot of every (source bucket, wave, direction) tally inside its
// destination bucket: offs has the layout of cnt
hipError_t launch_dest_offsets(const Geo &g, const int32_t *cnt, const int32_t *start, int32_t *offs,
                               hipStream_t s);
// The scan of the bucket totals and the offsets in one launch (when
// fused_scan_offsets(g)): tot is read, tot_next (the totals buffer of the
// next step) is cleared; otherwise launch_scan_dir + launch_dest_offsets.
bool fused_scan_offsets(const Geo &g);
hipError_t launch_scan_offsets(const Geo &g, const int32_t *tot, int32_t *tot_next, int32_t *start, int64_t n,
                               int64_t max_per_bucket, int step_mode, const int32_t *cnt, int32_t *offs,
                               const CtxDev &c, hipStream_t s);
hipError_t launch_step_push(const Geo &g, bool mixed, const Parts &src, const Parts &dst,
                            const int32_t *bstart, const int32_t *bstart_new, const int32_t *cnt,
                            const int32_t *offs, int32_t *farcnt, const double *E, const float *E32,
                            const PushC &pc, void *acc,
                            int32_t *perm, double *part, int32_t *deep, const CtxDev &c, hipStream_t s);

// field: accumulation buffer -> rho (FP64): rho = add + scale * acc
// (fixed-point sums with qacc set: their exact total is added to qacc)
hipError_t launch_rho(const Geo &g, bool mixed, void *acc, double *rho, double scale, double add,
                      int clear, unsigned long long *qacc, hipStream_t s);
// walls: rho of the odd extension along x: the physical interior nodes
// (add + scale acc), zero on the wall nodes, the negated mirror beyond
hipError_t launch_rho_odd(const Geo &g, bool mixed, void *acc, double *rho, double scale, double add, int clear,
                          unsigned long long *qacc, hipStream_t s);
int spectral_blocks(const Geo &g);
// phi_hat = rho_hat / K^2 (scaled for the inverse transform) and the field
// energy partials; then E = -(centred difference of phi) in real space
hipError_t launch_spectral(const Geo &g, const void *rho_hat, void *phi_hat, const CtxDev &c, hipStream_t s);
// (one extra workgroup of the same launch reduces the field diagnostics)
hipError_t launch_grad(const Geo &g, const double *phi, double *E, float *E32, const FinArgs &f,
                       const CtxDev &c, hipStream_t s);

// Fused periodic 2D field solve (apic_fft.hip): power-of-two nx, ny in
// [4, kFusedFftMax], walls included (nx the extended grid). acc -> rho (acc
// cleared when clear) -> E [2][G] (+ E32) and the diagnostics of f (nspec is
// set by the launcher). H: [ny][nx/2+1] complex, Z: [ny][nx] complex
// scratch. tw: the twiddle table of CtxDev for nmax = max(nx, ny).
constexpr int kFusedFftMax = 1024;
bool fused_fft_supported(int dim, int nx, int ny, int nz);
hipError_t launch_fused_field(const Geo &g, bool mixed_acc, void *acc, double scale, double add, int clear,
                              void *H, void *Z, double *E, float *E32, const double *tw, const FinArgs &f,
                              const CtxDev &c, hipStream_t s);
// Fused periodic 3D field solve (apic_fft3.hip): power-of-two nx, ny, nz in
// [4, kFusedFft3Max]. acc -> rho (acc cleared when clear; with qacc, the
// fixed-point node sums' exact total is added to it) -> phi (FP64 [G]) with
// the field-energy partials of fused_fft3_spec_blocks(g) workgroups in
// part_spec; E follows from phi by launch_grad. A: [nz][nx/2+1][ny] and B:
// [nx/2+1][ny][nz] complex scratch. tw: the twiddle table of CtxDev for
// nmax = max(nx, ny, nz).
constexpr int kFusedFft3Max = 256;
bool fused_fft3_supported(int dim, int nx, int ny, int nz);
int fused_fft3_spec_blocks(const Geo &g);
hipError_t launch_fused_field3(const Geo &g, bool mixed_acc, void *acc, double scale, double add, int clear,
                               void *A, void *B, double *phi, const double *tw, unsigned long long *qacc,
                               const CtxDev &c, hipStream_t s);
hipError_t launch_finalize(int npush, int nspec, double mass, double dV, double G, double rho_ion,
                           double *diag, double *we, double *charge, const CtxDev &c, hipStream_t s);
hipError_t launch_field1d(const Geo &g, bool mixed, void *acc, double scale, double add, double ion,
                          double dx, int clear, double *E, float *E32, double *we_out,
                          double *charge_out, int step_mode, double q_macro, const CtxDev &c, hipStream_t s);

// ---- electromagnetic step (FP64 2D3V, Yee grid; F = [6][G], J = [3][G]) ----
// F^0 from the potential phi [G]: (Ex, Ey) = -(forward differences of phi),
// Ez = Bx = By = 0, Bz = bz
hipError_t launch_em_init(const Geo &g, const double *phi, double bz, double *F, hipStream_t s);
// gather E, B + Boris (+ move), in place (no ordering needed)
hipError_t launch_em_gather_push(const Geo &g, bool mixed, const Parts &p, int64_t n, const double *F,
                                 const PushC &pc, const CtxDev &c, hipStream_t s);
// The whole field update of a step in one launch: reads F [6][G] and J
// [3][G], writes Fn [6][G] (a buffer other than F), clears Jnext [3][G] (the
// next step's current) and copies J to Jout when not NULL. With diag, one
// workgroup then writes diag[step] = (c^2/2 dV sum |B - B0|^2, 1/2 dV sum
// |E|^2, kinetic, momentum) from the field partials and the push partials.
hipError_t launch_fdtd_step(const Geo &g, const double *F, double *Fn, const double *J, double *Jnext, double *Jout,
                            double dt, double c2, double bz, double dV, double mass, int npush, double *diag,
                            const CtxDev &c, hipStream_t s);

}  // namespace apic
