/*
 * apic -- MI355X (gfx950) particle-in-cell coupling loop, C ABI.
 *
 * The loop is the electrostatic PIC cycle of the AlgoPlasma paper: its
 * "Core functionality" section names the modules (B_Scatter deposits particle
 * charge onto the grid, D_Poisson solves for the potential and evaluates E,
 * C_Gather interpolates E to the particles, A_Pusher advances velocities with
 * the Boris pusher), and the two-stream example's application driver fixes the
 * order (field of the initial charge, initial half push, then per step: full
 * push, position update with periodic boundaries, deposit, field). The paper
 * leaves data structures and execution order to the caller; so does this ABI:
 * every particle, grid and workspace array is allocated and owned by the
 * caller, and the library owns only its context (FFT plans, graph cache,
 * a few device words for error flags).
 *
 * Conventions shared by all entry points
 *   - Pointers marked [dev] are device (HBM) pointers on the current HIP
 *     device; [host] are host pointers. No entry point allocates device memory
 *     after apic_create / apic_batch_create, except the autotuning setup calls
 *     (apic_autotune_tiles, apic_batch_autotune_chunk).
 *   - All work is enqueued asynchronously on the given hipStream_t (pass the
 *     stream as void*; NULL = default stream). Argument errors are detected on
 *     the host and returned synchronously, before anything is enqueued.
 *     Errors found by kernels (a NaN/out-of-range particle, fixed-point
 *     headroom exceeded, an inconsistent bucket table) set a device flag that
 *     apic_sync_status() reads.
 *   - Units are the caller's (the reference workloads use omega_pe = 1,
 *     eps0 = 1, q/m = -1 for electrons).
 *   - Grids are periodic and node-centred: node j sits at X_j = j*dx.
 *     2D grid arrays are row-major [ny][nx]; a vector field is [dim][ny][nx].
 *     3D grid arrays are [nz][ny][nx]; a vector field is [3][nz][ny][nx].
 *     The 3D3V forms are the Cartesian three-dimensional scatter, gather and
 *     Boris routines the paper's two-stream driver calls (B01, C01, A01 in
 *     their "3Dxyz" form) with the 7-point finite-difference Poisson solve.
 *   - Return value: APIC_OK or a negative apic_status. No C++ exception
 *     crosses the ABI. apic_last_error() gives a message for the last failure.
 */
#ifndef APIC_H
#define APIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    APIC_OK = 0,
    APIC_EINVAL = -1,        /* bad argument (host-side check)                 */
    APIC_EHIP = -2,          /* a HIP / hipFFT call failed                     */
    APIC_ENOMEM = -3,        /* context allocation failed (apic_create only)   */
    APIC_EOVERFLOW = -4,     /* fixed-point deposit headroom exceeded          */
    APIC_EDOMAIN = -5,       /* NaN/Inf or out-of-range particle, or particles
                                not ordered as the bucket table says           */
    APIC_EUNSUPPORTED = -6   /* valid but not implemented combination          */
} apic_status;

/* Velocity advance (the paper's A_Pusher lists both). */
typedef enum {
    APIC_BORIS = 0,          /* Boris (1970); the state's velocities are v     */
    APIC_HIGUERA_CARY = 1    /* Higuera & Cary (2017), relativistic; the state's
                                velocities are u = gamma v, gamma =
                                sqrt(1 + |u|^2/c^2), and the move uses u/gamma.
                                Needs vdim = 3                                 */
} apic_pusher;

/* Field model (the paper's D_Poisson or E_Maxwell). */
typedef enum {
    APIC_ELECTROSTATIC = 0,  /* periodic Poisson solve each step (apic_step)  */
    APIC_ELECTROMAGNETIC = 1 /* Yee FDTD update with a charge-conserving
                                current deposit (apic_em_step); 2D3V, either
                                precision, Boris, c_light > 0 with the Courant
                                condition c dt sqrt(1/dx^2 + 1/dy^2) < 1     */
} apic_field_model;

typedef enum {
    APIC_FP64 = 0,  /* positions x,y in [0,L) and velocities as double          */
    APIC_MIXED = 1  /* cell index + binary32 in-cell offset, binary32 velocity,
                       int64 fixed-point deposit, FP64 field solve             */
} apic_precision;

/* One periodic plasma (one replica). */
typedef struct {
    int dim;              /* 1, 2 or 3 spatial dimensions                       */
    int vdim;             /* velocity components: 1 (dim 1), 2 or 3 (dim 2),
                             3 (dim 3)                                          */
    int nx, ny;           /* grid nodes per axis (ny = 1 when dim = 1); 2D
                             grids need nx, ny <= 32768                         */
    double lx, ly;        /* box lengths (ly ignored when dim = 1)              */
    double dt;            /* time step                                          */
    double qm;            /* charge-to-mass ratio of the particles              */
    double q_macro;       /* charge of one macro-particle; 0 selects the
                             neutralising charge -rho_ion * V / n (V the box
                             volume lx ly lz of the dimensions present, n the
                             particle count), the ion background of the
                             paper's two-stream example balanced by n equal
                             electrons; apic_q_macro() reports the value used  */
    double rho_ion;       /* uniform immobile background charge density         */
    double bz;            /* uniform magnetic field along z (needs vdim >= 2)   */
    apic_precision prec;
    int frac_bits;        /* mixed path: S, fixed-point weight bits per axis;
                             1..32 in 1D, 1..23 in 2D, 1..16 in 3D; 0 selects
                             32 (dim 1), 20 (dim 2) or 15 (dim 3)               */
    int tile_x, tile_y;   /* sort bucket = tile of tile_x * tile_y (* tile_z)
                             cells, powers of two; 0 selects the default for
                             the grid. A side longer than its axis is cut to
                             the largest power of two that fits. The fused
                             push's LDS (E tile + deposit region with a
                             one-cell halo) must fit 64 KiB                     */
    int nz;               /* 3D: grid nodes along z, 2..1024 (nx, ny <= 1024
                             too); 0 or 1 below 3D                              */
    double lz;            /* 3D: box length along z                             */
    int tile_z;           /* 3D: bucket tile size along z (0 = default)         */
    int pusher;           /* apic_pusher (0 = Boris)                            */
    double c_light;       /* speed of light (> 0) for APIC_HIGUERA_CARY and for
                             APIC_ELECTROMAGNETIC (either pusher)               */
    int model;            /* apic_field_model (0 = electrostatic)               */
    int walls_x;          /* 1: grounded absorbing walls at x = 0 and x = lx
                             (2D electrostatic; see "walls" below); 0: periodic */
} apic_grid_desc;

/* Particle arrays (structure of arrays), all [dev], caller-owned, length n.
 * FP64 path : x (and y when dim >= 2, z when dim = 3) are double positions
 *             in [0, L); vx, vy, vz are double.
 * MIXED path: cell is the packed cell word: ix in 1D, (iy << 16) | ix in 2D,
 *             (iz << 20) | (iy << 10) | ix in 3D; ox (and oy, oz) are binary32
 *             offsets in [0,1) in cell units; vx, vy, vz are float.
 * Unused components (y/oy in 1D, z/oz below 3D, vy when vdim = 1, vz when
 * vdim < 3) are NULL.
 * bucket_start [dev, int32, apic_num_buckets()+1] describes the current order:
 *             particles of bucket b occupy [bucket_start[b], bucket_start[b+1]).
 *             Written by apic_sort_by_cell and apic_step; read by apic_deposit,
 *             apic_gather_push and apic_step. NULL in apic_deposit /
 *             apic_gather_push selects the unsorted (untiled) kernels.
 * perm        [dev, int32, n] optional output of apic_sort_by_cell:
 *             sorted[i] = unsorted[perm[i]]. NULL = not written.
 * n may be 0 (an empty plasma: the particle arrays are not read and may be
 * NULL; the charge is the ion background alone and E stays zero). */
typedef struct {
    int64_t n;
    double *x, *y;
    int32_t *cell;
    float *ox, *oy;
    void *vx, *vy, *vz;
    int32_t *bucket_start;
    int32_t *perm;
    double *z;            /* 3D, FP64 path */
    float *oz;            /* 3D, mixed path */
} apic_particles;

typedef struct apic_ctx apic_ctx;

/* Create a context for one plasma of n_particles particles: validates the
 * descriptor, builds the FFT plans for 2D grids and allocates the context's
 * own small device words. Returns APIC_EINVAL for an invalid descriptor. */
apic_status apic_create(const apic_grid_desc *desc, int64_t n_particles, apic_ctx **out);
void apic_destroy(apic_ctx *ctx);

/* Bytes of caller-provided device workspace that apic_sort_by_cell and
 * apic_step need (second particle buffer, bucket counters, deposit and FFT
 * buffers). The workspace must stay untouched between calls that share it
 * only in that the library does not rely on its contents across calls. */
apic_status apic_workspace_size(const apic_ctx *ctx, size_t *bytes);

/* Number of sort buckets (tiles) of the context's grid. */
int64_t apic_num_buckets(const apic_ctx *ctx);

/* Fixed-point bits S the context uses (mixed path). */
int apic_frac_bits(const apic_ctx *ctx);

/* Charge of one macro-particle the context uses (the descriptor's q_macro, or
 * its neutralising default); NaN for a NULL context. */
double apic_q_macro(const apic_ctx *ctx);

/* Side, in cells, of the context's sort-bucket tile along axis 0 (x), 1 (y)
 * or 2 (z): 1 along an axis the grid does not have, -1 for a NULL context or
 * another axis. */
int apic_tile_size(const apic_ctx *ctx, int axis);

/* Counting sort of the particles by bucket: key = tile-major bucket of each
 * particle's cell; stable radix passes (tallies, exclusive scan, scatter),
 * the bucket table read off the sorted keys, a gather. Particles end up
 * ordered by ascending bucket, in place; bucket_start is written; perm is
 * written when non-NULL. The order inside a bucket is unspecified. The paper
 * leaves the particle data structures to the application ("Example setup and
 * implementation"); this order is the library's choice, so that the deposit
 * and the gather of one bucket touch one tile of the grid. */
apic_status apic_sort_by_cell(apic_ctx *ctx, apic_particles *p, void *ws, void *stream);

/* Charge deposit of the particles' current positions: the paper's B_Scatter
 * ("Core functionality", particle-grid coupling; module B01 of the two-stream
 * example) with cloud-in-cell (bilinear; linear in 1D, trilinear in 3D)
 * weights.
 * FP64 : rho [dev, double, G] is overwritten with
 *        rho_ion + (q_macro/dV) * sum_p W_j(x_p).
 * MIXED: rho [dev, int64, G] is overwritten with the fixed-point node sums
 *        I_j = sum_p w_pj, w = products of round-half-even(o * 2^S) weights;
 *        each particle contributes exactly 2^(S*dim) (exact, order-free).
 * G = nx*ny. With p->bucket_start set the particles must be bucket-ordered
 * (LDS-tiled kernel); with NULL any order is accepted. */
apic_status apic_deposit(apic_ctx *ctx, const apic_particles *p, void *rho, void *stream);

/* Periodic Poisson solve and field: the paper's D_Poisson ("Core
 * functionality"; modules D02, D05 and D06 of the two-stream example solve
 * for phi and form E). -lap_h phi = rho with the 3-point (1D) / 5-point (2D)
 * / 7-point (3D) finite-difference Laplacian, mean-free phi, and
 * E = -(centred difference of phi), solved by FFT on the periodic grid.
 * rho  [dev]: double [G] (FP64) or int64 fixed-point sums [G] (MIXED; converted
 *             with rho_ion + q_macro * I * 2^(-S*dim) / dV).
 * E    [dev, double, dim*G] output.
 * E32  [dev, float, dim*G] output copy for the mixed gather; may be NULL.
 * we   [dev, double, 1] output field energy 1/2 sum |E|^2 dV; may be NULL. */
apic_status apic_field_solve(apic_ctx *ctx, const void *rho, double *E, float *E32, double *we,
                             void *ws, void *stream);

/* Gather + velocity advance [+ position update]: the paper's C_Gather and
 * A_Pusher ("Core functionality"; modules C01 and A01 of the two-stream
 * example), then the position update with periodic boundaries that the
 * example's application code performs ("Example setup and implementation").
 * E [dev]: double [dim*G] (FP64) or float [dim*G] (MIXED).
 * The velocity advances by dt * dt_scale (dt_scale = -0.5 gives the initial
 * backward half push, a7). move != 0 then advances positions by dt (not
 * scaled) with periodic wrap. With p->bucket_start set, particles must be
 * bucket-ordered (E tile staged in LDS). */
apic_status apic_gather_push(apic_ctx *ctx, apic_particles *p, const void *E, double dt_scale,
                             int move, void *stream);

/* nsteps full PIC cycles in the order of the paper's two-stream driver
 * ("Example setup and implementation": full push, move with periodic
 * boundaries, then the field update of deposit and Poisson solve), with the
 * energy diagnostics its "Results and validation" section tracks, from the
 * leapfrog state (x^n, v^{n-1/2}),
 * bucket-ordered with a valid bucket_start, and the field E^n:
 *   gather E^n -> Boris -> move -> deposit rho^{n+1} -> counting sort ->
 *   Poisson -> E^{n+1}.
 * rho  [dev] optional output (NULL = none): the last step's deposit, in the
 *        format of apic_deposit (FP64 rho, or the int64 fixed-point sums).
 * E    [dev]: double [dim*G] in/out (E^n in, E^{n+nsteps} out). The mixed path
 *        rounds E to binary32 as it stages each tile for the gather.
 * E32  [dev]: optional float [dim*G] output (NULL = none): E^{n+nsteps} rounded
 *        to binary32.
 * diag [dev, double, nsteps*4] per step k (time level n+k -> n+k+1):
 *        [0] total deposited charge at n+k+1: FP64 path sum_j (rho_j - rho_ion)
 *            dV; mixed path q_macro times the exact integer total of the
 *            fixed-point node sums (see apic_charge_exact), which is
 *            q_macro * n bit for bit when every particle deposited its 2^(S*dim)
 *        [1] field energy W_E at n+k+1
 *        [2] kinetic energy at n+k: M/2 * sum_p (|v^{-}|^2 + |v^{+}|^2)/2
 *            with M = q_macro/qm
 *        [3] x-momentum M * sum_p vx^{n+k+1/2}
 *      may be NULL.
 * p->perm [dev, int32, n] optional: the last step's reordering,
 *        after[i] = before_last_step[perm[i]].
 * On return the particles are again bucket-ordered (bucket_start updated).
 * The order inside each bucket is a function of the previous order only
 * (slots come from per-bucket tallies, not from atomics), so repeated runs
 * give identical bits; the one exception is a particle that jumps more than
 * one tile in a step, which takes a slot at the end of its bucket in arrival
 * order. Workspace contents are not relied on across calls. */
apic_status apic_step(apic_ctx *ctx, apic_particles *p, void *rho, double *E, float *E32, int nsteps,
                      double *diag, void *ws, void *stream);

/* apic_step with a second, caller-owned particle buffer q (the same arrays
 * as p, bucket_start included, none shared with p) in place of the
 * workspace's: the steps alternate between p and q, and the call ends with
 * the state in q when nsteps is odd (*in_q = 1 [host]) and in p when it is
 * even (*in_q = 0), where apic_step copies an odd count's result back into p.
 * Saves that copy, a read and a write of every particle array, for callers
 * that step a few steps at a time (diagnostics between calls): the next
 * call passes the two buffers the other way round. The buffer that does not
 * hold the state is left with unspecified contents; q's content on entry is
 * not read. perm and the outputs are as in apic_step (perm from p). */
apic_status apic_step_pair(apic_ctx *ctx, apic_particles *p, apic_particles *q, void *rho, double *E, float *E32,
                           int nsteps, double *diag, int *in_q, void *ws, void *stream);

/* apic_step without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation). The workspace is a fixed array of
 * APIC_STATIC_WS_BYTES bytes inside the library, one per GPU the library runs
 * on (held until the process ends); the call allocates nothing and otherwise
 * behaves as apic_step with that array as ws (the same kernels, results and
 * errors). Returns APIC_EINVAL, with a message, when the context's workspace
 * (apic_workspace_size) exceeds the array, and APIC_EUNSUPPORTED for 3D
 * contexts and 2D grids whose sides are not powers of two in [4, 1024] (their
 * field solve goes through the FFT library). Every call on one GPU uses that
 * GPU's one array, so calls that overlap on one GPU (other streams, other
 * threads, other contexts) race; the array keeps the last call's contents,
 * and each call clears what it needs cleared. */
#define APIC_STATIC_WS_BYTES (64u << 20)
apic_status apic_step_static(apic_ctx *ctx, apic_particles *p, void *rho, double *E, float *E32, int nsteps,
                             double *diag, void *stream);

/* Per-phase timing of apic_step with HIP events recorded on the caller's
 * stream around each phase of each step (count pass, scan, push pass, field
 * solve). apic_profile_enable(ctx, max_steps) creates the events (host call,
 * not for capture; max_steps = 0 disables); apic_profile_read waits for the
 * last event and returns the summed milliseconds per phase in ms[4] and the
 * number of profiled steps, then rearms. Steps beyond max_steps are not timed. */
apic_status apic_profile_enable(apic_ctx *ctx, int max_steps);
apic_status apic_profile_read(apic_ctx *ctx, double ms[4], int *steps);

/* Which events apic_step records while profiling: all != 0 (the default) the
 * five per step above; all = 0 only the two around the push pass (ms[2];
 * the other phases read 0). Every recorded event makes the queue finish the
 * work before it, which costs time between kernels (about 16 us per step
 * with all five at 512^2, 16.8M particles), so a throughput measurement
 * records only the push pass. Discards the steps profiled so far. */
apic_status apic_profile_phases(apic_ctx *ctx, int all);

/* Profile one step in every `every` (>= 1; 1, the default, profiles each
 * step up to max_steps): the events are recorded on steps 0, every,
 * 2 every, ... of the calls after this one (counted from the last
 * apic_profile_enable, apic_profile_phases, apic_profile_every or
 * apic_profile_read), so that a throughput run pays their cost on a sample
 * of its steps only. Discards the steps profiled so far; APIC_EINVAL for
 * every < 1. */
apic_status apic_profile_every(apic_ctx *ctx, int every);

/* Convert a physical FP64 state to the context's particle representation (any
 * order): x, y, z [dev, double, n] positions (y NULL in 1D, z NULL below 3D),
 * vx, vy, vz [dev, double, n] velocities (NULL beyond vdim). FP64 path: copies
 * into p->x, p->y, p->z, p->vx.. ; mixed path: p->cell = floor(x/dx) (mod nx;
 * packed with iy in 2D, with iy and iz in 3D), p->ox = binary32(x/dx -
 * floor(x/dx)), an offset that rounds to 1 moving to the next cell with offset
 * 0, velocities rounded to binary32. Positions must lie in [0, L] (L is node
 * 0); a coordinate outside raises APIC_EDOMAIN at the next apic_sync_status.
 * Periodic contexts only (APIC_EUNSUPPORTED with walls). p->bucket_start and
 * p->perm are not touched. */
apic_status apic_import_state(apic_ctx *ctx, const double *x, const double *y, const double *z, const double *vx,
                              const double *vy, const double *vz, apic_particles *p, void *stream);

/* ---- adjoint ----------------------------------------------------------------
 * Gradient of the final field energy W = 1/2 sum_j |E_j^T|^2 dV of an
 * nsteps-step run with respect to every particle's initial position and
 * velocity (reverse-mode derivative of the discrete cycle; the paper has no
 * adjoint). The run is the cycle of the two-stream driver: sort, deposit,
 * Poisson -> E^0, backward half push v^0 -> v^{-1/2}, then nsteps apic_step
 * cycles. Reverse of each step: move (lam_v += dt lam_x), Boris (transpose of
 * its linear map in (v, E_p)), gather (adjoint = scatter of lam_Ep into a grid
 * lam_E, plus the field-slope term), Poisson (lam_rho = A^T lam_E, the same
 * FFT solve with the conjugate symbol), deposit (adjoint = gather of the slope
 * of lam_rho), sort (each step's permutation inverted). The derivative of the
 * CIC hat is its slope inside the particle's cell.
 *
 * With the Higuera-Cary advance (vdim = 3, state u = gamma v) the reverse of the
 * advance is the transpose of its Jacobian at the step's own velocity (the
 * advance is nonlinear in u through gamma), and the move's is
 * lam_u += dt (I - u u^T / (c^2 gamma^2)) lam_x / gamma; lam_vx, lam_vy and
 * lam_vz are then derivatives with respect to u^0.
 *
 * In 3D (trilinear weights, the 7-point solve) the same steps run with a
 * third position component and E_z kicking v_z; lam_Ep is then scattered to
 * the grid with global FP64 atomics rather than through per-tile LDS. The
 * electromagnetic model and absorbing walls return APIC_EUNSUPPORTED.
 *
 * Step checkpointing: apic_adjoint_forward stores the state every `stride`
 * steps in the caller's checkpoint buffer; apic_step_adjoint recomputes one
 * segment of at most `stride` steps at a time from its checkpoint and walks it
 * backwards. Memory: ckpt_bytes ~ (nsteps/stride + 1) states; ws_bytes holds
 * the context workspace plus `stride` per-step snapshots (positions, sort
 * permutation, E, and with Higuera-Cary the velocities) and the lam arrays.
 *
 * Precision: the mixed path runs the per-particle adjoint in binary32, the
 * FP64 path in FP64; grid adjoints are FP64 in both (accumulated with atomics,
 * so FP64 gradients are reproducible to rounding, not bitwise). */

/* Bytes of the checkpoint buffer and of the adjoint workspace. */
apic_status apic_adjoint_sizes(const apic_ctx *ctx, int nsteps, int stride, size_t *ckpt_bytes, size_t *ws_bytes);

/* Forward run with checkpoints. p0: the initial state (x^0, v^0) in the
 * context's representation, any order, read only (bucket_start and perm
 * ignored). ckpt [dev, ckpt_bytes], ws [dev, ws_bytes]: caller-owned.
 * W [dev, double, 1]: W_E(T), may be NULL. E_out [dev, double, dim*G]: E^T,
 * may be NULL. nsteps >= 0, stride >= 1. */
apic_status apic_adjoint_forward(apic_ctx *ctx, const apic_particles *p0, int nsteps, int stride, void *ckpt,
                                 double *W, double *E_out, void *ws, void *stream);

/* Reverse sweep over the checkpoints of the last apic_adjoint_forward with the
 * same nsteps and stride (ws contents between the two calls are not needed).
 * Writes seed * dW/d(state at t = 0) in the input order of p0, as FP64:
 * lam_x, lam_y, lam_z [dev, n] (lam_y NULL in 1D, lam_z NULL below 3D) with
 * respect to positions,
 * lam_vx, lam_vy, lam_vz [dev, n] (NULL beyond vdim) with respect to v^0.
 * grad_delta0 [dev, double, 1] (NULL = not computed): seed * dW/d delta0 for
 * the mode seeding of the paper's two-stream example ("Example setup and
 * implementation": every particle displaced by delta0 k/|k|^2 sin(k.x_u)),
 * i.e. sum_p lam_x[p] dx_ddelta0[p] + lam_y[p] dy_ddelta0[p], with
 * dx_ddelta0, dy_ddelta0 [dev, double, n] the derivative of each initial
 * position with respect to delta0 in the same order (dy NULL in 1D; the mode
 * has no z component, so a 3D seeding moves x and y only; the
 * caller knows its unperturbed positions x_u, the library does not); summed
 * in a fixed order on the device. */
apic_status apic_step_adjoint(apic_ctx *ctx, const void *ckpt, int nsteps, int stride, double seed, double *lam_x,
                              double *lam_y, double *lam_z, double *lam_vx, double *lam_vy, double *lam_vz,
                              const double *dx_ddelta0, const double *dy_ddelta0, double *grad_delta0, void *ws,
                              void *stream);

/* ---- walls: non-periodic Poisson with absorbing walls -----------------------
 * The paper's D_Poisson solves Poisson under general boundary conditions
 * (through HYPRE). A 2D electrostatic context created with walls_x = 1 has
 * grounded (phi = 0) walls at x = 0 and x = lx that absorb particles, and
 * stays periodic in y:
 *   - nodes X_i = i dx, i = 0..nx along x (dx = lx/nx); every grid array
 *     (rho, E, the fixed-point sums) has rows of 2 nx entries: entries
 *     0..nx are the physical nodes (0 and nx on the walls), the others the
 *     odd mirror the solver uses, so arrays are [ny][2 nx] and the context's
 *     G is 2 nx ny;
 *   - the field solves -lap(phi) = rho on the interior nodes with phi = 0 on
 *     the walls (5-point FD operator), exactly, as the periodic solve of the
 *     odd extension of rho (a type-I sine transform along x); E is the
 *     centred difference inside and the one-sided difference on the walls;
 *   - a particle whose move takes it to x < 0 or x >= lx is absorbed: it gets
 *     no slot in the next order, so apic_step leaves bucket_start[nb] (the
 *     live count) below n and the entries beyond it unused; the diagnostics
 *     then report charge = q_macro * live count, W_E = 1/2 dV sum w |E|^2
 *     over the physical nodes with w = 1/2 on the wall nodes, and the
 *     kinetic energy of every particle pushed in the step;
 *   - the tile along x divides nx (the walls are tile edges); particles must
 *     start inside [0, lx) (apic_sort_by_cell flags others with
 *     APIC_EDOMAIN);
 *   - the tiled forms of apic_deposit and apic_gather_push follow
 *     bucket_start; their untiled forms treat all n entries as particles.
 * 3D, 1D, the electromagnetic model, the adjoint and the tuner do not take
 * walls (APIC_EUNSUPPORTED). */

/* ---- electromagnetic step --------------------------------------------------
 * The paper lists B_Scatter of current densities and E_Maxwell
 * ("finite-difference time-domain updates", citing Yee 1966) among its
 * modules. A context created with model = APIC_ELECTROMAGNETIC runs the
 * electromagnetic PIC cycle on the same sorted, tiled particle layout, 2D3V,
 * on a periodic Yee grid in normalised units eps0 = 1, mu0 = 1/c^2
 * (c = c_light). The FP64 path pushes in FP64; the mixed path keeps its
 * particle representation (cell + binary32 offsets and velocities) and runs
 * the field tile, gather, velocity advance and the current weights in
 * binary32, the displacement of the current deposit being the binary32
 * product its move adds; the current sums, the field update and F stay FP64
 * in both. The velocity advance is Boris, or with pusher =
 * APIC_HIGUERA_CARY the general-field Higuera-Cary advance of u = gamma v,
 * the move and the current then using u / gamma (the same quotient):
 *   - F [dev, double, 6*G] holds Ex, Ey, Ez, Bx, By, Bz, each [ny][nx], with
 *     element [j][i] of Ex at ((i+1/2) dx, j dy), Ey at (i dx, (j+1/2) dy),
 *     Ez at (i dx, j dy), Bx at (i dx, (j+1/2) dy), By at ((i+1/2) dx, j dy)
 *     and Bz at ((i+1/2) dx, (j+1/2) dy); B includes the uniform bz (the grid
 *     Bz starts at bz and the update keeps a uniform field);
 *   - J [dev, double, 3*G]: Jx, Jy, Jz at the Ex, Ey, Ez locations;
 *   - one step: E and B interpolated to x^n (linear weights on each
 *     component's own staggered lattice), the advance v^{n-1/2} -> v^{n+1/2}
 *     in that E and B, move with periodic wrap, the current J^{n+1/2} of the move by the
 *     charge-conserving scheme of Esirkepov (2001) for the linear shape
 *     (a displacement of a cell or more along an axis is an APIC_EDOMAIN
 *     error), counting sort into the next bucket order, then
 *     B^{n+1/2} = B^n - dt/2 curl E^n, E^{n+1} = E^n + dt (c^2 curl B^{n+1/2}
 *     - J^{n+1/2}), B^{n+1} = B^{n+1/2} - dt/2 curl E^{n+1} (Yee leapfrog with
 *     B also held at integer times).
 * The discrete continuity equation holds for the CIC charge of the same
 * particles, so a field that satisfies Gauss's law at the start keeps it.
 * The electrostatic entry points (apic_step, apic_gather_push,
 * apic_field_solve, the adjoint and the tuner) return APIC_EUNSUPPORTED on an
 * electromagnetic context; apic_sort_by_cell and apic_deposit (charge) work
 * as for an electrostatic one. */

/* F^0: E as the staggered gradient -(phi(i+1) - phi(i))/d of the periodic
 * Poisson potential of the particles' charge (5-point Laplacian, so the
 * discrete Gauss law div E = rho holds), Ez = Bx = By = 0, Bz = bz. p sorted
 * (bucket_start valid) or not; ws: the context workspace. */
apic_status apic_em_init_fields(apic_ctx *ctx, const apic_particles *p, double *F, void *ws, void *stream);

/* E and B gathered at each particle, the context's velocity advance by
 * dt_scale * dt (the initial backward half push uses -0.5), then the move
 * when move != 0; in place, any order. */
apic_status apic_em_gather_push(apic_ctx *ctx, apic_particles *p, const double *F, double dt_scale, int move,
                                void *stream);

/* nsteps electromagnetic cycles from (x^n, v^{n-1/2}, F^n); p sorted by
 * bucket on entry and on exit (as apic_step), perm as apic_step. F is updated
 * in place. J [dev, double, 3*G] or NULL: J^{n+1/2} of the last step.
 * diag [dev, double, nsteps*4] or NULL: per step (W_B, W_E, kinetic energy,
 * x-momentum) with W_B = c^2/2 dV sum |B - bz z|^2 and W_E = 1/2 dV sum |E|^2
 * of F^{n+1}, the kinetic energy the mean over v^{n-1/2} and v^{n+1/2} as in
 * apic_step. */
apic_status apic_em_step(apic_ctx *ctx, apic_particles *p, double *F, double *J, int nsteps, double *diag,
                         void *ws, void *stream);

/* ---- batched replicas -------------------------------------------------------
 * The paper's modules serve any composition of small and large runs ("Core
 * functionality": components assembled at different levels of complexity);
 * this form fills the GPU with many small ones. Many independent 1D1V
 * periodic electrostatic plasmas ("replicas") with
 * their own grid and particle counts, advanced together. Each replica is the
 * single-plasma mixed-precision cycle (binary32 push of cell + offset
 * positions, int64 fixed-point CIC deposit with S = 32, FP64 1D field solve)
 * and gives the bits it gives alone. One persistent kernel launch per step
 * (replayed from a captured HIP graph): workgroups pull (replica, chunk)
 * items from a work counter, stage the replica's whole grid in LDS, and the
 * workgroup that finishes a replica's last chunk solves its field. Particles
 * keep their order (no sort: each replica's grid fits in LDS).
 * Every replica is a neutral electron plasma: q_macro = -rho_ion * lx / n.
 * A replica with n = 0 is the ion background alone: q_macro = 0, its field
 * stays zero to rounding and its diagnostics are zero. */
typedef struct {
    int nx;          /* grid nodes, 2..1024                                    */
    int64_t n;       /* particles                                              */
    double lx;       /* box length                                             */
} apic_replica;

typedef struct apic_batch apic_batch;

/* Packed state of all replicas, [dev], caller-owned: replica r owns particles
 * [part_off[r], part_off[r+1]) and grid nodes [grid_off[r], grid_off[r+1]).
 * cell: int32 cell index, ox: binary32 offset in [0,1), vx: binary32 velocity;
 * E: double node field (E^n in, E^{n+k} out). */
typedef struct {
    int32_t *cell;
    float *ox;
    float *vx;
    double *E;
} apic_batch_state;

/* chunk: particles per work item (0 = 8192; at most 65535, larger values are
 * clamped; at least 256). Fails with APIC_EINVAL for an
 * invalid replica (nx outside 2..1024, n < 0, lx <= 0) or a total particle
 * count above INT32_MAX - 1. Allocates the context's device tables. */
apic_status apic_batch_create(const apic_replica *reps, int nrep, double dt, double qm, double rho_ion, int chunk,
                              apic_batch **out);
void apic_batch_destroy(apic_batch *b);
/* Totals and the workspace size (int64 charge accumulator of all grids). */
apic_status apic_batch_sizes(const apic_batch *b, int64_t *n_total, int64_t *g_total, size_t *ws_bytes);
/* [host] part_off and grid_off, nrep + 1 entries each (either may be NULL). */
apic_status apic_batch_offsets(const apic_batch *b, int64_t *part_off, int64_t *grid_off);
/* Number of work items (for sizing external tuning loops). */
int apic_batch_work_items(const apic_batch *b);
/* E^0 from the initial positions, then the backward half push v^0 -> v^{-1/2}. */
apic_status apic_batch_init(apic_batch *b, apic_batch_state *st, void *ws, void *stream);
/* nsteps cycles. diag [dev, double, nsteps*nrep*4] (or NULL): per step k and
 * replica r at (k*nrep + r)*4: charge, W_E at n+k+1, kinetic energy at n+k,
 * x-momentum (as in apic_step). rho [dev, int64, g_total] optional: the last
 * step's fixed-point node sums. use_graph != 0 replays one captured launch per
 * step (captured on first use for the given pointers). */
apic_status apic_batch_step(apic_batch *b, apic_batch_state *st, int nsteps, double *diag, int64_t *rho, void *ws,
                            void *stream, int use_graph);
apic_status apic_batch_sync_status(apic_batch *b, void *stream);
const char *apic_batch_last_error(const apic_batch *b);

/* ---- autotuning -------------------------------------------------------------
 * Setup calls (host, synchronous; they allocate scratch device memory and
 * contexts of their own and must not run under graph capture). Each times
 * every candidate on a private copy of the caller's particles (tiles: four
 * warm-up steps, then the faster of two runs of nsteps steps, rounded up to
 * even; batch chunks: nsteps steps)
 * (the caller's arrays are only read), returns the fastest candidate and
 * its ms per step, and caches the pick for the process: a later call for the
 * same shape returns the cached pick with *ms_per_step = -1 (may be NULL).
 * Returns APIC_EINVAL for bad arguments, APIC_EHIP if no candidate ran.
 *
 * apic_autotune_tiles: sort-bucket tile (tile_x, tile_y, and tile_z in 3D) for
 *   apic_create, over powers of two 4x4 .. 32x32 (2D), 4x4x4 .. 16x16x8 (3D;
 *   shapes whose tiles do not fit a workgroup's LDS are skipped) or 8 .. 1024
 *   nodes (1D), plus the default (0, 0, 0). tile_z [host] may be NULL below
 *   3D (it is written 0 there). p: unsorted or sorted particles as for
 *   apic_sort_by_cell (n > 0); bucket_start and perm are ignored. Periodic
 *   electrostatic plasmas (walls and the electromagnetic model return
 *   APIC_EUNSUPPORTED). Cache key: dim, vdim, nx, ny, nz, precision,
 *   floor(log2(particles per cell)) and the velocity advance.
 * apic_batch_autotune_chunk: work-item size (particles per item, 1024 ..
 *   65535) for apic_batch_create. st: the packed initial state (cell, ox, vx;
 *   E is ignored). Cache key: total particles and replica count. */
apic_status apic_autotune_tiles(const apic_grid_desc *desc, const apic_particles *p, int nsteps, int *tile_x,
                                int *tile_y, int *tile_z, double *ms_per_step, void *stream);
apic_status apic_batch_autotune_chunk(const apic_replica *reps, int nrep, double dt, double qm, double rho_ion,
                                      const apic_batch_state *st, int nsteps, int *chunk, double *ms_per_step,
                                      void *stream);

/* Exact charge of the last field solve of a mixed-path context (apic_step,
 * apic_field_solve): the integer total of its int64
 * fixed-point node sums, computed on the device without rounding (each sum
 * split into whole particles and a remainder, both summed in 64-bit
 * integers), returned as *whole particles plus *frac units of 2^-(S*dim)
 * particle, 0 <= *frac < 2^(S*dim). A deposit of n particles gives
 * *whole = n and *frac = 0 (between walls: the particles still inside, as
 * the node sums of the physical nodes, walls included). The paper's
 * "Results and validation" judges its run by conserved totals; this is the
 * charge total of the fixed-point form. Waits for the stream. [host]
 * outputs. APIC_EUNSUPPORTED on an FP64 context. */
apic_status apic_charge_exact(apic_ctx *ctx, int64_t *whole, int64_t *frac, void *stream);

/* Waits for the stream, then returns and clears the device error flags
 * (APIC_OK, APIC_EDOMAIN or APIC_EOVERFLOW). */
apic_status apic_sync_status(apic_ctx *ctx, void *stream);

/* Message for the last error on this context (never NULL). */
const char *apic_last_error(const apic_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* APIC_H */
