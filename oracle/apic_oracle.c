/*
 * Serial FP64 reference ("oracle") for the electrostatic particle-in-cell
 * coupling loop: linear (cloud-in-cell) charge deposition, field gather,
 * Boris velocity advance and the position update with periodic wrap.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU baseline
 * leg of the benchmark do. It shares no source, header, table or constant with
 * the HIP path.
 *
 * Built with gcc -O2 -ffp-contract=off, no fast-math: every floating-point
 * operation below is a plain IEEE-754 double operation in the order written.
 *
 * The paper (AlgoPlasma, "Core functionality") names these operations as the
 * particle-space and particle-grid coupling modules (A_Pusher with the Boris
 * pusher, B_Scatter, C_Gather) and cites the textbook schemes of Birdsall &
 * Langdon and Hockney & Eastwood for them without restating formulas. The
 * formulas below are those textbook schemes:
 *   grid: periodic, node-centred, X_j = j*dx, j = 0..nx-1;
 *   shape: linear hat (CIC); in 2D and 3D the tensor product of 1D hats;
 *   deposit: rho_j += (Q/dV) * sum_p W_j(x_p);
 *   gather:  E_p = sum_j W_j(x_p) E_j (same weights as the deposit);
 *   Boris (1970): half electric kick, magnetic rotation, half electric kick.
 * The quantised deposit (integer CIC weights summed in int64) is not in the
 * paper; it is the fixed-point reading of the same deposit, documented at
 * or_deposit_q_1d / or_deposit_q_2d.
 *
 * Layout: 2D grid arrays are row-major [ny][nx], node index j = iy*nx + ix;
 * 3D grid arrays are [nz][ny][nx], node index (iz*ny + iy)*nx + ix. The 3D
 * routines are the Cartesian three-dimensional forms the paper's two-stream
 * driver calls (scatter B01, gather C01 and Boris A01 "3Dxyz").
 */
#include <math.h>
#include <stdint.h>

/* ---- cloud-in-cell weights --------------------------------------------- */

/* Cell index and fractional position of coordinate x on a periodic grid of n
 * nodes spaced d apart: i = floor(x/d), f = x/d - i. A coordinate that rounds
 * onto the right edge (i == n) belongs to node 0 with f = 0. */
static void cic_cell(double x, int n, double d, int64_t *i_out, double *f_out)
{
    double g = x / d;
    double fl = floor(g);
    int64_t i = (int64_t)fl;
    double f = g - fl;
    if (i >= n) { i -= n; }
    if (i < 0) { i += n; }
    if (i >= n || i < 0) { i = 0; f = 0.0; }
    *i_out = i;
    *f_out = f;
}

/* Periodic wrap of a coordinate into [0, L). */
static double wrap(double x, double L)
{
    x = fmod(x, L);
    if (x < 0.0) x += L;
    if (x >= L) x -= L;
    return x;
}

/* Weights of one particle on its two 1D nodes (i, i+1 mod n). */
void or_cic_weights_1d(double x, int n, double d, int64_t *i, int64_t *ip, double *w0, double *w1)
{
    double f;
    cic_cell(x, n, d, i, &f);
    *ip = (*i + 1) % n;
    *w0 = 1.0 - f;
    *w1 = f;
}

/* ---- deposit (B_Scatter) ----------------------------------------------- */

void or_deposit_1d(int64_t n, const double *x, int nx, double dx, double q_over_dv, double *rho)
{
    for (int64_t p = 0; p < n; ++p) {
        int64_t i; double f;
        cic_cell(x[p], nx, dx, &i, &f);
        int64_t ip = (i + 1) % nx;
        rho[i] += q_over_dv * (1.0 - f);
        rho[ip] += q_over_dv * f;
    }
}

void or_deposit_2d(int64_t n, const double *x, const double *y, int nx, int ny,
                   double dx, double dy, double q_over_dv, double *rho)
{
    for (int64_t p = 0; p < n; ++p) {
        int64_t i, j; double fx, fy;
        cic_cell(x[p], nx, dx, &i, &fx);
        cic_cell(y[p], ny, dy, &j, &fy);
        int64_t ip = (i + 1) % nx, jp = (j + 1) % ny;
        rho[j * nx + i]   += q_over_dv * ((1.0 - fx) * (1.0 - fy));
        rho[j * nx + ip]  += q_over_dv * (fx * (1.0 - fy));
        rho[jp * nx + i]  += q_over_dv * ((1.0 - fx) * fy);
        rho[jp * nx + ip] += q_over_dv * (fx * fy);
    }
}

/* 3D: the eight nodes of the particle's cell, weight (wx * wy) * wz with
 * wx in {1 - fx, fx} etc. */
void or_deposit_3d(int64_t n, const double *x, const double *y, const double *z, int nx, int ny, int nz,
                   double dx, double dy, double dz, double q_over_dv, double *rho)
{
    for (int64_t p = 0; p < n; ++p) {
        int64_t i[2], j[2], k[2]; double fx, fy, fz;
        cic_cell(x[p], nx, dx, &i[0], &fx);
        cic_cell(y[p], ny, dy, &j[0], &fy);
        cic_cell(z[p], nz, dz, &k[0], &fz);
        i[1] = (i[0] + 1) % nx; j[1] = (j[0] + 1) % ny; k[1] = (k[0] + 1) % nz;
        double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a)
                    rho[(k[c] * ny + j[b]) * nx + i[a]] += q_over_dv * ((wx[a] * wy[b]) * wz[c]);
    }
}

/* ---- quantised deposit (fixed-point reading of the same deposit) --------
 * A particle sits in cell (ix[, iy]) at in-cell offset o in [0,1) held in
 * binary32. Its 1D weights are the integers w1 = round-half-even(o * 2^S) and
 * w0 = 2^S - w1; o * 2^S is exact (a power-of-two scale), so the rounding is
 * the only approximation and the two weights sum to exactly 2^S. In 2D the
 * node weights are the integer products of the per-axis weights and sum to
 * exactly 2^(2S). The node sums are exact int64 additions, hence independent
 * of summation order. */
static int64_t qweight(float o, int S)
{
    double s = ldexp((double)o, S);
    return (int64_t)nearbyint(s);
}

void or_deposit_q_1d(int64_t n, const int32_t *ix, const float *ox, int nx, int S, int64_t *I)
{
    const int64_t one = (int64_t)1 << S;
    for (int64_t p = 0; p < n; ++p) {
        int64_t w1 = qweight(ox[p], S);
        int64_t w0 = one - w1;
        int64_t i = ix[p];
        int64_t ip = (i + 1) % nx;
        I[i] += w0;
        I[ip] += w1;
    }
}

void or_deposit_q_2d(int64_t n, const int32_t *ix, const int32_t *iy, const float *ox, const float *oy,
                     int nx, int ny, int S, int64_t *I)
{
    const int64_t one = (int64_t)1 << S;
    for (int64_t p = 0; p < n; ++p) {
        int64_t w1x = qweight(ox[p], S), w0x = one - w1x;
        int64_t w1y = qweight(oy[p], S), w0y = one - w1y;
        int64_t i = ix[p], j = iy[p];
        int64_t ip = (i + 1) % nx, jp = (j + 1) % ny;
        I[j * nx + i]   += w0x * w0y;
        I[j * nx + ip]  += w1x * w0y;
        I[jp * nx + i]  += w0x * w1y;
        I[jp * nx + ip] += w1x * w1y;
    }
}

/* 3D: node weight (w_a * w_b) * w_c of the per-axis integer weights; the
 * product of three S-bit weights is exact in int64 for S <= 20. */
void or_deposit_q_3d(int64_t n, const int32_t *ix, const int32_t *iy, const int32_t *iz, const float *ox,
                     const float *oy, const float *oz, int nx, int ny, int nz, int S, int64_t *I)
{
    const int64_t one = (int64_t)1 << S;
    for (int64_t p = 0; p < n; ++p) {
        int64_t wx[2], wy[2], wz[2];
        wx[1] = qweight(ox[p], S); wx[0] = one - wx[1];
        wy[1] = qweight(oy[p], S); wy[0] = one - wy[1];
        wz[1] = qweight(oz[p], S); wz[0] = one - wz[1];
        int64_t i[2] = {ix[p], (ix[p] + 1) % nx}, j[2] = {iy[p], (iy[p] + 1) % ny};
        int64_t k[2] = {iz[p], (iz[p] + 1) % nz};
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a)
                    I[(k[c] * ny + j[b]) * nx + i[a]] += (wx[a] * wy[b]) * wz[c];
    }
}

/* ---- gather (C_Gather) ------------------------------------------------- */

void or_gather_1d(int64_t n, const double *x, int nx, double dx, const double *E, double *Ep)
{
    for (int64_t p = 0; p < n; ++p) {
        int64_t i; double f;
        cic_cell(x[p], nx, dx, &i, &f);
        int64_t ip = (i + 1) % nx;
        Ep[p] = (1.0 - f) * E[i] + f * E[ip];
    }
}

void or_gather_2d(int64_t n, const double *x, const double *y, int nx, int ny, double dx, double dy,
                  const double *Ex, const double *Ey, double *Epx, double *Epy)
{
    for (int64_t p = 0; p < n; ++p) {
        int64_t i, j; double fx, fy;
        cic_cell(x[p], nx, dx, &i, &fx);
        cic_cell(y[p], ny, dy, &j, &fy);
        int64_t ip = (i + 1) % nx, jp = (j + 1) % ny;
        double w00 = (1.0 - fx) * (1.0 - fy), w10 = fx * (1.0 - fy);
        double w01 = (1.0 - fx) * fy, w11 = fx * fy;
        Epx[p] = w00 * Ex[j * nx + i] + w10 * Ex[j * nx + ip] + w01 * Ex[jp * nx + i] + w11 * Ex[jp * nx + ip];
        Epy[p] = w00 * Ey[j * nx + i] + w10 * Ey[j * nx + ip] + w01 * Ey[jp * nx + i] + w11 * Ey[jp * nx + ip];
    }
}

/* 3D: E_p = sum over the eight nodes of (wx * wy) * wz * E, for each of the
 * three components. */
void or_gather_3d(int64_t n, const double *x, const double *y, const double *z, int nx, int ny, int nz,
                  double dx, double dy, double dz, const double *Ex, const double *Ey, const double *Ez,
                  double *Epx, double *Epy, double *Epz)
{
    for (int64_t p = 0; p < n; ++p) {
        int64_t i[2], j[2], k[2]; double fx, fy, fz;
        cic_cell(x[p], nx, dx, &i[0], &fx);
        cic_cell(y[p], ny, dy, &j[0], &fy);
        cic_cell(z[p], nz, dz, &k[0], &fz);
        i[1] = (i[0] + 1) % nx; j[1] = (j[0] + 1) % ny; k[1] = (k[0] + 1) % nz;
        double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
        double ex = 0.0, ey = 0.0, ez = 0.0;
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) {
                    int64_t m = (k[c] * ny + j[b]) * nx + i[a];
                    double w = (wx[a] * wy[b]) * wz[c];
                    ex += w * Ex[m];
                    ey += w * Ey[m];
                    ez += w * Ez[m];
                }
        Epx[p] = ex;
        Epy[p] = ey;
        Epz[p] = ez;
    }
}

/* ---- Boris velocity advance (A_Pusher, Boris 1970) ----------------------
 * Uniform magnetic field along z (bz); the electric field has an x, y and
 * (3D only) z component.
 *   a   = (q/m) dt / 2
 *   v-  = v + a E
 *   t   = a bz z^ ,  s = 2 t / (1 + |t|^2)
 *   v'  = v- + v- x t
 *   v+  = v- + v' x s
 *   v   = v+ + a E
 * vdim = 1: only vx (no magnetic term); vdim = 2: (vx, vy), bz must be 0;
 * vdim = 3: (vx, vy, vz); the rotation about z leaves vz alone, so vz only
 * takes the two half kicks of Ez (none when Epz is NULL, Ez = 0 in 2D).
 * Epy may be NULL when vdim = 1 (1D electric field). */
void or_boris(int64_t n, int vdim, double *vx, double *vy, double *vz,
              const double *Epx, const double *Epy, const double *Epz, double qm, double dt, double bz)
{
    const double a = qm * dt * 0.5;
    const double t = a * bz;
    const double s = 2.0 * t / (1.0 + t * t);
    for (int64_t p = 0; p < n; ++p) {
        if (vdim == 3 && Epz) {
            double mz = vz[p] + a * Epz[p];
            vz[p] = mz + a * Epz[p];
        }
        if (vdim == 1) {
            double m1 = vx[p] + a * Epx[p];
            vx[p] = m1 + a * Epx[p];
            continue;
        }
        double ex = Epx[p], ey = Epy ? Epy[p] : 0.0;
        double mx = vx[p] + a * ex;
        double my = vy[p] + a * ey;
        double px = mx + my * t;
        double py = my - mx * t;
        double qx = mx + py * s;
        double qy = my - px * s;
        vx[p] = qx + a * ex;
        vy[p] = qy + a * ey;
    }
}

/* ---- Higuera-Cary velocity advance (A_Pusher, Higuera & Cary 2017) -------
 * The paper lists it beside Boris among A_Pusher's algorithms. The state is
 * u = gamma v (velocity units), gamma = sqrt(1 + |u|^2/c^2); B = bz z^.
 *   a = (q/m) dt / 2,  tau = a bz
 *   u-  = u + a E,  gamma-^2 = 1 + |u-|^2/c^2,  sigma = gamma-^2 - tau^2
 *   gamma+ = sqrt((sigma + sqrt(sigma^2 + 4 (tau^2 + (u-.tau)^2/c^2))) / 2)
 *   t = tau / gamma+ (along z),  s = 1 / (1 + t^2)
 *   u+  = s (u- + (u-.t) t + u- x t)
 *   u   = u+ + a E + u+ x t
 * As c -> infinity gamma+ -> 1 and the map is the Boris rotation. Epz may be
 * NULL (Ez = 0). vdim must be 3. */
void or_hc(int64_t n, double *ux, double *uy, double *uz, const double *Epx, const double *Epy,
           const double *Epz, double qm, double dt, double bz, double c)
{
    const double a = qm * dt * 0.5;
    const double tau = a * bz;
    const double ic2 = 1.0 / (c * c);
    for (int64_t p = 0; p < n; ++p) {
        double ex = Epx[p], ey = Epy[p], ez = Epz ? Epz[p] : 0.0;
        double mx = ux[p] + a * ex, my = uy[p] + a * ey, mz = uz[p] + a * ez;
        double g2 = 1.0 + (mx * mx + my * my + mz * mz) * ic2;
        double sig = g2 - tau * tau;
        double us = mz * tau;
        double gp = sqrt(0.5 * (sig + sqrt(sig * sig + 4.0 * (tau * tau + us * us * ic2))));
        double t = tau / gp;
        double s = 1.0 / (1.0 + t * t);
        double px = s * (mx + my * t);
        double py = s * (my - mx * t);
        double pz = s * (mz + (mz * t) * t);
        ux[p] = px + a * ex + py * t;
        uy[p] = py + a * ey - px * t;
        uz[p] = pz + a * ez;
    }
}

/* ---- position update with periodic boundaries ---------------------------
 * The paper leaves this to the application code ("move_particles" in the
 * two-stream driver): x <- x + v dt, then wrap into [0, L). */
void or_move_1d(int64_t n, double *x, const double *vx, double dt, double L)
{
    for (int64_t p = 0; p < n; ++p) x[p] = wrap(x[p] + vx[p] * dt, L);
}

void or_move_2d(int64_t n, double *x, double *y, const double *vx, const double *vy,
                double dt, double Lx, double Ly)
{
    for (int64_t p = 0; p < n; ++p) {
        x[p] = wrap(x[p] + vx[p] * dt, Lx);
        y[p] = wrap(y[p] + vy[p] * dt, Ly);
    }
}

void or_move_3d(int64_t n, double *x, double *y, double *z, const double *vx, const double *vy,
                const double *vz, double dt, double Lx, double Ly, double Lz)
{
    for (int64_t p = 0; p < n; ++p) {
        x[p] = wrap(x[p] + vx[p] * dt, Lx);
        y[p] = wrap(y[p] + vy[p] * dt, Ly);
        z[p] = wrap(z[p] + vz[p] * dt, Lz);
    }
}

/* Position update from u = gamma v: x <- x + (u / gamma) dt with
 * gamma = sqrt(1 + |u|^2/c^2), then wrap (dim 2 or 3; z, uz used in 3D). */
void or_move_u(int64_t n, int dim, double *x, double *y, double *z, const double *ux, const double *uy,
               const double *uz, double dt, double c, double Lx, double Ly, double Lz)
{
    const double ic2 = 1.0 / (c * c);
    for (int64_t p = 0; p < n; ++p) {
        double g = sqrt(1.0 + (ux[p] * ux[p] + uy[p] * uy[p] + uz[p] * uz[p]) * ic2);
        x[p] = wrap(x[p] + (ux[p] / g) * dt, Lx);
        y[p] = wrap(y[p] + (uy[p] / g) * dt, Ly);
        if (dim == 3) z[p] = wrap(z[p] + (uz[p] / g) * dt, Lz);
    }
}

/* ---- adjoint (transpose-Jacobian) operators -----------------------------
 * Discrete adjoints of the operators above, used to build the reference
 * gradient of a scalar loss through the time loop. "lam" arrays are the
 * adjoint variables; every routine ACCUMULATES (+=) into its outputs.
 *
 * Deposit  rho_j = rho0 + c * sum_p W_j(x_p):
 *   lam_x_p += c * sum_j lam_rho_j * dW_j/dx (x_p)        (a gradient gather)
 * Gather   E_p = sum_j W_j(x_p) E_j:
 *   lam_E_j += sum_p W_j(x_p) lam_Ep_p                    (a scatter)
 *   lam_x_p += sum_j dW_j/dx (x_p) E_j * lam_Ep_p
 * The CIC hat is piecewise linear; dW/dx is its one-sided slope inside the
 * cell that holds the particle (the derivative almost everywhere). */

void or_adj_deposit_1d(int64_t n, const double *x, int nx, double dx, double c,
                       const double *lrho, double *lx)
{
    for (int64_t p = 0; p < n; ++p) {
        int64_t i; double f;
        cic_cell(x[p], nx, dx, &i, &f);
        int64_t ip = (i + 1) % nx;
        lx[p] += c * ((lrho[ip] - lrho[i]) / dx);
    }
}

void or_adj_deposit_2d(int64_t n, const double *x, const double *y, int nx, int ny, double dx, double dy,
                       double c, const double *lrho, double *lx, double *ly)
{
    for (int64_t p = 0; p < n; ++p) {
        int64_t i, j; double fx, fy;
        cic_cell(x[p], nx, dx, &i, &fx);
        cic_cell(y[p], ny, dy, &j, &fy);
        int64_t ip = (i + 1) % nx, jp = (j + 1) % ny;
        double l00 = lrho[j * nx + i], l10 = lrho[j * nx + ip];
        double l01 = lrho[jp * nx + i], l11 = lrho[jp * nx + ip];
        /* d/dx of (1-fx)(1-fy), fx(1-fy), (1-fx)fy, fx fy  = (-(1-fy), (1-fy), -fy, fy)/dx */
        double gx = ((1.0 - fy) * (l10 - l00) + fy * (l11 - l01)) / dx;
        double gy = ((1.0 - fx) * (l01 - l00) + fx * (l11 - l10)) / dy;
        lx[p] += c * gx;
        ly[p] += c * gy;
    }
}

void or_adj_gather_1d(int64_t n, const double *x, int nx, double dx, const double *E,
                      const double *lEp, double *lE, double *lx)
{
    for (int64_t p = 0; p < n; ++p) {
        int64_t i; double f;
        cic_cell(x[p], nx, dx, &i, &f);
        int64_t ip = (i + 1) % nx;
        lE[i] += (1.0 - f) * lEp[p];
        lE[ip] += f * lEp[p];
        lx[p] += ((E[ip] - E[i]) / dx) * lEp[p];
    }
}

void or_adj_gather_2d(int64_t n, const double *x, const double *y, int nx, int ny, double dx, double dy,
                      const double *Ex, const double *Ey, const double *lEpx, const double *lEpy,
                      double *lEx, double *lEy, double *lx, double *ly)
{
    for (int64_t p = 0; p < n; ++p) {
        int64_t i, j; double fx, fy;
        cic_cell(x[p], nx, dx, &i, &fx);
        cic_cell(y[p], ny, dy, &j, &fy);
        int64_t ip = (i + 1) % nx, jp = (j + 1) % ny;
        int64_t a00 = j * nx + i, a10 = j * nx + ip, a01 = jp * nx + i, a11 = jp * nx + ip;
        double w00 = (1.0 - fx) * (1.0 - fy), w10 = fx * (1.0 - fy);
        double w01 = (1.0 - fx) * fy, w11 = fx * fy;
        double ax = lEpx[p], ay = lEpy[p];
        lEx[a00] += w00 * ax; lEx[a10] += w10 * ax; lEx[a01] += w01 * ax; lEx[a11] += w11 * ax;
        lEy[a00] += w00 * ay; lEy[a10] += w10 * ay; lEy[a01] += w01 * ay; lEy[a11] += w11 * ay;
        /* gradient of the interpolated field along x and y, dotted with lam_Ep */
        double dExdx = ((1.0 - fy) * (Ex[a10] - Ex[a00]) + fy * (Ex[a11] - Ex[a01])) / dx;
        double dEydx = ((1.0 - fy) * (Ey[a10] - Ey[a00]) + fy * (Ey[a11] - Ey[a01])) / dx;
        double dExdy = ((1.0 - fx) * (Ex[a01] - Ex[a00]) + fx * (Ex[a11] - Ex[a10])) / dy;
        double dEydy = ((1.0 - fx) * (Ey[a01] - Ey[a00]) + fx * (Ey[a11] - Ey[a10])) / dy;
        lx[p] += dExdx * ax + dEydx * ay;
        ly[p] += dExdy * ax + dEydy * ay;
    }
}

/* 3D deposit adjoint: lx, ly, lz += c * the slope of the trilinear hat, i.e.
 * d/dx of sum_abc (wx_a wy_b) wz_c lrho_abc over the particle's cell:
 * (sum_bc wy_b wz_c (lrho_1bc - lrho_0bc)) / dx, and likewise along y, z. */
void or_adj_deposit_3d(int64_t n, const double *x, const double *y, const double *z, int nx, int ny, int nz,
                       double dx, double dy, double dz, double c, const double *lrho, double *lx, double *ly,
                       double *lz)
{
    for (int64_t p = 0; p < n; ++p) {
        int64_t i[2], j[2], k[2]; double fx, fy, fz;
        cic_cell(x[p], nx, dx, &i[0], &fx);
        cic_cell(y[p], ny, dy, &j[0], &fy);
        cic_cell(z[p], nz, dz, &k[0], &fz);
        i[1] = (i[0] + 1) % nx; j[1] = (j[0] + 1) % ny; k[1] = (k[0] + 1) % nz;
        double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
        double l[2][2][2];
        for (int cc = 0; cc < 2; ++cc)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a)
                    l[cc][b][a] = lrho[(k[cc] * ny + j[b]) * nx + i[a]];
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (int u = 0; u < 2; ++u)
            for (int v = 0; v < 2; ++v) {
                gx += wy[u] * wz[v] * (l[v][u][1] - l[v][u][0]);
                gy += wx[u] * wz[v] * (l[v][1][u] - l[v][0][u]);
                gz += wx[u] * wy[v] * (l[1][v][u] - l[0][v][u]);
            }
        lx[p] += c * gx / dx;
        ly[p] += c * gy / dy;
        lz[p] += c * gz / dz;
    }
}

/* 3D gather adjoint: lam_E of each component += (wx wy) wz lam_Ep at the
 * particle's eight nodes; lx, ly, lz += the slope of the interpolated field
 * along each axis dotted with lam_Ep. */
void or_adj_gather_3d(int64_t n, const double *x, const double *y, const double *z, int nx, int ny, int nz,
                      double dx, double dy, double dz, const double *Ex, const double *Ey, const double *Ez,
                      const double *lEpx, const double *lEpy, const double *lEpz, double *lEx, double *lEy,
                      double *lEz, double *lx, double *ly, double *lz)
{
    for (int64_t p = 0; p < n; ++p) {
        int64_t i[2], j[2], k[2]; double fx, fy, fz;
        cic_cell(x[p], nx, dx, &i[0], &fx);
        cic_cell(y[p], ny, dy, &j[0], &fy);
        cic_cell(z[p], nz, dz, &k[0], &fz);
        i[1] = (i[0] + 1) % nx; j[1] = (j[0] + 1) % ny; k[1] = (k[0] + 1) % nz;
        double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
        double ax = lEpx[p], ay = lEpy[p], az = lEpz[p];
        double g[2][2][2];
        for (int cc = 0; cc < 2; ++cc)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) {
                    int64_t m = (k[cc] * ny + j[b]) * nx + i[a];
                    double w = (wx[a] * wy[b]) * wz[cc];
                    lEx[m] += w * ax;
                    lEy[m] += w * ay;
                    lEz[m] += w * az;
                    g[cc][b][a] = Ex[m] * ax + Ey[m] * ay + Ez[m] * az;
                }
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (int u = 0; u < 2; ++u)
            for (int v = 0; v < 2; ++v) {
                gx += wy[u] * wz[v] * (g[v][u][1] - g[v][u][0]);
                gy += wx[u] * wz[v] * (g[v][1][u] - g[v][0][u]);
                gz += wx[u] * wy[v] * (g[1][v][u] - g[0][v][u]);
            }
        lx[p] += gx / dx;
        ly[p] += gy / dy;
        lz[p] += gz / dz;
    }
}

/* Adjoint of the Boris map. For a fixed uniform bz the map is linear in
 * (v, E_p): v_new = R v + a (R + I) E_p, with R the rotation
 *   R = [[1 - s t, s], [-s, 1 - s t]]   acting on (vx, vy),
 * obtained by composing v' = v- + v- x t and v+ = v- + v' x s. Its adjoint is
 *   lam_v_old = R^T lam_v_new,   lam_Ep = a (R + I)^T lam_v_new.
 * On entry lv* hold lam for v_new; on return they hold lam for v_old. lEp*
 * are OVERWRITTEN with lam_Ep. vdim as in or_boris. */
void or_adj_boris(int64_t n, int vdim, double *lvx, double *lvy, double *lEpx, double *lEpy,
                  double qm, double dt, double bz)
{
    const double a = qm * dt * 0.5;
    const double t = a * bz;
    const double s = 2.0 * t / (1.0 + t * t);
    const double r = 1.0 - s * t;
    for (int64_t p = 0; p < n; ++p) {
        if (vdim == 1) {
            lEpx[p] = 2.0 * a * lvx[p];
            continue;
        }
        double gx = lvx[p], gy = lvy[p];
        /* R^T = [[r, -s], [s, r]] */
        double ox = r * gx - s * gy;
        double oy = s * gx + r * gy;
        /* (R + I)^T g = R^T g + g */
        lEpx[p] = a * (ox + gx);
        lEpy[p] = a * (oy + gy);
        lvx[p] = ox;
        lvy[p] = oy;
    }
}
