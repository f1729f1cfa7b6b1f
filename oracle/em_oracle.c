/*
 * Serial FP64 reference ("oracle") for the particle part of the
 * electromagnetic particle-in-cell step in 2D3V on a periodic Yee grid:
 * staggered field gather, Boris advance in a general magnetic field, and the
 * charge-conserving current deposit of Esirkepov (2001) for the linear shape.
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of this package: nothing in the
 * product library links, loads or calls it, and it shares no source, header,
 * table or constant with the HIP path.
 *
 * The paper names these modules (B_Scatter depositing "current densities",
 * C_Gather, A_Pusher, and E_Maxwell with finite-difference time-domain
 * updates citing Yee 1966) without restating formulas; the formulas below are
 * those of the cited schemes, written out:
 *
 * Yee grid (2D, periodic, node (i, j) at (i dx, j dy)); array element [j][i]
 * of each component sits at
 *   Ex, Jx: ((i+1/2) dx, j dy)      Bx: (i dx, (j+1/2) dy)
 *   Ey, Jy: (i dx, (j+1/2) dy)      By: ((i+1/2) dx, j dy)
 *   Ez, Jz: (i dx, j dy)            Bz: ((i+1/2) dx, (j+1/2) dy)
 * Field arrays are [6][ny][nx] in the order Ex, Ey, Ez, Bx, By, Bz; current
 * arrays [3][ny][nx] in the order Jx, Jy, Jz.
 *
 * Gather: every component is interpolated with the linear (CIC) hat on its
 * own staggered lattice (the particle's coordinate shifted by the component's
 * half-cell offset).
 *
 * Current (Esirkepov 2001, linear shape, 2D): with S0 and S1 the 1D hat
 * weights of the old and new positions on the nodes near the particle and
 * DS = S1 - S0 per axis,
 *   Wx = DSx (S0y + DSy/2),  Wy = DSy (S0x + DSx/2),
 *   Wz = S0x S0y + DSx S0y / 2 + S0x DSy / 2 + DSx DSy / 3;
 *   Jx(i+1/2, j) = Jx(i-1/2, j) - q Wx(i, j) / (dy dt)   (zero below the stencil),
 *   Jy(i, j+1/2) = Jy(i, j-1/2) - q Wy(i, j) / (dx dt),
 *   Jz(i, j)     = q vz Wz(i, j) / (dx dy).
 * Wx + Wy equals S1x S1y - S0x S0y, so the discrete continuity equation
 * (rho1 - rho0)/dt + div J = 0 holds for the CIC charge density. The window
 * is the four nodes around the old cell, which holds every displacement
 * smaller than one cell per axis; larger ones are counted and skipped.
 */
#include <math.h>
#include <stdint.h>

/* Index and fraction of coordinate g (in cells) on a periodic lattice of n
 * points: i = floor(g) wrapped into [0, n), f = g - floor(g). */
static void lattice(double g, int n, int64_t *i_out, double *f_out)
{
    double fl = floor(g);
    double f = g - fl;
    int64_t i = (int64_t)fl % n;
    if (i < 0) i += n;
    *i_out = i;
    *f_out = f;
}

/* Component offsets in cells (x, y), order Ex, Ey, Ez, Bx, By, Bz. */
static const double OFFX[6] = {0.5, 0.0, 0.0, 0.0, 0.5, 0.5};
static const double OFFY[6] = {0.0, 0.5, 0.0, 0.5, 0.0, 0.5};

/* out[c][p] = linear interpolation of component c of F at particle p. */
void or_em_gather_2d(int64_t n, const double *x, const double *y, int nx, int ny, double dx, double dy,
                     const double *F, double *out)
{
    const int64_t G = (int64_t)nx * ny;
    for (int64_t p = 0; p < n; ++p) {
        for (int c = 0; c < 6; ++c) {
            int64_t i, j;
            double fx, fy;
            lattice(x[p] / dx - OFFX[c], nx, &i, &fx);
            lattice(y[p] / dy - OFFY[c], ny, &j, &fy);
            int64_t ip = (i + 1) % nx, jp = (j + 1) % ny;
            const double *f = F + c * G;
            double v = (1.0 - fx) * (1.0 - fy) * f[j * nx + i] + fx * (1.0 - fy) * f[j * nx + ip]
                     + (1.0 - fx) * fy * f[jp * nx + i] + fx * fy * f[jp * nx + ip];
            out[c * n + p] = v;
        }
    }
}

/* Boris (1970) in a general magnetic field: a = (q/m) dt / 2,
 * v- = v + a E, t = a B, s = 2 t / (1 + |t|^2), v' = v- + v- x t,
 * v+ = v- + v' x s, v = v+ + a E. Ep and Bp are [3][n]. */
void or_boris3(int64_t n, double *vx, double *vy, double *vz, const double *Ep, const double *Bp, double qm,
               double dt)
{
    const double a = qm * dt * 0.5;
    for (int64_t p = 0; p < n; ++p) {
        double ex = Ep[p], ey = Ep[n + p], ez = Ep[2 * n + p];
        double tx = a * Bp[p], ty = a * Bp[n + p], tz = a * Bp[2 * n + p];
        double t2 = tx * tx + ty * ty + tz * tz;
        double sx = 2.0 * tx / (1.0 + t2), sy = 2.0 * ty / (1.0 + t2), sz = 2.0 * tz / (1.0 + t2);
        double mx = vx[p] + a * ex, my = vy[p] + a * ey, mz = vz[p] + a * ez;
        double qx = mx + (my * tz - mz * ty);
        double qy = my + (mz * tx - mx * tz);
        double qz = mz + (mx * ty - my * tx);
        double px = mx + (qy * sz - qz * sy);
        double py = my + (qz * sx - qx * sz);
        double pz = mz + (qx * sy - qy * sx);
        vx[p] = px + a * ex;
        vy[p] = py + a * ey;
        vz[p] = pz + a * ez;
    }
}

/* Higuera & Cary (2017) in a general field, state u = gamma v:
 * u- = u + a E, tau = a B, sigma = 1 + |u-|^2/c^2 - |tau|^2,
 * gamma+^2 = (sigma + sqrt(sigma^2 + 4 (|tau|^2 + (u- . tau)^2 / c^2))) / 2,
 * t = tau / gamma+, s = 1 / (1 + |t|^2),
 * u+ = s (u- + (u- . t) t + u- x t), u = u+ + a E + u+ x t. */
void or_hc3(int64_t n, double *ux, double *uy, double *uz, const double *Ep, const double *Bp, double qm, double dt,
            double c)
{
    const double a = qm * dt * 0.5;
    const double ic2 = 1.0 / (c * c);
    for (int64_t p = 0; p < n; ++p) {
        double ex = Ep[p], ey = Ep[n + p], ez = Ep[2 * n + p];
        double tx = a * Bp[p], ty = a * Bp[n + p], tz = a * Bp[2 * n + p];
        double mx = ux[p] + a * ex, my = uy[p] + a * ey, mz = uz[p] + a * ez;
        double tau2 = tx * tx + ty * ty + tz * tz;
        double sig = 1.0 + (mx * mx + my * my + mz * mz) * ic2 - tau2;
        double us = mx * tx + my * ty + mz * tz;
        double gp = sqrt(0.5 * (sig + sqrt(sig * sig + 4.0 * (tau2 + us * us * ic2))));
        double wx = tx / gp, wy = ty / gp, wz = tz / gp;
        double s = 1.0 / (1.0 + (wx * wx + wy * wy + wz * wz));
        double mw = mx * wx + my * wy + mz * wz;
        double px = s * (mx + mw * wx + (my * wz - mz * wy));
        double py = s * (my + mw * wy + (mz * wx - mx * wz));
        double pz = s * (mz + mw * wz + (mx * wy - my * wx));
        ux[p] = px + a * ex + (py * wz - pz * wy);
        uy[p] = py + a * ey + (pz * wx - px * wz);
        uz[p] = pz + a * ez + (px * wy - py * wx);
    }
}

/* Hat weights of a particle at fraction f0 of cell 0, moved by d cells, on the
 * local nodes k = -1..2 (index k + 1): S0, and S1 with the new cell in
 * {-1, 0, 1}. Returns 0 when |d| >= 1. */
static int hat_pair(double f0, double d, double S0[4], double S1[4])
{
    for (int k = 0; k < 4; ++k) { S0[k] = 0.0; S1[k] = 0.0; }
    if (!(fabs(d) < 1.0)) return 0;
    S0[1] = 1.0 - f0;
    S0[2] = f0;
    double g1 = f0 + d;
    double fl = floor(g1);
    int c = (int)fl;            /* -1, 0 or 1 */
    double f1 = g1 - fl;
    S1[c + 1] = 1.0 - f1;
    S1[c + 2] = f1;
    return 1;
}

/* Accumulate J of n particles moving from (x0, y0) by (ddx, ddy) (unwrapped)
 * with out-of-plane velocity vz, charge q each, over one step dt. J is
 * [3][ny][nx]. Returns the number of particles skipped for moving one cell or
 * more along an axis. */
int64_t or_esirkepov_2d(int64_t n, const double *x0, const double *y0, const double *ddx, const double *ddy,
                        const double *vz, int nx, int ny, double dx, double dy, double q, double dt, double *J)
{
    const int64_t G = (int64_t)nx * ny;
    double *Jx = J, *Jy = J + G, *Jz = J + 2 * G;
    int64_t skipped = 0;
    for (int64_t p = 0; p < n; ++p) {
        int64_t i0, j0;
        double fx0, fy0;
        lattice(x0[p] / dx, nx, &i0, &fx0);
        lattice(y0[p] / dy, ny, &j0, &fy0);
        double S0x[4], S1x[4], S0y[4], S1y[4];
        int okx = hat_pair(fx0, ddx[p] / dx, S0x, S1x);
        int oky = hat_pair(fy0, ddy[p] / dy, S0y, S1y);
        if (!okx || !oky) { ++skipped; continue; }
        double DSx[4], DSy[4];
        for (int k = 0; k < 4; ++k) { DSx[k] = S1x[k] - S0x[k]; DSy[k] = S1y[k] - S0y[k]; }
        const double cx = -q / (dy * dt), cy = -q / (dx * dt), cz = q * vz[p] / (dx * dy);
        for (int l = 0; l < 4; ++l) {
            /* Jx along x at row l: prefix sums of Wx over k */
            double run = 0.0;
            int64_t j = (j0 + l - 1 + ny) % ny;
            for (int k = 0; k < 3; ++k) {
                run += DSx[k] * (S0y[l] + 0.5 * DSy[l]);
                int64_t i = (i0 + k - 1 + nx) % nx;
                Jx[j * nx + i] += cx * run;
            }
        }
        for (int k = 0; k < 4; ++k) {
            double run = 0.0;
            int64_t i = (i0 + k - 1 + nx) % nx;
            for (int l = 0; l < 3; ++l) {
                run += DSy[l] * (S0x[k] + 0.5 * DSx[k]);
                int64_t j = (j0 + l - 1 + ny) % ny;
                Jy[j * nx + i] += cy * run;
            }
        }
        for (int l = 0; l < 4; ++l) {
            int64_t j = (j0 + l - 1 + ny) % ny;
            for (int k = 0; k < 4; ++k) {
                int64_t i = (i0 + k - 1 + nx) % nx;
                double wz = S0x[k] * S0y[l] + 0.5 * DSx[k] * S0y[l] + 0.5 * S0x[k] * DSy[l]
                          + DSx[k] * DSy[l] / 3.0;
                Jz[j * nx + i] += cz * wz;
            }
        }
    }
    return skipped;
}
