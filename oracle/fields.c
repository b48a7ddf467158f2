/*
 * Oracle field solver: Yee FDTD leapfrog, first-order Mur absorber, current
 * sheet laser antenna, CIC gather on the staggered grid, discrete div E.
 *
 * Paper: Methodology, the FDTD paragraphs (explicit time-domain Maxwell on a
 * uniform Cartesian grid), the boundary paragraph (first-order Mur absorbers
 * with coefficient (c dt - d)/(c dt + d)) and the laser paragraph (Gaussian
 * temporal and spatial envelopes applied to the E components by polarization).
 *
 * Normalized Maxwell equations: dB/dt = -curl E, dE/dt = curl B - J,
 * div E = rho.  Yee staggering (cell units):
 *   Ex (i+1/2, j, k)   Ey (i, j+1/2, k)   Ez (i, j, k+1/2)
 *   Bx (i, j+1/2, k+1/2)   By (i+1/2, j, k+1/2)   Bz (i+1/2, j+1/2, k)
 *   J like E, rho at nodes (i, j, k).
 * y and z are periodic.  In x the box is either periodic or open: node-type
 * components (Ey, Ez, Bx) live on planes i = 0..nx, half-type components
 * (Ex, By, Bz) on i = 0..nx-1, and Ey, Ez on the two wall planes follow Mur.
 */
#include "or_internal.h"

static int xwrap(const or_sim *s, int i) {
    return s->g.bc_x == OR_BC_PERIODIC ? or_wrap(i, s->g.nx) : i;
}

/* B <- B - (dt/2) curl E, over every valid sample. */
void or_yee_b_half(or_sim *s) {
    const or_grid *g = &s->g;
    double h = 0.5 * g->dt;
    double *Ex = s->f[OR_EX], *Ey = s->f[OR_EY], *Ez = s->f[OR_EZ];
    double *Bx = s->f[OR_BX], *By = s->f[OR_BY], *Bz = s->f[OR_BZ];
    int per = g->bc_x == OR_BC_PERIODIC;
    int inode = per ? g->nx - 1 : g->nx;   /* last node plane */
    int ihalf = g->nx - 1;                 /* last half plane */
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j) {
            int jp = or_wrap(j + 1, g->ny), kp = or_wrap(k + 1, g->nz);
            for (int i = 0; i <= inode; ++i) {
                size_t c = or_idx(s, i, j, k);
                double curlx = (Ez[or_idx(s, i, jp, k)] - Ez[c]) / g->dy -
                               (Ey[or_idx(s, i, j, kp)] - Ey[c]) / g->dz;
                Bx[c] -= h * curlx;
            }
            for (int i = 0; i <= ihalf; ++i) {
                int ip = xwrap(s, i + 1);
                size_t c = or_idx(s, i, j, k);
                double curly = (Ex[or_idx(s, i, j, kp)] - Ex[c]) / g->dz -
                               (Ez[or_idx(s, ip, j, k)] - Ez[c]) / g->dx;
                double curlz = (Ey[or_idx(s, ip, j, k)] - Ey[c]) / g->dx -
                               (Ex[or_idx(s, i, jp, k)] - Ex[c]) / g->dy;
                By[c] -= h * curly;
                Bz[c] -= h * curlz;
            }
        }
}

/* E <- E + dt (curl B - J); open x: Mur on Ey, Ez at the wall planes. */
void or_yee_e_full(or_sim *s) {
    const or_grid *g = &s->g;
    double dt = g->dt;
    double *Ex = s->f[OR_EX], *Ey = s->f[OR_EY], *Ez = s->f[OR_EZ];
    double *Bx = s->f[OR_BX], *By = s->f[OR_BY], *Bz = s->f[OR_BZ];
    double *Jx = s->f[OR_JX], *Jy = s->f[OR_JY], *Jz = s->f[OR_JZ];
    int per = g->bc_x == OR_BC_PERIODIC;
    int nx = g->nx;
    size_t plane = (size_t)g->ny * g->nz;
    /* Mur needs the wall and first interior planes at time n. */
    double *old = NULL;
    if (!per) {
        old = (double *)malloc(sizeof(double) * plane * 8);
        for (int k = 0; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j) {
                size_t p = (size_t)j + (size_t)g->ny * k;
                old[0 * plane + p] = Ey[or_idx(s, 0, j, k)];
                old[1 * plane + p] = Ey[or_idx(s, 1, j, k)];
                old[2 * plane + p] = Ez[or_idx(s, 0, j, k)];
                old[3 * plane + p] = Ez[or_idx(s, 1, j, k)];
                old[4 * plane + p] = Ey[or_idx(s, nx, j, k)];
                old[5 * plane + p] = Ey[or_idx(s, nx - 1, j, k)];
                old[6 * plane + p] = Ez[or_idx(s, nx, j, k)];
                old[7 * plane + p] = Ez[or_idx(s, nx - 1, j, k)];
            }
    }
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j) {
            int jm = or_wrap(j - 1, g->ny), km = or_wrap(k - 1, g->nz);
            for (int i = 0; i < nx; ++i) {      /* Ex on half planes */
                size_t c = or_idx(s, i, j, k);
                double curlx = (Bz[c] - Bz[or_idx(s, i, jm, k)]) / g->dy -
                               (By[c] - By[or_idx(s, i, j, km)]) / g->dz;
                Ex[c] += dt * (curlx - Jx[c]);
            }
            int i0 = per ? 0 : 1, i1 = per ? nx - 1 : nx - 1;
            for (int i = i0; i <= i1; ++i) {    /* Ey, Ez on node planes */
                int im = xwrap(s, i - 1);
                size_t c = or_idx(s, i, j, k);
                double curly = (Bx[c] - Bx[or_idx(s, i, j, km)]) / g->dz -
                               (Bz[c] - Bz[or_idx(s, im, j, k)]) / g->dx;
                double curlz = (By[c] - By[or_idx(s, im, j, k)]) / g->dx -
                               (Bx[c] - Bx[or_idx(s, i, jm, k)]) / g->dy;
                Ey[c] += dt * (curly - Jy[c]);
                Ez[c] += dt * (curlz - Jz[c]);
            }
        }
    if (!per) {
        /* First-order Mur: E(wall)^{n+1} = E(in)^n + cm (E(in)^{n+1} - E(wall)^n),
         * with cm = (c dt - dx)/(c dt + dx) as stated in the boundary paragraph. */
        double cm = (dt - g->dx) / (dt + g->dx);
        for (int k = 0; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j) {
                size_t p = (size_t)j + (size_t)g->ny * k;
                Ey[or_idx(s, 0, j, k)] =
                    old[1 * plane + p] + cm * (Ey[or_idx(s, 1, j, k)] - old[0 * plane + p]);
                Ez[or_idx(s, 0, j, k)] =
                    old[3 * plane + p] + cm * (Ez[or_idx(s, 1, j, k)] - old[2 * plane + p]);
                Ey[or_idx(s, nx, j, k)] =
                    old[5 * plane + p] + cm * (Ey[or_idx(s, nx - 1, j, k)] - old[4 * plane + p]);
                Ez[or_idx(s, nx, j, k)] =
                    old[7 * plane + p] + cm * (Ez[or_idx(s, nx - 1, j, k)] - old[6 * plane + p]);
            }
        free(old);
    }
}

/* Laser field at the antenna: Gaussian temporal and transverse envelopes on a
 * sin (y) / cos (z, circular only) carrier.  The sheet current that radiates a
 * field E on both sides is J = -2 E / dx on one node plane. */
void or_antenna(or_sim *s, double t) {
    const or_laser *L = &s->las;
    if (!L->enabled) return;
    const or_grid *g = &s->g;
    double tc = L->t_center > 0 ? L->t_center : 2.0 * L->duration;
    double env_t = exp(-((t - tc) / L->duration) * ((t - tc) / L->duration));
    double yc = 0.5 * g->ny * g->dy, zc = 0.5 * g->nz * g->dz;
    int ia = L->i_antenna;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j) {
            /* Jy sample at (ia, j+1/2, k) */
            double y = (j + 0.5) * g->dy - yc, z = k * g->dz - zc;
            double r2 = y * y + z * z;
            double ey = L->a0 * env_t * exp(-r2 / (L->waist * L->waist)) * sin(t);
            s->f[OR_JY][or_idx(s, ia, j, k)] += -2.0 * ey / g->dx;
            if (L->polarization == 1) {
                /* Jz sample at (ia, j, k+1/2) */
                double y2 = j * g->dy - yc, z2 = (k + 0.5) * g->dz - zc;
                double r22 = y2 * y2 + z2 * z2;
                double ez = L->a0 * env_t * exp(-r22 / (L->waist * L->waist)) * cos(t);
                s->f[OR_JZ][or_idx(s, ia, j, k)] += -2.0 * ez / g->dx;
            }
        }
}

/* Stagger offsets of each component, cell units. */
static const double OR_OFF[OR_NCOMP][3] = {
    {0.5, 0, 0}, {0, 0.5, 0}, {0, 0, 0.5},       /* E */
    {0, 0.5, 0.5}, {0.5, 0, 0.5}, {0.5, 0.5, 0}, /* B */
    {0.5, 0, 0}, {0, 0.5, 0}, {0, 0, 0.5}};      /* J */

/* Trilinear (CIC) interpolation of one staggered component at the position
 * cell c + offset o (cell units).  Open x: half-plane components are extended
 * past the walls by their value on the nearest plane. */
double or_gather(const or_sim *s, int comp, const int c[3], const double o[3]) {
    const or_grid *g = &s->g;
    int i0[3];
    double f[3];
    for (int d = 0; d < 3; ++d) {
        double u = o[d] - OR_OFF[comp][d];     /* in [-0.5, 1) */
        int fl = (int)floor(u);
        i0[d] = c[d] + fl;
        f[d] = u - fl;
    }
    int half = OR_OFF[comp][0] != 0.0;
    double acc = 0.0;
    for (int cc = 0; cc < 2; ++cc)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                int i = i0[0] + a;
                if (g->bc_x == OR_BC_PERIODIC) i = or_wrap(i, g->nx);
                else if (half) i = i < 0 ? 0 : (i > g->nx - 1 ? g->nx - 1 : i);
                else i = i < 0 ? 0 : (i > g->nx ? g->nx : i);
                int j = or_wrap(i0[1] + b, g->ny), k = or_wrap(i0[2] + cc, g->nz);
                double wgt = (a ? f[0] : 1 - f[0]) * (b ? f[1] : 1 - f[1]) * (cc ? f[2] : 1 - f[2]);
                acc += wgt * s->f[comp][or_idx(s, i, j, k)];
            }
    return acc;
}

/* Discrete divergence of E at nodes, the same difference stencil as Ampere's
 * law transposed; open x leaves the two wall planes at zero. */
void or_divE(const or_sim *s, double *out) {
    const or_grid *g = &s->g;
    memset(out, 0, sizeof(double) * s->nn);
    int per = g->bc_x == OR_BC_PERIODIC;
    int i0 = per ? 0 : 1, i1 = per ? g->nx - 1 : g->nx - 1;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = i0; i <= i1; ++i) {
                int im = per ? or_wrap(i - 1, g->nx) : i - 1;
                size_t c = or_idx(s, i, j, k);
                out[c] = (s->f[OR_EX][c] - s->f[OR_EX][or_idx(s, im, j, k)]) / g->dx +
                         (s->f[OR_EY][c] - s->f[OR_EY][or_idx(s, i, or_wrap(j - 1, g->ny), k)]) / g->dy +
                         (s->f[OR_EZ][c] - s->f[OR_EZ][or_idx(s, i, j, or_wrap(k - 1, g->nz))]) / g->dz;
            }
}
