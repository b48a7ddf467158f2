// Cold relativistic fluid for gfx950: node-centred density n and momentum u
// per fluid species, donor-cell fluxes on the Yee faces where J lives.
//
// Paper: Methodology, plasma-model paragraph (fluid continuity and momentum
// equations with relativistic gamma for the bulk plasma; the pressure and
// energy equations of the warm model are not part of the cold model).
//
// Scheme (per step, three passes, each one thread per node, x fastest):
//   1. us = Boris(u; E, B interpolated to the node), v = us / gamma(us)
//   2. on the face between node c and its +d neighbour: face velocity = mean
//      of the two nodes (or that of the only side above the density floor),
//      mass flux F = v_f n_donor, momentum flux G = F us_donor
//   3. n <- n - dt div F, n u <- n us - dt div G, J += q F
// The fluid current obeys the same discrete continuity equation as the
// Esirkepov particle current, so div E - rho is unchanged by the fluid.
// HBM-bound: each pass streams a few arrays of the grid once.
#include "hk_internal.h"

namespace {

constexpr int BS = 256;

__device__ inline void decompose(const GridP &g, long long c, int &i, int &j, int &k) {
    i = (int)(c % g.sx);
    long long r = c / g.sx;
    j = (int)(r % g.ny);
    k = (int)(r / g.ny);
}

// field component at node (i, j, k): trilinear at offset 0, i.e. the node
// value for node-type axes and the mean of the two neighbours for half axes
__device__ inline real node_val(const GridP &g, const real *F, int i, int j, int k, int hx, int hy,
                                int hz) {
    const int per = g.bcx == HK_BC_PERIODIC;
    int i0 = hx ? i - 1 : i, j0 = hy ? j - 1 : j, k0 = hz ? k - 1 : k;
    real acc = 0;
    for (int c = 0; c < (hz ? 2 : 1); ++c)
        for (int b = 0; b < (hy ? 2 : 1); ++b)
            for (int a = 0; a < (hx ? 2 : 1); ++a) {
                int ii = i0 + a;
                if (per) ii = wrapi(ii, g.nx);
                else if (hx) ii = ii < 0 ? 0 : (ii > g.nx - 1 ? g.nx - 1 : ii);
                int jj = wrapi(j0 + b, g.ny), kk = wrapi(k0 + c, g.nz);
                real wgt = (hx ? (real)0.5 : (real)1) * (hy ? (real)0.5 : (real)1) * (hz ? (real)0.5 : (real)1);
                acc += wgt * F[gidx(g, ii, jj, kk)];
            }
    return acc;
}

__global__ void __launch_bounds__(BS)
k_fluid_lorentz(GridP g, real qm, const real *__restrict__ n, const real *__restrict__ ux,
                const real *__restrict__ uy, const real *__restrict__ uz, const real *__restrict__ Ex,
                const real *__restrict__ Ey, const real *__restrict__ Ez, const real *__restrict__ Bx,
                const real *__restrict__ By, const real *__restrict__ Bz, real *__restrict__ sc) {
    long long c = (long long)blockIdx.x * BS + threadIdx.x;
    if (c >= g.nn) return;
    real us[3] = {0, 0, 0}, v[3] = {0, 0, 0};
    int i, j, k;
    decompose(g, c, i, j, k);
    const int nxn = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
    if (i < nxn && n[c] > (real)0) {
        real ex = node_val(g, Ex, i, j, k, 1, 0, 0), ey = node_val(g, Ey, i, j, k, 0, 1, 0);
        real ez = node_val(g, Ez, i, j, k, 0, 0, 1), bx = node_val(g, Bx, i, j, k, 0, 1, 1);
        real by = node_val(g, By, i, j, k, 1, 0, 1), bz = node_val(g, Bz, i, j, k, 1, 1, 0);
        const real h = (real)0.5 * qm * g.dt;
        real umx = ux[c] + h * ex, umy = uy[c] + h * ey, umz = uz[c] + h * ez;
        real gm = sqrt((real)1 + umx * umx + umy * umy + umz * umz);
        real tx = h * bx / gm, ty = h * by / gm, tz = h * bz / gm;
        real t2 = tx * tx + ty * ty + tz * tz;
        real sx = 2 * tx / (1 + t2), sy = 2 * ty / (1 + t2), sz = 2 * tz / (1 + t2);
        real upx = umx + (umy * tz - umz * ty), upy = umy + (umz * tx - umx * tz),
             upz = umz + (umx * ty - umy * tx);
        us[0] = umx + (upy * sz - upz * sy) + h * ex;
        us[1] = umy + (upz * sx - upx * sz) + h * ey;
        us[2] = umz + (upx * sy - upy * sx) + h * ez;
        real gam = sqrt((real)1 + us[0] * us[0] + us[1] * us[1] + us[2] * us[2]);
        v[0] = us[0] / gam; v[1] = us[1] / gam; v[2] = us[2] / gam;
    }
    const long long nn = g.nn;
    for (int d = 0; d < 3; ++d) {
        sc[d * nn + c] = us[d];
        sc[(3 + d) * nn + c] = v[d];
    }
}

// Fluxes on the three + faces of every node: F at sc[6..8], G at sc[9..17].
__global__ void __launch_bounds__(BS)
k_fluid_flux(GridP g, real n_floor, const real *__restrict__ n, real *__restrict__ sc) {
    long long c = (long long)blockIdx.x * BS + threadIdx.x;
    if (c >= g.nn) return;
    int i, j, k;
    decompose(g, c, i, j, k);
    const int per = g.bcx == HK_BC_PERIODIC;
    const int nxn = per ? g.nx : g.nx + 1;
    const long long nn = g.nn;
    for (int d = 0; d < 3; ++d) {
        real F = 0, G[3] = {0, 0, 0};
        bool has = i < nxn && !(d == 0 && !per && i == g.nx);
        if (has) {
            int ii = i, jj = j, kk = k;
            if (d == 0) ii = per ? (i + 1 == g.nx ? 0 : i + 1) : i + 1;
            else if (d == 1) jj = j + 1 == g.ny ? 0 : j + 1;
            else kk = k + 1 == g.nz ? 0 : k + 1;
            long long r = gidx(g, ii, jj, kk);
            real nl = n[c], nr = n[r];
            bool lok = nl > n_floor, rok = nr > n_floor;
            real vl = sc[(3 + d) * nn + c], vr = sc[(3 + d) * nn + r];
            real vf = (!lok && !rok) ? (real)0 : (!lok ? vr : (!rok ? vl : (real)0.5 * (vl + vr)));
            long long don = vf > (real)0 ? c : r;
            F = vf * n[don];
            for (int m = 0; m < 3; ++m) G[m] = F * sc[m * nn + don];
        }
        sc[(6 + d) * nn + c] = F;
        for (int m = 0; m < 3; ++m) sc[(9 + 3 * d + m) * nn + c] = G[m];
    }
}

__global__ void __launch_bounds__(BS)
k_fluid_update(GridP g, real q, real n_floor, real *__restrict__ n, real *__restrict__ ux,
               real *__restrict__ uy, real *__restrict__ uz, const real *__restrict__ sc,
               real *__restrict__ Jx, real *__restrict__ Jy, real *__restrict__ Jz) {
    long long c = (long long)blockIdx.x * BS + threadIdx.x;
    if (c >= g.nn) return;
    int i, j, k;
    decompose(g, c, i, j, k);
    const int per = g.bcx == HK_BC_PERIODIC;
    const int nxn = per ? g.nx : g.nx + 1;
    if (i >= nxn) return;
    const long long nn = g.nn;
    const real dxs[3] = {g.dx, g.dy, g.dz};
    real dn = 0, dm[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        int ii = i, jj = j, kk = k;
        bool has_minus = true;
        if (d == 0) {
            if (!per && i == 0) has_minus = false;
            ii = per ? (i == 0 ? g.nx - 1 : i - 1) : i - 1;
        } else if (d == 1) jj = j == 0 ? g.ny - 1 : j - 1;
        else kk = k == 0 ? g.nz - 1 : k - 1;
        long long cm = has_minus ? gidx(g, ii, jj, kk) : c;
        real fp = sc[(6 + d) * nn + c];
        real fm = has_minus ? sc[(6 + d) * nn + cm] : (real)0;
        dn += (fp - fm) / dxs[d];
        for (int m = 0; m < 3; ++m) {
            real gp = sc[(9 + 3 * d + m) * nn + c];
            real gmv = has_minus ? sc[(9 + 3 * d + m) * nn + cm] : (real)0;
            dm[m] += (gp - gmv) / dxs[d];
        }
    }
    real n0 = n[c];
    real nv = n0 - g.dt * dn;
    real mom[3];
    for (int m = 0; m < 3; ++m) mom[m] = n0 * sc[m * nn + c] - g.dt * dm[m];
    n[c] = nv;
    ux[c] = nv > n_floor ? mom[0] / nv : (real)0;
    uy[c] = nv > n_floor ? mom[1] / nv : (real)0;
    uz[c] = nv > n_floor ? mom[2] / nv : (real)0;
    // fluid current on the + faces (none beyond the open x wall)
    if (!(!per && i == g.nx)) Jx[c] += q * sc[6 * nn + c];
    Jy[c] += q * sc[7 * nn + c];
    Jz[c] += q * sc[8 * nn + c];
}

inline unsigned blocks(long long n) { return (unsigned)((n + BS - 1) / BS); }

}  // namespace

// scratch: 18 grid arrays
void launch_fluid(const GridP &g, const SpecP &sp, real *n, real *ux, real *uy, real *uz,
                  real *const f[9], real *scratch, real n_floor, hipStream_t s) {
    k_fluid_lorentz<<<blocks(g.nn), BS, 0, s>>>(g, sp.qm, n, ux, uy, uz, f[HK_EX], f[HK_EY],
                                                f[HK_EZ], f[HK_BX], f[HK_BY], f[HK_BZ], scratch);
    k_fluid_flux<<<blocks(g.nn), BS, 0, s>>>(g, n_floor, n, scratch);
    k_fluid_update<<<blocks(g.nn), BS, 0, s>>>(g, sp.q, n_floor, n, ux, uy, uz, scratch, f[HK_JX],
                                               f[HK_JY], f[HK_JZ]);
}
