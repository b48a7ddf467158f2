// Relativistic fluid for gfx950: node-centred density n and momentum u per
// fluid species, donor-cell fluxes on the Yee faces where J lives; a warm
// species also carries its entropy density S = n K (K = p / n^ga).
//
// Paper: Methodology, plasma-model paragraph (fluid continuity, momentum and
// energy equations with relativistic gamma and adiabatic pressure for the
// bulk plasma; the adiabatic energy equation is the advection of S).
//
// Scheme (per step, two passes, each one thread per node, x fastest):
//   1. us = Boris(u; E, B interpolated to the node), v = us / gamma(us),
//      stored only where n > 0 (nothing else reads them)
//   2. on the face between node c and its +d neighbour: face velocity = mean
//      of the two nodes (or that of the only side above the density floor),
//      mass flux F = v_f n_donor, momentum flux G = F us_donor; each node
//      evaluates its six faces itself (a face shared by two nodes gives both
//      the same bits), then n <- n - dt div F, n u <- n us - dt div G, J += q F
// Warm fluid, between 1 and 2: us -= dt grad p / (m n) at nodes above the
// density floor (p = S n^(ga-1), zero where n = 0; central differences,
// one-sided at the open x walls; non-relativistic pressure force), v again
// us / gamma; and S <- S - dt div(F K_donor) with the same face fluxes F.
// The fluid current obeys the same discrete continuity equation as the
// Esirkepov particle current, so div E - rho is unchanged by the fluid.
// HBM-bound; where there is no fluid only the density is read.
#include "hk_internal.h"

namespace {

constexpr int BS = 256;


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
    int i, j, k;
    node_ijk(g, c, i, j, k);
    const int nxn = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
    if (i >= nxn || !(n[c] > (real)0)) return;
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
    real us[3];
    us[0] = umx + (upy * sz - upz * sy) + h * ex;
    us[1] = umy + (upz * sx - upx * sz) + h * ey;
    us[2] = umz + (upx * sy - upy * sx) + h * ez;
    real gam = sqrt((real)1 + us[0] * us[0] + us[1] * us[1] + us[2] * us[2]);
    const long long nn = g.nn;
    for (int d = 0; d < 3; ++d) {
        sc[d * nn + c] = us[d];
        sc[(3 + d) * nn + c] = us[d] / gam;
    }
}

// Mass and momentum flux on the +d face of node (i, j, k); false where the
// face does not exist (beyond the open x wall).  us and v are read only at
// nodes with n > 0, the only ones where they were written.
__device__ inline bool face_flux(const GridP &g, real n_floor, const real *__restrict__ n,
                                 const real *__restrict__ sc, int i, int j, int k, int d, real &F,
                                 real G[3], long long *donor = nullptr) {
    const int per = g.bcx == HK_BC_PERIODIC;
    F = 0; G[0] = G[1] = G[2] = 0;
    if (donor) *donor = -1;
    if (d == 0 && !per && i == g.nx) return false;
    int ii = i, jj = j, kk = k;
    if (d == 0) ii = per ? (i + 1 == g.nx ? 0 : i + 1) : i + 1;
    else if (d == 1) jj = j + 1 == g.ny ? 0 : j + 1;
    else kk = k + 1 == g.nz ? 0 : k + 1;
    const long long c = gidx(g, i, j, k), r = gidx(g, ii, jj, kk);
    const real nl = n[c], nr = n[r];
    const bool lok = nl > n_floor && nl > (real)0, rok = nr > n_floor && nr > (real)0;
    if (!lok && !rok) return true;
    const long long nn = g.nn;
    real vf;
    if (!lok) vf = sc[(3 + d) * nn + r];
    else if (!rok) vf = sc[(3 + d) * nn + c];
    else vf = (real)0.5 * (sc[(3 + d) * nn + c] + sc[(3 + d) * nn + r]);
    const long long don = vf > (real)0 ? c : r;
    const real nd = vf > (real)0 ? nl : nr;
    F = vf * nd;
    if (donor) *donor = don;
    if (nd > (real)0)
        for (int m = 0; m < 3; ++m) G[m] = F * sc[m * nn + don];
    return true;
}

__global__ void __launch_bounds__(BS)
k_fluid_update(GridP g, real q, real n_floor, real *__restrict__ n, real *__restrict__ ux,
               real *__restrict__ uy, real *__restrict__ uz, const real *__restrict__ sc,
               real *__restrict__ Jx, real *__restrict__ Jy, real *__restrict__ Jz,
               real *__restrict__ nout) {
    long long c = (long long)blockIdx.x * BS + threadIdx.x;
    if (c >= g.nn) return;
    int i, j, k;
    node_ijk(g, c, i, j, k);
    const int per = g.bcx == HK_BC_PERIODIC;
    const int nxn = per ? g.nx : g.nx + 1;
    const real n0 = n[c];
    if (i >= nxn) { nout[c] = n0; return; }
    const long long nn = g.nn;
    const real dxs[3] = {g.dx, g.dy, g.dz};
    real dn = 0, dm[3] = {0, 0, 0}, fplus[3];
    for (int d = 0; d < 3; ++d) {
        real fp, gp[3], fm = 0, gm[3] = {0, 0, 0};
        face_flux(g, n_floor, n, sc, i, j, k, d, fp, gp);
        fplus[d] = fp;
        int ii = i, jj = j, kk = k;
        bool has_minus = true;
        if (d == 0) {
            if (!per && i == 0) has_minus = false;
            ii = per ? (i == 0 ? g.nx - 1 : i - 1) : i - 1;
        } else if (d == 1) jj = j == 0 ? g.ny - 1 : j - 1;
        else kk = k == 0 ? g.nz - 1 : k - 1;
        if (has_minus) face_flux(g, n_floor, n, sc, ii, jj, kk, d, fm, gm);
        dn += (fp - fm) / dxs[d];
        for (int m = 0; m < 3; ++m) dm[m] += (gp[m] - gm[m]) / dxs[d];
    }
    const real nv = n0 - g.dt * dn;
    nout[c] = nv;
    real mom[3];
    for (int m = 0; m < 3; ++m) mom[m] = (n0 > (real)0 ? n0 * sc[m * nn + c] : (real)0) - g.dt * dm[m];
    ux[c] = nv > n_floor ? mom[0] / nv : (real)0;
    uy[c] = nv > n_floor ? mom[1] / nv : (real)0;
    uz[c] = nv > n_floor ? mom[2] / nv : (real)0;
    // fluid current on the + faces (none beyond the open x wall)
    if (fplus[0] != (real)0) Jx[c] += q * fplus[0];
    if (fplus[1] != (real)0) Jy[c] += q * fplus[1];
    if (fplus[2] != (real)0) Jz[c] += q * fplus[2];
}

__device__ inline real pressure_at(const real *__restrict__ n, const real *__restrict__ S, real gm1,
                                   long long c) {
    const real nc = n[c];
    return nc > (real)0 ? S[c] * pow(nc, gm1) : (real)0;
}

// warm fluid: pressure force on the Boris result (us, v in sc)
__global__ void __launch_bounds__(BS)
k_fluid_pressure(GridP g, real mass, real n_floor, real gm1, const real *__restrict__ n,
                 const real *__restrict__ S, real *__restrict__ sc) {
    long long c = (long long)blockIdx.x * BS + threadIdx.x;
    if (c >= g.nn) return;
    int i, j, k;
    node_ijk(g, c, i, j, k);
    const int per = g.bcx == HK_BC_PERIODIC;
    const int nxn = per ? g.nx : g.nx + 1;
    const real nc = n[c];
    if (i >= nxn || !(nc > n_floor) || !(nc > (real)0)) return;
    real grad[3];
    if (per)
        grad[0] = (pressure_at(n, S, gm1, gidx(g, wrapi(i + 1, g.nx), j, k)) -
                   pressure_at(n, S, gm1, gidx(g, wrapi(i - 1, g.nx), j, k))) / (2 * g.dx);
    else if (i == 0)
        grad[0] = (pressure_at(n, S, gm1, gidx(g, 1, j, k)) - pressure_at(n, S, gm1, c)) / g.dx;
    else if (i == g.nx)
        grad[0] = (pressure_at(n, S, gm1, c) - pressure_at(n, S, gm1, gidx(g, i - 1, j, k))) / g.dx;
    else
        grad[0] = (pressure_at(n, S, gm1, gidx(g, i + 1, j, k)) - pressure_at(n, S, gm1, gidx(g, i - 1, j, k))) /
                  (2 * g.dx);
    grad[1] = (pressure_at(n, S, gm1, gidx(g, i, wrapi(j + 1, g.ny), k)) -
               pressure_at(n, S, gm1, gidx(g, i, wrapi(j - 1, g.ny), k))) / (2 * g.dy);
    grad[2] = (pressure_at(n, S, gm1, gidx(g, i, j, wrapi(k + 1, g.nz))) -
               pressure_at(n, S, gm1, gidx(g, i, j, wrapi(k - 1, g.nz)))) / (2 * g.dz);
    const long long nn = g.nn;
    real us[3];
    for (int d = 0; d < 3; ++d) us[d] = sc[d * nn + c] - g.dt * grad[d] / (mass * nc);
    const real gam = sqrt((real)1 + us[0] * us[0] + us[1] * us[1] + us[2] * us[2]);
    for (int d = 0; d < 3; ++d) {
        sc[d * nn + c] = us[d];
        sc[(3 + d) * nn + c] = us[d] / gam;
    }
}

// warm fluid: S_new = S - dt div(F K_donor), K = S / n (zero where n = 0)
__global__ void __launch_bounds__(BS)
k_fluid_entropy(GridP g, real n_floor, const real *__restrict__ n, const real *__restrict__ S,
                const real *__restrict__ sc, real *__restrict__ Sout) {
    long long c = (long long)blockIdx.x * BS + threadIdx.x;
    if (c >= g.nn) return;
    int i, j, k;
    node_ijk(g, c, i, j, k);
    const int per = g.bcx == HK_BC_PERIODIC;
    const int nxn = per ? g.nx : g.nx + 1;
    if (i >= nxn) { Sout[c] = S[c]; return; }
    const real dxs[3] = {g.dx, g.dy, g.dz};
    auto hflux = [&](int ii, int jj, int kk, int d) -> real {
        real F, G[3];
        long long don;
        face_flux(g, n_floor, n, sc, ii, jj, kk, d, F, G, &don);
        if (don < 0 || !(n[don] > (real)0)) return (real)0;
        return F * (S[don] / n[don]);
    };
    real ds = 0;
    for (int d = 0; d < 3; ++d) {
        const real hp = hflux(i, j, k, d);
        real hm = 0;
        int ii = i, jj = j, kk = k;
        bool has_minus = true;
        if (d == 0) {
            if (!per && i == 0) has_minus = false;
            ii = per ? (i == 0 ? g.nx - 1 : i - 1) : i - 1;
        } else if (d == 1) jj = j == 0 ? g.ny - 1 : j - 1;
        else kk = k == 0 ? g.nz - 1 : k - 1;
        if (has_minus) hm = hflux(ii, jj, kk, d);
        ds += (hp - hm) / dxs[d];
    }
    Sout[c] = S[c] - g.dt * ds;
}

// thermal energy sum p dV / (ga - 1) over the nodes
__global__ void __launch_bounds__(BS)
k_fluid_heat(GridP g, const real *__restrict__ n, const real *__restrict__ S, real gm1, double *out) {
    __shared__ double sh[BS];
    long long c = (long long)blockIdx.x * BS + threadIdx.x;
    double v = 0;
    if (c < g.nn) {
        int i, j, k;
        node_ijk(g, c, i, j, k);
        const int nxn = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
        if (i < nxn && n[c] > (real)0) v = (double)S[c] * pow((double)n[c], (double)gm1);
    }
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int h = BS / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0 && sh[0] != 0.0) atomicAdd(out, sh[0] * g.ddx * g.ddy * g.ddz / (double)gm1);
}

inline unsigned blocks(long long n) { return (unsigned)((n + BS - 1) / BS); }

}  // namespace

// scratch: 8 grid arrays (us, v, the new density and the new entropy
// density, copied back after every node has read the old ones)
void launch_fluid(const GridP &g, const SpecP &sp, real *n, real *ux, real *uy, real *uz, WarmP w,
                  real *const f[9], real *scratch, real n_floor, hipStream_t s) {
    k_fluid_lorentz<<<blocks(g.nn), BS, 0, s>>>(g, sp.qm, n, ux, uy, uz, f[HK_EX], f[HK_EY],
                                                f[HK_EZ], f[HK_BX], f[HK_BY], f[HK_BZ], scratch);
    real *nout = scratch + 6 * g.nn, *Sout = scratch + 7 * g.nn;
    if (w.S) {
        k_fluid_pressure<<<blocks(g.nn), BS, 0, s>>>(g, sp.m, n_floor, (real)(w.ga - 1.0), n, w.S, scratch);
        k_fluid_entropy<<<blocks(g.nn), BS, 0, s>>>(g, n_floor, n, w.S, scratch, Sout);
    }
    k_fluid_update<<<blocks(g.nn), BS, 0, s>>>(g, sp.q, n_floor, n, ux, uy, uz, scratch, f[HK_JX],
                                               f[HK_JY], f[HK_JZ], nout);
    hipMemcpyAsync(n, nout, sizeof(real) * g.nn, hipMemcpyDeviceToDevice, s);
    if (w.S) hipMemcpyAsync(w.S, Sout, sizeof(real) * g.nn, hipMemcpyDeviceToDevice, s);
}

void launch_fluid_heat(const GridP &g, const real *n, WarmP w, double *out, hipStream_t s) {
    if (w.S) k_fluid_heat<<<blocks(g.nn), BS, 0, s>>>(g, n, w.S, (real)(w.ga - 1.0), out);
}
