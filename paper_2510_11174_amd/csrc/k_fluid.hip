// Relativistic fluid for gfx950: node-centred density n and momentum u per
// fluid species, donor-cell fluxes on the Yee faces where J lives; a warm
// species also carries its entropy density S = n K (K = p / n^ga).
//
// Paper: Methodology, plasma-model paragraph (fluid continuity, momentum and
// energy equations with relativistic gamma and adiabatic pressure for the
// bulk plasma; the adiabatic energy equation is the advection of S).
//
// Scheme (per step, two passes over the nodes of the x window, x fastest):
//   1. us = Boris(u; E, B interpolated to the node); a warm species then
//      takes the pressure force, us -= dt grad p / (m n) at nodes above the
//      density floor (p = S n^(ga-1), zero where n = 0; central differences,
//      one-sided at the open x walls; non-relativistic), stored only where
//      n > 0 (nothing else reads it)
//   2. on the face between node c and its +d neighbour: face velocity = mean
//      of the two nodes' v = us / gamma(us) (or that of the only side above
//      the density floor),
//      mass flux F = v_f n_donor, momentum flux G = F us_donor, entropy flux
//      H = F K_donor (warm, K = S / n); each node evaluates its six faces
//      itself (a face shared by two nodes gives both the same bits), then
//      n <- n - dt div F, n u <- n us - dt div G, S <- max(S - dt div H, 0),
//      J += q F; the new n and S go to the species' second buffers, which
//      the host swaps with the first
// The fluid current obeys the same discrete continuity equation as the
// Esirkepov particle current, so div E - rho is unchanged by the fluid.
// HBM-bound; where there is no fluid only the density is read.
//
// x window (open x): every node with x index outside [xr[0], xr[1]] holds no
// fluid in either density buffer (and u = 0 there), so the passes leave the
// nodes outside [xr[0] - 1, xr[1] + 1] alone (a face flux reaches one node
// further per step).  The window only grows: the update widens xr[2..3] where
// it leaves fluid, the push's absorptions widen xr[4..5], and
// k_fluid_window_commit folds both into xr[0..1] once per step.  Periodic x
// keeps the full window.
#include "hk_internal.h"

namespace {

constexpr int BS = 256;
constexpr unsigned WIN_GRID = 8192;   // blocks of the window passes (a multiple of 8)


// The pass window of x range xr (see above): node columns lo .. lo + w - 1
// of every (y, z) row; false when it is empty.
__device__ inline bool pass_window(const GridP &g, const int *__restrict__ xr, int &lo, int &w) {
    lo = max(xr[0] - 1, 0);
    w = min(xr[1] + 1, g.sx - 1) - lo + 1;
    return w > 0;
}

// The window's nodes spread over a fixed grid (a multiple of 8 blocks):
// workgroups go round-robin to the 8 XCDs, and XCD x sweeps the x-th eighth
// of the window's nodes in row order, so that the y and z neighbour rows of
// its nodes sit in its own L2.  f(c, i, j, k) runs once per window node.
template <typename F>
__device__ inline void for_window_nodes(const GridP &g, const int *__restrict__ xr, F f) {
    int lo, w;
    if (!pass_window(g, xr, lo, w)) return;
    const unsigned total = (unsigned)w * (unsigned)g.ny * (unsigned)g.nz;
    const unsigned share = (total + 7u) / 8u, xcd = blockIdx.x & 7u, per_xcd = gridDim.x >> 3;
    const unsigned end = min(total, (xcd + 1u) * share);
    for (unsigned t = xcd * share + (blockIdx.x >> 3) * BS + threadIdx.x; t < end; t += per_xcd * BS) {
        const unsigned row = t / (unsigned)w;
        const int i = lo + (int)(t - row * (unsigned)w);
        const int j = (int)(row % (unsigned)g.ny), k = (int)(row / (unsigned)g.ny);
        f(i + (int)row * g.sx, i, j, k);
    }
}

// Linear indices of a node's neighbours (node counts stay below 2^31):
// y and z periodic, x periodic or open (no neighbour beyond an open wall).
struct Nbr {
    int xm, xp, ym, yp, zm, zp;
    bool hasxm, hasxp;
};

__device__ inline Nbr neighbours(const GridP &g, int c, int i, int j, int k) {
    Nbr b;
    const int sxy = g.sx * g.ny;
    if (g.bcx == HK_BC_PERIODIC) {
        b.xm = i == 0 ? c + g.nx - 1 : c - 1;
        b.xp = i + 1 == g.nx ? c - i : c + 1;
        b.hasxm = b.hasxp = true;
    } else {
        b.xm = c - 1;
        b.xp = c + 1;
        b.hasxm = i != 0;
        b.hasxp = i != g.nx;
    }
    b.ym = j == 0 ? c + (g.ny - 1) * g.sx : c - g.sx;
    b.yp = j + 1 == g.ny ? c - j * g.sx : c + g.sx;
    b.zm = k == 0 ? c + (g.nz - 1) * sxy : c - sxy;
    b.zp = k + 1 == g.nz ? c - k * sxy : c + sxy;
    return b;
}

// field component at a node: trilinear at offset 0, i.e. the node value for
// node-type axes and the mean of the two neighbours for half axes.  xs: the
// two x samples of a half axis (wrapped, or clamped to the last cell at an
// open wall); oy, oz: row offsets of the samples j - 1, j and k - 1, k.
__device__ inline real node_val(const real *__restrict__ F, const int xs[2], const int oy[2], const int oz[2],
                                int i, int hx, int hy, int hz) {
    real acc = 0;
    for (int c = 0; c < (hz ? 2 : 1); ++c)
        for (int b = 0; b < (hy ? 2 : 1); ++b)
            for (int a = 0; a < (hx ? 2 : 1); ++a) {
                const int ii = hx ? xs[a] : i;
                const int jo = hy ? oy[b] : oy[1], ko = hz ? oz[c] : oz[1];
                real wgt = (hx ? (real)0.5 : (real)1) * (hy ? (real)0.5 : (real)1) * (hz ? (real)0.5 : (real)1);
                acc += wgt * F[ii + jo + ko];
            }
    return acc;
}

// warm fluid: node pressure p = S n^(ga-1), zero where n = 0
__global__ void __launch_bounds__(BS)
k_fluid_p(GridP g, real gm1, const real *__restrict__ n, const real *__restrict__ S, real *__restrict__ P,
          const int *__restrict__ xr) {
    for_window_nodes(g, xr, [&](int c, int, int, int) {
        const real nc = n[c];
        P[c] = nc > (real)0 ? S[c] * pow(nc, gm1) : (real)0;
    });
}

__device__ inline void fluid_lorentz_node(const GridP &g, real qm, real mass, real n_floor,
                                          const real *__restrict__ n, const real *__restrict__ P,
                                          const real *__restrict__ ux, const real *__restrict__ uy,
                                          const real *__restrict__ uz, const real *__restrict__ Ex,
                                          const real *__restrict__ Ey, const real *__restrict__ Ez,
                                          const real *__restrict__ Bx, const real *__restrict__ By,
                                          const real *__restrict__ Bz, real *__restrict__ sc, int c, int i,
                                          int j, int k) {
    const int per = g.bcx == HK_BC_PERIODIC;
    const int nxn = per ? g.nx : g.nx + 1;
    const real nc = n[c];
    if (i >= nxn || !(nc > (real)0)) return;
    const int sxy = g.sx * g.ny;
    int xs[2];
    if (per) {
        xs[0] = i == 0 ? g.nx - 1 : i - 1;
        xs[1] = i;
    } else {
        xs[0] = i - 1 < 0 ? 0 : (i - 1 > g.nx - 1 ? g.nx - 1 : i - 1);
        xs[1] = i > g.nx - 1 ? g.nx - 1 : i;
    }
    const int oy[2] = {(j == 0 ? g.ny - 1 : j - 1) * g.sx, j * g.sx};
    const int oz[2] = {(k == 0 ? g.nz - 1 : k - 1) * sxy, k * sxy};
    real ex = node_val(Ex, xs, oy, oz, i, 1, 0, 0), ey = node_val(Ey, xs, oy, oz, i, 0, 1, 0);
    real ez = node_val(Ez, xs, oy, oz, i, 0, 0, 1), bx = node_val(Bx, xs, oy, oz, i, 0, 1, 1);
    real by = node_val(By, xs, oy, oz, i, 1, 0, 1), bz = node_val(Bz, xs, oy, oz, i, 1, 1, 0);
    const real h = (real)0.5 * qm * g.dt;
    real umx = ux[c] + h * ex, umy = uy[c] + h * ey, umz = uz[c] + h * ez;
    real gm = sqrt((real)1 + umx * umx + umy * umy + umz * umz);
    const real rg = h / gm;
    real tx = bx * rg, ty = by * rg, tz = bz * rg;
    real t2 = tx * tx + ty * ty + tz * tz;
    const real r2 = (real)2 / (1 + t2);
    real sx = tx * r2, sy = ty * r2, sz = tz * r2;
    real upx = umx + (umy * tz - umz * ty), upy = umy + (umz * tx - umx * tz),
         upz = umz + (umx * ty - umy * tx);
    real us[3];
    us[0] = umx + (upy * sz - upz * sy) + h * ex;
    us[1] = umy + (upz * sx - upx * sz) + h * ey;
    us[2] = umz + (upx * sy - upy * sx) + h * ez;
    if (P && nc > n_floor) {
        // pressure force: central differences, one-sided at the open x walls
        const Nbr b = neighbours(g, c, i, j, k);
        real grad[3];
        if (per) grad[0] = (P[b.xp] - P[b.xm]) / (2 * g.dx);
        else if (i == 0) grad[0] = (P[b.xp] - P[c]) / g.dx;
        else if (i == g.nx) grad[0] = (P[c] - P[b.xm]) / g.dx;
        else grad[0] = (P[b.xp] - P[b.xm]) / (2 * g.dx);
        grad[1] = (P[b.yp] - P[b.ym]) / (2 * g.dy);
        grad[2] = (P[b.zp] - P[b.zm]) / (2 * g.dz);
        const real rmn = g.dt / (mass * nc);
        for (int d = 0; d < 3; ++d) us[d] = us[d] - grad[d] * rmn;
    }
    const long long nn = g.nn;
    for (int d = 0; d < 3; ++d) sc[d * nn + c] = us[d];
}

// v = us / gamma(us), recomputed by the update from the us it reads (the
// same expression at every node, so the same bits wherever it is formed)
__device__ inline real rgamma_of(const real u[3]) {
    return (real)1 / sqrt((real)1 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
}

__global__ void __launch_bounds__(BS)
k_fluid_lorentz(GridP g, real qm, real mass, real n_floor, const real *__restrict__ n,
                const real *__restrict__ P, const real *__restrict__ ux,
                const real *__restrict__ uy, const real *__restrict__ uz, const real *__restrict__ Ex,
                const real *__restrict__ Ey, const real *__restrict__ Ez, const real *__restrict__ Bx,
                const real *__restrict__ By, const real *__restrict__ Bz, real *__restrict__ sc,
                const int *__restrict__ xr) {
    for_window_nodes(g, xr, [&](int c, int i, int j, int k) {
        fluid_lorentz_node(g, qm, mass, n_floor, n, P, ux, uy, uz, Ex, Ey, Ez, Bx, By, Bz, sc, c, i, j, k);
    });
}

// One side of a face: density, its velocity component normal to the face,
// its momentum, and whether it is above the density floor.
struct Side {
    real n, v, us[3];
    bool ok;
};

// Mass and momentum flux through the face between sides l and r (r on the
// +d side), from values already loaded; don receives the donor node (-1
// where neither side is above the density floor) and nd its density.  us
// and v are meaningful only at nodes with n > 0, the only ones where they
// were written; the selects below never use the others.
__device__ inline void face_flux(const Side &l, const Side &r, int lo, int hi, real &F, real G[3], int &don,
                                 real &nd) {
    const real vf = !l.ok ? r.v : (!r.ok ? l.v : (real)0.5 * (l.v + r.v));
    const bool pos = vf > (real)0;
    nd = pos ? l.n : r.n;
    F = vf * nd;
    for (int m = 0; m < 3; ++m) G[m] = nd > (real)0 ? F * (pos ? l.us[m] : r.us[m]) : (real)0;
    don = pos ? lo : hi;
    if (!l.ok && !r.ok) {
        F = 0; G[0] = G[1] = G[2] = 0;
        don = -1; nd = 0;
    }
}

__device__ inline void fluid_update_node(const GridP &g, real q, real n_floor, const real *__restrict__ n,
                                         real *__restrict__ ux, real *__restrict__ uy, real *__restrict__ uz,
                                         const real *__restrict__ sc, real *__restrict__ Jx,
                                         real *__restrict__ Jy, real *__restrict__ Jz, real *__restrict__ nout,
                                         const real *__restrict__ S, real *__restrict__ Sout,
                                         int *__restrict__ xr, int x0, int x1, int c, int i, int j, int k) {
    const int per = g.bcx == HK_BC_PERIODIC;
    const int nxn = per ? g.nx : g.nx + 1;
    const real n0 = n[c];
    if (i >= nxn) {
        nout[c] = n0;
        if (S) Sout[c] = S[c];
        return;
    }
    const long long nn = g.nn;
    const real *const us[3] = {sc, sc + nn, sc + 2 * nn};
    const real rdx[3] = {(real)1 / g.dx, (real)1 / g.dy, (real)1 / g.dz};
    const Nbr b = neighbours(g, c, i, j, k);
    const int pl[3] = {b.xp, b.yp, b.zp}, mi[3] = {b.xm, b.ym, b.zm};
    const bool hasp[3] = {b.hasxp, true, true}, hasm[3] = {b.hasxm, true, true};
    auto fok = [&](real v) { return v > n_floor && v > (real)0; };
    // the densities first: a node whose stencil holds no fluid above the
    // floor has no face flux, keeps its density and entropy and gets u = 0
    real np[3], nm[3];
    bool any = fok(n0);
    for (int d = 0; d < 3; ++d) {
        np[d] = hasp[d] ? n[pl[d]] : (real)0;
        nm[d] = hasm[d] ? n[mi[d]] : (real)0;
        any = any || (hasp[d] && fok(np[d])) || (hasm[d] && fok(nm[d]));
    }
    if (!any) {
        nout[c] = n0;
        if (S) Sout[c] = S[c];
        ux[c] = 0; uy[c] = 0; uz[c] = 0;
        return;
    }
    // every other value of the stencil, loaded before any is used
    Side C, P[3], M[3];
    C.n = n0; C.ok = fok(n0);
    for (int m = 0; m < 3; ++m) C.us[m] = us[m][c];
    real vc[3], Sc = 0, Sp[3] = {0, 0, 0}, Sm[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        const int pp = hasp[d] ? pl[d] : c, mm = hasm[d] ? mi[d] : c;
        P[d].n = np[d]; P[d].ok = hasp[d] && fok(np[d]);
        M[d].n = nm[d]; M[d].ok = hasm[d] && fok(nm[d]);
        for (int m = 0; m < 3; ++m) {
            P[d].us[m] = us[m][pp];
            M[d].us[m] = us[m][mm];
        }
        if (S) {
            Sp[d] = S[pp];
            Sm[d] = S[mm];
        }
    }
    if (S) Sc = S[c];
    // the normal velocity of each side (the pass before stores us only)
    const real rgc = rgamma_of(C.us);
    for (int d = 0; d < 3; ++d) {
        vc[d] = C.us[d] * rgc;
        P[d].v = P[d].us[d] * rgamma_of(P[d].us);
        M[d].v = M[d].us[d] * rgamma_of(M[d].us);
    }
    real dn = 0, dm[3] = {0, 0, 0}, fplus[3], ds = 0;
    for (int d = 0; d < 3; ++d) {
        C.v = vc[d];
        real fp = 0, gp[3] = {0, 0, 0}, fm = 0, gm[3] = {0, 0, 0}, ndp = 0, ndm = 0;
        int dp = -1, dmi = -1;
        if (hasp[d]) face_flux(C, P[d], c, pl[d], fp, gp, dp, ndp);
        if (hasm[d]) face_flux(M[d], C, mi[d], c, fm, gm, dmi, ndm);
        fplus[d] = fp;
        dn += (fp - fm) * rdx[d];
        for (int m = 0; m < 3; ++m) dm[m] += (gp[m] - gm[m]) * rdx[d];
        if (S) {
            // entropy flux F K_donor, K = S / n at the donor
            const real Sdp = dp == c ? Sc : Sp[d], Sdm = dmi == c ? Sc : Sm[d];
            const real hp = dp < 0 || !(ndp > (real)0) ? (real)0 : fp * (Sdp / ndp);
            const real hm = dmi < 0 || !(ndm > (real)0) ? (real)0 : fm * (Sdm / ndm);
            ds += (hp - hm) * rdx[d];
        }
    }
    const real nv = n0 - g.dt * dn;
    nout[c] = nv;
    // fluid left next to the window: widen it (x index i holds fluid now)
    if (nv != (real)0 && (i < x0 || i > x1)) {
        atomicMin(&xr[2], i);
        atomicMax(&xr[3], i);
    }
    if (S) {
        // kept non-negative: a node can lose more than it holds in one step
        const real sn = Sc - g.dt * ds;
        Sout[c] = sn > (real)0 ? sn : (real)0;
    }
    real mom[3];
    for (int m = 0; m < 3; ++m) mom[m] = (n0 > (real)0 ? n0 * C.us[m] : (real)0) - g.dt * dm[m];
    const bool live = nv > n_floor;
    const real rnv = live ? (real)1 / nv : (real)0;
    ux[c] = live ? mom[0] * rnv : (real)0;
    uy[c] = live ? mom[1] * rnv : (real)0;
    uz[c] = live ? mom[2] * rnv : (real)0;
    // fluid current on the + faces (none beyond the open x wall)
    if (fplus[0] != (real)0) Jx[c] += q * fplus[0];
    if (fplus[1] != (real)0) Jy[c] += q * fplus[1];
    if (fplus[2] != (real)0) Jz[c] += q * fplus[2];
}

__global__ void __launch_bounds__(BS)
k_fluid_update(GridP g, real q, real n_floor, const real *__restrict__ n, real *__restrict__ ux,
               real *__restrict__ uy, real *__restrict__ uz, const real *__restrict__ sc,
               real *__restrict__ Jx, real *__restrict__ Jy, real *__restrict__ Jz,
               real *__restrict__ nout, const real *__restrict__ S, real *__restrict__ Sout, int *__restrict__ xr) {
    // the window as this pass found it (the pass widens xr[2..3] only)
    const int x0 = xr[0], x1 = xr[1];
    for_window_nodes(g, xr, [&](int c, int i, int j, int k) {
        fluid_update_node(g, q, n_floor, n, ux, uy, uz, sc, Jx, Jy, Jz, nout, S, Sout, xr, x0, x1, c, i, j, k);
    });
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

// xr[0..1] the window, xr[2..3] the update's widening, xr[4..5] the
// absorptions' range: the window takes both, which then start empty again
__global__ void k_fluid_window_commit(int *xr, int empty_lo) {
    if (threadIdx.x != 0) return;
    xr[0] = min(xr[0], min(xr[2], xr[4]));
    xr[1] = max(xr[1], max(xr[3], xr[5]));
    xr[2] = xr[4] = empty_lo;
    xr[3] = xr[5] = -1;
}

}  // namespace

// scratch: 7 grid arrays (us in the first three, the pressure of a warm
// species in the seventh); nout
// and Sout receive the new density and entropy density (every node of the
// window, so the caller can swap them in); xr: the species' x window
void launch_fluid(const GridP &g, const SpecP &sp, const real *n, real *ux, real *uy, real *uz, WarmP w,
                  real *const f[9], real *scratch, real *nout, real *Sout, real n_floor, int *xr,
                  hipStream_t s) {
    real *P = nullptr;
    if (w.S) {
        P = scratch + 6 * g.nn;
        k_fluid_p<<<WIN_GRID, BS, 0, s>>>(g, (real)(w.ga - 1.0), n, w.S, P, xr);
    }
    k_fluid_lorentz<<<WIN_GRID, BS, 0, s>>>(g, sp.qm, sp.m, n_floor, n, P, ux, uy, uz, f[HK_EX],
                                                f[HK_EY], f[HK_EZ], f[HK_BX], f[HK_BY], f[HK_BZ], scratch, xr);
    k_fluid_update<<<WIN_GRID, BS, 0, s>>>(g, sp.q, n_floor, n, ux, uy, uz, scratch, f[HK_JX],
                                               f[HK_JY], f[HK_JZ], nout, w.S, Sout, xr);
}

void launch_fluid_window_commit(const GridP &g, int *xr, hipStream_t s) {
    k_fluid_window_commit<<<1, 64, 0, s>>>(xr, g.nx + 2);
}

void launch_fluid_heat(const GridP &g, const real *n, WarmP w, double *out, hipStream_t s) {
    if (w.S) k_fluid_heat<<<blocks(g.nn), BS, 0, s>>>(g, n, w.S, (real)(w.ga - 1.0), out);
}
