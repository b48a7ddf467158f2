// Regime switch and fluid <-> particle conversion for gfx950.
//
// Paper: abstract and Methodology (fluid in stable regions, PIC where the
// switch flags kinetic behaviour; instability thresholds as prior knowledge,
// Results after Table 1; charge and energy checks during regime switches,
// validation paragraph).  The paper gives neither threshold values nor a
// conversion rule; the definitions implemented here are:
//   indicators per node from nearest-node moments of the fluid species
//   (particles and fluid) and the node-interpolated E:
//     |E|; density gradient beyond three standard deviations of its shot
//     noise; momentum spread; ionization probability per step; quantum
//     parameter estimate.  Kinetic if any reaches its threshold, dilated by
//     `dilation` nodes; back to fluid after `hysteresis` calm evaluations.
//   absorb (done by the push, k_particles.hip): a fluid-species particle
//     whose nearest node is fluid, and which is not hot (|u| < thr_hot),
//     moves virtually to that node (Esirkepov current of the move) and joins
//     the node fluid (k_absorb_finish merges it); spawn: fluid mass M >= wmin
//     on a kinetic node becomes round(M / w0) particles (1 to 64; w0 the
//     species' reference weight) that move virtually from the node to Philox
//     positions in its dual cell.  A CIC particle on a node carries exactly
//     the node charge of the fluid, so div E - rho is unchanged by both.
//   Hot particles are also left out of the switch moments: a hot population
//     crossing a cold bulk stays kinetic by itself and does not decide the
//     regime of the bulk.
#include "hk_internal.h"
#include "hk_pic_device.h"

namespace {

using namespace hkdev;
constexpr int BS = 256;

// Node of this thread in an XCD-aware launch over the nodes: block b takes
// item (b mod 8) q + b / 8 of a grid of 8 q blocks, so each XCD sweeps a
// contiguous slab whose neighbour rows sit in its own L2.
__device__ inline long long xcd_node() {
    const int q = gridDim.x >> 3;
    const int item = (blockIdx.x & 7) * q + (blockIdx.x >> 3);
    return (long long)item * BS + threadIdx.x;
}
constexpr int NT = TILE + 1;          // node tile edge: nearest nodes 0 .. TILE
constexpr int NT3 = NT * NT * NT;


// Nearest node of a particle (cell + offset), wrapped in periodic directions.
__device__ inline long long nearest_node(const GridP &g, int ci, int cj, int ck, real rx, real ry,
                                         real rz, int &di, int &dj, int &dk) {
    di = rx >= (real)0.5; dj = ry >= (real)0.5; dk = rz >= (real)0.5;
    int i = ci + di, j = cj + dj, k = ck + dk;
    if (g.bcx == HK_BC_PERIODIC && i == g.nx) i = 0;
    if (j == g.ny) j = 0;
    if (k == g.nz) k = 0;
    return gidx(g, i, j, k);
}

// ---------------------------------------------------------------- moments -----------------
// mom layout (7 grid arrays): N = sum w, V = sum w^2, P (3), U2 = sum w |u|^2, NI.
// Nearest-node sums of one tile's particles in LDS.  The FP32 build adds
// fixed-point integers (2^40 units per a bound on each quantity's largest
// contribution): LDS integer atomics are far cheaper than float ones on this
// GPU, and the sums become independent of the order.  The bounds come from
// the species' weight bound and a per-tile bound on |u|^2 that every kernel
// changing momenta raises (push, ionization, spawn); the largest over the
// tile and its neighbours covers particles that changed tile since.  Without
// such a bound (umax2 == nullptr) a first pass over the tile finds it.
__device__ inline real tile_moment_term(int q, real w, real ux, real uy, real uz) {
    switch (q) {
        case 0: return w;
        case 1: return w * w;
        case 2: return w * ux;
        case 3: return w * uy;
        case 4: return w * uz;
        default: return w * (ux * ux + uy * uy + uz * uz);
    }
}

// fixed-point add with saturation: a term above its bound (a bound that was
// not raised) cannot leave the exact range of the conversion
__device__ inline void madd(jacc_t *p, real v, real inv) {
#ifdef HK_DOUBLE
    jadd(p, v, inv);
#else
    const float x = fminf(fmaxf(v * inv, -1e15f), 1e15f);
    const long long q = round_to_i64((double)x);
    if (q) atomicAdd(p, (unsigned long long)q);
#endif
}

constexpr int MOM_CHUNK = 8192;   // particles per workgroup of the tile moments
#ifndef MOM_UNROLL
#define MOM_UNROLL 2              // particle slots per thread and loop iteration
#endif
constexpr int MBS = 512;          // moments workgroup: LDS allows four per CU, 8 waves per SIMD

__global__ void __launch_bounds__(MBS)
k_moments(GridP g, SpecP sp, PArr a, Bins bins, int ion_only, int zmax, real hot2, real *__restrict__ mom,
          const unsigned *__restrict__ wmax_bits, const unsigned *__restrict__ umax2,
          const int *__restrict__ active, const int2 *__restrict__ items, const int *__restrict__ ctl) {
    __shared__ jacc_t sm[6 * NT3];
    __shared__ unsigned s_u2;
    const int2 it = plan_item(items, ctl, blockIdx.x);
    const int t = it.x;
    if (t < 0) return;
    int nf, nbv;
    const int nt_ = bin_count(sp, bins, t, nf, nbv);
    // this workgroup's chunk [p0, n) of the tile's bin slots
    const int chunk = tile_chunk(nt_, MOM_CHUNK);
    const int p0 = it.y * chunk, n = min(nt_, p0 + chunk);
    if (p0 >= n) return;
    if (ion_only && active && active[t] <= 0) return;   // every ion of the tile at z_max
    const int nq = ion_only ? 1 : 6;
    for (int e = threadIdx.x; e < nq * NT3; e += MBS) sm[e] = 0;
    if (threadIdx.x == 0) s_u2 = 0;
    __syncthreads();
    const int tx = t % g.ntx, ty = (t / g.ntx) % g.nty, tz = t / (g.ntx * g.nty);
    if (!ion_only) {
        if (umax2) {
            if (threadIdx.x < 27) {
                const int dx = threadIdx.x % 3 - 1, dy = (threadIdx.x / 3) % 3 - 1, dz = threadIdx.x / 9 - 1;
                int nx_ = tx + dx;
                const int ny_ = wrapi(ty + dy, g.nty), nz_ = wrapi(tz + dz, g.ntz);
                if (g.bcx == HK_BC_PERIODIC) nx_ = wrapi(nx_, g.ntx);
                if (nx_ >= 0 && nx_ < g.ntx) atomicMax(&s_u2, umax2[nx_ + g.ntx * (ny_ + g.nty * nz_)]);
            }
        } else {
            float l = 0.f;
            for (int p = p0 + threadIdx.x; p < n; p += MBS) {
                const long long ip = bin_slot(sp, t, p, nf, nbv);
                if (a.cell[ip] < 0) continue;
                const real ux = a.ux[ip], uy = a.uy[ip], uz = a.uz[ip];
                l = fmaxf(l, (float)(ux * ux + uy * uy + uz * uz));
            }
            for (int o = 32; o > 0; o >>= 1) l = fmaxf(l, __shfl_xor(l, o));
            if ((threadIdx.x & 63) == 0 && l > 0.f) atomicMax(&s_u2, __float_as_uint(l));
        }
        __syncthreads();
    }
    // bounds of |term| per quantity, with a margin for the FP32 products
    const double wb = (double)__uint_as_float(*wmax_bits) * 1.001;
    const double ub2 = (double)__uint_as_float(s_u2) * 1.001;
    const double bound[6] = {wb, wb * wb, wb * sqrt(ub2), wb * sqrt(ub2), wb * sqrt(ub2), wb * ub2};
    real inv[6], scl[6];
    for (int q = 0; q < 6; ++q) {
        inv[q] = bound[q] > 0.0 ? (real)((double)JFIX_UNITS / bound[q]) : (real)0;
        scl[q] = (real)(bound[q] / (double)JFIX_UNITS);
    }
    const int ox = tx * TILE, oy = ty * TILE, oz = tz * TILE;
    // MOM_UNROLL slots per thread and iteration, every field of every slot
    // loaded at once and one iteration ahead of its use: the loads of
    // 2 * MOM_UNROLL particles are in flight while the LDS sums run
    struct Slot {
        int cell, zc;
        real rx, ry, rz, w, ux, uy, uz;
    };
    auto ld = [&](int p, Slot &m) {
        m.cell = -1;
        if (p >= n) return;
        const long long ip = bin_slot(sp, t, p, nf, nbv);
        m.cell = a.cell[ip];
        m.rx = a.rx[ip]; m.ry = a.ry[ip]; m.rz = a.rz[ip]; m.w = a.w[ip];
        if (ion_only) m.zc = a.zc[ip];
        else { m.ux = a.ux[ip]; m.uy = a.uy[ip]; m.uz = a.uz[ip]; }
    };
    auto add = [&](const Slot &m) {
        if (m.cell < 0) return;
        int ci, cj, ck;
        cell_ijk(g, m.cell, ci, cj, ck);
        const int lx = ci - ox + (m.rx >= (real)0.5), ly = cj - oy + (m.ry >= (real)0.5),
                  lz = ck - oz + (m.rz >= (real)0.5);
        if ((unsigned)lx > TILE || (unsigned)ly > TILE || (unsigned)lz > TILE) return;
        const int e = lx + NT * (ly + NT * lz);
        if (ion_only) {
            if (m.zc < zmax) madd(&sm[e], m.w, inv[0]);
            return;
        }
        if (hot2 > (real)0 && m.ux * m.ux + m.uy * m.uy + m.uz * m.uz >= hot2) return;   // hot: not counted
        for (int q = 0; q < 6; ++q) madd(&sm[q * NT3 + e], tile_moment_term(q, m.w, m.ux, m.uy, m.uz), inv[q]);
    };
    constexpr int U = MOM_UNROLL;
    Slot cur[U], nxt[U];
    for (int u = 0; u < U; ++u) ld(p0 + threadIdx.x + u * MBS, cur[u]);
    for (int p = p0 + threadIdx.x; p < n; p += U * MBS) {
        for (int u = 0; u < U; ++u) ld(p + (U + u) * MBS, nxt[u]);
        for (int u = 0; u < U; ++u) add(cur[u]);
        for (int u = 0; u < U; ++u) cur[u] = nxt[u];
    }
    __syncthreads();
    const int per = g.bcx == HK_BC_PERIODIC;
    // nodes 1 .. TILE-1 of a tile that one workgroup covers belong to no other
    // tile's node block, a plain add (no atomic) suffices, when the tiles
    // divide every periodic direction into two or more: a partial last tile
    // would wrap its local nodes onto the first tile's
    const bool own = nt_ <= chunk && g.ny % TILE == 0 && g.ny > TILE && g.nz % TILE == 0 &&
                     g.nz > TILE && (!per || (g.nx % TILE == 0 && g.nx > TILE));
    for (int e = threadIdx.x; e < NT3; e += MBS) {
        int aa = e % NT, b = (e / NT) % NT, c = e / (NT * NT);
        int gi = ox + aa, gj = wrapi(oy + b, g.ny), gk = wrapi(oz + c, g.nz);
        if (per) gi = wrapi(gi, g.nx);
        else if (gi > g.nx) continue;
        const bool inner = own && aa > 0 && aa < TILE && b > 0 && b < TILE && c > 0 && c < TILE;
        long long node = gidx(g, gi, gj, gk);
        if (ion_only) {
            if (sm[e] == 0) continue;
            const real v = (real)jval(sm[e], scl[0]);
            if (inner) mom[6 * g.nn + node] += v;
            else atomicAdd(&mom[6 * g.nn + node], v);
            continue;
        }
        for (int q = 0; q < 6; ++q) {
            if (sm[q * NT3 + e] == 0) continue;
            const real v = (real)jval(sm[q * NT3 + e], scl[q]);
            if (inner) mom[q * g.nn + node] += v;
            else atomicAdd(&mom[q * g.nn + node], v);
        }
    }
}

// Fluid part of the moments.  `first`: the first fluid species overwrites all
// seven arrays (zero where it has no mass), so no separate clearing pass is
// needed before the particle moments are added.
__global__ void __launch_bounds__(BS)
k_fluid_moments(GridP g, real inv_ppc, const real *__restrict__ n, const real *__restrict__ ux,
                const real *__restrict__ uy, const real *__restrict__ uz, real *__restrict__ mom,
                int first) {
    long long c = (long long)blockIdx.x * BS + threadIdx.x;
    if (c >= g.nn) return;
    real m = n[c] * (g.dx * g.dy * g.dz);
    const long long nn = g.nn;
    real v[6] = {0, 0, 0, 0, 0, 0};
    if (m > (real)0) {
        real a = ux[c], b = uy[c], d = uz[c];
        v[0] = m;
        v[1] = m * m * inv_ppc;
        v[2] = m * a;
        v[3] = m * b;
        v[4] = m * d;
        v[5] = m * (a * a + b * b + d * d);
    } else if (!first) {
        return;
    }
    if (first) {
        for (int q = 0; q < 6; ++q) mom[q * nn + c] = v[q];
        mom[6 * nn + c] = 0;
    } else {
        for (int q = 0; q < 6; ++q) mom[q * nn + c] += v[q];
    }
}

// ------------------------------------------------------------- indicators -----------------
__device__ inline real node_field(const GridP &g, const real *F, int i, int j, int k, int hx, int hy,
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
                real wgt = (hx ? (real)0.5 : (real)1) * (hy ? (real)0.5 : (real)1) * (hz ? (real)0.5 : (real)1);
                acc += wgt * F[gidx(g, ii, wrapi(j0 + b, g.ny), wrapi(k0 + c, g.nz))];
            }
    return acc;
}

__device__ inline double adk_rate(const IonLevel &L, double F) {
    return L.c2 * L.ip_au * pow(2.0 * L.k3 / F, L.expo) * exp(-2.0 * L.k3 / (3.0 * F));
}
__device__ inline double ion_rate(const IonP *ion, int lev, double F) {
    if (F <= 0.0) return 0.0;
    const IonLevel &L = ion->lev[lev];
    double gk = ion->omega_au * sqrt(2.0 * L.ip_au) / F;
    double sig = 1.0 / (1.0 + exp(-(gk - 1.5) / 0.1));
    double wm = L.wfc * pow(fmin(F, L.fc) / L.fc, L.K2);
    return (sig * wm + (1.0 - sig) * adk_rate(L, F)) * ion->rate_norm;
}

struct IonSet {
    const IonP *p[4];
    int n;
};

__global__ void __launch_bounds__(BS)
k_indicators(GridP g, SwitchP P, const real *__restrict__ mom, const real *__restrict__ Ex,
             const real *__restrict__ Ey, const real *__restrict__ Ez, IonSet ions,
             uint8_t *__restrict__ hot, uint8_t *__restrict__ notcold) {
    long long c = xcd_node();
    if (c >= g.nn) return;
    int i, j, k;
    node_ijk(g, c, i, j, k);
    const int per = g.bcx == HK_BC_PERIODIC;
    const int nxn = per ? g.nx : g.nx + 1;
    if (i >= nxn) { hot[c] = 0; notcold[c] = 0; return; }
    const long long nn = g.nn;
    const real dv = g.dx * g.dy * g.dz;
    real ex = node_field(g, Ex, i, j, k, 1, 0, 0), ey = node_field(g, Ey, i, j, k, 0, 1, 0);
    real ez = node_field(g, Ez, i, j, k, 0, 0, 1);
    real emag = sqrt(ex * ex + ey * ey + ez * ez);
    auto cx = [&](int ii) { return per ? wrapi(ii, g.nx) : (ii < 0 ? 0 : (ii > g.nx ? g.nx : ii)); };
    long long xp = gidx(g, cx(i + 1), j, k), xm = gidx(g, cx(i - 1), j, k);
    long long yp = gidx(g, i, wrapi(j + 1, g.ny), k), ym = gidx(g, i, wrapi(j - 1, g.ny), k);
    long long zp = gidx(g, i, j, wrapi(k + 1, g.nz)), zm = gidx(g, i, j, wrapi(k - 1, g.nz));
    const real *N = mom, *V = mom + nn;
    real dgx = N[xp] - N[xm], dgy = N[yp] - N[ym], dgz = N[zp] - N[zm];
    real den = 2 * fmax(N[c], P.n_floor * dv);
    real grad = sqrt(dgx * dgx + dgy * dgy + dgz * dgz) / den;
    real sig = sqrt(V[xp] + V[xm] + V[yp] + V[ym] + V[zp] + V[zm]) / den;
    grad = grad - 3 * sig;
    real su = 0, g2 = 0;
    real Nc = N[c];
    if (Nc > 0) {
        real m2 = mom[5 * nn + c] / Nc;
        real mx = mom[2 * nn + c] / Nc, my = mom[3 * nn + c] / Nc, mz = mom[4 * nn + c] / Nc;
        su = sqrt(fmax((real)0, m2 - (mx * mx + my * my + mz * mz)));
        g2 = m2;
    }
    real NI = mom[6 * nn + c];
    double ionr = 0.0;
    if (NI > 0)
        for (int s = 0; s < ions.n; ++s)
            ionr = fmax(ionr, ion_rate(ions.p[s], 0, (double)emag * ions.p[s]->field_au) * g.ddt);
    double chi = P.enable_qed ? sqrt(1.0 + (double)g2) * (double)emag / P.a_s : 0.0;
    bool h = emag >= P.thr_a || grad >= P.thr_grad || su >= P.thr_su ||
             (NI > 0 && ionr >= (double)P.thr_ion) || (P.enable_qed && chi >= (double)P.thr_chi);
    bool nc = emag >= (real)0.5 * P.thr_a || grad >= (real)0.5 * P.thr_grad ||
              su >= (real)0.5 * P.thr_su || (NI > 0 && ionr >= 0.5 * (double)P.thr_ion) ||
              (P.enable_qed && chi >= 0.5 * (double)P.thr_chi);
    hot[c] = h;
    notcold[c] = nc;
}

// Training label of the learned switch at one step, per node of the
// canonical grid [nz][ny][NX] (x fastest): bit 0, a cold-fluid conversion
// would destroy more than 1e-3 of the node's kinetic energy (e = (1/2)(sum w
// |u|^2 - |sum w u|^2 / sum w) against (1/2) sum w |u|^2, small-u limit) and
// the momentum spread reaches the switch's spread threshold; bit 1, an
// ionization event is possible (per-step probability of the node's field at
// or above thr_ion while ionizable ions remain); bit 2, a QED event is
// possible (chi of the node's rms momentum at or above thr_chi).
__global__ void __launch_bounds__(BS)
k_label_cond(GridP g, SwitchP P, const real *__restrict__ mom, const real *__restrict__ Ex,
             const real *__restrict__ Ey, const real *__restrict__ Ez, IonSet ions,
             uint8_t *__restrict__ out) {
    const int per = g.bcx == HK_BC_PERIODIC;
    const int nxn = per ? g.nx : g.nx + 1;
    const long long n = (long long)nxn * g.ny * g.nz;
    const long long v = (long long)blockIdx.x * BS + threadIdx.x;
    if (v >= n) return;
    const int i = (int)(v % nxn), j = (int)((v / nxn) % g.ny), k = (int)(v / ((long long)nxn * g.ny));
    const long long c = gidx(g, i, j, k), nn = g.nn;
    const double N = mom[c];
    int bits = 0;
    double m2 = 0.0;
    if (N > 0.0) {
        const double U2 = mom[5 * nn + c];
        const double px = mom[2 * nn + c], py = mom[3 * nn + c], pz = mom[4 * nn + c];
        const double ehat = 0.5 * (U2 - (px * px + py * py + pz * pz) / N);
        m2 = U2 / N;
        const double su2 = 2.0 * ehat / N;
        if (ehat > 1e-3 * 0.5 * U2 && su2 >= (double)P.thr_su * (double)P.thr_su) bits |= 1;
    }
    const double ex = node_field(g, Ex, i, j, k, 1, 0, 0), ey = node_field(g, Ey, i, j, k, 0, 1, 0);
    const double ez = node_field(g, Ez, i, j, k, 0, 0, 1);
    const double emag = sqrt(ex * ex + ey * ey + ez * ez);
    if (mom[6 * nn + c] > 0) {
        double ionr = 0.0;
        for (int q = 0; q < ions.n; ++q)
            ionr = fmax(ionr, ion_rate(ions.p[q], 0, emag * ions.p[q]->field_au) * g.ddt);
        if (ionr >= (double)P.thr_ion) bits |= 2;
    }
    if (P.enable_qed && N > 0.0 && sqrt(1.0 + m2) * emag / P.a_s >= (double)P.thr_chi) bits |= 4;
    out[v] = (uint8_t)bits;
}

// Node flags from the grid layout to the canonical [nz][ny][NX] order.
__global__ void __launch_bounds__(BS)
k_flags_canonical(GridP g, const uint8_t *__restrict__ src, uint8_t *__restrict__ dst) {
    const int nxn = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
    const long long v = (long long)blockIdx.x * BS + threadIdx.x;
    if (v >= (long long)nxn * g.ny * g.nz) return;
    const int i = (int)(v % nxn), j = (int)((v / nxn) % g.ny), k = (int)(v / ((long long)nxn * g.ny));
    dst[v] = src[gidx(g, i, j, k)];
}

// Label accumulation over a window of steps: y |= (cond != 0).
__global__ void __launch_bounds__(BS)
k_label_or(long long n, const uint8_t *__restrict__ cond, uint8_t *__restrict__ y) {
    const long long v = (long long)blockIdx.x * BS + threadIdx.x;
    if (v < n && cond[v]) y[v] = 1;
}

// Dilation by the (2 D + 1)^3 box, as three one-axis passes (the OR over a
// box is the OR over its rows of the OR over their elements): bit 0 of the
// running mask is "hot", bit 1 "not cold".  Pass x also packs the two
// flags; pass z applies the result: a node near a hot one is kinetic and
// calm again; a kinetic node turns fluid after `hysteresis` evaluations in
// a row with no hot and no warm node in reach.
__global__ void __launch_bounds__(BS)
k_dilate_x(GridP g, int D, const uint8_t *__restrict__ hot, const uint8_t *__restrict__ notcold,
           uint8_t *__restrict__ out) {
    const long long c = xcd_node();
    if (c >= g.nn) return;
    int i, j, k;
    node_ijk(g, c, i, j, k);
    const int per = g.bcx == HK_BC_PERIODIC;
    const long long row = c - i;
    uint8_t m = 0;
    for (int di = -D; di <= D; ++di) {
        int ii = i + di;
        if (!per && (ii < 0 || ii > g.nx)) continue;
        if (per) ii = wrapi(ii, g.nx);
        m |= (uint8_t)(hot[row + ii] | (notcold[row + ii] << 1));
    }
    out[c] = m;
}
// axis 1 (y) or 2 (z), periodic
__global__ void __launch_bounds__(BS)
k_dilate_yz(GridP g, int D, int axis, const uint8_t *__restrict__ in, uint8_t *__restrict__ out) {
    const long long c = xcd_node();
    if (c >= g.nn) return;
    int i, j, k;
    node_ijk(g, c, i, j, k);
    uint8_t m = 0;
    for (int d = -D; d <= D; ++d)
        m |= axis == 1 ? in[gidx(g, i, wrapi(j + d, g.ny), k)] : in[gidx(g, i, j, wrapi(k + d, g.nz))];
    out[c] = m;
}
__global__ void __launch_bounds__(BS)
k_dilate_apply(GridP g, SwitchP P, const uint8_t *__restrict__ in, uint8_t *__restrict__ sw,
               uint8_t *__restrict__ calm) {
    const long long c = xcd_node();
    if (c >= g.nn) return;
    int i, j, k;
    node_ijk(g, c, i, j, k);
    const int nxn = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
    if (i >= nxn) return;
    uint8_t m = 0;
    for (int d = -P.dilation; d <= P.dilation; ++d) m |= in[gidx(g, i, j, wrapi(k + d, g.nz))];
    const int kin = m & 1, warm = m & 2;
    if (kin) { sw[c] = 1; calm[c] = 0; }
    else if (sw[c]) {
        if (warm) calm[c] = 0;
        else {
            int cc = calm[c] + 1;
            if (cc >= P.hysteresis) { sw[c] = 0; calm[c] = 0; }
            else calm[c] = (uint8_t)cc;
        }
    }
}

// --------------------------------------------------------------- conversion ---------------
// The Esirkepov currents of the particles a node spawns.  Each starts at the
// node and ends within half a cell of it, so its face currents lie in a fixed
// stencil of 54 faces around the node: Jx on the x offsets -1, 0 by the y and
// z offsets -1..1, Jy and Jz likewise.  Every particle's face values are the
// terms of a single deposit, each rounded once to the global unit and added
// to the node's stencil in LDS (shared by the node's lanes); the node then
// adds each face to the global accumulator once (54 atomics at most, against
// 12 per particle).
#ifdef HK_DOUBLE
typedef double jsum_t;
__device__ inline jsum_t jg_units(double v) { return v; }
__device__ inline void jg_add(jglob_t *p, jsum_t v) { if (v != 0.0) atomicAdd(p, v); }
__device__ inline void st_add(jsum_t *p, jsum_t v) { atomicAdd(p, v); }
#else
typedef long long jsum_t;
__device__ inline jsum_t jg_units(double v) { return __double2ll_rn(v * (double)(1ull << JG_BITS)); }
__device__ inline void jg_add(jglob_t *p, jsum_t v) { if (v) atomicAdd(p, (unsigned long long)v); }
// two's complement: the unsigned sum is the signed one
__device__ inline void st_add(jsum_t *p, jsum_t v) {
    atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v);
}
#endif
constexpr int SJ_FACES = 54;
// face slot of component d at node offsets (ox, oy, oz), or -1 outside the stencil
__device__ inline int spawn_face(int d, int ox, int oy, int oz) {
    const int nx = d == 0 ? 2 : 3, ny = d == 1 ? 2 : 3, nz = d == 2 ? 2 : 3;
    const int a = ox + 1, b = oy + 1, c = oz + 1;
    if (a < 0 || a >= nx || b < 0 || b >= ny || c < 0 || c >= nz) return -1;
    return 18 * d + (a * ny + b) * nz + c;
}
__device__ inline void spawn_current_add(const GridP &g, jsum_t *st, jglob_t *Jx, jglob_t *Jy, jglob_t *Jz,
                                         int ci, int cj, int ck, const AxisS &X, const AxisS &Y, const AxisS &Z,
                                         real cx, real cy, real cz) {
    const real third = (real)(1.0 / 3.0), half = (real)0.5;
    // a face outside the stencil (none for a move within half a cell) goes
    // straight to the global accumulator
    auto put = [&](int d, int a, int b, int c, real acc) {
        const jsum_t q = jg_units((double)acc);
        if (q == (jsum_t)0) return;
        const int f = spawn_face(d, X.base + a, Y.base + b, Z.base + c);
        if (f >= 0) {
            st_add(&st[f], q);
            return;
        }
        const int per = g.bcx == HK_BC_PERIODIC;
        const int i = ci + X.base + a, j = wrapi(cj + Y.base + b, g.ny), k = wrapi(ck + Z.base + c, g.nz);
        const int ii = per ? wrapi(i, g.nx) : i;
        const bool ok = per || (ii >= 0 && (d == 0 ? ii < g.nx : ii <= g.nx));
        if (ok) jg_add(&(d == 0 ? Jx : d == 1 ? Jy : Jz)[gidx(g, ii, j, k)], q);
    };
    for (int c = 0; c < 3; ++c)
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                if (a < 2) {
                    real acc = 0;
                    for (int a2 = 0; a2 <= a; ++a2)
                        acc -= cx * (X.DS[a2] * (Y.S0[b] * Z.S0[c] + half * Y.DS[b] * Z.S0[c] +
                                                 half * Y.S0[b] * Z.DS[c] + third * Y.DS[b] * Z.DS[c]));
                    put(0, a, b, c, acc);
                }
                if (b < 2) {
                    real acc = 0;
                    for (int b2 = 0; b2 <= b; ++b2)
                        acc -= cy * (Y.DS[b2] * (X.S0[a] * Z.S0[c] + half * X.DS[a] * Z.S0[c] +
                                                 half * X.S0[a] * Z.DS[c] + third * X.DS[a] * Z.DS[c]));
                    put(1, a, b, c, acc);
                }
                if (c < 2) {
                    real acc = 0;
                    for (int c2 = 0; c2 <= c; ++c2)
                        acc -= cz * (Z.DS[c2] * (X.S0[a] * Y.S0[b] + half * X.DS[a] * Y.S0[b] +
                                                 half * X.S0[a] * Y.DS[b] + third * X.DS[a] * Y.DS[b]));
                    put(2, a, b, c, acc);
                }
            }
}
// face f of the node's stencil into the global accumulator (no face beyond
// an open x wall)
__device__ inline void spawn_face_flush(const GridP &g, int f, jsum_t v, jglob_t *Jx, jglob_t *Jy, jglob_t *Jz,
                                        int ci, int cj, int ck) {
    if (v == (jsum_t)0) return;
    const int per = g.bcx == HK_BC_PERIODIC;
    const int d = f / 18, r = f - 18 * d;
    const int nyz = d == 0 ? 9 : 6, nz = d == 2 ? 2 : 3;
    const int a = r / nyz, b = (r - a * nyz) / nz, c = r - a * nyz - b * nz;
    const int i = ci + a - 1, j = wrapi(cj + b - 1, g.ny), k = wrapi(ck + c - 1, g.nz);
    const int ii = per ? wrapi(i, g.nx) : i;
    const bool ok = per || (ii >= 0 && (d == 0 ? ii < g.nx : ii <= g.nx));
    if (ok) jg_add(&(d == 0 ? Jx : d == 1 ? Jy : Jz)[gidx(g, ii, j, k)], v);
}

__device__ inline void block_add_d(double v, double *out) {
    __shared__ double red[BS / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0;
        for (int i = 0; i < BS / 64; ++i) s += red[i];
        if (s != 0.0) atomicAdd(out, s);
    }
    __syncthreads();
}

// macc layout (5 grid arrays, FP64, one set per fluid species, filled by the
// push): M = sum w, P (3) = sum w u of the absorbed particles, and for a warm
// fluid their kinetic energy per node (which then heats the node instead of
// going to the ledger).
__global__ void __launch_bounds__(BS)
k_absorb_finish(GridP g, real mass, double *__restrict__ macc, real *__restrict__ n,
                real *__restrict__ ux, real *__restrict__ uy, real *__restrict__ uz, WarmP wp,
                double *__restrict__ ledger, const int *__restrict__ xr) {
    // only the x range of this step's absorptions (xr[4..5]) has entries: the
    // grid strides over the node columns of that range alone, x fastest
    const int lo = xr[4], hi = xr[5];
    if (hi < lo) return;
    double dsum = 0;
    const unsigned w = (unsigned)(hi - lo + 1), total = w * (unsigned)g.ny * (unsigned)g.nz;
    // four nodes per thread and turn, their accumulators loaded together
    // (the scan is bound by load latency; few nodes have entries)
    constexpr int AF_U = 4;
    for (unsigned t0 = blockIdx.x * (AF_U * BS) + threadIdx.x; t0 < total; t0 += gridDim.x * (AF_U * BS)) {
    long long cs[AF_U];
    double ms[AF_U];
    for (int u = 0; u < AF_U; ++u) {
        const unsigned t = t0 + u * BS, row = t / w;
        cs[u] = (long long)(lo + (int)(t - row * w)) + (long long)row * g.sx;
        ms[u] = t < total ? macc[cs[u]] : 0.0;
    }
    for (int u = 0; u < AF_U; ++u) {
    const long long c = cs[u];
    if (ms[u] > 0.0) {
        const long long nn = g.nn;
        const double dv = g.ddx * g.ddy * g.ddz;
        double m0 = (double)n[c] * dv;
        double u0[3] = {ux[c], uy[c], uz[c]};
        double g0 = sqrt(1.0 + u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2]);
        double mt = m0 + macc[c];
        double un[3];
        for (int q = 0; q < 3; ++q) un[q] = (m0 * u0[q] + macc[(1 + q) * nn + c]) / mt;
        double gn = sqrt(1.0 + un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
        double d = m0 * (double)mass * (g0 - 1.0) - mt * (double)mass * (gn - 1.0);
        if (wp.S) {
            // the merge's kinetic energy loss heats the node: p += (ga - 1) dE / dV;
            // a node left without positive mass or pressure (its fluid density
            // had gone negative) keeps no entropy, the ledger takes that heat
            // and its previous thermal energy
            const double ga = wp.ga;
            const double pold = n[c] > (real)0 ? (double)wp.S[c] * pow((double)n[c], ga - 1.0) : 0.0;
            const double pnew = pold + (ga - 1.0) * (macc[4 * nn + c] + d) / dv;
            if (mt > 0.0 && pnew >= 0.0) {
                wp.S[c] = (real)(pnew * pow(mt / dv, 1.0 - ga));
                d = 0;
            } else {
                wp.S[c] = 0;
                d = macc[4 * nn + c] + d + pold * dv / (ga - 1.0);
            }
        }
        n[c] = (real)(mt / dv);
        ux[c] = (real)un[0]; uy[c] = (real)un[1]; uz[c] = (real)un[2];
        for (int q = 0; q < 5; ++q) macc[q * nn + c] = 0.0;
        dsum += d;
    }
    }
    }
    block_add_d(dsum, ledger);
}

// Spawn of node c (kinetic, fluid mass >= wmin).
// Particles a node of fluid mass `mass` becomes: about the reference weight
// each, at least one and at most 64.
__device__ inline int spawn_count(real mass, real w0) {
    const double mr = w0 > (real)0 ? floor((double)mass / (double)w0 + 0.5) : 1.0;
    return mr < 1.0 ? 1 : (mr > 64.0 ? 64 : (int)mr);
}

// The node's m particles go to inbox slots k0 .. k0 + m - 1 (reserved by the
// caller); nc is the node's fluid density.  SPAWN_LANES lanes of one wave
// share a node: lane `sub` makes particles sub, sub + SPAWN_LANES, ...; the
// node-wide updates (bounds, ledger, the fluid set to zero) come from lane 0
// of the group after the group's sums.
constexpr int SPAWN_LANES = 16;
__device__ inline void spawn_node(const GridP &g, const SpecP &sp, int isp, long long c, real nc, int m, int k0,
                                  int sub,
                                  real *__restrict__ n, real *__restrict__ ux, real *__restrict__ uy,
                                  real *__restrict__ uz, const WarmP &wp, jglob_t *__restrict__ Jx,
                                  jglob_t *__restrict__ Jy, jglob_t *__restrict__ Jz, uint64_t seed, int step,
                                  const PArr &inbox, int inbox_cap, int *__restrict__ deferred,
                                  unsigned *__restrict__ wmax_bits, unsigned *__restrict__ umax2,
                                  double *__restrict__ ledger, jsum_t *st) {
    int i, j, k;
    node_ijk(g, c, i, j, k);
    const int per = g.bcx == HK_BC_PERIODIC;
    const int nxn = per ? g.nx : g.nx + 1;
    const real dv = g.dx * g.dy * g.dz;
    const real mass = nc * dv;
    if (k0 + m > inbox_cap) {
        // no room this step: the node stays fluid; void the reserved slots
        for (int q = k0 + sub; q < inbox_cap && q < k0 + m; q += SPAWN_LANES) inbox.cell[q] = -1;
        if (sub == 0) atomicAdd(deferred, 1);
        return;
    }
    const real w = mass / (real)m;
    if (sub == 0 && __float_as_uint(fabsf((float)w)) > *wmax_bits)
        atomicMax(wmax_bits, __float_as_uint(fabsf((float)w)));
    const real u[3] = {ux[c], uy[c], uz[c]};
    double sig = 0.0, before = 0.0, after = 0.0;
    if (wp.S) {
        const double pr = (double)wp.S[c] * pow((double)nc, wp.ga - 1.0);
        sig = sqrt(fmax(pr / (double)nc, 0.0) / (double)sp.m);
        before = (double)mass * (double)sp.m *
                     (sqrt(1.0 + (double)u[0] * u[0] + (double)u[1] * u[1] + (double)u[2] * u[2]) - 1.0) +
                 pr * (double)dv / (wp.ga - 1.0);
    }
    // the new particles sit in cells next to the node: raise the bound of
    // the node's tile (the moments read the bounds of neighbouring tiles too)
    const int tile = (min(i, g.nx - 1) >> TLOG) + g.ntx * ((j >> TLOG) + g.nty * (k >> TLOG));
    float u2max = (float)(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const uint64_t node = (uint64_t)i + (uint64_t)nxn * ((uint64_t)j + (uint64_t)g.ny * k);
    const real qw = sp.q * w / dv;
    for (int q = sub; q < m; q += SPAWN_LANES) {
        uint32_t r[4];
        draw4(seed, node, (uint32_t)step, TAG_CONV, (uint32_t)q, r);
        real X1[3] = {u01(r[0]) - (real)0.5, u01(r[1]) - (real)0.5, u01(r[2]) - (real)0.5};
        if (!per && ((i == 0 && X1[0] < (real)0) || (i == g.nx && X1[0] >= (real)0))) X1[0] = -X1[0];
        AxisS SX = axis_shapes((real)0, X1[0]), SY = axis_shapes((real)0, X1[1]),
              SZ = axis_shapes((real)0, X1[2]);
        spawn_current_add(g, st, Jx, Jy, Jz, i, j, k, SX, SY, SZ, qw * g.dx / g.dt, qw * g.dy / g.dt,
                          qw * g.dz / g.dt);
        int cc[3] = {i, j, k};
        for (int d = 0; d < 3; ++d)
            if (X1[d] < (real)0) { cc[d] -= 1; X1[d] += (real)1; }
        if (per) cc[0] = wrapi(cc[0], g.nx);
        cc[1] = wrapi(cc[1], g.ny);
        cc[2] = wrapi(cc[2], g.nz);
        real uq[3] = {u[0], u[1], u[2]};
        const uint64_t pid = (1ull << 63) | ((uint64_t)step << 40) | ((uint64_t)isp << 37) | (node << 6) |
                             (uint64_t)q;
        if (wp.S) {
            uint32_t t4[4];
            draw4(seed, pid, (uint32_t)step, TAG_CONV_TH, 0, t4);
            const double r0 = u01d(t4[0]), r1 = u01d(t4[1]), r2 = u01d(t4[2]), r3 = u01d(t4[3]);
            const double m0 = sqrt(-2.0 * log(r0)), m1 = sqrt(-2.0 * log(r2));
            const double tp = 6.283185307179586;
            uq[0] = (real)((double)u[0] + sig * m0 * cos(tp * r1));
            uq[1] = (real)((double)u[1] + sig * m0 * sin(tp * r1));
            uq[2] = (real)((double)u[2] + sig * m1 * cos(tp * r3));
            after += (double)w * (double)sp.m *
                     (sqrt(1.0 + (double)uq[0] * uq[0] + (double)uq[1] * uq[1] + (double)uq[2] * uq[2]) - 1.0);
            u2max = fmaxf(u2max, (float)(uq[0] * uq[0] + uq[1] * uq[1] + uq[2] * uq[2]));
        }
        const long long s = k0 + q;
        inbox.cell[s] = cc[0] + g.nx * (cc[1] + g.ny * cc[2]);
        inbox.rx[s] = X1[0]; inbox.ry[s] = X1[1]; inbox.rz[s] = X1[2];
        inbox.ux[s] = uq[0]; inbox.uy[s] = uq[1]; inbox.uz[s] = uq[2];
        inbox.w[s] = w;
        inbox.id[s] = pid;
        if (sp.has_z) inbox.zc[s] = (int)sp.q;
        if (sp.has_tau) inbox.tau[s] = tau0(seed, inbox.id[s]);
    }
    // the node's stencil to the global current (the group's LDS atomics came
    // first: one wave's LDS operations complete in order), cleared for the
    // group's next node
    for (int f = sub; f < SJ_FACES; f += SPAWN_LANES) {
        spawn_face_flush(g, f, st[f], Jx, Jy, Jz, i, j, k);
        st[f] = 0;
    }
    // the group's sums (the lanes of a group are SPAWN_LANES consecutive lanes)
    for (int o = SPAWN_LANES / 2; o > 0; o >>= 1) {
        u2max = fmaxf(u2max, __shfl_xor(u2max, o, SPAWN_LANES));
        if (wp.S) after += __shfl_xor(after, o, SPAWN_LANES);
    }
    if (sub != 0) return;
    if (u2max > 0.f) atomicMax(&umax2[tile], __float_as_uint(u2max));
    if (wp.S) {
        wp.S[c] = 0;
        atomicAdd(ledger, before - after);
    }
    n[c] = 0; ux[c] = 0; uy[c] = 0; uz[c] = 0;
}


// Nodes that spawn: kinetic, with fluid mass >= wmin.  A light pass over the
// node grid (two loads per node) that lists them for k_spawn.
__global__ void __launch_bounds__(BS)
k_spawn_find(GridP g, const uint8_t *__restrict__ sw, const real *__restrict__ n, real wmin,
             int *__restrict__ list, int *__restrict__ list_n, const int *__restrict__ xr) {
    // fluid exists only inside the species' x window: the grid strides over
    // its node columns alone (every lane of a block takes the same number of
    // turns, for the wave-wide list appends)
    const int nxn = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
    const int lo = max(xr[0], 0), hi = min(xr[1], nxn - 1);
    if (hi < lo) return;
    // one list atomic per block and turn: atomics on one address serialize
    // across the chip (about 10 ns each), so waves pool their counts in LDS.
    // A turn covers SF_U nodes per thread, loaded together: the search is
    // bound by the latency of its loads, not by their bytes, so a workgroup
    // takes its share of the window in about one turn.
    constexpr int SF_U = 16;
    static_assert(SF_U * (BS / 64) == 64, "one wave scans the workgroup's counts");
    __shared__ int s_off[64];
    const int lane = __lane_id(), wv = threadIdx.x >> 6;
    const unsigned w = (unsigned)(hi - lo + 1), total = w * (unsigned)g.ny * (unsigned)g.nz;
    const real dv = g.dx * g.dy * g.dz;
    for (unsigned t0 = blockIdx.x * (SF_U * BS); t0 < total; t0 += gridDim.x * (SF_U * BS)) {
        // node indices stay below 2^31
        int c[SF_U];
        uint8_t sv[SF_U];
        for (int u = 0; u < SF_U; ++u) {
            const unsigned t = t0 + u * BS + threadIdx.x;
            const unsigned row = t / w;
            c[u] = lo + (int)(t - row * w) + (int)row * g.sx;
            sv[u] = t < total ? sw[c[u]] : 0;
        }
        bool want[SF_U];
        for (int u = 0; u < SF_U; ++u) {
            const real nc = sv[u] ? n[c[u]] : (real)0;
            want[u] = sv[u] && nc * dv >= wmin && nc > (real)0;
        }
        uint64_t b[SF_U];
        for (int u = 0; u < SF_U; ++u) {
            b[u] = __ballot(want[u]);
            if (lane == 0) s_off[u * (BS / 64) + wv] = __popcll(b[u]);
        }
        __syncthreads();
        // the first wave turns the 64 counts into list offsets: a scan over
        // its lanes and one atomic for the workgroup's total
        if (wv == 0) {
            const int v = s_off[lane];
            int incl = v;
            for (int o = 1; o < 64; o <<= 1) {
                const int t = __shfl_up(incl, o);
                if (lane >= o) incl += t;
            }
            const int tot = __shfl(incl, 63);
            int base = 0;
            if (lane == 0 && tot) base = atomicAdd(list_n, tot);
            base = __shfl(base, 0);
            s_off[lane] = base + incl - v;
        }
        __syncthreads();
        for (int u = 0; u < SF_U; ++u)
            if (want[u])
                list[s_off[u * (BS / 64) + wv] + __popcll(b[u] & ((1ull << lane) - 1ull))] = c[u];
        __syncthreads();
    }
}

// One listed node becomes particles (one thread per node).  A warm node's
// particles get the fluid momentum plus a Gaussian spread sqrt(T / m) per
// component, T = p / n (Box-Muller on Philox draws, tag TAG_CONV_TH, keyed by
// the particle's id); the ledger takes the fluid's kinetic plus thermal
// energy minus the sample's kinetic energy.  Positions (tag TAG_CONV) are
// keyed by (node, step, slot), shared by the species spawned on one node.
__global__ void __launch_bounds__(BS)
k_spawn(GridP g, SpecP sp, int isp, real *__restrict__ n, real *__restrict__ ux,
        real *__restrict__ uy, real *__restrict__ uz, WarmP wp, jglob_t *__restrict__ Jx,
        jglob_t *__restrict__ Jy, jglob_t *__restrict__ Jz, real w0, uint64_t seed, int step, PArr inbox,
        int *__restrict__ inbox_n, int inbox_cap, int *__restrict__ deferred,
        unsigned *__restrict__ wmax_bits, unsigned *__restrict__ umax2, double *__restrict__ ledger,
        const int *__restrict__ list, const int *__restrict__ list_n) {
    __shared__ jsum_t sst[BS / SPAWN_LANES][SJ_FACES];
    const int nl = *list_n;
    const int lane = __lane_id();
    const real dv = g.dx * g.dy * g.dz;
    jsum_t *st = sst[threadIdx.x / SPAWN_LANES];
    for (int f = lane % SPAWN_LANES; f < SJ_FACES; f += SPAWN_LANES) st[f] = 0;
    // SPAWN_LANES lanes per listed node, 64 / SPAWN_LANES nodes per wave and
    // turn; the wave reserves its nodes' inbox slots with one atomic (an
    // atomic per node on the one counter would serialize, about 10 ns each)
    constexpr int NPW = 64 / SPAWN_LANES;
    const int grp = lane / SPAWN_LANES, sub = lane % SPAWN_LANES;
    const int wave = (int)((blockIdx.x * BS + threadIdx.x) >> 6), nwaves = (int)((gridDim.x * BS) >> 6);
    for (int eb = wave * NPW; eb < nl; eb += nwaves * NPW) {
        const int e = eb + grp;
        const bool on = e < nl;
        const long long c = on ? list[e] : 0;
        const real nc = on ? n[c] : (real)0;
        const int m = on ? spawn_count(nc * dv, w0) : 0;
        int before = 0, tot = 0;
#pragma unroll
        for (int q = 0; q < NPW; ++q) {
            const int mq = __shfl(m, q * SPAWN_LANES);
            before += q < grp ? mq : 0;
            tot += mq;
        }
        int base = 0;
        if (lane == 0 && tot) base = atomicAdd(inbox_n, tot);
        base = __shfl(base, 0);
        if (on)
            spawn_node(g, sp, isp, c, nc, m, base + before, sub, n, ux, uy, uz, wp, Jx, Jy, Jz, seed, step, inbox,
                       inbox_cap, deferred, wmax_bits, umax2, ledger, st);
    }
}
inline unsigned blocks(long long n) { return (unsigned)((n + BS - 1) / BS); }
inline unsigned xcd_blocks(long long n) { return (blocks(n) + 7u) & ~7u; }

}  // namespace

void launch_moments_tiles(const GridP &g, const SpecP &sp, PArr a, Bins b, int ion_only,
                          int zmax, real hot2, real *mom, const unsigned *wmax_bits, const unsigned *umax2,
                          const int *active, int2 *items, int *ctl, long long capacity, hipStream_t s) {
    launch_tile_plan(g, sp, b, MOM_CHUNK, items, ctl, s);
    k_moments<<<tile_plan_grid(g, capacity, MOM_CHUNK), MBS, 0, s>>>(g, sp, a, b, ion_only, zmax, hot2, mom,
                                                                  wmax_bits, umax2, active, items, ctl);
}
void launch_fluid_moments_nodes(const GridP &g, real inv_ppc, const real *n, const real *ux,
                                const real *uy, const real *uz, real *mom, int first, hipStream_t s) {
    k_fluid_moments<<<blocks(g.nn), BS, 0, s>>>(g, inv_ppc, n, ux, uy, uz, mom, first);
}
void launch_indicators_nodes(const GridP &g, const SwitchP &P, const real *mom, real *const f[9],
                             const IonP *const *ions, int nion, uint8_t *hot, uint8_t *notcold,
                             hipStream_t s) {
    IonSet set{};
    set.n = nion < 4 ? nion : 4;
    for (int q = 0; q < set.n; ++q) set.p[q] = ions[q];
    k_indicators<<<xcd_blocks(g.nn), BS, 0, s>>>(g, P, mom, f[HK_EX], f[HK_EY], f[HK_EZ], set, hot, notcold);
}
void launch_label_nodes(const GridP &g, const SwitchP &P, const real *mom, real *const f[9],
                        const IonP *const *ions, int nion, uint8_t *cond, hipStream_t s) {
    IonSet set{};
    set.n = nion < 4 ? nion : 4;
    for (int q = 0; q < set.n; ++q) set.p[q] = ions[q];
    const int NX = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
    k_label_cond<<<blocks((long long)NX * g.ny * g.nz), BS, 0, s>>>(g, P, mom, f[HK_EX], f[HK_EY], f[HK_EZ],
                                                                    set, cond);
}
void launch_flags_canonical(const GridP &g, const uint8_t *src, uint8_t *dst, hipStream_t s) {
    const int NX = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
    k_flags_canonical<<<blocks((long long)NX * g.ny * g.nz), BS, 0, s>>>(g, src, dst);
}
void launch_label_or(long long n, const uint8_t *cond, uint8_t *y, hipStream_t s) {
    k_label_or<<<blocks(n), BS, 0, s>>>(n, cond, y);
}
void launch_dilate_nodes(const GridP &g, const SwitchP &P, const uint8_t *hot, const uint8_t *notcold,
                         uint8_t *sw, uint8_t *calm, uint8_t *tmp, hipStream_t s) {
    const unsigned nb = xcd_blocks(g.nn);
    k_dilate_x<<<nb, BS, 0, s>>>(g, P.dilation, hot, notcold, tmp);
    k_dilate_yz<<<nb, BS, 0, s>>>(g, P.dilation, 1, tmp, tmp + g.nn);
    k_dilate_apply<<<nb, BS, 0, s>>>(g, P, tmp + g.nn, sw, calm);
}
void launch_absorb_finish_nodes(const GridP &g, real mass, double *macc, real *n, real *ux,
                                real *uy, real *uz, WarmP w, double *ledger, const int *xr, hipStream_t s) {
    // few blocks: each adds its energy sum to the ledger with one atomic
    k_absorb_finish<<<512, BS, 0, s>>>(g, mass, macc, n, ux, uy, uz, w, ledger, xr);
}
void launch_spawn_nodes(const GridP &g, const SpecP &sp, int isp, const uint8_t *sw, real *n, real *ux,
                        real *uy, real *uz, WarmP w, jglob_t *jg, real wmin, real w0, uint64_t seed,
                        int step, PArr inbox, int *inbox_n, int inbox_cap, int *deferred,
                        unsigned *wmax_bits, unsigned *umax2, double *ledger, int *list, int *list_n,
                        const int *xr, hipStream_t s) {
    k_spawn_find<<<2048, BS, 0, s>>>(g, sw, n, wmin, list, list_n, xr);
    k_spawn<<<1024, BS, 0, s>>>(g, sp, isp, n, ux, uy, uz, w, jg, jg + g.nn, jg + 2 * g.nn, w0, seed, step,
                                inbox, inbox_n, inbox_cap, deferred, wmax_bits, umax2, ledger, list, list_n);
}
