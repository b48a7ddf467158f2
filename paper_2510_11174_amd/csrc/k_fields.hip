// Yee FDTD field kernels for gfx950: half-step B, full-step E with first-order
// Mur walls, current-sheet laser antenna, discrete div E.
//
// Paper: Methodology, FDTD paragraphs (explicit Maxwell on a uniform grid),
// boundary paragraph (first-order Mur, coefficient (c dt - d)/(c dt + d)) and
// laser paragraph (Gaussian temporal and spatial envelopes on E by
// polarization).  These kernels are bound by HBM traffic: one thread per
// grid sample, x fastest, so each wavefront streams 64 consecutive floats of
// every array it touches.
#include "hk_internal.h"

namespace {

constexpr int BS = 256;

// Node of this thread in an XCD-aware launch: workgroups go round-robin to
// the 8 XCDs, so block b takes item (b mod 8) q + b / 8 (q = grid / 8, the
// grid a multiple of 8) and each XCD sweeps a contiguous slab of nodes,
// whose y and z neighbour rows then sit in its own L2.
__device__ inline long long xcd_node() {
    const int q = gridDim.x >> 3;
    const int item = (blockIdx.x & 7) * q + (blockIdx.x >> 3);
    return (long long)item * BS + threadIdx.x;
}

__global__ void __launch_bounds__(BS) k_fill(uint32_t *p, size_t n, uint32_t v) {
    size_t i = (size_t)blockIdx.x * BS + threadIdx.x;
    if (i < n) p[i] = v;
}
// 16-byte stores for 16-byte aligned buffers (n counts uint4)
__global__ void __launch_bounds__(BS) k_fill16(uint4 *p, size_t n, uint32_t v) {
    for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS)
        p[i] = make_uint4(v, v, v, v);
}


// B <- B - dt/2 curl E.  Node-type Bx on x planes 0..nx (open) or 0..nx-1
// (periodic); half-type By, Bz on 0..nx-1.
__global__ void __launch_bounds__(BS)
k_b_half(GridP g, const real *__restrict__ Ex, const real *__restrict__ Ey,
         const real *__restrict__ Ez, real *__restrict__ Bx, real *__restrict__ By,
         real *__restrict__ Bz) {
    long long c = xcd_node();
    if (c >= g.nn) return;
    int i, j, k;
    node_ijk(g, c, i, j, k);
    const real h = (real)0.5 * g.dt;
    const int per = g.bcx == HK_BC_PERIODIC;
    const int jp = j + 1 == g.ny ? 0 : j + 1, kp = k + 1 == g.nz ? 0 : k + 1;
    const long long cjp = gidx(g, i, jp, k), ckp = gidx(g, i, j, kp);
    const int inode = per ? g.nx - 1 : g.nx;
    if (i <= inode) {
        real curlx = (Ez[cjp] - Ez[c]) / g.dy - (Ey[ckp] - Ey[c]) / g.dz;
        Bx[c] -= h * curlx;
    }
    if (i <= g.nx - 1) {
        const int ip = (per && i + 1 == g.nx) ? 0 : i + 1;
        const long long cip = gidx(g, ip, j, k);
        real curly = (Ex[ckp] - Ex[c]) / g.dz - (Ez[cip] - Ez[c]) / g.dx;
        real curlz = (Ey[cip] - Ey[c]) / g.dx - (Ex[cjp] - Ex[c]) / g.dy;
        By[c] -= h * curly;
        Bz[c] -= h * curlz;
    }
}

// E <- E + dt (curl B - J).  Ex on half planes 0..nx-1; Ey, Ez on interior
// node planes (1..nx-1 open, 0..nx-1 periodic).
__global__ void __launch_bounds__(BS)
k_e_full(GridP g, real *__restrict__ Ex, real *__restrict__ Ey, real *__restrict__ Ez,
         const real *__restrict__ Bx, const real *__restrict__ By, const real *__restrict__ Bz,
         const real *__restrict__ Jx, const real *__restrict__ Jy, const real *__restrict__ Jz) {
    long long c = xcd_node();
    if (c >= g.nn) return;
    int i, j, k;
    node_ijk(g, c, i, j, k);
    const real dt = g.dt;
    const int per = g.bcx == HK_BC_PERIODIC;
    const int jm = j == 0 ? g.ny - 1 : j - 1, km = k == 0 ? g.nz - 1 : k - 1;
    const long long cjm = gidx(g, i, jm, k), ckm = gidx(g, i, j, km);
    if (i <= g.nx - 1) {
        real curlx = (Bz[c] - Bz[cjm]) / g.dy - (By[c] - By[ckm]) / g.dz;
        Ex[c] += dt * (curlx - Jx[c]);
    }
    const int i0 = per ? 0 : 1;
    if (i >= i0 && i <= g.nx - 1) {
        const int im = (per && i == 0) ? g.nx - 1 : i - 1;
        const long long cim = gidx(g, im, j, k);
        real curly = (Bx[c] - Bx[ckm]) / g.dz - (Bz[c] - Bz[cim]) / g.dx;
        real curlz = (By[c] - By[cim]) / g.dx - (Bx[c] - Bx[cjm]) / g.dy;
        Ey[c] += dt * (curly - Jy[c]);
        Ez[c] += dt * (curlz - Jz[c]);
    }
}

// Keep planes 0, 1, nx-1, nx of Ey and Ez at time n for Mur.
__global__ void __launch_bounds__(BS)
k_mur_save(GridP g, const real *__restrict__ Ey, const real *__restrict__ Ez,
           real *__restrict__ old) {
    int p = blockIdx.x * BS + threadIdx.x;
    int plane = g.ny * g.nz;
    if (p >= plane) return;
    int j = p % g.ny, k = p / g.ny;
    old[0 * plane + p] = Ey[gidx(g, 0, j, k)];
    old[1 * plane + p] = Ey[gidx(g, 1, j, k)];
    old[2 * plane + p] = Ez[gidx(g, 0, j, k)];
    old[3 * plane + p] = Ez[gidx(g, 1, j, k)];
    old[4 * plane + p] = Ey[gidx(g, g.nx, j, k)];
    old[5 * plane + p] = Ey[gidx(g, g.nx - 1, j, k)];
    old[6 * plane + p] = Ez[gidx(g, g.nx, j, k)];
    old[7 * plane + p] = Ez[gidx(g, g.nx - 1, j, k)];
}

// First-order Mur: E(wall)^{n+1} = E(in)^n + cm (E(in)^{n+1} - E(wall)^n).
__global__ void __launch_bounds__(BS)
k_mur_apply(GridP g, real *__restrict__ Ey, real *__restrict__ Ez, const real *__restrict__ old) {
    int p = blockIdx.x * BS + threadIdx.x;
    int plane = g.ny * g.nz;
    if (p >= plane) return;
    int j = p % g.ny, k = p / g.ny;
    const real cm = (g.dt - g.dx) / (g.dt + g.dx);
    Ey[gidx(g, 0, j, k)] = old[1 * plane + p] + cm * (Ey[gidx(g, 1, j, k)] - old[0 * plane + p]);
    Ez[gidx(g, 0, j, k)] = old[3 * plane + p] + cm * (Ez[gidx(g, 1, j, k)] - old[2 * plane + p]);
    Ey[gidx(g, g.nx, j, k)] =
        old[5 * plane + p] + cm * (Ey[gidx(g, g.nx - 1, j, k)] - old[4 * plane + p]);
    Ez[gidx(g, g.nx, j, k)] =
        old[7 * plane + p] + cm * (Ez[gidx(g, g.nx - 1, j, k)] - old[6 * plane + p]);
}

// Sheet current J = -2 E_laser / dx on node plane ia.  Evaluated in FP64: t
// reaches a few hundred, where an FP32 carrier phase would lose 1e-5.
__global__ void __launch_bounds__(BS)
k_antenna(GridP g, hk_laser_desc L, double t, real *__restrict__ Jy, real *__restrict__ Jz) {
    int p = blockIdx.x * BS + threadIdx.x;
    if (p >= g.ny * g.nz) return;
    int j = p % g.ny, k = p / g.ny;
    double tc = L.t_center > 0 ? L.t_center : 2.0 * L.duration;
    double a = (t - tc) / L.duration;
    double env_t = exp(-a * a);
    double yc = 0.5 * g.ny * g.ddy, zc = 0.5 * g.nz * g.ddz;
    double w2 = L.waist * L.waist;
    double y = (j + 0.5) * g.ddy - yc, z = k * g.ddz - zc;
    double ey = L.a0 * env_t * exp(-(y * y + z * z) / w2) * sin(t);
    long long c = gidx(g, L.i_antenna, j, k);
    Jy[c] += (real)(-2.0 * ey / g.ddx);
    if (L.polarization == 1) {
        double y2 = j * g.ddy - yc, z2 = (k + 0.5) * g.ddz - zc;
        double ez = L.a0 * env_t * exp(-(y2 * y2 + z2 * z2) / w2) * cos(t);
        Jz[c] += (real)(-2.0 * ez / g.ddx);
    }
}

__global__ void __launch_bounds__(BS)
k_divE(GridP g, const real *__restrict__ Ex, const real *__restrict__ Ey,
       const real *__restrict__ Ez, double *__restrict__ out) {
    long long c = (long long)blockIdx.x * BS + threadIdx.x;
    if (c >= g.nn) return;
    int i, j, k;
    node_ijk(g, c, i, j, k);
    const int per = g.bcx == HK_BC_PERIODIC;
    double v = 0.0;
    if ((per && i < g.nx) || (!per && i >= 1 && i <= g.nx - 1)) {
        int im = (per && i == 0) ? g.nx - 1 : i - 1;
        v = ((double)Ex[c] - (double)Ex[gidx(g, im, j, k)]) / g.ddx +
            ((double)Ey[c] - (double)Ey[gidx(g, i, j == 0 ? g.ny - 1 : j - 1, k)]) / g.ddy +
            ((double)Ez[c] - (double)Ez[gidx(g, i, j, k == 0 ? g.nz - 1 : k - 1)]) / g.ddz;
    }
    out[c] = v;
}

inline unsigned blocks(long long n) { return (unsigned)((n + BS - 1) / BS); }
// grid of an XCD-aware launch over n nodes
inline unsigned xcd_blocks(long long n) { return (blocks(n) + 7u) & ~7u; }

}  // namespace

void launch_fill32(void *p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return;
    const size_t n16 = ((uintptr_t)p & 15) ? 0 : n / 4;
    if (n16 >= 1024) {
        const long long nb = std::min<long long>(blocks((long long)n16), 4096);
        k_fill16<<<(unsigned)nb, BS, 0, s>>>((uint4 *)p, n16, v);
        n -= 4 * n16;
        if (n == 0) return;
        p = (uint32_t *)p + 4 * n16;
    }
    k_fill<<<blocks((long long)n), BS, 0, s>>>((uint32_t *)p, n, v);
}

void launch_zero(void *p, size_t bytes, hipStream_t s) { launch_fill32(p, bytes / 4, 0u, s); }

void launch_yee_b_half(const GridP &g, real *const f[9], hipStream_t s) {
    k_b_half<<<xcd_blocks(g.nn), BS, 0, s>>>(g, f[HK_EX], f[HK_EY], f[HK_EZ], f[HK_BX], f[HK_BY],
                                         f[HK_BZ]);
}

void launch_yee_e_full(const GridP &g, real *const f[9], real *mur_old, hipStream_t s) {
    const int plane = g.ny * g.nz;
    if (g.bcx == HK_BC_OPEN) k_mur_save<<<blocks(plane), BS, 0, s>>>(g, f[HK_EY], f[HK_EZ], mur_old);
    k_e_full<<<xcd_blocks(g.nn), BS, 0, s>>>(g, f[HK_EX], f[HK_EY], f[HK_EZ], f[HK_BX], f[HK_BY],
                                         f[HK_BZ], f[HK_JX], f[HK_JY], f[HK_JZ]);
    if (g.bcx == HK_BC_OPEN) k_mur_apply<<<blocks(plane), BS, 0, s>>>(g, f[HK_EY], f[HK_EZ], mur_old);
}

void launch_antenna(const GridP &g, const hk_laser_desc &L, double t, real *jy, real *jz,
                    hipStream_t s) {
    if (!L.enabled) return;
    k_antenna<<<blocks(g.ny * g.nz), BS, 0, s>>>(g, L, t, jy, jz);
}

// J += the particle current of this step (global accumulator jg, 3 arrays of
// nn), which is cleared for the next step.  Only nodes with a deposit are
// written.  FP32 build: one rounding of the exact fixed-point sum.
__global__ void __launch_bounds__(BS)
k_jconvert(GridP g, jglob_t *__restrict__ jg, real *__restrict__ Jx, real *__restrict__ Jy,
           real *__restrict__ Jz) {
    long long c = xcd_node();
    if (c >= g.nn) return;
    real *J[3] = {Jx, Jy, Jz};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const jglob_t v = jg[q * g.nn + c];
        if (v == (jglob_t)0) continue;
#ifdef HK_DOUBLE
        J[q][c] += v;
#else
        J[q][c] += (real)((double)(long long)v * (1.0 / (double)(1ull << JG_BITS)));
#endif
        jg[q * g.nn + c] = 0;
    }
}

void launch_jconvert(const GridP &g, jglob_t *jg, real *const f[9], hipStream_t s) {
    k_jconvert<<<xcd_blocks(g.nn), BS, 0, s>>>(g, jg, f[HK_JX], f[HK_JY], f[HK_JZ]);
}

void launch_divE(const GridP &g, real *const f[9], double *out, hipStream_t s) {
    k_divE<<<blocks(g.nn), BS, 0, s>>>(g, f[HK_EX], f[HK_EY], f[HK_EZ], out);
}
