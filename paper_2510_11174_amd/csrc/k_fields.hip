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
    const real rdx = (real)1 / g.dx, rdy = (real)1 / g.dy, rdz = (real)1 / g.dz;
    const int per = g.bcx == HK_BC_PERIODIC;
    const int jp = j + 1 == g.ny ? 0 : j + 1, kp = k + 1 == g.nz ? 0 : k + 1;
    const long long cjp = gidx(g, i, jp, k), ckp = gidx(g, i, j, kp);
    const int inode = per ? g.nx - 1 : g.nx;
    if (i <= inode) {
        real curlx = (Ez[cjp] - Ez[c]) * rdy - (Ey[ckp] - Ey[c]) * rdz;
        Bx[c] -= h * curlx;
    }
    if (i <= g.nx - 1) {
        const int ip = (per && i + 1 == g.nx) ? 0 : i + 1;
        const long long cip = gidx(g, ip, j, k);
        real curly = (Ex[ckp] - Ex[c]) * rdz - (Ez[cip] - Ez[c]) * rdx;
        real curlz = (Ey[cip] - Ey[c]) * rdx - (Ex[cjp] - Ex[c]) * rdy;
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
    const real rdx = (real)1 / g.dx, rdy = (real)1 / g.dy, rdz = (real)1 / g.dz;
    const int per = g.bcx == HK_BC_PERIODIC;
    const int jm = j == 0 ? g.ny - 1 : j - 1, km = k == 0 ? g.nz - 1 : k - 1;
    const long long cjm = gidx(g, i, jm, k), ckm = gidx(g, i, j, km);
    if (i <= g.nx - 1) {
        real curlx = (Bz[c] - Bz[cjm]) * rdy - (By[c] - By[ckm]) * rdz;
        Ex[c] += dt * (curlx - Jx[c]);
    }
    const int i0 = per ? 0 : 1;
    if (i >= i0 && i <= g.nx - 1) {
        const int im = (per && i == 0) ? g.nx - 1 : i - 1;
        const long long cim = gidx(g, im, j, k);
        real curly = (Bx[c] - Bx[ckm]) * rdz - (Bz[c] - Bz[cim]) * rdx;
        real curlz = (By[c] - By[cim]) * rdx - (Bx[c] - Bx[cjm]) * rdy;
        Ey[c] += dt * (curly - Jy[c]);
        Ez[c] += dt * (curlz - Jz[c]);
    }
}

// ------------------------------------------------------------------ fused step
// The whole field update of a step (B half step, E full step with the Mur
// walls, B half step) in one pass: E^n and B^n are read from one buffer set
// and E^{n+1}, B^{n+1} written to the other, so no workgroup reads what
// another has written and every workgroup may recompute the values next to
// its tile.  A workgroup owns a YT_X x YT_Y column of nodes (x, y) and a
// chunk of YT_Z planes, and marches through the chunk in z.  Its threads form
// the column widened by one node below and two above in x and y: B^{n+1/2}
// at a node needs E^n at the +x, +y, +z neighbours, E^{n+1} needs B^{n+1/2}
// at -x, -y, -z, and B^{n+1} needs E^{n+1} at +x, +y, +z.  The in-plane
// neighbours come through LDS, the z neighbours through registers.  Each
// value is the same expression as in the separate kernels above (both
// multiply by the reciprocal spacings), so the result is the same bits.  Traffic per node: E, B, J read and E, B written
// once (60 B in FP32), against 120 B for the three separate passes.
constexpr int YT_TX = 32, YT_TY = 16;               // threads per workgroup in x, y
constexpr int YT_X = YT_TX - 3, YT_Y = YT_TY - 3;   // owned nodes in x, y
constexpr int YT_Z = 32;                            // planes per workgroup

struct YeeIn {
    const real *Ex, *Ey, *Ez, *Bx, *By, *Bz, *Jx, *Jy, *Jz;
};
struct YeeOut {
    real *Ex, *Ey, *Ez, *Bx, *By, *Bz;
};

__global__ void __launch_bounds__(YT_TX * YT_TY)
k_yee_step(GridP g, YeeIn F, YeeOut O, int tiles_x, int tiles_y) {
    typedef real Plane[3][YT_TY][YT_TX];
    __shared__ Plane sE;       // E^n of the plane being advanced
    __shared__ Plane sH;       // B^{n+1/2} of that plane
    __shared__ Plane sN[2];    // E^{n+1} of planes k and k + 1 (alternating)
    const int tx = threadIdx.x % YT_TX, ty = threadIdx.x / YT_TX;
    const int b = blockIdx.x;
    const int bx = b % tiles_x, by = (b / tiles_x) % tiles_y, bz = b / (tiles_x * tiles_y);
    const int per = g.bcx == HK_BC_PERIODIC;
    const int nxp = per ? g.nx : g.nx + 1;   // node columns
    const int iu = bx * YT_X - 1 + tx, ju = by * YT_Y - 1 + ty;   // unwrapped
    int i = iu;
    bool inx = true;
    if (per) i = i < 0 ? i + g.nx : (i >= g.nx ? i - g.nx : i);
    else inx = i >= 0 && i < nxp;
    const int j = wrapi(ju, g.ny);
    const bool own = tx >= 1 && tx <= YT_X && ty >= 1 && ty <= YT_Y && iu < nxp && ju < g.ny;
    // periodic x: the node column x = nx (storage padding, never computed)
    // keeps its values in the other buffer set too
    const bool pad = per && iu == g.nx && ty >= 1 && ty <= YT_Y && ju < g.ny;
    const int z0 = bz * YT_Z, z1 = min(g.nz, z0 + YT_Z);
    const real h = (real)0.5 * g.dt, dt = g.dt;
    const int inode = per ? g.nx - 1 : g.nx;
    const int i0 = per ? 0 : 1;
    const real cm = (g.dt - g.dx) / (g.dt + g.dx);
    const real rdx = (real)1 / g.dx, rdy = (real)1 / g.dy, rdz = (real)1 / g.dz;
    // a wall node in this workgroup's columns (the Mur pass below is skipped otherwise)
    const bool walls = !per && (bx == 0 || (bx * YT_X - 1 <= g.nx && g.nx <= bx * YT_X - 1 + YT_TX - 1));
    const long long col = inx ? (long long)i + (long long)g.sx * j : 0;
    const long long pl = (long long)g.sx * g.ny;
    const bool xp = tx + 1 < YT_TX, yp = ty + 1 < YT_TY, xm = tx > 0, ym = ty > 0;
    auto zw = [&](int k) { return k < 0 ? k + g.nz : (k >= g.nz ? k - g.nz : k); };
    auto load3 = [&](const real *A, const real *B, const real *C, int k, real o[3]) {
        const long long c = col + pl * k;
        o[0] = inx ? A[c] : (real)0;
        o[1] = inx ? B[c] : (real)0;
        o[2] = inx ? C[c] : (real)0;
    };
    auto put = [&](Plane &S, const real v[3]) {
        S[0][ty][tx] = v[0]; S[1][ty][tx] = v[1]; S[2][ty][tx] = v[2];
    };
    // B - dt/2 curl E at this node: E of the plane in S (the in-plane
    // neighbours +x, +y), e1 = E of the plane above at this node
    auto curl_b = [&](const Plane &S, const real bn[3], const real e1[3], real o[3]) {
        const real ex = S[0][ty][tx], ey = S[1][ty][tx], ez = S[2][ty][tx];
        const real ezjp = yp ? S[2][ty + 1][tx] : (real)0, exjp = yp ? S[0][ty + 1][tx] : (real)0;
        const real ezip = xp ? S[2][ty][tx + 1] : (real)0, eyip = xp ? S[1][ty][tx + 1] : (real)0;
        o[0] = bn[0]; o[1] = bn[1]; o[2] = bn[2];
        if (i <= inode) {
            real curlx = (ezjp - ez) * rdy - (e1[1] - ey) * rdz;
            o[0] = bn[0] - h * curlx;
        }
        if (i <= g.nx - 1) {
            real curly = (e1[0] - ex) * rdz - (ezip - ez) * rdx;
            real curlz = (eyip - ey) * rdx - (exjp - ex) * rdy;
            o[1] = bn[1] - h * curly;
            o[2] = bn[2] - h * curlz;
        }
    };
    // E^{n+1} of plane k' at this node from E^n (en; the plane's E^n is in sE),
    // B^{n+1/2} of the plane (hk) and of the plane below (hm, this node), then
    // the Mur walls; the result goes to nw and to S for every thread
    auto new_e = [&](int kk, const real en[3], const real hk[3], const real hm[3], real nw[3], Plane &S) {
        real jc[3];
        load3(F.Jx, F.Jy, F.Jz, kk, jc);
        put(sH, hk);
        __syncthreads();
        const real bx_ = sH[0][ty][tx], by_ = sH[1][ty][tx], bz_ = sH[2][ty][tx];
        const real bzjm = ym ? sH[2][ty - 1][tx] : (real)0, bxjm = ym ? sH[0][ty - 1][tx] : (real)0;
        const real bzim = xm ? sH[2][ty][tx - 1] : (real)0, byim = xm ? sH[1][ty][tx - 1] : (real)0;
        nw[0] = en[0]; nw[1] = en[1]; nw[2] = en[2];
        if (i <= g.nx - 1) {
            real curlx = (bz_ - bzjm) * rdy - (by_ - hm[1]) * rdz;
            nw[0] = en[0] + dt * (curlx - jc[0]);
        }
        if (i >= i0 && i <= g.nx - 1) {
            real curly = (bx_ - hm[0]) * rdz - (bz_ - bzim) * rdx;
            real curlz = (by_ - byim) * rdx - (bx_ - bxjm) * rdy;
            nw[1] = en[1] + dt * (curly - jc[1]);
            nw[2] = en[2] + dt * (curlz - jc[2]);
        }
        put(S, nw);
        __syncthreads();
        if (!walls) return;
        // first-order Mur at the open walls from the inner neighbour's E^{n+1}
        // and E^n of both nodes
        bool wall = false;
        real wy = 0, wz = 0;
        if (!per && i == 0 && xp) {
            wy = sE[1][ty][tx + 1] + cm * (S[1][ty][tx + 1] - sE[1][ty][tx]);
            wz = sE[2][ty][tx + 1] + cm * (S[2][ty][tx + 1] - sE[2][ty][tx]);
            wall = true;
        } else if (!per && i == g.nx && xm) {
            wy = sE[1][ty][tx - 1] + cm * (S[1][ty][tx - 1] - sE[1][ty][tx]);
            wz = sE[2][ty][tx - 1] + cm * (S[2][ty][tx - 1] - sE[2][ty][tx]);
            wall = true;
        }
        __syncthreads();
        if (wall) {
            nw[1] = wy; nw[2] = wz;
            S[1][ty][tx] = wy; S[2][ty][tx] = wz;
        }
        __syncthreads();
    };

    // prologue: B^{n+1/2} of planes z0 - 1 and z0, E^{n+1} of z0
    real en0[3], en1[3], bn[3], hm[3], hk[3], nk[3];
    load3(F.Ex, F.Ey, F.Ez, zw(z0 - 1), nk);
    load3(F.Ex, F.Ey, F.Ez, z0, en0);
    load3(F.Ex, F.Ey, F.Ez, zw(z0 + 1), en1);
    load3(F.Bx, F.By, F.Bz, zw(z0 - 1), bn);
    put(sE, nk);
    __syncthreads();
    curl_b(sE, bn, en0, hm);
    load3(F.Bx, F.By, F.Bz, z0, bn);
    __syncthreads();
    put(sE, en0);
    __syncthreads();
    curl_b(sE, bn, en1, hk);
    new_e(z0, en0, hk, hm, nk, sN[0]);
    // at plane k: en1 = E^n(k + 1), hk = B^{n+1/2}(k) and nk = E^{n+1}(k) at
    // this node, sN[(k - z0) & 1] = E^{n+1}(k) of every thread
    for (int k = z0; k < z1; ++k) {
        const int a = (k - z0) & 1;
        real en2[3], hk1[3], nk1[3], bo[3];
        load3(F.Ex, F.Ey, F.Ez, zw(k + 2), en2);
        load3(F.Bx, F.By, F.Bz, zw(k + 1), bn);
        // (every read of sE in the last plane came before its last barrier)
        put(sE, en1);
        __syncthreads();
        curl_b(sE, bn, en2, hk1);
        new_e(zw(k + 1), en1, hk1, hk, nk1, sN[a ^ 1]);
        // B^{n+1}(k) = B^{n+1/2}(k) - dt/2 curl E^{n+1}
        curl_b(sN[a], hk, nk1, bo);
        if (own) {
            const long long c = col + pl * k;
            O.Ex[c] = nk[0]; O.Ey[c] = nk[1]; O.Ez[c] = nk[2];
            O.Bx[c] = bo[0]; O.By[c] = bo[1]; O.Bz[c] = bo[2];
        } else if (pad) {
            const long long c = (long long)g.nx + (long long)g.sx * j + pl * k;
            O.Ex[c] = F.Ex[c]; O.Ey[c] = F.Ey[c]; O.Ez[c] = F.Ez[c];
            O.Bx[c] = F.Bx[c]; O.By[c] = F.By[c]; O.Bz[c] = F.Bz[c];
        }
        for (int q = 0; q < 3; ++q) { en1[q] = en2[q]; hk[q] = hk1[q]; nk[q] = nk1[q]; }
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

bool launch_yee_step(const GridP &g, real *const f[9], real *const out[6], hipStream_t s) {
    const int per = g.bcx == HK_BC_PERIODIC;
    const int nxp = per ? g.nx : g.nx + 1;
    // the wall node x = nx takes its Mur value from the E^{n+1} of node
    // nx - 1, which a workgroup forms from its second thread column on: not
    // when x = nx is the first node it owns
    if (!per && g.nx % YT_X == 0) return false;
    const int tiles_x = (nxp + YT_X - 1) / YT_X, tiles_y = (g.ny + YT_Y - 1) / YT_Y;
    const int tiles_z = (g.nz + YT_Z - 1) / YT_Z;
    YeeIn F{f[HK_EX], f[HK_EY], f[HK_EZ], f[HK_BX], f[HK_BY], f[HK_BZ], f[HK_JX], f[HK_JY], f[HK_JZ]};
    YeeOut O{out[0], out[1], out[2], out[3], out[4], out[5]};
    k_yee_step<<<tiles_x * tiles_y * tiles_z, YT_TX * YT_TY, 0, s>>>(g, F, O, tiles_x, tiles_y);
    return true;
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
