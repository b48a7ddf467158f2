// FP64 diagnostic reductions: field energy, particle and fluid kinetic energy,
// counts and charge, the Gauss residual, the kinetic fraction.
//
// Paper: Methodology, post-processing paragraph (total energy from the
// electromagnetic, kinetic and thermal parts) and validation paragraph
// (charge and energy conservation checks during switches and steps).  Every
// accumulator is FP64 in both builds; blocks reduce in LDS and add one value
// per block to the result with a global FP64 atomic.
#include "hk_internal.h"

namespace {

constexpr int BS = 256;

__device__ inline void block_add(double v, double *out) {
    __shared__ double red[BS / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0;
        for (int i = 0; i < BS / 64; ++i) s += red[i];
        atomicAdd(out, s);
    }
    __syncthreads();
}


__global__ void __launch_bounds__(BS)
k_field_energy(GridP g, const real *Ex, const real *Ey, const real *Ez, const real *Bx,
               const real *By, const real *Bz, double *out) {
    long long c = (long long)blockIdx.x * BS + threadIdx.x;
    double ee = 0, bb = 0;
    if (c < g.nn) {
        int i, j, k;
        node_ijk(g, c, i, j, k);
        const int per = g.bcx == HK_BC_PERIODIC;
        bool half_ok = i < g.nx, node_ok = per ? i < g.nx : true;
        if (half_ok) {
            double a = Ex[c], b = By[c], d = Bz[c];
            ee += a * a;
            bb += b * b + d * d;
        }
        if (node_ok) {
            double a = Ey[c], b = Ez[c], d = Bx[c];
            ee += a * a + b * b;
            bb += d * d;
        }
    }
    double dv = g.ddx * g.ddy * g.ddz;
    block_add(0.5 * ee * dv, out);
    block_add(0.5 * bb * dv, out + 1);
}

// out[0] kinetic energy, out[1] count, out[2] charge
__global__ void __launch_bounds__(BS)
k_particle_sums(GridP g, SpecP sp, PArr a, Bins bins, double *out) {
    const int t = blockIdx.x;
    int nf, nbv;
    const int n = bin_count(sp, bins, t, nf, nbv);
    double ke = 0, num = 0, ch = 0;
    for (int p = threadIdx.x; p < n; p += BS) {
        long long ip = bin_slot(sp, t, p, nf, nbv);
        if (a.cell[ip] < 0) continue;
        double ux = a.ux[ip], uy = a.uy[ip], uz = a.uz[ip], w = a.w[ip];
        double u2 = ux * ux + uy * uy + uz * uz;
        if (sp.kind == HK_PHOTON) ke += w * sqrt(u2);
        else ke += w * (double)sp.m * (sqrt(1.0 + u2) - 1.0);
        num += 1.0;
        ch += (sp.has_z ? (double)a.zc[ip] : (double)sp.q) * w;
    }
    block_add(ke, out);
    block_add(num, out + 1);
    block_add(ch, out + 2);
}

// out[0] fluid kinetic energy, out[1] mass (sum n dV), out[2] charge
__global__ void __launch_bounds__(BS)
k_fluid_sums(GridP g, SpecP sp, const real *n, const real *ux, const real *uy, const real *uz,
             double *out) {
    long long c = (long long)blockIdx.x * BS + threadIdx.x;
    double ke = 0, m = 0;
    if (c < g.nn) {
        double dv = g.ddx * g.ddy * g.ddz;
        double mm = (double)n[c] * dv;
        double a = ux[c], b = uy[c], d = uz[c];
        m = mm;
        ke = mm * (double)sp.m * (sqrt(1.0 + a * a + b * b + d * d) - 1.0);
    }
    block_add(ke, out);
    block_add(m, out + 1);
    block_add(m * (double)sp.q, out + 2);
}

// Gauss residual change: r = divE - rho - g0 over interior nodes (open x
// skips the wall planes and the antenna plane).  out[0] sum r^2, out[1] count,
// out[2] max |r| (as the bit pattern of a non-negative double).
__global__ void __launch_bounds__(BS)
k_gauss(GridP g, const double *dive, const double *rho, const double *g0, int skip_plane,
        double *out) {
    long long c = (long long)blockIdx.x * BS + threadIdx.x;
    double r2 = 0, num = 0, mx = 0;
    if (c < g.nn) {
        int i, j, k;
        node_ijk(g, c, i, j, k);
        const int per = g.bcx == HK_BC_PERIODIC;
        bool ok = i < g.nx && (per || (i != 0 && i != skip_plane));
        if (ok) {
            double r = dive[c] - rho[c] - g0[c];
            r2 = r * r;
            num = 1;
            mx = fabs(r);
        }
    }
    block_add(r2, out);
    block_add(num, out + 1);
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_down(mx, o));
    if ((threadIdx.x & 63) == 0 && mx > 0)
        atomicMax((unsigned long long *)(out + 2), (unsigned long long)__double_as_longlong(mx));
}

__global__ void __launch_bounds__(BS)
k_count_kinetic(GridP g, const uint8_t *sw, double *out) {
    long long c = (long long)blockIdx.x * BS + threadIdx.x;
    double kin = 0, tot = 0;
    if (c < g.nn) {
        int i = (int)(c % g.sx);
        int nxn = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
        if (i < nxn) { tot = 1; kin = sw[c] ? 1 : 0; }
    }
    block_add(kin, out);
    block_add(tot, out + 1);
}

__global__ void __launch_bounds__(BS)
k_fluid_rho(GridP g, real q, const real *n, double *rho) {
    long long c = (long long)blockIdx.x * BS + threadIdx.x;
    if (c < g.nn) rho[c] += (double)q * (double)n[c];
}

__global__ void __launch_bounds__(BS) k_sub(long long n, double *a, const double *b) {
    long long c = (long long)blockIdx.x * BS + threadIdx.x;
    if (c < n) a[c] -= b[c];
}

inline unsigned blocks(long long n) { return (unsigned)((n + BS - 1) / BS); }

}  // namespace

void launch_sub(long long n, double *a, const double *b, hipStream_t s) {
    k_sub<<<blocks(n), BS, 0, s>>>(n, a, b);
}

void launch_field_energy(const GridP &g, real *const f[9], double *out2, hipStream_t s) {
    k_field_energy<<<blocks(g.nn), BS, 0, s>>>(g, f[HK_EX], f[HK_EY], f[HK_EZ], f[HK_BX], f[HK_BY],
                                               f[HK_BZ], out2);
}
void launch_particle_sums(const GridP &g, const SpecP &sp, PArr a, Bins b, double *out3,
                          hipStream_t s) {
    k_particle_sums<<<g.ntiles, BS, 0, s>>>(g, sp, a, b, out3);
}
void launch_fluid_sums(const GridP &g, const SpecP &sp, const real *n, const real *ux,
                       const real *uy, const real *uz, double *out3, hipStream_t s) {
    k_fluid_sums<<<blocks(g.nn), BS, 0, s>>>(g, sp, n, ux, uy, uz, out3);
}
void launch_gauss(const GridP &g, const double *dive, const double *rho, const double *g0,
                  int skip_plane, double *out3, hipStream_t s) {
    k_gauss<<<blocks(g.nn), BS, 0, s>>>(g, dive, rho, g0, skip_plane, out3);
}
void launch_count_kinetic(const GridP &g, const uint8_t *sw, double *out2, hipStream_t s) {
    k_count_kinetic<<<blocks(g.nn), BS, 0, s>>>(g, sw, out2);
}
void launch_fluid_rho(const GridP &g, const SpecP &sp, const real *n, double *rho, hipStream_t s) {
    k_fluid_rho<<<blocks(g.nn), BS, 0, s>>>(g, sp.q, n, rho);
}
