// Particle kernels for gfx950.
//
// Paper: Methodology, plasma-model paragraph (macro-particles weighted by
// density and volume fraction, Boris pusher, ADK/multiphoton ionization joined
// by a Keldysh sigmoid), grid paragraph (deposition and gathering on the
// uniform grid) and boundary paragraph (velocity reversal at the walls).
// Literature: Boris (1970); Esirkepov, Comput. Phys. Commun. 135 (2001) 144;
// Ammosov, Delone, Krainov, Sov. Phys. JETP 64 (1986) 1191.
//
// Design.  Particles live in per-tile bins (TILE^3 cells) as SoA arrays with
// cell-relative offsets.  One workgroup owns one tile: it stages the tile's
// E and B (plus one guard cell) in LDS, gathers from LDS, pushes, deposits the
// Esirkepov current into an LDS J tile (guard 1 below, 2 above) with LDS
// atomics, flushes that tile to HBM with one global atomic per sample, and
// writes each pushed particle straight into its destination bin of the next
// buffer (wave-aggregated slot reservation for particles that stay).  Every
// particle byte is read once and written once per step.
#include "hk_internal.h"

namespace {

constexpr int BS = 256;
constexpr int FT = TILE + 2;       // field tile edge: cells -1 .. TILE
constexpr int FT3 = FT * FT * FT;
constexpr int JT = TILE + 3;       // current tile edge: nodes -1 .. TILE+1
constexpr int JT3 = JT * JT * JT;

__device__ inline int tile_of(const GridP &g, int cell) {
    int ci = cell % g.nx, r = cell / g.nx;
    int cj = r % g.ny, ck = r / g.ny;
    return (ci >> TLOG) + g.ntx * ((cj >> TLOG) + g.nty * (ck >> TLOG));
}

__device__ inline void copy_particle(const PArr &s, long long i, const PArr &d, long long j,
                                     int has_z, int has_tau) {
    d.cell[j] = s.cell[i];
    d.rx[j] = s.rx[i]; d.ry[j] = s.ry[i]; d.rz[j] = s.rz[i];
    d.ux[j] = s.ux[i]; d.uy[j] = s.uy[i]; d.uz[j] = s.uz[i];
    d.w[j] = s.w[i];
    d.id[j] = s.id[i];
    if (has_z) d.zc[j] = s.zc[i];
    if (has_tau) d.tau[j] = s.tau[i];
}

// ------------------------------------------------------------------ init ----------------
// Particle q of cell c: id = c * ppc + q; offsets from Philox tag 1, momenta by
// Box-Muller from tag 2 (FP64, rounded once to the storage type).
__global__ void __launch_bounds__(BS)
k_init(GridP g, int ppc, double u_th, double charge, uint64_t seed, const int *__restrict__ xcol,
       const double *__restrict__ wcol, int ncol, long long total, PArr out, int has_z,
       int has_tau) {
    long long tid = (long long)blockIdx.x * BS + threadIdx.x;
    if (tid >= total) return;
    int q = (int)(tid % ppc);
    long long r = tid / ppc;
    int col = (int)(r % ncol);
    long long jk = r / ncol;
    int j = (int)(jk % g.ny), k = (int)(jk / g.ny);
    int i = xcol[col];
    int cell = i + g.nx * (j + g.ny * k);
    uint64_t id = (uint64_t)cell * (uint64_t)ppc + (uint64_t)q;
    uint32_t rp[4], rm[4];
    draw4(seed, id, 0, TAG_POS, 0, rp);
    draw4(seed, id, 0, TAG_MOM, 0, rm);
    double r0 = u01d(rm[0]), r1 = u01d(rm[1]), r2 = u01d(rm[2]), r3 = u01d(rm[3]);
    double m0 = sqrt(-2.0 * log(r0)), m1 = sqrt(-2.0 * log(r2));
    const double tp = 6.283185307179586476925;
    out.cell[tid] = cell;
    out.rx[tid] = u01(rp[0]); out.ry[tid] = u01(rp[1]); out.rz[tid] = u01(rp[2]);
    out.ux[tid] = (real)(u_th * m0 * cos(tp * r1));
    out.uy[tid] = (real)(u_th * m0 * sin(tp * r1));
    out.uz[tid] = (real)(u_th * m1 * cos(tp * r3));
    out.w[tid] = (real)wcol[col];
    out.id[tid] = id;
    if (has_z) out.zc[tid] = (int)llround(charge);
    if (has_tau) out.tau[tid] = 0.0;
}

// --------------------------------------------------------- count / scatter ---------------
// Source bins: nsrc groups, group s holds slots [off[s], off[s] + min(cnt[s], cap[s])).
__global__ void __launch_bounds__(BS)
k_count(GridP g, PArr src, const long long *__restrict__ off, const int *__restrict__ cnt,
        const int *__restrict__ cap, int *__restrict__ newcnt) {
    int s = blockIdx.x;
    int n = min(cnt[s], cap[s]);
    long long b = off[s];
    for (int p = threadIdx.x; p < n; p += BS) {
        int cell = src.cell[b + p];
        if (cell >= 0) atomicAdd(&newcnt[tile_of(g, cell)], 1);
    }
}

__global__ void __launch_bounds__(BS)
k_scatter(GridP g, PArr src, const long long *__restrict__ off, const int *__restrict__ cnt,
          const int *__restrict__ cap, PArr dst, const long long *__restrict__ doff,
          int *__restrict__ dfill, int has_z, int has_tau) {
    int s = blockIdx.x;
    int n = min(cnt[s], cap[s]);
    long long b = off[s];
    for (int p = threadIdx.x; p < n; p += BS) {
        int cell = src.cell[b + p];
        if (cell < 0) continue;
        int t = tile_of(g, cell);
        int slot = atomicAdd(&dfill[t], 1);
        copy_particle(src, b + p, dst, doff[t] + slot, has_z, has_tau);
    }
}

// Inbox particles join their bins; those that do not fit go to `fail`.
__global__ void __launch_bounds__(BS)
k_merge(GridP g, SpecP sp, PArr inbox, const int *__restrict__ inbox_n, PArr dst,
        int *__restrict__ cnt, int *__restrict__ fail_n, PArr fail) {
    const long long n = *inbox_n;
    for (long long i = (long long)blockIdx.x * BS + threadIdx.x; i < n;
         i += (long long)gridDim.x * BS) {
        int cell = inbox.cell[i];
        if (cell < 0) continue;
        int t = tile_of(g, cell);
        int slot = atomicAdd(&cnt[t], 1);
        if (slot < sp.cap[t]) {
            copy_particle(inbox, i, dst, sp.off[t] + slot, sp.has_z, sp.has_tau);
        } else {
            int k = atomicAdd(fail_n, 1);
            copy_particle(inbox, i, fail, k, sp.has_z, sp.has_tau);
        }
    }
}

// ------------------------------------------------------------- the push -----------------
// CIC weights of a node-type (o) and a half-type (o - 1/2) sample along one
// axis, as an LDS index (field tile origin at cell -1) and fraction.
struct AxisW {
    int in_, ih;
    real fn, fh;
};
__device__ inline AxisW axis_weights(int l, real o) {
    AxisW a;
    a.in_ = l + 1;
    a.fn = o;
    if (o >= (real)0.5) { a.ih = l + 1; a.fh = o - (real)0.5; }
    else { a.ih = l; a.fh = o + (real)0.5; }
    return a;
}

__device__ inline real tri(const real *F, int i, int j, int k, real fx, real fy, real fz) {
    const int b = i + FT * (j + FT * k);
    real acc = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                real wgt = (a ? fx : 1 - fx) * (bb ? fy : 1 - fy) * (c ? fz : 1 - fz);
                acc += wgt * F[b + a + FT * (bb + FT * c)];
            }
    return acc;
}

// Esirkepov shape factors along one axis for a move from offset o to X1 = o +
// delta (relative to the old cell), written in terms of the displacement so
// that slow particles keep full relative precision.  Window nodes base..base+2
// relative to the old cell; base is -1 when the particle crossed downwards.
struct AxisS {
    int base;
    real S0[3], DS[3];
};
__device__ inline AxisS axis_shapes(real o, real X1) {
    AxisS s;
    if (X1 >= (real)1) {                // crossed up: nodes 0, 1, 2
        real e = X1 - (real)1;
        s.base = 0;
        s.S0[0] = (real)1 - o; s.S0[1] = o; s.S0[2] = 0;
        s.DS[0] = -((real)1 - o); s.DS[1] = ((real)1 - e) - o; s.DS[2] = e;
    } else if (X1 < (real)0) {          // crossed down: nodes -1, 0, 1
        real e = -X1;
        s.base = -1;
        s.S0[0] = 0; s.S0[1] = (real)1 - o; s.S0[2] = o;
        s.DS[0] = e; s.DS[1] = o - e; s.DS[2] = -o;
    } else {                            // stayed: nodes 0, 1, 2
        real d = X1 - o;
        s.base = 0;
        s.S0[0] = (real)1 - o; s.S0[1] = o; s.S0[2] = 0;
        s.DS[0] = -d; s.DS[1] = d; s.DS[2] = 0;
    }
    return s;
}

// Deposit the Esirkepov current of one particle into the LDS J tile.  (lx, ly,
// lz) is the old cell inside the tile; cx = q w / dV * dx / dt (per axis).
__device__ inline void esirkepov_lds(real *sJ, int lx, int ly, int lz, const AxisS &X,
                                     const AxisS &Y, const AxisS &Z, real cx, real cy, real cz) {
    const real third = (real)(1.0 / 3.0), half = (real)0.5;
    const int ox = lx + X.base + 1, oy = ly + Y.base + 1, oz = lz + Z.base + 1;
    // Jx on faces a = 0, 1 (prefix of W_x along x)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            real fyz = Y.S0[b] * Z.S0[c] + half * Y.DS[b] * Z.S0[c] + half * Y.S0[b] * Z.DS[c] +
                       third * Y.DS[b] * Z.DS[c];
            real acc = 0;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                acc -= cx * (X.DS[a] * fyz);
                if (acc != (real)0)
                    atomicAdd(&sJ[0 * JT3 + (ox + a) + JT * ((oy + b) + JT * (oz + c))], acc);
            }
        }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            real fxz = X.S0[a] * Z.S0[c] + half * X.DS[a] * Z.S0[c] + half * X.S0[a] * Z.DS[c] +
                       third * X.DS[a] * Z.DS[c];
            real acc = 0;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                acc -= cy * (Y.DS[b] * fxz);
                if (acc != (real)0)
                    atomicAdd(&sJ[1 * JT3 + (ox + a) + JT * ((oy + b) + JT * (oz + c))], acc);
            }
        }
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            real fxy = X.S0[a] * Y.S0[b] + half * X.DS[a] * Y.S0[b] + half * X.S0[a] * Y.DS[b] +
                       third * X.DS[a] * Y.DS[b];
            real acc = 0;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                acc -= cz * (Z.DS[c] * fxy);
                if (acc != (real)0)
                    atomicAdd(&sJ[2 * JT3 + (ox + a) + JT * ((oy + b) + JT * (oz + c))], acc);
            }
        }
}

__device__ inline real below_one() {
#ifdef HK_DOUBLE
    return 0.99999999999999988898;
#else
    return 0.99999994f;
#endif
}

__global__ void __launch_bounds__(BS)
k_push(GridP g, SpecP sp, PArr in, const int *__restrict__ cnt_in, PArr out,
       int *__restrict__ cnt_out, PArr inbox, int *__restrict__ inbox_n, int inbox_cap,
       const real *__restrict__ Ex, const real *__restrict__ Ey, const real *__restrict__ Ez,
       const real *__restrict__ Bx, const real *__restrict__ By, const real *__restrict__ Bz,
       real *__restrict__ Jx, real *__restrict__ Jy, real *__restrict__ Jz, int *__restrict__ err) {
    __shared__ real sF[6 * FT3];
    __shared__ real sJ[3 * JT3];
    const int t = blockIdx.x;
    const int n = min(cnt_in[t], sp.cap[t]);
    if (n <= 0) return;
    const int tx = t % g.ntx, ty = (t / g.ntx) % g.nty, tz = t / (g.ntx * g.nty);
    const int ox = tx * TILE, oy = ty * TILE, oz = tz * TILE;
    const int per = g.bcx == HK_BC_PERIODIC;

    for (int e = threadIdx.x; e < FT3; e += BS) {
        int a = e % FT, b = (e / FT) % FT, c = e / (FT * FT);
        int gi = ox - 1 + a;
        int gj = wrapi(oy - 1 + b, g.ny), gk = wrapi(oz - 1 + c, g.nz);
        int ih, in_;
        if (per) { ih = in_ = wrapi(gi, g.nx); }
        else {
            ih = gi < 0 ? 0 : (gi > g.nx - 1 ? g.nx - 1 : gi);
            in_ = gi < 0 ? 0 : (gi > g.nx ? g.nx : gi);
        }
        long long ch = gidx(g, ih, gj, gk), cn = gidx(g, in_, gj, gk);
        sF[0 * FT3 + e] = Ex[ch];
        sF[1 * FT3 + e] = Ey[cn];
        sF[2 * FT3 + e] = Ez[cn];
        sF[3 * FT3 + e] = Bx[cn];
        sF[4 * FT3 + e] = By[ch];
        sF[5 * FT3 + e] = Bz[ch];
    }
    for (int e = threadIdx.x; e < 3 * JT3; e += BS) sJ[e] = 0;
    __syncthreads();

    const long long base = sp.off[t];
    const real dv = g.dx * g.dy * g.dz;
    const real hq = (real)0.5 * sp.qm * g.dt;
    const int lane = __lane_id();
    for (int p0 = 0; p0 < n; p0 += BS) {
        const int p = p0 + threadIdx.x;
        int cell = p < n ? in.cell[base + p] : -1;
        bool valid = cell >= 0;
        int ncell = -1, ntile = -1;
        real nrx = 0, nry = 0, nrz = 0, ux = 0, uy = 0, uz = 0, w = 0;
        uint64_t id = 0;
        int zc = 0;
        double tau = 0;
        if (valid) {
            const long long ip = base + p;
            const int ci = cell % g.nx, rr = cell / g.nx;
            const int cj = rr % g.ny, ck = rr / g.ny;
            const int lx = ci - ox, ly = cj - oy, lz = ck - oz;
            if ((unsigned)lx >= TILE || (unsigned)ly >= TILE || (unsigned)lz >= TILE) {
                atomicOr(err, ERR_TILE);
                valid = false;
            }
        }
        if (valid) {
            const long long ip = base + p;
            const int ci = cell % g.nx, rr = cell / g.nx;
            const int cj = rr % g.ny, ck = rr / g.ny;
            const int lx = ci - ox, ly = cj - oy, lz = ck - oz;
            const real rx = in.rx[ip], ry = in.ry[ip], rz = in.rz[ip];
            ux = in.ux[ip]; uy = in.uy[ip]; uz = in.uz[ip];
            w = in.w[ip];
            id = in.id[ip];
            if (sp.has_z) zc = in.zc[ip];
            if (sp.has_tau) tau = in.tau[ip];
            // gather E^n, B^n (CIC on the Yee stagger)
            AxisW X = axis_weights(lx, rx), Y = axis_weights(ly, ry), Z = axis_weights(lz, rz);
            real ex = tri(sF + 0 * FT3, X.ih, Y.in_, Z.in_, X.fh, Y.fn, Z.fn);
            real ey = tri(sF + 1 * FT3, X.in_, Y.ih, Z.in_, X.fn, Y.fh, Z.fn);
            real ez = tri(sF + 2 * FT3, X.in_, Y.in_, Z.ih, X.fn, Y.fn, Z.fh);
            real bx = tri(sF + 3 * FT3, X.in_, Y.ih, Z.ih, X.fn, Y.fh, Z.fh);
            real by = tri(sF + 4 * FT3, X.ih, Y.in_, Z.ih, X.fh, Y.fn, Z.fh);
            real bz = tri(sF + 5 * FT3, X.ih, Y.ih, Z.in_, X.fh, Y.fh, Z.fn);
            // Boris rotation
            real umx = ux + hq * ex, umy = uy + hq * ey, umz = uz + hq * ez;
            real gm = sqrt((real)1 + umx * umx + umy * umy + umz * umz);
            real tx_ = hq * bx / gm, ty_ = hq * by / gm, tz_ = hq * bz / gm;
            real t2 = tx_ * tx_ + ty_ * ty_ + tz_ * tz_;
            real sx = 2 * tx_ / (1 + t2), sy = 2 * ty_ / (1 + t2), sz = 2 * tz_ / (1 + t2);
            real upx = umx + (umy * tz_ - umz * ty_);
            real upy = umy + (umz * tx_ - umx * tz_);
            real upz = umz + (umx * ty_ - umy * tx_);
            real uqx = umx + (upy * sz - upz * sy);
            real uqy = umy + (upz * sx - upx * sz);
            real uqz = umz + (upx * sy - upy * sx);
            ux = uqx + hq * ex; uy = uqy + hq * ey; uz = uqz + hq * ez;
            real gam = sqrt((real)1 + ux * ux + uy * uy + uz * uz);
            real X1 = rx + g.dt * ux / gam / g.dx;
            real Y1 = ry + g.dt * uy / gam / g.dy;
            real Z1 = rz + g.dt * uz / gam / g.dz;
            // specular reflection at the open x walls
            if (!per) {
                if (ci == 0 && X1 < (real)0) { X1 = -X1; ux = -ux; }
                else if (ci == g.nx - 1 && X1 >= (real)1) {
                    X1 = (real)2 - X1; ux = -ux;
                    if (X1 >= (real)1) X1 = below_one();
                }
            }
            if (!(isfinite(ux) && isfinite(uy) && isfinite(uz) && fabs(X1 - rx) < 1 &&
                  fabs(Y1 - ry) < 1 && fabs(Z1 - rz) < 1)) {
                atomicOr(err, isfinite(ux + uy + uz) ? ERR_CFL : ERR_NONFINITE);
                valid = false;
            } else {
                // Esirkepov deposit of J^{n+1/2}
                if (sp.q != (real)0) {
                    AxisS SX = axis_shapes(rx, X1), SY = axis_shapes(ry, Y1), SZ = axis_shapes(rz, Z1);
                    real qw = sp.q * w / dv;
                    esirkepov_lds(sJ, lx, ly, lz, SX, SY, SZ, qw * g.dx / g.dt, qw * g.dy / g.dt,
                                  qw * g.dz / g.dt);
                }
                // new cell and offsets
                int fx = X1 >= (real)1 ? 1 : (X1 < (real)0 ? -1 : 0);
                int fy = Y1 >= (real)1 ? 1 : (Y1 < (real)0 ? -1 : 0);
                int fz = Z1 >= (real)1 ? 1 : (Z1 < (real)0 ? -1 : 0);
                nrx = X1 - (real)fx; nry = Y1 - (real)fy; nrz = Z1 - (real)fz;
                if (nrx >= (real)1) nrx = below_one();
                if (nry >= (real)1) nry = below_one();
                if (nrz >= (real)1) nrz = below_one();
                int ni = ci + fx, nj = cj + fy, nk = ck + fz;
                if (per) ni = wrapi(ni, g.nx);
                nj = nj < 0 ? nj + g.ny : (nj >= g.ny ? nj - g.ny : nj);
                nk = nk < 0 ? nk + g.nz : (nk >= g.nz ? nk - g.nz : nk);
                ncell = ni + g.nx * (nj + g.ny * nk);
                ntile = (ni >> TLOG) + g.ntx * ((nj >> TLOG) + g.nty * (nk >> TLOG));
            }
        }
        // slot reservation: one global atomic per wave and destination tile
        // (lanes sharing a destination are ranked with ballot / popcount)
        const bool stay = valid && ntile == t;
        const uint64_t lt = (1ull << lane) - 1ull;
        const uint64_t m = __ballot(stay);
        int wbase = 0;
        if (lane == 0 && m) wbase = atomicAdd(&cnt_out[t], __popcll(m));
        wbase = __shfl(wbase, 0);
        int slot = stay ? wbase + __popcll(m & lt) : 0;
        uint64_t mv = __ballot(valid && !stay);
        while (mv) {
            const int leader = __ffsll((long long)mv) - 1;
            const int dest = __shfl(ntile, leader);
            const uint64_t grp = __ballot(valid && !stay && ntile == dest);
            int b = 0;
            if (lane == leader) b = atomicAdd(&cnt_out[dest], __popcll(grp));
            b = __shfl(b, leader);
            if ((grp >> lane) & 1ull) slot = b + __popcll(grp & lt);
            mv &= ~grp;
        }
        if (valid) {
            PArr dst = out;
            long long j;
            if (slot < sp.cap[ntile]) j = sp.off[ntile] + slot;
            else {
                int k = atomicAdd(inbox_n, 1);
                if (k >= inbox_cap) { atomicOr(err, ERR_INBOX); continue; }
                dst = inbox;
                j = k;
            }
            dst.cell[j] = ncell;
            dst.rx[j] = nrx; dst.ry[j] = nry; dst.rz[j] = nrz;
            dst.ux[j] = ux; dst.uy[j] = uy; dst.uz[j] = uz;
            dst.w[j] = w;
            dst.id[j] = id;
            if (sp.has_z) dst.zc[j] = zc;
            if (sp.has_tau) dst.tau[j] = tau;
        }
    }
    __syncthreads();
    // flush the LDS current tile (nodes ox-1 .. ox+TILE+1) to HBM
    for (int e = threadIdx.x; e < JT3; e += BS) {
        int a = e % JT, b = (e / JT) % JT, c = e / (JT * JT);
        int gi = ox - 1 + a;
        int gj = wrapi(oy - 1 + b, g.ny), gk = wrapi(oz - 1 + c, g.nz);
        bool okx, okn;
        if (per) { gi = wrapi(gi, g.nx); okx = okn = true; }
        else { okx = gi >= 0 && gi <= g.nx - 1; okn = gi >= 0 && gi <= g.nx; }
        long long c0 = gidx(g, gi < 0 ? 0 : gi, gj, gk);
        real vx = sJ[e], vy = sJ[JT3 + e], vz = sJ[2 * JT3 + e];
        if (okx && vx != (real)0) atomicAdd(&Jx[c0], vx);
        if (okn && vy != (real)0) atomicAdd(&Jy[c0], vy);
        if (okn && vz != (real)0) atomicAdd(&Jz[c0], vz);
    }
}

// --------------------------------------------------- immobile-ion ionization ---------------
// ADK tunnelling blended with the multiphoton continuation by a sigmoid in the
// Keldysh parameter; rates in FP64 (atomic units).
__device__ inline double adk(const IonLevel &L, double F) {
    return L.c2 * L.ip_au * pow(2.0 * L.k3 / F, L.expo) * exp(-2.0 * L.k3 / (3.0 * F));
}
__device__ inline double blended_rate(const IonLevel &L, double F, double omega) {
    if (F <= 0.0) return 0.0;
    double gk = omega * sqrt(2.0 * L.ip_au) / F;
    double sig = 1.0 / (1.0 + exp(-(gk - 1.5) / 0.1));
    double wm = L.wfc * pow(fmin(F, L.fc) / L.fc, L.K2);
    return sig * wm + (1.0 - sig) * adk(L, F);
}

__global__ void __launch_bounds__(BS)
k_ionize_static(GridP g, SpecP sp, PArr a, const int *__restrict__ cnt, const real *__restrict__ Ex,
                const real *__restrict__ Ey, const real *__restrict__ Ez,
                const uint8_t *__restrict__ sw, int hybrid, const IonP *__restrict__ ion,
                PArr eout, int *__restrict__ eout_n, int eout_cap, uint64_t seed, int step,
                double *__restrict__ ledger, int *__restrict__ err) {
    __shared__ real sF[3 * FT3];
    const int t = blockIdx.x;
    const int n = min(cnt[t], sp.cap[t]);
    if (n <= 0) return;
    const int tx = t % g.ntx, ty = (t / g.ntx) % g.nty, tz = t / (g.ntx * g.nty);
    const int ox = tx * TILE, oy = ty * TILE, oz = tz * TILE;
    const int per = g.bcx == HK_BC_PERIODIC;
    for (int e = threadIdx.x; e < FT3; e += BS) {
        int aa = e % FT, b = (e / FT) % FT, c = e / (FT * FT);
        int gi = ox - 1 + aa;
        int gj = wrapi(oy - 1 + b, g.ny), gk = wrapi(oz - 1 + c, g.nz);
        int ih, in_;
        if (per) { ih = in_ = wrapi(gi, g.nx); }
        else {
            ih = gi < 0 ? 0 : (gi > g.nx - 1 ? g.nx - 1 : gi);
            in_ = gi < 0 ? 0 : (gi > g.nx ? g.nx : gi);
        }
        sF[0 * FT3 + e] = Ex[gidx(g, ih, gj, gk)];
        sF[1 * FT3 + e] = Ey[gidx(g, in_, gj, gk)];
        sF[2 * FT3 + e] = Ez[gidx(g, in_, gj, gk)];
    }
    __syncthreads();
    const long long base = sp.off[t];
    const double omega = ion->omega_au;
    for (int p = threadIdx.x; p < n; p += BS) {
        const long long ip = base + p;
        int cell = a.cell[ip];
        if (cell < 0) continue;
        int zc = a.zc[ip];
        if (zc >= ion->z_max) continue;
        const int ci = cell % g.nx, rr = cell / g.nx;
        const int cj = rr % g.ny, ck = rr / g.ny;
        const real rx = a.rx[ip], ry = a.ry[ip], rz = a.rz[ip];
        if (hybrid) {
            int ni = ci + (rx >= (real)0.5), nj = cj + (ry >= (real)0.5), nk = ck + (rz >= (real)0.5);
            if (per) ni = wrapi(ni, g.nx);
            if (nj >= g.ny) nj -= g.ny;
            if (nk >= g.nz) nk -= g.nz;
            if (!sw[gidx(g, ni, nj, nk)]) continue;
        }
        const int lx = ci - ox, ly = cj - oy, lz = ck - oz;
        if ((unsigned)lx >= TILE || (unsigned)ly >= TILE || (unsigned)lz >= TILE) {
            atomicOr(err, ERR_TILE);
            continue;
        }
        AxisW X = axis_weights(lx, rx), Y = axis_weights(ly, ry), Z = axis_weights(lz, rz);
        double ex = tri(sF + 0 * FT3, X.ih, Y.in_, Z.in_, X.fh, Y.fn, Z.fn);
        double ey = tri(sF + 1 * FT3, X.in_, Y.ih, Z.in_, X.fn, Y.fh, Z.fn);
        double ez = tri(sF + 2 * FT3, X.in_, Y.in_, Z.ih, X.fn, Y.fn, Z.fh);
        double F = sqrt(ex * ex + ey * ey + ez * ez) * ion->field_au;
        const uint64_t pid = a.id[ip];
        int z0 = zc;
        for (int lev = zc; lev < ion->z_max; ++lev) {
            double wr = blended_rate(ion->lev[lev], F, omega) * ion->rate_norm;
            double P = -expm1(-wr * g.ddt);
            uint32_t r[4];
            draw4(seed, pid, (uint32_t)step, TAG_ION + (uint32_t)lev, 0, r);
            if (!(u01d(r[0]) < P)) break;
            zc = lev + 1;
            int k = atomicAdd(eout_n, 1);
            if (k >= eout_cap) { atomicOr(err, ERR_INBOX); break; }
            eout.cell[k] = cell;
            eout.rx[k] = rx; eout.ry[k] = ry; eout.rz[k] = rz;
            eout.ux[k] = a.ux[ip]; eout.uy[k] = a.uy[ip]; eout.uz[k] = a.uz[ip];
            eout.w[k] = a.w[ip];
            eout.id[k] = (1ull << 62) | ((uint64_t)lev << 56) | pid;
            atomicAdd(ledger, (double)a.w[ip] * ion->lev[lev].ip_au * 27.211386245988 / 510998.95);
        }
        if (zc != z0) a.zc[ip] = zc;
    }
}

// ----------------------------------------------------------- charge density ---------------
__global__ void __launch_bounds__(BS)
k_rho(GridP g, SpecP sp, PArr a, const int *__restrict__ cnt, double *__restrict__ rho) {
    const int t = blockIdx.x;
    const int n = min(cnt[t], sp.cap[t]);
    const long long base = sp.off[t];
    const double dv = g.ddx * g.ddy * g.ddz;
    const int per = g.bcx == HK_BC_PERIODIC;
    for (int p = threadIdx.x; p < n; p += BS) {
        const long long ip = base + p;
        int cell = a.cell[ip];
        if (cell < 0) continue;
        const int ci = cell % g.nx, rr = cell / g.nx;
        const int cj = rr % g.ny, ck = rr / g.ny;
        double fx = a.rx[ip], fy = a.ry[ip], fz = a.rz[ip];
        double q = sp.has_z ? (double)a.zc[ip] : (double)sp.q;
        double qw = q * (double)a.w[ip] / dv;
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int aa = 0; aa < 2; ++aa) {
                    int i = per ? wrapi(ci + aa, g.nx) : ci + aa;
                    int j = wrapi(cj + b, g.ny), k = wrapi(ck + c, g.nz);
                    double wgt = (aa ? fx : 1 - fx) * (b ? fy : 1 - fy) * (c ? fz : 1 - fz);
                    atomicAdd(&rho[gidx(g, i, j, k)], qw * wgt);
                }
    }
}

inline unsigned blocks(long long n) { return (unsigned)((n + BS - 1) / BS); }

}  // namespace

void launch_init_species_cols(const GridP &g, const hk_species_desc &d, uint64_t seed, PArr out,
                              const int *xcol, const double *wcol, int ncol, int has_z,
                              int has_tau, hipStream_t s) {
    long long total = (long long)ncol * g.ny * g.nz * d.ppc;
    if (total == 0) return;
    k_init<<<blocks(total), BS, 0, s>>>(g, d.ppc, d.u_th, d.charge, seed, xcol, wcol, ncol, total,
                                        out, has_z, has_tau);
}

void launch_count_groups(const GridP &g, PArr src, const long long *off, const int *cnt,
                         const int *cap, int ngroups, int *newcnt, hipStream_t s) {
    if (ngroups == 0) return;
    k_count<<<ngroups, BS, 0, s>>>(g, src, off, cnt, cap, newcnt);
}

void launch_scatter_groups(const GridP &g, PArr src, const long long *off, const int *cnt,
                           const int *cap, int ngroups, PArr dst, const long long *doff,
                           int *dfill, int has_z, int has_tau, hipStream_t s) {
    if (ngroups == 0) return;
    k_scatter<<<ngroups, BS, 0, s>>>(g, src, off, cnt, cap, dst, doff, dfill, has_z, has_tau);
}

void launch_merge_inbox(const GridP &g, const SpecP &sp, PArr inbox, const int *inbox_n,
                        long long max_n, PArr dst, int *cnt, int *fail_n, PArr fail,
                        hipStream_t s) {
    if (max_n == 0) return;
    unsigned nb = blocks(max_n);
    k_merge<<<nb < 1024u ? nb : 1024u, BS, 0, s>>>(g, sp, inbox, inbox_n, dst, cnt, fail_n, fail);
}

void launch_push_tiles(const GridP &g, const SpecP &sp, PArr in, const int *cnt_in, PArr out,
                       int *cnt_out, PArr inbox, int *inbox_n, int inbox_cap, real *const f[9],
                       int *err, hipStream_t s) {
    k_push<<<g.ntiles, BS, 0, s>>>(g, sp, in, cnt_in, out, cnt_out, inbox, inbox_n, inbox_cap,
                                   f[HK_EX], f[HK_EY], f[HK_EZ], f[HK_BX], f[HK_BY], f[HK_BZ],
                                   f[HK_JX], f[HK_JY], f[HK_JZ], err);
}

void launch_ionize_static(const GridP &g, const SpecP &sp, PArr a, const int *cnt,
                          real *const f[9], const uint8_t *sw, int hybrid, const IonP *ion,
                          PArr eout, int *eout_n, int eout_cap, uint64_t seed, int step,
                          double *ledger, int *err, hipStream_t s) {
    k_ionize_static<<<g.ntiles, BS, 0, s>>>(g, sp, a, cnt, f[HK_EX], f[HK_EY], f[HK_EZ], sw,
                                            hybrid, ion, eout, eout_n, eout_cap, seed, step,
                                            ledger, err);
}

void launch_rho_tiles(const GridP &g, const SpecP &sp, PArr a, const int *cnt, double *rho,
                      hipStream_t s) {
    k_rho<<<g.ntiles, BS, 0, s>>>(g, sp, a, cnt, rho);
}
