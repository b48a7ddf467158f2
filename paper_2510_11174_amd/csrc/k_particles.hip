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
// atomics and flushes that tile to HBM with one global atomic per sample.
// Particles that stay in the tile are written to the front of the tile's bin
// in the next buffer, ranked by an LDS counter, so the hot loop issues no
// global atomic with a return value (those cost a round trip to the memory
// side on a multi-die GPU).  Particles that leave go to the tile's mover
// region, also ranked in LDS; a migrate kernel then appends them to the back
// of their destination bins.  Every particle byte is read once and written
// once per step, movers twice.
#include "hk_internal.h"
#include "hk_pic_device.h"

namespace {

using namespace hkdev;
constexpr int BS = 256;

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
// Particle q of cell c: position index c * ppc + q, id (species << 52) |
// (c * ppc + q), unique over the species; offsets from Philox tag 1 keyed by
// the position index (the species of a cell start at the same points),
// momenta by Box-Muller from tag 2 keyed by the id (FP64, rounded once to
// the storage type).  Storage order: q slowest, so that consecutive particles
// (the lanes of a wave in the push, after binning) sit in distinct cells and
// their LDS current atomics go to distinct addresses.
__global__ void __launch_bounds__(BS)
k_init(GridP g, int ppc, int isp, double u_th, double charge, uint64_t seed, const int *__restrict__ xcol,
       const double *__restrict__ wcol, int ncol, long long total, PArr out, int has_z,
       int has_tau) {
    long long tid = (long long)blockIdx.x * BS + threadIdx.x;
    if (tid >= total) return;
    const long long cells = total / ppc;
    int q = (int)(tid / cells);
    long long r = tid - (long long)q * cells;
    int col = (int)(r % ncol);
    long long jk = r / ncol;
    int j = (int)(jk % g.ny), k = (int)(jk / g.ny);
    int i = xcol[col];
    int cell = i + g.nx * (j + g.ny * k);
    const uint64_t pos = (uint64_t)cell * (uint64_t)ppc + (uint64_t)q;
    const uint64_t id = ((uint64_t)isp << 52) | pos;
    uint32_t rp[4], rm[4];
    draw4(seed, pos, 0, TAG_POS, 0, rp);
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
    if (has_tau) out.tau[tid] = tau0(seed, id);
}

// --------------------------------------------------------- wave helpers ------------------
// Reserve `add` slots per active lane in ctr[key]: lanes of a wave that share a
// key are ranked by ballot and served by one atomic (up to four distinct keys
// per wave); the rest fall back to one atomic per lane.  Every lane calls it.
__device__ inline int wave_reserve(int *ctr, int key, bool active) {
    const int lane = __lane_id();
    const uint64_t lt = (1ull << lane) - 1ull;
    uint64_t pending = __ballot(active);
    int slot = 0;
    for (int it = 0; it < 4 && pending; ++it) {
        const int leader = __ffsll((long long)pending) - 1;
        const int k = __shfl(key, leader);
        const uint64_t grp = __ballot(active && key == k) & pending;
        int base = 0;
        if (lane == leader) base = atomicAdd(&ctr[k], __popcll(grp));
        base = __shfl(base, leader);
        if ((grp >> lane) & 1ull) slot = base + __popcll(grp & lt);
        pending &= ~grp;
    }
    if ((pending >> lane) & 1ull) slot = atomicAdd(&ctr[key], 1);
    return slot;
}

// --------------------------------------------------------- count / scatter ---------------
// Source groups: group s holds slots [off[s], off[s] + nf[s]) and
// [off[s] + cap[s] - nb[s], off[s] + cap[s]) (nb may be null: front only).
__device__ inline int group_count(const long long *off, const int *nf, const int *nb,
                                  const int *cap, int s, int &f, int &b) {
    const int c = cap[s];
    f = min(nf[s], c);
    b = nb ? min(nb[s], c - f) : 0;
    return f + b;
}

__global__ void __launch_bounds__(BS)
k_count(GridP g, PArr src, const long long *__restrict__ off, const int *__restrict__ nf,
        const int *__restrict__ nb, const int *__restrict__ cap, int *__restrict__ newcnt) {
    const int s = blockIdx.x;
    int f, b;
    const int n = group_count(off, nf, nb, cap, s, f, b);
    const int c = cap[s];
    const int stride = gridDim.y * BS;
    for (int p0 = blockIdx.y * BS; p0 < n; p0 += stride) {
        const int p = p0 + threadIdx.x;
        int cell = -1;
        if (p < n) cell = src.cell[off[s] + (p < f ? p : c - b + (p - f))];
        const bool ok = cell >= 0;
        wave_reserve(newcnt, ok ? tile_of(g, cell) : 0, ok);
    }
}

__global__ void __launch_bounds__(BS)
k_scatter(GridP g, PArr src, const long long *__restrict__ off, const int *__restrict__ nf,
          const int *__restrict__ nb, const int *__restrict__ cap, PArr dst,
          const long long *__restrict__ doff, int *__restrict__ dfill, int has_z, int has_tau) {
    const int s = blockIdx.x;
    int f, b;
    const int n = group_count(off, nf, nb, cap, s, f, b);
    const int c = cap[s];
    const int stride = gridDim.y * BS;
    for (int p0 = blockIdx.y * BS; p0 < n; p0 += stride) {
        const int p = p0 + threadIdx.x;
        long long i = 0;
        int cell = -1;
        if (p < n) {
            i = off[s] + (p < f ? p : c - b + (p - f));
            cell = src.cell[i];
        }
        const bool ok = cell >= 0;
        const int t = ok ? tile_of(g, cell) : 0;
        const int slot = wave_reserve(dfill, t, ok);
        if (ok) copy_particle(src, i, dst, doff[t] + slot, has_z, has_tau);
    }
}

// Append a list of particles to the back of their bins; those that do not
// fit go to `fail` (and force a re-bin).  Grid-stride over the list.
__global__ void __launch_bounds__(BS)
k_merge(GridP g, SpecP sp, PArr inbox, const int *__restrict__ inbox_n, int inbox_cap, PArr dst,
        const int *__restrict__ nf, int *__restrict__ nb, int *__restrict__ fail_n, PArr fail,
        int fail_cap, int *__restrict__ err) {
    const int n = min(*inbox_n, inbox_cap);
    for (int p0 = blockIdx.x * BS; p0 < n; p0 += gridDim.x * BS) {
        const int i = p0 + threadIdx.x;
        const int cell = i < n ? inbox.cell[i] : -1;
        const bool ok = cell >= 0;
        const int t = ok ? tile_of(g, cell) : 0;
        const int slot = wave_reserve(nb, t, ok);
        if (!ok) continue;
        if (nf[t] + slot < sp.cap[t]) {
            copy_particle(inbox, i, dst, sp.off[t] + sp.cap[t] - 1 - slot, sp.has_z, sp.has_tau);
        } else {
            int k = atomicAdd(fail_n, 1);
            if (k < fail_cap) copy_particle(inbox, i, fail, k, sp.has_z, sp.has_tau);
            else atomicOr(err, ERR_INBOX);
        }
    }
}

// Movers of tile t (its region of the mover buffer) join the back of their
// destination bins in the next buffer.
constexpr int MIGRATE_PARTS = 4;
__global__ void __launch_bounds__(BS)
k_migrate(GridP g, SpecP sp, PArr mig, const long long *__restrict__ moff,
          const int *__restrict__ mcnt, const int *__restrict__ mcap, PArr dst, const int *__restrict__ nf,
          int *__restrict__ nb, int *__restrict__ fail_n, PArr fail, int fail_cap, int *__restrict__ err,
          int nitems) {
    // (tile, part) items spread over the XCDs by slabs of tiles
    __shared__ int s_cnt[27], s_base[27];
    const int k = xcd_item(blockIdx.x, gridDim.x);
    if (k >= nitems) return;
    const int t = k / MIGRATE_PARTS, y = k % MIGRATE_PARTS;
    // movers beyond the region went to the inbox; the parts share the rest
    const int n = min(mcnt[t], mcap[t]);
    const int per = ((n + MIGRATE_PARTS - 1) / MIGRATE_PARTS + BS - 1) / BS * BS;
    const int beg = y * per, end = min(n, beg + per);
    const long long b0 = moff[t];
    const int tx = t % g.ntx, ty = (t / g.ntx) % g.nty, tz = t / (g.ntx * g.nty);
    const int per_x = g.bcx == HK_BC_PERIODIC;
    for (int p0 = beg; p0 < end; p0 += BS) {
        if (threadIdx.x < 27) s_cnt[threadIdx.x] = 0;
        __syncthreads();
        // the whole particle at once, then one global atomic per destination
        // tile and workgroup (ranks from LDS counters by direction)
        const int p = p0 + threadIdx.x;
        const long long i = b0 + p;
        int cell = -1, zc = 0;
        real rx = 0, ry = 0, rz = 0, ux = 0, uy = 0, uz = 0, w = 0;
        uint64_t id = 0;
        double tau = 0.0;
        if (p < end) {
            cell = mig.cell[i];
            rx = mig.rx[i]; ry = mig.ry[i]; rz = mig.rz[i];
            ux = mig.ux[i]; uy = mig.uy[i]; uz = mig.uz[i];
            w = mig.w[i]; id = mig.id[i];
            if (sp.has_z) zc = mig.zc[i];
            if (sp.has_tau) tau = mig.tau[i];
        }
        const bool ok = cell >= 0;
        int d = 0, dir = -1, rank = 0;
        if (ok) {
            int ci, cj, ck;
            cell_ijk(g, cell, ci, cj, ck);
            const int dtx_ = ci >> TLOG, dty_ = cj >> TLOG, dtz_ = ck >> TLOG;
            d = dtx_ + g.ntx * (dty_ + g.nty * dtz_);
            int ex = dtx_ - tx, ey = dty_ - ty, ez = dtz_ - tz;
            if (ex > 1) ex -= g.ntx; else if (ex < -1) ex += g.ntx;
            if (ey > 1) ey -= g.nty; else if (ey < -1) ey += g.nty;
            if (ez > 1) ez -= g.ntz; else if (ez < -1) ez += g.ntz;
            if (ex >= -1 && ex <= 1 && ey >= -1 && ey <= 1 && ez >= -1 && ez <= 1) {
                dir = (ex + 1) + 3 * ((ey + 1) + 3 * (ez + 1));
                rank = atomicAdd(&s_cnt[dir], 1);
            }
        }
        __syncthreads();
        if (threadIdx.x < 27 && s_cnt[threadIdx.x] > 0) {
            const int q = threadIdx.x;
            int nx_ = tx + q % 3 - 1;
            if (per_x) nx_ = wrapi(nx_, g.ntx);
            const int ny_ = wrapi(ty + (q / 3) % 3 - 1, g.nty), nz_ = wrapi(tz + q / 9 - 1, g.ntz);
            s_base[q] = atomicAdd(&nb[nx_ + g.ntx * (ny_ + g.nty * nz_)], s_cnt[q]);
        }
        __syncthreads();
        if (!ok) continue;
        // a destination beyond the neighbouring tiles (not reachable in one
        // step) takes a slot of its own
        const int slot = dir >= 0 ? s_base[dir] + rank : atomicAdd(&nb[d], 1);
        PArr to = dst;
        long long j;
        if (nf[d] + slot < sp.cap[d]) j = sp.off[d] + sp.cap[d] - 1 - slot;
        else {
            const int k = atomicAdd(fail_n, 1);
            if (k >= fail_cap) { atomicOr(err, ERR_INBOX); continue; }
            to = fail; j = k;
        }
        to.cell[j] = cell;
        to.rx[j] = rx; to.ry[j] = ry; to.rz[j] = rz;
        to.ux[j] = ux; to.uy[j] = uy; to.uz[j] = uz;
        to.w[j] = w; to.id[j] = id;
        if (sp.has_z) to.zc[j] = zc;
        if (sp.has_tau) to.tau[j] = tau;
    }
}

// ------------------------------------------------------------- the push -----------------
constexpr int PBS = 512;   // push workgroup: 8 waves share one tile
constexpr int PUSH_CHUNK = 16 * PBS; // tiles up to this many particles take one workgroup

// ------------------------------------------------------ work plan of tile kernels -----
constexpr int PLAN_BS = 1024;

// Two passes over the tiles, PLAN_PARTS workgroups each, every workgroup on
// the same contiguous range of tiles in both.  The items are sorted by
// decreasing chunk size through 32 power-of-two buckets: pass 1 counts each
// workgroup's items per bucket into ctl[4 + 32 w + b]; pass 2 places them,
// bucket b starting after every larger bucket's items and after the items
// of bucket b of the earlier workgroups.  ctl[0] = number of items; live
// (optional) receives it too: zero exactly when the bins are empty.
__device__ inline void plan_range(int ntiles, int &t0, int &t1) {
    const int per = (ntiles + (int)gridDim.x - 1) / (int)gridDim.x;
    t0 = min(ntiles, (int)blockIdx.x * per);
    t1 = min(ntiles, t0 + per);
}

__global__ void __launch_bounds__(PLAN_BS)
k_plan_count(int ntiles, SpecP sp, Bins bins, int cmin, int *__restrict__ ctl, int *__restrict__ zero3) {
    __shared__ int cnt[32];
    if (threadIdx.x < 32) cnt[threadIdx.x] = 0;
    // the push's output counters (3 ntiles ints), cleared here to save a launch
    if (zero3)
        for (int t = blockIdx.x * PLAN_BS + threadIdx.x; t < 3 * ntiles; t += gridDim.x * PLAN_BS) zero3[t] = 0;
    __syncthreads();
    int t0, t1;
    plan_range(ntiles, t0, t1);
    for (int t = t0 + (int)threadIdx.x; t < t1; t += PLAN_BS) {
        int nfi, nbi;
        const int n = bin_count(sp, bins, t, nfi, nbi);
        if (n > 0) {
            const int c = tile_chunk(n, cmin);
            atomicAdd(&cnt[31 - __clz(min(n, c))], (n + c - 1) / c);
        }
    }
    __syncthreads();
    if (threadIdx.x < 32) ctl[4 + 32 * blockIdx.x + threadIdx.x] = cnt[threadIdx.x];
}

__global__ void __launch_bounds__(PLAN_BS)
k_plan_place(int ntiles, SpecP sp, Bins bins, int cmin, int2 *__restrict__ items, int *__restrict__ ctl,
             int *__restrict__ live) {
    __shared__ int tot[32], cur[32];
    if (threadIdx.x < 32) {
        const int b = threadIdx.x;
        int all = 0, before = 0;
        for (int w = 0; w < (int)gridDim.x; ++w) {
            const int v = ctl[4 + 32 * w + b];
            all += v;
            if (w < (int)blockIdx.x) before += v;
        }
        tot[b] = all;
        cur[b] = before;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int total = 0;
        for (int b = 31; b >= 0; --b) { cur[b] += total; total += tot[b]; }
        if (blockIdx.x == 0) {
            ctl[0] = total;
            if (live) *live = total;
        }
    }
    __syncthreads();
    int t0, t1;
    plan_range(ntiles, t0, t1);
    for (int t = t0 + (int)threadIdx.x; t < t1; t += PLAN_BS) {
        int nfi, nbi;
        const int n = bin_count(sp, bins, t, nfi, nbi);
        if (n > 0) {
            const int c = tile_chunk(n, cmin), k = (n + c - 1) / c;
            const int at = atomicAdd(&cur[31 - __clz(min(n, c))], k);
            for (int j = 0; j < k; ++j) items[at + j] = make_int2(t, j);
        }
    }
}

void plan_tiles(const GridP &g, const SpecP &sp, Bins b, int cmin, int2 *items, int *ctl, int *zero3,
                int *live, hipStream_t s) {
    k_plan_count<<<PLAN_PARTS, PLAN_BS, 0, s>>>(g.ntiles, sp, b, cmin, ctl, zero3);
    k_plan_place<<<PLAN_PARTS, PLAN_BS, 0, s>>>(g.ntiles, sp, b, cmin, items, ctl, live);
}

// One particle's state as the push reads it.  Every field is loaded at once
// (no load waits on another) and one loop iteration ahead of its use.
struct PLoad {
    int cell;
    real rx, ry, rz, ux, uy, uz, w;
    uint64_t id;
    int zc;
    double tau;
};
__device__ inline PLoad pload(const PArr &in, const SpecP &sp, long long ip, bool ok) {
    PLoad L;
    L.cell = -1;
    L.rx = L.ry = L.rz = L.ux = L.uy = L.uz = L.w = 0;
    L.id = 0; L.zc = 0; L.tau = 0.0;
    if (ok) {
        L.cell = in.cell[ip];
        L.rx = in.rx[ip]; L.ry = in.ry[ip]; L.rz = in.rz[ip];
        L.ux = in.ux[ip]; L.uy = in.uy[ip]; L.uz = in.uz[ip];
        L.w = in.w[ip];
        L.id = in.id[ip];
        if (sp.has_z) L.zc = in.zc[ip];
        if (sp.has_tau) L.tau = in.tau[ip];
    }
    return L;
}

// MODE 0: charged particles; MODE 1: QED leptons (photon emission from the
// fields at x^n and u^{n-1/2}, before the Boris push); MODE 2: photons
// (Breit-Wheeler pair creation, then a ballistic move at c; no current).
// At most 128 VGPRs, four waves per SIMD: the LDS tiles already allow two
// workgroups of eight waves per CU, and the QED variant would otherwise take
// 141 registers and three waves per SIMD.
template <int MODE>
__global__ void __launch_bounds__(PBS) __attribute__((amdgpu_waves_per_eu(4)))
k_push(GridP g, SpecP sp, PArr in, Bins bin_in, long long dout, int *__restrict__ nf_out, long long mig0,
       const long long *__restrict__ moff, const int *__restrict__ mcap, int *__restrict__ mcnt,
       const PArr *__restrict__ inbox_p, int *__restrict__ inbox_n, int inbox_cap, const real *__restrict__ Ex,
       const real *__restrict__ Ey, const real *__restrict__ Ez, const real *__restrict__ Bx,
       const real *__restrict__ By, const real *__restrict__ Bz, jglob_t *__restrict__ Jx,
       jglob_t *__restrict__ Jy, jglob_t *__restrict__ Jz, int *__restrict__ err,
       unsigned long long *__restrict__ stats, const unsigned *__restrict__ wmax_bits,
       unsigned *__restrict__ umax2, const int2 *__restrict__ items, const int *__restrict__ ctl, QedP Q,
       AbsorbP A) {
    __shared__ real sF[6 * FT3];
    __shared__ jacc_t sJ[3 * JT3];
    __shared__ uint8_t sSw[JT3];   // switch map of nodes -1 .. TILE+1 (absorbing species)
    __shared__ int s_stay, s_move;
    __shared__ unsigned s_u2;
    const int2 it = plan_item(items, ctl, blockIdx.x);
    const int t = it.x, item = it.y;
    if (t < 0) return;
    int nfi, nbi;
    const int n = bin_count(sp, bin_in, t, nfi, nbi);
    // a dense tile's items go to several workgroups: they take the stayer and
    // mover ranks from the tile's global counters, a tile of one item from LDS
    const int chunk = tile_chunk(n, PUSH_CHUNK);
    const int pbeg = item * chunk, pend = min(n, pbeg + chunk);
    if (pbeg >= pend) return;
    const bool shared = n > chunk;
    const int tx = t % g.ntx, ty = (t / g.ntx) % g.nty, tz = t / (g.ntx * g.nty);
    const int ox = tx * TILE, oy = ty * TILE, oz = tz * TILE;
    const int per = g.bcx == HK_BC_PERIODIC;

    for (int e = threadIdx.x; e < FT3; e += PBS) {
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
    if (MODE != 2)
        for (int e = threadIdx.x; e < 3 * JT3; e += PBS) sJ[e] = 0;
    if (MODE != 2 && A.on)
        for (int e = threadIdx.x; e < JT3; e += PBS) {
            const int a = e % JT, b = (e / JT) % JT, c = e / (JT * JT);
            int gi = ox - 1 + a;
            const int gj = wrapi(oy - 1 + b, g.ny), gk = wrapi(oz - 1 + c, g.nz);
            if (per) gi = wrapi(gi, g.nx);
            // no node beyond an open wall: kinetic (nothing is absorbed there)
            sSw[e] = (!per && (gi < 0 || gi > g.nx)) ? 1 : A.sw[gidx(g, gi, gj, gk)];
        }
    if (threadIdx.x == 0) { s_stay = 0; s_move = 0; s_u2 = 0; }
    __syncthreads();

    const real dv = g.dx * g.dy * g.dz;
    const real hq = (real)0.5 * sp.qm * g.dt;
    float u2max = 0.f;   // largest |u|^2 pushed by this thread
    int pushed = 0;      // particles this wave ranked (shared tiles)
    double led = 0.0;    // photon ledger contributions of this thread
    double aled = 0.0;   // conversion ledger contributions (cold fluid absorption)
    const int lane = __lane_id();
    const uint64_t lt = (1ull << lane) - 1ull;
    const long long obase = sp.off[t];
    const long long mbase = moff[t];
    const int mlim = mcap[t];
    const real cdx = g.dx / g.dt, cdy = g.dy / g.dt, cdz = g.dz / g.dt;
    const real dtdx = g.dt / g.dx, dtdy = g.dt / g.dy, dtdz = g.dt / g.dz;
    // fixed-point scale: one particle's largest current contribution is
    // |q| w / dV * max(dx,dy,dz) / dt, with w bounded by the species' weight
    // bound (never lowered; raised by every kernel that creates particles)
    const double jmax = (double)fabsf((float)sp.q) * (double)__uint_as_float(*wmax_bits) / (double)dv *
                        (double)fmaxf(fmaxf((float)cdx, (float)cdy), (float)cdz);
#ifdef HK_DOUBLE
    const double jscale = 1.0;   // FP64 sums, no scale
    const int jshift = 0;
#else
    const int jexp = jdep_exp(jmax);
    const double jscale = ldexp(1.0, jexp);   // deposit unit of this species
    const int jshift = jexp + JG_BITS;        // tile sum -> global unit
#endif
    const real qsc = (real)((double)sp.q / (double)dv / jscale);   // q / dV in units
    PLoad nx_ = pload(in, sp, bin_slot(sp, t, min(pbeg + (int)threadIdx.x, pend - 1), nfi, nbi),
                      pbeg + (int)threadIdx.x < pend);
    for (int p0 = pbeg; p0 < pend; p0 += PBS) {
        const PLoad cur = nx_;
        if (p0 + PBS < pend) {
            const int pn = p0 + PBS + threadIdx.x;
            nx_ = pload(in, sp, bin_slot(sp, t, min(pn, pend - 1), nfi, nbi), pn < pend);
        }
        const int cell = cur.cell;
        bool valid = cell >= 0;
        int ncell = -1, ntile = -1;
        const real rx = cur.rx, ry = cur.ry, rz = cur.rz;
        real nrx = 0, nry = 0, nrz = 0, ux = cur.ux, uy = cur.uy, uz = cur.uz;
        const real w = cur.w;
        const uint64_t id = cur.id;
        const int zc = cur.zc;
        double tau = cur.tau;
        // QED event products: a photon (MODE 1) or a pair (MODE 2)
        bool want1 = false, want2 = false;
        double kx = 0, ky = 0, kz = 0, m1 = 0, m2 = 0;
        int ci = 0, cj = 0, ck = 0, lx = 0, ly = 0, lz = 0;
        if (valid) {
            cell_ijk(g, cell, ci, cj, ck);
            lx = ci - ox; ly = cj - oy; lz = ck - oz;
            if ((unsigned)lx >= TILE || (unsigned)ly >= TILE || (unsigned)lz >= TILE) {
                atomicOr(err, ERR_TILE);
                valid = false;
            }
        }
        if (valid) {
            // gather E^n, B^n (CIC on the Yee stagger)
            AxisW X = axis_weights(lx, rx), Y = axis_weights(ly, ry), Z = axis_weights(lz, rz);
            real ex = tri(sF + 0 * FT3, X.ih, Y.in_, Z.in_, X.fh, Y.fn, Z.fn);
            real ey = tri(sF + 1 * FT3, X.in_, Y.ih, Z.in_, X.fn, Y.fh, Z.fn);
            real ez = tri(sF + 2 * FT3, X.in_, Y.in_, Z.ih, X.fn, Y.fn, Z.fh);
            real bx = tri(sF + 3 * FT3, X.in_, Y.ih, Z.ih, X.fn, Y.fh, Z.fh);
            real by = tri(sF + 4 * FT3, X.ih, Y.in_, Z.ih, X.fh, Y.fn, Z.fh);
            real bz = tri(sF + 5 * FT3, X.ih, Y.ih, Z.in_, X.fh, Y.fh, Z.fn);
            real X1, Y1, Z1;
            bool gone = false;   // MODE 2: converted, or left through an open wall
            if (MODE == 2) {
                const double eps = sqrt((double)ux * ux + (double)uy * uy + (double)uz * uz);
                const bool low = qed_chi_below_floor((float)Q.a_s, (float)ex, (float)ey, (float)ez, (float)bx,
                                                     (float)by, (float)bz, (float)ux, (float)uy, (float)uz,
                                                     true, 1e-3f);
                const double chi = low ? 0.0 : qed_chi(Q.a_s, ex, ey, ez, bx, by, bz, ux, uy, uz, true);
                if (sp.qed && chi > 1e-3) {
                    tau -= Q.alpha_as / eps * qed_total(Q.Wb, chi) * g.ddt;
                    if (tau <= 0.0) {
                        uint32_t r[4];
                        draw4(Q.seed, id, (uint32_t)Q.step, TAG_PAIR, 0, r);
                        const double d = qed_fraction(Q.Xb, chi, u01d(r[0]));
                        const double ge = fmax(d * eps, 1.0), gp = fmax((1.0 - d) * eps, 1.0);
                        m1 = sqrt(ge * ge - 1.0) / eps;
                        m2 = sqrt(gp * gp - 1.0) / eps;
                        kx = ux; ky = uy; kz = uz;
                        want1 = Q.have1 && Q.have2;
                        want2 = want1;
                        led += want1 ? (double)w * (eps - ge - gp + 2.0) : (double)w * eps;
                        gone = true;
                    }
                }
                if (!gone) {
                    const real ie = (real)(1.0 / eps);
                    X1 = rx + dtdx * ux * ie;
                    Y1 = ry + dtdy * uy * ie;
                    Z1 = rz + dtdz * uz * ie;
                    if (!per && ((ci == 0 && X1 < (real)0) || (ci == g.nx - 1 && X1 >= (real)1))) {
                        led += (double)w * eps;
                        gone = true;
                    }
                }
            } else {
                if (MODE == 1) {
                    // every lepton particle radiates: one in a fluid node is hot,
                    // or the conversion takes it at the end of this step
                    const bool low = qed_chi_below_floor((float)Q.a_s, (float)ex, (float)ey, (float)ez,
                                                         (float)bx, (float)by, (float)bz, (float)ux, (float)uy,
                                                         (float)uz, false, 1e-3f);
                    const double chi = low ? 0.0 : qed_chi(Q.a_s, ex, ey, ez, bx, by, bz, ux, uy, uz, false);
                    if (chi > 1e-3) {
                        const double gam = sqrt(1.0 + (double)ux * ux + (double)uy * uy + (double)uz * uz);
                        tau -= Q.alpha_as / gam * qed_total(Q.We, chi) * g.ddt;
                        if (tau <= 0.0) {
                            uint32_t r[4];
                            draw4(Q.seed, id, (uint32_t)Q.step, TAG_EMIT, 0, r);
                            const double d = qed_fraction(Q.Xe, chi, u01d(r[0]));
                            kx = d * ux; ky = d * uy; kz = d * uz;
                            ux = (real)(ux - kx); uy = (real)(uy - ky); uz = (real)(uz - kz);
                            draw4(Q.seed, id, (uint32_t)Q.step, TAG_TAU, 0, r);
                            tau = -log(1.0 - u01d(r[0]));
                            const double kk = sqrt(kx * kx + ky * ky + kz * kz);
                            want1 = kk > 2.0 && Q.have1;
                            if (!want1) led += (double)w * kk;
                        }
                    }
                    // the photon is written here, while its momentum is at
                    // hand, rather than held in registers through the push
                    const int k1 = wave_slot(Q.out1_n, want1);
                    if (want1) {
                        if (k1 >= Q.out1_cap) atomicOr(err, ERR_INBOX);
                        else {
                            PArr o = Q.out1;
                            o.cell[k1] = cell;
                            o.rx[k1] = rx; o.ry[k1] = ry; o.rz[k1] = rz;
                            o.ux[k1] = (real)kx; o.uy[k1] = (real)ky; o.uz[k1] = (real)kz;
                            o.w[k1] = w;
                            const uint64_t cid = child_id(id, (uint32_t)Q.step, 1u);
                            o.id[k1] = cid;
                            if (Q.out1_tau) o.tau[k1] = tau0(Q.seed, cid);
                        }
                    }
                }
                // Boris rotation
                real umx = ux + hq * ex, umy = uy + hq * ey, umz = uz + hq * ez;
                real gm = sqrt_((real)1 + umx * umx + umy * umy + umz * umz);
                const real igm = hq * rcp_(gm);
                real tx_ = bx * igm, ty_ = by * igm, tz_ = bz * igm;
                real t2 = tx_ * tx_ + ty_ * ty_ + tz_ * tz_;
                const real is = (real)2 * rcp_(1 + t2);
                real sx = tx_ * is, sy = ty_ * is, sz = tz_ * is;
                real upx = umx + (umy * tz_ - umz * ty_);
                real upy = umy + (umz * tx_ - umx * tz_);
                real upz = umz + (umx * ty_ - umy * tx_);
                real uqx = umx + (upy * sz - upz * sy);
                real uqy = umy + (upz * sx - upx * sz);
                real uqz = umz + (upx * sy - upy * sx);
                ux = uqx + hq * ex; uy = uqy + hq * ey; uz = uqz + hq * ez;
                real gam = sqrt_((real)1 + ux * ux + uy * uy + uz * uz);
                const real igam = rcp_(gam);
                X1 = rx + dtdx * ux * igam;
                Y1 = ry + dtdy * uy * igam;
                Z1 = rz + dtdz * uz * igam;
                // specular reflection at the open x walls
                if (!per) {
                    if (ci == 0 && X1 < (real)0) { X1 = -X1; ux = -ux; }
                    else if (ci == g.nx - 1 && X1 >= (real)1) {
                        X1 = (real)2 - X1; ux = -ux;
                        if (X1 >= (real)1) X1 = below_one();
                    }
                }
            }
            if (gone) {
                valid = false;
            } else if (!(isfinite(ux) && isfinite(uy) && isfinite(uz) && fabs(X1 - rx) < 1 &&
                         fabs(Y1 - ry) < 1 && fabs(Z1 - rz) < 1)) {
                atomicOr(err, isfinite(ux + uy + uz) ? ERR_CFL : ERR_NONFINITE);
                valid = false;
            } else {
                u2max = fmaxf(u2max, (float)(ux * ux + uy * uy + uz * uz));
                // Esirkepov deposit of J^{n+1/2}
                if (MODE != 2 && sp.q != (real)0) {
                    AxisS SX = axis_shapes(rx, X1), SY = axis_shapes(ry, Y1), SZ = axis_shapes(rz, Z1);
                    const real qws = qsc * w;
                    // the axes some depositing lane of this wave crosses along
                    esirkepov_acc(sJ, lx, ly, lz, SX, SY, SZ, qws * cdx, qws * cdy, qws * cdz,
                                  wave_crossings(X1, Y1, Z1));
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
                if (MODE != 2 && A.on) {
                    // conversion: the nearest node after the move is fluid and the
                    // particle is not hot -> it moves virtually onto the node and
                    // joins the node fluid (the node lies in this tile's window)
                    const int dxn = nrx >= (real)0.5, dyn = nry >= (real)0.5, dzn = nrz >= (real)0.5;
                    const int lxn = lx + fx, lyn = ly + fy, lzn = lz + fz;
                    const real u2 = ux * ux + uy * uy + uz * uz;
                    const bool hot = A.hot2 > (real)0 && u2 >= A.hot2;
                    if (!hot && !sSw[(lxn + dxn + 1) + JT * ((lyn + dyn + 1) + JT * (lzn + dzn + 1))]) {
                        AxisS SX = axis_shapes(nrx, (real)dxn), SY = axis_shapes(nry, (real)dyn),
                              SZ = axis_shapes(nrz, (real)dzn);
                        const real qws = qsc * w;
                        // a move onto a node crosses no face
                        esirkepov_acc(sJ, lxn, lyn, lzn, SX, SY, SZ, qws * cdx, qws * cdy, qws * cdz, 0u);
                        int gi = ni + dxn, gj = nj + dyn, gk = nk + dzn;
                        if (per && gi == g.nx) gi = 0;
                        if (gj == g.ny) gj = 0;
                        if (gk == g.nz) gk = 0;
                        const long long node = gidx(g, gi, gj, gk), nn = g.nn;
                        const double dux = ux, duy = uy, duz = uz, dw = w;
                        const double kp = dw * (double)sp.m * (sqrt(1.0 + dux * dux + duy * duy + duz * duz) - 1.0);
                        if (A.warm) atomicAdd(&A.macc[4 * nn + node], kp);
                        else aled += kp;
                        atomicAdd(&A.macc[node], dw);
                        atomicAdd(&A.macc[nn + node], dw * dux);
                        atomicAdd(&A.macc[2 * nn + node], dw * duy);
                        atomicAdd(&A.macc[3 * nn + node], dw * duz);
                        // only when it can widen the range (a stale read costs an atomic)
                        if (gi < *(volatile int *)&A.xr[4]) atomicMin(&A.xr[4], gi);
                        if (gi > *(volatile int *)&A.xr[5]) atomicMax(&A.xr[5], gi);
                        valid = false;
                    }
                }
            }
        }
        // ranks from the tile's counters (zeroed before the launch): one atomic
        // per wave and class, shared by the workgroups of the tile
        const bool stay = valid && ntile == t;
        const bool move = valid && ntile != t;
        const uint64_t ms = __ballot(stay), mm = __ballot(move);
        int bs = 0, bm = 0;
        if (lane == 0) {
            if (ms) bs = atomicAdd(shared ? &nf_out[t] : &s_stay, __popcll(ms));
            if (mm) bm = atomicAdd(shared ? &mcnt[t] : &s_move, __popcll(mm));
            if (shared) pushed += __popcll(ms) + __popcll(mm);
        }
        bs = __shfl(bs, 0);
        bm = __shfl(bm, 0);
        if (valid) {
            // three store groups with uniform bases (no per-lane pointer choice)
            auto put = [&](const PArr &d, long long j) {
                d.cell[j] = ncell;
                d.rx[j] = nrx; d.ry[j] = nry; d.rz[j] = nrz;
                d.ux[j] = ux; d.uy[j] = uy; d.uz[j] = uz;
                d.w[j] = w;
                d.id[j] = id;
                if (sp.has_z) d.zc[j] = zc;
                if (sp.has_tau) d.tau[j] = tau;
            };
            // the output buffer has the input's layout, dout bytes further:
            // its stores reuse the input's field pointers (fewer live SGPRs)
            auto put_out = [&](long long j) {
                const long long o4 = j * 4 + dout, or_ = j * (long long)sizeof(real) + dout, o8 = j * 8 + dout;
                *(int *)((char *)in.cell + o4) = ncell;
                *(real *)((char *)in.rx + or_) = nrx; *(real *)((char *)in.ry + or_) = nry;
                *(real *)((char *)in.rz + or_) = nrz;
                *(real *)((char *)in.ux + or_) = ux; *(real *)((char *)in.uy + or_) = uy;
                *(real *)((char *)in.uz + or_) = uz;
                *(real *)((char *)in.w + or_) = w;
                *(uint64_t *)((char *)in.id + o8) = id;
                if (sp.has_z) *(int *)((char *)in.zc + o4) = zc;
                if (sp.has_tau) *(double *)((char *)in.tau + o8) = tau;
            };
            const int k = bm + __popcll(mm & lt);
            // the mover regions follow the bins in the output buffer; the inbox
            // descriptor is read only when a region overflows.  Stayers and
            // movers share one store sequence.
            if (stay || k < mlim) put_out(stay ? obase + bs + __popcll(ms & lt) : mig0 + mbase + k);
            else {
                const int q = atomicAdd(inbox_n, 1);
                if (q >= inbox_cap) atomicOr(err, ERR_INBOX);
                else put(*inbox_p, q);
            }
        }
        if (MODE == 2) {
            // new particles sit where their parent was at the start of the step
            const int k1 = wave_slot(Q.out1_n, want1);
            const int k2 = wave_slot(Q.out2_n, want2);
            if (want1) {
                if (k1 >= Q.out1_cap) atomicOr(err, ERR_INBOX);
                else {
                    PArr o = Q.out1;
                    o.cell[k1] = cell;
                    o.rx[k1] = rx; o.ry[k1] = ry; o.rz[k1] = rz;
                    const double f = MODE == 2 ? m1 : 1.0;
                    o.ux[k1] = (real)(f * kx); o.uy[k1] = (real)(f * ky); o.uz[k1] = (real)(f * kz);
                    o.w[k1] = w;
                    const uint64_t cid = child_id(id, (uint32_t)Q.step, MODE == 2 ? 2u : 1u);
                    o.id[k1] = cid;
                    if (Q.out1_tau) o.tau[k1] = tau0(Q.seed, cid);
                    if (MODE == 2 && __float_as_uint(fabsf((float)w)) > *Q.wmax1)
                        atomicMax(Q.wmax1, __float_as_uint(fabsf((float)w)));
                }
            }
            if (MODE == 2 && want2) {
                if (k2 >= Q.out2_cap) atomicOr(err, ERR_INBOX);
                else {
                    PArr o = Q.out2;
                    o.cell[k2] = cell;
                    o.rx[k2] = rx; o.ry[k2] = ry; o.rz[k2] = rz;
                    o.ux[k2] = (real)(m2 * kx); o.uy[k2] = (real)(m2 * ky); o.uz[k2] = (real)(m2 * kz);
                    o.w[k2] = w;
                    const uint64_t cid = child_id(id, (uint32_t)Q.step, 3u);
                    o.id[k2] = cid;
                    if (Q.out2_tau) o.tau[k2] = tau0(Q.seed, cid);
                    if (__float_as_uint(fabsf((float)w)) > *Q.wmax2)
                        atomicMax(Q.wmax2, __float_as_uint(fabsf((float)w)));
                }
            }
        }
    }
    if (MODE != 0) {
        for (int o = 32; o > 0; o >>= 1) led += __shfl_xor(led, o);
        if (lane == 0 && led != 0.0) atomicAdd(Q.ledger, led);
    }
    if (MODE != 2 && A.on) {
        for (int o = 32; o > 0; o >>= 1) aled += __shfl_xor(aled, o);
        if (lane == 0 && aled != 0.0) atomicAdd(A.ledger, aled);
    }
    // per-tile bound on |u|^2 of the pushed particles (non-negative float bits
    // order like unsigned integers); read by the next switch evaluation
    for (int o = 32; o > 0; o >>= 1) u2max = fmaxf(u2max, __shfl_xor(u2max, o));
    if (lane == 0 && u2max > 0.f) atomicMax(&s_u2, __float_as_uint(u2max));
    if (shared && lane == 0 && pushed) atomicAdd(&s_stay, pushed);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_u2) atomicMax(&umax2[t], s_u2);
        if (!shared) {
            nf_out[t] = s_stay;   // stayers never exceed the bin: they were in it
            mcnt[t] = s_move;     // the migration reads at most the region's capacity
        }
        atomicAdd(&stats[0], (unsigned long long)(s_stay + s_move));   // particles pushed
        if (item == 0) atomicAdd(&stats[1], 1ull);                     // tiles with particles
    }
    if (MODE == 2) return;
    // flush the LDS current tile (nodes ox-1 .. ox+TILE+1) to the global
    // accumulator: exact integer adds in the FP32 build
    for (int e = threadIdx.x; e < JT3; e += PBS) {
        int a = e % JT, b = (e / JT) % JT, c = e / (JT * JT);
        int gi = ox - 1 + a;
        int gj = wrapi(oy - 1 + b, g.ny), gk = wrapi(oz - 1 + c, g.nz);
        bool okx, okn;
        if (per) { gi = wrapi(gi, g.nx); okx = okn = true; }
        else { okx = gi >= 0 && gi <= g.nx - 1; okn = gi >= 0 && gi <= g.nx; }
        long long c0 = gidx(g, gi < 0 ? 0 : gi, gj, gk);
        if (okx) jg_flush(&Jx[c0], sJ[e], jshift);
        if (okn) jg_flush(&Jy[c0], sJ[JT3 + e], jshift);
        if (okn) jg_flush(&Jz[c0], sJ[2 * JT3 + e], jshift);
    }
}

// --------------------------------------------------- immobile-ion ionization ---------------
// ADK tunnelling blended with the multiphoton continuation by a sigmoid in the
// Keldysh parameter; rates in FP64 (atomic units).  active[t] counts the ions
// of tile t below full ionization; tiles with none are skipped.
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

// Immobile ions of tile t are shared by ION_PARTS workgroups (tile, part
// items spread over the XCDs by slabs of tiles).
constexpr int ION_PARTS = 4;
constexpr int INT_ = TILE + 1;   // nearest-node tile edge
constexpr int INT3 = INT_ * INT_ * INT_;

__global__ void __launch_bounds__(BS)
k_ionize_static(GridP g, SpecP sp, PArr a, Bins bins, int *__restrict__ active,
                const real *__restrict__ Ex, const real *__restrict__ Ey, const real *__restrict__ Ez,
                const uint8_t *__restrict__ sw, int hybrid, const IonP *__restrict__ ion, PArr eout,
                int *__restrict__ eout_n, int eout_cap, uint64_t seed, int step,
                double *__restrict__ ledger, int *__restrict__ err, unsigned *__restrict__ umax2,
                int eout_tau, int nitems) {
    __shared__ real sF[3 * FT3];
    __shared__ uint8_t sS[INT3];
    const int kk = xcd_item(blockIdx.x, gridDim.x);
    if (kk >= nitems) return;
    const int t = kk / ION_PARTS, part = kk % ION_PARTS;
    if (active[t] <= 0) return;   // every ion of the tile at z_max
    int nf = 0, nbv = 0;
    const int n = bin_count(sp, bins, t, nf, nbv);
    if (n > 0) {
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
        // switch map of the tile's nearest nodes ox .. ox + TILE (node nx exists
        // in open x; periodic directions wrap)
        if (hybrid)
            for (int e = threadIdx.x; e < INT3; e += BS) {
                int aa = e % INT_, b = (e / INT_) % INT_, c = e / (INT_ * INT_);
                int gi = ox + aa;
                if (per) gi = wrapi(gi, g.nx);
                sS[e] = sw[gidx(g, gi, wrapi(oy + b, g.ny), wrapi(oz + c, g.nz))];
            }
        __syncthreads();
        const double omega = ion->omega_au;
        const int zmax = ion->z_max;
        const int lane = __lane_id();
        int done = 0;
        const int span = ((n + ION_PARTS - 1) / ION_PARTS + BS - 1) / BS * BS;
        const int pbeg = part * span, pend = min(n, pbeg + span);
        // next iteration's slot, loaded one iteration ahead
        auto ld = [&](int p, int &cell, int &z, real &x, real &y, real &zz, uint64_t &id, long long &ip) {
            cell = -1; z = 0; x = y = zz = 0; id = 0; ip = 0;
            if (p < pend) {
                ip = bin_slot(sp, t, p, nf, nbv);
                cell = a.cell[ip]; z = a.zc[ip];
                x = a.rx[ip]; y = a.ry[ip]; zz = a.rz[ip];
                id = a.id[ip];
            }
        };
        int ncell, nz0; real nrx, nry, nrz; uint64_t nid; long long nip;
        ld(pbeg + threadIdx.x, ncell, nz0, nrx, nry, nrz, nid, nip);
        // uniform trip count so that every lane of a wave takes part in the
        // event-slot scan below
        for (int p0 = pbeg; p0 < pend; p0 += BS) {
            const int cell = ncell, z0 = ncell >= 0 ? nz0 : 0;
            const real rx = nrx, ry = nry, rz = nrz;
            const uint64_t pid = nid;
            const long long ip = nip;
            if (p0 + BS < pend) ld(p0 + BS + threadIdx.x, ncell, nz0, nrx, nry, nrz, nid, nip);
            int nev = 0;
            bool live = cell >= 0 && z0 < zmax;
            int ci = 0, cj = 0, ck = 0;
            if (live) cell_ijk(g, cell, ci, cj, ck);
            const int lx = ci - ox, ly = cj - oy, lz = ck - oz;
            if (live && ((unsigned)lx >= TILE || (unsigned)ly >= TILE || (unsigned)lz >= TILE)) {
                atomicOr(err, ERR_TILE);
                live = false;
            }
            if (live && hybrid) {
                const int e = (lx + (rx >= (real)0.5)) + INT_ * ((ly + (ry >= (real)0.5)) + INT_ * (lz + (rz >= (real)0.5)));
                if (!sS[e]) live = false;
            }
            if (live) {
                AxisW X = axis_weights(lx, rx), Y = axis_weights(ly, ry), Z = axis_weights(lz, rz);
                double ex = tri(sF + 0 * FT3, X.ih, Y.in_, Z.in_, X.fh, Y.fn, Z.fn);
                double ey = tri(sF + 1 * FT3, X.in_, Y.ih, Z.in_, X.fn, Y.fh, Z.fn);
                double ez = tri(sF + 2 * FT3, X.in_, Y.in_, Z.ih, X.fn, Y.fn, Z.fh);
                double F = sqrt(ex * ex + ey * ey + ez * ez) * ion->field_au;
                // levels ionize in sequence; below fskip the probability is under
                // the smallest uniform draw, so no event is possible; a draw at or
                // above the level's probability bound for this field decides
                // "no event" without evaluating the rate
                const float lf = __log2f((float)F);
                for (int lev = z0; lev < zmax; ++lev) {
                    const IonLevel &L = ion->lev[lev];
                    if (F < L.fskip) break;
                    uint32_t r[4];
                    draw4(seed, pid, (uint32_t)step, TAG_ION + (uint32_t)lev, 0, r);
                    const double u = u01d(r[0]);
                    const int b = min(max((int)((lf - L.lf0) * L.ilr), 0), ION_NBND - 1);
                    if (u >= (double)L.bnd[b]) break;
                    const double wr = blended_rate(L, F, omega) * ion->rate_norm;
                    const double P = -expm1(-wr * g.ddt);
                    if (!(u < P)) break;
                    nev++;
                }
            }
            // one slot reservation per wave: inclusive scan of the event counts
            int incl = nev;
            for (int o = 1; o < 64; o <<= 1) {
                const int v = __shfl_up(incl, o);
                if (lane >= o) incl += v;
            }
            const int tot = __shfl(incl, 63);
            if (tot == 0) continue;
            int base = 0;
            if (lane == 63) base = atomicAdd(eout_n, tot);
            base = __shfl(base, 63);
            double led = 0.0;
            if (nev) {
                const real ux = a.ux[ip], uy = a.uy[ip], uz = a.uz[ip], w = a.w[ip];
                const float u2 = (float)(ux * ux + uy * uy + uz * uz);
                if (u2 > 0.f) atomicMax(&umax2[t], __float_as_uint(u2));   // newborns keep the ion's u
                for (int e = 0; e < nev; ++e) {
                    const int k = base + incl - nev + e;
                    const int lev = z0 + e;
                    if (k >= eout_cap) { atomicOr(err, ERR_INBOX); break; }
                    eout.cell[k] = cell;
                    eout.rx[k] = rx; eout.ry[k] = ry; eout.rz[k] = rz;
                    eout.ux[k] = ux; eout.uy[k] = uy; eout.uz[k] = uz;
                    eout.w[k] = w;
                    eout.id[k] = (1ull << 62) | ((uint64_t)lev << 56) | pid;
                    if (eout_tau) eout.tau[k] = tau0(seed, eout.id[k]);
                    led += (double)w * ion->lev[lev].ip_au * 27.211386245988 / 510998.95;
                }
                a.zc[ip] = z0 + nev;
                if (z0 + nev >= zmax) done++;
            }
            for (int o = 32; o > 0; o >>= 1) led += __shfl_xor(led, o);
            if (lane == 0 && led != 0.0) atomicAdd(ledger, led);
        }
        if (done) atomicSub(&active[t], done);
    }
}

// Ions below full ionization per tile.
__global__ void __launch_bounds__(BS)
k_count_active(GridP g, SpecP sp, PArr a, Bins bins, int zmax, int *__restrict__ active) {
    const int t = blockIdx.x;
    int nf, nbv;
    const int n = bin_count(sp, bins, t, nf, nbv);
    int c = 0;
    for (int p = threadIdx.x; p < n; p += BS) {
        const long long ip = bin_slot(sp, t, p, nf, nbv);
        if (a.cell[ip] >= 0 && a.zc[ip] < zmax) c++;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(&active[t], c);
}

// ----------------------------------------------------------- charge density ---------------
__global__ void __launch_bounds__(BS)
k_rho(GridP g, SpecP sp, PArr a, Bins bins, double *__restrict__ rho) {
    const int t = blockIdx.x;
    int nf, nbv;
    const int n = bin_count(sp, bins, t, nf, nbv);
    const double dv = g.ddx * g.ddy * g.ddz;
    const int per = g.bcx == HK_BC_PERIODIC;
    for (int p = threadIdx.x; p < n; p += BS) {
        const long long ip = bin_slot(sp, t, p, nf, nbv);
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

void launch_init_species_cols(const GridP &g, const hk_species_desc &d, int isp, uint64_t seed, PArr out,
                              const int *xcol, const double *wcol, int ncol, int has_z,
                              int has_tau, hipStream_t s) {
    long long total = (long long)ncol * g.ny * g.nz * d.ppc;
    if (total == 0) return;
    k_init<<<blocks(total), BS, 0, s>>>(g, d.ppc, isp, d.u_th, d.charge, seed, xcol, wcol, ncol, total,
                                        out, has_z, has_tau);
}

// maxn bounds the entries of the largest group (sets the grid's x extent)
void launch_count_groups(const GridP &g, PArr src, const long long *off, const int *nf,
                         const int *nb, const int *cap, int ngroups, long long maxn, int *newcnt,
                         hipStream_t s) {
    if (ngroups == 0 || maxn == 0) return;
    unsigned bx = blocks(maxn);
    if (bx > 4096u) bx = 4096u;
    k_count<<<dim3(ngroups, bx), BS, 0, s>>>(g, src, off, nf, nb, cap, newcnt);
}

void launch_scatter_groups(const GridP &g, PArr src, const long long *off, const int *nf,
                           const int *nb, const int *cap, int ngroups, long long maxn, PArr dst,
                           const long long *doff, int *dfill, int has_z, int has_tau,
                           hipStream_t s) {
    if (ngroups == 0 || maxn == 0) return;
    unsigned bx = blocks(maxn);
    if (bx > 4096u) bx = 4096u;
    k_scatter<<<dim3(ngroups, bx), BS, 0, s>>>(g, src, off, nf, nb, cap, dst, doff, dfill, has_z,
                                               has_tau);
}

// The fail list has the inbox's capacity (max_n).
void launch_merge_inbox(const GridP &g, const SpecP &sp, PArr inbox, const int *inbox_n,
                        long long max_n, PArr dst, const int *nf, int *nb, int *fail_n, PArr fail,
                        int *err, hipStream_t s) {
    if (max_n == 0) return;
    unsigned nb_ = blocks(max_n);
    k_merge<<<nb_ < 1024u ? nb_ : 1024u, BS, 0, s>>>(g, sp, inbox, inbox_n, (int)max_n, dst, nf, nb,
                                                     fail_n, fail, (int)max_n, err);
}

void launch_migrate(const GridP &g, const SpecP &sp, PArr mig, const long long *moff,
                    const int *mcnt, const int *mcap, PArr dst, const int *nf, int *nb, int *fail_n,
                    PArr fail, int fail_cap, int *err, hipStream_t s) {
    const int n = g.ntiles * MIGRATE_PARTS;
    k_migrate<<<(n + 7) / 8 * 8, BS, 0, s>>>(g, sp, mig, moff, mcnt, mcap, dst, nf, nb, fail_n, fail,
                                              fail_cap, err, n);
}

long long tile_plan_items(const GridP &g) { return (long long)g.ntiles * TILE_SPLIT; }

// Items: at most TILE_SPLIT per tile, and at most one per tile plus one per
// cmin particles (chunks are never shorter than cmin but the last); surplus
// workgroups find the ticket past the end.
unsigned tile_plan_grid(const GridP &g, long long capacity, int cmin) {
    return (unsigned)std::min<long long>((long long)g.ntiles * TILE_SPLIT, g.ntiles + capacity / cmin + 1);
}

void launch_tile_plan(const GridP &g, const SpecP &sp, Bins b, int cmin, int2 *items, int *ctl,
                      hipStream_t s) {
    plan_tiles(g, sp, b, cmin, items, ctl, nullptr, nullptr, s);
}

void launch_push_tiles(const GridP &g, const SpecP &sp, PArr in, Bins bin_in, PArr out,
                       int *nf_out, long long mig0, const long long *moff, const int *mcap, int *mcnt,
                       const PArr *inbox_p, int *inbox_n, int inbox_cap, real *const f[9], jglob_t *jg,
                       int *err, unsigned long long *stats, const unsigned *wmax_bits, unsigned *umax2,
                       int mode, const QedP &Q, const AbsorbP &A, int2 *items, int *ctl,
                       long long capacity, int *live, hipStream_t s) {
#define HK_PUSH_ARGS g, sp, in, bin_in, dout, nf_out, mig0, moff, mcap, mcnt, inbox_p, inbox_n, inbox_cap, \
        f[HK_EX], f[HK_EY], f[HK_EZ], f[HK_BX], f[HK_BY], f[HK_BZ], jg, jg + g.nn, jg + 2 * g.nn, err, \
        stats, wmax_bits, umax2, items, ctl, Q, A
    // nf_out is the first of the next buffer's three counter arrays (front
    // fills, back fills, mover ranks), cleared by the planner
    plan_tiles(g, sp, bin_in, PUSH_CHUNK, items, ctl, nf_out, live, s);
    // the two bin buffers share one layout (checked when they are allocated):
    // every field of `out` sits the same byte distance from that of `in`
    const long long dout = (const char *)out.cell - (const char *)in.cell;
    const unsigned grid = tile_plan_grid(g, capacity, PUSH_CHUNK);
    if (mode == 1) k_push<1><<<grid, PBS, 0, s>>>(HK_PUSH_ARGS);
    else if (mode == 2) k_push<2><<<grid, PBS, 0, s>>>(HK_PUSH_ARGS);
    else k_push<0><<<grid, PBS, 0, s>>>(HK_PUSH_ARGS);
#undef HK_PUSH_ARGS
}

void launch_ionize_static(const GridP &g, const SpecP &sp, PArr a, Bins b, int *active,
                          real *const f[9], const uint8_t *sw, int hybrid, const IonP *ion,
                          PArr eout, int *eout_n, int eout_cap, uint64_t seed, int step,
                          double *ledger, int *err, unsigned *umax2, int eout_tau, hipStream_t s) {
    const int n = g.ntiles * ION_PARTS;
    k_ionize_static<<<(n + 7) / 8 * 8, BS, 0, s>>>(g, sp, a, b, active, f[HK_EX], f[HK_EY], f[HK_EZ],
                                                   sw, hybrid, ion, eout, eout_n, eout_cap, seed, step,
                                                   ledger, err, umax2, eout_tau, n);
}

void launch_count_active(const GridP &g, const SpecP &sp, PArr a, Bins b, int zmax, int *active,
                         hipStream_t s) {
    k_count_active<<<g.ntiles, BS, 0, s>>>(g, sp, a, b, zmax, active);
}

void launch_rho_tiles(const GridP &g, const SpecP &sp, PArr a, Bins b, double *rho, hipStream_t s) {
    k_rho<<<g.ntiles, BS, 0, s>>>(g, sp, a, b, rho);
}
