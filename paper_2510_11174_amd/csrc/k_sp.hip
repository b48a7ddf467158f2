// The next-state surrogate on gfx950: a residual 3D CNN (six "same" 3^3
// convolutions, widths 10-13-32-64-128-32-10) that maps a normalized state
// patch (E, B, J, rho at the nodes) to the state a few steps later, with its
// loss (Huber plus an energy-violation term), backward pass and packing.
//
// Paper: Results, Table 2 (StatePredictor layers) and the paragraph before it
// (residual blocks, dropout, Huber loss, physics term on the field energy).
//
// Storage: activations BF16, channels last, the channel count padded to a
// multiple of 16 (CP) with zeros.  Convolutions are implicit GEMMs on
// v_mfma_f32_16x16x32_bf16: rows are 16 consecutive voxels along x, columns
// output channels, K = (tap, input channel), k = t CP + ci, tap
// t = kx + 3 ky + 9 kz reading offset (kx - 1, ky - 1, kz - 1), zero outside
// the patch.  Lane l supplies A[l%16][8 (l/16) .. +8] (one 16-byte load of 8
// channels of one voxel), B[8 (l/16) .. +8][l%16] (16 bytes of the weight
// matrix stored column-major, [column][K]) and gets D[4 (l/16) + i][l%16].
// A wave owns MT row tiles x NT column tiles, so each fragment it loads feeds
// NT (A) or MT (B) matrix instructions.
//
// The data gradient is the same GEMM over input voxels with the transposed,
// tap-reversed weights (tap 26 - t): a "same" convolution of the output
// gradient.  Its epilogue finishes the layer below in place: it adds the
// residual path, applies the dropout factors and the ReLU derivative, and
// writes that layer's pre-activation gradient in BF16.
//
// The weight gradient contracts over voxels, which lie along x in memory only
// in a channel-major copy ([b][c][z][y][x]) that the forward and backward
// epilogues write beside the channels-last tensors.  A lane then loads 8
// consecutive x of one channel with one 16-byte load; the x shift of taps
// kx = 0 and 2 is done in registers from the neighbouring 8-voxel blocks.
#include "hk_internal.h"
#include "hk_sp_internal.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int SBS = 256;                  // 4 waves

__device__ inline u16 bf16_bits(float x) {
    // round to nearest even (finite inputs)
    const unsigned u = __float_as_uint(x);
    return (u16)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_val(u16 b) { return __uint_as_float((unsigned)b << 16); }

// dropout keep factor of channel c at voxel v: byte c % 16 of Philox draw
// sample * cols / 16 + c / 16 (counter: voxel, step) at or above drop_thr
// keeps the channel, scaled by drop_scale
__device__ inline float keep(const SpConv &a, uint64_t v, int c) {
    uint32_t r[4];
    draw4(a.seed, v, a.step, a.drop_tag, (uint32_t)(a.drop_sample * (a.cols >> 4) + (c >> 4)), r);
    const int byte = c & 15;
    return ((r[byte >> 2] >> (8 * (byte & 3))) & 0xffu) >= a.drop_thr ? a.drop_scale : 0.0f;
}

// blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous run
// of work items so neighbouring rows share one L2 (nb is a multiple of 8)
__device__ inline int xcd_block(int b, int nb) { return (b & 7) * (nb >> 3) + (b >> 3); }

// ------------------------------------------------------------ convolution
// Epilogue of one 16-voxel row tile (voxels x0 .. x0 + 15 of row (b, z, y)):
// lane (r, g) holds channel co = 16 (cg NT + nt) + r of voxels x0 + 4 g + i.
// Forward: bias, BF16 pre-activation (training), ReLU, residual copy,
// dropout, one rounding to BF16 (or the FP32 output of the last layer).
// Data gradient: residual-path gradient, dropout, ReLU derivative of the
// layer below (when it has one), BF16.  Both write the channel-major copy when asked.
// With `stage` (LDS, 16 rows of stride ST) the channels-last result goes
// there instead of to aout; the caller copies it out in 16-byte pieces.
template <int CPIN, int NT, bool BWD>
__device__ inline void store_row(const SpConv &a, const f32x4 (&acc)[NT], int b, int z, int y, int x0, int cg,
                                 int r, int g, u16 *stage = nullptr, int ST = 0) {
    const long long HW = (long long)a.H * a.W;
    const int xg = x0 + 4 * g;
    const long long vrow = ((long long)b * a.D + z) * HW + (long long)y * a.W;
    // dropout decisions of the lane's 4 NT elements, bit nt * 4 + i; one
    // rolled loop keeps a single copy of the Philox body in the code
    uint32_t dropped = 0;
    if (a.drop) {
#pragma unroll 1
        for (int q = 0; q < 4 * NT; ++q) {
            const int x = xg + (q & 3);
            if (x < a.W && keep(a, (uint64_t)(vrow + x), (cg * NT + (q >> 2)) * 16 + r) == 0.f) dropped |= 1u << q;
        }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int co = (cg * NT + nt) * 16 + r;
        const bool real_c = co < a.cout;
        const float bco = (!BWD && real_c) ? a.bias[co] : 0.f;
        u16 ov[4] = {0, 0, 0, 0};
        for (int i = 0; i < 4; ++i) {
            const int x = xg + i;
            if (x >= a.W) continue;
            const long long v = vrow + x;
            float s = acc[nt][i];
            if (!BWD) {
                s += bco;
                if (a.zout) a.zout[v * a.cols + co] = real_c ? bf16_bits(s) : (u16)0;
                float o = a.relu ? fmaxf(s, 0.f) : s;
                if (co < a.res) o += bf16_val(a.in[v * CPIN + co]);
                if (a.fout) {
                    if (real_c) a.fout[v * a.cout + co] = o;
                    continue;
                }
                if (a.drop) o *= (dropped >> (nt * 4 + i)) & 1u ? 0.f : a.drop_scale;
                ov[i] = real_c ? bf16_bits(o) : (u16)0;
            } else {
                if (co < a.gin_ch) s += a.gin[v * a.gin_stride + co];
                if (a.drop) s *= (dropped >> (nt * 4 + i)) & 1u ? 0.f : a.drop_scale;
                if (a.gout) a.gout[v * a.cols + co] = s;
                const float d = !a.zin || bf16_val(a.zin[v * a.cols + co]) > 0.f ? s : 0.f;
                ov[i] = real_c ? bf16_bits(d) : (u16)0;
            }
            if (stage) stage[(4 * g + i) * ST + nt * 16 + r] = ov[i];
            else a.aout[v * a.cols + co] = ov[i];
        }
        if (a.aT && xg < a.W) {
            // channel-major copy: 4 consecutive x of channel co (W % 4 == 0)
            const long long o = (((long long)b * a.cols + co) * a.D + z) * HW + (long long)y * a.W + xg;
            *reinterpret_cast<uint2 *>(a.aT + o) =
                make_uint2((unsigned)ov[0] | ((unsigned)ov[1] << 16), (unsigned)ov[2] | ((unsigned)ov[3] << 16));
        }
    }
}

// TAPS = 27: the "same" 3^3 convolution; TAPS = 1: a linear layer per voxel
// (the one tap reads the voxel itself).
template <int CPIN, int MT, int NT, bool BWD, int TAPS>
__global__ void __launch_bounds__(SBS) k_sp_conv(SpConv a) {
    constexpr int K = TAPS * CPIN, KPAD = (K + 31) / 32 * 32, NK = KPAD / 32;
    const int task = xcd_block(blockIdx.x, gridDim.x) * (SBS / 64) + (threadIdx.x >> 6);
    if (task >= a.ntask) return;
    const int cg = task % a.G, rg = task / a.G;
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    const int segs = (a.W + 15) >> 4;
    const long long nrows = (long long)a.B * a.D * a.H * segs;
    const long long HW = (long long)a.H * a.W;

    // per row tile: this lane's voxel and the taps that stay inside the patch
    long long vb[MT];
    unsigned tmask[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const long long row = (long long)rg * MT + m;
        vb[m] = 0;
        tmask[m] = 0;
        if (row >= nrows) continue;
        const int seg = (int)(row % segs);
        long long q = row / segs;
        const int y = (int)(q % a.H);
        q /= a.H;
        const int z = (int)(q % a.D);
        const int b = (int)(q / a.D);
        const int x = seg * 16 + r;
        if (x >= a.W) continue;
        vb[m] = ((long long)b * a.D + z) * HW + (long long)y * a.W + x;
        if (TAPS == 1) tmask[m] = 1u;
        else
            for (int t = 0; t < 27; ++t) {
                const int xx = x + t % 3 - 1, yy = y + (t / 3) % 3 - 1, zz = z + t / 9 - 1;
                if (xx >= 0 && xx < a.W && yy >= 0 && yy < a.H && zz >= 0 && zz < a.D) tmask[m] |= 1u << t;
            }
    }
    const u16 *wrow[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) wrow[nt] = a.wp + (long long)((cg * NT + nt) * 16 + r) * KPAD + 8 * g;

    auto loadA = [&](int ks, uint4 (&av)[MT]) {
        const int k = ks * 32 + 8 * g;
        const int t = k / CPIN, ci = k % CPIN;
        const int kx = TAPS == 1 ? 1 : t % 3, ky = TAPS == 1 ? 1 : (t / 3) % 3, kz = TAPS == 1 ? 1 : t / 9;
        const long long off = ((long long)(kz - 1) * a.H + (ky - 1)) * a.W + (kx - 1);
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            av[m] = make_uint4(0, 0, 0, 0);
            if (k < K && ((tmask[m] >> t) & 1u))
                av[m] = *reinterpret_cast<const uint4 *>(a.in + (vb[m] + off) * CPIN + ci);
        }
    };
    auto loadB = [&](int ks, uint4 (&bv)[NT]) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) bv[nt] = *reinterpret_cast<const uint4 *>(wrow[nt] + ks * 32);
    };

    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[m][nt] = f32x4{0, 0, 0, 0};
    uint4 av[MT], bv[NT];
    loadA(0, av);
    loadB(0, bv);
    for (int ks = 0; ks < NK; ++ks) {
        uint4 an[MT], bn[NT];
        if (ks + 1 < NK) {
            loadA(ks + 1, an);
            loadB(ks + 1, bn);
        } else {
#pragma unroll
            for (int m = 0; m < MT; ++m) an[m] = make_uint4(0, 0, 0, 0);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) bn[nt] = make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                acc[m][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av[m]),
                                                                    __builtin_bit_cast(bf16x8, bv[nt]),
                                                                    acc[m][nt], 0, 0, 0);
#pragma unroll
        for (int m = 0; m < MT; ++m) av[m] = an[m];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) bv[nt] = bn[nt];
    }

    // epilogue: D[4 g + i][r] is voxel x0 + 4 g + i, channel co
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const long long row = (long long)rg * MT + m;
        if (row >= nrows) continue;
        const int seg = (int)(row % segs);
        long long q = row / segs;
        const int y = (int)(q % a.H);
        q /= a.H;
        const int z = (int)(q % a.D);
        const int b = (int)(q / a.D);
        store_row<CPIN, NT, BWD>(a, acc[m], b, z, y, seg * 16, cg, r, g);
    }
}

// Halo-tiled variant for 32 or more input channels.  A workgroup owns 16 x MT
// x 4 output voxels (x segment, MT rows in y, 4 in z: wave w takes z slice w)
// and one column group.  For each 32-channel slice of the input it stages the
// tile's halo, 18 x (MT + 2) x 6 voxels of 64 bytes, in LDS with coalesced
// 16-byte loads, then runs the 27 taps of the slice: A fragments come from LDS
// (16 consecutive voxels of 64 bytes; the four 16-byte pieces of voxel h are
// stored in the order given by XOR with (h / 2) % 4, so eight consecutive
// lanes reading the same piece of eight voxels hit 32 different banks), one
// tap ahead; B fragments come from the weight matrix in global memory, three
// taps ahead (the four waves read the same B, so it stays in L1).  Each input
// voxel is fetched once per slice instead of once per tap.
constexpr int HZ = 4;   // tile depth in z (one slice per wave)
#ifndef SP_HALO_NT
#define SP_HALO_NT 2
#endif
template <int CPIN, int MT, int NT, bool BWD>
__global__ void __launch_bounds__(SBS) __attribute__((amdgpu_waves_per_eu(2, 8))) k_sp_conv_halo(SpConv a) {
    constexpr int HY = MT + 2, HX = 18, NV = HX * HY * (HZ + 2);
    constexpr int K = 27 * CPIN, KPAD = (K + 31) / 32 * 32;
    __shared__ __attribute__((aligned(16))) u16 sH[NV * 32];
    const int item = xcd_block(blockIdx.x, gridDim.x);
    if (item >= a.ntask) return;   // uniform over the workgroup
    const int cg = item % a.G;
    int q = item / a.G;
    const int segs = (a.W + 15) >> 4, nty = (a.H + MT - 1) / MT, ntz = (a.D + HZ - 1) / HZ;
    const int seg = q % segs;
    q /= segs;
    const int ty0 = (q % nty) * MT;
    q /= nty;
    const int tz0 = (q % ntz) * HZ;
    const int b = q / ntz;
    const int x0 = seg * 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
    const long long HW = (long long)a.H * a.W;
    const u16 *src = a.in + (long long)b * a.D * HW * CPIN;
    const u16 *wrow[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) wrow[nt] = a.wp + (long long)((cg * NT + nt) * 16 + r) * KPAD + 8 * g;
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[m][nt] = f32x4{0, 0, 0, 0};
    // B fragments of linear tap T = slice * 27 + t
    constexpr int NTAP = CPIN / 32 * 27;
    auto loadB = [&](int T, uint4 (&bv)[NT]) {
        // past the last tap: reload the last one (unused), so the loads stay
        // unconditional and their waits exact
        T = T < NTAP ? T : NTAP - 1;
        const int c = T / 27, t = T - 27 * c;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) bv[nt] = *reinterpret_cast<const uint4 *>(wrow[nt] + t * CPIN + 32 * c);
    };
    // A fragments of tap t for the wave's MT rows, from the halo
    auto loadA = [&](int t, uint4 (&av)[MT]) {
        const int kx = t % 3, ky = (t / 3) % 3, kz = t / 9;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int hv = ((wave + kz) * HY + (m + ky)) * HX + r + kx;
            av[m] = *reinterpret_cast<const uint4 *>(sH + hv * 32 + 8 * (g ^ ((hv >> 1) & 3)));
        }
    };
    auto mma = [&](const uint4 (&av)[MT], const uint4 (&bv)[NT]) {
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                acc[m][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av[m]),
                                                                    __builtin_bit_cast(bf16x8, bv[nt]), acc[m][nt],
                                                                    0, 0, 0);
    };
    uint4 b0[NT], b1[NT], b2[NT];
    loadB(0, b0);
    loadB(1, b1);
    loadB(2, b2);
    for (int c0 = 0; c0 < CPIN; c0 += 32) {
        __syncthreads();   // the previous slice is consumed
        for (int p = threadIdx.x; p < NV * 4; p += SBS) {
            const int hv = p >> 2, part = p & 3;
            const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
            const int x = x0 - 1 + hx, y = ty0 - 1 + hy, z = tz0 - 1 + hz;
            uint4 val = make_uint4(0, 0, 0, 0);
            if (x >= 0 && x < a.W && y >= 0 && y < a.H && z >= 0 && z < a.D)
                val = *reinterpret_cast<const uint4 *>(src + ((long long)z * HW + (long long)y * a.W + x) * CPIN +
                                                       c0 + part * 8);
            *reinterpret_cast<uint4 *>(sH + hv * 32 + 8 * (part ^ ((hv >> 1) & 3))) = val;
        }
        __syncthreads();
        const int T0 = c0 / 32 * 27;
        uint4 a0[MT], a1[MT];
        loadA(0, a0);
        for (int t = 0; t < 27; t += 3) {
            loadA(t + 1, a1);
            mma(a0, b0);
            loadB(T0 + t + 3, b0);
            loadA(t + 2, a0);
            mma(a1, b1);
            loadB(T0 + t + 4, b1);
            loadA(t + 3 < 27 ? t + 3 : 26, a1);
            mma(a0, b2);
            loadB(T0 + t + 5, b2);
#pragma unroll
            for (int m = 0; m < MT; ++m) a0[m] = a1[m];
        }
    }
    const int z = tz0 + wave;
    if (z >= a.D) return;
#pragma unroll
    for (int m = 0; m < MT; ++m)
        if (ty0 + m < a.H) store_row<CPIN, NT, BWD>(a, acc[m], b, z, ty0 + m, x0, cg, r, g);
}

// Linear layers (one tap) over n = B D H W voxels taken 16 at a time in
// storage order.  A workgroup owns one column group: its NT * 16 columns of
// the weight matrix (all of K) sit in LDS, rows padded by 16 bytes so that
// the 16 lanes reading one k range of 16 columns hit different banks; its
// four waves then walk row tiles of 4 x 16 voxels, A fragments from global
// memory (each row read once per column group).
template <int CPIN, int NT, bool BWD>
__global__ void __launch_bounds__(SBS) __attribute__((amdgpu_waves_per_eu(2, 8))) k_sp_lin(SpConv a) {
    constexpr int MT = 4, KPAD = (CPIN + 31) / 32 * 32, NK = KPAD / 32, KS = KPAD + 8, ST = NT * 16 + 8;
    __shared__ __attribute__((aligned(16))) u16 sB[NT * 16 * KS];
    __shared__ __attribute__((aligned(16))) u16 sS[SBS / 64 * 16 * ST];
    // block b runs on XCD b % 8: the G column groups of one set of rows go
    // to blocks b, b + 8, ... on the same XCD, so the rows are fetched into
    // that XCD's L2 once (gridDim.x = G * nwg, nwg a multiple of 8)
    const int cg = (blockIdx.x >> 3) % a.G, wgi = (blockIdx.x & 7) + 8 * ((blockIdx.x >> 3) / a.G);
    const int nwg = gridDim.x / a.G;
    const u16 *wsrc = a.wp + (long long)cg * NT * 16 * KPAD;
    for (int e = threadIdx.x; e < NT * 16 * KPAD / 8; e += SBS) {
        const int col = e / (KPAD / 8), k8 = e % (KPAD / 8);
        *reinterpret_cast<uint4 *>(sB + col * KS + 8 * k8) = reinterpret_cast<const uint4 *>(wsrc)[e];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
    const long long n = (long long)a.B * a.D * a.H * a.W;
    const long long ntiles = (n + 15) / 16;
    for (long long t0 = ((long long)wgi * (SBS / 64) + wave) * MT; t0 < ntiles; t0 += (long long)nwg * (SBS / 64) * MT) {
        f32x4 acc[MT][NT];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[m][nt] = f32x4{0, 0, 0, 0};
#pragma unroll 2
        for (int ks = 0; ks < NK; ++ks) {
            const int k = ks * 32 + 8 * g;
            uint4 av[MT], bv[NT];
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const long long v = (t0 + m) * 16 + r;
                av[m] = (v < n && k < CPIN) ? *reinterpret_cast<const uint4 *>(a.in + v * CPIN + k) : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) bv[nt] = *reinterpret_cast<const uint4 *>(sB + (nt * 16 + r) * KS + k);
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[m][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av[m]),
                                                                        __builtin_bit_cast(bf16x8, bv[nt]),
                                                                        acc[m][nt], 0, 0, 0);
        }
        // rows of 16 voxels in storage order: as x segments of one row when
        // the voxels are one line (B = D = H = 1).  The BF16 result goes
        // through the wave's LDS stage and out in 16-byte pieces.
        u16 *stage = sS + wave * 16 * ST;
        const bool staged = a.aout && !a.fout;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const long long v0 = (t0 + m) * 16;
            if (v0 >= n) continue;
            store_row<CPIN, NT, BWD>(a, acc[m], 0, 0, 0, (int)v0, cg, r, g, staged ? stage : nullptr, ST);
            if (!staged) continue;
            // the stage is written and read by this wave only: LDS keeps a
            // wave's accesses in order, the fences keep the compiler's
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int j = 0; j < (32 * NT + 63) / 64; ++j) {   // 16 rows x 2 NT pieces
                const int c = lane + 64 * j, per_row = NT * 2;
                if (c >= 16 * per_row) break;
                const int vr = c / per_row, part = c % per_row;
                const long long v = v0 + vr;
                if (v < n)
                    *reinterpret_cast<uint4 *>(a.aout + v * a.cols + cg * NT * 16 + part * 8) =
                        *reinterpret_cast<const uint4 *>(stage + vr * ST + part * 8);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// -------------------------------------------------------- weight gradient
// gw[t][ci][co] += sum_v a[v + off(t)][ci] dz[v][co].  K runs over 8-voxel
// blocks along x (W % 8 == 0), four blocks per step: lane (r, g) takes block
// 4 ks + g, A[r = ci][8 g + j] = a[x + j + kx - 1] of channel ci and B[8 g + j]
// [r = co] = dz[x + j] of channel co, both from the channel-major copies.  A
// workgroup owns one (ky, kz) pair, one 16-channel ci tile, NT co tiles and a
// chunk of K; its four waves take interleaved steps of the chunk, reduce in
// LDS, and wave 0 adds the three taps kx = 0, 1, 2 to gw.
// With ONE (a linear layer: the single tap is the voxel itself) there is
// one (ky, kz) pair and one kx.
template <int NT, bool ONE>
__global__ void __launch_bounds__(SBS) k_sp_wgrad(SpWgrad a) {
    constexpr int NKX = ONE ? 1 : 3;
    __shared__ f32x4 red[SBS / 64 - 1][NKX * NT][64];
    __shared__ float sb[NT * 16];
    const int item = xcd_block(blockIdx.x, gridDim.x);
    if (item >= a.nitems) return;   // uniform over the workgroup
    int q = item;
    const int p = ONE ? 4 : q % 9;
    if (!ONE) q /= 9;
    const int mt = q % a.mtn;
    q /= a.mtn;
    const int ng = q % a.ngn;
    const int chunk = q / a.ngn;
    const int ky = p % 3, kz = p / 3;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
    const int xbn = a.W >> 3;
    // the centre-tap workgroups of the first ci tile also sum dz: the bias
    // gradient, each voxel counted once per column group
    const bool bias = a.gb && p == 4 && mt == 0;
    float bsum[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) bsum[nt] = 0.f;
    if (threadIdx.x < NT * 16) sb[threadIdx.x] = 0.f;
    const long long HW = (long long)a.H * a.W, DHW = HW * a.D;
    const int ci = mt * 16 + r;
    f32x4 acc[NKX][NT];
#pragma unroll
    for (int kx = 0; kx < NKX; ++kx)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[kx][nt] = f32x4{0, 0, 0, 0};
    const long long ks0 = (long long)chunk * a.kpc;
    long long ks1 = ks0 + a.kpc;
    if (ks1 > a.nks) ks1 = a.nks;
    for (long long ks = ks0 + wave; ks < ks1; ks += SBS / 64) {
        const long long blk = ks * 4 + g;
        uint4 L = make_uint4(0, 0, 0, 0), M = L, R = L, Bv[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) Bv[nt] = L;
        if (blk < a.nblk) {
            const int xb = (int)(blk % xbn);
            long long rq = blk / xbn;
            const int y = (int)(rq % a.H);
            rq /= a.H;
            const int z = (int)(rq % a.D);
            const int b = (int)(rq / a.D);
            const int ys = y + ky - 1, zs = z + kz - 1;
            if (ys >= 0 && ys < a.H && zs >= 0 && zs < a.D) {
                const u16 *src = a.aT + ((long long)b * a.cpi + ci) * DHW + zs * HW + (long long)ys * a.W + 8 * xb;
                M = *reinterpret_cast<const uint4 *>(src);
                if (!ONE && xb > 0) L = *reinterpret_cast<const uint4 *>(src - 8);
                if (!ONE && xb + 1 < xbn) R = *reinterpret_cast<const uint4 *>(src + 8);
            }
            const long long dbase = (long long)b * a.cpo * DHW + z * HW + (long long)y * a.W + 8 * xb;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int co = (ng * NT + nt) * 16 + r;
                Bv[nt] = *reinterpret_cast<const uint4 *>(a.dT + dbase + (long long)co * DHW);
            }
        }
        // x shifted by -1 (kx = 0) and +1 (kx = 2): element j of the fragment
        // is a[x + j + kx - 1]; the low half of a word is the even element
        if (bias)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const uint4 v = Bv[nt];
                bsum[nt] += (bf16_val((u16)v.x) + bf16_val((u16)(v.x >> 16))) + (bf16_val((u16)v.y) + bf16_val((u16)(v.y >> 16))) +
                            (bf16_val((u16)v.z) + bf16_val((u16)(v.z >> 16))) + (bf16_val((u16)v.w) + bf16_val((u16)(v.w >> 16)));
            }
        const uint4 A0 = make_uint4((L.w >> 16) | (M.x << 16), (M.x >> 16) | (M.y << 16),
                                    (M.y >> 16) | (M.z << 16), (M.z >> 16) | (M.w << 16));
        const uint4 A2 = make_uint4((M.x >> 16) | (M.y << 16), (M.y >> 16) | (M.z << 16),
                                    (M.z >> 16) | (M.w << 16), (M.w >> 16) | (R.x << 16));
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const bf16x8 bb = __builtin_bit_cast(bf16x8, Bv[nt]);
            if constexpr (ONE) {
                acc[0][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, M), bb, acc[0][nt], 0, 0, 0);
            } else {
                acc[0][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A0), bb, acc[0][nt], 0, 0, 0);
                acc[1][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, M), bb, acc[1][nt], 0, 0, 0);
                acc[2][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A2), bb, acc[2][nt], 0, 0, 0);
            }
        }
    }
    if (wave > 0)
#pragma unroll
        for (int kx = 0; kx < NKX; ++kx)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) red[wave - 1][kx * NT + nt][lane] = acc[kx][nt];
    __syncthreads();
    if (bias) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) atomicAdd(&sb[nt * 16 + r], bsum[nt]);
        __syncthreads();   // uniform: bias depends on the workgroup only
        if (threadIdx.x < NT * 16) {
            const int co = ng * NT * 16 + threadIdx.x;
            if (co < a.cout && sb[threadIdx.x] != 0.f) atomicAdd(&a.gb[co], sb[threadIdx.x]);
        }
    }
    if (wave != 0) return;
#pragma unroll
    for (int kx = 0; kx < NKX; ++kx)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            f32x4 s = acc[kx][nt];
            for (int w = 0; w < SBS / 64 - 1; ++w) s += red[w][kx * NT + nt][lane];
            const int t = ONE ? 0 : kx + 3 * p;
            const int co = (ng * NT + nt) * 16 + r;
            for (int i = 0; i < 4; ++i) {
                const int c = mt * 16 + 4 * g + i;
                if (c < a.cin && co < a.cout && s[i] != 0.f)
                    atomicAdd(&a.gw[((long long)t * a.cin + c) * a.cout + co], s[i]);
            }
        }
}

// ------------------------------------------------------------------- loss
// per-sample field energies of prediction and target, sum_{c < 6} (x std + mean)^2
__global__ void __launch_bounds__(SBS)
k_sp_energy(long long n, long long per, const float *__restrict__ p, const float *__restrict__ y, SpNorm nm,
            double *__restrict__ U) {
    __shared__ double sp_[SBS], st_[SBS];
    const long long v = (long long)blockIdx.x * SBS + threadIdx.x;
    double up = 0.0, ut = 0.0;
    if (v < n)
        for (int c = 0; c < 6; ++c) {
            const double ep = (double)p[v * 10 + c] * nm.stdv[c] + nm.mean[c];
            const double et = (double)y[v * 10 + c] * nm.stdv[c] + nm.mean[c];
            up += ep * ep;
            ut += et * et;
        }
    const long long v0 = (long long)blockIdx.x * SBS;
    long long v1 = v0 + SBS - 1;
    if (v1 >= n) v1 = n - 1;
    if (v0 / per != v1 / per) {   // block spans samples
        if (v < n) {
            atomicAdd(&U[2 * (v / per)], up);
            atomicAdd(&U[2 * (v / per) + 1], ut);
        }
        return;
    }
    sp_[threadIdx.x] = up;
    st_[threadIdx.x] = ut;
    __syncthreads();
    for (int h = SBS / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            sp_[threadIdx.x] += sp_[threadIdx.x + h];
            st_[threadIdx.x] += st_[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(&U[2 * (v0 / per)], sp_[0]);
        atomicAdd(&U[2 * (v0 / per) + 1], st_[0]);
    }
}

// Huber loss and the output gradient: dz[v][c] (BF16, 16 channels, c >= 10
// zero) and its channel-major copy; thread 0 also adds the energy term
__global__ void __launch_bounds__(SBS)
k_sp_loss(long long n, long long per, int B, const float *__restrict__ p, const float *__restrict__ y, SpNorm nm,
          const double *__restrict__ U, float delta, float lambda, u16 *__restrict__ dz, u16 *__restrict__ dzT,
          double *__restrict__ loss) {
    __shared__ double sl[SBS];
    const long long v = (long long)blockIdx.x * SBS + threadIdx.x;
    double h = 0.0;
    if (v < n) {
        const long long b = v / per, s = v % per;
        const double ut = U[2 * b + 1], up = U[2 * b];
        const float kb = ut > 0.0 ? (float)(lambda * 2.0 * ((up - ut) / ut) / ut / B) : 0.f;
        const float inv = 1.0f / (float)(n * 10);
        for (int c = 0; c < 16; ++c) {
            float gd = 0.f;
            if (c < 10) {
                const float pv = p[v * 10 + c], d = pv - y[v * 10 + c], ad = fabsf(d);
                h += ad <= delta ? 0.5 * (double)d * d : (double)delta * (ad - 0.5 * (double)delta);
                gd = (ad <= delta ? d : (d > 0.f ? delta : -delta)) * inv;
                if (c < 6) gd += kb * 2.0f * (pv * nm.stdv[c] + nm.mean[c]) * nm.stdv[c];
            }
            const u16 bits = bf16_bits(gd);
            dz[v * 16 + c] = bits;
            dzT[(b * 16 + c) * per + s] = bits;
        }
    }
    sl[threadIdx.x] = h;
    __syncthreads();
    for (int k = SBS / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) sl[threadIdx.x] += sl[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double tot = sl[0] / (double)(n * 10);
        if (blockIdx.x == 0)
            for (int b = 0; b < B; ++b) {
                const double ut = U[2 * b + 1], up = U[2 * b];
                if (ut > 0.0) tot += lambda * ((up - ut) / ut) * ((up - ut) / ut) / B;
            }
        if (tot != 0.0) atomicAdd(loss, tot);
    }
}

// ------------------------------------------------------- packing, inputs
// BF16 weight matrices of one layer from the FP32 parameters W[27][cin][cout]:
// forward Wf[co][k = t cpi + ci] (kpf = 27 cpi rounded up to 32) and data
// gradient Wb[ci][k = t cpo + co] = W[26 - t][ci][co]; zeros in the padding
__global__ void __launch_bounds__(SBS)
k_sp_pack(const float *__restrict__ W, int cin, int cout, int cpi, int cpo, int taps, u16 *__restrict__ Wf,
          u16 *__restrict__ Wb) {
    const int i = blockIdx.x * SBS + threadIdx.x;
    const int kpf = (taps * cpi + 31) / 32 * 32, kpb = (taps * cpo + 31) / 32 * 32;
    if (i < cpo * kpf) {
        const int co = i / kpf, k = i % kpf, t = k / cpi, ci = k % cpi;
        Wf[i] = (k < taps * cpi && ci < cin && co < cout) ? bf16_bits(W[((long long)t * cin + ci) * cout + co])
                                                          : (u16)0;
    }
    if (Wb && i < cpi * kpb) {
        const int ci = i / kpb, k = i % kpb, t = k / cpo, co = k % cpo;
        Wb[i] = (k < taps * cpo && ci < cin && co < cout)
                    ? bf16_bits(W[((long long)(taps - 1 - t) * cin + ci) * cout + co]) : (u16)0;
    }
}

// SwitchNet loss from the logits: mean of BCE(p, y) + lambda (1 - p) e, and
// the logit gradient into column 0 of dz [n][16] (BF16, other columns zero)
// and of its channel-major copy (row stride ldT)
__global__ void __launch_bounds__(SBS)
k_swn_loss(long long n, const float *__restrict__ logit, const float *__restrict__ y, const float *__restrict__ e,
           float lambda, u16 *__restrict__ dz, u16 *__restrict__ dzT, long long ldT, double *__restrict__ loss) {
    __shared__ double sl[SBS];
    const long long v = (long long)blockIdx.x * SBS + threadIdx.x;
    double l = 0.0;
    if (v < n) {
        const float s = logit[v], p = 1.0f / (1.0f + __expf(-s));
        const float sp = s > 0.f ? s + log1pf(__expf(-s)) : log1pf(__expf(s));
        l = (double)(sp - y[v] * s + lambda * (1.0f - p) * e[v]) / (double)n;
        const u16 d = bf16_bits((p - y[v] - lambda * p * (1.0f - p) * e[v]) / (float)n);
        for (int c = 0; c < 16; ++c) {
            dz[v * 16 + c] = c ? (u16)0 : d;
            dzT[c * ldT + v] = c ? (u16)0 : d;
        }
    }
    sl[threadIdx.x] = l;
    __syncthreads();
    for (int k = SBS / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) sl[threadIdx.x] += sl[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0 && sl[0] != 0.0) atomicAdd(loss, sl[0]);
}

// FP32 inputs [n][10] -> BF16 [n][16] (zero padded) and the channel-major copy
__global__ void __launch_bounds__(SBS)
k_sp_input(long long n, long long per, const float *__restrict__ x, u16 *__restrict__ xb, u16 *__restrict__ xT) {
    const long long i = (long long)blockIdx.x * SBS + threadIdx.x;
    if (i >= n * 16) return;
    const long long v = i >> 4;
    const int c = (int)(i & 15);
    const u16 bits = c < 10 ? bf16_bits(x[v * 10 + c]) : (u16)0;
    xb[i] = bits;
    if (xT) xT[((v / per) * 16 + c) * per + v % per] = bits;
}

inline unsigned nblk(long long n) { return (unsigned)((n + SBS - 1) / SBS); }
inline unsigned grid8(long long items) { return (unsigned)((items + 7) / 8 * 8); }

template <int CPIN, int NT, bool BWD, int TAPS = 27>
void conv_go(SpConv a, hipStream_t s) {
    const int segs = (a.W + 15) / 16;
    a.G = a.cols / (16 * NT);
    if constexpr (TAPS == 1) {
        // persistent workgroups per column group, about 1024 in all
        const long long ntiles = ((long long)a.B * a.D * a.H * a.W + 15) / 16;
        long long per = (ntiles + 15) / 16;
        const long long cap = (1024 + a.G - 1) / a.G;
        if (per > cap) per = cap;
        per = (per + 7) / 8 * 8;
        a.ntask = 0;
        k_sp_lin<CPIN, NT, BWD><<<(unsigned)(per * a.G), SBS, 0, s>>>(a);
    } else if constexpr (TAPS == 27 && CPIN >= 32) {
        // eight rows per wave where a row feeds only one or two column tiles
        constexpr int MT = NT <= 2 ? 8 : 4;
        const long long tiles = (long long)a.B * ((a.D + HZ - 1) / HZ) * ((a.H + MT - 1) / MT) * segs;
        a.ntask = (int)(tiles * a.G);
        k_sp_conv_halo<CPIN, MT, NT, BWD><<<grid8(a.ntask), SBS, 0, s>>>(a);
    } else {
        constexpr int MT = 4;
        const long long rows = (long long)a.B * a.D * a.H * segs;
        a.ntask = (int)((rows + MT - 1) / MT * a.G);
        k_sp_conv<CPIN, MT, NT, BWD, TAPS><<<grid8((a.ntask + 3) / 4), SBS, 0, s>>>(a);
    }
}

}  // namespace

// ----------------------------------------------------------------- launchers
int sp_launch_conv(int cpin, int taps, bool bwd, const SpConv &a, hipStream_t s) {
    const int ct = a.cols / 16;
    if (taps == 1) {
        // linear layers take the voxels as one line (B = D = H = 1); four
        // row and up to four column tiles per wave
        if (a.B != 1 || a.D != 1 || a.H != 1) return -1;
        const int nt = ct < 4 ? ct : 4;
        switch (cpin * 100 + nt * 10 + (bwd ? 1 : 0)) {
        case 1640: conv_go<16, 4, false, 1>(a, s); break;
        case 12840: conv_go<128, 4, false, 1>(a, s); break;
        case 25640: conv_go<256, 4, false, 1>(a, s); break;
        case 25641: conv_go<256, 4, true, 1>(a, s); break;
        case 25610: conv_go<256, 1, false, 1>(a, s); break;
        case 1641: conv_go<16, 4, true, 1>(a, s); break;
        default: return -1;
        }
        return 0;
    }
    if (taps != 27) return -1;
    // column tiles per wave: up to 4 on the 16-channel inputs; on the halo
    // path two (with eight rows per wave), which keeps the wave's working set
    // in registers at two waves per SIMD
    const int nt = cpin >= 32 ? (ct < SP_HALO_NT ? ct : SP_HALO_NT) : (ct < 4 ? ct : 4);
    const int key = cpin * 100 + nt * 10 + (bwd ? 1 : 0);
    switch (key) {
    case 1610: conv_go<16, 1, false>(a, s); break;
    case 1620: conv_go<16, 2, false>(a, s); break;
    case 1621: conv_go<16, 2, true>(a, s); break;
    case 3210: conv_go<32, 1, false>(a, s); break;
    case 3211: conv_go<32, 1, true>(a, s); break;
    case 3220: conv_go<32, 2, false>(a, s); break;
    case 3221: conv_go<32, 2, true>(a, s); break;
    case 6420: conv_go<64, 2, false>(a, s); break;
    case 6421: conv_go<64, 2, true>(a, s); break;
    case 12820: conv_go<128, 2, false>(a, s); break;
    case 12821: conv_go<128, 2, true>(a, s); break;
#if SP_HALO_NT >= 4
    case 3240: conv_go<32, 4, false>(a, s); break;
    case 3241: conv_go<32, 4, true>(a, s); break;
    case 6440: conv_go<64, 4, false>(a, s); break;
    case 6441: conv_go<64, 4, true>(a, s); break;
    case 12840: conv_go<128, 4, false>(a, s); break;
    case 12841: conv_go<128, 4, true>(a, s); break;
#endif
    default: return -1;
    }
    return 0;
}

int sp_launch_wgrad(int nt, int taps, const SpWgrad &a, hipStream_t s) {
    const unsigned grid = grid8(a.nitems);
    switch (nt * 100 + taps) {
    case 127: k_sp_wgrad<1, false><<<grid, SBS, 0, s>>>(a); break;
    case 227: k_sp_wgrad<2, false><<<grid, SBS, 0, s>>>(a); break;
    case 427: k_sp_wgrad<4, false><<<grid, SBS, 0, s>>>(a); break;
    case 101: k_sp_wgrad<1, true><<<grid, SBS, 0, s>>>(a); break;
    case 401: k_sp_wgrad<4, true><<<grid, SBS, 0, s>>>(a); break;
    default: return -1;
    }
    return 0;
}

void sp_launch_energy(long long n, long long per, const float *p, const float *y, const SpNorm &nm, double *U,
                      hipStream_t s) {
    k_sp_energy<<<nblk(n), SBS, 0, s>>>(n, per, p, y, nm, U);
}

void sp_launch_loss(long long n, long long per, int B, const float *p, const float *y, const SpNorm &nm,
                    const double *U, float delta, float lambda, unsigned short *dz, unsigned short *dzT,
                    double *loss, hipStream_t s) {
    k_sp_loss<<<nblk(n), SBS, 0, s>>>(n, per, B, p, y, nm, U, delta, lambda, dz, dzT, loss);
}

void sp_launch_pack(const float *W, int cin, int cout, int cpi, int cpo, int taps, unsigned short *Wf,
                    unsigned short *Wb, hipStream_t s) {
    const long long nf = (long long)cpo * ((taps * cpi + 31) / 32 * 32);
    const long long nb = (long long)cpi * ((taps * cpo + 31) / 32 * 32);
    k_sp_pack<<<nblk(nf > nb ? nf : nb), SBS, 0, s>>>(W, cin, cout, cpi, cpo, taps, Wf, Wb);
}

void swn_launch_loss(long long n, const float *logit, const float *y, const float *e, float lambda,
                     unsigned short *dz, unsigned short *dzT, long long ldT, double *loss, hipStream_t s) {
    k_swn_loss<<<nblk(n), SBS, 0, s>>>(n, logit, y, e, lambda, dz, dzT, ldT, loss);
}

void sp_launch_input(long long n, long long per, const float *x, unsigned short *xb, unsigned short *xT,
                     hipStream_t s) {
    k_sp_input<<<nblk(n * 16), SBS, 0, s>>>(n, per, x, xb, xT);
}
