// The learned regime switch on gfx950: a 4-layer 3D CNN (valid 3^3
// convolutions, 32 channels, GELU) with a 1x1x1 head, in BF16 with FP32
// accumulation on the matrix cores, its backward pass and AdamW.
//
// Paper: abstract and Methodology (a neural network picks fluid or kinetic
// treatment per region; Monte Carlo dropout gives its uncertainty; physics
// thresholds are the fallback; it is trained on data the simulation makes,
// with an energy penalty).
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16: rows are 16
// consecutive output voxels along x, columns the 32 output channels (two
// 16-wide halves), and K runs over (tap, input channel), k = tap * CIN + ci,
// tap = kx + 3 ky + 9 kz, padded to a multiple of 32.  Lane l holds A[l%16]
// [8 (l/16) .. +8] (8 input channels of one voxel: one 16-byte load, channels
// last), B[8 (l/16) .. +8][l%16] (16 bytes of the weight matrix stored
// co-major), and D[4 (l/16) + i][l%16], i < 4.  The weight matrix of a layer
// sits in LDS.  The forward passes order their K steps by (kz, ky) so that a
// loaded input row serves several steps (see k_conv_fwd_first and
// k_conv_fwd_rows); the GELU of their outputs takes a rational erf.
// The data gradient is the same GEMM over input voxels with K = (tap, co) and
// the transposed weights; the weight gradient is a GEMM with K over voxels on
// v_mfma_f32_32x32x16_bf16 (rows (tap, ci), columns co).
//
// Activations are stored channels last in BF16 (round to nearest even from
// FP32); pre-activations in FP32 when the backward pass needs them.
#include "hk_internal.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int NC = 32;
constexpr int CBS = 256;                  // 4 waves

__device__ inline unsigned short bf16_bits(float x) {
    // round to nearest even (finite inputs)
    const unsigned u = __float_as_uint(x);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_val(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

// GELU of the forward passes, with erfc(u) (u = |z| / sqrt 2) from the
// rational approximation of Abramowitz & Stegun 7.1.26 (Hastings): absolute
// error at most 1.5e-7, far below the BF16 rounding of the activations it
// feeds, in a dozen instructions instead of a full erff.
__device__ inline float gelu_fwd(float z) {
    const float u = fabsf(z) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, u, 1.0f));
    float p = fmaf(1.061405429f, t, -1.453152027f);
    p = fmaf(p, t, 1.421413741f);
    p = fmaf(p, t, -0.284496736f);
    p = fmaf(p, t, 0.254829592f);
    const float q = p * t * __expf(-u * u);
    return 0.5f * z * (z >= 0.f ? 2.0f - q : q);
}
__device__ inline float gelu_d(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * __expf(-0.5f * z * z) * 0.3989422804014327f;
}

struct Dims { int B, D, H, W; };   // voxel grid of an activation

__device__ inline long long vidx(const Dims &d, int b, int z, int y, int x) {
    return (((long long)b * d.D + z) * d.H + y) * d.W + x;
}

// ------------------------------------------------------------------ forward
// out dims = in dims - 2.  Wf: [NC][kpad] BF16 (co-major), kpad = 27 CIN
// rounded up to 32 with zeros, k = tap CIN + ci, tap = kx + 3 ky + 9 kz.  A
// workgroup of 8 waves shares the weight matrix in LDS and loops over groups
// of output rows, a wave per group.
constexpr int FBS = 512;
// xwin (may be null): output x indices outside [xwin[0], xwin[1] + 6] are
// skipped (the switch's plasma window; see k_cnn_window).
// raw buffer resource of the gfx9 family: byte range BUF_RECORDS from the
// base (offsets at or past it read zeros), dword 3 as for untyped dword data
constexpr int BUF_RECORDS = 0x7ffffff0;
constexpr int BUF_DWORD3 = 0x00020000;
constexpr unsigned BUF_OUT = 0x80000000u;

// The first layer (8 input channels).  K step (ky, kz) holds the three kx taps
// of 8 channels in the lane groups g = 0, 1, 2 (k = 8 kx + ci) and zeros in
// g = 3, so that lane (r, g) loads the 8 channels of one voxel, x0 + r + g; a
// wave owns RY output rows of 16 voxels and, for each kz, loads the RY + 2
// input rows once (raw buffer loads, as below) and runs 3 x RY x 2 MFMAs.
// Nine K steps, a quarter of them zeros, against seven dense ones: a load per
// input row and kz instead of a gather per K step.
template <int RY>
__global__ void __launch_bounds__(FBS)
k_conv_fwd_first(Dims in, const unsigned short *__restrict__ act, const unsigned short *__restrict__ Wf,
                 const float *__restrict__ bias, float *__restrict__ zout, unsigned short *__restrict__ aout,
                 const int *__restrict__ xwin) {
    // LDS rows of the weights padded to KS shorts (KS / 2 = 4 mod 64 dwords)
    constexpr int CIN = 8, KPAD = 224, KS = KPAD + 2 * ((4 - (KPAD / 2) % 64 + 64) % 64);
    static_assert((KS / 2) % 64 == 4, "padded LDS row");
    __shared__ __attribute__((aligned(16))) unsigned short sW[NC * KS];
    for (int e = threadIdx.x; e < NC * KPAD / 8; e += FBS) {
        const int row = e / (KPAD / 8), col = e - row * (KPAD / 8);
        reinterpret_cast<uint4 *>(sW)[row * (KS / 8) + col] = reinterpret_cast<const uint4 *>(Wf)[e];
    }
    __syncthreads();
    const Dims out{in.B, in.D - 2, in.H - 2, in.W - 2};
    int seg0 = 0, segs = (out.W + 15) / 16;
    if (xwin) {
        const int lo = xwin[0], hi = min(xwin[1] + 6, out.W - 1);
        seg0 = lo / 16;
        segs = xwin[1] >= lo && hi >= lo ? hi / 16 - seg0 + 1 : 0;
    }
    const int ygroups = (out.H + RY - 1) / RY;
    const long long nrows = (long long)out.B * out.D * ygroups * segs;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const float b0 = bias[r], b1 = bias[16 + r];
    const unsigned short *wr0 = sW + r * KS + 8 * g, *wr1 = sW + (16 + r) * KS + 8 * g;
    for (long long row = (long long)blockIdx.x * (FBS / 64) + wave; row < nrows;
         row += (long long)gridDim.x * (FBS / 64)) {
        const int seg = seg0 + (int)(row % segs);
        long long q = row / segs;
        const int yg = (int)(q % ygroups); q /= ygroups;
        const int z = (int)(q % out.D);
        const int b = (int)(q / out.D);
        const int x0 = seg * 16, y0 = yg * RY;
        const bool xin = g < 3 && x0 + r + g < in.W;
        const unsigned long long ba = (unsigned long long)(act + vidx(in, b, z, y0, x0) * CIN);
        const unsigned long long bu = ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(ba >> 32)) << 32) |
                                      (unsigned)__builtin_amdgcn_readfirstlane((unsigned)ba);
        const __amdgpu_buffer_rsrc_t rsrc =
            __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void *>(bu), (short)0, BUF_RECORDS, BUF_DWORD3);
        const unsigned lane_off = 2u * (unsigned)((r + g) * CIN);
        const unsigned rs = 2u * (unsigned)(in.W * CIN), ps = 2u * (unsigned)(in.H * in.W * CIN);
        f32x4 acc[RY][2];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            acc[j][0] = f32x4{0, 0, 0, 0};
            acc[j][1] = f32x4{0, 0, 0, 0};
        }
#pragma unroll 1
        for (int kz = 0; kz < 3; ++kz) {
            uint4 av[RY + 2];
#pragma unroll
            for (int j = 0; j < RY + 2; ++j) {
                const unsigned off = xin && y0 + j < in.H ? lane_off + (unsigned)kz * ps + (unsigned)j * rs : BUF_OUT;
                av[j] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)off, 0, 0));
            }
#pragma unroll
            for (int ky = 0; ky < 3; ++ky) {
                // lane group g takes tap (g, ky, kz); g = 3 reads the next tap's
                // weights (within the zero-padded row), against zeros of A
                const int k = (3 * ky + 9 * kz) * CIN;
                const bf16x8 w0 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(wr0 + k));
                const bf16x8 w1 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(wr1 + k));
#pragma unroll
                for (int j = 0; j < RY; ++j) {
                    const bf16x8 a = __builtin_bit_cast(bf16x8, av[j + ky]);
                    acc[j][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, w0, acc[j][0], 0, 0, 0);
                    acc[j][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, w1, acc[j][1], 0, 0, 0);
                }
            }
        }
        const long long vb = vidx(out, b, z, y0, x0) * NC;
        const int ors = out.W * NC;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int y = y0 + j;
            if (y >= out.H) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int xo = 4 * g + i;
                if (x0 + xo >= out.W) continue;
                const long long v = vb + j * ors + xo * NC;
                const float z0 = acc[j][0][i] + b0, z1 = acc[j][1][i] + b1;
                if (zout) { zout[v + r] = z0; zout[v + 16 + r] = z1; }
                aout[v + r] = bf16_bits(gelu_fwd(z0));
                aout[v + 16 + r] = bf16_bits(gelu_fwd(z1));
            }
        }
    }
}

// The 32-channel layers with RY output rows per wave: the wave owns output
// voxels (z, y0 .. y0 + RY - 1, x0 .. x0 + 13).  For each kz it loads the A
// fragments (16 voxels x0 .. x0 + 15 of the RY + 2 input rows y0 .. y0 + RY +
// 1) once; the taps kx = 1, 2 take them shifted down one lane within each
// 16-lane row (DPP row_shl:1), so that lane r holds voxel x0 + r + kx, and the
// two lanes whose voxel would lie beyond x0 + 15 give outputs that are not
// stored: 14 of every 16 MFMA rows are kept, for a third of the loads.  The B
// fragments of the three ky taps come from LDS once per (kz, kx); output row j
// takes input row j + ky.
constexpr int ROW_TW = 14;
__device__ inline uint4 shift_down_lane(uint4 a) {
    // lane r of each 16-lane row takes lane r + 1's value (lane 15 keeps its own)
    a.x = __builtin_amdgcn_update_dpp(a.x, a.x, 0x101, 0xf, 0xf, false);
    a.y = __builtin_amdgcn_update_dpp(a.y, a.y, 0x101, 0xf, 0xf, false);
    a.z = __builtin_amdgcn_update_dpp(a.z, a.z, 0x101, 0xf, 0xf, false);
    a.w = __builtin_amdgcn_update_dpp(a.w, a.w, 0x101, 0xf, 0xf, false);
    return a;
}
template <int RY>
__global__ void __launch_bounds__(FBS)
k_conv_fwd_rows(Dims in, const unsigned short *__restrict__ act, const unsigned short *__restrict__ Wf,
                const float *__restrict__ bias, float *__restrict__ zout, unsigned short *__restrict__ aout,
                const int *__restrict__ xwin) {
    // LDS rows of the weights padded from 432 to 452 dwords: the 16 output
    // channels of one fragment read start 4 banks apart (452 = 4 mod 64), so
    // a 16-lane group covers the 64 banks once
    constexpr int CIN = NC, KPAD = 27 * NC, KS = KPAD + 40;
    __shared__ __attribute__((aligned(16))) unsigned short sW[NC * KS];
    for (int e = threadIdx.x; e < NC * KPAD / 8; e += FBS) {
        const int row = e / (KPAD / 8), col = e - row * (KPAD / 8);
        reinterpret_cast<uint4 *>(sW)[row * (KS / 8) + col] = reinterpret_cast<const uint4 *>(Wf)[e];
    }
    __syncthreads();
    const Dims out{in.B, in.D - 2, in.H - 2, in.W - 2};
    int seg0 = 0, segs = (out.W + ROW_TW - 1) / ROW_TW;
    if (xwin) {
        const int lo = xwin[0], hi = min(xwin[1] + 6, out.W - 1);
        seg0 = lo / ROW_TW;
        segs = xwin[1] >= lo && hi >= lo ? hi / ROW_TW - seg0 + 1 : 0;
    }
    const int ygroups = (out.H + RY - 1) / RY;
    const long long nrows = (long long)out.B * out.D * ygroups * segs;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const float b0 = bias[r], b1 = bias[16 + r];
    for (long long row = (long long)blockIdx.x * (FBS / 64) + wave; row < nrows;
         row += (long long)gridDim.x * (FBS / 64)) {
        const int seg = seg0 + (int)(row % segs);
        long long q = row / segs;
        const int yg = (int)(q % ygroups); q /= ygroups;
        const int z = (int)(q % out.D);
        const int b = (int)(q / out.D);
        const int x0 = seg * ROW_TW, y0 = yg * RY;
        const bool xin = x0 + r < in.W;
        // the row group's input as a raw buffer from its first voxel: lanes
        // address it with 32-bit byte offsets, and the rows beyond the grid
        // and the lanes beyond x take an offset past the buffer's end, for
        // which the load returns zeros without touching memory
        const unsigned long long ba = (unsigned long long)(act + vidx(in, b, z, y0, x0) * CIN);
        const unsigned long long bu = ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(ba >> 32)) << 32) |
                                      (unsigned)__builtin_amdgcn_readfirstlane((unsigned)ba);
        const __amdgpu_buffer_rsrc_t rsrc =
            __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void *>(bu), (short)0, BUF_RECORDS, BUF_DWORD3);
        const unsigned lane_off = 2u * (unsigned)(r * CIN + 8 * g);
        const unsigned rs = 2u * (unsigned)(in.W * CIN), ps = 2u * (unsigned)(in.H * in.W * CIN);
        f32x4 acc[RY][2];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            acc[j][0] = f32x4{0, 0, 0, 0};
            acc[j][1] = f32x4{0, 0, 0, 0};
        }
        const unsigned short *wr0 = sW + r * KS + 8 * g, *wr1 = sW + (16 + r) * KS + 8 * g;
#pragma unroll 1
        for (int kz = 0; kz < 3; ++kz) {
            uint4 av[RY + 2];
#pragma unroll
            for (int j = 0; j < RY + 2; ++j) {
                const unsigned off = xin && y0 + j < in.H ? lane_off + (unsigned)kz * ps + (unsigned)j * rs : BUF_OUT;
                av[j] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)off, 0, 0));
            }
            // the B fragments of tap (kx, ky) are read one tap ahead of their MFMAs
            uint4 wn0 = *reinterpret_cast<const uint4 *>(wr0 + 9 * kz * CIN);
            uint4 wn1 = *reinterpret_cast<const uint4 *>(wr1 + 9 * kz * CIN);
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                if (kx > 0) {
#pragma unroll
                    for (int j = 0; j < RY + 2; ++j) av[j] = shift_down_lane(av[j]);
                }
#pragma unroll
                for (int ky = 0; ky < 3; ++ky) {
                    const bf16x8 w0 = __builtin_bit_cast(bf16x8, wn0);
                    const bf16x8 w1 = __builtin_bit_cast(bf16x8, wn1);
                    if (kx < 2 || ky < 2) {
                        const int nkx = ky < 2 ? kx : kx + 1, nky = ky < 2 ? ky + 1 : 0;
                        const int k = (nkx + 3 * nky + 9 * kz) * CIN;
                        wn0 = *reinterpret_cast<const uint4 *>(wr0 + k);
                        wn1 = *reinterpret_cast<const uint4 *>(wr1 + k);
                    }
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        const bf16x8 a = __builtin_bit_cast(bf16x8, av[j + ky]);
                        acc[j][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, w0, acc[j][0], 0, 0, 0);
                        acc[j][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, w1, acc[j][1], 0, 0, 0);
                    }
                }
            }
        }
        const long long vb = vidx(out, b, z, y0, x0) * NC;
        const int ors = out.W * NC;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int y = y0 + j;
            if (y >= out.H) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int xo = 4 * g + i, x = x0 + xo;
                if (xo >= ROW_TW || x >= out.W) continue;
                const long long v = vb + j * ors + xo * NC;
                const float z0 = acc[j][0][i] + b0, z1 = acc[j][1][i] + b1;
                if (zout) { zout[v + r] = z0; zout[v + 16 + r] = z1; }
                aout[v + r] = bf16_bits(gelu_fwd(z0));
                aout[v + 16 + r] = bf16_bits(gelu_fwd(z1));
            }
        }
    }
}

// ---------------------------------------------------------- data gradient
// din[u][ci] = sum_{t, co} dz[u - off(t)][co] W[t][ci][co] over the input
// voxels u (dims `in`; dz lives on in - 2), then times GELU'(z_in[u][ci]) and
// stored in BF16: the pre-activation gradient of the layer below.  Wb:
// [CIN][864] BF16 with k = t * 32 + co.  CIN = 32 here (layer 1's input needs
// no gradient).
__global__ void __launch_bounds__(CBS)
k_conv_bwd_data(Dims in, const unsigned short *__restrict__ dz, const unsigned short *__restrict__ Wb,
                const float *__restrict__ zin, unsigned short *__restrict__ dzin) {
    constexpr int KPAD = 27 * NC;
    __shared__ __attribute__((aligned(16))) unsigned short sW[NC * KPAD];
    for (int e = threadIdx.x; e < NC * KPAD / 8; e += CBS)
        reinterpret_cast<uint4 *>(sW)[e] = reinterpret_cast<const uint4 *>(Wb)[e];
    __syncthreads();
    const Dims out{in.B, in.D - 2, in.H - 2, in.W - 2};
    const int segs = (in.W + 15) / 16;
    const long long nrows = (long long)in.B * in.D * in.H * segs;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    for (long long row = (long long)blockIdx.x * 4 + wave; row < nrows; row += (long long)gridDim.x * 4) {
        const int seg = (int)(row % segs);
        long long q = row / segs;
        const int y = (int)(q % in.H); q /= in.H;
        const int z = (int)(q % in.D);
        const int b = (int)(q / in.D);
        const int x0 = seg * 16;
        const int u = x0 + r;
        f32x4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
        for (int kb = 0; kb < KPAD; kb += 32) {
            const int k = kb + 8 * g;
            const int t = k / NC, co = k % NC;
            const int kx = t % 3, ky = (t / 3) % 3, kz = t / 9;
            const int ox = u - kx, oy = y - ky, oz = z - kz;
            uint4 raw = make_uint4(0, 0, 0, 0);
            if (u < in.W && ox >= 0 && ox < out.W && oy >= 0 && oy < out.H && oz >= 0 && oz < out.D)
                raw = *reinterpret_cast<const uint4 *>(dz + vidx(out, b, oz, oy, ox) * NC + co);
            const bf16x8 a = __builtin_bit_cast(bf16x8, raw);
            const bf16x8 w0 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(sW + r * KPAD + k));
            const bf16x8 w1 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(sW + (16 + r) * KPAD + k));
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, w0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, w1, acc1, 0, 0, 0);
        }
        for (int i = 0; i < 4; ++i) {
            const int x = x0 + 4 * g + i;
            if (x >= in.W) continue;
            const long long v = vidx(in, b, z, y, x);
            dzin[v * NC + r] = bf16_bits(acc0[i] * gelu_d(zin[v * NC + r]));
            dzin[v * NC + 16 + r] = bf16_bits(acc1[i] * gelu_d(zin[v * NC + 16 + r]));
        }
    }
}

// -------------------------------------------------------- weight gradient
// gW[t][ci][co] += sum_v act[v + off(t)][ci] dz[v][co], over the output
// voxels v (dims in - 2).  One wave per (tap, chunk of 16-voxel x-segments);
// MFMA 32x32x16: A[m = ci][k = voxel], B[k = voxel][n = co]; lane l holds
// A[l%32][8 (l/32) .. +8], B[8 (l/32) .. +8][l%32], D[8 (i/4) + 4 (l/32) + i%4][l%32].
template <int CIN>
__global__ void __launch_bounds__(CBS)
k_conv_bwd_weight(Dims in, const unsigned short *__restrict__ act, const unsigned short *__restrict__ dz,
                  float *__restrict__ gW, int seg_per_wave) {
    const Dims out{in.B, in.D - 2, in.H - 2, in.W - 2};
    const int segs = (out.W + 15) / 16;
    const long long nrows = (long long)out.B * out.D * out.H * segs;
    const int lane = threadIdx.x & 63;
    const long long wid = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int t = (int)(wid % 27);
    const long long chunk = wid / 27;
    const int kx = t % 3, ky = (t / 3) % 3, kz = t / 9;
    const int m = lane & 31, h = lane >> 5;
    f32x16 acc = {};
    const long long r0 = chunk * seg_per_wave;
    for (long long row = r0; row < r0 + seg_per_wave && row < nrows; ++row) {
        const int seg = (int)(row % segs);
        long long q = row / segs;
        const int y = (int)(q % out.H); q /= out.H;
        const int z = (int)(q % out.D);
        const int b = (int)(q / out.D);
        bf16x8 a, bb;
        for (int i = 0; i < 8; ++i) {
            const int x = seg * 16 + 8 * h + i;
            unsigned short av = 0, dv = 0;
            if (x < out.W) {
                if (m < CIN) av = act[vidx(in, b, z + kz, y + ky, x + kx) * CIN + m];
                dv = dz[vidx(out, b, z, y, x) * NC + m];
            }
            a[i] = __builtin_bit_cast(__bf16, av);
            bb[i] = __builtin_bit_cast(__bf16, dv);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc, 0, 0, 0);
    }
    if (r0 >= nrows) return;
    for (int i = 0; i < 16; ++i) {
        const int ci = 8 * (i / 4) + 4 * h + (i % 4), co = m;
        if (ci < CIN && acc[i] != 0.f) atomicAdd(&gW[((long long)t * CIN + ci) * NC + co], acc[i]);
    }
}

// bias gradient: gb[co] += sum_v dz[v][co]
__global__ void __launch_bounds__(CBS)
k_bias_grad(long long n, const unsigned short *__restrict__ dz, float *__restrict__ gb) {
    __shared__ float s[NC];
    if (threadIdx.x < NC) s[threadIdx.x] = 0.f;
    __syncthreads();
    const int co = threadIdx.x & 31;
    float acc = 0.f;
    for (long long v = (long long)blockIdx.x * (CBS / 32) + threadIdx.x / 32; v < n;
         v += (long long)gridDim.x * (CBS / 32))
        acc += bf16_val(dz[v * NC + co]);
    atomicAdd(&s[co], acc);
    __syncthreads();
    if (threadIdx.x < NC && s[threadIdx.x] != 0.f) atomicAdd(&gb[threadIdx.x], s[threadIdx.x]);
}

// ------------------------------------------------------------------- head
// dropout keep factors of channel c: byte c of Philox draws (tag TAG_DROP,
// draws 2s and 2s + 1) >= 26 keeps it, scaled by 256/230
__device__ inline void drop_mask(uint64_t seed, uint64_t id, uint32_t step, int sample, float m[NC]) {
    for (int hh = 0; hh < 2; ++hh) {
        uint32_t r[4];
        draw4(seed, id, step, TAG_DROP, (uint32_t)(2 * sample + hh), r);
        for (int c = 0; c < 16; ++c) {
            const uint32_t byte = (r[c / 4] >> (8 * (c % 4))) & 0xffu;
            m[16 * hh + c] = byte >= 26u ? 256.0f / 230.0f : 0.0f;
        }
    }
}

// logits (optionally with the training dropout mask of (id = v, step))
__global__ void __launch_bounds__(CBS)
k_head(long long n, const unsigned short *__restrict__ a4, const unsigned short *__restrict__ wh,
       const float *__restrict__ bh, int use_mask, uint64_t seed, uint32_t step, float *__restrict__ logit) {
    const long long v = (long long)blockIdx.x * CBS + threadIdx.x;
    if (v >= n) return;
    float m[NC];
    if (use_mask) drop_mask(seed, (uint64_t)v, step, 0, m);
    float s = bh[0];
    for (int c = 0; c < NC; ++c) s += bf16_val(wh[c]) * bf16_val(a4[v * NC + c]) * (use_mask ? m[c] : 1.0f);
    logit[v] = s;
}

// loss, head gradient and the pre-activation gradient of layer 4 (BF16)
__global__ void __launch_bounds__(CBS)
k_head_bwd(long long n, const unsigned short *__restrict__ a4, const float *__restrict__ z4,
           const unsigned short *__restrict__ wh, const float *__restrict__ bh, int use_mask, uint64_t seed,
           uint32_t step, const float *__restrict__ y, const float *__restrict__ e, float lambda,
           unsigned short *__restrict__ dz4, float *__restrict__ gwh, double *__restrict__ loss) {
    __shared__ float sg[NC + 1];
    __shared__ double sl;
    if (threadIdx.x <= NC) sg[threadIdx.x] = 0.f;
    if (threadIdx.x == 0) sl = 0.0;
    __syncthreads();
    const long long v = (long long)blockIdx.x * CBS + threadIdx.x;
    if (v < n) {
        float m[NC];
        if (use_mask) drop_mask(seed, (uint64_t)v, step, 0, m);
        float s = bh[0];
        for (int c = 0; c < NC; ++c) s += bf16_val(wh[c]) * bf16_val(a4[v * NC + c]) * (use_mask ? m[c] : 1.0f);
        const float p = 1.0f / (1.0f + __expf(-s));
        const float sp = s > 0.f ? s + log1pf(__expf(-s)) : log1pf(__expf(s));
        atomicAdd(&sl, (double)(sp - y[v] * s + lambda * (1.0f - p) * e[v]) / (double)n);
        const float dl = (p - y[v] - lambda * p * (1.0f - p) * e[v]) / (float)n;
        for (int c = 0; c < NC; ++c) {
            const float mc = use_mask ? m[c] : 1.0f;
            atomicAdd(&sg[c], dl * bf16_val(a4[v * NC + c]) * mc);
            dz4[v * NC + c] = bf16_bits(dl * bf16_val(wh[c]) * mc * gelu_d(z4[v * NC + c]));
        }
        atomicAdd(&sg[NC], dl);
    }
    __syncthreads();
    if (threadIdx.x <= NC && sg[threadIdx.x] != 0.f) atomicAdd(&gwh[threadIdx.x], sg[threadIdx.x]);
    if (threadIdx.x == 0 && sl != 0.0) atomicAdd(loss, sl);
}

// AdamW on the FP32 master parameters (decoupled weight decay)
__global__ void __launch_bounds__(CBS)
k_adamw(int n, float *__restrict__ p, const float *__restrict__ gr, float *__restrict__ m,
        float *__restrict__ v, float lr, float b1, float b2, float eps, float wd, float c1, float c2) {
    const int i = blockIdx.x * CBS + threadIdx.x;
    if (i >= n) return;
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g, vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1 / (sqrtf(vi / c2) + eps) + wd * p[i]);
}

// BF16 copies of the weights: forward (co-major, k = t CIN + ci, padded) and
// data-gradient (ci-major, k = t 32 + co) layouts, and the head
__global__ void __launch_bounds__(CBS)
k_pack(const float *__restrict__ p, int cin, long long woff, int kpad, unsigned short *__restrict__ Wf,
       unsigned short *__restrict__ Wb) {
    const int i = blockIdx.x * CBS + threadIdx.x;
    if (i >= NC * kpad) return;
    const int co = i / kpad, k = i % kpad;
    const int K = 27 * cin;
    Wf[i] = k < K ? bf16_bits(p[woff + (long long)k * NC + co]) : (unsigned short)0;
    if (Wb && i < cin * 27 * NC) {
        const int ci = i / (27 * NC), kk = i % (27 * NC);
        const int t = kk / NC, c2 = kk % NC;
        Wb[i] = bf16_bits(p[woff + ((long long)t * cin + ci) * NC + c2]);
    }
}

__global__ void k_pack_head(const float *__restrict__ p, long long off, unsigned short *__restrict__ wh) {
    if (threadIdx.x < NC) wh[threadIdx.x] = bf16_bits(p[off + threadIdx.x]);
}

// FP32 (normalized) inputs -> BF16
__global__ void __launch_bounds__(CBS)
k_to_bf16(long long n, const float *__restrict__ x, unsigned short *__restrict__ o) {
    const long long i = (long long)blockIdx.x * CBS + threadIdx.x;
    if (i < n) o[i] = bf16_bits(x[i]);
}

// ------------------------------------------------------------- the switch
// Node inputs of the canonical node grid into the padded BF16 grid
// [nz + 8][ny + 8][NX + 8][8] (halo 4: wrap in y, z and periodic x; the wall
// node repeated in open x), normalized with the frozen statistics.
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

struct Norm { float mean[8], inv_std[8]; };

__global__ void __launch_bounds__(CBS)
k_cnn_inputs(GridP g, const real *__restrict__ Ex, const real *__restrict__ Ey, const real *__restrict__ Ez,
             const real *__restrict__ Bx, const real *__restrict__ By, const real *__restrict__ Bz,
             const real *__restrict__ mom, Norm nm, unsigned short *__restrict__ x, const int *__restrict__ xwin) {
    const int per = g.bcx == HK_BC_PERIODIC;
    const int NX = per ? g.nx : g.nx + 1;
    const int W = NX + 8, H = g.ny + 8, D = g.nz + 8;
    const long long n = (long long)W * H * D;
    const long long v = (long long)blockIdx.x * CBS + threadIdx.x;
    if (v >= n) return;
    const unsigned uv = (unsigned)v, ur = uv / (unsigned)W;
    const int i = (int)(uv - ur * (unsigned)W), j = (int)(ur % (unsigned)H), k = (int)(ur / (unsigned)H);
    // padded x indices the windowed layers read: nodes xwin[0] - 4 .. xwin[1] + 4
    if (xwin && (xwin[1] < xwin[0] || i < xwin[0] || i > xwin[1] + 8)) return;
    int ii = i - 4;
    if (per) ii = wrapi(ii, g.nx);
    else ii = ii < 0 ? 0 : (ii > NX - 1 ? NX - 1 : ii);
    const int jj = wrapi(j - 4, g.ny), kk = wrapi(k - 4, g.nz);
    const long long c = gidx(g, ii, jj, kk);
    const double dv = (double)g.dx * g.dy * g.dz;
    float f[8];
    f[0] = node_field(g, Ex, ii, jj, kk, 1, 0, 0);
    f[1] = node_field(g, Ey, ii, jj, kk, 0, 1, 0);
    f[2] = node_field(g, Ez, ii, jj, kk, 0, 0, 1);
    f[3] = node_field(g, Bx, ii, jj, kk, 0, 1, 1);
    f[4] = node_field(g, By, ii, jj, kk, 1, 0, 1);
    f[5] = node_field(g, Bz, ii, jj, kk, 1, 1, 0);
    const float N = mom[c], U2 = mom[5 * g.nn + c];
    f[6] = (float)(N / dv);
    f[7] = N > 0.f ? sqrtf(U2 / N) : 0.f;
    for (int q = 0; q < 8; ++q) x[v * 8 + q] = bf16_bits((f[q] - nm.mean[q]) * nm.inv_std[q]);
}

// Raw node inputs (8 channels) and the conversion energy per node of the
// canonical node grid [nz][ny][NX]: e = (sum w |u|^2 - |sum w u|^2 / sum w) / 2,
// the thermal energy (m_e c^2, small-u limit) a cold fluid would not carry.
__global__ void __launch_bounds__(CBS)
k_node_raw(GridP g, const real *__restrict__ Ex, const real *__restrict__ Ey, const real *__restrict__ Ez,
           const real *__restrict__ Bx, const real *__restrict__ By, const real *__restrict__ Bz,
           const real *__restrict__ mom, float *__restrict__ out) {
    const int NX = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
    const long long n = (long long)NX * g.ny * g.nz;
    const long long v = (long long)blockIdx.x * CBS + threadIdx.x;
    if (v >= n) return;
    // node counts stay below 2^31: 32-bit index arithmetic
    const unsigned uv = (unsigned)v, ur = uv / (unsigned)NX;
    const int i = (int)(uv - ur * (unsigned)NX), j = (int)(ur % (unsigned)g.ny), k = (int)(ur / (unsigned)g.ny);
    const long long c = gidx(g, i, j, k);
    const double dv = (double)g.dx * g.dy * g.dz;
    float *o = out + 9 * v;
    o[0] = node_field(g, Ex, i, j, k, 1, 0, 0);
    o[1] = node_field(g, Ey, i, j, k, 0, 1, 0);
    o[2] = node_field(g, Ez, i, j, k, 0, 0, 1);
    o[3] = node_field(g, Bx, i, j, k, 0, 1, 1);
    o[4] = node_field(g, By, i, j, k, 1, 0, 1);
    o[5] = node_field(g, Bz, i, j, k, 1, 1, 0);
    const double N = mom[c], U2 = mom[5 * g.nn + c];
    const double px = mom[2 * g.nn + c], py = mom[3 * g.nn + c], pz = mom[4 * g.nn + c];
    o[6] = (float)(N / dv);
    o[7] = N > 0.0 ? (float)sqrt(U2 / N) : 0.f;
    o[8] = N > 0.0 ? (float)fmax(0.0, 0.5 * (U2 - (px * px + py * py + pz * pz) / N)) : 0.f;
}

// States of the canonical node grid [nz][ny][NX] for the next-state
// surrogate, 10 channels per node: E and B averaged to the node as above, J
// averaged like E (its components sit where E's do), and the charge density.
__global__ void __launch_bounds__(CBS)
k_node_state(GridP g, const real *__restrict__ Ex, const real *__restrict__ Ey, const real *__restrict__ Ez,
             const real *__restrict__ Bx, const real *__restrict__ By, const real *__restrict__ Bz,
             const real *__restrict__ Jx, const real *__restrict__ Jy, const real *__restrict__ Jz,
             const double *__restrict__ rho, float *__restrict__ out) {
    const int NX = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
    const long long n = (long long)NX * g.ny * g.nz;
    const long long v = (long long)blockIdx.x * CBS + threadIdx.x;
    if (v >= n) return;
    // node counts stay below 2^31: 32-bit index arithmetic
    const unsigned uv = (unsigned)v, ur = uv / (unsigned)NX;
    const int i = (int)(uv - ur * (unsigned)NX), j = (int)(ur % (unsigned)g.ny), k = (int)(ur / (unsigned)g.ny);
    float *o = out + 10 * v;
    o[0] = node_field(g, Ex, i, j, k, 1, 0, 0);
    o[1] = node_field(g, Ey, i, j, k, 0, 1, 0);
    o[2] = node_field(g, Ez, i, j, k, 0, 0, 1);
    o[3] = node_field(g, Bx, i, j, k, 0, 1, 1);
    o[4] = node_field(g, By, i, j, k, 1, 0, 1);
    o[5] = node_field(g, Bz, i, j, k, 1, 1, 0);
    o[6] = node_field(g, Jx, i, j, k, 1, 0, 0);
    o[7] = node_field(g, Jy, i, j, k, 0, 1, 0);
    o[8] = node_field(g, Jz, i, j, k, 0, 0, 1);
    o[9] = (float)rho[gidx(g, i, j, k)];
}

// 16 dropout samples of the head per node: mean p > 0.5 is kinetic unless the
// samples' standard deviation exceeds 0.2 (then the threshold flags stay).
// The threads loop over the nodes of the x window only (outside it the
// threshold decision stays); 32-bit node arithmetic (counts below 2^31).
constexpr int DECIDE_GRID = 4096;
__global__ void __launch_bounds__(CBS)
k_cnn_decide(GridP g, const unsigned short *__restrict__ a4, const unsigned short *__restrict__ wh,
             const float *__restrict__ bh, uint64_t seed, uint32_t eval, uint8_t *__restrict__ hot,
             uint8_t *__restrict__ notcold, int *__restrict__ nfall, float *__restrict__ pmean,
             const int *__restrict__ xwin) {
    const int per = g.bcx == HK_BC_PERIODIC;
    const int NX = per ? g.nx : g.nx + 1;
    int x0 = 0, x1 = NX - 1;
    if (xwin) { x0 = max(xwin[0], 0); x1 = min(xwin[1], NX - 1); }
    const unsigned wx = x1 >= x0 ? (unsigned)(x1 - x0 + 1) : 0u;
    const unsigned nw = wx * (unsigned)g.ny * (unsigned)g.nz;
    const float K = 256.0f / 230.0f, b = bh[0];
    float w[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) w[q] = bf16_val(wh[q]);
    int nf = 0;
    for (unsigned t = blockIdx.x * CBS + threadIdx.x; t < nw; t += gridDim.x * CBS) {
        const unsigned r = t / wx, i = x0 + (t - r * wx);
        const unsigned j = r % (unsigned)g.ny, k = r / (unsigned)g.ny;
        const unsigned v = i + (unsigned)NX * r;
        const long long c = gidx(g, (int)i, (int)j, (int)k);
        // the terms w h of the logit, loaded as 4 x 16 bytes
        float t_[NC];
        const uint4 *src = reinterpret_cast<const uint4 *>(a4 + (size_t)v * NC);
#pragma unroll
        for (int u = 0; u < NC / 8; ++u) {
            const uint4 q4 = src[u];
            const unsigned int wds[4] = {q4.x, q4.y, q4.z, q4.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                t_[8 * u + 2 * e] = w[8 * u + 2 * e] * __uint_as_float(wds[e] << 16);
                t_[8 * u + 2 * e + 1] = w[8 * u + 2 * e + 1] * __uint_as_float(wds[e] & 0xffff0000u);
            }
        }
        // Every dropout sample's logit lies in [b + K neg, b + K pos] (pos and
        // neg the sums of the positive and negative terms): when that whole
        // range, widened by a rounding margin, sits on one side of 0 and its
        // sigmoids span less than 0.38, every sample decides alike and their
        // spread stays under 0.2, so the 16 samples would give this decision;
        // they are drawn only otherwise.
        bool done = false;
        if (!pmean) {
            float pos = 0.f, neg = 0.f;
#pragma unroll
            for (int q = 0; q < NC; ++q) {
                pos += fmaxf(t_[q], 0.f);
                neg += fminf(t_[q], 0.f);
            }
            const float eps = 1e-4f * (fabsf(b) + K * (pos - neg)) + 1e-3f;
            const float lo = b + K * neg - eps, hi = b + K * pos + eps;
            const float span = 1.0f / (1.0f + expf(-hi)) - 1.0f / (1.0f + expf(-lo));
            if (span < 0.38f && (lo > 0.f || hi < 0.f)) {
                hot[c] = lo > 0.f;
                notcold[c] = lo > 0.f;
                done = true;
            }
        }
        if (done) continue;
        // channel q of sample s is kept when byte q of the Philox draws
        // (TAG_DROP; draws 2s, 2s + 1) is 26 or more, and then scaled by K
        float ps[16], mean = 0.f;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            float z = b;
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                uint32_t rr[4];
                draw4(seed, (uint64_t)c, eval, TAG_DROP, (uint32_t)(2 * s + hh), rr);
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const uint32_t byte = (rr[q >> 2] >> (8 * (q & 3))) & 0xffu;
                    z = fmaf(byte >= 26u ? K : 0.0f, t_[16 * hh + q], z);
                }
            }
            ps[s] = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
            mean += ps[s];
        }
        mean *= 1.0f / 16.0f;
        float var = 0.f;
#pragma unroll
        for (int s = 0; s < 16; ++s) var += (ps[s] - mean) * (ps[s] - mean);
        const float sd = sqrtf(var * (1.0f / 16.0f));
        if (pmean) pmean[v] = mean;
        if (sd > 0.2f) {
            ++nf;
        } else {
            hot[c] = mean > 0.5f;
            notcold[c] = mean > 0.5f;
        }
    }
    // one atomic per wave
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nf += __shfl_xor(nf, o, 64);
    if ((threadIdx.x & 63) == 0 && nf) atomicAdd(nfall, nf);
}

// The switch's plasma window along x: the node columns holding particles or
// fluid of the fluid species, or ionizable ions (switch moments N or NI > 0),
// widened by `margin` nodes.  win[0..1] accumulate the extent (start at
// INT_MAX and -1), win[2..3] receive the window (empty when win[3] < win[2]).
__global__ void __launch_bounds__(CBS)
k_cnn_extent(GridP g, const real *__restrict__ mom, int *__restrict__ win) {
    const int NX = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
    const long long n = (long long)NX * g.ny * g.nz;
    const long long v = (long long)blockIdx.x * CBS + threadIdx.x;
    int lo = INT_MAX, hi = -1;
    if (v < n) {
        // node counts stay below 2^31: 32-bit index arithmetic
        const unsigned uv = (unsigned)v, ur = uv / (unsigned)NX;
        const int i = (int)(uv - ur * (unsigned)NX), j = (int)(ur % (unsigned)g.ny), k = (int)(ur / (unsigned)g.ny);
        const long long c = gidx(g, i, j, k);
        if (mom[c] > 0 || mom[6 * g.nn + c] > 0) { lo = i; hi = i; }
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o, 64));
        hi = max(hi, __shfl_xor(hi, o, 64));
    }
    // one wave per atomic, and only when it can move the extent: a read of the
    // current value (possibly stale, which only costs an atomic) avoids the
    // serialisation of every wave on the same two words
    if ((threadIdx.x & 63) == 0 && hi >= 0) {
        if (lo < *(volatile int *)win) atomicMin(win, lo);
        if (hi > *(volatile int *)(win + 1)) atomicMax(win + 1, hi);
    }
}

__global__ void k_cnn_window(int NX, int margin, int *__restrict__ win) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (win[1] < 0) { win[2] = 1; win[3] = 0; return; }
    win[2] = max(0, win[0] - margin);
    win[3] = min(NX - 1, win[1] + margin);
}

__global__ void k_cnn_window_init(int *__restrict__ win) {
    if (threadIdx.x == 0 && blockIdx.x == 0) { win[0] = INT_MAX; win[1] = -1; }
}

inline unsigned nblk(long long n) { return (unsigned)((n + CBS - 1) / CBS); }
inline unsigned rows_grid(long long rows) {
    long long b = (rows + 3) / 4;
    return (unsigned)(b < 4096 ? b : 4096);
}

}  // namespace

// ----------------------------------------------------------------- launchers
void cnn_launch_to_bf16(long long n, const float *x, unsigned short *o, hipStream_t s) {
    k_to_bf16<<<nblk(n), CBS, 0, s>>>(n, x, o);
}

void cnn_launch_conv_fwd(int cin, int B, int D, int H, int W, const unsigned short *act,
                         const unsigned short *Wf, const float *bias, float *zout, unsigned short *aout,
                         const int *xwin, hipStream_t s) {
    Dims in{B, D, H, W};
    // at most two workgroups per CU, every one looping over row groups: the
    // weight matrix is read into LDS once per workgroup
    if (cin == 8) {
        constexpr int RY = 4;
        const long long groups = (long long)B * (D - 2) * ((H - 2 + RY - 1) / RY) * ((W - 2 + 15) / 16);
        const long long nb4 = (groups + FBS / 64 - 1) / (FBS / 64);
        k_conv_fwd_first<RY><<<(unsigned)(nb4 < 512 ? nb4 : 512), FBS, 0, s>>>(in, act, Wf, bias, zout, aout, xwin);
    } else {
        constexpr int RY = 4;
        const long long groups = (long long)B * (D - 2) * ((H - 2 + RY - 1) / RY) * ((W - 2 + ROW_TW - 1) / ROW_TW);
        const long long nb4 = (groups + FBS / 64 - 1) / (FBS / 64);
        k_conv_fwd_rows<RY><<<(unsigned)(nb4 < 512 ? nb4 : 512), FBS, 0, s>>>(in, act, Wf, bias, zout, aout, xwin);
    }
}

void cnn_launch_conv_bwd_data(int B, int D, int H, int W, const unsigned short *dz,
                              const unsigned short *Wb, const float *zin, unsigned short *dzin,
                              hipStream_t s) {
    Dims in{B, D, H, W};
    const long long rows = (long long)B * D * H * ((W + 15) / 16);
    k_conv_bwd_data<<<rows_grid(rows), CBS, 0, s>>>(in, dz, Wb, zin, dzin);
}

void cnn_launch_conv_bwd_weight(int cin, int B, int D, int H, int W, const unsigned short *act,
                                const unsigned short *dz, float *gW, float *gb, hipStream_t s) {
    Dims in{B, D, H, W};
    const long long rows = (long long)B * (D - 2) * (H - 2) * ((W - 2 + 15) / 16);
    const int spw = 32;
    const long long waves = 27 * ((rows + spw - 1) / spw);
    const unsigned grid = (unsigned)((waves + 3) / 4);
    if (cin == 8) k_conv_bwd_weight<8><<<grid, CBS, 0, s>>>(in, act, dz, gW, spw);
    else k_conv_bwd_weight<32><<<grid, CBS, 0, s>>>(in, act, dz, gW, spw);
    const long long n = (long long)B * (D - 2) * (H - 2) * (W - 2);
    k_bias_grad<<<1024, CBS, 0, s>>>(n, dz, gb);
}

void cnn_launch_head(long long n, const unsigned short *a4, const unsigned short *wh, const float *bh,
                     int use_mask, uint64_t seed, uint32_t step, float *logit, hipStream_t s) {
    k_head<<<nblk(n), CBS, 0, s>>>(n, a4, wh, bh, use_mask, seed, step, logit);
}

void cnn_launch_head_bwd(long long n, const unsigned short *a4, const float *z4, const unsigned short *wh,
                         const float *bh, int use_mask, uint64_t seed, uint32_t step, const float *y,
                         const float *e, float lambda, unsigned short *dz4, float *gwh, double *loss,
                         hipStream_t s) {
    k_head_bwd<<<nblk(n), CBS, 0, s>>>(n, a4, z4, wh, bh, use_mask, seed, step, y, e, lambda, dz4, gwh, loss);
}

void cnn_launch_adamw(int n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2,
                      float eps, float wd, int t, hipStream_t s) {
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    k_adamw<<<nblk(n), CBS, 0, s>>>(n, p, g, m, v, lr, b1, b2, eps, wd, c1, c2);
}

void cnn_launch_pack(const float *p, int layer_cin, long long woff, int kpad, unsigned short *Wf,
                     unsigned short *Wb, hipStream_t s) {
    k_pack<<<nblk((long long)NC * kpad), CBS, 0, s>>>(p, layer_cin, woff, kpad, Wf, Wb);
}

void cnn_launch_pack_head(const float *p, long long off, unsigned short *wh, hipStream_t s) {
    k_pack_head<<<1, 64, 0, s>>>(p, off, wh);
}

void cnn_launch_inputs(const GridP &g, real *const f[9], const real *mom, const float mean[8],
                       const float inv_std[8], unsigned short *x, const int *xwin, hipStream_t s) {
    Norm nm;
    for (int q = 0; q < 8; ++q) { nm.mean[q] = mean[q]; nm.inv_std[q] = inv_std[q]; }
    const int NX = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
    const long long n = (long long)(NX + 8) * (g.ny + 8) * (g.nz + 8);
    k_cnn_inputs<<<nblk(n), CBS, 0, s>>>(g, f[HK_EX], f[HK_EY], f[HK_EZ], f[HK_BX], f[HK_BY], f[HK_BZ], mom,
                                         nm, x, xwin);
}

void cnn_launch_node_raw(const GridP &g, real *const f[9], const real *mom, float *out, hipStream_t s) {
    const int NX = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
    const long long n = (long long)NX * g.ny * g.nz;
    k_node_raw<<<nblk(n), CBS, 0, s>>>(g, f[HK_EX], f[HK_EY], f[HK_EZ], f[HK_BX], f[HK_BY], f[HK_BZ], mom, out);
}

void cnn_launch_node_state(const GridP &g, real *const f[9], const double *rho, float *out, hipStream_t s) {
    const int NX = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
    const long long n = (long long)NX * g.ny * g.nz;
    k_node_state<<<nblk(n), CBS, 0, s>>>(g, f[HK_EX], f[HK_EY], f[HK_EZ], f[HK_BX], f[HK_BY], f[HK_BZ], f[HK_JX],
                                          f[HK_JY], f[HK_JZ], rho, out);
}

void cnn_launch_decide(const GridP &g, const unsigned short *a4, const unsigned short *wh, const float *bh,
                       uint64_t seed, uint32_t eval, uint8_t *hot, uint8_t *notcold, int *nfall,
                       float *pmean, const int *xwin, hipStream_t s) {
    const int NX = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
    const long long n = (long long)NX * g.ny * g.nz;
    const unsigned grid = std::min<unsigned>(nblk(n), DECIDE_GRID);
    k_cnn_decide<<<grid, CBS, 0, s>>>(g, a4, wh, bh, seed, eval, hot, notcold, nfall, pmean, xwin);
}
void cnn_launch_window(const GridP &g, const real *mom, int margin, int *win, hipStream_t s) {
    const int NX = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
    k_cnn_window_init<<<1, 64, 0, s>>>(win);
    k_cnn_extent<<<nblk((long long)NX * g.ny * g.nz), CBS, 0, s>>>(g, mom, win);
    k_cnn_window<<<1, 64, 0, s>>>(NX, margin, win);
}
