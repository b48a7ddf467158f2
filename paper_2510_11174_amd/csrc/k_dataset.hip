// Training set of the learned switch on the device: per-channel statistics of
// the node inputs, crops sampled with Philox, normalized inputs with their
// 4-node halo, labels and energy weights.
//
// Paper: Methodology, pipeline paragraph (the switch network is trained on
// data the simulation itself generates, on inputs normalized per channel,
// with a penalty on energy the regime choice would violate).
//
// A crop is 24^3 input nodes around 16^3 output nodes.  Its snapshot and
// origin come from one Philox draw (tag TAG_CROP, counter (crop index, AdamW
// iteration)); the halo wraps in y and z, and in x for a periodic grid, else
// repeats the wall node.  The energy weight of an output node is its
// conversion energy over the crop's kinetic energy (sum over the 16^3 output
// nodes of (1/2) n dV |p|_rms^2), times the 4096 nodes of the crop.
#include "hk_internal.h"
#include "hk_dataset_internal.h"

namespace {

constexpr int DBS = 256;
constexpr int CROP = 24, OUT = 16, HALO = 4;
constexpr int TAG_CROP = 28;

struct Norm {
    float mean[8], inv_std[8];
};

struct Pick {
    int k, z0, y0, x0;
};

__device__ inline Pick pick_crop(const DsSnap *tab, int nsnap, uint64_t seed, int b, int it) {
    uint32_t r[4];
    draw4(seed, (uint64_t)b, (uint32_t)it, TAG_CROP, 0, r);
    Pick p;
    p.k = min((int)(u01d(r[0]) * nsnap), nsnap - 1);
    const DsSnap &S = tab[p.k];
    p.z0 = min((int)(u01d(r[1]) * (S.D - OUT + 1)), S.D - OUT);
    p.y0 = min((int)(u01d(r[2]) * (S.H - OUT + 1)), S.H - OUT);
    p.x0 = min((int)(u01d(r[3]) * (S.W - OUT + 1)), S.W - OUT);
    return p;
}

// node of the snapshot that input voxel (z, y, x) of a window starting at
// node (z0 - 4, y0 - 4, x0 - 4) reads
__device__ inline long long src_node(const DsSnap &S, int z, int y, int x) {
    const int zz = wrapi(z, S.D), yy = wrapi(y, S.H);
    const int xx = S.per_x ? wrapi(x, S.W) : (x < 0 ? 0 : (x >= S.W ? S.W - 1 : x));
    return ((long long)zz * S.H + yy) * S.W + xx;
}

__global__ void __launch_bounds__(DBS)
k_ds_crops(const DsSnap *__restrict__ tab, int nsnap, uint64_t seed, int it, Norm nm, float *__restrict__ x,
           float *__restrict__ y, float *__restrict__ e) {
    const int b = blockIdx.y;
    const int t = blockIdx.x * DBS + threadIdx.x;
    if (t >= CROP * CROP * CROP) return;
    const Pick p = pick_crop(tab, nsnap, seed, b, it);
    const DsSnap &S = tab[p.k];
    const int dz = t / (CROP * CROP), dy = (t / CROP) % CROP, dx = t % CROP;
    const long long v = src_node(S, p.z0 + dz - HALO, p.y0 + dy - HALO, p.x0 + dx - HALO);
    const float *r = S.raw9 + 9 * v;
    float *o = x + ((long long)b * CROP * CROP * CROP + t) * 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) o[q] = (r[q] - nm.mean[q]) * nm.inv_std[q];
    if (dz >= HALO && dz < HALO + OUT && dy >= HALO && dy < HALO + OUT && dx >= HALO && dx < HALO + OUT) {
        const long long oi = (long long)b * OUT * OUT * OUT + ((dz - HALO) * OUT + (dy - HALO)) * OUT + (dx - HALO);
        y[oi] = (float)S.y[v];
        e[oi] = r[8];
    }
}

// one block per crop: the crop's kinetic energy, then the weights
__global__ void __launch_bounds__(DBS)
k_ds_weights(const DsSnap *__restrict__ tab, int nsnap, uint64_t seed, int it, float *__restrict__ e) {
    __shared__ double part[DBS];
    const int b = blockIdx.x;
    const Pick p = pick_crop(tab, nsnap, seed, b, it);
    const DsSnap &S = tab[p.k];
    double ke = 0.0;
    for (int o = threadIdx.x; o < OUT * OUT * OUT; o += DBS) {
        const int dz = o / (OUT * OUT), dy = (o / OUT) % OUT, dx = o % OUT;
        const long long v = ((long long)(p.z0 + dz) * S.H + (p.y0 + dy)) * S.W + (p.x0 + dx);
        const float *r = S.raw9 + 9 * v;
        ke += 0.5 * (double)r[6] * S.dv * (double)r[7] * (double)r[7];
    }
    part[threadIdx.x] = ke;
    __syncthreads();
    for (int h = DBS / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    const double scale = (double)(OUT * OUT * OUT) / (part[0] + 1e-30);
    for (int o = threadIdx.x; o < OUT * OUT * OUT; o += DBS) {
        float &w = e[(long long)b * OUT * OUT * OUT + o];
        w = (float)((double)w * scale);
    }
}

// Whole snapshot with its halo, normalized: x[D+8][H+8][W+8][8].
__global__ void __launch_bounds__(DBS)
k_ds_pad(DsSnap S, Norm nm, float *__restrict__ x) {
    const int PD = S.D + 2 * HALO, PH = S.H + 2 * HALO, PW = S.W + 2 * HALO;
    const long long t = (long long)blockIdx.x * DBS + threadIdx.x;
    if (t >= (long long)PD * PH * PW) return;
    const int dz = (int)(t / ((long long)PH * PW)), dy = (int)((t / PW) % PH), dx = (int)(t % PW);
    const float *r = S.raw9 + 9 * src_node(S, dz - HALO, dy - HALO, dx - HALO);
    float *o = x + 8 * t;
#pragma unroll
    for (int q = 0; q < 8; ++q) o[q] = (r[q] - nm.mean[q]) * nm.inv_std[q];
}

// Per-channel sums and sums of squares of the 8 inputs (FP64).
__global__ void __launch_bounds__(DBS)
k_ds_stats(const float *__restrict__ raw9, long long n, double *__restrict__ acc) {
    __shared__ double part[16][DBS / 64];
    double s[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) s[q] = 0.0;
    for (long long v = (long long)blockIdx.x * DBS + threadIdx.x; v < n; v += (long long)gridDim.x * DBS) {
        const float *r = raw9 + 9 * v;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double a = r[q];
            s[q] += a;
            s[8 + q] += a * a;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        double a = s[q];
        for (int o = 32; o > 0; o >>= 1) a += __shfl_down(a, o, 64);
        if (lane == 0) part[q][wave] = a;
    }
    __syncthreads();
    if (threadIdx.x < 16) {
        double a = 0.0;
        for (int w = 0; w < DBS / 64; ++w) a += part[threadIdx.x][w];
        atomicAdd(acc + threadIdx.x, a);
    }
}

Norm make_norm(const float *mean, const float *inv_std) {
    Norm nm;
    for (int q = 0; q < 8; ++q) { nm.mean[q] = mean[q]; nm.inv_std[q] = inv_std[q]; }
    return nm;
}

}  // namespace

void ds_launch_crops(const DsSnap *tab, int nsnap, uint64_t seed, int it, int B, const float *mean,
                     const float *inv_std, float *x, float *y, float *e, hipStream_t s) {
    dim3 grid((CROP * CROP * CROP + DBS - 1) / DBS, B);
    k_ds_crops<<<grid, DBS, 0, s>>>(tab, nsnap, seed, it, make_norm(mean, inv_std), x, y, e);
    k_ds_weights<<<B, DBS, 0, s>>>(tab, nsnap, seed, it, e);
}

void ds_launch_pad(const DsSnap &S, const float *mean, const float *inv_std, float *x, hipStream_t s) {
    const long long n = (long long)(S.D + 2 * HALO) * (S.H + 2 * HALO) * (S.W + 2 * HALO);
    k_ds_pad<<<(unsigned)((n + DBS - 1) / DBS), DBS, 0, s>>>(S, make_norm(mean, inv_std), x);
}

void ds_launch_stats(const float *raw9, long long n, double *acc, hipStream_t s) {
    long long blocks = (n + DBS - 1) / DBS;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    k_ds_stats<<<(unsigned)blocks, DBS, 0, s>>>(raw9, n, acc);
}
