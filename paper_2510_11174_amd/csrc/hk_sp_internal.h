// Kernel arguments and launchers of the next-state surrogate (k_sp.hip),
// used by its host side (hk_sp.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

// One "same" 3^3 convolution as an implicit GEMM (forward or data gradient).
struct SpConv {
    int B, D, H, W;                 // voxel grid, shared by input and output
    const unsigned short *in;       // [n][CPIN] BF16, channels last
    const unsigned short *wp;       // [cols][KPAD] BF16 weight matrix
    int cols, cout;                 // padded (output stride) and real output channels
    // forward epilogue
    const float *bias;              // [cout]
    int relu, res;                  // res: leading channels of `in` added after the ReLU
    float *fout;                    // last layer: FP32 [n][cout] (no BF16 output)
    // both epilogues
    int drop;                       // apply the dropout factors of (seed, voxel, step, sample)
    uint64_t seed;
    uint32_t step;
    uint32_t drop_tag, drop_thr;    // Philox tag; a byte below drop_thr drops the channel
    float drop_scale;               // factor of a kept channel
    int drop_sample;                // Monte Carlo sample: draws sample * cols / 16 + c / 16
    unsigned short *zout;           // forward: BF16 pre-activations (for the backward pass), or null
    unsigned short *aout, *aT;      // BF16 result, channels last and channel-major (or null)
    // data-gradient epilogue
    const float *gin;               // residual-path gradient of the layer above (or null)
    int gin_ch, gin_stride;
    float *gout;                    // gradient after dropout of the layer below (or null)
    const unsigned short *zin;      // BF16 pre-activations of the layer below (null: it has no ReLU)
    int ntask, G;                   // work items, column groups (set by the launcher)
};

// Weight gradient of one convolution from the channel-major copies.
struct SpWgrad {
    int B, D, H, W;
    const unsigned short *aT;       // [B][cpi][D][H][W] layer input
    const unsigned short *dT;       // [B][cpo][D][H][W] pre-activation gradient
    int cpi, cpo, cin, cout;
    float *gw;                      // [27][cin][cout], accumulated
    float *gb;                      // [cout] bias gradient, accumulated (or null)
    int mtn, ngn, nitems;           // ci tiles, co groups, workgroups
    long long nblk, nks, kpc;       // 8-voxel blocks, K steps (4 blocks), steps per chunk
};

struct SpNorm { float mean[10], stdv[10]; };

// taps: 27 ("same" 3^3 convolution) or 1 (a linear layer per voxel)
int sp_launch_conv(int cpin, int taps, bool bwd, const SpConv &a, hipStream_t s);
int sp_launch_wgrad(int nt, int taps, const SpWgrad &a, hipStream_t s);
void sp_launch_energy(long long n, long long per, const float *p, const float *y, const SpNorm &nm, double *U,
                      hipStream_t s);
void sp_launch_loss(long long n, long long per, int B, const float *p, const float *y, const SpNorm &nm,
                    const double *U, float delta, float lambda, unsigned short *dz, unsigned short *dzT,
                    double *loss, hipStream_t s);
void sp_launch_pack(const float *W, int cin, int cout, int cpi, int cpo, int taps, unsigned short *Wf,
                    unsigned short *Wb, hipStream_t s);
void swn_launch_loss(long long n, const float *logit, const float *y, const float *e, float lambda,
                     unsigned short *dz, unsigned short *dzT, long long ldT, double *loss, hipStream_t s);
void sp_launch_input(long long n, long long per, const float *x, unsigned short *xb, unsigned short *xT,
                     hipStream_t s);
