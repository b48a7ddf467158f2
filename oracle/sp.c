/*
 * Oracle of the next-state surrogate (the paper's StatePredictor): a residual
 * 3D CNN mapping a 10-channel state patch to the state a few steps later, its
 * loss gradient and its dropout masks.  Test infrastructure: only the tests,
 * the smoke check and the bench's CPU leg call it.
 *
 * Paper: Results, Table 2 (StatePredictor architecture) and the paragraph
 * before it (residual blocks, dropout, Huber loss with delta 0.01, physics
 * term 0.1 on energy violation).  Readings:
 *   channels (10): Ex, Ey, Ez, Bx, By, Bz, Jx, Jy, Jz and rho at the nodes,
 *   each normalized (x - mean) / std with frozen statistics; inputs rounded
 *   to BF16;
 *   "same" 3^3 convolutions with zero padding (the patch keeps its size, 16^3
 *   in the paper); tap t = kx + 3 ky + 9 kz reads offset (kx-1, ky-1, kz-1);
 *   blocks 1-3 (10->13, 13->32, 32->64): a = bf16(relu(conv(x) + b) + P x),
 *   P copying the block's input into its first channels (zeros in the rest):
 *   a residual across a change of width with no extra weights;
 *   dropout on block 2's output (32 channels): byte c of two Philox draws
 *   (tag 25, draws 2s and 2s + 1 for sample s, counter = voxel id and step)
 *   below 26 drops the channel, kept channels are scaled by 256/230; the
 *   activation is rounded to BF16 once, after the dropout factor;
 *   block 4 (the 128-32-10 row of Table 2): conv 64->128 + relu, conv
 *   128->32 + relu, conv 32->10, linear: the output is the normalized next
 *   state, signed, in FP32 (not rounded);
 *   weights used rounded to BF16 (round to nearest even from FP32), biases as
 *   they are, sums in FP64 here (FP32 on the GPU);
 *   loss: mean over voxels and channels of Huber_delta(pred - target) plus
 *   lambda times the mean over samples of ((U_pred - U_true) / U_true)^2,
 *   U = sum over the patch of sum_{c < 6} (x_c std_c + mean_c)^2, the field
 *   energy in the de-normalized units.
 * Parameter vector: per layer W[27][cin][cout] then b[cout], in layer order
 * (410,733 values).
 */
#include "or_internal.h"

#define SP_NL 6
static const int sp_cin[SP_NL] = {10, 13, 32, 64, 128, 32};
static const int sp_cout[SP_NL] = {13, 32, 64, 128, 32, 10};
static const int sp_res[SP_NL] = {1, 1, 1, 0, 0, 0};
static const int sp_relu[SP_NL] = {1, 1, 1, 1, 1, 0};
#define SP_DROP_LAYER 1   /* dropout on this layer's output */

static size_t sp_woff(int l) {
    size_t o = 0;
    for (int q = 0; q < l; ++q) o += 27 * (size_t)sp_cin[q] * sp_cout[q] + sp_cout[q];
    return o;
}

int or_sp_nparam(void) { return (int)sp_woff(SP_NL); }

/* 32 keep factors (0 or 256/230) for one (voxel id, step, sample) */
void or_sp_mask(uint64_t seed, uint64_t id, uint32_t step, int sample, double out[32]) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int h = 0; h < 2; ++h) {
        uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), step, (25u << 8) | (uint32_t)(2 * sample + h)};
        uint32_t r[4];
        or_philox4x32_10(ctr, key, r);
        for (int c = 0; c < 16; ++c) {
            uint32_t byte = (r[c / 4] >> (8 * (c % 4))) & 0xffu;
            out[16 * h + c] = byte >= 26u ? 256.0 / 230.0 : 0.0;
        }
    }
}

typedef struct {
    int B, D, H, W;
    size_t n;                     /* voxels */
    double *a[SP_NL + 1];         /* activations, channels last: a[0] input, a[l+1] layer l output */
    double *z[SP_NL];             /* pre-activations of layer l */
} sp_fwd_t;

/* s[v][co] = sum_t sum_ci a[v + off(t)][ci] W[t][ci][co] (zero padding) */
static void conv_same(const sp_fwd_t *f, const double *a, int ci, const double *Wt, int co, double *s) {
    for (int b = 0; b < f->B; ++b)
        for (int z = 0; z < f->D; ++z)
            for (int y = 0; y < f->H; ++y)
                for (int x = 0; x < f->W; ++x) {
                    size_t o = (((size_t)b * f->D + z) * f->H + y) * f->W + x;
                    for (int c = 0; c < co; ++c) s[o * co + c] = 0.0;
                    for (int t = 0; t < 27; ++t) {
                        int xx = x + t % 3 - 1, yy = y + (t / 3) % 3 - 1, zz = z + t / 9 - 1;
                        if (xx < 0 || xx >= f->W || yy < 0 || yy >= f->H || zz < 0 || zz >= f->D) continue;
                        size_t iv = (((size_t)b * f->D + zz) * f->H + yy) * f->W + xx;
                        for (int i = 0; i < ci; ++i) {
                            double av = a[iv * ci + i];
                            if (av == 0.0) continue;
                            for (int c = 0; c < co; ++c) s[o * co + c] += av * or_bf16(Wt[((size_t)t * ci + i) * co + c]);
                        }
                    }
                }
}

static void sp_forward(const double *par, const double *x, int B, int D, int H, int W, const double *mask,
                       sp_fwd_t *f) {
    f->B = B; f->D = D; f->H = H; f->W = W;
    f->n = (size_t)B * D * H * W;
    f->a[0] = (double *)malloc(sizeof(double) * f->n * 10);
    for (size_t i = 0; i < f->n * 10; ++i) f->a[0][i] = or_bf16(x[i]);
    for (int l = 0; l < SP_NL; ++l) {
        const int ci = sp_cin[l], co = sp_cout[l];
        const double *Wt = par + sp_woff(l), *bias = Wt + 27 * (size_t)ci * co;
        f->z[l] = (double *)malloc(sizeof(double) * f->n * co);
        f->a[l + 1] = (double *)malloc(sizeof(double) * f->n * co);
        conv_same(f, f->a[l], ci, Wt, co, f->z[l]);
        for (size_t v = 0; v < f->n; ++v)
            for (int c = 0; c < co; ++c) {
                double zz = f->z[l][v * co + c] += bias[c];
                double o = sp_relu[l] ? (zz > 0.0 ? zz : 0.0) : zz;
                if (sp_res[l] && c < ci) o += f->a[l][v * ci + c];
                if (l == SP_NL - 1) { f->a[l + 1][v * co + c] = o; continue; }   /* FP32 output */
                if (l == SP_DROP_LAYER && mask) o *= mask[v * 32 + c];
                f->a[l + 1][v * co + c] = or_bf16(o);
            }
    }
}

static void sp_free(sp_fwd_t *f) {
    for (int l = 0; l <= SP_NL; ++l) free(f->a[l]);
    for (int l = 0; l < SP_NL; ++l) free(f->z[l]);
}

/* Next states (normalized) of B patches x[B][D][H][W][10]; mask: per voxel 32
 * factors for block 2's output, or NULL. */
void or_sp_forward(const double *par, const double *x, int B, int D, int H, int W, const double *mask,
                   double *out) {
    sp_fwd_t f;
    sp_forward(par, x, B, D, H, W, mask, &f);
    memcpy(out, f.a[SP_NL], sizeof(double) * f.n * 10);
    sp_free(&f);
}

/* Loss and its gradient with respect to the parameters (BF16 rounding passed
 * straight through); y: target next states, normalized like x. */
double or_sp_loss_grad(const double *par, const double *x, const double *y, int B, int D, int H, int W,
                       const double mean[10], const double stdv[10], double delta, double lambda,
                       const double *mask, double *grad) {
    sp_fwd_t f;
    sp_forward(par, x, B, D, H, W, mask, &f);
    memset(grad, 0, sizeof(double) * or_sp_nparam());
    const size_t n = f.n, per = n / B;
    const double *p = f.a[SP_NL];
    double loss = 0.0;
    double *da = (double *)calloc(n * 10, sizeof(double));
    for (size_t i = 0; i < n * 10; ++i) {
        double d = p[i] - y[i];
        double ad = fabs(d);
        loss += ad <= delta ? 0.5 * d * d : delta * (ad - 0.5 * delta);
        da[i] = (ad <= delta ? d : (d > 0 ? delta : -delta)) / (double)(n * 10);
    }
    loss /= (double)(n * 10);
    for (int b = 0; b < B; ++b) {
        double up = 0.0, ut = 0.0;
        for (size_t v = b * per; v < (b + 1) * per; ++v)
            for (int c = 0; c < 6; ++c) {
                double ep = p[v * 10 + c] * stdv[c] + mean[c], et = y[v * 10 + c] * stdv[c] + mean[c];
                up += ep * ep; ut += et * et;
            }
        if (ut <= 0.0) continue;
        double r = (up - ut) / ut;
        loss += lambda * r * r / B;
        double k = lambda * 2.0 * r / ut / B;
        for (size_t v = b * per; v < (b + 1) * per; ++v)
            for (int c = 0; c < 6; ++c)
                da[v * 10 + c] += k * 2.0 * (p[v * 10 + c] * stdv[c] + mean[c]) * stdv[c];
    }
    for (int l = SP_NL - 1; l >= 0; --l) {
        const int ci = sp_cin[l], co = sp_cout[l];
        const double *Wt = par + sp_woff(l);
        double *gW = grad + sp_woff(l), *gb = gW + 27 * (size_t)ci * co;
        /* through dropout, then relu */
        double *dz = (double *)malloc(sizeof(double) * n * co);
        for (size_t v = 0; v < n; ++v)
            for (int c = 0; c < co; ++c) {
                double g = da[v * co + c];
                if (l == SP_DROP_LAYER && mask) g *= mask[v * 32 + c];
                da[v * co + c] = g;   /* gradient of the block output before dropout */
                dz[v * co + c] = sp_relu[l] ? (f.z[l][v * co + c] > 0.0 ? g : 0.0) : g;
            }
        double *dprev = (double *)calloc(n * ci, sizeof(double));
        for (int b = 0; b < B; ++b)
            for (int z = 0; z < D; ++z)
                for (int yy = 0; yy < H; ++yy)
                    for (int xx = 0; xx < W; ++xx) {
                        size_t o = (((size_t)b * D + z) * H + yy) * W + xx;
                        for (int c = 0; c < co; ++c) gb[c] += dz[o * co + c];
                        for (int t = 0; t < 27; ++t) {
                            int x2 = xx + t % 3 - 1, y2 = yy + (t / 3) % 3 - 1, z2 = z + t / 9 - 1;
                            if (x2 < 0 || x2 >= W || y2 < 0 || y2 >= H || z2 < 0 || z2 >= D) continue;
                            size_t iv = (((size_t)b * D + z2) * H + y2) * W + x2;
                            for (int i = 0; i < ci; ++i) {
                                double av = f.a[l][iv * ci + i], acc = 0.0;
                                const double *wr = Wt + ((size_t)t * ci + i) * co;
                                double *gw = gW + ((size_t)t * ci + i) * co;
                                for (int c = 0; c < co; ++c) {
                                    double g = dz[o * co + c];
                                    gw[c] += av * g;
                                    acc += or_bf16(wr[c]) * g;
                                }
                                dprev[iv * ci + i] += acc;
                            }
                        }
                    }
        if (sp_res[l])
            for (size_t v = 0; v < n; ++v)
                for (int i = 0; i < ci; ++i) dprev[v * ci + i] += da[v * co + i];
        free(dz);
        free(da);
        da = dprev;
    }
    free(da);
    sp_free(&f);
    return loss;
}
