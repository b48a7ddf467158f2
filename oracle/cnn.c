/*
 * Oracle of the learned regime switch: a small 3D CNN, its training step, and
 * its use as the switch with Monte Carlo dropout and a threshold fallback.
 *
 * Paper: abstract and Methodology (a neural network decides fluid or kinetic
 * treatment per region, with uncertainty estimates from Monte Carlo dropout
 * and the physics thresholds as fallback; training on data the simulations
 * generate, with a physics penalty on energy violation).  The paper's own
 * classifier is a per-cell network with attention; the readings used here are:
 *
 *   inputs per node, 8 channels: E (3) and B (3) at the node, the electron
 *   density N/dV, and the rms momentum sqrt(sum w |u|^2 / sum w); each
 *   normalized with frozen statistics (x - mean) / std and rounded to BF16;
 *   4 layers: valid 3^3 convolution (8 -> 32, then 32 -> 32 channels), bias,
 *   exact GELU 0.5 z (1 + erf(z / sqrt 2)), output rounded to BF16;
 *   head: 1 x 1 x 1, 32 -> 1, logit; p = 1 / (1 + exp(-logit));
 *   weights are used rounded to BF16 (round to nearest even from FP32), biases as they
 *   are; sums in FP64 here (FP32 on the GPU);
 *   the network sees a node through a 4-node halo (24^3 inputs give 16^3
 *   outputs); on the whole grid the halo wraps in periodic directions and
 *   repeats the wall node in open x;
 *   dropout on the head input only: channel c of a sample is kept when byte c
 *   of two Philox draws (tag 24, draws 2s and 2s + 1 for sample s) is >= 26,
 *   i.e. dropped with probability 26/256, and kept channels are scaled by
 *   256/230;  the switch runs 16 samples per node, counter (node, evaluation
 *   number); mean p > 0.5 means kinetic unless the samples' standard
 *   deviation exceeds 0.2, where the threshold decision is kept;
 *   loss per output node: BCE(p, y) + lambda (1 - p) e, averaged;
 *   AdamW on FP64 master parameters (decoupled weight decay on everything).
 *
 * Parameter vector (90017 values): W1[27][8][32], b1[32], then for layers
 * 2..4 W[27][32][32], b[32], then the head w[32], b.  Tap t = kx + 3 ky + 9 kz.
 */
#include "or_internal.h"

#define NC 32

static int cin_of(int l) { return l == 0 ? 8 : NC; }
static size_t w_off(int l) {   /* offset of layer l's weights */
    size_t o = 0;
    for (int q = 0; q < l; ++q) o += 27 * (size_t)cin_of(q) * NC + NC;
    return o;
}
static size_t head_off(void) { return w_off(4); }

int or_cnn_nparam(void) { return (int)(head_off() + NC + 1); }

/* BF16 from FP32, round to nearest even (the GPU stores FP32 results this
 * way): the double is first rounded to FP32, then to 8 significant bits.
 * or_cnn_set_rounding(0) turns the rounding off (for finite-difference checks
 * of the gradients). */
static int g_round = 1;
void or_cnn_set_rounding(int on) { g_round = on; }
double or_bf16(double x) {
    if (!g_round || x == 0.0 || !isfinite(x)) return x;
    double f = (double)(float)x;        /* RNE to FP32 */
    int e;
    double m = frexp(f, &e);            /* f = m 2^e, 0.5 <= |m| < 1 */
    double r = nearbyint(ldexp(m, 8));  /* 8 significant bits, ties to even */
    return ldexp(r, e - 8);
}

static double gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }
static double gelu_d(double z) {
    return 0.5 * (1.0 + erf(z / sqrt(2.0))) + z * exp(-0.5 * z * z) / sqrt(2.0 * OR_PI);
}

/* 32 keep factors (0 or 256/230) for one (id, step, sample) */
void or_cnn_mask(uint64_t seed, uint64_t id, uint32_t step, int sample, double out[NC]) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int h = 0; h < 2; ++h) {
        uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), step, (24u << 8) | (uint32_t)(2 * sample + h)};
        uint32_t r[4];
        or_philox4x32_10(ctr, key, r);
        for (int c = 0; c < 16; ++c) {
            uint32_t byte = (r[c / 4] >> (8 * (c % 4))) & 0xffu;
            out[16 * h + c] = byte >= 26u ? 256.0 / 230.0 : 0.0;
        }
    }
}

typedef struct {
    int B, D[5], H[5], W[5];     /* dims of activation l (0 = input) */
    double *a[5];                /* activations (BF16 values), channels last */
    double *z[5];                /* pre-activations of layers 1..4 */
} fwd_t;

static size_t vox(const fwd_t *f, int l) { return (size_t)f->B * f->D[l] * f->H[l] * f->W[l]; }

static void forward(const double *par, const double *x, int B, int D, int H, int W, fwd_t *f) {
    f->B = B;
    for (int l = 0; l < 5; ++l) { f->D[l] = D - 2 * l; f->H[l] = H - 2 * l; f->W[l] = W - 2 * l; }
    f->a[0] = (double *)malloc(sizeof(double) * vox(f, 0) * 8);
    for (size_t i = 0; i < vox(f, 0) * 8; ++i) f->a[0][i] = or_bf16(x[i]);
    f->z[0] = NULL;
    for (int l = 0; l < 4; ++l) {
        const int ci = cin_of(l);
        const double *Wt = par + w_off(l), *bias = Wt + 27 * (size_t)ci * NC;
        size_t n = vox(f, l + 1);
        f->z[l + 1] = (double *)malloc(sizeof(double) * n * NC);
        f->a[l + 1] = (double *)malloc(sizeof(double) * n * NC);
        for (int b = 0; b < B; ++b)
            for (int z = 0; z < f->D[l + 1]; ++z)
                for (int y = 0; y < f->H[l + 1]; ++y)
                    for (int xx = 0; xx < f->W[l + 1]; ++xx) {
                        size_t o = (((size_t)b * f->D[l + 1] + z) * f->H[l + 1] + y) * f->W[l + 1] + xx;
                        for (int co = 0; co < NC; ++co) {
                            double s = bias[co];
                            for (int t = 0; t < 27; ++t) {
                                int kx = t % 3, ky = (t / 3) % 3, kz = t / 9;
                                size_t iv = (((size_t)b * f->D[l] + z + kz) * f->H[l] + y + ky) * f->W[l] + xx + kx;
                                for (int c = 0; c < ci; ++c)
                                    s += f->a[l][iv * ci + c] * or_bf16(Wt[((size_t)t * ci + c) * NC + co]);
                            }
                            f->z[l + 1][o * NC + co] = s;
                            f->a[l + 1][o * NC + co] = or_bf16(gelu(s));
                        }
                    }
    }
}

static void fwd_free(fwd_t *f) {
    for (int l = 0; l < 5; ++l) { free(f->a[l]); if (l) free(f->z[l]); }
}

static double head_logit(const double *par, const double *h, const double *mask) {
    const double *wh = par + head_off();
    double s = wh[NC];
    for (int c = 0; c < NC; ++c) s += or_bf16(wh[c]) * h[c] * (mask ? mask[c] : 1.0);
    return s;
}

/* Logits of B crops (D x H x W x 8 normalized inputs, channels last) over the
 * (D-8)(H-8)(W-8) valid outputs; mask: per output voxel 32 factors, or NULL. */
void or_cnn_forward(const double *par, const double *x, int B, int D, int H, int W,
                    const double *mask, double *logit) {
    fwd_t f;
    forward(par, x, B, D, H, W, &f);
    size_t n = vox(&f, 4);
    for (size_t v = 0; v < n; ++v) logit[v] = head_logit(par, f.a[4] + v * NC, mask ? mask + v * NC : NULL);
    fwd_free(&f);
}

/* Loss and its gradient with respect to the parameters (BF16 rounding passed
 * straight through). */
double or_cnn_loss_grad(const double *par, const double *x, const double *y, const double *e,
                        int B, int D, int H, int W, double lambda, const double *mask, double *grad) {
    fwd_t f;
    forward(par, x, B, D, H, W, &f);
    const int np = or_cnn_nparam();
    memset(grad, 0, sizeof(double) * np);
    size_t n = vox(&f, 4);
    double loss = 0.0;
    double *da = (double *)calloc(n * NC, sizeof(double));
    const double *wh = par + head_off();
    double *gh = grad + head_off();
    for (size_t v = 0; v < n; ++v) {
        const double *mk = mask ? mask + v * NC : NULL;
        double lg = head_logit(par, f.a[4] + v * NC, mk);
        double p = 1.0 / (1.0 + exp(-lg));
        /* BCE from the logit: softplus(l) - y l */
        double sp = lg > 0 ? lg + log1p(exp(-lg)) : log1p(exp(lg));
        loss += sp - y[v] * lg + lambda * (1.0 - p) * e[v];
        double dl = (p - y[v] - lambda * p * (1.0 - p) * e[v]) / (double)n;
        for (int c = 0; c < NC; ++c) {
            double m = mk ? mk[c] : 1.0;
            gh[c] += dl * f.a[4][v * NC + c] * m;
            da[v * NC + c] = dl * or_bf16(wh[c]) * m;
        }
        gh[NC] += dl;
    }
    loss /= (double)n;
    for (int l = 3; l >= 0; --l) {
        const int ci = cin_of(l);
        const double *Wt = par + w_off(l);
        double *gW = grad + w_off(l), *gb = gW + 27 * (size_t)ci * NC;
        size_t no = vox(&f, l + 1), ni = vox(&f, l);
        double *dz = (double *)malloc(sizeof(double) * no * NC);
        for (size_t i = 0; i < no * NC; ++i) dz[i] = da[i] * gelu_d(f.z[l + 1][i]);
        double *dprev = l > 0 ? (double *)calloc(ni * ci, sizeof(double)) : NULL;
        for (int b = 0; b < B; ++b)
            for (int z = 0; z < f.D[l + 1]; ++z)
                for (int yy = 0; yy < f.H[l + 1]; ++yy)
                    for (int xx = 0; xx < f.W[l + 1]; ++xx) {
                        size_t o = (((size_t)b * f.D[l + 1] + z) * f.H[l + 1] + yy) * f.W[l + 1] + xx;
                        for (int co = 0; co < NC; ++co) {
                            double g = dz[o * NC + co];
                            gb[co] += g;
                            for (int t = 0; t < 27; ++t) {
                                int kx = t % 3, ky = (t / 3) % 3, kz = t / 9;
                                size_t iv = (((size_t)b * f.D[l] + z + kz) * f.H[l] + yy + ky) * f.W[l] + xx + kx;
                                for (int c = 0; c < ci; ++c) {
                                    gW[((size_t)t * ci + c) * NC + co] += f.a[l][iv * ci + c] * g;
                                    if (dprev) dprev[iv * ci + c] += or_bf16(Wt[((size_t)t * ci + c) * NC + co]) * g;
                                }
                            }
                        }
                    }
        free(dz);
        free(da);
        da = dprev;
    }
    fwd_free(&f);
    return loss;
}

/* AdamW (Loshchilov and Hutter): decoupled weight decay, bias-corrected moments. */
void or_cnn_adamw(double *par, const double *grad, double *m, double *v, int t, double lr,
                  double b1, double b2, double eps, double wd, int n) {
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
        v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
        par[i] -= lr * (m[i] / c1 / (sqrt(v[i] / c2) + eps) + wd * par[i]);
    }
}

/* ------------------------------------------------------------ the switch */

typedef struct {
    double *par;
    double mean[8], std[8];
    int have;
    uint32_t evals;
} or_cnn_state;

int or_set_cnn(or_sim *s, const double *par, const double mean[8], const double stdv[8]) {
    or_cnn_state *c = (or_cnn_state *)s->cnn;
    if (!c) { c = (or_cnn_state *)calloc(1, sizeof(or_cnn_state)); s->cnn = c; }
    free(c->par);
    c->par = (double *)malloc(sizeof(double) * or_cnn_nparam());
    memcpy(c->par, par, sizeof(double) * or_cnn_nparam());
    memcpy(c->mean, mean, sizeof(c->mean));
    for (int k = 0; k < 8; ++k) c->std[k] = stdv[k] > 0.0 ? stdv[k] : 1.0;
    c->have = 1;
    return 0;
}

void or_cnn_free(or_sim *s) {
    or_cnn_state *c = (or_cnn_state *)s->cnn;
    if (c) free(c->par);
    free(c);
    s->cnn = NULL;
}

/* Node inputs (raw, before normalization) of the canonical node grid. */
void or_cnn_node_inputs(or_sim *s, const double *N, const double *U2, double *raw) {
    const or_grid *g = &s->g;
    double dv = g->dx * g->dy * g->dz;
    int nxn = g->bc_x == OR_BC_PERIODIC ? g->nx : g->nx + 1;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < nxn; ++i) {
                size_t c = or_idx(s, i, j, k);
                size_t o = (((size_t)k * g->ny + j) * nxn + i) * 8;
                int node[3] = {i, j, k};
                double z0[3] = {0, 0, 0};
                for (int d = 0; d < 6; ++d) raw[o + d] = or_gather(s, OR_EX + d, node, z0);
                raw[o + 6] = N[c] / dv;
                raw[o + 7] = N[c] > 0 ? sqrt(U2[c] / N[c]) : 0.0;
            }
}

/* Switch decisions from the CNN where it is confident; returns the fraction
 * of nodes that kept the threshold decision. */
double or_cnn_switch(or_sim *s, const double *N, const double *U2, const double *NI, uint8_t *hot,
                     uint8_t *cold) {
    or_cnn_state *cs = (or_cnn_state *)s->cnn;
    if (!cs || !cs->have) return 1.0;
    const or_grid *g = &s->g;
    int nxn = g->bc_x == OR_BC_PERIODIC ? g->nx : g->nx + 1;
    size_t nodes = (size_t)nxn * g->ny * g->nz;
    /* The network decides in the plasma's x extent (columns with N or NI > 0)
     * widened by the nodes plasma can reach before the next evaluation
     * (switch_every + dilation + 4); the threshold decision stays elsewhere. */
    int lo = nxn, hi = -1;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < nxn; ++i) {
                size_t c = or_idx(s, i, j, k);
                if (N[c] > 0 || NI[c] > 0) {
                    if (i < lo) lo = i;
                    if (i > hi) hi = i;
                }
            }
    int margin = s->run.switch_every + s->run.dilation + 4;
    int w0 = lo - margin < 0 ? 0 : lo - margin;
    int w1 = hi + margin > nxn - 1 ? nxn - 1 : hi + margin;
    if (hi < 0) { w0 = 1; w1 = 0; }
    double *raw = (double *)malloc(sizeof(double) * nodes * 8);
    or_cnn_node_inputs(s, N, U2, raw);
    int D = g->nz + 8, H = g->ny + 8, W = nxn + 8;
    double *x = (double *)malloc(sizeof(double) * (size_t)D * H * W * 8);
    for (int k = 0; k < D; ++k)
        for (int j = 0; j < H; ++j)
            for (int i = 0; i < W; ++i) {
                int kk = or_wrap(k - 4, g->nz), jj = or_wrap(j - 4, g->ny), ii = i - 4;
                if (g->bc_x == OR_BC_PERIODIC) ii = or_wrap(ii, g->nx);
                else ii = ii < 0 ? 0 : (ii > nxn - 1 ? nxn - 1 : ii);
                const double *r = raw + (((size_t)kk * g->ny + jj) * nxn + ii) * 8;
                double *o = x + (((size_t)k * H + j) * W + i) * 8;
                for (int c = 0; c < 8; ++c) o[c] = (r[c] - cs->mean[c]) / cs->std[c];
            }
    fwd_t f;
    forward(cs->par, x, 1, D, H, W, &f);
    size_t fall = 0;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < nxn; ++i) {
                size_t v = ((size_t)k * g->ny + j) * nxn + i;
                size_t c = or_idx(s, i, j, k);
                if (i < w0 || i > w1) continue;
                double ps[16], mean = 0.0, var = 0.0;
                for (int q = 0; q < 16; ++q) {
                    double mk[NC];
                    or_cnn_mask(s->run.seed, c, cs->evals, q, mk);
                    ps[q] = 1.0 / (1.0 + exp(-head_logit(cs->par, f.a[4] + v * NC, mk)));
                    mean += ps[q];
                }
                mean /= 16.0;
                for (int q = 0; q < 16; ++q) var += (ps[q] - mean) * (ps[q] - mean);
                double sd = sqrt(var / 16.0);
                if (sd > 0.2) { fall++; continue; }
                hot[c] = mean > 0.5;
                cold[c] = hot[c];
            }
    cs->evals++;
    fwd_free(&f);
    free(x);
    free(raw);
    return (double)fall / (double)nodes;
}
