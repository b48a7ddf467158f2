/*
 * Oracle of the paper's SwitchNet: a per-node classifier (fluid or kinetic)
 * made of two residual linear blocks, a 4-head attention layer and a sigmoid
 * head, with its loss gradient and dropout masks.  Test infrastructure: only
 * the tests, the smoke check and the bench's CPU leg call it.
 *
 * Paper: Results, Table 1 (SwitchNet layers) and the paragraph after it
 * (residuals and attention, BCE with a physics regularizer, AUC).  Readings:
 *   features (10): the node state E, B, J at the node and rho, normalized
 *   (x - mean) / std with frozen statistics, rounded to BF16;
 *   block 1: h1 = bf16(relu(W1 x + b1) + P x), 10 -> 128, P copying the
 *   input into the first channels (a residual across a change of width);
 *   block 2: h2 = bf16((relu(W2 h1 + b2) + P h1) m), 128 -> 256, m the
 *   dropout factors: byte c % 16 of Philox draw 16 s + c / 16 (tag 26,
 *   counter = node id and step, sample s) below 51 drops channel c (p close
 *   to the paper's 0.2), kept channels scaled by 256/205;
 *   attention: 4 heads of 64 over the one token a node is: per head the
 *   score q.k / 8 goes through a softmax over that single key, so each head
 *   returns its value; v = bf16(Wv h2 + bv), a = bf16(Wo v + bo); the query
 *   and key projections are evaluated but do not change the output, and
 *   their gradient is zero;
 *   head: logit = wh . a + bh (not rounded), p = sigmoid(logit);
 *   weights used rounded to BF16, biases as they are, sums in FP64;
 *   loss: mean over nodes of BCE(p, y) + lambda (1 - p) e, the physics term
 *   of the switch CNN (e the energy a cold-fluid conversion would destroy).
 * Parameter vector: W1[10][128], b1, W2[128][256], b2, then Wq, bq, Wk, bk,
 * Wv, bv, Wo, bo (each W[256][256] indexed [in][out]), then wh[256], bh
 * (297,857 values).
 */
#include "or_internal.h"

#define SW_IN 10
#define SW_H1 128
#define SW_H2 256
#define SW_HEADS 4

enum { O_W1 = 0, O_B1 = O_W1 + SW_IN * SW_H1, O_W2 = O_B1 + SW_H1, O_B2 = O_W2 + SW_H1 * SW_H2,
       O_WQ = O_B2 + SW_H2, O_BQ = O_WQ + SW_H2 * SW_H2, O_WK = O_BQ + SW_H2, O_BK = O_WK + SW_H2 * SW_H2,
       O_WV = O_BK + SW_H2, O_BV = O_WV + SW_H2 * SW_H2, O_WO = O_BV + SW_H2, O_BO = O_WO + SW_H2 * SW_H2,
       O_WH = O_BO + SW_H2, O_BH = O_WH + SW_H2, O_END = O_BH + 1 };

int or_swn_nparam(void) { return O_END; }

/* 256 keep factors (0 or 256/205) for one (node id, step, sample) */
void or_swn_mask(uint64_t seed, uint64_t id, uint32_t step, int sample, double out[256]) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int d = 0; d < 16; ++d) {
        uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), step, (26u << 8) | (uint32_t)(16 * sample + d)};
        uint32_t r[4];
        or_philox4x32_10(ctr, key, r);
        for (int c = 0; c < 16; ++c) {
            uint32_t byte = (r[c / 4] >> (8 * (c % 4))) & 0xffu;
            out[16 * d + c] = byte >= 51u ? 256.0 / 205.0 : 0.0;
        }
    }
}

/* y[o] = sum_i x[i] bf16(W[i][o]) + b[o] */
static void linear(const double *W, const double *b, const double *x, int ni, int no, double *y) {
    for (int o = 0; o < no; ++o) y[o] = b[o];
    for (int i = 0; i < ni; ++i)
        for (int o = 0; o < no; ++o) y[o] += x[i] * or_bf16(W[(size_t)i * no + o]);
}

typedef struct {
    double x[SW_IN], z1[SW_H1], h1[SW_H1], z2[SW_H2], h2[SW_H2], q[SW_H2], k[SW_H2], v[SW_H2], att[SW_H2],
        a[SW_H2], logit;
} sw_node;

static void forward_node(const double *par, const double *xin, const double *m, sw_node *s) {
    for (int i = 0; i < SW_IN; ++i) s->x[i] = or_bf16(xin[i]);
    linear(par + O_W1, par + O_B1, s->x, SW_IN, SW_H1, s->z1);
    for (int o = 0; o < SW_H1; ++o) s->h1[o] = or_bf16((s->z1[o] > 0 ? s->z1[o] : 0) + (o < SW_IN ? s->x[o] : 0));
    linear(par + O_W2, par + O_B2, s->h1, SW_H1, SW_H2, s->z2);
    for (int o = 0; o < SW_H2; ++o) {
        double h = (s->z2[o] > 0 ? s->z2[o] : 0) + (o < SW_H1 ? s->h1[o] : 0);
        if (m) h *= m[o];
        s->h2[o] = or_bf16(h);
    }
    /* attention over the single token */
    linear(par + O_WQ, par + O_BQ, s->h2, SW_H2, SW_H2, s->q);
    linear(par + O_WK, par + O_BK, s->h2, SW_H2, SW_H2, s->k);
    linear(par + O_WV, par + O_BV, s->h2, SW_H2, SW_H2, s->v);
    for (int o = 0; o < SW_H2; ++o) s->v[o] = or_bf16(s->v[o]);
    const int dh = SW_H2 / SW_HEADS;
    for (int h = 0; h < SW_HEADS; ++h) {
        double score = 0.0;
        for (int d = 0; d < dh; ++d) score += s->q[h * dh + d] * s->k[h * dh + d];
        score /= sqrt((double)dh);
        /* softmax over one key: exp(score - max) / sum = 1 */
        double wgt = exp(score - score) / exp(score - score);
        for (int d = 0; d < dh; ++d) s->att[h * dh + d] = wgt * s->v[h * dh + d];
    }
    linear(par + O_WO, par + O_BO, s->att, SW_H2, SW_H2, s->a);
    for (int o = 0; o < SW_H2; ++o) s->a[o] = or_bf16(s->a[o]);
    s->logit = par[O_BH];
    for (int i = 0; i < SW_H2; ++i) s->logit += s->a[i] * or_bf16(par[O_WH + i]);
}

/* logits of n nodes x[n][10]; mask: per node 256 factors, or NULL */
void or_swn_forward(const double *par, const double *x, int n, const double *mask, double *logit) {
    sw_node *s = (sw_node *)malloc(sizeof(sw_node));
    for (int v = 0; v < n; ++v) {
        forward_node(par, x + (size_t)v * SW_IN, mask ? mask + (size_t)v * SW_H2 : NULL, s);
        logit[v] = s->logit;
    }
    free(s);
}

/* dx[i] += sum_o bf16(W[i][o]) dy[o]; dW[i][o] += x[i] dy[o]; db[o] += dy[o] */
static void linear_back(const double *W, const double *x, const double *dy, int ni, int no, double *dW,
                        double *db, double *dx) {
    for (int o = 0; o < no; ++o) db[o] += dy[o];
    for (int i = 0; i < ni; ++i) {
        double acc = 0.0;
        for (int o = 0; o < no; ++o) {
            dW[(size_t)i * no + o] += x[i] * dy[o];
            acc += or_bf16(W[(size_t)i * no + o]) * dy[o];
        }
        if (dx) dx[i] += acc;
    }
}

/* Loss and gradient (BF16 rounding passed straight through; the softmax of
 * one key has zero derivative, so Wq, bq, Wk, bk get none). */
double or_swn_loss_grad(const double *par, const double *x, const double *y, const double *e, int n,
                        double lambda, const double *mask, double *grad) {
    memset(grad, 0, sizeof(double) * O_END);
    sw_node *s = (sw_node *)malloc(sizeof(sw_node));
    double loss = 0.0;
    for (int v = 0; v < n; ++v) {
        const double *m = mask ? mask + (size_t)v * SW_H2 : NULL;
        forward_node(par, x + (size_t)v * SW_IN, m, s);
        const double lg = s->logit, p = 1.0 / (1.0 + exp(-lg));
        const double sp = lg > 0 ? lg + log1p(exp(-lg)) : log1p(exp(lg));
        loss += (sp - y[v] * lg + lambda * (1.0 - p) * e[v]) / n;
        const double dl = (p - y[v] - lambda * p * (1.0 - p) * e[v]) / n;
        double da[SW_H2], dv[SW_H2], dh2[SW_H2], dz2[SW_H2], dh1[SW_H1], dz1[SW_H1];
        grad[O_BH] += dl;
        for (int i = 0; i < SW_H2; ++i) {
            grad[O_WH + i] += dl * s->a[i];
            da[i] = dl * or_bf16(par[O_WH + i]);
        }
        double datt[SW_H2];
        memset(datt, 0, sizeof(datt));
        linear_back(par + O_WO, s->att, da, SW_H2, SW_H2, grad + O_WO, grad + O_BO, datt);
        for (int i = 0; i < SW_H2; ++i) dv[i] = datt[i];   /* weight 1 per head */
        memset(dh2, 0, sizeof(dh2));
        linear_back(par + O_WV, s->h2, dv, SW_H2, SW_H2, grad + O_WV, grad + O_BV, dh2);
        for (int o = 0; o < SW_H2; ++o) {
            double g = dh2[o] * (m ? m[o] : 1.0);
            dz2[o] = s->z2[o] > 0 ? g : 0.0;
            dh2[o] = g;   /* residual path */
        }
        memset(dh1, 0, sizeof(dh1));
        linear_back(par + O_W2, s->h1, dz2, SW_H1, SW_H2, grad + O_W2, grad + O_B2, dh1);
        for (int o = 0; o < SW_H1; ++o) {
            double g = dh1[o] + dh2[o];
            dz1[o] = s->z1[o] > 0 ? g : 0.0;
        }
        linear_back(par + O_W1, s->x, dz1, SW_IN, SW_H1, grad + O_W1, grad + O_B1, NULL);
    }
    free(s);
    return loss;
}
