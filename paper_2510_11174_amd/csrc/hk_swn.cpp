// Host side of the paper's SwitchNet: parameters (FP32 masters and BF16
// weight matrices), AdamW state, workspace, and the forward / gradient /
// training calls of the C ABI (include/hk.h, hk_swn_*).
//
// Paper: Results, Table 1 (SwitchNet) and the paragraph after it.  Layers
// (per node): 10 -> 128 and 128 -> 256, each ReLU plus a residual copy of its
// input, dropout on the 256-wide output; 4-head attention over the node's
// single token, which returns each head's value projection, so it runs as
// the value and output projections (256 -> 256, twice); a 256 -> 1 head.
// Every layer is a linear map per node: the one-tap instantiation of the
// surrogate's matrix-core convolution kernels.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/hk.h"
#include "hk_sp_internal.h"

void cnn_launch_adamw(int n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2,
                      float eps, float wd, int t, hipStream_t s);

namespace {

constexpr int NL = 5;
constexpr int CIN[NL] = {10, 128, 256, 256, 256};
constexpr int COUT[NL] = {128, 256, 256, 256, 1};
constexpr int RES[NL] = {10, 128, 0, 0, 0};   // input channels copied into the output
constexpr int RELU[NL] = {1, 1, 0, 0, 0};
constexpr int DROP_LAYER = 1;
// parameter vector: W1, b1, W2, b2, Wq, bq, Wk, bk, Wv, bv, Wo, bo, wh, bh
constexpr long long P_W1 = 0, P_B1 = P_W1 + 10 * 128, P_W2 = P_B1 + 128, P_B2 = P_W2 + 128 * 256,
                    P_WQ = P_B2 + 256, P_WK = P_WQ + 256 * 256 + 256, P_WV = P_WK + 256 * 256 + 256,
                    P_WO = P_WV + 256 * 256 + 256, P_WH = P_WO + 256 * 256 + 256, P_END = P_WH + 256 + 1;
constexpr long long W_OFF[NL] = {P_W1, P_W2, P_WV, P_WO, P_WH};
constexpr long long B_OFF[NL] = {P_B1, P_B2, P_WV + 256 * 256, P_WO + 256 * 256, P_WH + 256};

int cp(int c) { return (c + 15) / 16 * 16; }
int kpad(int cpin) { return (cpin + 31) / 32 * 32; }
int ntile(int cols) { return cols / 16 < 4 ? cols / 16 : 4; }

enum { W_ACT = 0, W_ACTT = NL, W_Z = 2 * NL, W_OUT = 3 * NL, W_DZ, W_DZ2, W_DZT, W_DZT2, W_G1, W_N };

}  // namespace

struct hk_swn {
    hipStream_t s = nullptr;
    hk_alloc_fn alloc = nullptr;
    hk_free_fn free = nullptr;
    void *alloc_ctx = nullptr;
    uint64_t seed = 0;
    float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    double *loss = nullptr;
    unsigned short *Wf[NL] = {}, *Wb[NL] = {};
    int t = 0;
    void *w[W_N] = {};
    size_t cap[W_N] = {};
    std::vector<void *> allocs;
    std::string err;
};

namespace {

int fail(hk_swn *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->err = buf;
    return code;
}

#define WCHK(c, x)                                                                                  \
    do {                                                                                            \
        hipError_t e_ = (x);                                                                        \
        if (e_ != hipSuccess) return fail(c, HK_EDEVICE, "%s: %s", #x, hipGetErrorString(e_));      \
    } while (0)

void *nalloc(hk_swn *c, size_t bytes) {
    void *p = nullptr;
    if (c->alloc) p = c->alloc(bytes, c->alloc_ctx);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    if (p) c->allocs.push_back(p);
    return p;
}

void nrelease(hk_swn *c, void *p) {
    if (!p) return;
    for (size_t i = 0; i < c->allocs.size(); ++i)
        if (c->allocs[i] == p) {
            c->allocs.erase(c->allocs.begin() + i);
            break;
        }
    if (c->free) c->free(p, c->alloc_ctx);
    else (void)hipFree(p);
}

template <typename T>
T *ws(hk_swn *c, int slot, size_t bytes) {
    if (c->cap[slot] >= bytes && c->w[slot]) return (T *)c->w[slot];
    (void)hipStreamSynchronize(c->s);
    nrelease(c, c->w[slot]);
    c->w[slot] = nalloc(c, bytes);
    c->cap[slot] = c->w[slot] ? bytes : 0;
    return (T *)c->w[slot];
}

void pack(hk_swn *c) {
    for (int l = 0; l < NL; ++l)
        sp_launch_pack(c->p + W_OFF[l], CIN[l], COUT[l], cp(CIN[l]), cp(COUT[l]), 1, c->Wf[l], c->Wb[l], c->s);
}

// n nodes laid out as one row of n voxels
SpConv layer_args(int n, int cols, uint64_t seed, int mask_step, int sample) {
    SpConv a{};
    a.B = 1; a.D = 1; a.H = 1; a.W = n;
    a.cols = cols;
    // dropout p = 51/256 (Philox tag 26), kept channels scaled by 256/205
    a.seed = seed;
    a.step = (uint32_t)(mask_step >= 0 ? mask_step : 0);
    a.drop_tag = 26;
    a.drop_thr = 51;
    a.drop_scale = 256.0f / 205.0f;
    a.drop_sample = sample;
    return a;
}

int forward(hk_swn *c, const float *x, int n, int mask_step, int sample, bool train, float *logit) {
    unsigned short *act[NL] = {}, *actT[NL] = {}, *z[NL] = {};
    for (int l = 0; l < NL; ++l) {
        const size_t bytes = (size_t)n * cp(CIN[l]) * 2;
        act[l] = ws<unsigned short>(c, W_ACT + l, bytes);
        if (!act[l]) return fail(c, HK_ENOMEM, "SwitchNet activations");
        if (train) {
            actT[l] = ws<unsigned short>(c, W_ACTT + l, bytes);
            z[l] = RELU[l] ? ws<unsigned short>(c, W_Z + l, (size_t)n * cp(COUT[l]) * 2) : nullptr;
            if (!actT[l] || (RELU[l] && !z[l])) return fail(c, HK_ENOMEM, "SwitchNet activations");
        }
    }
    sp_launch_input(n, n, x, act[0], actT[0], c->s);
    for (int l = 0; l < NL; ++l) {
        const int cpin = cp(CIN[l]), cols = cp(COUT[l]);
        SpConv a = layer_args(n, cols, c->seed, mask_step, sample);
        a.in = act[l];
        a.wp = c->Wf[l];
        a.cout = COUT[l];
        a.bias = c->p + B_OFF[l];
        a.relu = RELU[l];
        a.res = RES[l];
        a.drop = l == DROP_LAYER && mask_step >= 0;
        a.zout = train ? z[l] : nullptr;
        if (l == NL - 1) a.fout = logit;
        else {
            a.aout = act[l + 1];
            a.aT = train ? actT[l + 1] : nullptr;
        }
        if (sp_launch_conv(cpin, 1, false, a, c->s))
            return fail(c, HK_EINVAL, "no linear-layer kernel for %d -> %d channels", cpin, cols);
    }
    return HK_OK;
}

int check_n(hk_swn *c, int n, bool train) {
    if (n <= 0) return fail(c, HK_EINVAL, "no nodes");
    if (n > (1 << 26)) return fail(c, HK_EINVAL, "more than 2^26 nodes in one call");
    if (train && n % 8) return fail(c, HK_EINVAL, "training needs n %% 8 == 0 (got %d)", n);
    return HK_OK;
}

}  // namespace

extern "C" {

int hk_swn_nparams(void) { return (int)P_END; }

int hk_swn_create(const hk_cnn_desc *d, hk_swn **out) {
    if (!d || !out) return HK_EINVAL;
    hk_swn *c = new hk_swn();
    c->s = (hipStream_t)d->stream;
    c->alloc = d->alloc;
    c->free = d->free;
    c->alloc_ctx = d->alloc_ctx;
    c->seed = d->seed;
    const int np = hk_swn_nparams();
    c->p = (float *)nalloc(c, sizeof(float) * np);
    c->m = (float *)nalloc(c, sizeof(float) * np);
    c->v = (float *)nalloc(c, sizeof(float) * np);
    c->g = (float *)nalloc(c, sizeof(float) * np);
    c->loss = (double *)nalloc(c, sizeof(double));
    bool ok = c->p && c->m && c->v && c->g && c->loss;
    for (int l = 0; l < NL && ok; ++l) {
        c->Wf[l] = (unsigned short *)nalloc(c, 2 * (size_t)cp(COUT[l]) * kpad(cp(CIN[l])));
        c->Wb[l] = (unsigned short *)nalloc(c, 2 * (size_t)cp(CIN[l]) * kpad(cp(COUT[l])));
        ok = c->Wf[l] && c->Wb[l];
    }
    if (!ok) {
        hk_swn_destroy(c);
        return HK_ENOMEM;
    }
    (void)hipMemsetAsync(c->p, 0, sizeof(float) * np, c->s);
    (void)hipMemsetAsync(c->m, 0, sizeof(float) * np, c->s);
    (void)hipMemsetAsync(c->v, 0, sizeof(float) * np, c->s);
    pack(c);
    if (hipStreamSynchronize(c->s) != hipSuccess) {
        hk_swn_destroy(c);
        return HK_EDEVICE;
    }
    *out = c;
    return HK_OK;
}

void hk_swn_destroy(hk_swn *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->s);
    std::vector<void *> all = c->allocs;
    for (void *p : all) nrelease(c, p);
    delete c;
}

int hk_swn_set_params(hk_swn *c, const float *params, size_t n) {
    if (!c || !params || n != (size_t)hk_swn_nparams()) return HK_EINVAL;
    WCHK(c, hipMemcpyAsync(c->p, params, sizeof(float) * n, hipMemcpyHostToDevice, c->s));
    WCHK(c, hipMemsetAsync(c->m, 0, sizeof(float) * n, c->s));
    WCHK(c, hipMemsetAsync(c->v, 0, sizeof(float) * n, c->s));
    c->t = 0;
    pack(c);
    WCHK(c, hipStreamSynchronize(c->s));
    return HK_OK;
}

int hk_swn_get_params(hk_swn *c, float *params, size_t n) {
    if (!c || !params || n != (size_t)hk_swn_nparams()) return HK_EINVAL;
    WCHK(c, hipMemcpyAsync(params, c->p, sizeof(float) * n, hipMemcpyDeviceToHost, c->s));
    WCHK(c, hipStreamSynchronize(c->s));
    return HK_OK;
}

int hk_swn_forward(hk_swn *c, const float *x, int n, int mask_step, int sample, float *logit) {
    if (!c || !x || !logit) return HK_EINVAL;
    int rc = check_n(c, n, false);
    if (rc) return rc;
    if (sample < 0 || sample > 15) return fail(c, HK_EINVAL, "dropout sample %d outside 0..15", sample);
    rc = forward(c, x, n, mask_step, sample, false, logit);
    if (rc) return rc;
    WCHK(c, hipStreamSynchronize(c->s));
    return HK_OK;
}

int hk_swn_loss_grad(hk_swn *c, const float *x, const float *y, const float *e, int n, double lambda,
                     int mask_step, float *grad_host, double *loss) {
    if (!c || !x || !y || !e) return HK_EINVAL;
    int rc = check_n(c, n, true);
    if (rc) return rc;
    hipStream_t s = c->s;
    float *logit = ws<float>(c, W_OUT, (size_t)n * 4);
    unsigned short *dz[2] = {ws<unsigned short>(c, W_DZ, (size_t)n * 256 * 2),
                             ws<unsigned short>(c, W_DZ2, (size_t)n * 256 * 2)};
    unsigned short *dzT[2] = {ws<unsigned short>(c, W_DZT, (size_t)n * 256 * 2),
                              ws<unsigned short>(c, W_DZT2, (size_t)n * 256 * 2)};
    float *g1 = ws<float>(c, W_G1, (size_t)n * cp(COUT[DROP_LAYER]) * 4);
    if (!logit || !dz[0] || !dz[1] || !dzT[0] || !dzT[1] || !g1) return fail(c, HK_ENOMEM, "SwitchNet gradients");
    rc = forward(c, x, n, mask_step, 0, true, logit);
    if (rc) return rc;
    const int np = hk_swn_nparams();
    WCHK(c, hipMemsetAsync(c->g, 0, sizeof(float) * np, s));
    WCHK(c, hipMemsetAsync(c->loss, 0, sizeof(double), s));
    swn_launch_loss(n, logit, y, e, (float)lambda, dz[0], dzT[0], n, c->loss, s);
    int cur = 0;
    for (int l = NL - 1; l >= 0; --l) {
        const int cpi = cp(CIN[l]), cpo = cp(COUT[l]);
        SpWgrad wg{};
        wg.B = 1; wg.D = 1; wg.H = 1; wg.W = n;
        wg.aT = (const unsigned short *)c->w[W_ACTT + l];
        wg.dT = dzT[cur];
        wg.cpi = cpi; wg.cpo = cpo; wg.cin = CIN[l]; wg.cout = COUT[l];
        wg.gw = c->g + W_OFF[l];
        wg.gb = c->g + B_OFF[l];
        const int wnt = ntile(cpo);
        wg.mtn = cpi / 16;
        wg.ngn = cpo / (16 * wnt);
        wg.nblk = n / 8;
        wg.nks = (wg.nblk + 3) / 4;
        const long long base = (long long)wg.mtn * wg.ngn;
        long long chunks = (1024 + base - 1) / base;
        if (chunks > (wg.nks + 15) / 16) chunks = (wg.nks + 15) / 16;
        if (chunks < 1) chunks = 1;
        wg.kpc = (wg.nks + chunks - 1) / chunks;
        chunks = (wg.nks + wg.kpc - 1) / wg.kpc;
        wg.nitems = (int)(base * chunks);
        if (sp_launch_wgrad(wnt, 1, wg, s)) return fail(c, HK_EINVAL, "no weight-gradient kernel");
        if (l == 0) break;
        SpConv a = layer_args(n, cpi, c->seed, mask_step, 0);
        a.in = dz[cur];
        a.wp = c->Wb[l];
        a.cout = CIN[l];
        a.gin = RES[l] ? g1 : nullptr;   // only block 2's residual carries a gradient back
        a.gin_ch = RES[l];
        a.gin_stride = cpo;
        a.drop = l - 1 == DROP_LAYER && mask_step >= 0;
        a.gout = l - 1 == DROP_LAYER ? g1 : nullptr;
        a.zin = RELU[l - 1] ? (const unsigned short *)c->w[W_Z + l - 1] : nullptr;
        a.aout = dz[cur ^ 1];
        a.aT = dzT[cur ^ 1];
        if (sp_launch_conv(cpo, 1, true, a, s))
            return fail(c, HK_EINVAL, "no data-gradient kernel for %d -> %d channels", cpo, cpi);
        cur ^= 1;
    }
    if (grad_host) WCHK(c, hipMemcpyAsync(grad_host, c->g, sizeof(float) * np, hipMemcpyDeviceToHost, s));
    double lh = 0.0;
    WCHK(c, hipMemcpyAsync(&lh, c->loss, sizeof(double), hipMemcpyDeviceToHost, s));
    WCHK(c, hipStreamSynchronize(s));
    if (loss) *loss = lh;
    return HK_OK;
}

int hk_swn_train_step(hk_swn *c, const float *x, const float *y, const float *e, int n,
                      const hk_cnn_train_desc *t, double *loss) {
    if (!c || !t) return HK_EINVAL;
    int rc = hk_swn_loss_grad(c, x, y, e, n, t->lambda_e, t->dropout ? c->t : -1, nullptr, loss);
    if (rc) return rc;
    c->t += 1;
    cnn_launch_adamw(hk_swn_nparams(), c->p, c->g, c->m, c->v, (float)t->lr, (float)t->beta1, (float)t->beta2,
                     (float)t->eps, (float)t->weight_decay, c->t, c->s);
    pack(c);
    WCHK(c, hipStreamSynchronize(c->s));
    return HK_OK;
}

const char *hk_swn_last_error(const hk_swn *c) { return c ? c->err.c_str() : "null network"; }

}  // extern "C"
