// Host side of the next-state surrogate: parameters (FP32 masters and BF16
// weight matrices), AdamW state, workspace, and the forward / gradient /
// training calls of the C ABI (include/hk.h, hk_sp_*).
//
// Paper: Results, Table 2 (StatePredictor) and the paragraph before it.
// Layers (input -> output channels): 10->13, 13->32, 32->64 with residual
// copies of the block input, then 64->128, 128->32, 32->10; ReLU after all
// but the last; dropout on the 32-channel output of the second layer.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hk.h"
#include "hk_sp_internal.h"

void cnn_launch_adamw(int n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2,
                      float eps, float wd, int t, hipStream_t s);

namespace {

constexpr int NL = 6;
constexpr int CIN[NL] = {10, 13, 32, 64, 128, 32};
constexpr int COUT[NL] = {13, 32, 64, 128, 32, 10};
constexpr int RES[NL] = {1, 1, 1, 0, 0, 0};
constexpr int DROP_LAYER = 1;

int cp(int c) { return (c + 15) / 16 * 16; }
long long w_off(int l) {
    long long o = 0;
    for (int q = 0; q < l; ++q) o += 27LL * CIN[q] * COUT[q] + COUT[q];
    return o;
}
long long b_off(int l) { return w_off(l) + 27LL * CIN[l] * COUT[l]; }
int kpad(int cpin) { return (27 * cpin + 31) / 32 * 32; }
int ntile(int cols) { return cols / 16 < 4 ? cols / 16 : 4; }

// workspace slots
enum { W_ACT = 0, W_ACTT = NL, W_Z = 2 * NL, W_OUT = 3 * NL, W_DZ, W_DZ2, W_DZT, W_DZT2, W_G1, W_G2, W_U, W_N };

}  // namespace

struct hk_sp {
    hipStream_t s = nullptr;
    hk_alloc_fn alloc = nullptr;
    hk_free_fn free = nullptr;
    void *alloc_ctx = nullptr;
    uint64_t seed = 0;
    float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    double *loss = nullptr;
    unsigned short *Wf[NL] = {}, *Wb[NL] = {};
    SpNorm nm;
    int t = 0;
    void *w[W_N] = {};
    size_t cap[W_N] = {};
    std::vector<void *> allocs;
    std::string err;
};

namespace {

int fail(hk_sp *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->err = buf;
    return code;
}

#define SCHK(c, x)                                                                                  \
    do {                                                                                            \
        hipError_t e_ = (x);                                                                        \
        if (e_ != hipSuccess) return fail(c, HK_EDEVICE, "%s: %s", #x, hipGetErrorString(e_));      \
    } while (0)

void *sp_alloc(hk_sp *c, size_t bytes) {
    void *p = nullptr;
    if (c->alloc) p = c->alloc(bytes, c->alloc_ctx);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    if (p) c->allocs.push_back(p);
    return p;
}

void sp_release(hk_sp *c, void *p) {
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
T *ws(hk_sp *c, int slot, size_t bytes) {
    if (c->cap[slot] >= bytes && c->w[slot]) return (T *)c->w[slot];
    (void)hipStreamSynchronize(c->s);
    sp_release(c, c->w[slot]);
    c->w[slot] = sp_alloc(c, bytes);
    c->cap[slot] = c->w[slot] ? bytes : 0;
    return (T *)c->w[slot];
}

void pack(hk_sp *c) {
    for (int l = 0; l < NL; ++l)
        sp_launch_pack(c->p + w_off(l), CIN[l], COUT[l], cp(CIN[l]), cp(COUT[l]), 27, c->Wf[l], c->Wb[l], c->s);
}

int check_shape(hk_sp *c, int B, int D, int H, int W, bool train) {
    if (B <= 0 || D <= 0 || H <= 0 || W <= 0) return fail(c, HK_EINVAL, "empty patch batch");
    if ((long long)B * D * H * W * 128 >= (1LL << 40)) return fail(c, HK_EINVAL, "patch batch too large");
    if ((long long)B * (D * H) * ((W + 15) / 16) >= (1LL << 30)) return fail(c, HK_EINVAL, "patch batch too large");
    if (train && W % 8) return fail(c, HK_EINVAL, "training needs W %% 8 == 0 (got %d)", W);
    return HK_OK;
}

SpConv conv_args(int B, int D, int H, int W, int cols) {
    SpConv a{};
    a.B = B; a.D = D; a.H = H; a.W = W;
    a.cols = cols;
    // dropout p = 26/256 (Philox tag 25), kept channels scaled by 256/230
    a.drop_tag = 25;
    a.drop_thr = 26;
    a.drop_scale = 256.0f / 230.0f;
    return a;
}

// Forward pass from FP32 inputs; with `train` every layer's input is kept in
// both layouts and the pre-activations in BF16.
int forward(hk_sp *c, const float *x, int B, int D, int H, int W, int mask_step, bool train, float *out) {
    const long long n = (long long)B * D * H * W, per = (long long)D * H * W;
    unsigned short *act[NL + 1] = {}, *actT[NL + 1] = {}, *z[NL] = {};
    for (int l = 0; l < NL; ++l) {
        const size_t bytes = (size_t)n * cp(CIN[l]) * 2;
        act[l] = ws<unsigned short>(c, W_ACT + l, bytes);
        if (!act[l]) return fail(c, HK_ENOMEM, "surrogate activations");
        if (train) {
            actT[l] = ws<unsigned short>(c, W_ACTT + l, bytes);
            z[l] = l < NL - 1 ? ws<unsigned short>(c, W_Z + l, (size_t)n * cp(COUT[l]) * 2) : nullptr;
            if (!actT[l] || (l < NL - 1 && !z[l])) return fail(c, HK_ENOMEM, "surrogate activations");
        }
    }
    sp_launch_input(n, per, x, act[0], actT[0], c->s);
    for (int l = 0; l < NL; ++l) {
        const int cpin = cp(CIN[l]), cols = cp(COUT[l]);
        SpConv a = conv_args(B, D, H, W, cols);
        a.in = act[l];
        a.wp = c->Wf[l];
        a.cout = COUT[l];
        a.bias = c->p + b_off(l);
        a.relu = l < NL - 1;
        a.res = RES[l] ? CIN[l] : 0;
        a.drop = l == DROP_LAYER && mask_step >= 0;
        a.seed = c->seed;
        a.step = (uint32_t)(mask_step >= 0 ? mask_step : 0);
        a.zout = train ? z[l] : nullptr;
        if (l == NL - 1) a.fout = out;
        else {
            a.aout = act[l + 1];
            a.aT = train ? actT[l + 1] : nullptr;
        }
        if (sp_launch_conv(cpin, 27, false, a, c->s))
            return fail(c, HK_EINVAL, "no convolution kernel for %d -> %d channels", cpin, cols);
    }
    return HK_OK;
}

}  // namespace

extern "C" {

int hk_sp_nparams(void) { return (int)w_off(NL); }

int hk_sp_create(const hk_cnn_desc *d, hk_sp **out) {
    if (!d || !out) return HK_EINVAL;
    hk_sp *c = new hk_sp();
    c->s = (hipStream_t)d->stream;
    c->alloc = d->alloc;
    c->free = d->free;
    c->alloc_ctx = d->alloc_ctx;
    c->seed = d->seed;
    const int np = hk_sp_nparams();
    c->p = (float *)sp_alloc(c, sizeof(float) * np);
    c->m = (float *)sp_alloc(c, sizeof(float) * np);
    c->v = (float *)sp_alloc(c, sizeof(float) * np);
    c->g = (float *)sp_alloc(c, sizeof(float) * np);
    c->loss = (double *)sp_alloc(c, sizeof(double));
    bool ok = c->p && c->m && c->v && c->g && c->loss;
    for (int l = 0; l < NL && ok; ++l) {
        c->Wf[l] = (unsigned short *)sp_alloc(c, 2 * (size_t)cp(COUT[l]) * kpad(cp(CIN[l])));
        c->Wb[l] = (unsigned short *)sp_alloc(c, 2 * (size_t)cp(CIN[l]) * kpad(cp(COUT[l])));
        ok = c->Wf[l] && c->Wb[l];
    }
    if (!ok) {
        hk_sp_destroy(c);
        return HK_ENOMEM;
    }
    for (int q = 0; q < 10; ++q) { c->nm.mean[q] = 0.f; c->nm.stdv[q] = 1.f; }
    (void)hipMemsetAsync(c->p, 0, sizeof(float) * np, c->s);
    (void)hipMemsetAsync(c->m, 0, sizeof(float) * np, c->s);
    (void)hipMemsetAsync(c->v, 0, sizeof(float) * np, c->s);
    pack(c);
    if (hipStreamSynchronize(c->s) != hipSuccess) {
        hk_sp_destroy(c);
        return HK_EDEVICE;
    }
    *out = c;
    return HK_OK;
}

void hk_sp_destroy(hk_sp *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->s);
    std::vector<void *> all = c->allocs;
    for (void *p : all) sp_release(c, p);
    delete c;
}

int hk_sp_set_params(hk_sp *c, const float *params, size_t n) {
    if (!c || !params || n != (size_t)hk_sp_nparams()) return HK_EINVAL;
    SCHK(c, hipMemcpyAsync(c->p, params, sizeof(float) * n, hipMemcpyHostToDevice, c->s));
    SCHK(c, hipMemsetAsync(c->m, 0, sizeof(float) * n, c->s));
    SCHK(c, hipMemsetAsync(c->v, 0, sizeof(float) * n, c->s));
    c->t = 0;
    pack(c);
    SCHK(c, hipStreamSynchronize(c->s));
    return HK_OK;
}

int hk_sp_get_params(hk_sp *c, float *params, size_t n) {
    if (!c || !params || n != (size_t)hk_sp_nparams()) return HK_EINVAL;
    SCHK(c, hipMemcpyAsync(params, c->p, sizeof(float) * n, hipMemcpyDeviceToHost, c->s));
    SCHK(c, hipStreamSynchronize(c->s));
    return HK_OK;
}

int hk_sp_set_norm(hk_sp *c, const float *mean, const float *stdv) {
    if (!c || !mean || !stdv) return HK_EINVAL;
    for (int q = 0; q < 10; ++q) {
        c->nm.mean[q] = mean[q];
        c->nm.stdv[q] = stdv[q];
    }
    return HK_OK;
}

int hk_sp_forward(hk_sp *c, const float *x, int B, int D, int H, int W, int mask_step, float *out) {
    if (!c || !x || !out) return HK_EINVAL;
    int rc = check_shape(c, B, D, H, W, false);
    if (rc) return rc;
    rc = forward(c, x, B, D, H, W, mask_step, false, out);
    if (rc) return rc;
    SCHK(c, hipStreamSynchronize(c->s));
    return HK_OK;
}

int hk_sp_loss_grad(hk_sp *c, const float *x, const float *y, int B, int D, int H, int W, double delta,
                    double lambda, int mask_step, float *grad_host, double *loss) {
    if (!c || !x || !y) return HK_EINVAL;
    int rc = check_shape(c, B, D, H, W, true);
    if (rc) return rc;
    hipStream_t s = c->s;
    const long long n = (long long)B * D * H * W, per = (long long)D * H * W;
    float *out = ws<float>(c, W_OUT, (size_t)n * 10 * 4);
    unsigned short *dz[2] = {ws<unsigned short>(c, W_DZ, (size_t)n * 128 * 2),
                             ws<unsigned short>(c, W_DZ2, (size_t)n * 128 * 2)};
    unsigned short *dzT[2] = {ws<unsigned short>(c, W_DZT, (size_t)n * 128 * 2),
                              ws<unsigned short>(c, W_DZT2, (size_t)n * 128 * 2)};
    float *gres[NL] = {};
    gres[1] = ws<float>(c, W_G1, (size_t)n * cp(COUT[1]) * 4);
    gres[2] = ws<float>(c, W_G2, (size_t)n * cp(COUT[2]) * 4);
    double *U = ws<double>(c, W_U, (size_t)B * 2 * 8);
    if (!out || !dz[0] || !dz[1] || !dzT[0] || !dzT[1] || !gres[1] || !gres[2] || !U)
        return fail(c, HK_ENOMEM, "surrogate gradients");
    rc = forward(c, x, B, D, H, W, mask_step, true, out);
    if (rc) return rc;
    const int np = hk_sp_nparams();
    SCHK(c, hipMemsetAsync(c->g, 0, sizeof(float) * np, s));
    SCHK(c, hipMemsetAsync(c->loss, 0, sizeof(double), s));
    SCHK(c, hipMemsetAsync(U, 0, sizeof(double) * 2 * B, s));
    sp_launch_energy(n, per, out, y, c->nm, U, s);
    sp_launch_loss(n, per, B, out, y, c->nm, U, (float)delta, (float)lambda, dz[0], dzT[0], c->loss, s);
    int cur = 0;
    for (int l = NL - 1; l >= 0; --l) {
        const int cpi = cp(CIN[l]), cpo = cp(COUT[l]);
        // weight and bias gradients: K = 8-voxel blocks, chunks sized for
        // ~1024 workgroups
        SpWgrad wg{};
        wg.B = B; wg.D = D; wg.H = H; wg.W = W;
        wg.aT = (const unsigned short *)c->w[W_ACTT + l];
        wg.dT = dzT[cur];
        wg.cpi = cpi; wg.cpo = cpo; wg.cin = CIN[l]; wg.cout = COUT[l];
        wg.gw = c->g + w_off(l);
        wg.gb = c->g + b_off(l);
        const int wnt = ntile(cpo);
        wg.mtn = cpi / 16;
        wg.ngn = cpo / (16 * wnt);
        wg.nblk = n / 8;
        wg.nks = (wg.nblk + 3) / 4;
        const long long base = 9LL * wg.mtn * wg.ngn;
        long long chunks = (1024 + base - 1) / base;
        if (chunks > (wg.nks + 15) / 16) chunks = (wg.nks + 15) / 16;
        if (chunks < 1) chunks = 1;
        wg.kpc = (wg.nks + chunks - 1) / chunks;
        chunks = (wg.nks + wg.kpc - 1) / wg.kpc;
        wg.nitems = (int)(base * chunks);
        if (sp_launch_wgrad(wnt, 27, wg, s)) return fail(c, HK_EINVAL, "no weight-gradient kernel");
        if (l == 0) break;
        // data gradient into the layer below's pre-activation gradient
        SpConv a = conv_args(B, D, H, W, cpi);
        a.in = dz[cur];
        a.wp = c->Wb[l];
        a.cout = CIN[l];
        a.gin = RES[l] ? gres[l] : nullptr;
        a.gin_ch = RES[l] ? CIN[l] : 0;
        a.gin_stride = cpo;
        a.drop = l - 1 == DROP_LAYER && mask_step >= 0;
        a.seed = c->seed;
        a.step = (uint32_t)(mask_step >= 0 ? mask_step : 0);
        a.gout = l - 1 >= 1 && RES[l - 1] ? gres[l - 1] : nullptr;
        a.zin = (const unsigned short *)c->w[W_Z + l - 1];
        a.aout = dz[cur ^ 1];
        a.aT = dzT[cur ^ 1];
        if (sp_launch_conv(cpo, 27, true, a, s))
            return fail(c, HK_EINVAL, "no data-gradient kernel for %d -> %d channels", cpo, cpi);
        cur ^= 1;
    }
    if (grad_host) SCHK(c, hipMemcpyAsync(grad_host, c->g, sizeof(float) * np, hipMemcpyDeviceToHost, s));
    double lh = 0.0;
    SCHK(c, hipMemcpyAsync(&lh, c->loss, sizeof(double), hipMemcpyDeviceToHost, s));
    SCHK(c, hipStreamSynchronize(s));
    if (loss) *loss = lh;
    return HK_OK;
}

int hk_sp_train_step(hk_sp *c, const float *x, const float *y, int B, int D, int H, int W,
                     const hk_sp_train_desc *t, double *loss) {
    if (!c || !t) return HK_EINVAL;
    int rc = hk_sp_loss_grad(c, x, y, B, D, H, W, t->delta, t->lambda_e, t->dropout ? c->t : -1, nullptr, loss);
    if (rc) return rc;
    c->t += 1;
    cnn_launch_adamw(hk_sp_nparams(), c->p, c->g, c->m, c->v, (float)t->lr, (float)t->beta1, (float)t->beta2,
                     (float)t->eps, (float)t->weight_decay, c->t, c->s);
    pack(c);
    SCHK(c, hipStreamSynchronize(c->s));
    return HK_OK;
}

const char *hk_sp_last_error(const hk_sp *c) { return c ? c->err.c_str() : "null network"; }

}  // extern "C"
