// Host side of the switch network: parameters (FP32 masters and BF16 copies),
// AdamW state, workspace, and the forward / gradient / training calls of the
// C ABI (include/hk.h, hk_cnn_*).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hk_internal.h"
#include "hk_cnn_internal.h"

void cnn_launch_to_bf16(long long n, const float *x, unsigned short *o, hipStream_t s);
void cnn_launch_conv_fwd(int cin, int B, int D, int H, int W, const unsigned short *act,
                         const unsigned short *Wf, const float *bias, float *zout, unsigned short *aout,
                         const int *xwin, hipStream_t s);
void cnn_launch_conv_bwd_data(int B, int D, int H, int W, const unsigned short *dz,
                              const unsigned short *Wb, const float *zin, unsigned short *dzin,
                              hipStream_t s);
void cnn_launch_conv_bwd_weight(int cin, int B, int D, int H, int W, const unsigned short *act,
                                const unsigned short *dz, float *gW, float *gb, hipStream_t s);
void cnn_launch_head(long long n, const unsigned short *a4, const unsigned short *wh, const float *bh,
                     int use_mask, uint64_t seed, uint32_t step, float *logit, hipStream_t s);
void cnn_launch_head_bwd(long long n, const unsigned short *a4, const float *z4, const unsigned short *wh,
                         const float *bh, int use_mask, uint64_t seed, uint32_t step, const float *y,
                         const float *e, float lambda, unsigned short *dz4, float *gwh, double *loss,
                         hipStream_t s);
void cnn_launch_adamw(int n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2,
                      float eps, float wd, int t, hipStream_t s);
void cnn_launch_pack(const float *p, int layer_cin, long long woff, int kpad, unsigned short *Wf,
                     unsigned short *Wb, hipStream_t s);
void cnn_launch_pack_head(const float *p, long long off, unsigned short *wh, hipStream_t s);

namespace {

constexpr int NC = 32;

int cin_of(int l) { return l == 0 ? 8 : NC; }
long long w_off(int l) {
    long long o = 0;
    for (int q = 0; q < l; ++q) o += 27LL * cin_of(q) * NC + NC;
    return o;
}
int kpad_of(int l) { return (27 * cin_of(l) + 31) / 32 * 32; }

int cnn_fail(hk_cnn *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->err = buf;
    return code;
}

#define CCHK(c, x)                                                                                  \
    do {                                                                                            \
        hipError_t e_ = (x);                                                                        \
        if (e_ != hipSuccess) return cnn_fail(c, HK_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

}  // namespace

void *cnn_alloc(hk_cnn *c, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    void *p = nullptr;
    if (c->alloc) p = c->alloc(bytes, c->alloc_ctx);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    if (p) c->allocs.push_back(p);
    return p;
}

void cnn_release(hk_cnn *c, void *p) {
    if (!p) return;
    for (size_t i = 0; i < c->allocs.size(); ++i)
        if (c->allocs[i] == p) {
            c->allocs.erase(c->allocs.begin() + i);
            break;
        }
    if (c->free) c->free(p, c->alloc_ctx);
    else (void)hipFree(p);
}

// grow a workspace buffer to at least `bytes`
static void *ws(hk_cnn *c, void *&slot, size_t &cap, size_t bytes) {
    if (cap >= bytes && slot) return slot;
    (void)hipStreamSynchronize(c->s);
    cnn_release(c, slot);
    slot = cnn_alloc(c, bytes);
    cap = slot ? bytes : 0;
    return slot;
}

int cnn_pack(hk_cnn *c, hipStream_t s) {
    for (int l = 0; l < 4; ++l)
        cnn_launch_pack(c->p, cin_of(l), w_off(l), kpad_of(l), c->Wf[l], l ? c->Wb[l] : nullptr, s);
    cnn_launch_pack_head(c->p, w_off(4), c->wh, s);
    return HK_OK;
}

// Forward over B x D x H x W x 8 BF16 inputs; activations of every layer (and
// pre-activations when keep_z) stay in the workspace.  Returns a4.  With
// `pingpong` the activations alternate between those two caller buffers
// instead (layer l writes pingpong[l & 1]; no pre-activations, nothing grown).
int cnn_forward_bf16(hk_cnn *c, const unsigned short *x, int B, int D, int H, int W, bool keep_z,
                     hipStream_t s, const unsigned short **a4, unsigned short *const *pingpong,
                     const int *xwin) {
    if (D < 9 || H < 9 || W < 9) return cnn_fail(c, HK_EINVAL, "input smaller than the receptive field");
    if (pingpong && keep_z) return cnn_fail(c, HK_EINVAL, "pre-activations need the workspace");
    // the convolutions address three input planes of 32 BF16 channels from a
    // row group's first voxel with 32-bit byte offsets below 2^31
    if (3LL * H * W * NC * 2 >= (1LL << 31) - 16)
        return cnn_fail(c, HK_EINVAL, "an input plane of %d x %d voxels is beyond the convolutions' range", H, W);
    const unsigned short *in = x;
    for (int l = 0; l < 4; ++l) {
        const int d = D - 2 * (l + 1), h = H - 2 * (l + 1), w = W - 2 * (l + 1);
        const size_t n = (size_t)B * d * h * w;
        unsigned short *a = pingpong ? pingpong[l & 1]
                                     : (unsigned short *)ws(c, c->wa[l], c->wa_cap[l], n * NC * 2);
        float *z = keep_z ? (float *)ws(c, c->wz[l], c->wz_cap[l], n * NC * 4) : nullptr;
        if (!a || (keep_z && !z)) return cnn_fail(c, HK_ENOMEM, "CNN activations");
        cnn_launch_conv_fwd(cin_of(l), B, D - 2 * l, H - 2 * l, W - 2 * l, in, c->Wf[l], c->p + w_off(l) + 27LL * cin_of(l) * NC,
                            z, a, xwin, s);
        in = a;
    }
    *a4 = in;
    return HK_OK;
}

extern "C" {

int hk_cnn_nparams(void) { return (int)(w_off(4) + NC + 1); }

int hk_cnn_create(const hk_cnn_desc *d, hk_cnn **out) {
    if (!d || !out) return HK_EINVAL;
    hk_cnn *c = new hk_cnn();
    c->s = (hipStream_t)d->stream;
    c->alloc = d->alloc;
    c->free = d->free;
    c->alloc_ctx = d->alloc_ctx;
    c->seed = d->seed;
    const int np = hk_cnn_nparams();
    c->p = (float *)cnn_alloc(c, sizeof(float) * np);
    c->m = (float *)cnn_alloc(c, sizeof(float) * np);
    c->v = (float *)cnn_alloc(c, sizeof(float) * np);
    c->g = (float *)cnn_alloc(c, sizeof(float) * np);
    c->loss = (double *)cnn_alloc(c, sizeof(double));
    bool ok = c->p && c->m && c->v && c->g && c->loss;
    for (int l = 0; l < 4 && ok; ++l) {
        c->Wf[l] = (unsigned short *)cnn_alloc(c, 2 * (size_t)NC * kpad_of(l));
        c->Wb[l] = l ? (unsigned short *)cnn_alloc(c, 2 * (size_t)NC * 27 * NC) : nullptr;
        ok = c->Wf[l] && (l == 0 || c->Wb[l]);
    }
    c->wh = ok ? (unsigned short *)cnn_alloc(c, 2 * NC) : nullptr;
    if (!ok || !c->wh) {
        hk_cnn_destroy(c);
        return HK_ENOMEM;
    }
    for (int q = 0; q < 8; ++q) { c->mean[q] = 0.f; c->inv_std[q] = 1.f; }
    (void)hipMemsetAsync(c->p, 0, sizeof(float) * np, c->s);
    (void)hipMemsetAsync(c->m, 0, sizeof(float) * np, c->s);
    (void)hipMemsetAsync(c->v, 0, sizeof(float) * np, c->s);
    cnn_pack(c, c->s);
    if (hipStreamSynchronize(c->s) != hipSuccess) {
        hk_cnn_destroy(c);
        return HK_EDEVICE;
    }
    *out = c;
    return HK_OK;
}

void hk_cnn_destroy(hk_cnn *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->s);
    std::vector<void *> all = c->allocs;
    for (void *p : all) cnn_release(c, p);
    delete c;
}

int hk_cnn_set_params(hk_cnn *c, const float *params, size_t n) {
    if (!c || !params || n != (size_t)hk_cnn_nparams()) return HK_EINVAL;
    CCHK(c, hipMemcpyAsync(c->p, params, sizeof(float) * n, hipMemcpyHostToDevice, c->s));
    CCHK(c, hipMemsetAsync(c->m, 0, sizeof(float) * n, c->s));
    CCHK(c, hipMemsetAsync(c->v, 0, sizeof(float) * n, c->s));
    c->t = 0;
    cnn_pack(c, c->s);
    CCHK(c, hipStreamSynchronize(c->s));
    return HK_OK;
}

int hk_cnn_get_params(hk_cnn *c, float *params, size_t n) {
    if (!c || !params || n != (size_t)hk_cnn_nparams()) return HK_EINVAL;
    CCHK(c, hipMemcpyAsync(params, c->p, sizeof(float) * n, hipMemcpyDeviceToHost, c->s));
    CCHK(c, hipStreamSynchronize(c->s));
    return HK_OK;
}

int hk_cnn_set_norm(hk_cnn *c, const float *mean, const float *stdv) {
    if (!c || !mean || !stdv) return HK_EINVAL;
    for (int q = 0; q < 8; ++q) {
        c->mean[q] = mean[q];
        c->inv_std[q] = stdv[q] > 0.f ? 1.0f / stdv[q] : 1.0f;
    }
    return HK_OK;
}

int hk_cnn_forward(hk_cnn *c, const float *x, int B, int D, int H, int W, float *logit) {
    if (!c || !x || !logit || B <= 0) return HK_EINVAL;
    const size_t nin = (size_t)B * D * H * W * 8;
    unsigned short *xb = (unsigned short *)ws(c, c->wx, c->wx_cap, nin * 2);
    if (!xb) return cnn_fail(c, HK_ENOMEM, "CNN input");
    cnn_launch_to_bf16((long long)nin, x, xb, c->s);
    const unsigned short *a4;
    int rc = cnn_forward_bf16(c, xb, B, D, H, W, false, c->s, &a4, nullptr);
    if (rc) return rc;
    const long long n = (long long)B * (D - 8) * (H - 8) * (W - 8);
    cnn_launch_head(n, a4, c->wh, c->p + w_off(4) + NC, 0, 0, 0, logit, c->s);
    CCHK(c, hipStreamSynchronize(c->s));
    return HK_OK;
}

int hk_cnn_loss_grad(hk_cnn *c, const float *x, const float *y, const float *e, int B, int D, int H, int W,
                     float lambda, int mask_step, float *grad_host, double *loss) {
    if (!c || !x || !y || !e || B <= 0) return HK_EINVAL;
    hipStream_t s = c->s;
    const int np = hk_cnn_nparams();
    const size_t nin = (size_t)B * D * H * W * 8;
    unsigned short *xb = (unsigned short *)ws(c, c->wx, c->wx_cap, nin * 2);
    if (!xb) return cnn_fail(c, HK_ENOMEM, "CNN input");
    cnn_launch_to_bf16((long long)nin, x, xb, s);
    const unsigned short *a4;
    int rc = cnn_forward_bf16(c, xb, B, D, H, W, true, s, &a4, nullptr);
    if (rc) return rc;
    CCHK(c, hipMemsetAsync(c->g, 0, sizeof(float) * np, s));
    CCHK(c, hipMemsetAsync(c->loss, 0, sizeof(double), s));
    const long long n4 = (long long)B * (D - 8) * (H - 8) * (W - 8);
    // two ping-pong buffers for the pre-activation gradients (BF16)
    size_t maxn = (size_t)B * (D - 2) * (H - 2) * (W - 2) * NC * 2;
    unsigned short *dzA = (unsigned short *)ws(c, c->wd[0], c->wd_cap[0], maxn);
    unsigned short *dzB = (unsigned short *)ws(c, c->wd[1], c->wd_cap[1], maxn);
    if (!dzA || !dzB) return cnn_fail(c, HK_ENOMEM, "CNN gradients");
    cnn_launch_head_bwd(n4, a4, (const float *)c->wz[3], c->wh, c->p + w_off(4) + NC, mask_step >= 0,
                        c->seed, (uint32_t)(mask_step >= 0 ? mask_step : 0), y, e, lambda, dzA,
                        c->g + w_off(4), c->loss, s);
    unsigned short *dz = dzA, *dzn = dzB;
    for (int l = 3; l >= 0; --l) {
        // layer l maps activation l (input dims Dl) to l + 1
        const int Dl = D - 2 * l, Hl = H - 2 * l, Wl = W - 2 * l;
        const unsigned short *act = l ? (const unsigned short *)c->wa[l - 1] : xb;
        cnn_launch_conv_bwd_weight(cin_of(l), B, Dl, Hl, Wl, act, dz, c->g + w_off(l),
                                   c->g + w_off(l) + 27LL * cin_of(l) * NC, s);
        if (l > 0) {
            cnn_launch_conv_bwd_data(B, Dl, Hl, Wl, dz, c->Wb[l], (const float *)c->wz[l - 1], dzn, s);
            std::swap(dz, dzn);
        }
    }
    if (grad_host) CCHK(c, hipMemcpyAsync(grad_host, c->g, sizeof(float) * np, hipMemcpyDeviceToHost, s));
    double lh = 0.0;
    CCHK(c, hipMemcpyAsync(&lh, c->loss, sizeof(double), hipMemcpyDeviceToHost, s));
    CCHK(c, hipStreamSynchronize(s));
    if (loss) *loss = lh;
    return HK_OK;
}

int hk_cnn_train_step(hk_cnn *c, const float *x, const float *y, const float *e, int B, int D, int H, int W,
                      const hk_cnn_train_desc *t, double *loss) {
    if (!c || !t) return HK_EINVAL;
    int rc = hk_cnn_loss_grad(c, x, y, e, B, D, H, W, (float)t->lambda_e, t->dropout ? c->t : -1, nullptr,
                              loss);
    if (rc) return rc;
    c->t += 1;
    cnn_launch_adamw(hk_cnn_nparams(), c->p, c->g, c->m, c->v, (float)t->lr, (float)t->beta1,
                     (float)t->beta2, (float)t->eps, (float)t->weight_decay, c->t, c->s);
    cnn_pack(c, c->s);
    CCHK(c, hipStreamSynchronize(c->s));
    return HK_OK;
}

const char *hk_cnn_last_error(const hk_cnn *c) { return c ? c->err.c_str() : "null network"; }

}  // extern "C"

// ------------------------------------------------------------------------------------------
// Allocation-free forward.  Its working memory is one static device array per
// GPU: the BF16 copy of the input, then two activation buffers that the four
// layers alternate between (layer l writes buffer l & 1, reads the other or
// the input).  Kernels take the array's device address, looked up once per
// device with hipGetSymbolAddress; the array's name itself is a host-side
// stand-in and never reaches a kernel.
namespace {

constexpr size_t NOALLOC_IN = (size_t)HK_CNN_NOALLOC_MAX_VOXELS * 8 * 2;    // BF16 inputs
constexpr size_t NOALLOC_ACT = (size_t)HK_CNN_NOALLOC_MAX_VOXELS * NC * 2;  // one activation buffer
static_assert(HK_CNN_NOALLOC_SCRATCH_BYTES == NOALLOC_IN + 2 * NOALLOC_ACT, "scratch layout");

__device__ __align__(256) unsigned char scratch[HK_CNN_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mu;
unsigned char *noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// device address of this device's scratch array (looked up on first use)
int noalloc_scratch(hk_cnn *c, unsigned char **out) {
    int dev = -1;
    CCHK(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return cnn_fail(c, HK_EDEVICE, "device %d beyond the %d the scratch table covers", dev,
                        NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (!noalloc_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return cnn_fail(c, HK_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                            hipGetErrorString(e));
        noalloc_ptr[dev] = (unsigned char *)p;
    }
    *out = noalloc_ptr[dev];
    return HK_OK;
}

}  // namespace

extern "C" {

int hk_cnn_forward_noalloc(hk_cnn *c, const float *x, int B, int D, int H, int W, float *logit) {
    if (!c || !x || !logit || B <= 0 || D <= 0 || H <= 0 || W <= 0) return HK_EINVAL;
    const long long vox = (long long)B * D * H * W;
    if (vox > HK_CNN_NOALLOC_MAX_VOXELS)
        return cnn_fail(c, HK_EINVAL, "hk_cnn_forward_noalloc: %lld input voxels exceed the limit of %d",
                        vox, HK_CNN_NOALLOC_MAX_VOXELS);
    if (D < 9 || H < 9 || W < 9) return cnn_fail(c, HK_EINVAL, "input smaller than the receptive field");
    unsigned char *base = nullptr;
    int rc = noalloc_scratch(c, &base);
    if (rc) return rc;
    unsigned short *xb = (unsigned short *)base;
    unsigned short *pp[2] = {(unsigned short *)(base + NOALLOC_IN),
                             (unsigned short *)(base + NOALLOC_IN + NOALLOC_ACT)};
    cnn_launch_to_bf16(vox * 8, x, xb, c->s);
    const unsigned short *a4;
    rc = cnn_forward_bf16(c, xb, B, D, H, W, false, c->s, &a4, pp);
    if (rc) return rc;
    const long long n = (long long)B * (D - 8) * (H - 8) * (W - 8);
    cnn_launch_head(n, a4, c->wh, c->p + w_off(4) + NC, 0, 0, 0, logit, c->s);
    CCHK(c, hipGetLastError());
    return HK_OK;
}

}  // extern "C"
