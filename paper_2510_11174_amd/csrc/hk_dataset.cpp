// Host side of the learned switch's training set (include/hk.h, hk_dataset_*
// and hk_train): snapshot storage in device memory, per-channel statistics,
// the training loop over device-sampled crops, and prediction over a whole
// snapshot.  hk_dump_training, which fills the set from a simulation, lives
// with the simulation (hk_api.cpp).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "hk_internal.h"
#include "hk_cnn_internal.h"
#include "hk_dataset_internal.h"

void ds_launch_crops(const DsSnap *tab, int nsnap, uint64_t seed, int it, int B, const float *mean,
                     const float *inv_std, float *x, float *y, float *e, hipStream_t s);
void ds_launch_pad(const DsSnap &S, const float *mean, const float *inv_std, float *x, hipStream_t s);
void ds_launch_stats(const float *raw9, long long n, double *acc, hipStream_t s);

#define DCHK(d, x)                                                                                 \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) return ds_fail(d, HK_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

int ds_fail(hk_dataset *d, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    d->err = buf;
    return code;
}

void *ds_alloc(hk_dataset *d, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    void *p = nullptr;
    if (d->alloc) p = d->alloc(bytes, d->alloc_ctx);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    if (p) d->allocs.push_back(p);
    return p;
}

void ds_release(hk_dataset *d, void *p) {
    if (!p) return;
    for (size_t i = 0; i < d->allocs.size(); ++i)
        if (d->allocs[i] == p) {
            d->allocs.erase(d->allocs.begin() + i);
            break;
        }
    if (d->free) d->free(p, d->alloc_ctx);
    else (void)hipFree(p);
}

int ds_append(hk_dataset *d, int D, int H, int W, int per_x, double dv, hipStream_t s, DsSnap **out) {
    const size_t n = (size_t)D * H * W;
    DsSnap S{};
    S.raw9 = (float *)ds_alloc(d, sizeof(float) * 9 * n);
    S.y = (uint8_t *)ds_alloc(d, n);
    S.thr = (uint8_t *)ds_alloc(d, n);
    if (!S.raw9 || !S.y || !S.thr) {
        ds_release(d, S.raw9);
        ds_release(d, S.y);
        ds_release(d, S.thr);
        return ds_fail(d, HK_ENOMEM, "snapshot of %zu nodes", n);
    }
    S.D = D; S.H = H; S.W = W; S.per_x = per_x; S.dv = dv;
    DCHK(d, hipMemsetAsync(S.y, 0, n, s));
    d->snaps.push_back(S);
    d->dirty = true;
    *out = &d->snaps.back();
    return HK_OK;
}

namespace {

int upload_table(hk_dataset *d) {
    if (!d->dirty) return HK_OK;
    const size_t bytes = sizeof(DsSnap) * d->snaps.size();
    if (d->dtab_cap < bytes) {
        DCHK(d, hipStreamSynchronize(d->s));
        ds_release(d, d->dtab);
        d->dtab = (DsSnap *)ds_alloc(d, 2 * bytes);
        d->dtab_cap = d->dtab ? 2 * bytes : 0;
        if (!d->dtab) return ds_fail(d, HK_ENOMEM, "snapshot table");
    }
    DCHK(d, hipMemcpyAsync(d->dtab, d->snaps.data(), bytes, hipMemcpyHostToDevice, d->s));
    DCHK(d, hipStreamSynchronize(d->s));
    d->dirty = false;
    return HK_OK;
}

}  // namespace

extern "C" {

int hk_dataset_create(const hk_cnn_desc *desc, hk_dataset **out) {
    if (!desc || !out) return HK_EINVAL;
    hk_dataset *d = new hk_dataset();
    d->s = (hipStream_t)desc->stream;
    d->alloc = desc->alloc;
    d->free = desc->free;
    d->alloc_ctx = desc->alloc_ctx;
    *out = d;
    return HK_OK;
}

void hk_dataset_destroy(hk_dataset *d) {
    if (!d) return;
    (void)hipStreamSynchronize(d->s);
    while (!d->allocs.empty()) ds_release(d, d->allocs.back());
    delete d;
}

int hk_dataset_size(const hk_dataset *d) { return d ? (int)d->snaps.size() : 0; }

int hk_dataset_get(hk_dataset *d, int k, int *dims, float *raw, float *ehat, uint8_t *y, uint8_t *thr,
                   size_t n) {
    if (!d || k < 0 || k >= (int)d->snaps.size()) return HK_EINVAL;
    const DsSnap &S = d->snaps[k];
    const size_t nodes = (size_t)S.D * S.H * S.W;
    if (dims) { dims[0] = S.D; dims[1] = S.H; dims[2] = S.W; }
    if (!raw && !ehat && !y && !thr) return HK_OK;
    if (n != nodes) return ds_fail(d, HK_EINVAL, "node count %zu, snapshot has %zu", n, nodes);
    std::vector<float> h;
    if (raw || ehat) {
        h.resize(9 * nodes);
        DCHK(d, hipMemcpyAsync(h.data(), S.raw9, sizeof(float) * 9 * nodes, hipMemcpyDeviceToHost, d->s));
    }
    if (y) DCHK(d, hipMemcpyAsync(y, S.y, nodes, hipMemcpyDeviceToHost, d->s));
    if (thr) DCHK(d, hipMemcpyAsync(thr, S.thr, nodes, hipMemcpyDeviceToHost, d->s));
    DCHK(d, hipStreamSynchronize(d->s));
    for (size_t v = 0; v < nodes && (raw || ehat); ++v) {
        if (raw) for (int q = 0; q < 8; ++q) raw[8 * v + q] = h[9 * v + q];
        if (ehat) ehat[v] = h[9 * v + 8];
    }
    return HK_OK;
}

int hk_dataset_stats(hk_dataset *d, float *mean, float *stdv) {
    if (!d || !mean || !stdv) return HK_EINVAL;
    if (d->snaps.empty()) return ds_fail(d, HK_EINVAL, "empty training set");
    double *acc = (double *)ds_alloc(d, sizeof(double) * 16);
    if (!acc) return ds_fail(d, HK_ENOMEM, "statistics");
    DCHK(d, hipMemsetAsync(acc, 0, sizeof(double) * 16, d->s));
    long long total = 0;
    for (const DsSnap &S : d->snaps) {
        const long long n = (long long)S.D * S.H * S.W;
        ds_launch_stats(S.raw9, n, acc, d->s);
        total += n;
    }
    double h[16];
    const hipError_t e1 = hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, d->s);
    const hipError_t e2 = hipStreamSynchronize(d->s);
    ds_release(d, acc);
    if (e1 != hipSuccess || e2 != hipSuccess) return ds_fail(d, HK_EDEVICE, "statistics: %s",
                                                             hipGetErrorString(e1 ? e1 : e2));
    for (int q = 0; q < 8; ++q) {
        const double m = h[q] / (double)total;
        const double var = std::fmax(0.0, h[8 + q] / (double)total - m * m);
        mean[q] = (float)m;
        stdv[q] = var > 0.0 ? (float)std::sqrt(var) : 1.0f;
    }
    return HK_OK;
}

int hk_train(hk_cnn *c, hk_dataset *d, int iters, int B, const hk_cnn_train_desc *t, uint64_t seed,
             double *losses) {
    if (!c || !d || !t || iters < 0 || B < 1 || B > 1024) return HK_EINVAL;
    if (d->snaps.empty()) return ds_fail(d, HK_EINVAL, "empty training set");
    if (iters == 0) return HK_OK;
    int rc = upload_table(d);
    if (rc) return rc;
    const size_t nx = (size_t)B * 24 * 24 * 24 * 8, ny = (size_t)B * 16 * 16 * 16;
    float *x = (float *)ds_alloc(d, sizeof(float) * nx);
    float *y = (float *)ds_alloc(d, sizeof(float) * ny);
    float *e = (float *)ds_alloc(d, sizeof(float) * ny);
    if (!x || !y || !e) {
        ds_release(d, x); ds_release(d, y); ds_release(d, e);
        return ds_fail(d, HK_ENOMEM, "crop buffers for a batch of %d", B);
    }
    rc = HK_OK;
    for (int it = 0; it < iters && rc == HK_OK; ++it) {
        // crops are keyed by the network's AdamW step: repeated calls draw new ones
        ds_launch_crops(d->dtab, (int)d->snaps.size(), seed, c->t, B, c->mean, c->inv_std, x, y, e, c->s);
        double loss = 0.0;
        rc = hk_cnn_train_step(c, x, y, e, B, 24, 24, 24, t, &loss);
        if (rc) ds_fail(d, rc, "training step %d: %s", it, c->err.c_str());
        else if (losses) losses[it] = loss;
    }
    (void)hipStreamSynchronize(c->s);
    ds_release(d, x); ds_release(d, y); ds_release(d, e);
    return rc;
}

int hk_dataset_predict(hk_cnn *c, hk_dataset *d, int k, float *logit) {
    if (!c || !d || !logit || k < 0 || k >= (int)d->snaps.size()) return HK_EINVAL;
    const DsSnap &S = d->snaps[k];
    const size_t n = (size_t)(S.D + 8) * (S.H + 8) * (S.W + 8) * 8;
    float *x = (float *)ds_alloc(d, sizeof(float) * n);
    if (!x) return ds_fail(d, HK_ENOMEM, "padded snapshot");
    DCHK(d, hipStreamSynchronize(d->s));   // the snapshot was written on the dataset's stream
    ds_launch_pad(S, c->mean, c->inv_std, x, c->s);
    int rc = hk_cnn_forward(c, x, 1, S.D + 8, S.H + 8, S.W + 8, logit);
    if (rc) ds_fail(d, rc, "forward: %s", c->err.c_str());
    (void)hipStreamSynchronize(c->s);
    ds_release(d, x);
    return rc;
}

const char *hk_dataset_last_error(const hk_dataset *d) { return d ? d->err.c_str() : "null dataset"; }

}  // extern "C"
