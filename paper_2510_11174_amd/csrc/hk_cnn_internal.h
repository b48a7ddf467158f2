// State of a switch network context (host side); shared by the CNN calls and
// the simulation's CNN switch mode.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/hk.h"

struct hk_cnn {
    hipStream_t s = nullptr;
    hk_alloc_fn alloc = nullptr;
    hk_free_fn free = nullptr;
    void *alloc_ctx = nullptr;
    uint64_t seed = 0;
    float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;  // FP32 masters, AdamW moments, gradient
    double *loss = nullptr;
    unsigned short *Wf[4] = {}, *Wb[4] = {}, *wh = nullptr;         // BF16 copies
    float mean[8], inv_std[8];
    int t = 0;                                                       // AdamW steps taken
    // workspace, grown on demand
    void *wx = nullptr, *wa[4] = {}, *wz[4] = {}, *wd[2] = {};
    size_t wx_cap = 0, wa_cap[4] = {}, wz_cap[4] = {}, wd_cap[2] = {};
    std::vector<void *> allocs;
    std::string err;
};

void *cnn_alloc(hk_cnn *c, size_t bytes);
void cnn_release(hk_cnn *c, void *p);
// xwin (device, may be null): only output x columns xwin[0] .. xwin[1] (+ the
// halo the next layers read) are computed, for B = 1 on the switch's grid
int cnn_forward_bf16(hk_cnn *c, const unsigned short *x, int B, int D, int H, int W, bool keep_z,
                     hipStream_t s, const unsigned short **a4, unsigned short *const *pingpong,
                     const int *xwin = nullptr);
