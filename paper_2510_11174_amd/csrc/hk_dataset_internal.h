// Training set of the learned switch, held in device memory: snapshots of a
// simulation's node inputs with their labels (hk_dump_training appends, the
// crop sampler of hk_train reads).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/hk.h"

// One snapshot: nodes [D][H][W] (z, y, x; x fastest), per node the 8 network
// inputs before normalization and the conversion energy e (9 floats), the
// label (0/1) and the threshold criterion's flags at the snapshot's step.
struct DsSnap {
    float *raw9;
    uint8_t *y, *thr;
    int D, H, W, per_x;
    double dv;
};

struct hk_dataset {
    hipStream_t s = nullptr;
    hk_alloc_fn alloc = nullptr;
    hk_free_fn free = nullptr;
    void *alloc_ctx = nullptr;
    std::vector<DsSnap> snaps;
    DsSnap *dtab = nullptr;       // device copy of snaps (crop sampler)
    size_t dtab_cap = 0;
    bool dirty = true;
    std::vector<void *> allocs;
    std::string err;
};

void *ds_alloc(hk_dataset *d, size_t bytes);
void ds_release(hk_dataset *d, void *p);
int ds_fail(hk_dataset *d, int code, const char *fmt, ...);
// a new snapshot of D x H x W nodes; its raw9 is left for the caller to fill
// and its labels are zeroed on stream s
int ds_append(hk_dataset *d, int D, int H, int W, int per_x, double dv, hipStream_t s, DsSnap **out);
