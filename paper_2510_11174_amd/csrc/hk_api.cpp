// C ABI of the hybrid fluid-kinetic step: context, device memory, the step
// schedule and the host-side accessors.  Every arithmetic step of the method
// runs in the kernels of k_*.hip; this file only orders launches, owns memory
// and moves data across the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hk_internal.h"
#include "hk_cnn_internal.h"
#include "hk_dataset_internal.h"

void cnn_launch_inputs(const GridP &g, real *const f[9], const real *mom, const float mean[8],
                       const float inv_std[8], unsigned short *x, const int *xwin, hipStream_t s);
void cnn_launch_node_raw(const GridP &g, real *const f[9], const real *mom, float *out, hipStream_t s);
void cnn_launch_node_state(const GridP &g, real *const f[9], const double *rho, float *out, hipStream_t s);
void cnn_launch_decide(const GridP &g, const unsigned short *a4, const unsigned short *wh, const float *bh,
                       uint64_t seed, uint32_t eval, uint8_t *hot, uint8_t *notcold, int *nfall,
                       float *pmean, const int *xwin, hipStream_t s);
void cnn_launch_window(const GridP &g, const real *mom, int margin, int *win, hipStream_t s);

// device status words copied to the host once per merge (see hk_sim::status)
#define HK_NSTATUS 32

namespace {

// Physical constants (CODATA 2018) for the SI scale of ionization and QED.
constexpr double PHYS_C = 299792458.0, PHYS_ME = 9.1093837015e-31, PHYS_QE = 1.602176634e-19;
constexpr double PHYS_HBAR = 1.054571817e-34, PHYS_EA = 5.14220674763e11;
constexpr double PHYS_TA = 2.4188843265857e-17, PHYS_HARTREE_EV = 27.211386245988;
constexpr double PI = 3.14159265358979323846;

struct DevSpecies {
    hk_species_desc d{};
    int has_z = 0, has_tau = 0;
    PArr buf[2]{};
    int cur = 0;
    long long capacity = 0;
    long long *off = nullptr;  // device [ntiles]
    int *cap = nullptr;        // device [ntiles]
    int *nf[2] = {nullptr, nullptr}, *nb[2] = {nullptr, nullptr};  // bin front / back counts
    std::vector<long long> h_off;
    std::vector<int> h_cap;
    int max_cap = 0;
    long long mig0 = 0;        // slot of the first per-tile mover region in each bin buffer
    long long alloc_slots = 0; // slots allocated per bin buffer (both alike)
    long long *moff = nullptr;
    int *mcap = nullptr;
    int *active = nullptr;     // immobile ionizable ions: ions below z_max per tile
    PArr inbox{}, fail{};
    PArr *inbox_dev = nullptr;    // device copy of the inbox descriptor (the push reads it
                                  // only when a mover region overflows)
    int inbox_cap = 0;
    long long *g_off0 = nullptr;  // device {0}
    int *g_capmax = nullptr;      // device {INT_MAX}
    real *fn = nullptr, *fu[3] = {nullptr, nullptr, nullptr};  // fluid density and momentum
    real *fs = nullptr;           // warm fluid: entropy density n K, K = p / n^gamma_ad
    real *fn2 = nullptr, *fs2 = nullptr;   // the fluid pass writes n and S here, then swaps
    double *macc = nullptr;       // particles the push absorbed into the fluid this step (5 grid arrays)
    int *xr = nullptr;            // device [8]: x window of the fluid (see launch_fluid)
    IonP *ion = nullptr;          // device rate constants
    long long reserve_hint = 0;   // expected peak count (ionization targets)
    unsigned *umax2 = nullptr;    // device [ntiles]: bound on |u|^2 (float bits) since the
                                  // last switch evaluation, raised by push, ionization, spawn
    bool umax_ok = false;         // false: particles changed outside those kernels
    // an empty species is not pushed: `idle` when its bins were empty at the
    // last push and nothing arrived since (inbox entries, counted per step)
    bool idle = false;
    long long arrived = 0;
};

}  // namespace

struct hk_sim {
    GridP g{};
    double *qed_tab = nullptr;   // device copy of the QED tables (enable_qed)
    hk_cnn *cnn = nullptr;       // learned switch (borrowed)
    uint32_t cnn_evals = 0;      // evaluations so far (dropout counter)
    unsigned short *cnn_x = nullptr;   // padded BF16 node inputs of the grid
    int *cnn_nfall = nullptr;    // [0] nodes that kept the threshold decision, last evaluation;
                                 // [4..7] the network's x window (k_cnn_window)
    float *cnn_raw = nullptr;    // node inputs and conversion energy (hk_node_inputs)
    uint8_t *lab = nullptr;      // training-label condition per node (hk_dump_training)
    uint8_t *dil = nullptr;      // 2 nn bytes: the dilation's one-axis passes
    double a_s = 0.0;            // Schwinger field in normalized units
    int photon_sp = -1, electron_sp = -1, positron_sp = -1;   // QED sinks (first of each kind)
    hk_grid_desc gd{};
    hk_laser_desc las{};
    hk_run_desc run{};
    int nsp = 0;
    DevSpecies sp[HK_MAX_SPECIES];
    hipStream_t s = nullptr;
    real *fblock = nullptr;      // the 9 field arrays, contiguous
    real *falt = nullptr;        // a second set of E and B: the fused field update writes there
    real *f_alt[6] = {};         // and the two sets swap (f[0..5] is always the current one)
    real *f[9]{};
    jglob_t *jg = nullptr;       // particle current of the step (3 arrays), zero between steps
    real *mur_old = nullptr;
    uint8_t *sw = nullptr, *calm = nullptr, *hot = nullptr, *notcold = nullptr;
    real *mom = nullptr;         // switch moments (7 grid arrays)
    int *spawn_list = nullptr;   // nodes that spawn this step (one species at a time)
    int *spawn_n = nullptr;      // their count
    real *fluid_scratch = nullptr;
    double *gauss0 = nullptr, *tmp_a = nullptr, *tmp_b = nullptr;
    double *dsum = nullptr;      // diagnostic accumulators
    double *ledger = nullptr;    // [0] conversion loss, [1] ionization, [2] photons
    int *status = nullptr;       // [0] error bits, [1 + 2s] inbox count, [2 + 2s] fail count,
                                 // [13] spawns deferred for lack of inbox room, [16 + s] push
                                 // work items of species s at its last push (0: bins empty)
    int *h_status = nullptr;     // pinned
    hipEvent_t status_ev = nullptr;  // recorded after the status copy to h_status
    int have_gauss0 = 0;
    int64_t step = 0;
    double t = 0;
    int poisoned = 0;
    std::string err;
    std::vector<void *> allocs;
    bool timing = false;
    double timers[HK_NTIMERS]{};
    // timing events: recorded without waiting, resolved when the timers are read
    std::vector<hipEvent_t> ev_free;
    struct Span { hipEvent_t a, b; int slot; };
    std::vector<Span> spans;
    hipEvent_t last_mark = nullptr;
    unsigned long long *dstat = nullptr;   // [0] particles pushed, [1] tiles pushed
    unsigned *wmax = nullptr;       // per species: bound on |w| (FP32 bits), never lowered
    int2 *plan = nullptr;           // push work items (tile, chunk), rebuilt before every push
    int *plan_ctl = nullptr;        // [0] items of the current plan, then the planner's counts
    unsigned long long stat0[2]{};  // device counters when timing was enabled
    double fallback_fraction = 0;
};

namespace {

int fail(hk_sim *S, int code, const char *fmt, ...) {
    if (S) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        S->err = buf;
        if (code == HK_EDEVICE || code == HK_ENUMERIC || code == HK_EOVERFLOW) S->poisoned = 1;
    }
    return code;
}

#define HIPCHK(S, x)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) return fail(S, HK_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

void *dalloc(hk_sim *S, size_t bytes, bool zero = true) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (S->run.alloc) p = S->run.alloc(bytes, S->run.alloc_ctx);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    if (p) {
        S->allocs.push_back(p);
        if (zero) launch_zero(p, bytes, S->s);
    }
    return p;
}

void dfree(hk_sim *S, void *p) {
    if (!p) return;
    auto it = std::find(S->allocs.begin(), S->allocs.end(), p);
    if (it != S->allocs.end()) S->allocs.erase(it);
    if (S->run.free) S->run.free(p, S->run.alloc_ctx);
    else (void)hipFree(p);
}

// One allocation per particle array set, fields on 256-byte boundaries.  Slots
// are written before they are read (bins count only filled slots); cells start
// at -1, the mark of an empty slot, and nothing else is cleared.
bool alloc_parr(hk_sim *S, PArr &a, long long n, int has_z, int has_tau) {
    a = PArr{};
    if (n <= 0) n = 1;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t s4 = al(4 * (size_t)n), s8 = al(8 * (size_t)n), sr = al(sizeof(real) * (size_t)n);
    const size_t total = s4 + 7 * sr + s8 + (has_z ? s4 : 0) + (has_tau ? s8 : 0);
    char *base = (char *)dalloc(S, total, false);
    if (!base) return false;
    size_t o = 0;
    a.cell = (int *)(base + o); o += s4;
    real **rs[] = {&a.rx, &a.ry, &a.rz, &a.ux, &a.uy, &a.uz, &a.w};
    for (real **r : rs) { *r = (real *)(base + o); o += sr; }
    a.id = (uint64_t *)(base + o); o += s8;
    if (has_z) { a.zc = (int *)(base + o); o += s4; }
    if (has_tau) { a.tau = (double *)(base + o); o += s8; }
    launch_fill32(a.cell, (size_t)n, 0xFFFFFFFFu, S->s);
    return true;
}

// Every field of b at the same byte distance from that of a.
bool same_layout(const PArr &a, const PArr &b) {
    const char *pa[] = {(const char *)a.rx, (const char *)a.ry, (const char *)a.rz, (const char *)a.ux,
                        (const char *)a.uy, (const char *)a.uz, (const char *)a.w, (const char *)a.id,
                        (const char *)a.zc, (const char *)a.tau};
    const char *pb[] = {(const char *)b.rx, (const char *)b.ry, (const char *)b.rz, (const char *)b.ux,
                        (const char *)b.uy, (const char *)b.uz, (const char *)b.w, (const char *)b.id,
                        (const char *)b.zc, (const char *)b.tau};
    const long long d = (const char *)b.cell - (const char *)a.cell;
    for (int k = 0; k < 10; ++k)
        if ((pa[k] == nullptr) != (pb[k] == nullptr) || (pa[k] && pb[k] - pa[k] != d)) return false;
    return true;
}

// The same arrays from slot k on.
PArr shifted(const PArr &a, long long k) {
    PArr v = a;
    v.cell += k; v.rx += k; v.ry += k; v.rz += k; v.ux += k; v.uy += k; v.uz += k; v.w += k;
    v.id += k;
    if (v.zc) v.zc += k;
    if (v.tau) v.tau += k;
    return v;
}

void free_parr(hk_sim *S, PArr &a) {
    dfree(S, a.cell);   // the base of the set's one allocation
    a = PArr{};
}

Bins bins(const DevSpecies &d, int which) { return Bins{d.nf[which], d.nb[which]}; }
Bins cur_bins(const DevSpecies &d) { return bins(d, d.cur); }

SpecP specp(const DevSpecies &d) {
    SpecP p{};
    p.kind = d.d.kind;
    p.mobile = d.d.mobile;
    p.fluid = d.d.fluid;
    p.ionizable = d.d.ionizable;
    p.z_max = d.d.z_max;
    p.qed = d.d.qed;
    p.has_z = d.has_z;
    p.has_tau = d.has_tau;
    p.q = (real)d.d.charge;
    p.m = (real)d.d.mass;
    p.qm = d.d.mass > 0 ? (real)(d.d.charge / d.d.mass) : (real)0;
    p.off = d.off;
    p.cap = d.cap;
    return p;
}

double profile(const hk_species_desc &d, double x) {
    switch (d.profile) {
    case HK_PROF_UNIFORM: return d.n0;
    case HK_PROF_RAMP: return x < d.x0 ? 0.0 : d.n0 * std::min(1.0, (x - d.x0) / d.length);
    case HK_PROF_FOIL: return (x >= d.x0 && x < d.x0 + d.length) ? d.n0 : 0.0;
    default: return 0.0;
    }
}

// Particles a species starts with: ppc in every cell whose centre has n > 0.
long long initial_count(const hk_grid_desc &g, const hk_species_desc &d) {
    if (d.ppc <= 0 || d.profile == HK_PROF_NONE) return 0;
    long long cols = 0;
    for (int x = 0; x < g.nx; ++x)
        if (profile(d, (x + 0.5) * g.dx) > 0) cols++;
    return cols * (long long)g.ny * g.nz * d.ppc;
}

// Re-bin a species from its current bins plus unbinned lists into a fresh
// layout whose per-tile capacity leaves headroom for density changes.
// list_max[l] bounds the entries of list l (its capacity).
int rebuild(hk_sim *S, int isp, bool use_tiles, PArr *lists, int **list_n, const long long *list_max,
            int nlists) {
    DevSpecies &D = S->sp[isp];
    S->timers[7] += 1;   // re-bin count (reported with the timers)
    const GridP &g = S->g;
    const int nt = g.ntiles;
    int *newcnt = (int *)dalloc(S, sizeof(int) * nt);
    if (!newcnt) return fail(S, HK_ENOMEM, "rebuild: counts");
    PArr cur = D.buf[D.cur];
    if (use_tiles && D.capacity > 0)
        launch_count_groups(g, cur, D.off, D.nf[D.cur], D.nb[D.cur], D.cap, nt, D.max_cap, newcnt, S->s);
    for (int l = 0; l < nlists; ++l)
        launch_count_groups(g, lists[l], D.g_off0, list_n[l], nullptr, D.g_capmax, 1, list_max[l],
                            newcnt, S->s);
    std::vector<int> h(nt);
    HIPCHK(S, hipMemcpyAsync(h.data(), newcnt, sizeof(int) * nt, hipMemcpyDeviceToHost, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    // capacity: three times the larger of the tile's count and the species'
    // mean count per tile, plus 256 slots, at least the reserve hint share.
    // A large species (over 2^26 particles, as in a 512 x 256 x 256 box with a
    // dense target) takes twice its count and a floor of 1024 instead of the
    // mean in tiles it barely fills, with an eighth of slack instead of a
    // quarter: two buffers of 2^28 particles at three times would take a
    // quarter of the 288 GB HBM, and the spare vacuum tiles most of it.  Local
    // density spikes (a laser snow-plough) then rarely overflow a bin; spare
    // slots cost memory only, never traffic (kernels touch occupied slots).
    long long hint_per_tile = D.reserve_hint > 0 ? (D.reserve_hint + nt - 1) / nt : 0;
    long long hsum = 0;
    for (int t = 0; t < nt; ++t) hsum += h[t];
    const long long mean = (hsum + nt - 1) / nt;
    const bool large = std::max(hsum, D.reserve_hint) > (1LL << 26);
    const long long factor = large ? 2 : 3;
    const long long tfloor = large ? std::min<long long>(mean, 1024) : mean;
    std::vector<long long> off(nt), moff(nt);
    std::vector<int> cap(nt), mcap(nt);
    long long total = 0, mtotal = 0;
    int maxc = 0;
    // Lay the bins out with a fraction sg of each tile's headroom above its
    // count (1: the capacity above); below 1 a tile keeps at least a quarter
    // of its count and 256 slots of room, and its reserve hint share.
    auto lay = [&](double sg) {
        total = mtotal = 0;
        maxc = 0;
        for (int t = 0; t < nt; ++t) {
            long long c = factor * std::max<long long>(h[t], tfloor) + 256;
            long long hc = hint_per_tile + hint_per_tile / 4 + 128;
            c = std::max(c, std::min<long long>(hc, INT_MAX / 4));
            if (sg < 1.0) {
                const long long lo = std::max<long long>(h[t] + h[t] / 4 + 256, std::min(c, hc));
                c = std::max(lo, h[t] + (long long)std::ceil(sg * (double)(c - h[t])));
            }
            c = (c + 63) & ~63LL;
            off[t] = total;
            cap[t] = (int)c;
            total += c;
            maxc = std::max(maxc, (int)c);
            long long m = (c / 4 + 63) & ~63LL;
            moff[t] = mtotal;
            mcap[t] = (int)m;
            mtotal += m;
        }
        return total + (D.d.mobile ? mtotal : 0);
    };
    // each bin buffer carries the per-tile mover regions after its bins.  The
    // spare buffer (the push's output, idle now) takes the scatter when it is
    // large enough, with less headroom in every tile if need be (a bin that
    // fills up sooner costs a re-bin, milliseconds; a new pair of buffers of a
    // large species costs a fraction of a second of allocation); otherwise both
    // are allocated anew with a quarter of slack, so that re-binning a large
    // species rarely allocates
    long long slots = lay(1.0);
    const bool spare = D.buf[1 - D.cur].cell != nullptr;
    if (spare && slots > D.alloc_slots) {
        if (lay(0.0) <= D.alloc_slots) {
            double a = 0.0, b = 1.0;
            for (int it = 0; it < 24; ++it) {
                const double m = 0.5 * (a + b);
                if (lay(m) <= D.alloc_slots) a = m;
                else b = m;
            }
            slots = lay(a);
        } else {
            slots = lay(1.0);
        }
    }
    const bool reuse = spare && D.alloc_slots >= slots;
    PArr nbuf[2];
    if (!reuse) {
        const long long n_alloc = slots + (large ? slots / 8 : slots / 4);
        // the idle buffer holds nothing: free it before the new pair is taken,
        // so the peak is the current buffer plus the new pair
        HIPCHK(S, hipStreamSynchronize(S->s));
        free_parr(S, D.buf[1 - D.cur]);
        D.buf[1 - D.cur] = PArr{};
        if (!alloc_parr(S, nbuf[0], n_alloc, D.has_z, D.has_tau) ||
            !alloc_parr(S, nbuf[1], n_alloc, D.has_z, D.has_tau)) {
            free_parr(S, nbuf[0]);
            free_parr(S, nbuf[1]);
            S->poisoned = 1;
            return fail(S, HK_ENOMEM, "rebuild: %lld particle slots", n_alloc);
        }
        // the push addresses its output through the input's field pointers plus
        // one byte distance: both buffers must have the same layout
        if (!same_layout(nbuf[0], nbuf[1])) {
            S->poisoned = 1;
            return fail(S, HK_ENOMEM, "rebuild: buffer layouts differ");
        }
        D.alloc_slots = n_alloc;
    }
    const int dst_i = reuse ? 1 - D.cur : 0;
    const PArr dst = reuse ? D.buf[dst_i] : nbuf[0];
    long long *doff = (long long *)dalloc(S, sizeof(long long) * nt);
    long long *dmoff = (long long *)dalloc(S, sizeof(long long) * nt);
    int *dcap = (int *)dalloc(S, sizeof(int) * nt);
    int *dmcap = (int *)dalloc(S, sizeof(int) * nt);
    // per buffer one block of 3 nt counters: front fills, back fills, mover
    // ranks (cleared together before a push into that buffer)
    int *dfill = (int *)dalloc(S, sizeof(int) * 3 * nt);
    int *f1 = (int *)dalloc(S, sizeof(int) * 3 * nt);
    // the idle buffer may be gone already: a failure from here on leaves the
    // species without a push output, and the context is unusable
    if (!doff || !dmoff || !dcap || !dmcap || !dfill || !f1) {
        S->poisoned = 1;
        return fail(S, HK_ENOMEM, "rebuild: tables");
    }
    HIPCHK(S, hipMemcpyAsync(doff, off.data(), sizeof(long long) * nt, hipMemcpyHostToDevice, S->s));
    HIPCHK(S, hipMemcpyAsync(dmoff, moff.data(), sizeof(long long) * nt, hipMemcpyHostToDevice, S->s));
    HIPCHK(S, hipMemcpyAsync(dcap, cap.data(), sizeof(int) * nt, hipMemcpyHostToDevice, S->s));
    HIPCHK(S, hipMemcpyAsync(dmcap, mcap.data(), sizeof(int) * nt, hipMemcpyHostToDevice, S->s));
    if (use_tiles && D.capacity > 0)
        launch_scatter_groups(g, cur, D.off, D.nf[D.cur], D.nb[D.cur], D.cap, nt, D.max_cap, dst,
                              doff, dfill, D.has_z, D.has_tau, S->s);
    for (int l = 0; l < nlists; ++l)
        launch_scatter_groups(g, lists[l], D.g_off0, list_n[l], nullptr, D.g_capmax, 1, list_max[l],
                              dst, doff, dfill, D.has_z, D.has_tau, S->s);
    HIPCHK(S, hipStreamSynchronize(S->s));
    if (!reuse) {
        free_parr(S, D.buf[0]);
        free_parr(S, D.buf[1]);
        D.buf[0] = nbuf[0];
        D.buf[1] = nbuf[1];
    }
    int *olds[] = {D.nf[0], D.nf[1], D.cap, D.mcap};
    for (int *q : olds) dfree(S, q);
    dfree(S, D.off); dfree(S, D.moff);
    dfree(S, newcnt);
    D.mig0 = total;
    D.cur = dst_i;
    D.off = doff;
    D.cap = dcap;
    D.moff = dmoff;
    D.mcap = dmcap;
    // the scatter fill counts are the new front counts of the current buffer
    D.nf[dst_i] = dfill;
    D.nf[1 - dst_i] = f1;
    D.nb[dst_i] = dfill + nt;
    D.nb[1 - dst_i] = f1 + nt;
    D.capacity = total;
    D.max_cap = maxc;
    D.idle = false;
    D.h_off = off;
    D.h_cap = cap;
    if (D.d.ionizable) {
        dfree(S, D.active);
        D.active = (int *)dalloc(S, sizeof(int) * nt);
        if (!D.active) {
            S->poisoned = 1;
            return fail(S, HK_ENOMEM, "rebuild: active counts");
        }
        launch_count_active(g, specp(D), D.buf[D.cur], cur_bins(D), D.d.z_max, D.active, S->s);
    }
    return HK_OK;
}

// Raise species isp's weight bound to at least w (host side).
int raise_wmax(hk_sim *S, int isp, double w) {
    unsigned cur = 0;
    HIPCHK(S, hipMemcpyAsync(&cur, S->wmax + isp, sizeof(unsigned), hipMemcpyDeviceToHost, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    float f = (float)std::fabs(w);
    f = std::nextafter(f, INFINITY);   // round up: a bound, not an estimate
    unsigned bits;
    std::memcpy(&bits, &f, 4);
    if (bits > cur) HIPCHK(S, hipMemcpyAsync(S->wmax + isp, &bits, sizeof(unsigned), hipMemcpyHostToDevice, S->s));
    return HK_OK;
}

int ensure_inbox(hk_sim *S, int isp, long long need) {
    DevSpecies &D = S->sp[isp];
    if (need <= D.inbox_cap) return HK_OK;
    // an eighth of room beyond the need, so that the few percent a re-bin adds
    // to the capacity do not allocate again (a new inbox and fail list of a
    // large species, gigabytes, cost a fraction of a second); small lists double
    long long c = need + need / 8;
    if (D.inbox_cap < (1 << 20)) c = std::max<long long>(c, 2LL * D.inbox_cap);
    c = std::min<long long>(c, INT_MAX / 2);
    free_parr(S, D.inbox);
    free_parr(S, D.fail);
    if (!alloc_parr(S, D.inbox, c, D.has_z, D.has_tau) || !alloc_parr(S, D.fail, c, D.has_z, D.has_tau)) {
        // no inbox now: kernels must not see the old capacity
        free_parr(S, D.inbox);
        free_parr(S, D.fail);
        D.inbox_cap = 0;
        S->poisoned = 1;
        return fail(S, HK_ENOMEM, "inbox of %lld", c);
    }
    D.inbox_cap = (int)c;
    if (!D.inbox_dev) D.inbox_dev = (PArr *)dalloc(S, sizeof(PArr));
    if (!D.inbox_dev) {
        S->poisoned = 1;
        return fail(S, HK_ENOMEM, "inbox descriptor");
    }
    HIPCHK(S, hipMemcpyAsync(D.inbox_dev, &D.inbox, sizeof(PArr), hipMemcpyHostToDevice, S->s));
    int capv[1] = {(int)INT_MAX};
    HIPCHK(S, hipMemcpyAsync(D.g_capmax, capv, sizeof(int), hipMemcpyHostToDevice, S->s));
    return HK_OK;
}

int build_ion_table(hk_sim *S, int isp) {
    DevSpecies &D = S->sp[isp];
    IonP P{};
    double omega0 = 2.0 * PI * PHYS_C / (S->las.lambda_um * 1e-6);
    double eunit = PHYS_ME * PHYS_C * omega0 / PHYS_QE;
    P.field_au = eunit / PHYS_EA;
    P.omega_au = omega0 * PHYS_TA;
    P.rate_norm = 1.0 / P.omega_au;
    P.dt_au = S->gd.dt / P.omega_au;
    P.z_max = D.d.z_max;
    P.target = D.d.target;
    for (int l = 0; l < D.d.z_max && l < HK_MAX_LEVELS; ++l) {
        IonLevel &L = P.lev[l];
        L.ip_au = D.d.ip_ev[l] / PHYS_HARTREE_EV;
        L.zres = l + 1;
        double ns = L.zres / std::sqrt(2.0 * L.ip_au);
        L.c2 = std::pow(2.0, 2.0 * ns) / (ns * std::tgamma(2.0 * ns));
        L.k3 = std::pow(2.0 * L.ip_au, 1.5);
        L.expo = 2.0 * ns - 1.0;
        L.fc = P.omega_au * std::sqrt(2.0 * L.ip_au) / 1.5;
        L.wfc = L.c2 * L.ip_au * std::pow(2.0 * L.k3 / L.fc, L.expo) * std::exp(-2.0 * L.k3 / (3.0 * L.fc));
        L.K2 = 2.0 * std::ceil(L.ip_au / P.omega_au);
        // Below F_skip the blended rate is under max(w_MPI, w_ADK), which rises
        // monotonically up to the ADK maximum at F = 2 k3 / (3 expo); keep the
        // step probability under 1e-9, far below the smallest uniform draw
        // (2^-24), so skipping the rate there changes no event.
        auto bound = [&](double F) {
            double wm = L.wfc * std::pow(std::fmin(F, L.fc) / L.fc, L.K2);
            double wa = L.c2 * L.ip_au * std::pow(2.0 * L.k3 / F, L.expo) * std::exp(-2.0 * L.k3 / (3.0 * F));
            return std::fmax(wm, wa) * P.rate_norm * S->gd.dt;
        };
        double lo = 1e-12, hi = std::fmin(1.0, 2.0 * L.k3 / (3.0 * std::fmax(L.expo, 1e-3)));
        if (!(bound(lo) < 1e-9)) L.fskip = 0.0;
        else if (bound(hi) < 1e-9) L.fskip = hi;
        else {
            for (int it = 0; it < 200; ++it) {
                double mid = std::sqrt(lo * hi);
                if (bound(mid) < 1e-9) lo = mid; else hi = mid;
            }
            L.fskip = lo;
        }
        // probability bounds over field bins: the blend is a convex combination
        // of w_MPI (rising in F) and w_ADK (rising up to F* = 2 k3 / (3 expo),
        // falling after), so over [Fa, Fb] it stays under max(w_MPI(Fb),
        // w_ADK at F* clamped to the bin); and 1 - exp(-w dt) <= w dt
        const double f0 = L.fskip > 0.0 ? L.fskip : 1e-9;
        const double octaves = 24.0;
        L.lf0 = (float)std::log2(f0);
        L.ilr = (float)(ION_NBND / octaves);
        const double fstar = L.expo > 0.0 ? 2.0 * L.k3 / (3.0 * L.expo) : 1e300;
        std::vector<double> b1(ION_NBND);
        for (int b = 0; b < ION_NBND; ++b) {
            // bins widened by 1e-3 of a bin on both sides against FP32 edge rounding
            const double fa = std::exp2((double)L.lf0 + (b - 1e-3) / (double)L.ilr);
            const double fb = std::exp2((double)L.lf0 + (b + 1 + 1e-3) / (double)L.ilr);
            const double wm = L.wfc * std::pow(std::fmin(fb, L.fc) / L.fc, L.K2);
            const double fm = std::fmin(std::fmax(fstar, fa), fb);
            const double wa = L.c2 * L.ip_au * std::pow(2.0 * L.k3 / fm, L.expo) *
                              std::exp(-2.0 * L.k3 / (3.0 * fm));
            const double x = std::fmax(wm, wa) * P.rate_norm * S->gd.dt * (1.0 + 1e-6);
            b1[b] = std::isfinite(x) ? x : 2.0;
        }
        for (int b = 0; b < ION_NBND; ++b) {
            double m = b1[b];
            if (b > 0) m = std::fmax(m, b1[b - 1]);
            if (b + 1 < ION_NBND) m = std::fmax(m, b1[b + 1]);
            // the top bin also stands for every larger field: no bound there
            if (b >= ION_NBND - 2) m = 2.0;
            L.bnd[b] = m >= 1.0 ? 2.0f : std::nextafter((float)m, 2.0f);
        }
    }
    D.ion = (IonP *)dalloc(S, sizeof(IonP));
    if (!D.ion) return fail(S, HK_ENOMEM, "ion table");
    HIPCHK(S, hipMemcpyAsync(D.ion, &P, sizeof(IonP), hipMemcpyHostToDevice, S->s));
    return HK_OK;
}

int init_species(hk_sim *S, int isp) {
    DevSpecies &D = S->sp[isp];
    const GridP &g = S->g;
    const hk_species_desc &d = D.d;
    D.g_off0 = (long long *)dalloc(S, sizeof(long long));
    D.g_capmax = (int *)dalloc(S, sizeof(int));
    D.umax2 = (unsigned *)dalloc(S, sizeof(unsigned) * g.ntiles);
    if (!D.g_off0 || !D.g_capmax || !D.umax2) return fail(S, HK_ENOMEM, "species tables");
    launch_zero(D.umax2, sizeof(unsigned) * g.ntiles, S->s);
    D.umax_ok = false;
    std::vector<int> xcol;
    std::vector<double> wcol;
    double dv = g.ddx * g.ddy * g.ddz;
    if (d.ppc > 0 && d.profile != HK_PROF_NONE)
        for (int i = 0; i < g.nx; ++i) {
            double n = profile(d, (i + 0.5) * g.ddx);
            if (n > 0) { xcol.push_back(i); wcol.push_back(n * dv / d.ppc); }
        }
    long long total = (long long)xcol.size() * g.ny * g.nz * std::max(d.ppc, 0);
    int rc = ensure_inbox(S, isp, std::max<long long>(total, 1 << 16));
    if (rc) return rc;
    double wm = 0;
    for (double w : wcol) wm = std::max(wm, w);
    rc = raise_wmax(S, isp, wm);
    if (rc) return rc;
    if (total > 0) {
        int *dx = (int *)dalloc(S, sizeof(int) * xcol.size());
        double *dw = (double *)dalloc(S, sizeof(double) * wcol.size());
        if (!dx || !dw) return fail(S, HK_ENOMEM, "init columns");
        HIPCHK(S, hipMemcpyAsync(dx, xcol.data(), sizeof(int) * xcol.size(), hipMemcpyHostToDevice, S->s));
        HIPCHK(S, hipMemcpyAsync(dw, wcol.data(), sizeof(double) * wcol.size(), hipMemcpyHostToDevice, S->s));
        launch_init_species_cols(g, d, isp, S->run.seed, D.inbox, dx, dw, (int)xcol.size(), D.has_z,
                                 D.has_tau, S->s);
        int n32 = (int)total;
        HIPCHK(S, hipMemcpyAsync(S->status + 1 + 2 * isp, &n32, sizeof(int), hipMemcpyHostToDevice, S->s));
        HIPCHK(S, hipStreamSynchronize(S->s));
        dfree(S, dx);
        dfree(S, dw);
    }
    int *ln = S->status + 1 + 2 * isp;
    PArr lists[1] = {D.inbox};
    long long lmax[1] = {total};
    rc = rebuild(S, isp, false, lists, &ln, lmax, total > 0 ? 1 : 0);
    if (rc) return rc;
    HIPCHK(S, hipMemsetAsync(S->status + 1 + 2 * isp, 0, sizeof(int), S->s));
    return HK_OK;
}

hipEvent_t ev_get(hk_sim *S) {
    hipEvent_t e = nullptr;
    if (!S->ev_free.empty()) { e = S->ev_free.back(); S->ev_free.pop_back(); }
    else (void)hipEventCreate(&e);
    (void)hipEventRecord(e, S->s);
    return e;
}

// Accumulate every recorded span into the timers and recycle the events.
void ev_resolve(hk_sim *S) {
    if (S->spans.empty()) return;
    (void)hipEventSynchronize(S->spans.back().b);
    std::vector<hipEvent_t> used;
    for (auto &sp : S->spans) {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, sp.a, sp.b);
        S->timers[sp.slot] += ms;
        used.push_back(sp.a);
        used.push_back(sp.b);
    }
    S->spans.clear();
    std::sort(used.begin(), used.end());
    used.erase(std::unique(used.begin(), used.end()), used.end());
    for (hipEvent_t e : used)
        if (e != S->last_mark) S->ev_free.push_back(e);
}

// Group timing: the interval since the previous mark is charged to `slot`
// (slot < 0 starts a new sequence).
void time_mark(hk_sim *S, int slot) {
    if (!S->timing) return;
    hipEvent_t e = ev_get(S);
    if (slot >= 0 && S->last_mark) S->spans.push_back({S->last_mark, e, slot});
    S->last_mark = e;
    if (S->spans.size() > 2048) ev_resolve(S);
}

int status_error(hk_sim *S) {
    int e = S->h_status[0];
    if (e & ERR_NONFINITE) return fail(S, HK_ENUMERIC, "non-finite momentum at step %lld", (long long)S->step);
    if (e & ERR_CFL) return fail(S, HK_ENUMERIC, "particle moved a cell or more at step %lld", (long long)S->step);
    if (e & ERR_INBOX) return fail(S, HK_EOVERFLOW, "particle inbox overflow at step %lld", (long long)S->step);
    if (e & ERR_TILE) return fail(S, HK_EDEVICE, "particle outside its tile at step %lld", (long long)S->step);
    return HK_OK;
}

int gauss_snapshot(hk_sim *S);

// Kernel variant of a species' push: 0 charged particles, 1 QED leptons,
// 2 photons; -1 for photons without QED (they are not advanced).
int push_mode(const hk_sim *S, int isp) {
    const hk_species_desc &d = S->sp[isp].d;
    if (d.kind == HK_PHOTON) return S->run.enable_qed ? 2 : -1;
    if (S->run.enable_qed && d.qed && (d.kind == HK_ELECTRON || d.kind == HK_POSITRON)) return 1;
    return 0;
}

// Inbox size of a species: the particles one step can send past full bins
// (a quarter of the capacity; bins keep 25% headroom) plus every electron the
// ions targeting it can free in one step, plus room for spawning (a quarter
// of the capacity: a node whose particles find no room stays fluid and
// spawns in a later step).
long long inbox_need(hk_sim *S, int isp) {
    long long need = std::max<long long>(S->sp[isp].capacity / 4, 1 << 16);
    if (S->sp[isp].d.fluid && S->run.switch_mode != HK_SW_ALL_PIC)
        need += std::min<long long>(S->g.nn * std::max(1, S->sp[isp].d.ppc),
                                    std::max<long long>(S->sp[isp].capacity / 4, 1 << 20));
    for (int j = 0; j < S->nsp; ++j)
        if (S->sp[j].d.ionizable && S->sp[j].d.target == isp && S->run.enable_ionization)
            need += S->sp[j].capacity * std::max(1, S->sp[j].d.z_max);
    if (S->run.enable_qed) {
        // one photon per QED lepton per step; one pair member per photon
        if (isp == S->photon_sp)
            for (int j = 0; j < S->nsp; ++j)
                if (push_mode(S, j) == 1) need += std::max<long long>(S->sp[j].capacity, S->sp[j].reserve_hint);
        if ((isp == S->electron_sp || isp == S->positron_sp) && S->photon_sp >= 0)
            need += std::max<long long>(S->sp[S->photon_sp].capacity, S->sp[S->photon_sp].reserve_hint);
    }
    return need;
}

// Whether kernels of a step can send particles to species isp's inbox: its own
// push (overflowing mover regions), ionization of ions that target it, QED
// products, or fluid-to-particle spawning.
bool receives(const hk_sim *S, int isp) {
    const DevSpecies &D = S->sp[isp];
    if (D.d.mobile) return true;
    if (D.d.fluid && S->run.switch_mode != HK_SW_ALL_PIC) return true;
    for (int j = 0; j < S->nsp; ++j)
        if (S->sp[j].d.ionizable && S->sp[j].d.target == isp && S->run.enable_ionization) return true;
    return S->run.enable_qed && (isp == S->photon_sp || isp == S->electron_sp || isp == S->positron_sp);
}

// Append every species' inbox to the back of its current bins and start the
// copy of the device status to the host (merge_launch); work that does not
// touch the particle bins may be enqueued before merge_finish waits for the
// status, re-bins species whose bins were full and clears the counters.
int merge_launch(hk_sim *S) {
    for (int isp = 0; isp < S->nsp; ++isp) {
        DevSpecies &D = S->sp[isp];
        if (D.capacity == 0 || !receives(S, isp)) continue;
        SpecP P = specp(D);
        int *inbox_n = S->status + 1 + 2 * isp, *fail_n = S->status + 2 + 2 * isp;
        launch_merge_inbox(S->g, P, D.inbox, inbox_n, D.inbox_cap, D.buf[D.cur], D.nf[D.cur],
                           D.nb[D.cur], fail_n, D.fail, S->status, S->s);
    }
    HIPCHK(S, hipMemcpyAsync(S->h_status, S->status, sizeof(int) * HK_NSTATUS, hipMemcpyDeviceToHost, S->s));
    HIPCHK(S, hipEventRecord(S->status_ev, S->s));
    return HK_OK;
}

int merge_finish(hk_sim *S) {
    HIPCHK(S, hipEventSynchronize(S->status_ev));
    int rc = status_error(S);
    if (rc) return rc;
    for (int isp = 0; isp < S->nsp; ++isp) S->sp[isp].arrived += S->h_status[1 + 2 * isp];
    bool rebinned = false;
    for (int isp = 0; isp < S->nsp; ++isp) {
        DevSpecies &D = S->sp[isp];
        int nfail = S->h_status[2 + 2 * isp];
        if (nfail > 0) {
            int *ln = S->status + 2 + 2 * isp;
            PArr lists[1] = {D.fail};
            long long lmax[1] = {D.inbox_cap};
            rc = rebuild(S, isp, true, lists, &ln, lmax, 1);
            if (rc) return rc;
            rebinned = true;
        }
    }
    // inbox and fail counters of every species (status[1 .. 2 nsp])
    launch_zero(S->status + 1, sizeof(int) * 2 * HK_MAX_SPECIES, S->s);
    if (rebinned)
        for (int isp = 0; isp < S->nsp; ++isp) {
            DevSpecies &D = S->sp[isp];
            if (S->h_status[2 + 2 * isp] > 0 && D.d.mobile) {
                rc = ensure_inbox(S, isp, inbox_need(S, isp));
                if (rc) return rc;
            }
        }
    return HK_OK;
}

SwitchP switch_params(const hk_sim *S) {
    SwitchP P{};
    P.thr_a = (real)S->run.thr_a;
    P.thr_grad = (real)S->run.thr_grad;
    P.thr_su = (real)S->run.thr_sigma_u;
    P.thr_ion = (real)S->run.thr_ion;
    P.thr_chi = (real)S->run.thr_chi;
    P.n_floor = (real)S->run.n_floor;
    P.dilation = S->run.dilation;
    P.hysteresis = S->run.hysteresis;
    P.enable_qed = S->run.enable_qed;
    P.enable_ion = S->run.enable_ionization;
    if (S->run.enable_qed) {
        double omega0 = 2.0 * PI * PHYS_C / (S->las.lambda_um * 1e-6);
        P.a_s = PHYS_ME * PHYS_C * PHYS_C / (PHYS_HBAR * omega0);
    }
    return P;
}

// Learned switch on the whole node grid: inputs with a 4-node halo, the four
// convolutions, then 16 dropout samples of the head decide where the network
// is confident; elsewhere the threshold flags stay.
void cnn_switch(hk_sim *S) {
    const GridP &g = S->g;
    hk_cnn *c = S->cnn;
    const int NX = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
    const int D = g.nz + 8, H = g.ny + 8, W = NX + 8;
    if (!S->cnn_x) S->cnn_x = (unsigned short *)dalloc(S, sizeof(unsigned short) * 8 * (size_t)D * H * W);
    if (!S->cnn_nfall) S->cnn_nfall = (int *)dalloc(S, sizeof(int) * 8);
    if (!S->cnn_x || !S->cnn_nfall) { fail(S, HK_ENOMEM, "CNN switch inputs"); return; }
    // the network decides within the plasma's x extent widened by the nodes
    // plasma can reach before the next evaluation; the threshold elsewhere
    int *win = S->cnn_nfall + 4;
    cnn_launch_window(g, S->mom, S->run.switch_every + S->run.dilation + 4, win, S->s);
    cnn_launch_inputs(g, S->f, S->mom, c->mean, c->inv_std, S->cnn_x, win + 2, S->s);
    const unsigned short *a4;
    if (cnn_forward_bf16(c, S->cnn_x, 1, D, H, W, false, S->s, &a4, nullptr, win + 2) != HK_OK) {
        fail(S, HK_ENOMEM, "CNN switch: %s", c->err.c_str());
        return;
    }
    launch_zero(S->cnn_nfall, sizeof(int), S->s);
    const long long head = 27LL * 8 * 32 + 32 + 3 * (27LL * 32 * 32 + 32);
    cnn_launch_decide(g, a4, c->wh, c->p + head + 32, S->run.seed, S->cnn_evals, S->hot, S->notcold,
                      S->cnn_nfall, nullptr, win + 2, S->s);
    S->cnn_evals++;
}

// Square of the hot-particle threshold (0: no particle is hot).
real hot2(const hk_sim *S) {
    return S->run.thr_hot > 0.0 ? (real)(S->run.thr_hot * S->run.thr_hot) : (real)0;
}

// Threshold criterion: nearest-node moments, indicators, dilation, hysteresis.
// Switch moments of every fluid species (particles and fluid) and of the
// ionizable ions.  use_bounds: particle moments take their fixed-point scale
// from the per-tile |u|^2 bounds (the switch evaluation, which then restarts
// them); otherwise they scan the tiles for it.
int switch_moments(hk_sim *S, bool use_bounds, const IonP **ions) {
    hipStream_t s = S->s;
    const GridP &g = S->g;
    // fluid moments first: the first fluid species overwrites the arrays
    int first = 1;
    for (int isp = 0; isp < S->nsp; ++isp) {
        DevSpecies &D = S->sp[isp];
        if (!D.d.fluid || !D.fn) continue;
        launch_fluid_moments_nodes(g, (real)(1.0 / std::max(1, D.d.ppc)), D.fn, D.fu[0], D.fu[1],
                                   D.fu[2], S->mom, first, s);
        first = 0;
    }
    if (first) launch_zero(S->mom, sizeof(real) * 7 * (size_t)g.nn, s);
    int nion = 0;
    for (int isp = 0; isp < S->nsp; ++isp) {
        DevSpecies &D = S->sp[isp];
        SpecP P = specp(D);
        if (D.d.fluid && D.capacity)
            launch_moments_tiles(g, P, D.buf[D.cur], cur_bins(D), 0, 0, hot2(S), S->mom, S->wmax + isp,
                                 use_bounds && D.d.mobile && D.umax_ok ? D.umax2 : nullptr, nullptr,
                                 S->plan, S->plan_ctl, D.capacity, s);
        if (D.d.ionizable && S->run.enable_ionization && D.capacity) {
            launch_moments_tiles(g, P, D.buf[D.cur], cur_bins(D), 1, D.d.z_max, (real)0, S->mom, S->wmax + isp,
                                 nullptr, D.d.mobile ? nullptr : D.active, S->plan, S->plan_ctl,
                                 D.capacity, s);
            if (nion < 4) ions[nion++] = D.ion;
        }
    }
    return nion;
}

void switch_eval(hk_sim *S) {
    hipStream_t s = S->s;
    const GridP &g = S->g;
    const IonP *ions[4];
    const int nion = switch_moments(S, true, ions);
    // the |u|^2 bounds start again from here
    for (int isp = 0; isp < S->nsp; ++isp) {
        DevSpecies &D = S->sp[isp];
        if (!D.d.fluid || !D.d.mobile) continue;
        launch_zero(D.umax2, sizeof(unsigned) * g.ntiles, s);
        D.umax_ok = true;
    }
    SwitchP P = switch_params(S);
    launch_indicators_nodes(g, P, S->mom, S->f, ions, nion, S->hot, S->notcold, s);
    if (S->run.switch_mode == HK_SW_CNN && S->cnn) cnn_switch(S);
    if (!S->dil) S->dil = (uint8_t *)dalloc(S, 2 * (size_t)g.nn);
    if (!S->dil) { fail(S, HK_ENOMEM, "switch dilation scratch"); return; }
    launch_dilate_nodes(g, P, S->hot, S->notcold, S->sw, S->calm, S->dil, s);
}

// Fluid <-> particle conversion for every fluid species with a fluid array.
void reconcile(hk_sim *S) {
    hipStream_t s = S->s;
    const GridP &g = S->g;
    for (int isp = 0; isp < S->nsp; ++isp) {
        DevSpecies &D = S->sp[isp];
        if (!D.d.fluid || !D.fn) continue;
        SpecP P = specp(D);
        const WarmP W{D.fs, D.d.gamma_ad};
        // particles the push absorbed join the node fluid
        if (D.capacity)
            launch_absorb_finish_nodes(g, P.m, D.macc, D.fn, D.fu[0], D.fu[1], D.fu[2], W, S->ledger, D.xr, s);
        launch_fluid_window_commit(g, D.xr, s);
        double dv = g.ddx * g.ddy * g.ddz;
        const double w0 = D.d.n0 * dv / std::max(1, D.d.ppc);
        real wmin = (real)(S->run.spawn_frac * w0);
        launch_zero(S->spawn_n, sizeof(int), s);
        launch_spawn_nodes(g, P, isp, S->sw, D.fn, D.fu[0], D.fu[1], D.fu[2], W, S->jg, wmin, (real)w0,
                           S->run.seed, (int)S->step, D.inbox, S->status + 1 + 2 * isp, D.inbox_cap,
                           S->status + 13, S->wmax + isp, D.umax2, S->ledger, S->spawn_list, S->spawn_n, D.xr,
                           s);
    }
}

// Sinks and tables of the QED events: photons go to the first photon species,
// pairs to the first electron and positron species.
QedP qed_params(hk_sim *S, int mode) {
    QedP Q{};
    if (mode == 0) return Q;
    Q.We = S->qed_tab;
    Q.Wb = S->qed_tab + QED_NCHI;
    Q.Xe = S->qed_tab + 2 * QED_NCHI;
    Q.Xb = S->qed_tab + 2 * QED_NCHI + QED_NCHI * QED_NU;
    Q.a_s = S->a_s;
    Q.alpha_as = 7.2973525693e-3 * S->a_s;
    Q.ledger = S->ledger + 2;
    Q.sw = S->sw;
    Q.hybrid = S->run.switch_mode != HK_SW_ALL_PIC;
    Q.seed = S->run.seed;
    Q.step = (int)S->step;
    auto sink = [&](int sp, PArr &o, int *&n, int &cap, int &tau, int &have, unsigned *&wm) {
        if (sp < 0) return;
        DevSpecies &T = S->sp[sp];
        o = T.inbox;
        n = S->status + 1 + 2 * sp;
        cap = T.inbox_cap;
        tau = T.has_tau;
        have = T.inbox_cap > 0;
        wm = S->wmax + sp;
    };
    if (mode == 1) {
        sink(S->photon_sp, Q.out1, Q.out1_n, Q.out1_cap, Q.out1_tau, Q.have1, Q.wmax1);
    } else {
        sink(S->electron_sp, Q.out1, Q.out1_n, Q.out1_cap, Q.out1_tau, Q.have1, Q.wmax1);
        sink(S->positron_sp, Q.out2, Q.out2_n, Q.out2_cap, Q.out2_tau, Q.have2, Q.wmax2);
    }
    if (!Q.out1_n) Q.out1_n = S->status + 15;   // a dummy counter: nothing requests it
    if (!Q.out2_n) Q.out2_n = S->status + 15;
    if (!Q.wmax1) Q.wmax1 = S->wmax + HK_MAX_SPECIES;
    if (!Q.wmax2) Q.wmax2 = S->wmax + HK_MAX_SPECIES;
    return Q;
}

int one_step(hk_sim *S) {
    hipStream_t s = S->s;
    const GridP &g = S->g;
    const int mode = S->run.switch_mode;
    const int hybrid = mode != HK_SW_ALL_PIC;
    time_mark(S, -1);
    // 1. switch evaluation
    if ((mode == HK_SW_THRESHOLD || mode == HK_SW_CNN) &&
        S->step % std::max(1, S->run.switch_every) == 0)
        switch_eval(S);
    time_mark(S, 0);
    // 2. J = 0, antenna current at t^{n+1/2}
    launch_zero(S->f[HK_JX], sizeof(real) * 3 * (size_t)g.nn, s);
    launch_antenna(g, S->las, S->t + 0.5 * g.ddt, S->f[HK_JY], S->f[HK_JZ], s);
    // 3. particles (mobile species push into the next bins; immobile ions ionize in
    // place; QED leptons emit photons; photons create pairs and fly straight)
    for (int isp = 0; isp < S->nsp; ++isp) S->sp[isp].arrived = 0;
    for (int isp = 0; isp < S->nsp; ++isp) {
        DevSpecies &D = S->sp[isp];
        if (D.capacity == 0) continue;
        SpecP P = specp(D);
        const int mode = push_mode(S, isp);
        if (mode < 0) continue;
        if (D.d.mobile && D.idle) continue;   // empty bins, nothing arrived: nothing to push
        if (D.d.mobile) {
            int nxt = 1 - D.cur;
            // front and back fills of the next buffer and the mover ranks start
            // at zero (cleared by the push's planner): several push workgroups
            // share a dense tile
            int *mcnt = D.nf[nxt] + 2 * g.ntiles;
            QedP Q = qed_params(S, mode);
            AbsorbP A{};
            if (hybrid && D.d.fluid && D.fn && D.macc && mode != 2) {
                A.on = 1;
                A.sw = S->sw;
                A.macc = D.macc;
                A.ledger = S->ledger;
                A.hot2 = hot2(S);
                A.xr = D.xr;
                A.warm = D.fs != nullptr;
            }
            hipEvent_t pa = S->timing ? ev_get(S) : nullptr;
            launch_push_tiles(g, P, D.buf[D.cur], cur_bins(D), D.buf[nxt], D.nf[nxt], D.mig0, D.moff,
                              D.mcap, mcnt, D.inbox_dev, S->status + 1 + 2 * isp, D.inbox_cap, S->f,
                              S->jg, S->status, S->dstat, S->wmax + isp, D.umax2, mode, Q, A, S->plan,
                              S->plan_ctl, D.capacity, S->status + 16 + isp, s);
            if (S->timing) {
                S->spans.push_back({pa, ev_get(S), 6});
                S->timers[8] += 1;
            }
            launch_migrate(g, P, shifted(D.buf[nxt], D.mig0), D.moff, mcnt, D.mcap, D.buf[nxt], D.nf[nxt], D.nb[nxt],
                           S->status + 2 + 2 * isp, D.fail, D.inbox_cap, S->status, s);
        } else if (D.d.ionizable && S->run.enable_ionization) {
            DevSpecies &T = S->sp[D.d.target];
            launch_ionize_static(g, P, D.buf[D.cur], cur_bins(D), D.active, S->f, S->sw, hybrid,
                                 D.ion, T.inbox, S->status + 1 + 2 * D.d.target, T.inbox_cap,
                                 S->run.seed, (int)S->step, S->ledger + 1, S->status, T.umax2,
                                 T.has_tau, s);
        }
    }
    bool pushed[HK_MAX_SPECIES] = {};
    for (int isp = 0; isp < S->nsp; ++isp) {
        DevSpecies &D = S->sp[isp];
        if (D.capacity && D.d.mobile && push_mode(S, isp) >= 0 && !D.idle) {
            D.cur = 1 - D.cur;
            pushed[isp] = true;
        }
    }
    time_mark(S, 1);
    // 4. cold fluid and 5. conversion (neither reads the bins: spawned particles
    // go to the inboxes behind the push's products); 6. newborn and overflow
    // particles join their bins; 7. fields, enqueued before the host waits for
    // the status of the merge
    if (hybrid) {
        for (int isp = 0; isp < S->nsp; ++isp) {
            DevSpecies &D = S->sp[isp];
            if (!D.fn) continue;
            launch_fluid(g, specp(D), D.fn, D.fu[0], D.fu[1], D.fu[2], WarmP{D.fs, D.d.gamma_ad}, S->f,
                         S->fluid_scratch, D.fn2, D.fs2, (real)S->run.n_floor, D.xr, s);
            std::swap(D.fn, D.fn2);
            if (D.fs) std::swap(D.fs, D.fs2);
        }
        time_mark(S, 2);
        reconcile(S);
        time_mark(S, 3);
    }
    int rc = merge_launch(S);
    if (rc) return rc;
    time_mark(S, 5);
    // the particles' current (deposits and conversion moves) joins J
    launch_jconvert(g, S->jg, S->f, s);
    if (S->falt && launch_yee_step(g, S->f, S->f_alt, s)) {
        for (int c = 0; c < 6; ++c) std::swap(S->f[c], S->f_alt[c]);
    } else {
        launch_yee_b_half(g, S->f, s);
        launch_yee_e_full(g, S->f, S->mur_old, s);
        launch_yee_b_half(g, S->f, s);
    }
    time_mark(S, 4);
    rc = merge_finish(S);
    if (rc) return rc;
    time_mark(S, 5);
    // a species whose bins were empty at this push and which received nothing
    // is skipped until something arrives (a re-bin or a host write resets it)
    for (int isp = 0; isp < S->nsp; ++isp) {
        DevSpecies &D = S->sp[isp];
        if (pushed[isp]) D.idle = S->h_status[16 + isp] == 0;
        if (D.arrived > 0) D.idle = false;
    }
    S->step++;
    S->t = S->step * g.ddt;
    return HK_OK;
}

// The x window of species isp's fluid: every node (full) or none (a fluid
// that is zero everywhere); periodic x always takes every node.
int set_fluid_window(hk_sim *S, int isp, bool full) {
    const GridP &g = S->g;
    const int per = g.bcx == HK_BC_PERIODIC;
    const int empty = g.nx + 2;
    int h[8] = {0, per ? g.nx - 1 : g.nx, empty, -1, empty, -1, 0, 0};
    if (!full && !per) { h[0] = empty; h[1] = -1; }
    HIPCHK(S, hipMemcpyAsync(S->sp[isp].xr, h, sizeof(h), hipMemcpyHostToDevice, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    return HK_OK;
}

// Fluid arrays exist for fluid species whenever the mode is not all-PIC.
int ensure_fluid(hk_sim *S) {
    const GridP &g = S->g;
    if (!S->mom) {
        S->mom = (real *)dalloc(S, sizeof(real) * 7 * (size_t)g.nn);
        S->spawn_list = (int *)dalloc(S, sizeof(int) * (size_t)g.nn, false);
        S->spawn_n = (int *)dalloc(S, sizeof(int) * 8);
        S->hot = (uint8_t *)dalloc(S, (size_t)g.nn);
        S->notcold = (uint8_t *)dalloc(S, (size_t)g.nn);
        S->fluid_scratch = (real *)dalloc(S, sizeof(real) * 7 * (size_t)g.nn);
        if (!S->mom || !S->spawn_list || !S->spawn_n || !S->hot || !S->notcold || !S->fluid_scratch)
            return fail(S, HK_ENOMEM, "switch arrays");
    }
    for (int isp = 0; isp < S->nsp; ++isp) {
        DevSpecies &D = S->sp[isp];
        if (!D.d.fluid || D.fn) continue;
        D.fn = (real *)dalloc(S, sizeof(real) * (size_t)g.nn);
        D.fn2 = (real *)dalloc(S, sizeof(real) * (size_t)g.nn);
        for (int d = 0; d < 3; ++d) D.fu[d] = (real *)dalloc(S, sizeof(real) * (size_t)g.nn);
        D.macc = (double *)dalloc(S, sizeof(double) * 5 * (size_t)g.nn);
        D.xr = (int *)dalloc(S, sizeof(int) * 8, false);
        if (D.xr) {
            int rc = set_fluid_window(S, isp, false);
            if (rc) return rc;
        }
        if (D.d.gamma_ad > 0.0) {
            D.fs = (real *)dalloc(S, sizeof(real) * (size_t)g.nn);
            D.fs2 = (real *)dalloc(S, sizeof(real) * (size_t)g.nn);
        }
        if (!D.fn || !D.fn2 || !D.fu[0] || !D.fu[1] || !D.fu[2] || !D.macc || !D.xr ||
            (D.d.gamma_ad > 0.0 && (!D.fs || !D.fs2)))
            return fail(S, HK_ENOMEM, "fluid arrays");
        int rc = ensure_inbox(S, isp, inbox_need(S, isp));
        if (rc) return rc;
    }
    return HK_OK;
}

int rho_total(hk_sim *S, double *rho) {
    launch_zero(rho, sizeof(double) * (size_t)S->g.nn, S->s);
    for (int isp = 0; isp < S->nsp; ++isp) {
        DevSpecies &D = S->sp[isp];
        if (D.d.kind == HK_PHOTON) continue;
        SpecP P = specp(D);
        if (D.capacity) launch_rho_tiles(S->g, P, D.buf[D.cur], cur_bins(D), rho, S->s);
        if (D.fn) launch_fluid_rho(S->g, P, D.fn, rho, S->s);
    }
    return HK_OK;
}

int gauss_snapshot(hk_sim *S) {
    launch_divE(S->g, S->f, S->gauss0, S->s);
    rho_total(S, S->tmp_a);
    launch_sub(S->g.nn, S->gauss0, S->tmp_a, S->s);   // gauss0 = divE - rho
    S->have_gauss0 = 1;
    return HK_OK;
}

bool check_grid(const hk_grid_desc *g) {
    return g && g->nx >= 4 && g->ny >= 2 && g->nz >= 2 && g->dx > 0 && g->dy > 0 && g->dz > 0 &&
           g->dt > 0 && (g->bc_x == HK_BC_OPEN || g->bc_x == HK_BC_PERIODIC) &&
           (long long)(g->nx + 1) * g->ny * g->nz < (1LL << 31) &&   // nodes: 32-bit indices
           g->dt < 1.0 / std::sqrt(1.0 / (g->dx * g->dx) + 1.0 / (g->dy * g->dy) + 1.0 / (g->dz * g->dz));
}

// Host copy of the valid slots of a species' current bins, in storage order.
int valid_slots(hk_sim *S, DevSpecies &D, std::vector<long long> &slots) {
    slots.clear();
    if (D.capacity == 0) return HK_OK;
    const int nt = S->g.ntiles;
    std::vector<int> nf(nt), nb(nt), cells((size_t)D.capacity);
    HIPCHK(S, hipMemcpyAsync(nf.data(), D.nf[D.cur], sizeof(int) * nt, hipMemcpyDeviceToHost, S->s));
    HIPCHK(S, hipMemcpyAsync(nb.data(), D.nb[D.cur], sizeof(int) * nt, hipMemcpyDeviceToHost, S->s));
    HIPCHK(S, hipMemcpyAsync(cells.data(), D.buf[D.cur].cell, sizeof(int) * D.capacity,
                             hipMemcpyDeviceToHost, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    for (int t = 0; t < nt; ++t) {
        int c = D.h_cap[t];
        int f = std::min(nf[t], c), b = std::min(nb[t], c - f);
        for (int p = 0; p < f + b; ++p) {
            long long i = D.h_off[t] + (p < f ? p : c - b + (p - f));
            if (cells[i] >= 0) slots.push_back(i);
        }
    }
    return HK_OK;
}

// Replace species isp's particles by n particles in the library's own
// representation (cell, offsets, u, w, id, z, tau) and re-bin them.
int upload_particles(hk_sim *S, int isp, size_t n, const std::vector<int> &cell, const std::vector<real> r[7],
                     const std::vector<uint64_t> &id, const std::vector<int> &zc, const std::vector<double> &tau,
                     double wm) {
    DevSpecies &D = S->sp[isp];
    D.umax_ok = false;
    int rc = ensure_inbox(S, isp, (long long)n + 1024);
    if (rc) return rc;
    rc = raise_wmax(S, isp, wm);
    if (rc) return rc;
    const PArr &a = D.inbox;
    hipStream_t s = S->s;
    if (n) {
        HIPCHK(S, hipMemcpyAsync(a.cell, cell.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
        real *dst[7] = {a.rx, a.ry, a.rz, a.ux, a.uy, a.uz, a.w};
        for (int k = 0; k < 7; ++k)
            HIPCHK(S, hipMemcpyAsync(dst[k], r[k].data(), sizeof(real) * n, hipMemcpyHostToDevice, s));
        HIPCHK(S, hipMemcpyAsync(a.id, id.data(), sizeof(uint64_t) * n, hipMemcpyHostToDevice, s));
        if (D.has_z) HIPCHK(S, hipMemcpyAsync(a.zc, zc.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
        if (D.has_tau) HIPCHK(S, hipMemcpyAsync(a.tau, tau.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
    }
    int n32 = (int)n;
    HIPCHK(S, hipMemcpyAsync(S->status + 1 + 2 * isp, &n32, sizeof(int), hipMemcpyHostToDevice, s));
    int *ln = S->status + 1 + 2 * isp;
    PArr lists[1] = {D.inbox};
    long long lmax[1] = {(long long)n};
    rc = rebuild(S, isp, false, lists, &ln, lmax, 1);
    if (rc) return rc;
    HIPCHK(S, hipMemsetAsync(S->status + 1 + 2 * isp, 0, sizeof(int), s));
    HIPCHK(S, hipStreamSynchronize(s));
    return ensure_inbox(S, isp, inbox_need(S, isp));
}

constexpr uint32_t CK_MAGIC = 0x4b434b48u;   // "HKCK"
constexpr uint32_t CK_VERSION = 1;

struct CkFile {
    FILE *f = nullptr;
    bool ok = true;
    ~CkFile() { if (f) fclose(f); }
    void put(const void *p, size_t n) { if (ok && n && fwrite(p, 1, n, f) != n) ok = false; }
    void get(void *p, size_t n) { if (ok && n && fread(p, 1, n, f) != n) ok = false; }
    template <class T> void put(const T &v) { put(&v, sizeof(T)); }
    template <class T> void get(T &v) { get(&v, sizeof(T)); }
};

// device -> file and file -> device through a host buffer
int ck_dev_out(hk_sim *S, CkFile &F, const void *dev, size_t bytes) {
    std::vector<char> h(bytes);
    if (bytes) HIPCHK(S, hipMemcpyAsync(h.data(), dev, bytes, hipMemcpyDeviceToHost, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    F.put(h.data(), bytes);
    return HK_OK;
}
int ck_dev_in(hk_sim *S, CkFile &F, void *dev, size_t bytes) {
    std::vector<char> h(bytes);
    F.get(h.data(), bytes);
    if (!F.ok) return fail(S, HK_EIO, "checkpoint: file ends early");
    if (bytes) HIPCHK(S, hipMemcpyAsync(dev, h.data(), bytes, hipMemcpyHostToDevice, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    return HK_OK;
}

}  // namespace

// ====================================================================== ABI ===============

extern "C" {

int hk_node_inputs(hk_sim *S, double *raw, double *ehat, uint8_t *hot, size_t nodes) {
    if (!S) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    const GridP &g = S->g;
    const int NX = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
    const size_t n = (size_t)NX * g.ny * g.nz;
    if (nodes != n) return fail(S, HK_EINVAL, "node count %zu, expected %zu", nodes, n);
    int rc = ensure_fluid(S);
    if (rc) return rc;
    if (!S->cnn_raw) {
        S->cnn_raw = (float *)dalloc(S, sizeof(float) * 9 * n);
        if (!S->cnn_raw) return fail(S, HK_ENOMEM, "node inputs");
    }
    const IonP *ions[4];
    const int nion = switch_moments(S, false, ions);
    SwitchP P = switch_params(S);
    // indicators into scratch flags; the switch map and its hysteresis state stay
    launch_indicators_nodes(g, P, S->mom, S->f, ions, nion, S->hot, S->notcold, S->s);
    cnn_launch_node_raw(g, S->f, S->mom, S->cnn_raw, S->s);
    std::vector<float> h(9 * n);
    std::vector<uint8_t> hh(g.nn);
    HIPCHK(S, hipMemcpyAsync(h.data(), S->cnn_raw, sizeof(float) * 9 * n, hipMemcpyDeviceToHost, S->s));
    HIPCHK(S, hipMemcpyAsync(hh.data(), S->hot, g.nn, hipMemcpyDeviceToHost, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    for (size_t v = 0; v < n; ++v) {
        if (raw) for (int q = 0; q < 8; ++q) raw[8 * v + q] = h[9 * v + q];
        if (ehat) ehat[v] = h[9 * v + 8];
        if (hot) {
            const int i = (int)(v % NX), j = (int)((v / NX) % g.ny), k = (int)(v / ((size_t)NX * g.ny));
            hot[v] = hh[(size_t)i + (size_t)g.sx * ((size_t)j + (size_t)g.ny * k)];
        }
    }
    return HK_OK;
}

int hk_dump_training(hk_sim *S, hk_dataset *ds, int steps, int every, int window) {
    if (!S || !ds || steps < 0 || every < 1 || window < 0) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    if (S->run.switch_mode != HK_SW_ALL_PIC)
        return fail(S, HK_EINVAL, "training data come from an all-PIC run");
    const GridP &g = S->g;
    const int per = g.bcx == HK_BC_PERIODIC;
    const int NX = per ? g.nx : g.nx + 1;
    if (g.nz < 16 || g.ny < 16 || NX < 16)
        return fail(S, HK_EINVAL, "grid of %d x %d x %d nodes: crops need 16 in each direction", g.nz, g.ny, NX);
    const long long n = (long long)NX * g.ny * g.nz;
    int rc = ensure_fluid(S);
    if (rc) return rc;
    if (!S->lab) {
        S->lab = (uint8_t *)dalloc(S, (size_t)n);
        if (!S->lab) return fail(S, HK_ENOMEM, "label scratch");
    }
    // snapshots are written on the simulation's stream, which is drained
    // before the call returns
    HIPCHK(S, hipStreamSynchronize(ds->s));
    const SwitchP P = switch_params(S);
    const double dv = g.ddx * g.ddy * g.ddz;
    std::vector<int> open;   // indices into ds->snaps still accumulating labels
    std::vector<int> r0s;
    for (int r = 0; r <= steps + window; ++r) {
        const IonP *ions[4];
        const int nion = switch_moments(S, false, ions);
        launch_label_nodes(g, P, S->mom, S->f, ions, nion, S->lab, S->s);
        if (r <= steps && r % every == 0) {
            DsSnap *snap = nullptr;
            rc = ds_append(ds, g.nz, g.ny, NX, per, dv, S->s, &snap);
            if (rc) return fail(S, rc, "training snapshot: %s", ds->err.c_str());
            cnn_launch_node_raw(g, S->f, S->mom, snap->raw9, S->s);
            launch_indicators_nodes(g, P, S->mom, S->f, ions, nion, S->hot, S->notcold, S->s);
            launch_flags_canonical(g, S->hot, snap->thr, S->s);
            open.push_back((int)ds->snaps.size() - 1);
            r0s.push_back(r);
        }
        for (size_t q = 0; q < open.size(); ++q)
            launch_label_or(n, S->lab, ds->snaps[open[q]].y, S->s);
        // a snapshot's window closes after steps r0 .. r0 + window
        for (size_t q = 0; q < open.size();) {
            if (r >= r0s[q] + window) {
                open.erase(open.begin() + q);
                r0s.erase(r0s.begin() + q);
            } else {
                ++q;
            }
        }
        if (r < steps + window) {
            rc = one_step(S);
            if (rc) {
                S->poisoned = 1;
                return rc;
            }
        }
    }
    HIPCHK(S, hipStreamSynchronize(S->s));
    return HK_OK;
}

int hk_set_cnn(hk_sim *S, hk_cnn *cnn) {
    if (!S) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    S->cnn = cnn;
    return HK_OK;
}

int hk_qed_tables(double *We, double *Wb, double *Xe, double *Xb) {
    if (!We || !Wb || !Xe || !Xb) return HK_EINVAL;
    const double *t = hk_qed_host_tables();
    std::memcpy(We, t, sizeof(double) * QED_NCHI);
    std::memcpy(Wb, t + QED_NCHI, sizeof(double) * QED_NCHI);
    std::memcpy(Xe, t + 2 * QED_NCHI, sizeof(double) * QED_NCHI * QED_NU);
    std::memcpy(Xb, t + 2 * QED_NCHI + QED_NCHI * QED_NU, sizeof(double) * QED_NCHI * QED_NU);
    return HK_OK;
}

int hk_real_size(void) { return HK_REAL_BYTES; }

const char *hk_strerror(int code) {
    switch (code) {
    case HK_OK: return "ok";
    case HK_EINVAL: return "invalid argument";
    case HK_ENOMEM: return "out of memory";
    case HK_EDEVICE: return "device error";
    case HK_ENUMERIC: return "numerical failure";
    case HK_EOVERFLOW: return "particle storage overflow";
    case HK_ESTATE: return "context poisoned or call invalid in this state";
    case HK_EIO: return "i/o error";
    case HK_ENOTSUP: return "not supported by this library";
    default: return "unknown error";
    }
}

const char *hk_last_error(const hk_sim *sim) { return sim ? sim->err.c_str() : "no context"; }

int hk_create(const hk_grid_desc *grid, const hk_species_desc *species, int nspecies,
              const hk_laser_desc *laser, const hk_run_desc *run, hk_sim **out) {
    if (!out) return HK_EINVAL;
    *out = nullptr;
    if (!check_grid(grid) || !laser || !run || nspecies < 0 || nspecies > HK_MAX_SPECIES ||
        (nspecies > 0 && !species))
        return HK_EINVAL;
    if (run->switch_mode < HK_SW_ALL_PIC || run->switch_mode > HK_SW_FIXED) return HK_EINVAL;
    if (laser->enabled && (laser->i_antenna < 1 || laser->i_antenna >= grid->nx || laser->duration <= 0 ||
                           laser->waist <= 0 || laser->lambda_um <= 0))
        return HK_EINVAL;
    for (int i = 0; i < nspecies; ++i) {
        const hk_species_desc &d = species[i];
        if (d.kind < HK_ELECTRON || d.kind > HK_PHOTON || d.ppc < 0 || d.ppc > 64) return HK_EINVAL;
        if (d.kind != HK_PHOTON && d.mass <= 0) return HK_EINVAL;
        if (d.ionizable && (d.kind != HK_ION || d.z_max < 1 || d.z_max > HK_MAX_LEVELS ||
                            d.target < 0 || d.target >= nspecies || d.mobile))
            return HK_EINVAL;
    }
    if (run->switch_every < 0 || run->dilation < 0 || run->dilation > 4 || run->hysteresis < 1 ||
        run->hysteresis > 255)
        return HK_EINVAL;
    hk_sim *S = new hk_sim();
    S->gd = *grid;
    S->las = *laser;
    S->run = *run;
    S->nsp = nspecies;
    S->s = (hipStream_t)run->stream;
    GridP &g = S->g;
    g.nx = grid->nx; g.ny = grid->ny; g.nz = grid->nz; g.sx = grid->nx + 1;
    g.bcx = grid->bc_x;
    g.ntx = (g.nx + TILE - 1) / TILE; g.nty = (g.ny + TILE - 1) / TILE; g.ntz = (g.nz + TILE - 1) / TILE;
    g.ntiles = g.ntx * g.nty * g.ntz;
    g.nn = (long long)g.sx * g.ny * g.nz;
    g.dx = (real)grid->dx; g.dy = (real)grid->dy; g.dz = (real)grid->dz; g.dt = (real)grid->dt;
    g.ddx = grid->dx; g.ddy = grid->dy; g.ddz = grid->dz; g.ddt = grid->dt;
    int rc = HK_OK;
    S->fblock = (real *)dalloc(S, sizeof(real) * 9 * (size_t)g.nn);
    S->falt = (real *)dalloc(S, sizeof(real) * 6 * (size_t)g.nn);
    S->jg = (jglob_t *)dalloc(S, sizeof(jglob_t) * 3 * (size_t)g.nn);
    S->mur_old = (real *)dalloc(S, sizeof(real) * 8 * (size_t)g.ny * g.nz);
    S->sw = (uint8_t *)dalloc(S, (size_t)g.nn);
    S->calm = (uint8_t *)dalloc(S, (size_t)g.nn);
    S->gauss0 = (double *)dalloc(S, sizeof(double) * (size_t)g.nn);
    S->tmp_a = (double *)dalloc(S, sizeof(double) * (size_t)g.nn);
    S->tmp_b = (double *)dalloc(S, sizeof(double) * (size_t)g.nn);
    S->dsum = (double *)dalloc(S, sizeof(double) * 64);
    S->ledger = (double *)dalloc(S, sizeof(double) * 8);
    S->status = (int *)dalloc(S, sizeof(int) * HK_NSTATUS);
    S->dstat = (unsigned long long *)dalloc(S, sizeof(unsigned long long) * 4);
    // species weight bounds, plus one spare slot that QED kernels may raise
    // when a sink species does not exist
    S->wmax = (unsigned *)dalloc(S, sizeof(unsigned) * (HK_MAX_SPECIES + 1));
    S->plan = (int2 *)dalloc(S, sizeof(int2) * (size_t)tile_plan_items(g));
    S->plan_ctl = (int *)dalloc(S, sizeof(int) * PLAN_CTL);
    if (hipHostMalloc((void **)&S->h_status, sizeof(int) * HK_NSTATUS, 0) != hipSuccess)
        S->h_status = nullptr;
    if (hipEventCreateWithFlags(&S->status_ev, hipEventDisableTiming) != hipSuccess)
        S->status_ev = nullptr;
    if (!S->fblock || !S->falt || !S->jg || !S->mur_old || !S->sw || !S->calm || !S->gauss0 || !S->tmp_a || !S->tmp_b ||
        !S->dsum || !S->ledger || !S->status || !S->h_status || !S->dstat || !S->wmax ||
        !S->plan || !S->plan_ctl || !S->status_ev) {
        hk_destroy(S);
        return HK_ENOMEM;
    }
    for (int c = 0; c < 9; ++c) S->f[c] = S->fblock + (size_t)c * g.nn;
    for (int c = 0; c < 6; ++c) S->f_alt[c] = S->falt + (size_t)c * g.nn;
    (void)hipMemsetAsync(S->sw, run->switch_mode == HK_SW_ALL_FLUID ? 0 : 1, (size_t)g.nn, S->s);
    for (int i = 0; i < nspecies; ++i) {
        DevSpecies &D = S->sp[i];
        D.d = species[i];
        D.has_z = D.d.kind == HK_ION;
        D.has_tau = D.d.qed != 0;
    }
    if (run->enable_qed) {
        for (int i = nspecies - 1; i >= 0; --i) {
            if (species[i].kind == HK_PHOTON) S->photon_sp = i;
            if (species[i].kind == HK_ELECTRON) S->electron_sp = i;
            if (species[i].kind == HK_POSITRON) S->positron_sp = i;
        }
        // bins for the particles QED creates: photons up to the QED leptons'
        // count, pairs a quarter of that (re-binning grows them when needed)
        long long leptons = 0;
        for (int i = 0; i < nspecies; ++i)
            if (species[i].qed && (species[i].kind == HK_ELECTRON || species[i].kind == HK_POSITRON))
                leptons += initial_count(*grid, species[i]);
        if (S->photon_sp >= 0) S->sp[S->photon_sp].reserve_hint += leptons;
        if (S->electron_sp >= 0) S->sp[S->electron_sp].reserve_hint += leptons / 4;
        if (S->positron_sp >= 0) S->sp[S->positron_sp].reserve_hint += leptons / 4;
        double omega0 = 2.0 * PI * PHYS_C / (laser->lambda_um * 1e-6);
        S->a_s = PHYS_ME * PHYS_C * PHYS_C / (PHYS_HBAR * omega0);
        const size_t nt = 2 * QED_NCHI + 2 * (size_t)QED_NCHI * QED_NU;
        S->qed_tab = (double *)dalloc(S, sizeof(double) * nt);
        if (!S->qed_tab) rc = HK_ENOMEM;
        else if (hipMemcpyAsync(S->qed_tab, hk_qed_host_tables(), sizeof(double) * nt,
                                hipMemcpyHostToDevice, S->s) != hipSuccess) rc = HK_EDEVICE;
    }
    // ionization targets: reserve bins for the electrons the ions can free
    for (int i = 0; i < nspecies; ++i)
        if (species[i].ionizable && run->enable_ionization) {
            S->sp[species[i].target].reserve_hint += initial_count(*grid, species[i]) * species[i].z_max;
        }
    for (int i = 0; i < nspecies && rc == HK_OK; ++i) rc = init_species(S, i);
    for (int i = 0; i < nspecies && rc == HK_OK; ++i)
        if (species[i].ionizable && run->enable_ionization) {
            rc = build_ion_table(S, i);
            unsigned b = 0;
            if (rc == HK_OK && hipMemcpy(&b, S->wmax + i, 4, hipMemcpyDeviceToHost) != hipSuccess) rc = HK_EDEVICE;
            float f;
            std::memcpy(&f, &b, 4);
            if (rc == HK_OK) rc = raise_wmax(S, species[i].target, f);
        }
    if (rc == HK_OK && run->enable_qed) {
        // photons carry their parent's weight and pairs their photon's: one bound
        // covers the leptons and photons of QED (spawns raise it further)
        float wq = 0.f;
        for (int i = 0; i < nspecies && rc == HK_OK; ++i) {
            if (species[i].kind == HK_ION) continue;
            unsigned b = 0;
            if (hipMemcpy(&b, S->wmax + i, 4, hipMemcpyDeviceToHost) != hipSuccess) rc = HK_EDEVICE;
            float f;
            std::memcpy(&f, &b, 4);
            wq = std::max(wq, f);
        }
        for (int i = 0; i < nspecies && rc == HK_OK; ++i)
            if (species[i].kind != HK_ION) rc = raise_wmax(S, i, wq);
    }
    for (int i = 0; i < nspecies && rc == HK_OK; ++i) rc = ensure_inbox(S, i, inbox_need(S, i));
    if (rc == HK_OK && run->switch_mode != HK_SW_ALL_PIC) rc = ensure_fluid(S);
    if (rc == HK_OK && hipStreamSynchronize(S->s) != hipSuccess) rc = HK_EDEVICE;
    if (rc != HK_OK) {
        hk_destroy(S);
        return rc;
    }
    *out = S;
    return HK_OK;
}

void hk_destroy(hk_sim *S) {
    if (!S) return;
    if (S->s) (void)hipStreamSynchronize(S->s);
    else (void)hipDeviceSynchronize();
    std::vector<void *> all = S->allocs;
    for (void *p : all) dfree(S, p);
    if (S->h_status) (void)hipHostFree(S->h_status);
    ev_resolve(S);
    for (hipEvent_t e : S->ev_free) (void)hipEventDestroy(e);
    if (S->last_mark) (void)hipEventDestroy(S->last_mark);
    if (S->status_ev) (void)hipEventDestroy(S->status_ev);
    delete S;
}

int hk_step(hk_sim *S, int nsteps) {
    if (!S || nsteps < 0) return HK_EINVAL;
    if (S->poisoned) return fail(S, HK_ESTATE, "context poisoned: %s", S->err.c_str());
    if (!S->have_gauss0) {
        int rc = gauss_snapshot(S);
        if (rc) return rc;
    }
    for (int n = 0; n < nsteps; ++n) {
        int rc = one_step(S);
        // a step that stops part-way leaves particles or fluid half-moved:
        // nothing may run on that state
        if (rc) {
            S->poisoned = 1;
            return rc;
        }
    }
    HIPCHK(S, hipStreamSynchronize(S->s));
    return HK_OK;
}

int hk_set_switch_mode(hk_sim *S, int mode) {
    if (!S || mode < HK_SW_ALL_PIC || mode > HK_SW_FIXED) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    if (mode == HK_SW_ALL_PIC) {
        for (int i = 0; i < S->nsp; ++i)
            if (S->sp[i].fn) return fail(S, HK_ESTATE, "fluid present: cannot return to all-PIC");
    }
    S->run.switch_mode = mode;
    if (mode != HK_SW_ALL_PIC) {
        int rc = ensure_fluid(S);
        if (rc) return rc;
    }
    if (mode == HK_SW_ALL_PIC || mode == HK_SW_ALL_FLUID)
        HIPCHK(S, hipMemsetAsync(S->sw, mode == HK_SW_ALL_PIC ? 1 : 0, (size_t)S->g.nn, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    return HK_OK;
}

int hk_switch_map(hk_sim *S, uint8_t *out, size_t n) {
    if (!S || !out || n != (size_t)S->g.nn) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    HIPCHK(S, hipMemcpyAsync(out, S->sw, n, hipMemcpyDeviceToHost, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    return HK_OK;
}

int hk_set_switch_map(hk_sim *S, const uint8_t *in, size_t n) {
    if (!S || !in || n != (size_t)S->g.nn) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    S->run.switch_mode = HK_SW_FIXED;
    int rc = ensure_fluid(S);
    if (rc) return rc;
    HIPCHK(S, hipMemcpyAsync(S->sw, in, n, hipMemcpyHostToDevice, S->s));
    HIPCHK(S, hipMemsetAsync(S->calm, 0, n, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    return HK_OK;
}

int hk_get_field(hk_sim *S, int comp, void *host_out, size_t bytes) {
    if (!S || !host_out || comp < 0 || comp >= HK_NCOMP || bytes != sizeof(real) * (size_t)S->g.nn)
        return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    HIPCHK(S, hipMemcpyAsync(host_out, S->f[comp], bytes, hipMemcpyDeviceToHost, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    return HK_OK;
}

int hk_set_field(hk_sim *S, int comp, const void *host_in, size_t bytes) {
    if (!S || !host_in || comp < 0 || comp >= HK_NCOMP || bytes != sizeof(real) * (size_t)S->g.nn)
        return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    HIPCHK(S, hipMemcpyAsync(S->f[comp], host_in, bytes, hipMemcpyHostToDevice, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    S->have_gauss0 = 0;
    return HK_OK;
}

int hk_node_state(hk_sim *S, float *dev_out, size_t nodes) {
    if (!S || !dev_out) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    const GridP &g = S->g;
    const size_t n = (size_t)(g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1) * g.ny * g.nz;
    if (nodes != n) return fail(S, HK_EINVAL, "node count %zu, expected %zu", nodes, n);
    rho_total(S, S->tmp_a);
    cnn_launch_node_state(g, S->f, S->tmp_a, dev_out, S->s);
    HIPCHK(S, hipStreamSynchronize(S->s));
    return HK_OK;
}

int hk_get_rho(hk_sim *S, double *host_out, size_t n) {
    if (!S || !host_out || n != (size_t)S->g.nn) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    rho_total(S, S->tmp_a);
    HIPCHK(S, hipMemcpyAsync(host_out, S->tmp_a, sizeof(double) * n, hipMemcpyDeviceToHost, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    return HK_OK;
}

int hk_get_divE(hk_sim *S, double *host_out, size_t n) {
    if (!S || !host_out || n != (size_t)S->g.nn) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    launch_divE(S->g, S->f, S->tmp_a, S->s);
    HIPCHK(S, hipMemcpyAsync(host_out, S->tmp_a, sizeof(double) * n, hipMemcpyDeviceToHost, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    return HK_OK;
}


int hk_particle_count(hk_sim *S, int isp, size_t *n) {
    if (!S || !n || isp < 0 || isp >= S->nsp) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    std::vector<long long> slots;
    int rc = valid_slots(S, S->sp[isp], slots);
    if (rc) return rc;
    *n = slots.size();
    return HK_OK;
}

int hk_get_particles(hk_sim *S, int isp, const hk_particles *out) {
    if (!S || !out || isp < 0 || isp >= S->nsp) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    DevSpecies &D = S->sp[isp];
    std::vector<long long> slots;
    int rc = valid_slots(S, D, slots);
    if (rc) return rc;
    const size_t n = slots.size();
    if (out->n != n) return fail(S, HK_EINVAL, "hk_get_particles: n = %zu, have %zu", out->n, n);
    if (n == 0) return HK_OK;
    const long long C = D.capacity;
    std::vector<int> cell(C), zc(D.has_z ? C : 0);
    std::vector<real> r[7];
    for (auto &v : r) v.resize(C);
    std::vector<uint64_t> id(C);
    std::vector<double> tau(D.has_tau ? C : 0);
    const PArr &a = D.buf[D.cur];
    hipStream_t s = S->s;
    HIPCHK(S, hipMemcpyAsync(cell.data(), a.cell, sizeof(int) * C, hipMemcpyDeviceToHost, s));
    real *src[7] = {a.rx, a.ry, a.rz, a.ux, a.uy, a.uz, a.w};
    for (int k = 0; k < 7; ++k)
        HIPCHK(S, hipMemcpyAsync(r[k].data(), src[k], sizeof(real) * C, hipMemcpyDeviceToHost, s));
    HIPCHK(S, hipMemcpyAsync(id.data(), a.id, sizeof(uint64_t) * C, hipMemcpyDeviceToHost, s));
    if (D.has_z) HIPCHK(S, hipMemcpyAsync(zc.data(), a.zc, sizeof(int) * C, hipMemcpyDeviceToHost, s));
    if (D.has_tau) HIPCHK(S, hipMemcpyAsync(tau.data(), a.tau, sizeof(double) * C, hipMemcpyDeviceToHost, s));
    HIPCHK(S, hipStreamSynchronize(s));
    const GridP &g = S->g;
    for (size_t q = 0; q < n; ++q) {
        const long long i = slots[q];
        int c = cell[i];
        int ci = c % g.nx, cj = (c / g.nx) % g.ny, ck = c / (g.nx * g.ny);
        if (out->x) {
            out->x[3 * q] = (ci + (double)r[0][i]) * g.ddx;
            out->x[3 * q + 1] = (cj + (double)r[1][i]) * g.ddy;
            out->x[3 * q + 2] = (ck + (double)r[2][i]) * g.ddz;
        }
        if (out->u) {
            out->u[3 * q] = r[3][i]; out->u[3 * q + 1] = r[4][i]; out->u[3 * q + 2] = r[5][i];
        }
        if (out->w) out->w[q] = r[6][i];
        if (out->id) out->id[q] = id[i];
        if (out->z) out->z[q] = D.has_z ? zc[i] : (int32_t)std::llround(D.d.charge);
        if (out->tau) out->tau[q] = D.has_tau ? tau[i] : 0.0;
    }
    return HK_OK;
}

int hk_set_particles(hk_sim *S, int isp, const hk_particles *in) {
    if (!S || !in || isp < 0 || isp >= S->nsp || (in->n > 0 && (!in->x || !in->u || !in->w)))
        return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    DevSpecies &D = S->sp[isp];
    const GridP &g = S->g;
    D.umax_ok = false;   // momenta set from the host: the next evaluation scans them
    const size_t n = in->n;
    std::vector<int> cell(n), zc(n);
    std::vector<real> r[7];
    for (auto &v : r) v.resize(n);
    std::vector<uint64_t> id(n);
    std::vector<double> tau(n, 0.0);
    const double dxs[3] = {g.ddx, g.ddy, g.ddz};
    const int dims[3] = {g.nx, g.ny, g.nz};
    for (size_t q = 0; q < n; ++q) {
        int c[3];
        for (int d = 0; d < 3; ++d) {
            double X = in->x[3 * q + d] / dxs[d];
            c[d] = (int)std::floor(X);
            if (c[d] < 0 || c[d] >= dims[d]) return fail(S, HK_EINVAL, "particle %zu outside the box", q);
            r[d][q] = (real)(X - c[d]);
            if (r[d][q] >= (real)1) r[d][q] = std::nextafter((real)1, (real)0);
        }
        cell[q] = c[0] + g.nx * (c[1] + g.ny * c[2]);
        for (int d = 0; d < 3; ++d) r[3 + d][q] = (real)in->u[3 * q + d];
        r[6][q] = (real)in->w[q];
        id[q] = in->id ? in->id[q] : q;
        zc[q] = in->z ? in->z[q] : (int)std::llround(D.d.charge);
        if (in->tau) tau[q] = in->tau[q];
        else if (D.has_tau) tau[q] = tau0(S->run.seed, id[q]);   // as a new particle draws it
    }
    double wm = 0;
    for (size_t q = 0; q < n; ++q) wm = std::max(wm, std::fabs(in->w[q]));
    int rc = upload_particles(S, isp, n, cell, r, id, zc, tau, wm);
    S->have_gauss0 = 0;
    return rc;
}


int hk_get_fluid(hk_sim *S, int isp, double *n, double *u, size_t nodes) {
    if (!S || !n || !u || isp < 0 || isp >= S->nsp || nodes != (size_t)S->g.nn) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    DevSpecies &D = S->sp[isp];
    if (!D.fn) return fail(S, HK_EINVAL, "species %d has no fluid", isp);
    std::vector<real> h[4];
    real *src[4] = {D.fn, D.fu[0], D.fu[1], D.fu[2]};
    for (int q = 0; q < 4; ++q) {
        h[q].resize(nodes);
        HIPCHK(S, hipMemcpyAsync(h[q].data(), src[q], sizeof(real) * nodes, hipMemcpyDeviceToHost, S->s));
    }
    HIPCHK(S, hipStreamSynchronize(S->s));
    for (size_t c = 0; c < nodes; ++c) {
        n[c] = h[0][c];
        for (int d = 0; d < 3; ++d) u[3 * c + d] = h[1 + d][c];
    }
    return HK_OK;
}

int hk_set_fluid(hk_sim *S, int isp, const double *n, const double *u, size_t nodes) {
    if (!S || !n || !u || isp < 0 || isp >= S->nsp || nodes != (size_t)S->g.nn) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    DevSpecies &D = S->sp[isp];
    if (!D.fn) return fail(S, HK_EINVAL, "species %d has no fluid", isp);
    std::vector<real> h[4];
    for (int q = 0; q < 4; ++q) h[q].resize(nodes);
    for (size_t c = 0; c < nodes; ++c) {
        h[0][c] = (real)n[c];
        for (int d = 0; d < 3; ++d) h[1 + d][c] = (real)u[3 * c + d];
    }
    real *dst[4] = {D.fn, D.fu[0], D.fu[1], D.fu[2]};
    for (int q = 0; q < 4; ++q)
        HIPCHK(S, hipMemcpyAsync(dst[q], h[q].data(), sizeof(real) * nodes, hipMemcpyHostToDevice, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    S->have_gauss0 = 0;
    return set_fluid_window(S, isp, true);   // fluid may sit anywhere now
}

// Warm fluid pressure p = S n^(gamma_ad - 1) per node (host FP64); setting
// converts with the density already on the device.
int hk_get_fluid_p(hk_sim *S, int isp, double *p, size_t nodes) {
    if (!S || !p || isp < 0 || isp >= S->nsp || nodes != (size_t)S->g.nn) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    DevSpecies &D = S->sp[isp];
    if (!D.fs) return fail(S, HK_EINVAL, "species %d has no warm fluid", isp);
    std::vector<real> hn(nodes), hs(nodes);
    HIPCHK(S, hipMemcpyAsync(hn.data(), D.fn, sizeof(real) * nodes, hipMemcpyDeviceToHost, S->s));
    HIPCHK(S, hipMemcpyAsync(hs.data(), D.fs, sizeof(real) * nodes, hipMemcpyDeviceToHost, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    for (size_t c = 0; c < nodes; ++c)
        p[c] = hn[c] > 0 ? (double)hs[c] * std::pow((double)hn[c], D.d.gamma_ad - 1.0) : 0.0;
    return HK_OK;
}

int hk_set_fluid_p(hk_sim *S, int isp, const double *p, size_t nodes) {
    if (!S || !p || isp < 0 || isp >= S->nsp || nodes != (size_t)S->g.nn) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    DevSpecies &D = S->sp[isp];
    if (!D.fs) return fail(S, HK_EINVAL, "species %d has no warm fluid", isp);
    std::vector<real> hn(nodes), hs(nodes);
    HIPCHK(S, hipMemcpyAsync(hn.data(), D.fn, sizeof(real) * nodes, hipMemcpyDeviceToHost, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    for (size_t c = 0; c < nodes; ++c)
        hs[c] = hn[c] > 0 ? (real)(p[c] * std::pow((double)hn[c], 1.0 - D.d.gamma_ad)) : (real)0;
    HIPCHK(S, hipMemcpyAsync(D.fs, hs.data(), sizeof(real) * nodes, hipMemcpyHostToDevice, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    return set_fluid_window(S, isp, true);
}

int hk_enable_timing(hk_sim *S, int on) {
    if (!S) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    ev_resolve(S);
    S->timing = on != 0;
    for (int i = 0; i < HK_NTIMERS; ++i)
        if (i != 7) S->timers[i] = 0;
    HIPCHK(S, hipMemcpyAsync(S->stat0, S->dstat, sizeof(S->stat0), hipMemcpyDeviceToHost, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    return HK_OK;
}

int hk_timers(hk_sim *S, double *ms, int n) {
    if (!S || !ms || n < 0) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    ev_resolve(S);
    unsigned long long now[2];
    HIPCHK(S, hipMemcpyAsync(now, S->dstat, sizeof(now), hipMemcpyDeviceToHost, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    S->timers[9] = (double)(now[0] - S->stat0[0]);
    S->timers[10] = (double)(now[1] - S->stat0[1]);
    for (int i = 0; i < n && i < HK_NTIMERS; ++i) ms[i] = S->timers[i];
    return HK_OK;
}

int hk_diagnostics(hk_sim *S, hk_diag *d) {
    if (!S || !d) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    hipStream_t s = S->s;
    const GridP &g = S->g;
    if (!S->have_gauss0) gauss_snapshot(S);
    std::memset(d, 0, sizeof(*d));
    launch_zero(S->dsum, sizeof(double) * 64, s);
    launch_field_energy(g, S->f, S->dsum, s);
    for (int isp = 0; isp < S->nsp; ++isp) {
        DevSpecies &D = S->sp[isp];
        SpecP P = specp(D);
        if (D.capacity) launch_particle_sums(g, P, D.buf[D.cur], cur_bins(D), S->dsum + 2 + 3 * isp, s);
        if (D.fn) launch_fluid_sums(g, P, D.fn, D.fu[0], D.fu[1], D.fu[2], S->dsum + 20 + 3 * isp, s);
        if (D.fs) launch_fluid_heat(g, D.fn, WarmP{D.fs, D.d.gamma_ad}, S->dsum + 46 + isp, s);
    }
    // Gauss: (divE - rho) now minus (divE - rho) at the snapshot
    launch_divE(g, S->f, S->tmp_a, s);
    rho_total(S, S->tmp_b);
    launch_gauss(g, S->tmp_a, S->tmp_b, S->gauss0, S->las.enabled ? S->las.i_antenna : -1,
                 S->dsum + 40, s);
    launch_count_kinetic(g, S->sw, S->dsum + 44, s);
    double h[64], led[8];
    HIPCHK(S, hipMemcpyAsync(h, S->dsum, sizeof(double) * 64, hipMemcpyDeviceToHost, s));
    HIPCHK(S, hipMemcpyAsync(led, S->ledger, sizeof(double) * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(S, hipStreamSynchronize(s));
    d->t = S->t;
    d->step = S->step;
    d->u_e = h[0];
    d->u_b = h[1];
    for (int isp = 0; isp < S->nsp; ++isp) {
        d->kin[isp] = h[2 + 3 * isp];
        d->count[isp] = h[3 + 3 * isp];
        d->charge_total += h[4 + 3 * isp];
        d->fluid_kin[isp] = h[20 + 3 * isp];
        d->fluid_mass[isp] = h[21 + 3 * isp];
        d->charge_total += h[22 + 3 * isp];
        d->fluid_th[isp] = h[46 + isp];
    }
    d->gauss_l2 = h[41] > 0 ? std::sqrt(h[40] / h[41]) : 0.0;
    uint64_t mb;
    std::memcpy(&mb, &h[42], 8);
    double mx;
    std::memcpy(&mx, &mb, 8);
    d->gauss_max = mx;
    d->kinetic_fraction = h[45] > 0 ? h[44] / h[45] : 0.0;
    d->conv_loss = led[0];
    d->ion_energy = led[1];
    d->photon_energy = led[2];
    d->fallback_fraction = 0.0;
    if (S->run.switch_mode == HK_SW_CNN) {
        int nf = 0;
        if (S->cnn && !S->cnn_nfall) {
            d->fallback_fraction = 0.0;   // not evaluated yet
        } else if (S->cnn) {
            HIPCHK(S, hipMemcpyAsync(&nf, S->cnn_nfall, sizeof(int), hipMemcpyDeviceToHost, S->s));
            HIPCHK(S, hipStreamSynchronize(S->s));
            const int NX = g.bcx == HK_BC_PERIODIC ? g.nx : g.nx + 1;
            d->fallback_fraction = (double)nf / ((double)NX * g.ny * g.nz);
        } else {
            d->fallback_fraction = 1.0;   // no network: every node decided by the thresholds
        }
    }
    return HK_OK;
}


// ------------------------------------------------------------------ checkpoint ----------
// File: "HKCK", version, real size, grid and species kinds (checked on load),
// step and time, then fixed sections in order: the 9 field components, the
// Mur planes, switch map and calm counters, ledgers, species weight bounds,
// the Gauss baseline, CNN evaluation count, then per species the particles
// (count, then cell, offsets, u, w, id, z, tau in the library's own layout)
// and the fluid (n, u) when the species has one.  Little endian, as written.

int hk_save(hk_sim *S, const char *path) {
    if (!S || !path) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    ev_resolve(S);
    CkFile F;
    F.f = fopen(path, "wb");
    if (!F.f) return fail(S, HK_EIO, "checkpoint: cannot open %s for writing", path);
    const GridP &g = S->g;
    F.put(CK_MAGIC); F.put(CK_VERSION); F.put((uint32_t)sizeof(real));
    F.put(g.nx); F.put(g.ny); F.put(g.nz); F.put(S->nsp);
    for (int i = 0; i < S->nsp; ++i) F.put(S->sp[i].d.kind);
    F.put(S->step); F.put(S->t); F.put(S->have_gauss0);
    int rc;
    // the nine field arrays in component order (the current E and B set)
    for (int c = 0; c < 9; ++c)
        if ((rc = ck_dev_out(S, F, S->f[c], sizeof(real) * (size_t)g.nn))) return rc;
    if ((rc = ck_dev_out(S, F, S->mur_old, sizeof(real) * 8 * (size_t)g.ny * g.nz))) return rc;
    if ((rc = ck_dev_out(S, F, S->sw, (size_t)g.nn))) return rc;
    if ((rc = ck_dev_out(S, F, S->calm, (size_t)g.nn))) return rc;
    if ((rc = ck_dev_out(S, F, S->ledger, sizeof(double) * 8))) return rc;
    if ((rc = ck_dev_out(S, F, S->wmax, sizeof(unsigned) * (HK_MAX_SPECIES + 1)))) return rc;
    if ((rc = ck_dev_out(S, F, S->gauss0, S->have_gauss0 ? sizeof(double) * (size_t)g.nn : 0))) return rc;
    F.put(S->cnn_evals);
    for (int isp = 0; isp < S->nsp; ++isp) {
        DevSpecies &D = S->sp[isp];
        std::vector<long long> slots;
        if ((rc = valid_slots(S, D, slots))) return rc;
        const uint64_t n = slots.size();
        F.put(n);
        const long long C = D.capacity;
        const PArr &a = D.buf[D.cur];
        // one field at a time: copy the whole buffer, keep the valid slots
        auto field = [&](const void *dev, size_t esz) -> int {
            std::vector<char> h((size_t)C * esz), o((size_t)n * esz);
            if (C) HIPCHK(S, hipMemcpyAsync(h.data(), dev, (size_t)C * esz, hipMemcpyDeviceToHost, S->s));
            HIPCHK(S, hipStreamSynchronize(S->s));
            for (uint64_t q = 0; q < n; ++q) memcpy(&o[q * esz], &h[(size_t)slots[q] * esz], esz);
            F.put(o.data(), o.size());
            return HK_OK;
        };
        if ((rc = field(a.cell, sizeof(int)))) return rc;
        const real *rs[7] = {a.rx, a.ry, a.rz, a.ux, a.uy, a.uz, a.w};
        for (const real *r : rs)
            if ((rc = field(r, sizeof(real)))) return rc;
        if ((rc = field(a.id, sizeof(uint64_t)))) return rc;
        if (D.has_z && (rc = field(a.zc, sizeof(int)))) return rc;
        if (D.has_tau && (rc = field(a.tau, sizeof(double)))) return rc;
        // 0: no fluid; 1: n and u; 2: n, u and the warm fluid's entropy density
        const int has_fluid = D.fn == nullptr ? 0 : (D.fs ? 2 : 1);
        F.put(has_fluid);
        if (has_fluid) {
            real *fl[4] = {D.fn, D.fu[0], D.fu[1], D.fu[2]};
            for (real *q : fl)
                if ((rc = ck_dev_out(S, F, q, sizeof(real) * (size_t)g.nn))) return rc;
            if (has_fluid == 2 && (rc = ck_dev_out(S, F, D.fs, sizeof(real) * (size_t)g.nn))) return rc;
        }
    }
    if (!F.ok) return fail(S, HK_EIO, "checkpoint: write to %s failed", path);
    return HK_OK;
}

static int load_body(hk_sim *S, CkFile &F, const char *path, const GridP &g, int nsp, int64_t step, double t,
                     int have_g0) {
    int rc;
    for (int c = 0; c < 9; ++c)
        if ((rc = ck_dev_in(S, F, S->f[c], sizeof(real) * (size_t)g.nn))) return rc;
    if ((rc = ck_dev_in(S, F, S->mur_old, sizeof(real) * 8 * (size_t)g.ny * g.nz))) return rc;
    if ((rc = ck_dev_in(S, F, S->sw, (size_t)g.nn))) return rc;
    if ((rc = ck_dev_in(S, F, S->calm, (size_t)g.nn))) return rc;
    if ((rc = ck_dev_in(S, F, S->ledger, sizeof(double) * 8))) return rc;
    std::vector<unsigned> wmax(HK_MAX_SPECIES + 1);
    F.get(wmax.data(), sizeof(unsigned) * wmax.size());
    if ((rc = ck_dev_in(S, F, S->gauss0, have_g0 ? sizeof(double) * (size_t)g.nn : 0))) return rc;
    uint32_t evals = 0;
    F.get(evals);
    for (int isp = 0; isp < nsp; ++isp) {
        DevSpecies &D = S->sp[isp];
        uint64_t n = 0;
        F.get(n);
        if (!F.ok || n > (uint64_t)INT_MAX) return fail(S, HK_EIO, "checkpoint: bad particle count");
        std::vector<int> cell(n), zc(n);
        std::vector<real> r[7];
        std::vector<uint64_t> id(n);
        std::vector<double> tau(n, 0.0);
        F.get(cell.data(), sizeof(int) * n);
        for (auto &v : r) { v.resize(n); F.get(v.data(), sizeof(real) * n); }
        F.get(id.data(), sizeof(uint64_t) * n);
        if (D.has_z) F.get(zc.data(), sizeof(int) * n);
        if (D.has_tau) F.get(tau.data(), sizeof(double) * n);
        if (!F.ok) return fail(S, HK_EIO, "checkpoint: file ends early");
        for (uint64_t q = 0; q < n; ++q)
            if (cell[q] < 0 || cell[q] >= g.nx * g.ny * g.nz) return fail(S, HK_EIO, "checkpoint: bad cell");
        double wm = 0;
        for (uint64_t q = 0; q < n; ++q) wm = std::max(wm, std::fabs((double)r[6][q]));
        if ((rc = upload_particles(S, isp, n, cell, r, id, zc, tau, wm))) return rc;
        int has_fluid = 0;
        F.get(has_fluid);
        if (has_fluid) {
            if ((rc = ensure_fluid(S))) return rc;
            if (!D.fn) return fail(S, HK_EINVAL, "checkpoint: species %d has a fluid here only in the file", isp);
            if ((has_fluid == 2) != (D.fs != nullptr))
                return fail(S, HK_EINVAL, "checkpoint: species %d is warm in one of file and run only", isp);
            real *fl[4] = {D.fn, D.fu[0], D.fu[1], D.fu[2]};
            for (real *q : fl)
                if ((rc = ck_dev_in(S, F, q, sizeof(real) * (size_t)g.nn))) return rc;
            if (has_fluid == 2 && (rc = ck_dev_in(S, F, D.fs, sizeof(real) * (size_t)g.nn))) return rc;
            if ((rc = set_fluid_window(S, isp, true))) return rc;
        }
    }
    if (!F.ok) return fail(S, HK_EIO, "checkpoint: file ends early");
    // weight bounds exactly as saved (they set the fixed-point scales)
    HIPCHK(S, hipMemcpyAsync(S->wmax, wmax.data(), sizeof(unsigned) * wmax.size(), hipMemcpyHostToDevice, S->s));
    HIPCHK(S, hipStreamSynchronize(S->s));
    S->step = step;
    S->t = t;
    S->have_gauss0 = have_g0;
    S->cnn_evals = evals;
    return HK_OK;
}

int hk_load(hk_sim *S, const char *path) {
    if (!S || !path) return HK_EINVAL;
    if (S->poisoned) return HK_ESTATE;
    ev_resolve(S);
    CkFile F;
    F.f = fopen(path, "rb");
    if (!F.f) return fail(S, HK_EIO, "checkpoint: cannot open %s", path);
    const GridP &g = S->g;
    uint32_t magic = 0, version = 0, rsz = 0;
    int nx = 0, ny = 0, nz = 0, nsp = 0;
    F.get(magic); F.get(version); F.get(rsz);
    F.get(nx); F.get(ny); F.get(nz); F.get(nsp);
    if (!F.ok || magic != CK_MAGIC || version != CK_VERSION)
        return fail(S, HK_EIO, "checkpoint: %s is not a checkpoint of this version", path);
    if (rsz != sizeof(real) || nx != g.nx || ny != g.ny || nz != g.nz || nsp != S->nsp)
        return fail(S, HK_EINVAL, "checkpoint: precision, grid or species count differ from this context");
    for (int i = 0; i < nsp; ++i) {
        int kind = -1;
        F.get(kind);
        if (kind != S->sp[i].d.kind) return fail(S, HK_EINVAL, "checkpoint: species %d has another kind", i);
    }
    int64_t step = 0;
    double t = 0;
    int have_g0 = 0;
    F.get(step); F.get(t); F.get(have_g0);
    // from here on the context is overwritten: a failure leaves it partly
    // restored, so it is poisoned
    const int rc = load_body(S, F, path, g, nsp, step, t, have_g0);
    if (rc) S->poisoned = 1;
    return rc;
}

}  // extern "C"
