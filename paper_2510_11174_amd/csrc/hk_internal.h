// Internal declarations of the MI355X hybrid-step library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hk.h"

#ifdef HK_DOUBLE
typedef double real;
#define HK_REAL_BYTES 8
#else
typedef float real;
#define HK_REAL_BYTES 4
#endif

// Global accumulator of the current that particles deposit (push, absorption
// and spawning moves), converted into J once per step before the field
// update.  FP32 build: 64-bit fixed point with JG_BITS fractional bits, so
// the integer sums are exact and the current does not depend on the order in
// which workgroups add (two runs of the same input give the same bits; the
// range is +-2^(63 - JG_BITS) = 32768 in units of n_c e c).  FP64 build: FP64
// sums.
#ifdef HK_DOUBLE
typedef double jglob_t;
#else
typedef unsigned long long jglob_t;
#endif
#define JG_BITS 48

// Particles are binned in cubic tiles of TILE^3 cells; one workgroup owns a tile.
#define TILE 8
#define TLOG 3

// Grid parameters passed by value to every kernel.
struct GridP {
    int nx, ny, nz, sx;         // sx = nx + 1: x extent of every grid array
    int bcx;                    // HK_BC_PERIODIC / HK_BC_OPEN
    int ntx, nty, ntz, ntiles;  // tiles per axis
    long long nn;               // nodes in the canonical layout: sx * ny * nz
    real dx, dy, dz, dt;
    double ddx, ddy, ddz, ddt;  // the same in FP64 (set-up, antenna, diagnostics)
};

__host__ __device__ inline long long gidx(const GridP &g, int i, int j, int k) {
    return (long long)i + (long long)g.sx * ((long long)j + (long long)g.ny * (long long)k);
}
// (i, j, k) of canonical node c; node counts stay below 2^31 (checked when a
// simulation is created), so 32-bit unsigned division is exact
__device__ inline void node_ijk(const GridP &g, long long c, int &i, int &j, int &k) {
    const unsigned u = (unsigned)c, sx = (unsigned)g.sx, ny = (unsigned)g.ny;
    const unsigned r = u / sx;
    i = (int)(u - r * sx);
    j = (int)(r % ny);
    k = (int)(r / ny);
}
__host__ __device__ inline int wrapi(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

// ---------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): counter (id lo, id hi, step, tag<<8|draw),
// key (seed lo, seed hi).  Ten rounds; the key advances by the Weyl constants
// between rounds.
__host__ __device__ inline void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t a = (uint64_t)0xD2511F53u * c0;
        uint64_t b = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
        uint32_t n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

__host__ __device__ inline void draw4(uint64_t seed, uint64_t id, uint32_t step, uint32_t tag,
                                      uint32_t draw, uint32_t out[4]) {
    philox10((uint32_t)id, (uint32_t)(id >> 32), step, (tag << 8) | draw, (uint32_t)seed,
             (uint32_t)(seed >> 32), out);
}

// Uniform in (0,1) with 24 significant bits: exact in FP32 and FP64 alike.
__host__ __device__ inline real u01(uint32_t x) {
    return ((real)(x >> 9) + (real)0.5) * (real)(1.0 / 8388608.0);
}
__host__ __device__ inline double u01d(uint32_t x) {
    return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0);
}

// Philox tags (one stream per purpose).
enum { TAG_POS = 1, TAG_MOM = 2, TAG_ION = 3, TAG_CONV = 12, TAG_CONV_TH = 13, TAG_EMIT = 16,
       TAG_TAU = 17, TAG_PAIR = 18, TAG_DROP = 24 };

// Ids of particles born in QED events: splitmix64 (S. Vigna's finaliser)
// of the parent id mixed with the step and the kind k (1 photon, 2 electron,
// 3 positron); collisions are as unlikely as for any 64-bit hash.
__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t child_id(uint64_t parent, uint32_t step, uint32_t k) {
    return splitmix64(parent ^ splitmix64(((uint64_t)step << 8) | k));
}
// Optical depth of a new QED particle: -ln(1 - r), r drawn from its id alone.
__host__ __device__ inline double tau0(uint64_t seed, uint64_t id) {
    uint32_t r[4];
    draw4(seed, id, 0xffffffffu, TAG_TAU, 0, r);
    return -log(1.0 - u01d(r[0]));
}

// ---------------------------------------------------------------------------------------
// Particle storage: structure of arrays, binned per tile.  Tile t owns slots
// [off[t], off[t] + cap[t]) in both buffers; cnt[t] particles are valid
// (a slot whose cell is < 0 is a hole).  cell is the global linear cell index
// i + nx (j + ny k); r* are offsets in [0,1) inside that cell.
struct PArr {
    int *cell;
    real *rx, *ry, *rz, *ux, *uy, *uz, *w;
    uint64_t *id;
    int *zc;      // ion charge state (ions only)
    double *tau;  // optical depth (QED species only)
};

// Occupancy of one buffer's bins: tile t holds nf[t] particles from the front
// of its region and nb[t] from the back (arrivals from other tiles).
struct Bins {
    const int *nf, *nb;
};

// Per-species state visible to kernels.
struct SpecP {
    int kind, mobile, fluid, ionizable, z_max, qed, has_z, has_tau;
    real q, m, qm;
    const long long *off;
    const int *cap;
};

__device__ inline int bin_count(const SpecP &sp, const Bins &b, int t, int &nf, int &nbv) {
    const int cap = sp.cap[t];
    nf = min(b.nf[t], cap);
    nbv = min(b.nb[t], cap - nf);
    return nf + nbv;
}
// Slot of the p-th valid particle of tile t.
__device__ inline long long bin_slot(const SpecP &sp, int t, int p, int nf, int nbv) {
    return sp.off[t] + (p < nf ? p : sp.cap[t] - nbv + (p - nf));
}

// QED Monte Carlo: device tables and the particle sinks of the events.
// Tables: We/Wb[256] spectrum totals over chi_i = 10^(-3 + 6 i / 255);
// Xe/Xb[256][128] inverse cumulative spectra at u_j = (j + 1/2) / 128 in the
// variable x of delta = x^3 / (x^3 + (1 - x)^3).
#define QED_NCHI 256
#define QED_NU 128
struct QedP {
    const double *We, *Wb, *Xe, *Xb;
    double a_s, alpha_as;         // Schwinger field and alpha * a_s (normalized units)
    PArr out1;                    // emitted photons (leptons) / pair electrons (photons)
    int *out1_n;
    int out1_cap, out1_tau;       // capacity; the sink species keeps optical depths
    PArr out2;                    // pair positrons
    int *out2_n;
    int out2_cap, out2_tau;
    int have1, have2;             // the sink species exist
    unsigned *wmax1, *wmax2;      // weight bounds of the pair species (float bits)
    double *ledger;               // photon ledger
    const uint8_t *sw;            // switch map (emission only in kinetic nodes)
    int hybrid;
    uint64_t seed;
    int step;
};

// Conversion of particles into the node fluid, done by the push (hybrid runs,
// fluid species): a particle whose nearest node after its move is fluid and
// which is not hot (|u|^2 < hot2, or hot2 <= 0) moves virtually onto that
// node; its weight and momentum go to macc (5 grid arrays, FP64: weight,
// momentum, and kinetic energy for a warm fluid), a cold fluid's lost kinetic
// energy to the ledger; k_absorb_finish merges macc into the fluid.
struct AbsorbP {
    const uint8_t *sw;   // switch map (1 kinetic)
    double *macc;        // the species' absorption accumulators
    double *ledger;      // conversion ledger
    real hot2;           // thr_hot^2 (<= 0: nothing is hot)
    int *xr;             // the species' fluid x window: absorptions widen xr[4..5]
    int on, warm;
};

// Error flags raised by kernels (bitmask in a device int).
enum { ERR_NONFINITE = 1, ERR_CFL = 2, ERR_INBOX = 4, ERR_TILE = 8 };

// Device-side rate tables for ionization (per species, per level).
// Bounds of the step probability over bins of the field: bin b holds fields
// F with log2(F) in [lf0 + b / ilr, lf0 + (b + 1) / ilr); bnd[b] bounds the
// probability over bins b - 1 .. b + 1 (so an index off by one from rounding
// still finds a bound), rounded up.  A draw at or above the bound decides "no
// event" without the rate.
#define ION_NBND 512
struct IonLevel {
    double ip_au, zres, c2, k3, expo, fc, wfc, K2;  // constants of the ADK/MPI blend
    double fskip;  // fields below this give a step probability under the smallest draw
    float lf0, ilr;
    float bnd[ION_NBND];
};
struct IonP {
    double field_au;   // atomic field units per normalized field unit
    double rate_norm;  // normalized rate per atomic rate (1 / (omega0 t_a))
    double dt_au;      // unused in kernels: kept for the host
    double omega_au;
    int z_max;
    int target;
    IonLevel lev[HK_MAX_LEVELS];
};

// ----------------------------------------------------------------- launchers ------------
// fields (k_fields.hip)
void launch_zero(void *p, size_t bytes, hipStream_t s);
void launch_fill32(void *p, size_t n, uint32_t v, hipStream_t s);   // n 32-bit words
void launch_yee_b_half(const GridP &g, real *const f[9], hipStream_t s);
void launch_yee_e_full(const GridP &g, real *const f[9], real *mur_old, hipStream_t s);
// The step's whole field update (B half, E full with the Mur walls, B half)
// in one pass from f[0..5] (E, B) and f[6..8] (J) into out[0..5]; false
// (nothing launched) where the fused pass does not apply.
bool launch_yee_step(const GridP &g, real *const f[9], real *const out[6], hipStream_t s);
void launch_antenna(const GridP &g, const hk_laser_desc &L, double t, real *jy, real *jz,
                    hipStream_t s);
void launch_divE(const GridP &g, real *const f[9], double *out, hipStream_t s);
// J += the particle current accumulated in jg (3 grid arrays); jg is left zero
void launch_jconvert(const GridP &g, jglob_t *jg, real *const f[9], hipStream_t s);

// particles (k_particles.hip): declared in hk_api.cpp where they are used

// diagnostics (k_diag.hip)
void launch_field_energy(const GridP &g, real *const f[9], double *out2, hipStream_t s);
void launch_particle_sums(const GridP &g, const SpecP &sp, PArr a, Bins b, double *out3,
                          hipStream_t s);
void launch_gauss(const GridP &g, const double *dive, const double *rho, const double *g0,
                  int skip_plane, double *out2, hipStream_t s);
void launch_fluid_sums(const GridP &g, const SpecP &sp, const real *n, const real *ux,
                       const real *uy, const real *uz, double *out3, hipStream_t s);
void launch_count_kinetic(const GridP &g, const uint8_t *sw, double *out, hipStream_t s);
void launch_sub(long long n, double *a, const double *b, hipStream_t s);

// fluid (k_fluid.hip).  A warm fluid species carries its entropy density
// S = n K (K = p / n^ga) beside n and u; S == nullptr is a cold fluid.
struct WarmP {
    real *S;
    double ga;   // adiabatic index
};
// xr (6 ints per fluid species): x window of the nodes that may hold fluid
// (open x; periodic x keeps the full range), its widening by the update, and
// the x range of this step's absorptions (k_fluid.hip explains the protocol)
void launch_fluid(const GridP &g, const SpecP &sp, const real *n, real *ux, real *uy, real *uz, WarmP w,
                  real *const f[9], real *scratch, real *nout, real *Sout, real n_floor, int *xr,
                  hipStream_t s);
void launch_fluid_window_commit(const GridP &g, int *xr, hipStream_t s);
void launch_fluid_heat(const GridP &g, const real *n, WarmP w, double *out, hipStream_t s);
void launch_fluid_rho(const GridP &g, const SpecP &sp, const real *n, double *rho,
                      hipStream_t s);

// switch and conversion (k_switch.hip)
struct SwitchP {
    real thr_a, thr_grad, thr_su, thr_ion, thr_chi, n_floor;
    int dilation, hysteresis, enable_qed, enable_ion;
    double a_s;   // QED normalized Schwinger field
};

// particle, switch and conversion launchers (k_particles.hip, k_switch.hip)
void launch_init_species_cols(const GridP &g, const hk_species_desc &d, int isp, uint64_t seed, PArr out,
                              const int *xcol, const double *wcol, int ncol, int has_z,
                              int has_tau, hipStream_t s);
void launch_count_groups(const GridP &g, PArr src, const long long *off, const int *nf,
                         const int *nb, const int *cap, int ngroups, long long maxn, int *newcnt,
                         hipStream_t s);
void launch_scatter_groups(const GridP &g, PArr src, const long long *off, const int *nf,
                           const int *nb, const int *cap, int ngroups, long long maxn, PArr dst,
                           const long long *doff, int *dfill, int has_z, int has_tau,
                           hipStream_t s);
void launch_merge_inbox(const GridP &g, const SpecP &sp, PArr inbox, const int *inbox_n,
                        long long max_n, PArr dst, const int *nf, int *nb, int *fail_n, PArr fail,
                        int *err, hipStream_t s);
void launch_migrate(const GridP &g, const SpecP &sp, PArr mig, const long long *moff,
                    const int *mcnt, const int *mcap, PArr dst, const int *nf, int *nb, int *fail_n,
                    PArr fail, int fail_cap, int *err, hipStream_t s);
void launch_push_tiles(const GridP &g, const SpecP &sp, PArr in, Bins bin_in, PArr out,
                       int *nf_out, long long mig0, const long long *moff, const int *mcap, int *mcnt,
                       const PArr *inbox_p, int *inbox_n, int inbox_cap, real *const f[9], jglob_t *jg,
                       int *err, unsigned long long *stats, const unsigned *wmax_bits, unsigned *umax2,
                       int mode, const QedP &Q, const AbsorbP &A, int2 *items, int *ctl,
                       long long capacity, int *live, hipStream_t s);
// Work plans of the per-tile particle kernels: items (tile, chunk) for grid g
// (tile_plan_items entries) and ctl[0] (the item count); ctl holds PLAN_CTL
// ints (the planner's per-workgroup bucket counts follow the count).  The
// plan lists the chunks of at least cmin particles of bins b by decreasing
// size; tile_plan_grid is the launch size that covers every item of a
// species of this capacity.
constexpr int PLAN_PARTS = 64;
constexpr int PLAN_CTL = 4 + 32 * PLAN_PARTS;
long long tile_plan_items(const GridP &g);
unsigned tile_plan_grid(const GridP &g, long long capacity, int cmin);
void launch_tile_plan(const GridP &g, const SpecP &sp, Bins b, int cmin, int2 *items, int *ctl,
                      hipStream_t s);
void launch_ionize_static(const GridP &g, const SpecP &sp, PArr a, Bins b, int *active,
                          real *const f[9], const uint8_t *sw, int hybrid, const IonP *ion,
                          PArr eout, int *eout_n, int eout_cap, uint64_t seed, int step,
                          double *ledger, int *err, unsigned *umax2, int eout_tau, hipStream_t s);
void launch_count_active(const GridP &g, const SpecP &sp, PArr a, Bins b, int zmax, int *active,
                         hipStream_t s);
void launch_rho_tiles(const GridP &g, const SpecP &sp, PArr a, Bins b, double *rho, hipStream_t s);
void launch_moments_tiles(const GridP &g, const SpecP &sp, PArr a, Bins b, int ion_only,
                          int zmax, real hot2, real *mom, const unsigned *wmax_bits, const unsigned *umax2,
                          const int *active, int2 *items, int *ctl, long long capacity, hipStream_t s);
void launch_fluid_moments_nodes(const GridP &g, real inv_ppc, const real *n, const real *ux,
                                const real *uy, const real *uz, real *mom, int first,
                                hipStream_t s);
void launch_indicators_nodes(const GridP &g, const SwitchP &P, const real *mom, real *const f[9],
                             const IonP *const *ions, int nion, uint8_t *hot, uint8_t *notcold,
                             hipStream_t s);
// training labels of the learned switch: condition bits per canonical node
// (k_label_cond), and their accumulation y |= cond over a window of steps
void launch_label_nodes(const GridP &g, const SwitchP &P, const real *mom, real *const f[9],
                        const IonP *const *ions, int nion, uint8_t *cond, hipStream_t s);
void launch_label_or(long long n, const uint8_t *cond, uint8_t *y, hipStream_t s);
void launch_flags_canonical(const GridP &g, const uint8_t *src, uint8_t *dst, hipStream_t s);
// tmp: 2 nn bytes of scratch
void launch_dilate_nodes(const GridP &g, const SwitchP &P, const uint8_t *hot, const uint8_t *notcold,
                         uint8_t *sw, uint8_t *calm, uint8_t *tmp, hipStream_t s);
// macc: 5 grid arrays (FP64): absorbed weight, momentum (3), kinetic energy
// merges macc into the fluid at the nodes of the absorptions' x range xr[4..5]
void launch_absorb_finish_nodes(const GridP &g, real mass, double *macc, real *n, real *ux,
                                real *uy, real *uz, WarmP w, double *ledger, const int *xr, hipStream_t s);
// Spawning: the kinetic nodes with fluid mass >= wmin are listed first (list
// of node indices, count in list_n, cleared by the caller), then each listed
// node becomes round(M / w0) particles (1 to 64) of species isp.
void launch_spawn_nodes(const GridP &g, const SpecP &sp, int isp, const uint8_t *sw, real *n, real *ux,
                        real *uy, real *uz, WarmP w, jglob_t *jg, real wmin, real w0, uint64_t seed,
                        int step, PArr inbox, int *inbox_n, int inbox_cap, int *deferred,
                        unsigned *wmax_bits, unsigned *umax2, double *ledger, int *list, int *list_n,
                        const int *xr, hipStream_t s);

// QED tables built on the host (hk_qed.cpp): We[256], Wb[256], Xe[256*128], Xb[256*128]
const double *hk_qed_host_tables();
