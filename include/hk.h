/*
 * hk.h - C ABI of the MI355X hybrid fluid-kinetic laser-plasma step.
 *
 * Paper: "Machine Learning-Integrated Hybrid Fluid-Kinetic Framework for QED
 * Laser-Plasma Simulations" (arXiv 2510.11174).  The calls follow the
 * paper's statement of the problem (Methodology, pipeline paragraph): set up
 * plasma parameters and fields (hk_create), run the time loop of laser
 * excitation, ionization, particle movement, fluid changes and field updates
 * (hk_step), switch between fluid and kinetic treatment per region
 * (hk_switch_map / hk_set_switch_map / hk_set_switch_mode) and report the
 * conservation checks and energies (hk_diagnostics; validation and
 * post-processing paragraphs).
 *
 * Units: normalized laser units, c = omega0 = m_e = e = 1.  Lengths in
 * c/omega0, times in 1/omega0, densities in n_c, fields in m_e c omega0 / e.
 *
 * Grid and layout.  nx * ny * nz cells, y and z periodic, x periodic or open
 * (Mur-absorbing fields, reflecting particles).  Every grid array exchanged
 * through this ABI has the canonical shape (nz, ny, nx + 1), x fastest:
 * element (i, j, k) sits at i + (nx + 1) * (j + ny * k).  Yee staggering in
 * cell units: Ex (i+1/2, j, k), Ey (i, j+1/2, k), Ez (i, j, k+1/2),
 * Bx (i, j+1/2, k+1/2), By (i+1/2, j, k+1/2), Bz (i+1/2, j+1/2, k); J as E;
 * nodes (rho, fluid, switch map) at (i, j, k).  Unused samples (the last x
 * plane of half-staggered components, or the last plane when x is periodic)
 * read as zero.
 *
 * Precision.  The library is built twice from one source: libhk_f32.so
 * (fields and particles in FP32; FP64 optical depth and diagnostics) and
 * libhk_f64.so (everything FP64).  hk_real_size() tells which one is loaded.
 * Exchange buffers are FP64 on the host in both builds except hk_get_field /
 * hk_set_field, which move the build's own real type (4 or 8 bytes).
 *
 * Memory ownership.  Device state is owned by the library.  It is allocated
 * through hk_run_desc.alloc/free when given (for example a caching allocator
 * of the host framework), else with hipMalloc.  Work is enqueued on
 * hk_run_desc.stream (a hipStream_t, NULL = default stream).  Host pointers
 * passed to any call are borrowed for the duration of that call only.
 *
 * Errors.  Every int-returning call returns HK_OK (0) or a negative code.
 * hk_last_error() returns a message for the last failure of that context.
 * The library never aborts or prints.  After HK_EDEVICE, HK_ENUMERIC or
 * HK_EOVERFLOW the context is poisoned: later calls return HK_ESTATE until
 * hk_destroy.  A context is not thread safe; separate contexts are
 * independent.
 */
#ifndef HK_H
#define HK_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HK_MAX_SPECIES 6
#define HK_MAX_LEVELS 8

enum hk_status {
    HK_OK = 0,
    HK_EINVAL = -1,    /* bad argument or size mismatch; nothing written */
    HK_ENOMEM = -2,    /* device or host allocation failed */
    HK_EDEVICE = -3,   /* HIP runtime error (poisons the context) */
    HK_ENUMERIC = -4,  /* non-finite field or momentum, CFL breach (poisons) */
    HK_EOVERFLOW = -5, /* particle storage could not grow (poisons) */
    HK_ESTATE = -6,    /* context poisoned, or call not valid in this state */
    HK_EIO = -7,       /* file I/O */
    HK_ENOTSUP = -8    /* feature not built into this library */
};

enum hk_bc { HK_BC_PERIODIC = 0, HK_BC_OPEN = 1 };
enum hk_kind { HK_ELECTRON = 0, HK_ION = 1, HK_POSITRON = 2, HK_PHOTON = 3 };
enum hk_profile { HK_PROF_NONE = 0, HK_PROF_UNIFORM = 1, HK_PROF_RAMP = 2, HK_PROF_FOIL = 3 };
enum hk_switch_mode {
    HK_SW_ALL_PIC = 0,    /* every node kinetic, no fluid (the reference run) */
    HK_SW_THRESHOLD = 1,  /* physics-threshold switch */
    HK_SW_CNN = 2,        /* learned switch with threshold fallback */
    HK_SW_ALL_FLUID = 3,  /* every node fluid */
    HK_SW_FIXED = 4       /* map set by hk_set_switch_map, never re-evaluated */
};
enum hk_comp { HK_EX = 0, HK_EY, HK_EZ, HK_BX, HK_BY, HK_BZ, HK_JX, HK_JY, HK_JZ, HK_NCOMP };

/* Grid: cells, x boundary, cell sizes and time step (1/omega0). */
typedef struct {
    int32_t nx, ny, nz, bc_x;
    double dx, dy, dz, dt;
} hk_grid_desc;

/* One species.  Particles are created in every cell whose centre has
 * density > 0 (ppc per cell, Philox positions and Gaussian momenta).
 * kind HK_ION uses `charge` as the initial charge state; `ionizable` ions
 * ionize level by level up to z_max with potentials ip_ev[level] (eV) and put
 * the freed electrons into species `target`.  `fluid` species may be held as
 * a fluid in fluid nodes: cold (gamma_ad = 0) or warm, with adiabatic
 * pressure p = K n^gamma_ad (Methodology, plasma-model paragraph): the fluid
 * then carries S = n K, advected with its mass flux, feels the force
 * -grad p / n (taken non-relativistically), is heated by the kinetic energy
 * an absorption loses, and gives spawned particles a Gaussian spread
 * sqrt(T / m), T = p / n.  `mobile` = 0 freezes the species (no push, no
 * current).  `qed`: photon emission (leptons) or pair creation (photons). */
typedef struct {
    int32_t kind, ppc, profile, mobile;
    int32_t fluid, ionizable, z_max, target;
    int32_t qed, pad;
    double charge, mass;       /* e units, m_e units */
    double n0, x0, length;     /* peak density; ramp start/length or foil start/thickness */
    double u_th;               /* Gaussian momentum spread per component (m_e c) */
    double ip_ev[HK_MAX_LEVELS];
    double gamma_ad;           /* adiabatic index of the species' warm fluid; 0 = cold fluid */
} hk_species_desc;

/* Laser antenna: a current sheet on node plane i_antenna radiating a
 * Gaussian pulse, E = a0 exp(-((t - t_center)/duration)^2) exp(-r^2/waist^2)
 * times sin t (y) and, for circular polarization, cos t (z).  t_center <= 0
 * means 2 * duration.  lambda_um fixes the SI scale used by ionization and
 * QED rates. */
typedef struct {
    int32_t enabled, polarization;   /* 0 linear (E along y), 1 circular */
    int32_t i_antenna, pad;
    double a0, waist, duration, t_center, lambda_um;
} hk_laser_desc;

typedef void *(*hk_alloc_fn)(size_t bytes, void *ctx);
typedef void (*hk_free_fn)(void *ptr, void *ctx);

/* Run control.  Thresholds of the switch criterion (kinetic when any is
 * reached): |E| >= thr_a; density gradient beyond its shot noise >= thr_grad;
 * momentum spread >= thr_sigma_u; ionization probability per step >= thr_ion;
 * estimated quantum parameter >= thr_chi.  `dilation` widens the kinetic
 * region by that many nodes; a kinetic node returns to fluid after
 * `hysteresis` calm evaluations.  Fluid below n_floor has no velocity.
 * Fluid mass M >= spawn_frac * w0 on a kinetic node, w0 = n0 dV / ppc the
 * species' reference weight, becomes round(M / w0) particles (1 to 64).
 * A particle with |u| >= thr_hot (thr_hot > 0) is hot: a kinetic population
 * wherever it is, never absorbed into a fluid node and left out of the
 * switch moments (thr_hot <= 0: no particle is hot). */
typedef struct {
    uint64_t seed;
    int32_t switch_mode, switch_every;
    int32_t dilation, hysteresis;
    int32_t enable_ionization, enable_qed;
    double thr_a, thr_grad, thr_sigma_u, thr_ion, thr_chi;
    double n_floor;
    double spawn_frac;
    double thr_hot;
    void *stream;          /* hipStream_t or NULL */
    hk_alloc_fn alloc;     /* optional device allocator */
    hk_free_fn free;
    void *alloc_ctx;
} hk_run_desc;

/* QED (run.enable_qed).  Species with `qed` set carry an optical depth.
 * Electrons and positrons with `qed` emit photons (quantum-synchrotron
 * spectrum, Airy form) into the first HK_PHOTON species; photons convert into
 * pairs (Breit-Wheeler) in the first HK_ELECTRON and HK_POSITRON species and
 * otherwise fly at c, leaving through open x walls.  Soft photons (|k| <= 2),
 * escaped photons and the pairs' rest energy go to the photon ledger
 * (hk_diag.photon_energy).  Paper: abstract and Methodology, plasma-model
 * paragraph (QED effects with Airy-function approximations). */

/* FP64 diagnostics (energies in m_e c^2 n_c (c/omega0)^3). */
typedef struct {
    double t;
    int64_t step;
    double u_e, u_b;                       /* field energies */
    double kin[HK_MAX_SPECIES];            /* particle kinetic energy per species */
    double fluid_kin[HK_MAX_SPECIES];      /* fluid kinetic energy per species */
    double count[HK_MAX_SPECIES];          /* macro-particles per species */
    double fluid_mass[HK_MAX_SPECIES];     /* sum n dV per fluid species */
    double charge_total;                   /* particles + fluids */
    double gauss_max, gauss_l2;            /* change of div E - rho since step 0 */
    double conv_loss;                      /* kinetic energy lost by absorption */
    double ion_energy;                     /* ionization potential energy spent */
    double photon_energy;                  /* photon ledger: radiated energy not held by photon
                                              particles, escaped photons, pair rest energy */
    double kinetic_fraction;               /* kinetic nodes / all nodes */
    double fallback_fraction;              /* CNN nodes that fell back to threshold */
    double fluid_th[HK_MAX_SPECIES];       /* warm fluid thermal energy, sum p dV / (gamma_ad - 1) */
} hk_diag;

/* Host-side particle arrays, FP64 regardless of the build: x[3n] absolute
 * positions, u[3n] momenta, w[n] weights, id[n], z[n] charge state (ions),
 * tau[n] optical depth (QED species).  Any pointer may be NULL on get. */
typedef struct {
    size_t n;
    double *x, *u, *w;
    uint64_t *id;
    int32_t *z;
    double *tau;
} hk_particles;

typedef struct hk_sim hk_sim;

/* Build the context: validates the descriptors (HK_EINVAL; among others the
 * node count (nx+1)*ny*nz must stay below 2^31), allocates device state,
 * initialises species on the device and zeroes the fields. */
int hk_create(const hk_grid_desc *grid, const hk_species_desc *species, int nspecies,
              const hk_laser_desc *laser, const hk_run_desc *run, hk_sim **out);
void hk_destroy(hk_sim *sim);

/* Advance nsteps time steps on the run stream; returns after they complete.
 * Each step waits on the host once, for a device status word read after the
 * step's field update has been queued: an error ends the call with its code
 * (HK_ENUMERIC, HK_EOVERFLOW, HK_EDEVICE) at that step; bins that overflowed
 * are re-binned before the next step's push. */
int hk_step(hk_sim *sim, int nsteps);

/* Switch map: n must be (nx+1)*ny*nz bytes; 1 kinetic, 0 fluid. */
int hk_switch_map(hk_sim *sim, uint8_t *out, size_t n);
int hk_set_switch_map(hk_sim *sim, const uint8_t *in, size_t n);  /* implies FIXED */
int hk_set_switch_mode(hk_sim *sim, int mode);

int hk_diagnostics(hk_sim *sim, hk_diag *out);

/* Field component `comp` (hk_comp) in the canonical layout; bytes must be
 * (nx+1)*ny*nz*hk_real_size(). */
int hk_get_field(hk_sim *sim, int comp, void *host_out, size_t bytes);
int hk_set_field(hk_sim *sim, int comp, const void *host_in, size_t bytes);

/* Node charge density and discrete div E (FP64, canonical layout, n values). */
int hk_get_rho(hk_sim *sim, double *host_out, size_t n);
int hk_get_divE(hk_sim *sim, double *host_out, size_t n);

int hk_particle_count(hk_sim *sim, int species, size_t *n);
/* out->n must equal hk_particle_count; particles come in storage order. */
int hk_get_particles(hk_sim *sim, int species, const hk_particles *out);
/* Replaces the species' particles (positions must lie inside the box). */
int hk_set_particles(hk_sim *sim, int species, const hk_particles *in);

/* Cold fluid of a fluid species: n[(nx+1)*ny*nz], u[3*(nx+1)*ny*nz]. */
int hk_get_fluid(hk_sim *sim, int species, double *n, double *u, size_t nodes);
int hk_set_fluid(hk_sim *sim, int species, const double *n, const double *u, size_t nodes);
/* Warm fluid pressure per node (host FP64, canonical layout, same size as
 * the fluid density); HK_EINVAL for a cold or missing fluid.  Set the density
 * first: the pressure is stored as S = p n^(1 - gamma_ad). */
int hk_get_fluid_p(hk_sim *sim, int species, double *p, size_t nodes);
int hk_set_fluid_p(hk_sim *sim, int species, const double *p, size_t nodes);

/* Timers since the last hk_enable_timing(sim, 1), collected with HIP events
 * on the run stream (they add synchronisation, so timed runs are slower):
 *   0 switch evaluation, 1 particle phase (push, migrate, ionization),
 *   2 fluid, 3 conversion, 4 fields, 5 inbox merge and re-binning (ms);
 *   6 the push kernel alone (ms), 7 re-binnings since creation,
 *   8 push launches, 9 particles pushed, 10 tiles pushed (counts).
 * hk_timers copies min(n, HK_NTIMERS) values. */
#define HK_NTIMERS 12
int hk_enable_timing(hk_sim *sim, int on);
int hk_timers(hk_sim *sim, double *ms, int n);

/* Checkpoint and resume.  hk_save writes the whole state a step depends on:
 * fields (E, B, J), the Mur boundary planes, the switch map and its calm
 * counters, the energy ledgers, the species weight bounds, the Gauss
 * baseline, the CNN evaluation count, every species' particles in the
 * library's own representation (cell, cell-relative offsets, u, w, id, z,
 * tau) and fluid arrays, the step counter and the time.  hk_load restores it
 * into a context created with the same descriptors (grid, species kinds,
 * precision: HK_EINVAL otherwise, nothing changed); particles are re-binned,
 * so a resumed run draws the same Philox numbers (counters are id, step and
 * tag) and takes the same decisions as an uninterrupted one.  An attached
 * CNN is not part of the file: save it with hk_cnn_get_params.  The path is
 * borrowed for the call; file errors return HK_EIO.  A file whose header
 * does not match (magic, version, precision, grid, species kinds) changes
 * nothing; a failure after the header (a short or corrupt body) leaves the
 * state partly restored and poisons the context (HK_ESTATE from then on).
 * Paper: Methodology (keeping code, parameters and outputs together for
 * reproducible runs). */
int hk_save(hk_sim *sim, const char *path);
int hk_load(hk_sim *sim, const char *path);

/* The QED tables the library built (host FP64, independent of any context):
 * We[256] and Wb[256] are the emission and pair spectra integrated over the
 * energy fraction at chi_i = 10^(-3 + 6 i / 255); Xe and Xb [256 * 128], row
 * i, hold the inverse cumulative spectra at u_j = (j + 1/2) / 128 in the
 * variable x of delta = x^3 / (x^3 + (1 - x)^3).  The caller owns the arrays.
 * Paper: Methodology, plasma-model paragraph (Airy-function QED rates). */
int hk_qed_tables(double *We, double *Wb, double *Xe, double *Xb);

/* ------------------------------------------------------------------------
 * The learned switch (Methodology: a neural network selects fluid or kinetic
 * treatment per region, Monte Carlo dropout measures its uncertainty, the
 * physics thresholds are the fallback; it is trained on the simulation's own
 * data with an energy penalty).
 *
 * Network: 8 input channels per node (E, B at the node, electron density,
 * rms momentum), normalized with frozen statistics (hk_cnn_set_norm); four
 * valid 3^3 convolutions of 32 channels with exact GELU; a 1x1x1 head to one
 * logit.  BF16 inputs, weights and activations, FP32 accumulation (matrix
 * cores).  90017 parameters (hk_cnn_nparams), FP32 masters, laid out as
 * W1[27][8][32], b1[32], then W[27][32][32], b[32] for layers 2..4, then the
 * head w[32], b (tap = kx + 3 ky + 9 kz).
 *
 * Crops: x[B][D][H][W][8] FP32 normalized inputs, channels last (device
 * pointers); outputs cover the valid (D-8)(H-8)(W-8) nodes, x fastest.
 * Loss per output node: BCE(p, y) + lambda_e (1 - p) e, averaged; y the
 * kinetic label (0/1), e the energy a cold-fluid conversion would destroy.
 * Training dropout (p = 26/256 on the head input) uses Philox (seed, output
 * node index, AdamW step); the switch uses 16 samples per node with counter
 * (node, evaluation number), mean p > 0.5 = kinetic unless the samples' std
 * exceeds 0.2 (then the threshold decision stays). */
typedef struct hk_cnn hk_cnn;
typedef struct {
    uint64_t seed;          /* dropout streams */
    void *stream;           /* hipStream_t or NULL */
    hk_alloc_fn alloc;      /* optional device allocator */
    hk_free_fn free;
    void *alloc_ctx;
} hk_cnn_desc;
typedef struct {
    double lr, beta1, beta2, eps, weight_decay;   /* AdamW */
    double lambda_e;                               /* energy penalty weight */
    int32_t dropout, pad;                          /* train with head-input dropout */
} hk_cnn_train_desc;

int hk_cnn_nparams(void);
int hk_cnn_create(const hk_cnn_desc *desc, hk_cnn **out);
void hk_cnn_destroy(hk_cnn *cnn);
/* host FP32 parameters in and out (n = hk_cnn_nparams()); setting resets AdamW */
int hk_cnn_set_params(hk_cnn *cnn, const float *params, size_t n);
int hk_cnn_get_params(hk_cnn *cnn, float *params, size_t n);
/* input statistics: 8 means and 8 standard deviations (host) */
int hk_cnn_set_norm(hk_cnn *cnn, const float *mean, const float *stdv);
/* logits (device FP32, B (D-8)(H-8)(W-8)) of crops x (device), no dropout */
int hk_cnn_forward(hk_cnn *cnn, const float *x, int B, int D, int H, int W, float *logit);
/* loss and gradient (host FP32, n = hk_cnn_nparams(), may be NULL); y and e
 * device FP32 per output node; mask_step < 0: no dropout */
int hk_cnn_loss_grad(hk_cnn *cnn, const float *x, const float *y, const float *e, int B, int D, int H,
                     int W, float lambda_e, int mask_step, float *grad_host, double *loss);
/* one AdamW step on a batch (dropout masks keyed by the step count) */
int hk_cnn_train_step(hk_cnn *cnn, const float *x, const float *y, const float *e, int B, int D, int H,
                      int W, const hk_cnn_train_desc *train, double *loss);
const char *hk_cnn_last_error(const hk_cnn *cnn);
/* Allocation-free variant of hk_cnn_forward, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, layouts and results as
 * hk_cnn_forward (the same kernels); the BF16 input copy and the activations
 * live in one static device array of HK_CNN_NOALLOC_SCRATCH_BYTES per GPU,
 * held until the process ends, so the call makes no hipMalloc, hipFree or
 * other allocation.  B * D * H * W may not exceed HK_CNN_NOALLOC_MAX_VOXELS
 * (HK_EINVAL, message in hk_cnn_last_error).  The work is only enqueued on
 * the network's stream: the logits are ready once the stream gets there.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (any network, any stream) race and must be serialized by the caller.  The
 * first call on a device looks the array up there (HK_EDEVICE on failure). */
#define HK_CNN_NOALLOC_MAX_VOXELS (1 << 18)
#define HK_CNN_NOALLOC_SCRATCH_BYTES ((size_t)HK_CNN_NOALLOC_MAX_VOXELS * (8 * 2 + 2 * 32 * 2))
int hk_cnn_forward_noalloc(hk_cnn *cnn, const float *x, int B, int D, int H, int W, float *logit);
/* Training data from a simulation, per node of the grid [nz][ny][NX] (NX = nx
 * for periodic x, nx + 1 for open x), x fastest, all host arrays (NULL skips
 * one): raw[8 n] the network's 8 inputs before normalization; ehat[n] the
 * thermal energy (m_e c^2 n_c (c/omega0)^3, small-u limit) a cold-fluid
 * conversion would destroy; hot[n] the threshold criterion's undilated flags
 * now.  The switch map is left unchanged.  n must equal NX ny nz. */
int hk_node_inputs(hk_sim *sim, double *raw, double *ehat, uint8_t *hot, size_t n);
/* States for the next-state surrogate, per node of the grid [nz][ny][NX] as
 * above: out (device FP32, 10 n values, channels last) = Ex, Ey, Ez, Bx, By,
 * Bz averaged to the node from their Yee positions (neighbour means; open x
 * repeats the wall cell), Jx, Jy, Jz averaged the same way as E, and the
 * charge density rho at the node (particles and fluid); not normalized.  The
 * simulation is left unchanged.  n must equal NX ny nz. */
int hk_node_state(hk_sim *sim, float *out, size_t n);
/* the network the simulation's HK_SW_CNN mode uses (borrowed; NULL detaches;
 * without one the mode decides by the thresholds alone) */
int hk_set_cnn(hk_sim *sim, hk_cnn *cnn);

/* Training set of the learned switch, in device memory (Methodology,
 * pipeline paragraph: the switch network learns from data the simulation
 * itself generates, with inputs normalized per channel and an energy
 * penalty).  desc gives the stream and the optional allocator (its seed is
 * unused).  Snapshots of D x H x W nodes (z, y, x; x fastest) hold per node
 * the 8 network inputs before normalization, the conversion energy e (as
 * for hk_node_inputs) and the 0/1 kinetic label. */
typedef struct hk_dataset hk_dataset;
int hk_dataset_create(const hk_cnn_desc *desc, hk_dataset **out);
void hk_dataset_destroy(hk_dataset *ds);
int hk_dataset_size(const hk_dataset *ds);   /* snapshots held */
/* snapshot k to the host: dims[3] = D, H, W; raw[8 n], ehat[n], y[n] the
 * label, thr[n] the threshold criterion's undilated flags at the snapshot's
 * step (the method without the network; each may be NULL; n must be D H W
 * when any is given) */
int hk_dataset_get(hk_dataset *ds, int k, int *dims, float *raw, float *ehat, uint8_t *y, uint8_t *thr,
                   size_t n);
/* per-channel mean and standard deviation of the 8 inputs over every node of
 * every snapshot (FP64 sums on the device; a constant channel gets std 1);
 * the caller hands them to hk_cnn_set_norm */
int hk_dataset_stats(hk_dataset *ds, float *mean, float *stdv);
/* Append snapshots of an all-PIC run (HK_EINVAL in any other mode, or for a
 * grid under 16 nodes in a direction): the simulation advances steps +
 * window steps from where it is; at relative steps 0, every, 2 every, ...
 * <= steps the node inputs are stored, and the label of a node is 1 when,
 * at any of that step and the window steps after it, (a) a cold-fluid
 * conversion would destroy more than 1e-3 of the node's kinetic energy while
 * its momentum spread is at or above thr_sigma_u, or (b) an ionization is
 * possible there (per-step probability >= thr_ion with ionizable ions left),
 * or (c) a QED emission is possible (chi >= thr_chi).  Everything runs on
 * the simulation's stream, drained before return; a failed step poisons the
 * simulation as hk_step does.  Snapshots appended before a failure stay. */
int hk_dump_training(hk_sim *sim, hk_dataset *ds, int steps, int every, int window);
/* iters AdamW steps of the network on batches of B crops sampled on the
 * device: snapshot and origin from Philox (seed, crop index, the network's
 * AdamW step), 24^3 input nodes normalized with the network's statistics
 * (halo: wrap in y, z and periodic x, wall node repeated in open x), labels
 * and energy weights e / (crop kinetic energy) x 4096 on the 16^3 output
 * nodes.  losses[iters] (host, may be NULL) receives each batch loss. */
int hk_train(hk_cnn *cnn, hk_dataset *ds, int iters, int B, const hk_cnn_train_desc *train, uint64_t seed,
             double *losses);
/* logits (device FP32, D H W) of snapshot k, no dropout */
int hk_dataset_predict(hk_cnn *cnn, hk_dataset *ds, int k, float *logit);
const char *hk_dataset_last_error(const hk_dataset *ds);

/* ------------------------------------------------------------------------
 * Next-state surrogate (Results, Table 2 and the paragraph before it: a
 * residual 3D CNN, the StatePredictor, trained with a Huber loss and a
 * physics penalty on the field energy).
 *
 * Network: 10 channels per node in and out (Ex, Ey, Ez, Bx, By, Bz, Jx, Jy,
 * Jz, rho, each normalized (x - mean) / std with frozen statistics); six
 * "same" 3^3 convolutions with zero padding, widths 10->13->32->64->128->32->
 * 10; ReLU after all but the last; the first three add their input to their
 * first output channels (residual copy, no weights); dropout (p = 26/256,
 * kept channels scaled by 256/230) on the 32-channel output of the second,
 * keyed by Philox (seed, voxel index in the batch, mask step), tag 25.  BF16
 * inputs, weights and activations (rounded to nearest even; the dropped-out
 * activation is rounded once, after scaling), FP32 accumulation on the matrix
 * cores, FP32 output.  410733 parameters (hk_sp_nparams), FP32 masters,
 * per layer W[27][cin][cout] then b[cout] (tap = kx + 3 ky + 9 kz reads the
 * offset (kx - 1, ky - 1, kz - 1)).
 *
 * Patches: x[B][D][H][W][10] FP32 normalized states, channels last, x
 * fastest (device pointers); the output has the same shape.  Loss: the mean
 * over voxels and channels of Huber_delta(pred - y) plus lambda_e times the
 * mean over patches of ((U_pred - U_y) / U_y)^2, U = sum over the patch of
 * sum_{c < 6} (x_c std_c + mean_c)^2 (hk_sp_set_norm; patches with U_y = 0
 * add no energy term).  Training needs W % 8 == 0; errors: HK_EINVAL for a
 * bad shape or argument, HK_ENOMEM when the workspace cannot grow,
 * HK_EDEVICE for a failed HIP call (hk_sp_last_error has the text).  The
 * workspace (about 3 KB per voxel when training) is kept between calls and
 * freed by hk_sp_destroy; calls on one network are serialized on its stream. */
typedef struct hk_sp hk_sp;
typedef struct {
    double lr, beta1, beta2, eps, weight_decay;   /* AdamW */
    double delta;                                  /* Huber threshold */
    double lambda_e;                               /* energy penalty weight */
    int32_t dropout, pad;                          /* train with dropout (mask step = AdamW step) */
} hk_sp_train_desc;

int hk_sp_nparams(void);
/* desc as for hk_cnn_create: dropout seed, stream, optional allocator */
int hk_sp_create(const hk_cnn_desc *desc, hk_sp **out);
void hk_sp_destroy(hk_sp *sp);
/* host FP32 parameters in and out (n = hk_sp_nparams()); setting resets AdamW */
int hk_sp_set_params(hk_sp *sp, const float *params, size_t n);
int hk_sp_get_params(hk_sp *sp, float *params, size_t n);
/* 10 means and 10 standard deviations (host) of the raw channels: only the
 * energy term uses them (the inputs arrive normalized) */
int hk_sp_set_norm(hk_sp *sp, const float *mean, const float *stdv);
/* out (device FP32, same shape as x) = the predicted normalized next states;
 * mask_step >= 0 applies that step's dropout masks (Monte Carlo samples),
 * < 0 none */
int hk_sp_forward(hk_sp *sp, const float *x, int B, int D, int H, int W, int mask_step, float *out);
/* loss (host) and gradient (host FP32, n = hk_sp_nparams(), may be NULL) for
 * targets y (device, same shape as x) */
int hk_sp_loss_grad(hk_sp *sp, const float *x, const float *y, int B, int D, int H, int W, double delta,
                    double lambda_e, int mask_step, float *grad_host, double *loss);
/* one AdamW step on a batch */
int hk_sp_train_step(hk_sp *sp, const float *x, const float *y, int B, int D, int H, int W,
                     const hk_sp_train_desc *train, double *loss);
const char *hk_sp_last_error(const hk_sp *sp);

/* ------------------------------------------------------------------------
 * The paper's SwitchNet (Results, Table 1 and the paragraph after it): a
 * per-node fluid/kinetic classifier.  10 features per node (the node state
 * of hk_node_state, normalized with frozen statistics); Linear 10->128 +
 * ReLU + residual copy of the input, Linear 128->256 + ReLU + residual copy
 * with dropout (p = 51/256, kept channels scaled by 256/205, Philox tag 26
 * keyed by (seed, node index in the call, mask step), sample s using draws
 * 16 s .. 16 s + 15); 4-head attention over the node's single token (the
 * softmax over one key is 1, so each head passes its value projection: the
 * layer computes v = Wv h + bv then Wo v + bo, and the query and key
 * projections get no gradient); Linear 256->1 to the logit.  BF16 weights
 * and activations, FP32 accumulation on the matrix cores, FP32 logits.
 * 297857 parameters (hk_swn_nparams), FP32 masters: W1[10][128], b1,
 * W2[128][256], b2, Wq, bq, Wk, bk, Wv, bv, Wo, bo (W[256][256] indexed
 * [in][out]), wh[256], bh.  Loss per node: BCE(p, y) + lambda_e (1 - p) e,
 * averaged (y the kinetic label, e the energy a cold-fluid conversion would
 * destroy).  x[n][10], y[n], e[n] and logits are device FP32; training needs
 * n % 8 == 0; n <= 2^26.  Errors as for hk_sp_*. */
typedef struct hk_swn hk_swn;
int hk_swn_nparams(void);
int hk_swn_create(const hk_cnn_desc *desc, hk_swn **out);
void hk_swn_destroy(hk_swn *swn);
/* host FP32 parameters in and out (n = hk_swn_nparams()); setting resets AdamW */
int hk_swn_set_params(hk_swn *swn, const float *params, size_t n);
int hk_swn_get_params(hk_swn *swn, float *params, size_t n);
/* logits of n nodes; mask_step >= 0 applies dropout sample `sample` (0..15)
 * of that step (Monte Carlo samples), < 0 none */
int hk_swn_forward(hk_swn *swn, const float *x, int n, int mask_step, int sample, float *logit);
/* loss (host) and gradient (host FP32, may be NULL) */
int hk_swn_loss_grad(hk_swn *swn, const float *x, const float *y, const float *e, int n, double lambda_e,
                     int mask_step, float *grad_host, double *loss);
/* one AdamW step (train->lambda_e, dropout keyed by the step count) */
int hk_swn_train_step(hk_swn *swn, const float *x, const float *y, const float *e, int n,
                      const hk_cnn_train_desc *train, double *loss);
const char *hk_swn_last_error(const hk_swn *swn);

int hk_real_size(void);
const char *hk_strerror(int code);
const char *hk_last_error(const hk_sim *sim);

#ifdef __cplusplus
}
#endif
#endif
