/*
 * Plain FP64 CPU oracle of the hybrid fluid-kinetic time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP library; every formula is
 * written out here from the paper and the literature it names.
 *
 * Paper: "Machine Learning-Integrated Hybrid Fluid-Kinetic Framework for QED
 * Laser-Plasma Simulations" (arXiv 2510.11174).  The step follows the stage
 * order given in the Methodology section (laser excitation, ionization,
 * particle movement, fluid changes, field modifications).
 *
 * Units: normalized laser units, c = omega0 = m_e = e = 1; lengths in c/omega0,
 * times in 1/omega0, densities in n_c, fields in m_e c omega0 / e.
 *
 * Every function is plain loops in double precision.  Nothing is blocked,
 * fused or reordered beyond what the definitions state.
 */
#ifndef HK_ORACLE_H
#define HK_ORACLE_H
#include <stdint.h>
#include <stddef.h>

#define OR_MAX_SPECIES 6
#define OR_MAX_LEVELS 8

enum { OR_BC_PERIODIC = 0, OR_BC_OPEN = 1 };
enum { OR_ELECTRON = 0, OR_ION = 1, OR_POSITRON = 2, OR_PHOTON = 3 };
enum { OR_PROF_NONE = 0, OR_PROF_UNIFORM = 1, OR_PROF_RAMP = 2, OR_PROF_FOIL = 3 };
enum { OR_SW_ALL_PIC = 0, OR_SW_THRESHOLD = 1, OR_SW_CNN = 2, OR_SW_ALL_FLUID = 3,
       OR_SW_FIXED = 4 };

/* Field component ids (same numbering as the library's canonical dump). */
enum { OR_EX = 0, OR_EY, OR_EZ, OR_BX, OR_BY, OR_BZ, OR_JX, OR_JY, OR_JZ, OR_NCOMP };

typedef struct {
    int32_t nx, ny, nz, bc_x;
    double dx, dy, dz, dt;
} or_grid;

typedef struct {
    int32_t kind, ppc, profile, mobile;
    int32_t fluid;       /* may be represented by the cold fluid in fluid nodes */
    int32_t ionizable;   /* field ionization of this (ion) species */
    int32_t z_max;       /* fully stripped charge state */
    int32_t target;      /* species index that receives ionization electrons */
    int32_t qed;         /* photon emission (leptons) / pair creation (photons) */
    int32_t pad;
    double charge, mass;    /* initial charge state (e units), mass (m_e units) */
    double n0, x0, length;  /* peak density; ramp start/length or foil start/thickness */
    double u_th;            /* Gaussian momentum spread per component */
    double ip_ev[OR_MAX_LEVELS];
    double gamma_ad;        /* adiabatic index of the warm fluid; 0 = cold fluid */
} or_species;

typedef struct {
    int32_t enabled, polarization;   /* 0 linear (E along y), 1 circular */
    int32_t i_antenna, pad;
    double a0, waist, duration, t_center, lambda_um;
} or_laser;

typedef struct {
    uint64_t seed;
    int32_t switch_mode, switch_every;
    int32_t dilation, hysteresis;
    int32_t enable_ionization, enable_qed;
    double thr_a, thr_grad, thr_sigma_u, thr_ion, thr_chi;
    double n_floor;      /* fluid density floor (n_c) */
    double spawn_frac;   /* spawn fluid mass >= spawn_frac * n0 dV / ppc */
    double thr_hot;      /* |u| >= thr_hot: never absorbed, not in the switch moments (<= 0: none) */
} or_run;

typedef struct {
    double t;
    int64_t step;
    double u_e, u_b;                       /* field energies */
    double kin[OR_MAX_SPECIES];            /* particle kinetic energy per species */
    double fluid_kin[OR_MAX_SPECIES];      /* fluid kinetic energy per species */
    double count[OR_MAX_SPECIES];          /* particles per species */
    double fluid_mass[OR_MAX_SPECIES];     /* sum n dV per fluid species */
    double charge_total;                   /* sum of particle and fluid charge */
    double gauss_max, gauss_l2;            /* max / rms of (div E - rho) - initial */
    double conv_loss;                      /* kinetic energy lost at absorption */
    double ion_energy;                     /* ionization potential energy spent */
    double photon_energy;                  /* photon ledger: radiated energy not held by photon
                                              particles, escaped photons, pair rest energy */
    double kinetic_fraction;               /* fraction of kinetic nodes */
    double fallback_fraction;
    double fluid_th[OR_MAX_SPECIES];       /* warm fluid thermal energy, sum p dV / (gamma_ad - 1) */
} or_diag;

typedef struct or_sim or_sim;

/* Lifecycle */
or_sim *or_create(const or_grid *g, const or_species *sp, int nspecies,
                  const or_laser *l, const or_run *r);
void or_destroy(or_sim *s);
int or_step(or_sim *s, int nsteps);

/* Field access in the canonical layout: (nz, ny, nx+1), x fastest. */
size_t or_field_size(const or_sim *s);
int or_get_field(const or_sim *s, int comp, double *out);
int or_set_field(or_sim *s, int comp, const double *in);

/* Particles: positions in c/omega0, momenta u = gamma v. */
size_t or_particle_count(const or_sim *s, int species);
int or_get_particles(const or_sim *s, int species, double *x, double *u, double *w,
                     uint64_t *id, int32_t *z, double *tau);
int or_set_particles(or_sim *s, int species, size_t n, const double *x, const double *u,
                     const double *w, const uint64_t *id, const int32_t *z,
                     const double *tau);

/* Fluid: node density n and momentum u per node, canonical layout. */
int or_get_fluid(const or_sim *s, int species, double *n, double *u);
int or_set_fluid(or_sim *s, int species, const double *n, const double *u);
/* Warm fluid pressure per node (canonical layout); set after the density. */
int or_get_fluid_p(const or_sim *s, int species, double *p);
int or_set_fluid_p(or_sim *s, int species, const double *p);

/* Switch map, one byte per node (canonical layout): 1 kinetic, 0 fluid. */
int or_get_switch(const or_sim *s, uint8_t *out);
int or_set_switch(or_sim *s, const uint8_t *in);
int or_set_switch_mode(or_sim *s, int mode);
/* Training data of the learned switch at the current step, canonical node
 * grid [nz][ny][NX] (NX = nx periodic, nx + 1 open): raw9 (may be NULL) the 8
 * network inputs and the conversion energy per node, cond the label
 * condition bits (1 thermal, 2 ionization possible, 4 QED possible). */
void or_training_node(or_sim *s, double *raw9, uint8_t *cond);
/* The next step's Monte Carlo decisions, for comparisons of events decided
 * in another precision: per particle of species isp (the oracle's order),
 * ionization P and draw r per level [n][z_max] (event when r < P), and QED
 * optical depth tau and its decrement dtau (event when tau - dtau <= 0). */
void or_ion_probe(or_sim *s, int isp, double *P, double *r);
void or_qed_probe(or_sim *s, int isp, double *tau, double *dtau);

int or_diagnostics(or_sim *s, or_diag *d);
/* Charge density (nodes) and div E, canonical layout. */
int or_get_rho(const or_sim *s, double *rho);
int or_get_divE(const or_sim *s, double *dive);

/* Building blocks exposed for the closed-form pins. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_uniform(uint32_t x);
void or_boris(double qm, double dt, const double e[3], const double b[3], double u[3]);
double or_adk_rate(double field_au, double ip_au, double zres);
double or_ionization_rate(double field_au, double ip_au, double zres, double omega_au);
void or_esirkepov(const double x0[3], const double x1[3], double qw_dv, double dt,
                  const double dx[3], double jx[27], double jy[27], double jz[27],
                  int base[3]);
/* QED building blocks: Airy functions (z > 0), spectra, totals over delta
 * (kind 0 emission, 1 pairs, 2 emitted energy fraction), the tables
 * (256 chi values; 256 x 128 inverse spectra in the x variable), chi. */
void or_airy(double z, double *ai, double *aip, double *iai);
double or_qed_emission_spectrum(double chi, double delta);
double or_qed_pair_spectrum(double chi, double delta);
double or_qed_total(int kind, double chi);
void or_qed_build_tables(double *We, double *Wb, double *Xe, double *Xb);
double or_qed_chi(double a_s, const double e[3], const double b[3], const double u[3], int photon);
double or_schwinger_field(double lambda_um);
/* CNN switch: parameter count, BF16 rounding, forward over crops, loss and
 * gradient, AdamW, dropout masks, node inputs; or_set_cnn installs the
 * network and its input statistics for switch mode CNN. */
int or_cnn_nparam(void);
void or_cnn_set_rounding(int on);
double or_bf16(double x);
void or_cnn_forward(const double *par, const double *x, int B, int D, int H, int W,
                    const double *mask, double *logit);
double or_cnn_loss_grad(const double *par, const double *x, const double *y, const double *e,
                        int B, int D, int H, int W, double lambda, const double *mask, double *grad);
void or_cnn_adamw(double *par, const double *grad, double *m, double *v, int t, double lr,
                  double b1, double b2, double eps, double wd, int n);
void or_cnn_mask(uint64_t seed, uint64_t id, uint32_t step, int sample, double out[32]);
int or_set_cnn(or_sim *s, const double *par, const double mean[8], const double stdv[8]);

/* Next-state surrogate (sp.c): parameter count, forward over B patches of
 * D x H x W x 10 normalized inputs (same-size output), loss (Huber + energy
 * term) and gradient, dropout factors. */
int or_sp_nparam(void);
void or_sp_forward(const double *par, const double *x, int B, int D, int H, int W, const double *mask,
                   double *out);
double or_sp_loss_grad(const double *par, const double *x, const double *y, int B, int D, int H, int W,
                       const double mean[10], const double stdv[10], double delta, double lambda,
                       const double *mask, double *grad);
void or_sp_mask(uint64_t seed, uint64_t id, uint32_t step, int sample, double out[32]);

/* SwitchNet (swn.c): parameter count, logits of n nodes' 10 features, loss
 * (BCE + lambda (1 - p) e) and gradient, dropout factors of its 256-wide
 * block. */
int or_swn_nparam(void);
void or_swn_forward(const double *par, const double *x, int n, const double *mask, double *logit);
double or_swn_loss_grad(const double *par, const double *x, const double *y, const double *e, int n,
                        double lambda, const double *mask, double *grad);
void or_swn_mask(uint64_t seed, uint64_t id, uint32_t step, int sample, double out[256]);

#endif
