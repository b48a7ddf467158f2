/* Internal state of the FP64 oracle (test infrastructure only). */
#ifndef HK_OR_INTERNAL_H
#define HK_OR_INTERNAL_H
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    size_t n, cap;
    int32_t *ci, *cj, *ck;    /* cell holding the particle */
    double *ox, *oy, *oz;     /* offset inside that cell, [0,1) in cell units */
    double *ux, *uy, *uz;     /* momentum u = gamma v (photons: k) */
    double *w;                /* weight: number of real particles / n_c */
    double *tau;              /* remaining optical depth (QED) */
    uint64_t *id;
    int32_t *zc;              /* ion charge state */
} or_parts;

typedef struct {           /* one spawn event, appended after the particle phase */
    int species;
    int32_t ci, cj, ck;
    double ox, oy, oz, ux, uy, uz, w, tau;
    uint64_t id;
    int32_t zc;
} or_spawn;

struct or_sim {
    or_grid g;
    or_species sp[OR_MAX_SPECIES];
    int nsp;
    or_laser las;
    or_run run;
    int sx;                    /* x extent of every array: nx + 1 */
    size_t nn;                 /* sx * ny * nz */
    double *f[OR_NCOMP];
    or_parts p[OR_MAX_SPECIES];
    double *fn[OR_MAX_SPECIES], *fu[OR_MAX_SPECIES][3];  /* fluid n, u at nodes */
    double *fs[OR_MAX_SPECIES];   /* warm fluid: n K, K = p / n^gamma_ad (NULL: cold fluid) */
    uint8_t *sw, *calm;
    double *gauss0;
    int have_gauss0;
    int64_t step;
    double t;
    /* ledgers */
    double conv_loss, ion_energy, photon_ledger;
    double fallback_fraction;
    /* spawn buffer */
    or_spawn *ev;
    size_t nev, cap_ev;
    /* QED tables (filled by or_qed_init when QED is on) */
    void *qed;
    /* CNN (switch network) parameters, owned by cnn.c */
    void *cnn;
};

static inline size_t or_idx(const or_sim *s, int i, int j, int k) {
    return (size_t)i + (size_t)s->sx * ((size_t)j + (size_t)s->g.ny * (size_t)k);
}
static inline int or_wrap(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

/* Physical constants (CODATA 2018) used only for SI <-> normalized conversion. */
#define OR_C 299792458.0
#define OR_ME 9.1093837015e-31
#define OR_QE 1.602176634e-19
#define OR_HBAR 1.054571817e-34
#define OR_EPS0 8.8541878128e-12
#define OR_ALPHA 7.2973525693e-3
#define OR_EA 5.14220674763e11        /* atomic unit of field, V/m */
#define OR_TA 2.4188843265857e-17     /* atomic unit of time, s */
#define OR_HARTREE_EV 27.211386245988
#define OR_PI 3.14159265358979323846

/* philox.c */
void or_draw4(const or_sim *s, uint64_t id, uint32_t step, uint32_t tag, uint32_t draw,
              uint32_t out[4]);
/* fields.c */
void or_yee_b_half(or_sim *s);
void or_yee_e_full(or_sim *s);
void or_antenna(or_sim *s, double t);
double or_gather(const or_sim *s, int comp, const int c[3], const double o[3]);
void or_divE(const or_sim *s, double *out);
/* particles.c */
void or_parts_reserve(or_parts *p, size_t cap);
void or_parts_push_back(or_parts *p, int32_t ci, int32_t cj, int32_t ck, double ox,
                        double oy, double oz, double ux, double uy, double uz, double w,
                        double tau, uint64_t id, int32_t zc);
void or_parts_remove(or_parts *p, size_t i);
void or_init_species(or_sim *s, int sp);
void or_particle_phase(or_sim *s);
void or_deposit_move(or_sim *s, double q, double w, const int cell[3], const double X0[3],
                     const double X1[3]);
void or_rho(const or_sim *s, double *rho);
void or_spawn_flush(or_sim *s);
void or_spawn_add(or_sim *s, const or_spawn *e);
void or_carry(const or_sim *s, int c[3], double X[3]);
void or_reflect_x(const or_sim *s, int ci, double *X, double *ux);
/* fluid.c */
void or_fluid_phase(or_sim *s);
/* switch.c */
void or_switch_eval(or_sim *s);
void or_training_node(or_sim *s, double *raw9, uint8_t *cond);
void or_cnn_node_inputs(or_sim *s, const double *N, const double *U2, double *raw);
void or_absorb(or_sim *s);
void or_spawn_fluid(or_sim *s);
int or_is_hot(const or_sim *s, const double u[3]);
/* ionize.c */
double or_lambda_field_unit(double lambda_um);
double or_lambda_omega_au(double lambda_um);
void or_ionize_particle(or_sim *s, int sp, size_t i, double emag);
double or_ion_rate_norm(const or_sim *s, int sp, int level, double emag);
/* qed.c */
void or_qed_init(or_sim *s);
void or_qed_free(or_sim *s);
void or_qed_emit(or_sim *s, int sp, size_t i, const double e[3], const double b[3]);
void or_photon_phase(or_sim *s);
double or_qed_tau0(const or_sim *s, uint64_t id);
uint64_t or_child_id(uint64_t parent, uint32_t step, uint32_t k);
/* cnn.c */
void or_cnn_free(or_sim *s);
#endif
