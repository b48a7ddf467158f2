/*
 * Oracle driver: set-up, the time step in the paper's stage order, and the
 * FP64 diagnostics.
 *
 * Paper: Methodology, pipeline paragraph (set-up of plasma parameters and
 * fields, then a time loop of laser excitation, ionization, particle
 * movement, fluid changes and field modifications) and post-processing /
 * validation paragraphs (total energy from electromagnetic, kinetic and
 * thermal parts; charge and energy conservation checks).
 *
 * Step n (E^n, B^n at integer time; particle x^n, u^{n-1/2}; fluid n^n, u^{n-1/2}):
 *   1. switch evaluation every `switch_every` steps (threshold / CNN modes);
 *   2. J = 0; laser antenna current at t^{n+1/2};
 *   3. particles: gather, ionization, photon emission, Boris, move, deposit;
 *   4. photons: pair creation, ballistic push; the particles born in 3 and 4
 *      then join their species (they move from the next step on);
 *   5. fluid update (adds its face current to J);
 *   6. conversion: particles of fluid-capable species whose nearest node is
 *      fluid (and which are not hot) join the node fluid, then fluid mass on
 *      kinetic nodes becomes particles (both add their moves' current to J);
 *   7. B^{n+1/2} = B^n - dt/2 curl E^n; E^{n+1} = E^n + dt (curl B - J)
 *      with Mur walls; B^{n+1} = B^{n+1/2} - dt/2 curl E^{n+1}.
 */
#include "or_internal.h"

or_sim *or_create(const or_grid *g, const or_species *sp, int nspecies, const or_laser *l,
                  const or_run *r) {
    if (nspecies < 0 || nspecies > OR_MAX_SPECIES) return NULL;
    or_sim *s = (or_sim *)calloc(1, sizeof(or_sim));
    s->g = *g;
    s->nsp = nspecies;
    for (int i = 0; i < nspecies; ++i) s->sp[i] = sp[i];
    s->las = *l;
    s->run = *r;
    s->sx = g->nx + 1;
    s->nn = (size_t)s->sx * g->ny * g->nz;
    for (int c = 0; c < OR_NCOMP; ++c) s->f[c] = (double *)calloc(s->nn, sizeof(double));
    s->sw = (uint8_t *)calloc(s->nn, 1);
    s->calm = (uint8_t *)calloc(s->nn, 1);
    uint8_t init_sw = r->switch_mode == OR_SW_ALL_FLUID ? 0 : 1;
    memset(s->sw, init_sw, s->nn);
    for (int i = 0; i < nspecies; ++i) {
        or_init_species(s, i);
        if (sp[i].fluid && r->switch_mode != OR_SW_ALL_PIC) {
            s->fn[i] = (double *)calloc(s->nn, sizeof(double));
            for (int d = 0; d < 3; ++d) s->fu[i][d] = (double *)calloc(s->nn, sizeof(double));
            if (sp[i].gamma_ad > 0.0) s->fs[i] = (double *)calloc(s->nn, sizeof(double));
        }
    }
    if (r->enable_qed) or_qed_init(s);
    s->gauss0 = (double *)calloc(s->nn, sizeof(double));
    return s;
}

void or_destroy(or_sim *s) {
    if (!s) return;
    for (int c = 0; c < OR_NCOMP; ++c) free(s->f[c]);
    for (int i = 0; i < s->nsp; ++i) {
        or_parts *p = &s->p[i];
        free(p->ci); free(p->cj); free(p->ck); free(p->ox); free(p->oy); free(p->oz); free(p->ux); free(p->uy); free(p->uz);
        free(p->w); free(p->tau); free(p->id); free(p->zc);
        free(s->fn[i]);
        free(s->fs[i]);
        for (int d = 0; d < 3; ++d) free(s->fu[i][d]);
    }
    free(s->sw); free(s->calm); free(s->gauss0); free(s->ev);
    or_qed_free(s);
    or_cnn_free(s);
    free(s);
}

static void gauss_snapshot(or_sim *s) {
    double *rho = (double *)malloc(sizeof(double) * s->nn);
    or_divE(s, s->gauss0);
    or_rho(s, rho);
    for (size_t c = 0; c < s->nn; ++c) s->gauss0[c] -= rho[c];
    free(rho);
    s->have_gauss0 = 1;
}

int or_step(or_sim *s, int nsteps) {
    const or_grid *g = &s->g;
    if (!s->have_gauss0) gauss_snapshot(s);
    for (int it = 0; it < nsteps; ++it) {
        int mode = s->run.switch_mode;
        if ((mode == OR_SW_THRESHOLD || mode == OR_SW_CNN) &&
            s->step % (s->run.switch_every > 0 ? s->run.switch_every : 1) == 0)
            or_switch_eval(s);
        for (int c = OR_JX; c <= OR_JZ; ++c) memset(s->f[c], 0, sizeof(double) * s->nn);
        or_antenna(s, s->t + 0.5 * g->dt);
        or_particle_phase(s);
        if (s->run.enable_qed) or_photon_phase(s);
        or_spawn_flush(s);   /* particles born this step move from the next one */
        if (mode != OR_SW_ALL_PIC) {
            or_fluid_phase(s);
            or_absorb(s);
            or_spawn_fluid(s);
        }
        or_yee_b_half(s);
        or_yee_e_full(s);
        or_yee_b_half(s);
        s->step++;
        s->t = s->step * g->dt;
    }
    return 0;
}

size_t or_field_size(const or_sim *s) { return s->nn; }

int or_get_field(const or_sim *s, int comp, double *out) {
    if (comp < 0 || comp >= OR_NCOMP) return -1;
    memcpy(out, s->f[comp], sizeof(double) * s->nn);
    return 0;
}

int or_set_field(or_sim *s, int comp, const double *in) {
    if (comp < 0 || comp >= OR_NCOMP) return -1;
    memcpy(s->f[comp], in, sizeof(double) * s->nn);
    s->have_gauss0 = 0;
    return 0;
}

size_t or_particle_count(const or_sim *s, int sp) {
    return (sp >= 0 && sp < s->nsp) ? s->p[sp].n : 0;
}

int or_get_particles(const or_sim *s, int sp, double *x, double *u, double *w, uint64_t *id,
                     int32_t *z, double *tau) {
    if (sp < 0 || sp >= s->nsp) return -1;
    const or_parts *p = &s->p[sp];
    for (size_t n = 0; n < p->n; ++n) {
        if (x) {
            x[3 * n] = (p->ci[n] + p->ox[n]) * s->g.dx;
            x[3 * n + 1] = (p->cj[n] + p->oy[n]) * s->g.dy;
            x[3 * n + 2] = (p->ck[n] + p->oz[n]) * s->g.dz;
        }
        if (u) { u[3 * n] = p->ux[n]; u[3 * n + 1] = p->uy[n]; u[3 * n + 2] = p->uz[n]; }
        if (w) w[n] = p->w[n];
        if (id) id[n] = p->id[n];
        if (z) z[n] = p->zc[n];
        if (tau) tau[n] = p->tau[n];
    }
    return 0;
}

int or_set_particles(or_sim *s, int sp, size_t n, const double *x, const double *u,
                     const double *w, const uint64_t *id, const int32_t *z, const double *tau) {
    if (sp < 0 || sp >= s->nsp) return -1;
    or_parts *p = &s->p[sp];
    p->n = 0;
    or_parts_reserve(p, n);
    double dxs[3] = {s->g.dx, s->g.dy, s->g.dz};
    for (size_t q = 0; q < n; ++q) {
        /* absolute position -> cell index + offset (same rule as the library) */
        int c[3];
        double o[3];
        for (int d = 0; d < 3; ++d) {
            double X = x[3 * q + d] / dxs[d];
            c[d] = (int)floor(X);
            o[d] = X - c[d];
        }
        uint64_t pid = id ? id[q] : q;
        /* without given optical depths a QED particle draws its own, as a new one does */
        double t0 = tau ? tau[q] : (s->sp[sp].qed ? or_qed_tau0(s, pid) : 0.0);
        or_parts_push_back(p, c[0], c[1], c[2], o[0], o[1], o[2], u[3 * q], u[3 * q + 1],
                           u[3 * q + 2], w[q], t0, pid,
                           z ? z[q] : (int32_t)llround(s->sp[sp].charge));
    }
    s->have_gauss0 = 0;
    return 0;
}

int or_get_fluid(const or_sim *s, int sp, double *n, double *u) {
    if (sp < 0 || sp >= s->nsp || !s->fn[sp]) return -1;
    memcpy(n, s->fn[sp], sizeof(double) * s->nn);
    for (size_t c = 0; c < s->nn; ++c)
        for (int d = 0; d < 3; ++d) u[3 * c + d] = s->fu[sp][d][c];
    return 0;
}

int or_set_fluid(or_sim *s, int sp, const double *n, const double *u) {
    if (sp < 0 || sp >= s->nsp || !s->fn[sp]) return -1;
    memcpy(s->fn[sp], n, sizeof(double) * s->nn);
    for (size_t c = 0; c < s->nn; ++c)
        for (int d = 0; d < 3; ++d) s->fu[sp][d][c] = u[3 * c + d];
    s->have_gauss0 = 0;
    return 0;
}

/* p = (n K) n^(gamma - 1) */
int or_get_fluid_p(const or_sim *s, int sp, double *p) {
    if (sp < 0 || sp >= s->nsp || !s->fs[sp]) return -1;
    const double ga = s->sp[sp].gamma_ad;
    for (size_t c = 0; c < s->nn; ++c) {
        double n = s->fn[sp][c];
        p[c] = n > 0.0 ? s->fs[sp][c] * pow(n, ga - 1.0) : 0.0;
    }
    return 0;
}

int or_set_fluid_p(or_sim *s, int sp, const double *p) {
    if (sp < 0 || sp >= s->nsp || !s->fs[sp]) return -1;
    const double ga = s->sp[sp].gamma_ad;
    for (size_t c = 0; c < s->nn; ++c) {
        double n = s->fn[sp][c];
        s->fs[sp][c] = n > 0.0 ? p[c] * pow(n, 1.0 - ga) : 0.0;
    }
    return 0;
}

int or_get_switch(const or_sim *s, uint8_t *out) { memcpy(out, s->sw, s->nn); return 0; }

int or_set_switch(or_sim *s, const uint8_t *in) {
    memcpy(s->sw, in, s->nn);
    memset(s->calm, 0, s->nn);
    s->run.switch_mode = OR_SW_FIXED;
    return 0;
}

int or_set_switch_mode(or_sim *s, int mode) {
    s->run.switch_mode = mode;
    if (mode == OR_SW_ALL_PIC) memset(s->sw, 1, s->nn);
    if (mode == OR_SW_ALL_FLUID) memset(s->sw, 0, s->nn);
    return 0;
}

int or_get_rho(const or_sim *s, double *rho) { or_rho(s, rho); return 0; }
int or_get_divE(const or_sim *s, double *d) { or_divE(s, d); return 0; }

int or_diagnostics(or_sim *s, or_diag *d) {
    const or_grid *g = &s->g;
    memset(d, 0, sizeof(*d));
    double dv = g->dx * g->dy * g->dz;
    int per = g->bc_x == OR_BC_PERIODIC;
    d->t = s->t;
    d->step = s->step;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i <= g->nx; ++i) {
                size_t c = or_idx(s, i, j, k);
                int half_ok = i < g->nx;
                int node_ok = per ? i < g->nx : 1;
                double ee = 0, bb = 0;
                if (half_ok) ee += s->f[OR_EX][c] * s->f[OR_EX][c];
                if (node_ok) ee += s->f[OR_EY][c] * s->f[OR_EY][c] + s->f[OR_EZ][c] * s->f[OR_EZ][c];
                if (node_ok) bb += s->f[OR_BX][c] * s->f[OR_BX][c];
                if (half_ok) bb += s->f[OR_BY][c] * s->f[OR_BY][c] + s->f[OR_BZ][c] * s->f[OR_BZ][c];
                d->u_e += 0.5 * ee * dv;
                d->u_b += 0.5 * bb * dv;
            }
    for (int isp = 0; isp < s->nsp; ++isp) {
        const or_parts *p = &s->p[isp];
        const or_species *sp = &s->sp[isp];
        d->count[isp] = (double)p->n;
        for (size_t n = 0; n < p->n; ++n) {
            double u2 = p->ux[n] * p->ux[n] + p->uy[n] * p->uy[n] + p->uz[n] * p->uz[n];
            if (sp->kind == OR_PHOTON) d->kin[isp] += p->w[n] * sqrt(u2);
            else d->kin[isp] += p->w[n] * sp->mass * (sqrt(1.0 + u2) - 1.0);
            double q = sp->kind == OR_ION ? p->zc[n] : sp->charge;
            d->charge_total += q * p->w[n];
        }
        if (s->fn[isp])
            for (size_t c = 0; c < s->nn; ++c) {
                double m = s->fn[isp][c] * dv;
                double u2 = 0;
                for (int q = 0; q < 3; ++q) u2 += s->fu[isp][q][c] * s->fu[isp][q][c];
                d->fluid_mass[isp] += m;
                d->fluid_kin[isp] += m * sp->mass * (sqrt(1.0 + u2) - 1.0);
                d->charge_total += sp->charge * m;
                if (s->fs[isp] && s->fn[isp][c] > 0.0)
                    d->fluid_th[isp] += s->fs[isp][c] * pow(s->fn[isp][c], sp->gamma_ad - 1.0) * dv /
                                        (sp->gamma_ad - 1.0);
            }
    }
    /* Gauss: change of (div E - rho) since the first step, over interior
     * nodes (open x: without the wall planes and the antenna plane). */
    double *dive = (double *)malloc(sizeof(double) * s->nn);
    double *rho = (double *)malloc(sizeof(double) * s->nn);
    or_divE(s, dive);
    or_rho(s, rho);
    if (!s->have_gauss0) gauss_snapshot(s);
    double mx = 0, l2 = 0;
    size_t cnt = 0;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                if (!per && (i == 0 || (s->las.enabled && i == s->las.i_antenna))) continue;
                size_t c = or_idx(s, i, j, k);
                double r = dive[c] - rho[c] - s->gauss0[c];
                mx = fmax(mx, fabs(r));
                l2 += r * r;
                cnt++;
            }
    d->gauss_max = mx;
    d->gauss_l2 = cnt ? sqrt(l2 / cnt) : 0.0;
    free(dive); free(rho);
    size_t kin = 0, tot = 0;
    int nxn = per ? g->nx : g->nx + 1;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < nxn; ++i) { kin += s->sw[or_idx(s, i, j, k)]; tot++; }
    d->kinetic_fraction = (double)kin / (double)tot;
    d->conv_loss = s->conv_loss;
    d->ion_energy = s->ion_energy;
    d->photon_energy = s->photon_ledger;
    d->fallback_fraction = s->fallback_fraction;
    return 0;
}
