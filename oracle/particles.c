/*
 * Oracle particle kernel: species initialisation, CIC field gather,
 * relativistic Boris push, position advance with wall reflection, and the
 * charge-conserving Esirkepov current deposition.
 *
 * Paper: Methodology, plasma-model paragraph (macro-particles weighted by
 * density and volume fraction, Boris pusher), grid paragraph (particle
 * deposition and field gathering on the uniform grid) and boundary paragraph
 * (particles reverse their velocity at the domain walls).
 * Literature: J. P. Boris (1970) rotation; T. Zh. Esirkepov, Comput. Phys.
 * Commun. 135 (2001) 144, density decomposition for CIC form factors.
 */
#include "or_internal.h"

void or_parts_reserve(or_parts *p, size_t cap) {
    if (cap <= p->cap) return;
    size_t c = p->cap ? p->cap : 64;
    while (c < cap) c *= 2;
#define GROW(f, T) p->f = (T *)realloc(p->f, sizeof(T) * c)
    GROW(ci, int32_t); GROW(cj, int32_t); GROW(ck, int32_t);
    GROW(ox, double); GROW(oy, double); GROW(oz, double);
    GROW(ux, double); GROW(uy, double); GROW(uz, double);
    GROW(w, double); GROW(tau, double); GROW(id, uint64_t); GROW(zc, int32_t);
#undef GROW
    p->cap = c;
}

void or_parts_push_back(or_parts *p, int32_t ci, int32_t cj, int32_t ck, double ox,
                        double oy, double oz, double ux, double uy, double uz, double w,
                        double tau, uint64_t id, int32_t zc) {
    or_parts_reserve(p, p->n + 1);
    size_t i = p->n++;
    p->ci[i] = ci; p->cj[i] = cj; p->ck[i] = ck;
    p->ox[i] = ox; p->oy[i] = oy; p->oz[i] = oz;
    p->ux[i] = ux; p->uy[i] = uy; p->uz[i] = uz;
    p->w[i] = w; p->tau[i] = tau; p->id[i] = id; p->zc[i] = zc;
}

/* Order-preserving removal. */
void or_parts_remove(or_parts *p, size_t i) {
    size_t m = p->n - i - 1;
#define SHIFT(f) memmove(p->f + i, p->f + i + 1, sizeof(*p->f) * m)
    SHIFT(ci); SHIFT(cj); SHIFT(ck); SHIFT(ox); SHIFT(oy); SHIFT(oz); SHIFT(ux); SHIFT(uy); SHIFT(uz);
    SHIFT(w); SHIFT(tau); SHIFT(id); SHIFT(zc);
#undef SHIFT
    p->n--;
}

/* Density profile n(x) in n_c, evaluated at a cell centre. */
static double profile(const or_species *sp, double x) {
    switch (sp->profile) {
    case OR_PROF_UNIFORM: return sp->n0;
    case OR_PROF_RAMP:
        if (x < sp->x0) return 0.0;
        return sp->n0 * fmin(1.0, (x - sp->x0) / sp->length);
    case OR_PROF_FOIL:
        return (x >= sp->x0 && x < sp->x0 + sp->length) ? sp->n0 : 0.0;
    default: return 0.0;
    }
}

/* ppc particles per cell whose centre has n > 0.  Particle k of cell c has
 * position index c*ppc + k and id (species << 52) | (c*ppc + k), unique over
 * the species.  Its position offsets are Philox draws (tag 1) keyed by the
 * position index, so the species of one cell start at the same points (a
 * neutral plasma starts without charge separation); its momentum components
 * are Gaussian draws by Box-Muller (tag 2) keyed by the id, independent from
 * species to species.  Weight n dV / ppc. */
void or_init_species(or_sim *s, int isp) {
    const or_species *sp = &s->sp[isp];
    const or_grid *g = &s->g;
    or_parts *p = &s->p[isp];
    if (sp->ppc <= 0 || sp->profile == OR_PROF_NONE) return;
    double dv = g->dx * g->dy * g->dz;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                double n = profile(sp, (i + 0.5) * g->dx);
                if (n <= 0) continue;
                uint64_t cell = (uint64_t)i + (uint64_t)g->nx * ((uint64_t)j + (uint64_t)g->ny * k);
                for (int q = 0; q < sp->ppc; ++q) {
                    uint64_t pos = cell * (uint64_t)sp->ppc + (uint64_t)q;
                    uint64_t id = ((uint64_t)isp << 52) | pos;
                    uint32_t rp[4], rm[4];
                    or_draw4(s, pos, 0, 1, 0, rp);
                    or_draw4(s, id, 0, 2, 0, rm);
                    double r0 = or_uniform(rm[0]), r1 = or_uniform(rm[1]);
                    double r2 = or_uniform(rm[2]), r3 = or_uniform(rm[3]);
                    double m0 = sqrt(-2.0 * log(r0)), m1 = sqrt(-2.0 * log(r2));
                    double ux = sp->u_th * m0 * cos(2.0 * OR_PI * r1);
                    double uy = sp->u_th * m0 * sin(2.0 * OR_PI * r1);
                    double uz = sp->u_th * m1 * cos(2.0 * OR_PI * r3);
                    or_parts_push_back(p, i, j, k, or_uniform(rp[0]), or_uniform(rp[1]),
                                       or_uniform(rp[2]), ux, uy, uz, n * dv / sp->ppc,
                                       sp->qed ? or_qed_tau0(s, id) : 0.0, id,
                                       (int32_t)llround(sp->charge));
                }
            }
}

/* Relativistic Boris rotation; u = gamma v, fields already interpolated. */
void or_boris(double qm, double dt, const double e[3], const double b[3], double u[3]) {
    double h = 0.5 * qm * dt;
    double um[3] = {u[0] + h * e[0], u[1] + h * e[1], u[2] + h * e[2]};
    double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    double t[3] = {h * b[0] / gm, h * b[1] / gm, h * b[2] / gm};
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    double sv[3] = {2 * t[0] / (1 + t2), 2 * t[1] / (1 + t2), 2 * t[2] / (1 + t2)};
    double up[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]),
                    um[1] + (um[2] * t[0] - um[0] * t[2]),
                    um[2] + (um[0] * t[1] - um[1] * t[0])};
    double uq[3] = {um[0] + (up[1] * sv[2] - up[2] * sv[1]),
                    um[1] + (up[2] * sv[0] - up[0] * sv[2]),
                    um[2] + (up[0] * sv[1] - up[1] * sv[0])};
    u[0] = uq[0] + h * e[0];
    u[1] = uq[1] + h * e[1];
    u[2] = uq[2] + h * e[2];
}

static double cic(double d) { d = fabs(d); return d < 1.0 ? 1.0 - d : 0.0; }

/* Esirkepov decomposition for CIC shapes on a 3x3x3 node window starting at
 * base = min(floor(old), floor(new)) per axis.  Positions in cell units.
 * jx[a][b][c] is the current on the x face (base+a+1/2, base+b, base+c), and
 * cyclically for jy, jz.  qw_dv = q w / dV; dx are the cell sizes. */
void or_esirkepov(const double x0[3], const double x1[3], double qw_dv, double dt,
                  const double dx[3], double jx[27], double jy[27], double jz[27],
                  int base[3]) {
    double S0[3][3], DS[3][3];
    for (int d = 0; d < 3; ++d) {
        int f0 = (int)floor(x0[d]), f1 = (int)floor(x1[d]);
        base[d] = f0 < f1 ? f0 : f1;
        for (int a = 0; a < 3; ++a) {
            double s0 = cic(x0[d] - (base[d] + a));
            double s1 = cic(x1[d] - (base[d] + a));
            S0[d][a] = s0;
            DS[d][a] = s1 - s0;
        }
    }
    double W[3][27];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) {
                int n = a + 3 * (b + 3 * c);
                W[0][n] = DS[0][a] * (S0[1][b] * S0[2][c] + 0.5 * DS[1][b] * S0[2][c] +
                                      0.5 * S0[1][b] * DS[2][c] + DS[1][b] * DS[2][c] / 3.0);
                W[1][n] = DS[1][b] * (S0[0][a] * S0[2][c] + 0.5 * DS[0][a] * S0[2][c] +
                                      0.5 * S0[0][a] * DS[2][c] + DS[0][a] * DS[2][c] / 3.0);
                W[2][n] = DS[2][c] * (S0[0][a] * S0[1][b] + 0.5 * DS[0][a] * S0[1][b] +
                                      0.5 * S0[0][a] * DS[1][b] + DS[0][a] * DS[1][b] / 3.0);
            }
    /* J(face a+1/2) = J(face a-1/2) - q w/dV * (dx/dt) * W(a): prefix along the axis. */
    for (int b = 0; b < 3; ++b)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int a = 0; a < 3; ++a) {
                int n = a + 3 * (b + 3 * c);
                acc -= qw_dv * dx[0] / dt * W[0][n];
                jx[n] = acc;
            }
        }
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int b = 0; b < 3; ++b) {
                int n = a + 3 * (b + 3 * c);
                acc -= qw_dv * dx[1] / dt * W[1][n];
                jy[n] = acc;
            }
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int c = 0; c < 3; ++c) {
                int n = a + 3 * (b + 3 * c);
                acc -= qw_dv * dx[2] / dt * W[2][n];
                jz[n] = acc;
            }
        }
}

/* Add the Esirkepov current of a move X0 -> X1 to the grid J.  X0 and X1 are
 * positions relative to the node `cell` (cell units; X1 may leave [0,1) by
 * less than one cell).  The last face of each x row carries the total, which
 * is zero; entries outside an open x box are zero too. */
void or_deposit_move(or_sim *s, double q, double w, const int cell[3], const double X0[3],
                     const double X1[3]) {
    const or_grid *g = &s->g;
    double dv = g->dx * g->dy * g->dz;
    double dx[3] = {g->dx, g->dy, g->dz};
    double jx[27], jy[27], jz[27];
    int base[3];
    or_esirkepov(X0, X1, q * w / dv, g->dt, dx, jx, jy, jz, base);
    int per = g->bc_x == OR_BC_PERIODIC;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) {
                int n = a + 3 * (b + 3 * c);
                int i = cell[0] + base[0] + a;
                int j = or_wrap(cell[1] + base[1] + b, g->ny);
                int k = or_wrap(cell[2] + base[2] + c, g->nz);
                int ii = per ? or_wrap(i, g->nx) : i;
                /* x faces: a = 2 is the closing face (total zero) */
                if (a < 2 && (per || (ii >= 0 && ii < g->nx)))
                    s->f[OR_JX][or_idx(s, ii, j, k)] += jx[n];
                if (per || (ii >= 0 && ii <= g->nx)) {
                    if (b < 2) s->f[OR_JY][or_idx(s, ii, j, k)] += jy[n];
                    if (c < 2) s->f[OR_JZ][or_idx(s, ii, j, k)] += jz[n];
                }
            }
}

/* Charge density at nodes from particles (CIC) and fluids (node values). */
void or_rho(const or_sim *s, double *rho) {
    const or_grid *g = &s->g;
    double dv = g->dx * g->dy * g->dz;
    memset(rho, 0, sizeof(double) * s->nn);
    int per = g->bc_x == OR_BC_PERIODIC;
    for (int isp = 0; isp < s->nsp; ++isp) {
        const or_parts *p = &s->p[isp];
        if (s->sp[isp].kind == OR_PHOTON) continue;
        for (size_t n = 0; n < p->n; ++n) {
            int i0 = p->ci[n], j0 = p->cj[n], k0 = p->ck[n];
            double fx = p->ox[n], fy = p->oy[n], fz = p->oz[n];
            double q = s->sp[isp].kind == OR_ION ? (double)p->zc[n] : s->sp[isp].charge;
            for (int c = 0; c < 2; ++c)
                for (int b = 0; b < 2; ++b)
                    for (int a = 0; a < 2; ++a) {
                        int i = per ? or_wrap(i0 + a, g->nx) : i0 + a;
                        int j = or_wrap(j0 + b, g->ny), k = or_wrap(k0 + c, g->nz);
                        double wgt = (a ? fx : 1 - fx) * (b ? fy : 1 - fy) * (c ? fz : 1 - fz);
                        rho[or_idx(s, i, j, k)] += q * p->w[n] * wgt / dv;
                    }
        }
        if (s->fn[isp]) {
            double q = s->sp[isp].charge;
            for (size_t c = 0; c < s->nn; ++c) rho[c] += q * s->fn[isp][c];
        }
    }
}

void or_spawn_add(or_sim *s, const or_spawn *e) {
    if (s->nev == s->cap_ev) {
        s->cap_ev = s->cap_ev ? 2 * s->cap_ev : 256;
        s->ev = (or_spawn *)realloc(s->ev, sizeof(or_spawn) * s->cap_ev);
    }
    s->ev[s->nev++] = *e;
}

static int cmp_spawn(const void *a, const void *b) {
    const or_spawn *x = (const or_spawn *)a, *y = (const or_spawn *)b;
    if (x->species != y->species) return x->species < y->species ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

/* Particles created during the particle phase join their species after it,
 * in id order, so that no newborn particle is pushed in its birth step. */
void or_spawn_flush(or_sim *s) {
    qsort(s->ev, s->nev, sizeof(or_spawn), cmp_spawn);
    for (size_t n = 0; n < s->nev; ++n) {
        or_spawn *e = &s->ev[n];
        or_parts_push_back(&s->p[e->species], e->ci, e->cj, e->ck, e->ox, e->oy, e->oz,
                           e->ux, e->uy, e->uz, e->w, e->tau, e->id, e->zc);
    }
    s->nev = 0;
}

/* Nearest node of a particle (open x clamps to the wall planes). */
static size_t nearest_node(const or_sim *s, const or_parts *p, size_t n) {
    const or_grid *g = &s->g;
    int i = p->ci[n] + (p->ox[n] >= 0.5), j = p->cj[n] + (p->oy[n] >= 0.5);
    int k = p->ck[n] + (p->oz[n] >= 0.5);
    if (g->bc_x == OR_BC_PERIODIC) i = or_wrap(i, g->nx);
    else i = i > g->nx ? g->nx : i;
    return or_idx(s, i, or_wrap(j, g->ny), or_wrap(k, g->nz));
}

/* Carry a position relative to cell c into [0,1) offsets of its new cell. */
void or_carry(const or_sim *s, int c[3], double X[3]) {
    const or_grid *g = &s->g;
    for (int d = 0; d < 3; ++d) {
        int f = (int)floor(X[d]);
        c[d] += f;
        X[d] -= f;
    }
    if (g->bc_x == OR_BC_PERIODIC) c[0] = or_wrap(c[0], g->nx);
    c[1] = or_wrap(c[1], g->ny);
    c[2] = or_wrap(c[2], g->nz);
}

/* Specular reflection at the open x walls of a position X (relative to cell
 * index ci) after a move: the normal momentum changes sign. */
void or_reflect_x(const or_sim *s, int ci, double *X, double *ux) {
    const or_grid *g = &s->g;
    if (g->bc_x != OR_BC_OPEN) return;
    double a = ci + *X;                          /* absolute, cell units */
    if (a < 0.0) { *X = -a - ci; *ux = -*ux; }
    else if (a >= g->nx) {
        *X = (2.0 * g->nx - a) - ci;
        *ux = -*ux;
        if (ci + *X >= g->nx) *X = nextafter(1.0, 0.0) + (g->nx - 1 - ci);
    }
}

/* One pass over every charged particle in species then storage order:
 * gather E^n, B^n at x^n; ionization (ions); photon emission (leptons);
 * Boris push to u^{n+1/2}; x^{n+1} = x^n + dt u/gamma; wall reflection in
 * open x, wrap in periodic directions; Esirkepov deposit of J^{n+1/2}. */
void or_particle_phase(or_sim *s) {
    const or_grid *g = &s->g;
    int hybrid = s->run.switch_mode != OR_SW_ALL_PIC;
    double dxs[3] = {g->dx, g->dy, g->dz};
    for (int isp = 0; isp < s->nsp; ++isp) {
        const or_species *sp = &s->sp[isp];
        if (sp->kind == OR_PHOTON) continue;
        or_parts *p = &s->p[isp];
        size_t n0 = p->n;
        for (size_t n = 0; n < n0; ++n) {
            int kinetic = !hybrid || s->sw[nearest_node(s, p, n)];
            if (!sp->mobile && !kinetic) continue;
            int c[3] = {p->ci[n], p->cj[n], p->ck[n]};
            double X0[3] = {p->ox[n], p->oy[n], p->oz[n]};
            double e[3], b[3];
            for (int d = 0; d < 3; ++d) {
                e[d] = or_gather(s, OR_EX + d, c, X0);
                b[d] = or_gather(s, OR_BX + d, c, X0);
            }
            if (sp->kind == OR_ION && sp->ionizable && s->run.enable_ionization && kinetic)
                or_ionize_particle(s, isp, n, sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]));
            /* every lepton particle radiates: in a fluid node it is a hot
             * particle the conversion keeps, or one the conversion takes at
             * the end of this step */
            if (sp->kind != OR_ION && sp->qed && s->run.enable_qed)
                or_qed_emit(s, isp, n, e, b);
            if (!sp->mobile) continue;
            double q = sp->kind == OR_ION ? (double)p->zc[n] : sp->charge;
            double u[3] = {p->ux[n], p->uy[n], p->uz[n]};
            or_boris(q / sp->mass, g->dt, e, b, u);
            double gam = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            double X1[3];
            for (int d = 0; d < 3; ++d) X1[d] = X0[d] + g->dt * u[d] / gam / dxs[d];
            or_reflect_x(s, c[0], &X1[0], &u[0]);
            if (q != 0.0) or_deposit_move(s, q, p->w[n], c, X0, X1);
            or_carry(s, c, X1);
            p->ci[n] = c[0]; p->cj[n] = c[1]; p->ck[n] = c[2];
            p->ox[n] = X1[0]; p->oy[n] = X1[1]; p->oz[n] = X1[2];
            p->ux[n] = u[0]; p->uy[n] = u[1]; p->uz[n] = u[2];
        }
    }
}
