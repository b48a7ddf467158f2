/*
 * Oracle regime switch and fluid <-> particle conversion.
 *
 * Paper: abstract and Methodology (fluid in stable regions, PIC where the
 * switch flags instability; instability thresholds used as prior knowledge
 * for the switch, Results after Table 1; charge and energy conservation
 * checks during regime switches, validation paragraph).  The paper gives no
 * threshold values and no conversion rule; the readings used here are:
 *
 *  indicators per node, from nearest-node moments of the fluid-capable
 *  species (particles plus fluid) and the node-interpolated E:
 *    a   = |E|
 *    g   = |(N(+1)-N(-1)) per axis| / (2 max(N, n_floor dV)), N = node moment
 *          sum w; the gradient counts only beyond three standard deviations
 *          of its shot noise, sigma_g = sqrt(sum of the six neighbours' sum w^2)
 *          / (2 max(N, n_floor dV)), i.e. the test is g - 3 sigma_g >= thr_grad;
 *          fluid mass M on a node counts as ppc particles of weight M/ppc
 *    s_u = sqrt(<|u|^2> - |<u>|^2)
 *    ion: ionizable ions present and level-0 rate * dt >= thr_ion
 *    chi: gamma_rms |E| / a_S >= thr_chi (QED runs)
 *  kinetic if any indicator reaches its threshold (>=), dilated by
 *  `dilation` nodes; a kinetic node returns to fluid only after
 *  `hysteresis` consecutive evaluations with every indicator below half its
 *  threshold in the dilated neighbourhood.
 *
 *  hot particles: a particle with |u| >= thr_hot (when thr_hot > 0) is a
 *  kinetic population wherever it is: it is never absorbed and does not enter
 *  the switch moments, so a hot beam crossing a cold bulk leaves the bulk
 *  fluid (the bulk's own state decides its regime).
 *
 *  conversion (after the fluid update of every hybrid step):
 *    absorb: a particle of a fluid-capable species whose nearest node is
 *      fluid, and which is not hot, is moved virtually to that node
 *      (Esirkepov current of the move) and its weight and momentum join the
 *      node fluid, at one time level (x^{n+1}, u^{n+1/2} with n^{n+1},
 *      u^{n+1/2});
 *    spawn: fluid mass M = n dV >= spawn_frac * w0 on
 *      a kinetic node, w0 = n0 dV / ppc the species' reference weight, becomes
 *      m = round(M / w0) particles (at least 1, at most 64) of weight M/m with
 *      the fluid momentum, moved virtually from the node to Philox positions
 *      in the node's dual cell.
 *  A CIC particle sitting on a node has exactly the node-delta charge of the
 *  fluid, so both conversions keep div E - rho unchanged.
 *  Warm fluid (gamma_ad > 0): the kinetic energy an absorption loses (the
 *  particles' spread about the merged flow) heats the node, p += (gamma_ad -
 *  1) dE / dV, instead of going to the ledger (unless the merged mass or
 *  pressure is not positive, which a node whose fluid density had gone
 *  negative can give: then S = 0 and the ledger takes that heat and the
 *  node's previous thermal energy); a spawned particle gets the
 *  fluid momentum plus a Gaussian spread sqrt(T / m) per component, T = p / n
 *  (Box-Muller on Philox draws, tag 13), and the ledger takes the difference
 *  between the fluid's kinetic plus thermal energy and the sample's.
 *  A spawned particle's id is 2^63 | step << 40 | species << 37 | node << 6 |
 *  slot; its position draws (tag 12) are keyed by (node, step, slot), shared
 *  by the species spawned on one node (a neutral fluid spawns neutral), its
 *  thermal draws by its id.
 */
#include "or_internal.h"

static int clampx(const or_sim *s, int i) {
    if (s->g.bc_x == OR_BC_PERIODIC) return or_wrap(i, s->g.nx);
    return i < 0 ? 0 : (i > s->g.nx ? s->g.nx : i);
}

static int node_x_count(const or_sim *s) {
    return s->g.bc_x == OR_BC_PERIODIC ? s->g.nx : s->g.nx + 1;
}

/* Nearest node of particle n; rel receives the node's offset (0 or 1 per
 * axis) relative to the particle's cell. */
static size_t nearest(const or_sim *s, const or_parts *p, size_t n, int *rel) {
    int r[3] = {p->ox[n] >= 0.5, p->oy[n] >= 0.5, p->oz[n] >= 0.5};
    if (rel) { rel[0] = r[0]; rel[1] = r[1]; rel[2] = r[2]; }
    return or_idx(s, clampx(s, p->ci[n] + r[0]), or_wrap(p->cj[n] + r[1], s->g.ny),
                  or_wrap(p->ck[n] + r[2], s->g.nz));
}

/* A hot particle (|u| >= thr_hot, thr_hot > 0). */
int or_is_hot(const or_sim *s, const double u[3]) {
    double h = s->run.thr_hot;
    return h > 0.0 && u[0] * u[0] + u[1] * u[1] + u[2] * u[2] >= h * h;
}

extern double or_cnn_switch(or_sim *s, const double *nmom, const double *u2mom, const double *nimom,
                            uint8_t *hot, uint8_t *cold);

/* Nearest-node moments of the fluid species (particles that are not hot,
 * then fluid mass): N = sum w, V = sum w^2, P = sum w u, U2 = sum w |u|^2;
 * NI = weight of ionizable ions not yet at their last charge state. */
static void node_moments(const or_sim *s, double *N, double *P, double *U2, double *NI, double *V) {
    size_t nn = s->nn;
    double dv = s->g.dx * s->g.dy * s->g.dz;
    for (int isp = 0; isp < s->nsp; ++isp) {
        const or_species *sp = &s->sp[isp];
        const or_parts *p = &s->p[isp];
        if (sp->fluid) {
            for (size_t n = 0; n < p->n; ++n) {
                double u[3] = {p->ux[n], p->uy[n], p->uz[n]};
                if (or_is_hot(s, u)) continue;
                size_t c = nearest(s, p, n, NULL);
                N[c] += p->w[n];
                V[c] += p->w[n] * p->w[n];
                for (int d = 0; d < 3; ++d) P[3 * c + d] += p->w[n] * u[d];
                U2[c] += p->w[n] * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            }
            if (s->fn[sp - s->sp])
                for (size_t c = 0; c < nn; ++c) {
                    double m = s->fn[isp][c] * dv;
                    if (m <= 0) continue;
                    double u[3] = {s->fu[isp][0][c], s->fu[isp][1][c], s->fu[isp][2][c]};
                    N[c] += m;
                    V[c] += m * m / (sp->ppc > 0 ? sp->ppc : 1);
                    for (int d = 0; d < 3; ++d) P[3 * c + d] += m * u[d];
                    U2[c] += m * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                }
        }
        if (sp->kind == OR_ION && sp->ionizable && s->run.enable_ionization)
            for (size_t n = 0; n < p->n; ++n)
                if (p->zc[n] < sp->z_max) {
                    size_t c = nearest(s, p, n, NULL);
                    NI[c] += p->w[n];
                }
    }
}

void or_switch_eval(or_sim *s) {
    const or_grid *g = &s->g;
    size_t nn = s->nn;
    double dv = g->dx * g->dy * g->dz;
    int nxn = node_x_count(s);
    double *N = (double *)calloc(nn, sizeof(double));
    double *P = (double *)calloc(nn * 3, sizeof(double));
    double *U2 = (double *)calloc(nn, sizeof(double));
    double *NI = (double *)calloc(nn, sizeof(double));
    double *V = (double *)calloc(nn, sizeof(double));
    node_moments(s, N, P, U2, NI, V);
    uint8_t *hot = (uint8_t *)calloc(nn, 1), *notcold = (uint8_t *)calloc(nn, 1);
    double a_s = 0.0;
    if (s->run.enable_qed) {
        double lam = s->las.lambda_um * 1e-6;
        double omega0 = 2.0 * OR_PI * OR_C / lam;
        a_s = OR_ME * OR_C * OR_C / (OR_HBAR * omega0);
    }
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < nxn; ++i) {
                size_t c = or_idx(s, i, j, k);
                double e[3];
                int node[3] = {i, j, k};
                double z0[3] = {0, 0, 0};
                for (int d = 0; d < 3; ++d) e[d] = or_gather(s, OR_EX + d, node, z0);
                double emag = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
                size_t xp = or_idx(s, clampx(s, i + 1), j, k), xm = or_idx(s, clampx(s, i - 1), j, k);
                size_t yp = or_idx(s, i, or_wrap(j + 1, g->ny), k), ym = or_idx(s, i, or_wrap(j - 1, g->ny), k);
                size_t zp = or_idx(s, i, j, or_wrap(k + 1, g->nz)), zm = or_idx(s, i, j, or_wrap(k - 1, g->nz));
                double dgx = N[xp] - N[xm], dgy = N[yp] - N[ym], dgz = N[zp] - N[zm];
                double den = 2.0 * fmax(N[c], s->run.n_floor * dv);
                double grad = sqrt(dgx * dgx + dgy * dgy + dgz * dgz) / den;
                double sig = sqrt(V[xp] + V[xm] + V[yp] + V[ym] + V[zp] + V[zm]) / den;
                grad = grad - 3.0 * sig;
                double su = 0.0, g2 = 0.0;
                if (N[c] > 0) {
                    double m2 = U2[c] / N[c];
                    double mx = P[3 * c] / N[c], my = P[3 * c + 1] / N[c], mz = P[3 * c + 2] / N[c];
                    su = sqrt(fmax(0.0, m2 - (mx * mx + my * my + mz * mz)));
                    g2 = m2;
                }
                double ionr = 0.0;
                if (NI[c] > 0)
                    for (int isp = 0; isp < s->nsp; ++isp)
                        if (s->sp[isp].kind == OR_ION && s->sp[isp].ionizable)
                            ionr = fmax(ionr, or_ion_rate_norm(s, isp, 0, emag) * g->dt);
                double chi = s->run.enable_qed ? sqrt(1.0 + g2) * emag / a_s : 0.0;
                const or_run *r = &s->run;
                int h = emag >= r->thr_a || grad >= r->thr_grad || su >= r->thr_sigma_u ||
                        (NI[c] > 0 && ionr >= r->thr_ion) ||
                        (r->enable_qed && chi >= r->thr_chi);
                int nc = emag >= 0.5 * r->thr_a || grad >= 0.5 * r->thr_grad ||
                         su >= 0.5 * r->thr_sigma_u || (NI[c] > 0 && ionr >= 0.5 * r->thr_ion) ||
                         (r->enable_qed && chi >= 0.5 * r->thr_chi);
                hot[c] = (uint8_t)h;
                notcold[c] = (uint8_t)nc;
            }
    s->fallback_fraction = 0.0;
    if (s->run.switch_mode == OR_SW_CNN)
        s->fallback_fraction = or_cnn_switch(s, N, U2, NI, hot, notcold);
    /* dilation + hysteresis */
    int D = s->run.dilation;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < nxn; ++i) {
                size_t c = or_idx(s, i, j, k);
                int kin = 0, warm = 0;
                for (int dk = -D; dk <= D; ++dk)
                    for (int dj = -D; dj <= D; ++dj)
                        for (int di = -D; di <= D; ++di) {
                            int ii = i + di;
                            if (g->bc_x == OR_BC_OPEN && (ii < 0 || ii > g->nx)) continue;
                            size_t q = or_idx(s, clampx(s, ii), or_wrap(j + dj, g->ny),
                                              or_wrap(k + dk, g->nz));
                            kin |= hot[q];
                            warm |= notcold[q];
                        }
                if (kin) { s->sw[c] = 1; s->calm[c] = 0; }
                else if (s->sw[c]) {
                    if (warm) s->calm[c] = 0;
                    else if (++s->calm[c] >= s->run.hysteresis) { s->sw[c] = 0; s->calm[c] = 0; }
                }
            }
    free(N); free(P); free(U2); free(NI); free(V); free(hot); free(notcold);
}

/* Training data of the learned switch at the current step, per node of the
 * canonical grid [nz][ny][NX] (x fastest).  raw9 (may be NULL): the network's
 * 8 inputs (as the CNN switch builds them) and the conversion energy
 * e = (1/2)(U2 - |P|^2 / N), the thermal energy a cold fluid at the mean
 * momentum drops (small-u limit).  cond: the label condition, bit 0 when e
 * exceeds 1e-3 of the node's kinetic energy U2 / 2 and the momentum spread
 * sqrt(2 e / N) reaches thr_sigma_u, bit 1 when an ionization is possible
 * (per-step probability at the node's field >= thr_ion, ionizable ions
 * present), bit 2 when a QED emission is possible (chi of the rms momentum
 * >= thr_chi).  The reading of the label is the one stated with
 * hk_dump_training; the paper leaves the training labels unstated. */
void or_training_node(or_sim *s, double *raw9, uint8_t *cond) {
    const or_grid *g = &s->g;
    size_t nn = s->nn;
    int nxn = node_x_count(s);
    double *N = (double *)calloc(nn, sizeof(double));
    double *P = (double *)calloc(nn * 3, sizeof(double));
    double *U2 = (double *)calloc(nn, sizeof(double));
    double *NI = (double *)calloc(nn, sizeof(double));
    double *V = (double *)calloc(nn, sizeof(double));
    node_moments(s, N, P, U2, NI, V);
    size_t nodes = (size_t)nxn * g->ny * g->nz;
    double *raw = NULL;
    if (raw9) {
        raw = (double *)malloc(sizeof(double) * nodes * 8);
        or_cnn_node_inputs(s, N, U2, raw);
    }
    double a_s = 0.0;
    if (s->run.enable_qed) {
        double omega0 = 2.0 * OR_PI * OR_C / (s->las.lambda_um * 1e-6);
        a_s = OR_ME * OR_C * OR_C / (OR_HBAR * omega0);
    }
    const or_run *r = &s->run;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < nxn; ++i) {
                size_t c = or_idx(s, i, j, k);
                size_t v = ((size_t)k * g->ny + j) * nxn + i;
                double e = 0.0;
                int bits = 0;
                if (N[c] > 0) {
                    double p2 = P[3 * c] * P[3 * c] + P[3 * c + 1] * P[3 * c + 1] + P[3 * c + 2] * P[3 * c + 2];
                    e = 0.5 * (U2[c] - p2 / N[c]);
                    if (e > 1e-3 * 0.5 * U2[c] && 2.0 * e / N[c] >= r->thr_sigma_u * r->thr_sigma_u) bits |= 1;
                }
                int node[3] = {i, j, k};
                double z0[3] = {0, 0, 0}, f[3];
                for (int d = 0; d < 3; ++d) f[d] = or_gather(s, OR_EX + d, node, z0);
                double emag = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
                if (NI[c] > 0) {
                    double ionr = 0.0;
                    for (int isp = 0; isp < s->nsp; ++isp)
                        if (s->sp[isp].kind == OR_ION && s->sp[isp].ionizable)
                            ionr = fmax(ionr, or_ion_rate_norm(s, isp, 0, emag) * g->dt);
                    if (ionr >= r->thr_ion) bits |= 2;
                }
                if (r->enable_qed && N[c] > 0 && sqrt(1.0 + U2[c] / N[c]) * emag / a_s >= r->thr_chi) bits |= 4;
                cond[v] = (uint8_t)bits;
                if (raw9) {
                    for (int q = 0; q < 8; ++q) raw9[9 * v + q] = raw[8 * v + q];
                    raw9[9 * v + 8] = e;
                }
            }
    free(N); free(P); free(U2); free(NI); free(V); free(raw);
}

/* Absorption part of the conversion (see the header comment). */
void or_absorb(or_sim *s) {
    const or_grid *g = &s->g;
    double dv = g->dx * g->dy * g->dz;
    for (int isp = 0; isp < s->nsp; ++isp) {
        const or_species *sp = &s->sp[isp];
        if (!sp->fluid || !s->fn[isp]) continue;
        or_parts *p = &s->p[isp];
        double *n = s->fn[isp];
        double *M = (double *)calloc(s->nn, sizeof(double));
        double *Pm = (double *)calloc(s->nn * 3, sizeof(double));
        double *KEa = (double *)calloc(s->nn, sizeof(double));   /* absorbed kinetic energy (warm) */
        double *S = s->fs[isp];
        const double ga = sp->gamma_ad;
        uint8_t *touched = (uint8_t *)calloc(s->nn, 1);
        /* absorb, in storage order */
        size_t keep = 0;
        for (size_t q = 0; q < p->n; ++q) {
            int rel[3];
            size_t c = nearest(s, p, q, rel);
            double uq[3] = {p->ux[q], p->uy[q], p->uz[q]};
            if (s->sw[c] || or_is_hot(s, uq)) {
                if (keep != q) {
                    p->ci[keep] = p->ci[q]; p->cj[keep] = p->cj[q]; p->ck[keep] = p->ck[q];
                    p->ox[keep] = p->ox[q]; p->oy[keep] = p->oy[q]; p->oz[keep] = p->oz[q];
                    p->ux[keep] = p->ux[q]; p->uy[keep] = p->uy[q]; p->uz[keep] = p->uz[q];
                    p->w[keep] = p->w[q]; p->tau[keep] = p->tau[q]; p->id[keep] = p->id[q];
                    p->zc[keep] = p->zc[q];
                }
                keep++;
                continue;
            }
            int cell[3] = {p->ci[q], p->cj[q], p->ck[q]};
            double X[3] = {p->ox[q], p->oy[q], p->oz[q]};
            double Xn[3] = {(double)rel[0], (double)rel[1], (double)rel[2]};
            or_deposit_move(s, sp->charge, p->w[q], cell, X, Xn);
            double u[3] = {p->ux[q], p->uy[q], p->uz[q]};
            double gam = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            if (S) KEa[c] += p->w[q] * sp->mass * (gam - 1.0);
            else s->conv_loss += p->w[q] * sp->mass * (gam - 1.0);
            M[c] += p->w[q];
            for (int d = 0; d < 3; ++d) Pm[3 * c + d] += p->w[q] * u[d];
            touched[c] = 1;
        }
        p->n = keep;
        for (size_t c = 0; c < s->nn; ++c) {
            if (!touched[c]) continue;
            double m0 = n[c] * dv;
            double u0[3] = {s->fu[isp][0][c], s->fu[isp][1][c], s->fu[isp][2][c]};
            double g0 = sqrt(1.0 + u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2]);
            double mt = m0 + M[c];
            double un[3];
            for (int d = 0; d < 3; ++d) un[d] = (m0 * u0[d] + Pm[3 * c + d]) / mt;
            double gn = sqrt(1.0 + un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
            double loss = m0 * sp->mass * (g0 - 1.0) - mt * sp->mass * (gn - 1.0);
            if (S) {
                /* the kinetic energy the merge loses becomes heat of the node;
                 * a node left without positive mass or pressure (its fluid
                 * density had gone negative) keeps no entropy, and that heat
                 * and its previous thermal energy go to the ledger */
                double pold = n[c] > 0.0 ? S[c] * pow(n[c], ga - 1.0) : 0.0;
                double pnew = pold + (ga - 1.0) * (KEa[c] + loss) / dv;
                if (mt > 0.0 && pnew >= 0.0) {
                    S[c] = pnew * pow(mt / dv, 1.0 - ga);
                } else {
                    S[c] = 0.0;
                    s->conv_loss += KEa[c] + loss + pold * dv / (ga - 1.0);
                }
            } else s->conv_loss += loss;
            n[c] = mt / dv;
            for (int d = 0; d < 3; ++d) s->fu[isp][d][c] = un[d];
        }
        free(M); free(Pm); free(KEa); free(touched);
    }
}

/* Spawning part of the conversion (see the header comment), after the fluid update. */
void or_spawn_fluid(or_sim *s) {
    const or_grid *g = &s->g;
    double dv = g->dx * g->dy * g->dz;
    int nxn = node_x_count(s);
    for (int isp = 0; isp < s->nsp; ++isp) {
        const or_species *sp = &s->sp[isp];
        if (!sp->fluid || !s->fn[isp]) continue;
        or_parts *p = &s->p[isp];
        double *n = s->fn[isp];
        double *S = s->fs[isp];
        const double ga = sp->gamma_ad;
        /* spawn, in node order */
        double w0 = sp->n0 * dv / (sp->ppc > 0 ? sp->ppc : 1);
        double wmin = s->run.spawn_frac * w0;
        for (int k = 0; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < nxn; ++i) {
                    size_t c = or_idx(s, i, j, k);
                    if (!s->sw[c] || n[c] <= 0.0) continue;
                    double mass = n[c] * dv;
                    if (mass < wmin) continue;
                    double mr = w0 > 0.0 ? floor(mass / w0 + 0.5) : 1.0;
                    int m = mr < 1.0 ? 1 : (mr > 64.0 ? 64 : (int)mr);
                    double w = mass / m;
                    double u[3] = {s->fu[isp][0][c], s->fu[isp][1][c], s->fu[isp][2][c]};
                    /* warm fluid: thermal spread sqrt(T / m) per component, T = p / n */
                    double sig = 0.0, before = 0.0, after = 0.0;
                    if (S) {
                        double pr = S[c] * pow(n[c], ga - 1.0);
                        sig = sqrt(fmax(pr / n[c], 0.0) / sp->mass);
                        before = mass * sp->mass * (sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) - 1.0) +
                                 pr * dv / (ga - 1.0);
                    }
                    uint64_t node = (uint64_t)i + (uint64_t)nxn * ((uint64_t)j + (uint64_t)g->ny * k);
                    for (int q = 0; q < m; ++q) {
                        uint32_t r[4];
                        or_draw4(s, node, (uint32_t)s->step, 12, (uint32_t)q, r);
                        /* move from the node to node + (r - 1/2) in each axis */
                        int cell[3] = {i, j, k};
                        double X0[3] = {0.0, 0.0, 0.0};
                        double X1[3] = {or_uniform(r[0]) - 0.5, or_uniform(r[1]) - 0.5,
                                        or_uniform(r[2]) - 0.5};
                        double uq[3] = {u[0], u[1], u[2]};
                        uint64_t id = (1ull << 63) | ((uint64_t)s->step << 40) | ((uint64_t)isp << 37) |
                                      (node << 6) | (uint64_t)q;
                        if (S) {
                            /* Box-Muller on Philox draws, tag 13 */
                            uint32_t t[4];
                            or_draw4(s, id, (uint32_t)s->step, 13, 0, t);
                            double r0 = or_uniform(t[0]), r1 = or_uniform(t[1]), r2 = or_uniform(t[2]),
                                   r3 = or_uniform(t[3]);
                            double m0 = sqrt(-2.0 * log(r0)), m1 = sqrt(-2.0 * log(r2));
                            const double tp = 6.283185307179586;
                            uq[0] += sig * m0 * cos(tp * r1);
                            uq[1] += sig * m0 * sin(tp * r1);
                            uq[2] += sig * m1 * cos(tp * r3);
                            after += w * sp->mass * (sqrt(1.0 + uq[0] * uq[0] + uq[1] * uq[1] + uq[2] * uq[2]) - 1.0);
                        }
                        double ux = uq[0];
                        or_reflect_x(s, i, &X1[0], &ux);
                        or_deposit_move(s, sp->charge, w, cell, X0, X1);
                        or_carry(s, cell, X1);
                        or_parts_push_back(p, cell[0], cell[1], cell[2], X1[0], X1[1], X1[2],
                                           uq[0], uq[1], uq[2], w, sp->qed ? or_qed_tau0(s, id) : 0.0, id,
                                           (int32_t)llround(sp->charge));
                    }
                    if (S) {
                        s->conv_loss += before - after;   /* the sample's energy differs from the fluid's */
                        S[c] = 0.0;
                    }
                    n[c] = 0.0;
                    s->fu[isp][0][c] = s->fu[isp][1][c] = s->fu[isp][2][c] = 0.0;
                }
    }
}
