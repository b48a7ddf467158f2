/*
 * Oracle cold relativistic fluid (one fluid per fluid-capable species).
 *
 * Paper: Methodology, plasma-model paragraph (continuity, momentum and
 * energy equations with relativistic gamma and adiabatic pressure for the
 * bulk plasma).  A species with gamma_ad = 0 is a cold fluid (density n and
 * momentum u = gamma v); with gamma_ad > 0 it is warm: it also carries the
 * entropy density S = n K, K = p / n^gamma_ad, constant along the flow of an
 * adiabatic fluid, so the energy equation becomes the advection of S.
 *
 * Discretisation (node-centred n, u; fluxes on the faces where J lives):
 *  1. us = Boris(u^{n-1/2}; E^n, B^n interpolated to the node);
 *  2. v = us / gamma(us);
 *  3. face velocity = mean of the two nodes, or the velocity of the only side
 *     above the density floor; donor-cell mass flux F = v_f n_donor and
 *     momentum flux G = F us_donor;
 *  4. n^{n+1} = n - dt div F, (n u)^{n+1/2} = n us - dt div G;
 *  5. J^{n+1/2} += q F on the faces, which makes the fluid charge obey the
 *     same discrete continuity equation as the Esirkepov particle current.
 * Warm fluid, in addition:
 *  1b. after the Boris step, at nodes above the density floor,
 *      us -= dt grad p / (m n), p = S n^(gamma_ad - 1) at the nodes (zero
 *      where n = 0), central differences (one-sided at the open x walls); the
 *      pressure force is taken non-relativistically (modest temperatures);
 *  3b. entropy flux H = F K_donor, K = S / n;
 *  4b. S^{n+1} = max(S - dt div H, 0).  The face velocity is the mean of two
 *      nodes, so a node can lose more than it holds in one step (its density
 *      may then go negative, which every reader of n treats as no fluid);
 *      the entropy density is kept non-negative so that p and the
 *      temperature p / n never turn negative where n stays positive.
 */
#include "or_internal.h"

void or_fluid_phase(or_sim *s) {
    const or_grid *g = &s->g;
    int per = g->bc_x == OR_BC_PERIODIC;
    double floor_n = s->run.n_floor;
    double dxs[3] = {g->dx, g->dy, g->dz};
    int nmax[3] = {per ? g->nx : g->nx + 1, g->ny, g->nz};
    for (int isp = 0; isp < s->nsp; ++isp) {
        if (!s->fn[isp]) continue;
        const or_species *sp = &s->sp[isp];
        double qm = sp->charge / sp->mass;
        double *n = s->fn[isp];
        size_t nn = s->nn;
        double *us = (double *)calloc(nn * 3, sizeof(double));  /* us */
        double *v = (double *)calloc(nn * 3, sizeof(double));
        /* 1-2: Lorentz force at every node holding fluid. */
        for (int k = 0; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < nmax[0]; ++i) {
                    size_t c = or_idx(s, i, j, k);
                    if (n[c] <= 0.0) continue;
                    double e[3], b[3], u[3];
                    int nc[3] = {i, j, k};
                    double z0[3] = {0, 0, 0};
                    for (int d = 0; d < 3; ++d) {
                        e[d] = or_gather(s, OR_EX + d, nc, z0);
                        b[d] = or_gather(s, OR_BX + d, nc, z0);
                        u[d] = s->fu[isp][d][c];
                    }
                    or_boris(qm, g->dt, e, b, u);
                    double gam = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                    for (int d = 0; d < 3; ++d) {
                        us[3 * c + d] = u[d];
                        v[3 * c + d] = u[d] / gam;
                    }
                }
        /* 1b: pressure force of a warm fluid. */
        double *S = s->fs[isp];
        const double ga = sp->gamma_ad;
        if (S) {
            double *pr = (double *)calloc(nn, sizeof(double));
            for (size_t c = 0; c < nn; ++c) pr[c] = n[c] > 0.0 ? S[c] * pow(n[c], ga - 1.0) : 0.0;
            for (int k = 0; k < g->nz; ++k)
                for (int j = 0; j < g->ny; ++j)
                    for (int i = 0; i < nmax[0]; ++i) {
                        size_t c = or_idx(s, i, j, k);
                        if (!(n[c] > floor_n) || !(n[c] > 0.0)) continue;
                        double grad[3];
                        /* x */
                        if (per) grad[0] = (pr[or_idx(s, or_wrap(i + 1, g->nx), j, k)] -
                                            pr[or_idx(s, or_wrap(i - 1, g->nx), j, k)]) / (2.0 * dxs[0]);
                        else if (i == 0) grad[0] = (pr[or_idx(s, 1, j, k)] - pr[c]) / dxs[0];
                        else if (i == g->nx) grad[0] = (pr[c] - pr[or_idx(s, i - 1, j, k)]) / dxs[0];
                        else grad[0] = (pr[or_idx(s, i + 1, j, k)] - pr[or_idx(s, i - 1, j, k)]) / (2.0 * dxs[0]);
                        grad[1] = (pr[or_idx(s, i, or_wrap(j + 1, g->ny), k)] -
                                   pr[or_idx(s, i, or_wrap(j - 1, g->ny), k)]) / (2.0 * dxs[1]);
                        grad[2] = (pr[or_idx(s, i, j, or_wrap(k + 1, g->nz))] -
                                   pr[or_idx(s, i, j, or_wrap(k - 1, g->nz))]) / (2.0 * dxs[2]);
                        for (int d = 0; d < 3; ++d) us[3 * c + d] -= g->dt * grad[d] / (sp->mass * n[c]);
                        double gam = sqrt(1.0 + us[3 * c] * us[3 * c] + us[3 * c + 1] * us[3 * c + 1] +
                                          us[3 * c + 2] * us[3 * c + 2]);
                        for (int d = 0; d < 3; ++d) v[3 * c + d] = us[3 * c + d] / gam;
                    }
            free(pr);
        }
        /* 3: fluxes on the faces between node c and its +d neighbour. */
        double *F = (double *)calloc(nn * 3, sizeof(double));
        double *G = (double *)calloc(nn * 9, sizeof(double));
        double *Hs = (double *)calloc(nn * 3, sizeof(double));   /* entropy flux (warm) */
        for (int k = 0; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < nmax[0]; ++i) {
                    size_t c = or_idx(s, i, j, k);
                    for (int d = 0; d < 3; ++d) {
                        int ii = i, jj = j, kk = k;
                        if (d == 0) {
                            if (!per && i == g->nx) continue;   /* no face beyond the wall */
                            ii = per ? or_wrap(i + 1, g->nx) : i + 1;
                        } else if (d == 1) jj = or_wrap(j + 1, g->ny);
                        else kk = or_wrap(k + 1, g->nz);
                        size_t r = or_idx(s, ii, jj, kk);
                        double nl = n[c], nr = n[r];
                        int lok = nl > floor_n, rok = nr > floor_n;
                        double vf;
                        if (!lok && !rok) vf = 0.0;
                        else if (!lok) vf = v[3 * r + d];
                        else if (!rok) vf = v[3 * c + d];
                        else vf = 0.5 * (v[3 * c + d] + v[3 * r + d]);
                        size_t don = vf > 0.0 ? c : r;
                        double flux = vf * n[don];
                        F[3 * c + d] = flux;
                        for (int m = 0; m < 3; ++m) G[9 * c + 3 * d + m] = flux * us[3 * don + m];
                        if (S) Hs[3 * c + d] = n[don] > 0.0 ? flux * (S[don] / n[don]) : 0.0;
                    }
                }
        /* 4: conservative update. */
        double *nnew = (double *)calloc(nn, sizeof(double));
        double *Snew = S ? (double *)calloc(nn, sizeof(double)) : NULL;
        for (int k = 0; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < nmax[0]; ++i) {
                    size_t c = or_idx(s, i, j, k);
                    double dn = 0.0, dm[3] = {0, 0, 0}, ds = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        int ii = i, jj = j, kk = k;
                        int has_minus = 1;
                        if (d == 0) {
                            if (!per && i == 0) has_minus = 0;
                            ii = per ? or_wrap(i - 1, g->nx) : i - 1;
                        } else if (d == 1) jj = or_wrap(j - 1, g->ny);
                        else kk = or_wrap(k - 1, g->nz);
                        double fplus = (d == 0 && !per && i == g->nx) ? 0.0 : F[3 * c + d];
                        double fminus = has_minus ? F[3 * or_idx(s, ii, jj, kk) + d] : 0.0;
                        dn += (fplus - fminus) / dxs[d];
                        if (S) {
                            double hp = (d == 0 && !per && i == g->nx) ? 0.0 : Hs[3 * c + d];
                            double hm = has_minus ? Hs[3 * or_idx(s, ii, jj, kk) + d] : 0.0;
                            ds += (hp - hm) / dxs[d];
                        }
                        for (int m = 0; m < 3; ++m) {
                            double gp = (d == 0 && !per && i == g->nx) ? 0.0 : G[9 * c + 3 * d + m];
                            double gm = has_minus ? G[9 * or_idx(s, ii, jj, kk) + 3 * d + m] : 0.0;
                            dm[m] += (gp - gm) / dxs[d];
                        }
                    }
                    double nv = n[c] - g->dt * dn;
                    nnew[c] = nv;
                    if (S) Snew[c] = fmax(S[c] - g->dt * ds, 0.0);
                    for (int m = 0; m < 3; ++m) {
                        double mom = n[c] * us[3 * c + m] - g->dt * dm[m];
                        s->fu[isp][m][c] = nv > floor_n ? mom / nv : 0.0;
                    }
                }
        memcpy(n, nnew, sizeof(double) * nn);
        if (S) memcpy(S, Snew, sizeof(double) * nn);
        /* 5: fluid current on the J faces. */
        for (int k = 0; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < nmax[0]; ++i) {
                    size_t c = or_idx(s, i, j, k);
                    for (int d = 0; d < 3; ++d) {
                        if (d == 0 && !per && i == g->nx) continue;
                        s->f[OR_JX + d][c] += sp->charge * F[3 * c + d];
                    }
                }
        free(us); free(v); free(F); free(G); free(Hs); free(nnew); free(Snew);
    }
}
