/*
 * Oracle field ionization: ADK tunnelling rate blended with a multiphoton
 * rate by a sigmoid in the Keldysh parameter, Monte Carlo per ion and level.
 *
 * Paper: abstract and Methodology, plasma-model paragraph (ADK tunnelling and
 * multiphoton rates joined by a sigmoid transition at Keldysh parameter about
 * 1.5).  Literature: Ammosov, Delone, Krainov, Sov. Phys. JETP 64 (1986) 1191
 * (static rate, m = 0, l* = n* - 1); Keldysh, Sov. Phys. JETP 20 (1965) 1307.
 *
 * Readings (the paper gives no formula):
 *   w_ADK(F) = 2^{2n*} / (n* Gamma(2n*)) * Ip * (2 (2Ip)^{3/2} / F)^{2n*-1}
 *              * exp(-2 (2Ip)^{3/2} / (3F)),   n* = Z / sqrt(2 Ip), atomic units;
 *   multiphoton continuation below the crossover field F_c (where the Keldysh
 *   parameter omega sqrt(2 Ip) / F equals 1.5):
 *              w_MPI(F) = w_ADK(F_c) (min(F, F_c) / F_c)^{2K},  K = ceil(Ip / omega);
 *   blend      w = s w_MPI + (1 - s) w_ADK,  s = 1 / (1 + exp(-(gamma_K - 1.5) / 0.1));
 *   step probability P = 1 - exp(-w dt); successive levels are tried in one
 *   step while each draw succeeds (Philox tag 3 + level).
 *   The laser wavelength lambda_um sets the SI scale of the normalized units.
 */
#include "or_internal.h"

double or_lambda_field_unit(double lambda_um) {
    double omega0 = 2.0 * OR_PI * OR_C / (lambda_um * 1e-6);
    return OR_ME * OR_C * omega0 / OR_QE;      /* V/m per normalized field unit */
}

double or_lambda_omega_au(double lambda_um) {
    double omega0 = 2.0 * OR_PI * OR_C / (lambda_um * 1e-6);
    return omega0 * OR_TA;                     /* photon energy in Hartree */
}

double or_adk_rate(double F, double ip, double zres) {
    if (F <= 0.0) return 0.0;
    double ns = zres / sqrt(2.0 * ip);
    double k3 = pow(2.0 * ip, 1.5);
    double c2 = pow(2.0, 2.0 * ns) / (ns * tgamma(2.0 * ns));
    return c2 * ip * pow(2.0 * k3 / F, 2.0 * ns - 1.0) * exp(-2.0 * k3 / (3.0 * F));
}

double or_ionization_rate(double F, double ip, double zres, double omega) {
    if (F <= 0.0) return 0.0;
    double gk = omega * sqrt(2.0 * ip) / F;
    double fc = omega * sqrt(2.0 * ip) / 1.5;
    double K = ceil(ip / omega);
    double sig = 1.0 / (1.0 + exp(-(gk - 1.5) / 0.1));
    double wmpi = or_adk_rate(fc, ip, zres) * pow(fmin(F, fc) / fc, 2.0 * K);
    return sig * wmpi + (1.0 - sig) * or_adk_rate(F, ip, zres);
}

/* Rate of level `level` of species sp at normalized field emag, per 1/omega0. */
double or_ion_rate_norm(const or_sim *s, int sp, int level, double emag) {
    double eu = or_lambda_field_unit(s->las.lambda_um);
    double om = or_lambda_omega_au(s->las.lambda_um);
    double F = emag * eu / OR_EA;
    double ip = s->sp[sp].ip_ev[level] / OR_HARTREE_EV;
    double w_au = or_ionization_rate(F, ip, (double)(level + 1), om);
    return w_au / om;   /* 1/t_a -> 1/(1/omega0): multiply by 1/(omega0 t_a) */
}

void or_ionize_particle(or_sim *s, int isp, size_t i, double emag) {
    const or_species *sp = &s->sp[isp];
    or_parts *p = &s->p[isp];
    double dt = s->g.dt;
    for (int lev = p->zc[i]; lev < sp->z_max; ++lev) {
        double w = or_ion_rate_norm(s, isp, lev, emag);
        double P = -expm1(-w * dt);
        uint32_t r[4];
        or_draw4(s, p->id[i], (uint32_t)s->step, 3 + (uint32_t)lev, 0, r);
        if (!(or_uniform(r[0]) < P)) break;
        p->zc[i] = lev + 1;
        or_spawn e;
        e.species = sp->target;
        e.ci = p->ci[i]; e.cj = p->cj[i]; e.ck = p->ck[i];
        e.ox = p->ox[i]; e.oy = p->oy[i]; e.oz = p->oz[i];
        e.ux = p->ux[i]; e.uy = p->uy[i]; e.uz = p->uz[i];
        e.w = p->w[i];
        e.id = (1ull << 62) | ((uint64_t)lev << 56) | p->id[i];
        e.tau = s->sp[sp->target].qed ? or_qed_tau0(s, e.id) : 0.0;
        e.zc = -1;
        or_spawn_add(s, &e);
        s->ion_energy += p->w[i] * sp->ip_ev[lev] / 510998.95;   /* m_e c^2 units */
    }
}

/* What the next step's ionization of ion species isp decides, per particle i
 * (the oracle's order) and level l < z_max: the probability P[i z_max + l] of
 * the transition l -> l + 1 in that step at the field the push gathers and
 * the uniform draw r[i z_max + l] it compares with (event when r < P); both 0
 * for levels below the particle's charge.  Test infrastructure: it lets a
 * comparison check that an event decided differently elsewhere lay within
 * rounding of its threshold. */
void or_ion_probe(or_sim *s, int isp, double *P, double *r) {
    const or_species *sp = &s->sp[isp];
    const or_parts *p = &s->p[isp];
    int zm = sp->z_max;
    for (size_t i = 0; i < p->n; ++i) {
        int c[3] = {p->ci[i], p->cj[i], p->ck[i]};
        double X0[3] = {p->ox[i], p->oy[i], p->oz[i]}, e[3];
        for (int d = 0; d < 3; ++d) e[d] = or_gather(s, OR_EX + d, c, X0);
        double emag = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        for (int l = 0; l < zm; ++l) {
            P[i * zm + l] = 0.0;
            r[i * zm + l] = 0.0;
            if (l < p->zc[i]) continue;
            uint32_t q[4];
            or_draw4(s, p->id[i], (uint32_t)s->step, 3 + (uint32_t)l, 0, q);
            P[i * zm + l] = -expm1(-or_ion_rate_norm(s, isp, l, emag) * s->g.dt);
            r[i * zm + l] = or_uniform(q[0]);
        }
    }
}
