/*
 * Oracle QED module: quantum-synchrotron photon emission by leptons and
 * Breit-Wheeler pair creation by photons, in the locally-constant-field
 * approximation with Airy-function rates, sampled by Monte Carlo with an
 * optical depth per particle.
 *
 * Paper: abstract and Methodology, plasma-model paragraph (QED photon
 * emission and pair creation with Airy-function approximations and local
 * field adjustments).  Literature: V. I. Ritus, J. Sov. Laser Res. 6 (1985)
 * 497 and V. N. Baier, V. M. Katkov, Sov. Phys. JETP 26 (1968) 854 for the
 * spectra; the optical-depth Monte Carlo follows Duclous, Kirk and Bell,
 * Plasma Phys. Control. Fusion 53 (2011) 015009.
 *
 * Normalized units (c = omega0 = m_e = e = 1).  a_s = m c^2 / (hbar omega0)
 * is the Schwinger field in these units (3.2972e5 at lambda = 0.8 um).
 *
 *   emission, lepton with gamma, momentum u, velocity v = u / gamma:
 *     chi_e = (gamma / a_s) sqrt(|E + v x B|^2 - (v.E)^2)
 *     dW/d(delta) = (alpha a_s / gamma) F_e(chi_e, delta),  delta = photon / lepton energy,
 *     F_e = -Int_z^inf Ai - (2/z + chi delta sqrt z) Ai'(z),  z = (delta / (chi (1 - delta)))^(2/3)
 *   pair creation, photon with energy eps = |k|, direction n = k / |k|:
 *     chi_g = (eps / a_s) sqrt(|E + n x B|^2 - (n.E)^2)
 *     dW/d(delta) = (alpha a_s / eps) F_b(chi_g, delta),  delta = electron / photon energy,
 *     F_b = Int_z^inf Ai + (2/z - chi sqrt z) Ai'(z),  z = (1 / (chi delta (1 - delta)))^(2/3)
 *
 * Airy functions for z >= 0 from the modified Bessel functions (zeta =
 * 2/3 z^(3/2)):  Ai = sqrt(z/3) K_{1/3}(zeta) / pi,  Ai' = -z K_{2/3}(zeta) / (pi sqrt 3),
 * Int_z^inf Ai = Int_zeta^inf K_{1/3} / (pi sqrt 3), with
 * K_nu(zeta) = Int_0^inf exp(-zeta cosh t) cosh(nu t) dt and
 * Int_zeta^inf K_nu = Int_0^inf exp(-zeta cosh t) cosh(nu t) / cosh t dt,
 * each by the trapezoidal rule (the integrands are smooth and decay
 * double-exponentially).
 *
 * Readings (the paper gives no numbers):
 *   tables over chi_i = 10^(-3 + 6 i / 255), i = 0..255, of
 *     W_e(chi) = Int_0^1 F_e d(delta),  W_b(chi) = Int_0^1 F_b d(delta)
 *   and of the inverse cumulative spectra at u_j = (j + 1/2) / 128, j = 0..127,
 *   stored in the variable x of delta = x^3 / (x^3 + (1 - x)^3), which keeps
 *   both ends of the spectra smooth; lookups interpolate linearly in
 *   (log10 chi, u), clamping chi to [1e-3, 1e3] and u to [u_0, u_127];
 *   no emission or pair creation below chi = 1e-3;
 *   per step: chi from the fields at x^n and u^{n-1/2}; tau -= W dt; if tau <= 0
 *   one event: emission takes k = delta u from the lepton (momentum exact), a new
 *   tau = -ln(1 - r) (Philox tag 17), and a photon with momentum k if |k| > 2,
 *   else the energy w |k| goes to the photon ledger; a photon that converts
 *   gives an electron and a positron along n with gamma = max(delta eps, 1) and
 *   max((1 - delta) eps, 1), the ledger takes w (eps - gamma_e - gamma_p + 2)
 *   (rest energy and the threshold residue); photons move ballistically and
 *   leave through open x walls into the ledger; new particles start to move in
 *   the step after their birth;
 *   a new QED particle has tau = -ln(1 - r), r from Philox (id, 2^32 - 1, 17, 0);
 *   child ids: splitmix64(parent ^ splitmix64((step << 8) | k)), k = 1 photon,
 *   2 electron, 3 positron (S. Vigna's splitmix64 finaliser).
 */
#include "or_internal.h"

#define OR_NCHI 256
#define OR_NU 128
#define OR_CHI_MIN 1e-3

typedef struct {
    double a_s;
    double We[OR_NCHI], Wb[OR_NCHI];
    double Xe[OR_NCHI][OR_NU], Xb[OR_NCHI][OR_NU];
    int photon_sp, electron_sp, positron_sp;
} or_qed;

/* ---------------------------------------------------------------- Airy */

/* Int_0^inf exp(-zeta cosh t) cosh(nu t) / cosh(t)^p dt, p = 0 or 1.  The step
 * resolves the peak at t = 0 (width 1/sqrt(zeta)) and the strip of
 * analyticity (|Im t| < pi/2); the sum stops where exp(-zeta cosh t) < e^-745. */
static double bessel_int(double zeta, double nu, int p) {
    double tmax = acosh(745.0 / zeta + 1.0);
    double h = 0.3 / sqrt(zeta + 1.0);
    if (h > 0.1) h = 0.1;
    int n = (int)ceil(tmax / h);
    double s = 0.5 * exp(-zeta);   /* t = 0 term, weight 1/2 */
    for (int k = 1; k <= n; ++k) {
        double t = k * h, c = cosh(t);
        double v = exp(-zeta * c) * cosh(nu * t);
        if (p) v /= c;
        s += v;
    }
    return s * h;
}

/* Ai(z), Ai'(z) and Int_z^inf Ai for z > 0. */
void or_airy(double z, double *ai, double *aip, double *iai) {
    double zeta = 2.0 / 3.0 * pow(z, 1.5);
    if (zeta > 700.0) { *ai = *aip = *iai = 0.0; return; }
    *ai = sqrt(z / 3.0) * bessel_int(zeta, 1.0 / 3.0, 0) / OR_PI;
    *aip = -z * bessel_int(zeta, 2.0 / 3.0, 0) / (OR_PI * sqrt(3.0));
    *iai = bessel_int(zeta, 1.0 / 3.0, 1) / (OR_PI * sqrt(3.0));
}

/* --------------------------------------------------------------- spectra */

static double delta_of_x(double x) {
    double a = x * x * x, b = (1.0 - x) * (1.0 - x) * (1.0 - x);
    return a / (a + b);
}
static double ddelta_dx(double x) {
    double a = x * x * x, b = (1.0 - x) * (1.0 - x) * (1.0 - x);
    return 3.0 * x * x * (1.0 - x) * (1.0 - x) / ((a + b) * (a + b));
}

double or_qed_emission_spectrum(double chi, double delta) {
    if (delta <= 0.0 || delta >= 1.0) return 0.0;
    double z = pow(delta / (chi * (1.0 - delta)), 2.0 / 3.0);
    double ai, aip, iai;
    or_airy(z, &ai, &aip, &iai);
    return -iai - (2.0 / z + chi * delta * sqrt(z)) * aip;
}

double or_qed_pair_spectrum(double chi, double delta) {
    if (delta <= 0.0 || delta >= 1.0) return 0.0;
    double z = pow(1.0 / (chi * delta * (1.0 - delta)), 2.0 / 3.0);
    double ai, aip, iai;
    or_airy(z, &ai, &aip, &iai);
    return iai + (2.0 / z - chi * sqrt(z)) * aip;
}

/* Integrand in x (the delta substitution) of kind 0 emission, 1 pairs, 2 emitted
 * energy (delta F_e).  At x = 0 the emission spectrum times d(delta)/dx tends to
 * -6 Ai'(0) chi^(2/3), with Ai'(0) = -1 / (3^(1/3) Gamma(1/3)). */
static double x_integrand(int kind, double chi, double x) {
    if (x <= 0.0) {
        if (kind != 0) return 0.0;
        return 6.0 / (cbrt(3.0) * tgamma(1.0 / 3.0)) * pow(chi, 2.0 / 3.0);
    }
    if (x >= 1.0) return 0.0;
    double d = delta_of_x(x), j = ddelta_dx(x);
    if (kind == 1) return or_qed_pair_spectrum(chi, d) * j;
    double f = or_qed_emission_spectrum(chi, d) * j;
    return kind == 2 ? d * f : f;
}

#define OR_NSIMP 4096   /* Simpson intervals over x in [0, 1] */

/* Total of the spectrum (kind 0 / 1) or the emitted energy fraction (kind 2):
 * composite Simpson over x. */
double or_qed_total(int kind, double chi) {
    const double h = 1.0 / OR_NSIMP;
    double s = x_integrand(kind, chi, 0.0) + x_integrand(kind, chi, 1.0);
    for (int k = 1; k < OR_NSIMP; ++k) s += (k & 1 ? 4.0 : 2.0) * x_integrand(kind, chi, k * h);
    return s * h / 3.0;
}

/* Cubic through (t_m, f_m), m = 0..3, as monomial coefficients in t
 * (Newton divided differences expanded). */
static void cubic_coeffs(const double t[4], const double f[4], double c[4]) {
    double d1[3], d2[2], d3;
    for (int m = 0; m < 3; ++m) d1[m] = (f[m + 1] - f[m]) / (t[m + 1] - t[m]);
    for (int m = 0; m < 2; ++m) d2[m] = (d1[m + 1] - d1[m]) / (t[m + 2] - t[m]);
    d3 = (d2[1] - d2[0]) / (t[3] - t[0]);
    /* p(t) = f0 + d1 (t-t0) + d2 (t-t0)(t-t1) + d3 (t-t0)(t-t1)(t-t2) */
    double a = t[0], b = t[1], e = t[2];
    c[0] = f[0] - d1[0] * a + d2[0] * a * b - d3 * a * b * e;
    c[1] = d1[0] - d2[0] * (a + b) + d3 * (a * b + a * e + b * e);
    c[2] = d2[0] - d3 * (a + b + e);
    c[3] = d3;
}
static double cubic_int(const double c[4], double t) {   /* Int_0^t p */
    return t * (c[0] + t * (c[1] / 2.0 + t * (c[2] / 3.0 + t * c[3] / 4.0)));
}
static double cubic_val(const double c[4], double t) {
    return c[0] + t * (c[1] + t * (c[2] + t * c[3]));
}

/* The cubic of interval [x_k, x_k+1] (in t = (x - x_k)/h) through the four
 * nearest nodes. */
static void interval_cubic(const double *f, int N, int k, double c[4]) {
    int m0 = k - 1;
    if (m0 < 0) m0 = 0;
    if (m0 > N - 3) m0 = N - 3;
    double t[4], v[4];
    for (int m = 0; m < 4; ++m) { t[m] = m0 + m - k; v[m] = f[m0 + m]; }
    cubic_coeffs(t, v, c);
}

/* Inverse cumulative spectrum: x with Int_0^x f = u Int_0^1 f, for the 128 u_j.
 * f is sampled once on the Simpson grid; the cumulative integral and its
 * inverse use the cubic through the four nodes nearest each interval. */
static void inverse_cdf(int kind, double chi, double out[OR_NU]) {
    const int N = OR_NSIMP;
    const double h = 1.0 / N;
    double *f = (double *)malloc(sizeof(double) * (N + 1));
    double *C = (double *)malloc(sizeof(double) * (N + 1));
    for (int k = 0; k <= N; ++k) f[k] = x_integrand(kind, chi, k * h);
    C[0] = 0.0;
    for (int k = 0; k < N; ++k) {
        double c[4];
        interval_cubic(f, N, k, c);
        C[k + 1] = C[k] + h * cubic_int(c, 1.0);
    }
    double tot = C[N];
    for (int j = 0; j < OR_NU; ++j) {
        double u = (j + 0.5) / OR_NU;
        if (!(tot > 0.0)) { out[j] = u; continue; }
        double target = u * tot;
        int k = 0;
        while (k < N - 1 && C[k + 1] < target) ++k;
        double c[4];
        interval_cubic(f, N, k, c);
        /* bisection then Newton on C[k] + h Int_0^t p = target, t in [0, 1] */
        double lo = 0.0, hi = 1.0;
        for (int it = 0; it < 30; ++it) {
            double mid = 0.5 * (lo + hi);
            if (C[k] + h * cubic_int(c, mid) < target) lo = mid; else hi = mid;
        }
        double t = 0.5 * (lo + hi);
        for (int it = 0; it < 4; ++it) {
            double pv = cubic_val(c, t);
            if (!(pv > 0.0)) break;
            double tn = t - (C[k] + h * cubic_int(c, t) - target) / (h * pv);
            if (tn < 0.0 || tn > 1.0) break;
            t = tn;
        }
        out[j] = (k + t) * h;
    }
    free(f);
    free(C);
}

void or_qed_build_tables(double *We, double *Wb, double *Xe, double *Xb) {
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < OR_NCHI; ++i) {
        double chi = pow(10.0, -3.0 + 6.0 * i / (OR_NCHI - 1));
        We[i] = or_qed_total(0, chi);
        Wb[i] = or_qed_total(1, chi);
        inverse_cdf(0, chi, Xe + (size_t)i * OR_NU);
        inverse_cdf(1, chi, Xb + (size_t)i * OR_NU);
    }
}

/* cached tables (they depend on nothing but the definitions) */
static double *g_tab = NULL;
static void tables(const double **We, const double **Wb, const double **Xe, const double **Xb) {
    if (!g_tab) {
        double *t = (double *)malloc(sizeof(double) * (2 * OR_NCHI + 2 * OR_NCHI * OR_NU));
        or_qed_build_tables(t, t + OR_NCHI, t + 2 * OR_NCHI, t + 2 * OR_NCHI + OR_NCHI * OR_NU);
        g_tab = t;
    }
    *We = g_tab; *Wb = g_tab + OR_NCHI;
    *Xe = g_tab + 2 * OR_NCHI; *Xb = g_tab + 2 * OR_NCHI + OR_NCHI * OR_NU;
}

/* table position of chi: index i0 and fraction f */
static void chi_pos(double chi, int *i0, double *f) {
    double x = (log10(chi) + 3.0) * (OR_NCHI - 1) / 6.0;
    if (x < 0.0) x = 0.0;
    if (x > OR_NCHI - 1) x = OR_NCHI - 1;
    int i = (int)floor(x);
    if (i > OR_NCHI - 2) i = OR_NCHI - 2;
    *i0 = i;
    *f = x - i;
}
static double lookup_w(const double *W, double chi) {
    int i; double f;
    chi_pos(chi, &i, &f);
    return (1.0 - f) * W[i] + f * W[i + 1];
}
static double lookup_delta(const double *X, double chi, double r) {
    int i; double f;
    chi_pos(chi, &i, &f);
    double y = r * OR_NU - 0.5;
    if (y < 0.0) y = 0.0;
    if (y > OR_NU - 1) y = OR_NU - 1;
    int j = (int)floor(y);
    if (j > OR_NU - 2) j = OR_NU - 2;
    double g = y - j;
    const double *a = X + (size_t)i * OR_NU, *b = X + (size_t)(i + 1) * OR_NU;
    double x = (1.0 - f) * ((1.0 - g) * a[j] + g * a[j + 1]) + f * ((1.0 - g) * b[j] + g * b[j + 1]);
    return delta_of_x(x);
}

/* ----------------------------------------------------------- Monte Carlo */

static uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
uint64_t or_child_id(uint64_t parent, uint32_t step, uint32_t k) {
    return splitmix64(parent ^ splitmix64(((uint64_t)step << 8) | k));
}

double or_qed_tau0(const or_sim *s, uint64_t id) {
    uint32_t r[4];
    or_draw4(s, id, 0xffffffffu, 17, 0, r);
    return -log(1.0 - or_uniform(r[0]));
}

double or_schwinger_field(double lambda_um) {
    double omega0 = 2.0 * OR_PI * OR_C / (lambda_um * 1e-6);
    return OR_ME * OR_C * OR_C / (OR_HBAR * omega0);
}

void or_qed_init(or_sim *s) {
    if (!s->run.enable_qed || s->qed) return;
    or_qed *q = (or_qed *)calloc(1, sizeof(or_qed));
    q->a_s = or_schwinger_field(s->las.lambda_um);
    const double *We, *Wb, *Xe, *Xb;
    tables(&We, &Wb, &Xe, &Xb);
    memcpy(q->We, We, sizeof(q->We));
    memcpy(q->Wb, Wb, sizeof(q->Wb));
    memcpy(q->Xe, Xe, sizeof(q->Xe));
    memcpy(q->Xb, Xb, sizeof(q->Xb));
    q->photon_sp = q->electron_sp = q->positron_sp = -1;
    /* emitted photons and pairs go to the first species of each kind */
    for (int i = s->nsp - 1; i >= 0; --i) {
        if (s->sp[i].kind == OR_PHOTON) q->photon_sp = i;
        if (s->sp[i].kind == OR_ELECTRON) q->electron_sp = i;
        if (s->sp[i].kind == OR_POSITRON) q->positron_sp = i;
    }
    s->qed = q;
}

void or_qed_free(or_sim *s) {
    free(s->qed);
    s->qed = NULL;
}

/* chi of a lepton (u) or photon (k, photon = 1) in fields e, b */
double or_qed_chi(double a_s, const double e[3], const double b[3], const double u[3], int photon) {
    double p = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    double en = photon ? p : sqrt(1.0 + p * p);
    if (!(p > 0.0)) return 0.0;
    double v[3] = {u[0] / en, u[1] / en, u[2] / en};   /* velocity (unit vector for photons) */
    double f[3] = {e[0] + v[1] * b[2] - v[2] * b[1], e[1] + v[2] * b[0] - v[0] * b[2],
                   e[2] + v[0] * b[1] - v[1] * b[0]};
    double ve = v[0] * e[0] + v[1] * e[1] + v[2] * e[2];
    double q2 = f[0] * f[0] + f[1] * f[1] + f[2] * f[2] - ve * ve;
    return en / a_s * sqrt(q2 > 0.0 ? q2 : 0.0);
}

void or_qed_emit(or_sim *s, int isp, size_t i, const double e[3], const double b[3]) {
    or_qed *q = (or_qed *)s->qed;
    if (!q) return;
    or_parts *p = &s->p[isp];
    double u[3] = {p->ux[i], p->uy[i], p->uz[i]};
    double chi = or_qed_chi(q->a_s, e, b, u, 0);
    if (!(chi > OR_CHI_MIN)) return;
    double gam = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    double W = OR_ALPHA * q->a_s / gam * lookup_w(q->We, chi);
    p->tau[i] -= W * s->g.dt;
    if (p->tau[i] > 0.0) return;
    uint32_t r[4];
    or_draw4(s, p->id[i], (uint32_t)s->step, 16, 0, r);
    double delta = lookup_delta(&q->Xe[0][0], chi, or_uniform(r[0]));
    double k[3] = {delta * u[0], delta * u[1], delta * u[2]};
    p->ux[i] = u[0] - k[0]; p->uy[i] = u[1] - k[1]; p->uz[i] = u[2] - k[2];
    or_draw4(s, p->id[i], (uint32_t)s->step, 17, 0, r);
    p->tau[i] = -log(1.0 - or_uniform(r[0]));
    double kk = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    if (kk > 2.0 && q->photon_sp >= 0) {
        or_spawn ev;
        ev.species = q->photon_sp;
        ev.ci = p->ci[i]; ev.cj = p->cj[i]; ev.ck = p->ck[i];
        ev.ox = p->ox[i]; ev.oy = p->oy[i]; ev.oz = p->oz[i];
        ev.ux = k[0]; ev.uy = k[1]; ev.uz = k[2];
        ev.w = p->w[i];
        ev.id = or_child_id(p->id[i], (uint32_t)s->step, 1);
        ev.tau = or_qed_tau0(s, ev.id);
        ev.zc = 0;
        or_spawn_add(s, &ev);
    } else {
        s->photon_ledger += p->w[i] * kk;
    }
}

/* Photons: gather at x^n, pair creation, ballistic move at c; photons that
 * leave through an open x wall go to the ledger. */
void or_photon_phase(or_sim *s) {
    or_qed *q = (or_qed *)s->qed;
    if (!q) return;
    const or_grid *g = &s->g;
    double dxs[3] = {g->dx, g->dy, g->dz};
    for (int isp = 0; isp < s->nsp; ++isp) {
        if (s->sp[isp].kind != OR_PHOTON) continue;
        or_parts *p = &s->p[isp];
        size_t n = 0;
        while (n < p->n) {
            int c[3] = {p->ci[n], p->cj[n], p->ck[n]};
            double X0[3] = {p->ox[n], p->oy[n], p->oz[n]};
            double k[3] = {p->ux[n], p->uy[n], p->uz[n]};
            double eps = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
            double e[3], b[3];
            for (int d = 0; d < 3; ++d) {
                e[d] = or_gather(s, OR_EX + d, c, X0);
                b[d] = or_gather(s, OR_BX + d, c, X0);
            }
            double chi = or_qed_chi(q->a_s, e, b, k, 1);
            if (chi > OR_CHI_MIN && s->sp[isp].qed) {
                double W = OR_ALPHA * q->a_s / eps * lookup_w(q->Wb, chi);
                p->tau[n] -= W * g->dt;
                if (p->tau[n] <= 0.0) {
                    uint32_t r[4];
                    or_draw4(s, p->id[n], (uint32_t)s->step, 18, 0, r);
                    double delta = lookup_delta(&q->Xb[0][0], chi, or_uniform(r[0]));
                    double ge = fmax(delta * eps, 1.0), gp = fmax((1.0 - delta) * eps, 1.0);
                    double nk[3] = {k[0] / eps, k[1] / eps, k[2] / eps};
                    double ue = sqrt(ge * ge - 1.0), up = sqrt(gp * gp - 1.0);
                    int made = 0;
                    for (int which = 0; which < 2; ++which) {
                        int tsp = which == 0 ? q->electron_sp : q->positron_sp;
                        if (tsp < 0) continue;
                        double m = which == 0 ? ue : up;
                        or_spawn ev;
                        ev.species = tsp;
                        ev.ci = c[0]; ev.cj = c[1]; ev.ck = c[2];
                        ev.ox = X0[0]; ev.oy = X0[1]; ev.oz = X0[2];
                        ev.ux = m * nk[0]; ev.uy = m * nk[1]; ev.uz = m * nk[2];
                        ev.w = p->w[n];
                        ev.id = or_child_id(p->id[n], (uint32_t)s->step, 2 + which);
                        ev.tau = or_qed_tau0(s, ev.id);
                        ev.zc = which == 0 ? -1 : 1;
                        or_spawn_add(s, &ev);
                        made++;
                    }
                    if (made == 2) s->photon_ledger += p->w[n] * (eps - ge - gp + 2.0);
                    else s->photon_ledger += p->w[n] * eps;   /* no lepton species to hold the pair */
                    or_parts_remove(p, n);
                    continue;
                }
            }
            double X1[3];
            for (int d = 0; d < 3; ++d) X1[d] = X0[d] + g->dt * k[d] / eps / dxs[d];
            int out = 0;
            if (g->bc_x == OR_BC_OPEN) {
                if (c[0] == 0 && X1[0] < 0.0) out = 1;
                if (c[0] == g->nx - 1 && X1[0] >= 1.0) out = 1;
            }
            if (out) {
                s->photon_ledger += p->w[n] * eps;
                or_parts_remove(p, n);
                continue;
            }
            or_carry(s, c, X1);
            p->ci[n] = c[0]; p->cj[n] = c[1]; p->ck[n] = c[2];
            p->ox[n] = X1[0]; p->oy[n] = X1[1]; p->oz[n] = X1[2];
            ++n;
        }
    }
}

/* What the next step's QED decides for species isp (leptons: emission,
 * photons: pair creation), per particle i in the oracle's order: its optical
 * depth tau[i] and the decrement dtau[i] = W dt at the fields the push
 * gathers (0 below chi_min); the event fires when tau - dtau <= 0.  Test
 * infrastructure, as or_ion_probe. */
void or_qed_probe(or_sim *s, int isp, double *tau, double *dtau) {
    or_qed *q = (or_qed *)s->qed;
    const or_parts *p = &s->p[isp];
    int photon = s->sp[isp].kind == OR_PHOTON;
    for (size_t i = 0; i < p->n; ++i) {
        tau[i] = p->tau[i];
        dtau[i] = 0.0;
        if (!q) continue;
        int c[3] = {p->ci[i], p->cj[i], p->ck[i]};
        double X0[3] = {p->ox[i], p->oy[i], p->oz[i]}, e[3], b[3];
        for (int d = 0; d < 3; ++d) {
            e[d] = or_gather(s, OR_EX + d, c, X0);
            b[d] = or_gather(s, OR_BX + d, c, X0);
        }
        double u[3] = {p->ux[i], p->uy[i], p->uz[i]};
        double chi = or_qed_chi(q->a_s, e, b, u, photon);
        if (!(chi > OR_CHI_MIN)) continue;
        double pm = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        double en = photon ? pm : sqrt(1.0 + pm * pm);
        dtau[i] = OR_ALPHA * q->a_s / en * lookup_w(photon ? q->Wb : q->We, chi) * s->g.dt;
    }
}
