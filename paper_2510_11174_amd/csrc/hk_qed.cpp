// Rate and spectrum tables of the QED Monte Carlo, built once on the host in
// FP64 and copied to the device.
//
// Paper: abstract and Methodology, plasma-model paragraph (photon emission
// and pair creation with Airy-function approximations).  Spectra in the
// locally-constant-field approximation (Ritus 1985; Baier and Katkov 1968):
//   emission: F_e(chi, d) = -Int_z^inf Ai - (2/z + chi d sqrt z) Ai'(z),
//             z = (d / (chi (1 - d)))^(2/3), d = photon / lepton energy;
//   pairs:    F_b(chi, d) = Int_z^inf Ai + (2/z - chi sqrt z) Ai'(z),
//             z = (1 / (chi d (1 - d)))^(2/3), d = electron / photon energy.
// Tables: chi_i = 10^(-3 + 6 i / 255), i < 256; W(chi) = Int_0^1 F d(d); the
// inverse cumulative spectrum at u_j = (j + 1/2) / 128, j < 128, stored as x
// with d = x^3 / (x^3 + (1 - x)^3) (smooth at both ends of the spectrum).
//
// Airy functions on z >= 0: the Airy equation y'' = z y integrated backwards
// (RK4, step 1/4096) from z0 = 12, where the asymptotic expansions
// (Abramowitz and Stegun 10.4.59 and 10.4.61) start it; along the way
// F(z) = Int_z^inf Ai obeys F' = -Ai.  Backwards, Ai is the growing solution,
// so the integration is stable.  Values between grid points come from cubic
// Hermite interpolation (y'' = z y gives the slope of Ai').  On [z0, 120] the
// expansions, and F by Gauss-Legendre quadrature of them, are tabulated once
// scaled by exp(2/3 z^(3/2)) (smooth there) and interpolated the same way;
// beyond 120 the functions underflow and are taken as zero.
// Integrals over x use 1024 Gauss-Legendre panels of 8 points.
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

namespace {

constexpr int NCHI = 256, NU = 128;
constexpr double Z0 = 12.0;
constexpr int NZ = 12 * 4096;   // grid steps on [0, Z0]
constexpr double HZ = Z0 / NZ;
constexpr double PI_ = 3.14159265358979323846;

// asymptotic Ai and Ai' for z >= Z0 (A&S 10.4.59, 10.4.61)
void airy_asym(double z, double &ai, double &aip) {
    const double zeta = 2.0 / 3.0 * z * std::sqrt(z);
    double su = 1.0, sv = 1.0, u = 1.0, p = 1.0;
    for (int k = 1; k < 40; ++k) {
        u *= (6.0 * k - 5.0) * (6.0 * k - 3.0) * (6.0 * k - 1.0) / ((2.0 * k - 1.0) * 216.0 * k);
        const double v = -(6.0 * k + 1.0) / (6.0 * k - 1.0) * u;
        p *= -1.0 / zeta;
        su += u * p;
        sv += v * p;
        if (std::fabs(u * p) < 1e-18 && std::fabs(v * p) < 1e-18) break;
    }
    // scaled by exp(zeta): the caller multiplies by exp(-zeta)
    const double e = 1.0 / (2.0 * std::sqrt(PI_));
    ai = e / std::pow(z, 0.25) * su;
    aip = -e * std::pow(z, 0.25) * sv;
}

constexpr double ZT = 120.0;         // end of the scaled tail table
constexpr int NT = (int)((ZT - Z0) * 64);
constexpr double HT = (ZT - Z0) / NT;

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n)
void gauss_legendre(int n, double *x, double *w) {
    for (int i = 0; i < n; ++i) {
        double t = std::cos(PI_ * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double dp = n * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        double p0 = 1.0, p1 = t;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        double dp = n * (t * p1 - p0) / (t * t - 1.0);
        x[i] = t;
        w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

struct Airy {
    std::vector<double> A, Ap, F;   // Ai, Ai', Int_z^inf Ai on the grid z_k = k HZ
    double glx[32], glw[32];

    std::vector<double> TA, TAp, TF;   // on [Z0, ZT], scaled by exp(zeta(z))

    // exp(zeta(z)) Int_z^inf Ai from the expansion, z >= Z0
    double tail_integral(double z) const {
        const double len = 40.0 / std::sqrt(z), zz = 2.0 / 3.0 * z * std::sqrt(z);
        const int panels = 4;
        double s = 0.0;
        for (int p = 0; p < panels; ++p) {
            const double a = z + len * p / panels, b = z + len * (p + 1) / panels;
            for (int q = 0; q < 32; ++q) {
                double t = 0.5 * (a + b) + 0.5 * (b - a) * glx[q], ai, aip;
                airy_asym(t, ai, aip);
                s += 0.5 * (b - a) * glw[q] * ai * std::exp(zz - 2.0 / 3.0 * t * std::sqrt(t));
            }
        }
        return s;
    }

    Airy() : A(NZ + 1), Ap(NZ + 1), F(NZ + 1), TA(NT + 1), TAp(NT + 1), TF(NT + 1) {
        gauss_legendre(32, glx, glw);
        for (int k = 0; k <= NT; ++k) {
            const double z = Z0 + k * HT;
            airy_asym(z, TA[k], TAp[k]);
            TF[k] = tail_integral(z);
        }
        const double e0 = std::exp(-2.0 / 3.0 * Z0 * std::sqrt(Z0));
        double y = TA[0] * e0, yp = TAp[0] * e0, f = TF[0] * e0;
        A[NZ] = y; Ap[NZ] = yp; F[NZ] = f;
        // state (y, y', F) with d/dz = (y', z y, -y), stepped by -HZ
        for (int k = NZ; k > 0; --k) {
            const double z = k * HZ, h = -HZ;
            auto der = [](double zz, const double s[3], double d[3]) {
                d[0] = s[1]; d[1] = zz * s[0]; d[2] = -s[0];
            };
            double s0[3] = {y, yp, f}, k1[3], k2[3], k3[3], k4[3], s1[3];
            der(z, s0, k1);
            for (int m = 0; m < 3; ++m) s1[m] = s0[m] + 0.5 * h * k1[m];
            der(z + 0.5 * h, s1, k2);
            for (int m = 0; m < 3; ++m) s1[m] = s0[m] + 0.5 * h * k2[m];
            der(z + 0.5 * h, s1, k3);
            for (int m = 0; m < 3; ++m) s1[m] = s0[m] + h * k3[m];
            der(z + h, s1, k4);
            for (int m = 0; m < 3; ++m) s0[m] += h / 6.0 * (k1[m] + 2.0 * k2[m] + 2.0 * k3[m] + k4[m]);
            y = s0[0]; yp = s0[1]; f = s0[2];
            A[k - 1] = y; Ap[k - 1] = yp; F[k - 1] = f;
        }
    }

    // cubic Hermite on [z_k, z_k+1] from values and slopes
    static double hermite(double t, double h, double y0, double y1, double d0, double d1) {
        const double t2 = t * t, t3 = t2 * t;
        return (2 * t3 - 3 * t2 + 1) * y0 + (t3 - 2 * t2 + t) * h * d0 + (-2 * t3 + 3 * t2) * y1 +
               (t3 - t2) * h * d1;
    }

    void eval(double z, double &ai, double &aip, double &iai) const {
        if (z >= ZT) { ai = aip = iai = 0.0; return; }
        if (z >= Z0) {
            // scaled values g = f exp(zeta): g' = f' exp(zeta) + sqrt(z) g
            int k = (int)((z - Z0) / HT);
            if (k >= NT) k = NT - 1;
            const double t = (z - Z0 - k * HT) / HT, z0 = Z0 + k * HT, z1 = z0 + HT;
            const double r0 = std::sqrt(z0), r1 = std::sqrt(z1);
            const double e = std::exp(-2.0 / 3.0 * z * std::sqrt(z));
            ai = e * hermite(t, HT, TA[k], TA[k + 1], TAp[k] + r0 * TA[k], TAp[k + 1] + r1 * TA[k + 1]);
            aip = e * hermite(t, HT, TAp[k], TAp[k + 1], z0 * TA[k] + r0 * TAp[k], z1 * TA[k + 1] + r1 * TAp[k + 1]);
            iai = e * hermite(t, HT, TF[k], TF[k + 1], -TA[k] + r0 * TF[k], -TA[k + 1] + r1 * TF[k + 1]);
            return;
        }
        int k = (int)(z / HZ);
        if (k >= NZ) k = NZ - 1;
        const double t = (z - k * HZ) / HZ, z0 = k * HZ, z1 = (k + 1) * HZ;
        ai = hermite(t, HZ, A[k], A[k + 1], Ap[k], Ap[k + 1]);
        aip = hermite(t, HZ, Ap[k], Ap[k + 1], z0 * A[k], z1 * A[k + 1]);
        iai = hermite(t, HZ, F[k], F[k + 1], -A[k], -A[k + 1]);
    }
};

const Airy &airy() {
    static Airy a;
    return a;
}

double emission_spectrum(double chi, double d) {
    if (d <= 0.0 || d >= 1.0) return 0.0;
    const double z = std::pow(d / (chi * (1.0 - d)), 2.0 / 3.0);
    double ai, aip, iai;
    airy().eval(z, ai, aip, iai);
    return -iai - (2.0 / z + chi * d * std::sqrt(z)) * aip;
}

double pair_spectrum(double chi, double d) {
    if (d <= 0.0 || d >= 1.0) return 0.0;
    const double z = std::pow(1.0 / (chi * d * (1.0 - d)), 2.0 / 3.0);
    if (z > 120.0) return 0.0;   // exp(-2/3 z^1.5) underflows
    double ai, aip, iai;
    airy().eval(z, ai, aip, iai);
    return iai + (2.0 / z - chi * std::sqrt(z)) * aip;
}

// spectrum in the x variable, times d(d)/dx
double in_x(int kind, double chi, double x) {
    const double a = x * x * x, b = (1.0 - x) * (1.0 - x) * (1.0 - x);
    const double d = a / (a + b), j = 3.0 * x * x * (1.0 - x) * (1.0 - x) / ((a + b) * (a + b));
    return (kind == 0 ? emission_spectrum(chi, d) : pair_spectrum(chi, d)) * j;
}

constexpr int NPAN = 1024, NGL = 8;

struct Quad {
    double x[NGL], w[NGL];
    Quad() { gauss_legendre(NGL, x, w); }
    double integrate(int kind, double chi, double a, double b) const {
        double s = 0.0;
        for (int q = 0; q < NGL; ++q) s += w[q] * in_x(kind, chi, 0.5 * (a + b) + 0.5 * (b - a) * x[q]);
        return 0.5 * (b - a) * s;
    }
};

void build_row(const Quad &Q, int kind, double chi, double &W, double *X) {
    std::vector<double> C(NPAN + 1);
    C[0] = 0.0;
    for (int p = 0; p < NPAN; ++p)
        C[p + 1] = C[p] + Q.integrate(kind, chi, (double)p / NPAN, (double)(p + 1) / NPAN);
    W = C[NPAN];
    for (int j = 0; j < NU; ++j) {
        const double u = (j + 0.5) / NU;
        if (!(W > 0.0)) { X[j] = u; continue; }
        const double target = u * W;
        int p = 0;
        while (p < NPAN - 1 && C[p + 1] < target) ++p;
        const double a = (double)p / NPAN, b = (double)(p + 1) / NPAN;
        // Newton on C[p] + Int_a^x f = target, safeguarded by bisection
        double lo = a, hi = b, x = a + (b - a) * (target - C[p]) / (C[p + 1] - C[p]);
        for (int it = 0; it < 60; ++it) {
            const double g = C[p] + Q.integrate(kind, chi, a, x) - target;
            if (g < 0.0) lo = x; else hi = x;
            const double fx = in_x(kind, chi, x);
            double xn = fx > 0.0 ? x - g / fx : 0.5 * (lo + hi);
            if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
            if (std::fabs(xn - x) < 1e-15) { x = xn; break; }
            x = xn;
        }
        X[j] = x;
    }
}

std::mutex g_mu;
std::vector<double> g_tables;   // We[256], Wb[256], Xe[256][128], Xb[256][128]

}  // namespace

// Tables of the emission (W_e, X_e) and pair (W_b, X_b) spectra; built on
// the first call (about a second) and cached for the process.
const double *hk_qed_host_tables() {
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_tables.empty()) {
        std::vector<double> t(2 * NCHI + 2 * NCHI * NU);
        Quad Q;
        airy();
        for (int i = 0; i < NCHI; ++i) {
            const double chi = std::pow(10.0, -3.0 + 6.0 * i / (NCHI - 1));
            build_row(Q, 0, chi, t[i], &t[2 * NCHI + (size_t)i * NU]);
            build_row(Q, 1, chi, t[NCHI + i], &t[2 * NCHI + (size_t)NCHI * NU + (size_t)i * NU]);
        }
        g_tables.swap(t);
    }
    return g_tables.data();
}

// host Airy values for the tests of the table builder
void hk_qed_host_airy(double z, double *ai, double *aip, double *iai) { airy().eval(z, *ai, *aip, *iai); }
