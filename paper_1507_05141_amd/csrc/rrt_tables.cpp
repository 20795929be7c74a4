// Host-side FP64 tables of the library: ordinate quadrature, real spherical
// harmonics on the ordinates and the Klein-Nishina group-to-group tables.
// Built once per problem (rrt_create); uploaded to the device in the working
// precision.
#include "rrt_internal.h"

#include <cmath>
#include <vector>

namespace rrt {

static const double kPi = 3.14159265358979323846;

// Gauss-Legendre nodes on [-1, 1] (ascending) and weights.  Newton iteration
// on P_n, evaluated by the three-term recurrence, from the asymptotic first
// guess cos(pi (4i - 1) / (4n + 2)) of the i-th largest root.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 1; i <= n; ++i) {
        double t = std::cos(kPi * (4.0 * i - 1.0) / (4.0 * n + 2.0));
        double dpn = 1.0;
        for (int iter = 0; iter < 100; ++iter) {
            double pm1 = 1.0, p = t;          // P_0, P_1
            for (int k = 1; k < n; ++k) {
                double pn = ((2.0 * k + 1.0) * t * p - k * pm1) / (k + 1.0);
                pm1 = p;
                p = pn;
            }
            if (n == 1) { p = t; pm1 = 1.0; }
            dpn = n * (pm1 - t * p) / (1.0 - t * t);
            double step = p / dpn;
            t -= step;
            if (std::fabs(step) <= 1e-16 * std::fmax(1.0, std::fabs(t))) {
                // one more evaluation of the derivative at the final node
                pm1 = 1.0; p = t;
                for (int k = 1; k < n; ++k) {
                    double pn = ((2.0 * k + 1.0) * t * p - k * pm1) / (k + 1.0);
                    pm1 = p;
                    p = pn;
                }
                if (n == 1) { p = t; pm1 = 1.0; }
                dpn = n * (pm1 - t * p) / (1.0 - t * t);
                break;
            }
        }
        x[n - i] = t;
        w[n - i] = 2.0 / ((1.0 - t * t) * dpn * dpn);
    }
}

// Real orthonormal spherical harmonics (q = l*l + l + m) at one direction,
// from fully normalised associated Legendre functions:
//   Pbar_0^0 = 1/sqrt(4 pi), Pbar_m^m = sqrt((2m+1)/(2m)) s Pbar_{m-1}^{m-1},
//   Pbar_{m+1}^m = sqrt(2m+3) mu Pbar_m^m,
//   Pbar_l^m = a_lm (mu Pbar_{l-1}^m - b_lm Pbar_{l-2}^m),
//   a_lm = sqrt((4l^2-1)/(l^2-m^2)), b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)),
// times sqrt(2) cos(m phi) (m > 0), 1 (m = 0), sqrt(2) sin(|m| phi) (m < 0).
void real_sh(int lmax, double mu, double phi, double *Y)
{
    const double s = std::sqrt(std::fmax(0.0, 1.0 - mu * mu));
    double pmm = 1.0 / std::sqrt(4.0 * kPi);
    for (int m = 0; m <= lmax; ++m) {
        if (m > 0) pmm *= std::sqrt((2.0 * m + 1.0) / (2.0 * m)) * s;
        const double cm = (m == 0) ? 1.0 : std::sqrt(2.0) * std::cos(m * phi);
        const double sm = (m == 0) ? 0.0 : std::sqrt(2.0) * std::sin(m * phi);
        double p2 = 0.0, p1 = pmm;           // Pbar_{l-2}^m, Pbar_{l-1}^m
        for (int l = m; l <= lmax; ++l) {
            double p;
            if (l == m) {
                p = pmm;
            } else if (l == m + 1) {
                p = std::sqrt(2.0 * m + 3.0) * mu * pmm;
            } else {
                double a = std::sqrt((4.0 * l * l - 1.0) / (double(l) * l - double(m) * m));
                double b = std::sqrt((double(l - 1) * (l - 1) - double(m) * m) / (4.0 * (l - 1) * (l - 1) - 1.0));
                p = a * (mu * p1 - b * p2);
            }
            if (l > m) { p2 = p1; p1 = p; }
            if (m == 0) {
                Y[l * l + l] = p;
            } else {
                Y[l * l + l + m] = p * cm;
                Y[l * l + l - m] = p * sm;
            }
        }
    }
}

// Klein-Nishina dsigma/dOmega / r0^2 with the scattered-to-incident frequency
// ratio entering squared (the textbook Klein-Nishina formula).
static double kn_cross(double x, double mu)
{
    const double r = 1.0 / (1.0 + x * (1.0 - mu));
    return 0.5 * r * r * (r + 1.0 / r - (1.0 - mu * mu));
}

static double legendre(int l, double t)
{
    double a = 1.0, b = t;
    if (l == 0) return a;
    for (int k = 2; k <= l; ++k) {
        double c = ((2 * k - 1) * t * b - (k - 1) * a) / k;
        a = b;
        b = c;
    }
    return b;
}

// Composite 24-point Gauss-Legendre (16 panels) of kn_cross(x, mu) P_l(mu) for
// l = 0..lmax over [lo, hi]; out[l] accumulates.
static void kn_moments(double x, double lo, double hi, int lmax, const std::vector<double> &gx,
                       const std::vector<double> &gw, double *out)
{
    const int panels = 16;
    const double h = (hi - lo) / panels;
    for (int pnl = 0; pnl < panels; ++pnl) {
        const double a = lo + pnl * h, c = a + 0.5 * h;
        for (size_t i = 0; i < gx.size(); ++i) {
            const double mu = c + 0.5 * h * gx[i];
            const double f = kn_cross(x, mu) * gw[i] * 0.5 * h;
            double p0 = 1.0, p1 = mu;
            out[0] += f;
            if (lmax >= 1) out[1] += f * mu;
            for (int l = 2; l <= lmax; ++l) {
                double p2 = ((2 * l - 1) * mu * p1 - (l - 1) * p0) / l;
                out[l] += f * p2;
                p0 = p1;
                p1 = p2;
            }
        }
    }
}

// Multi-group Compton scattering on electrons at rest with photons at the bin
// centres.  s[i] = sigma_KN(nu_i)/sigma_T; the source coefficient of Legendre
// order l from group i into group j is
//   A[l][j][i] = s_i (nu_j dnu_i)/(nu_i dnu_j) p_l^{i->j} / (2l+1),
// where p^{i->j}(mu) = 4 pi dsigma/dOmega(nu_i, mu) / sigma_KN(nu_i) on the
// scattering cosines whose scattered frequency nu_i/(1 + x_i (1 - mu)) lies in
// bin j, and p_l = (2l+1)/2 int p P_l dmu.
void compton_tables(int G, const double *edges, const double *centres, double mec2, int lmax,
                    std::vector<double> &s, std::vector<double> &A, std::vector<double> &p_out)
{
    std::vector<double> gx, gw;
    gauss_legendre(24, gx, gw);
    s.assign(G, 0.0);
    A.assign((size_t)(lmax + 1) * G * G, 0.0);
    p_out.assign((size_t)(lmax + 1) * G * G, 0.0);
    std::vector<double> mom(lmax + 1);
    for (int i = 0; i < G; ++i) {
        const double nu = centres[i], x = nu / mec2;
        std::fill(mom.begin(), mom.end(), 0.0);
        kn_moments(x, -1.0, 1.0, 0, gx, gw, mom.data());
        const double sig = 2.0 * kPi * mom[0];           // r0^2 units
        s[i] = sig / (8.0 * kPi / 3.0);
        for (int j = 0; j < G; ++j) {
            // cosine of the scattering angle that lands exactly on a frequency
            auto mu_of = [&](double e) { return e > 0.0 ? 1.0 - (nu / e - 1.0) / x : -2.0; };
            double lo = std::fmax(-1.0, mu_of(edges[j]));
            double hi = std::fmin(1.0, mu_of(edges[j + 1]));
            if (!(hi > lo)) continue;
            std::fill(mom.begin(), mom.end(), 0.0);
            kn_moments(x, lo, hi, lmax, gx, gw, mom.data());
            for (int l = 0; l <= lmax; ++l) {
                const double pl = (2.0 * l + 1.0) * 0.5 * 4.0 * kPi / sig * mom[l];
                p_out[((size_t)l * G + i) * G + j] = pl;
                const double dnu_i = edges[i + 1] - edges[i], dnu_j = edges[j + 1] - edges[j];
                A[((size_t)l * G + j) * G + i] = s[i] * (centres[j] * dnu_i) / (centres[i] * dnu_j) * pl / (2.0 * l + 1.0);
            }
        }
    }
}

}  // namespace rrt
