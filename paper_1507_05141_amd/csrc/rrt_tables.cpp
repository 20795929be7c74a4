// Host-side FP64 tables of the library: ordinate quadrature and real
// spherical harmonics on the ordinates.  Built once per problem (rrt_create);
// uploaded to the device in the working precision.
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
    gauss_legendre(n, x.data(), w.data());
}

void gauss_legendre(int n, double *x, double *w)
{
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

}  // namespace rrt
