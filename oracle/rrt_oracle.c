/*
 * Oracle for the mixed-frame relativistic SHDOM source iteration of
 * Tominaga, Shibata & Blinnikov (2015), "Time-dependent multi-group
 * multidimensional relativistic radiative transfer code based on SHDOM".
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 CPU implementation
 * written straight from the paper's equations, used to check the HIP library.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * Where the paper defers to the SHDOM papers (Evans 1998; Pincus & Evans 2009)
 * and to de la Cruz Rodriguez & Piskunov (2013) for details it does not print,
 * the reading followed here is the one documented with the repository's design
 * notes (grid, ordinates, interpolation, Bezier derivative rule, boundaries).
 *
 * Array layouts (point index p = (z*ny + y)*nx + x, ordinate k = a*nphi + b):
 *   SH arrays            [P][G][NLM]          (q = l*l + l + m)
 *   comoving DO arrays   [P][G][K]
 *   lab DO arrays        [K][G][P]
 *   fields               kappa, bnu [P][G]; sigma [P]; beta [P][3]
 *   z-boundary inflow    [K][G][ny][nx]
 *
 * Functions whose result is not pinned by a test against something other than
 * this file say so in their comment.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
    /* grid: x, y periodic with nx, ny points; z has nz points on [0, lz] */
    int nx, ny, nz;
    double lx, ly, lz;
    /* angular mesh and spherical-harmonic order */
    int nmu, nphi, lmax;
    /* frequency groups */
    int ng;
    int grey;               /* 1: one frequency-integrated group */
    const double *edges;    /* [ng+1] */
    const double *centres;  /* [ng]   */
    /* scattering: 0 = Thomson, 1 = Compton */
    int compton;
    const double *kn_s;     /* [nt][ng]  sigma(nu_i; T_n) / sigma_T                    */
    const double *kn_p;     /* [nt][lmax+1][ng][ng]  Legendre moment p_l^{i->j}(T_n)    */
    /* fields */
    const double *kappa;    /* [P][ng] */
    const double *sigma;    /* [P]     */
    const double *bnu;      /* [P][ng] */
    const double *beta;     /* [P][3] or NULL */
    const double *bc_bot;   /* [K][ng][ny][nx] or NULL */
    const double *bc_top;   /* [K][ng][ny][nx] or NULL */
    /* ordinate tables */
    const double *mu;       /* [nmu] Gauss-Legendre nodes, ascending */
    const double *wmu;      /* [nmu] Gauss-Legendre weights          */
    const double *Y;        /* [K][NLM] real SH at the ordinates     */
    /* electron temperature: ntemp = 0 for electrons at rest (one table);
       else the tables above are given at ntemp nodes, log10 of the node
       temperatures in lt_nodes (ascending), and kte [P] is the field */
    int ntemp;
    const double *lt_nodes;
    const double *kte;
} or_problem;

static int nlm_of(int lmax) { return (lmax + 1) * (lmax + 1); }
static long npts(const or_problem *pr) { return (long)pr->nx * pr->ny * pr->nz; }
static int nord(const or_problem *pr) { return pr->nmu * pr->nphi; }

/* ------------------------------------------------------------------------ */
/* Quadrature and spherical harmonics (Eq. 9: real orthonormal Y_lm)         */
/* ------------------------------------------------------------------------ */

/* Gauss-Legendre nodes (ascending) and weights on [-1, 1] by Newton iteration
   on the three-term Legendre recurrence. */
int or_gauss_legendre(int n, double *x, double *w)
{
    if (n < 1) return -1;
    for (int i = 0; i < n; i++) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        double pn = 0.0, dp = 1.0;
        for (int it = 0; it < 200; it++) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            pn = p1;
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = pn / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {   /* derivative at the converged root */
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    return 0;
}

/* Real orthonormal spherical harmonics at (mu, phi), all l <= lmax, index
   q = l*l + l + m.  Y_lm = N_l^|m| P_l^|m|(mu) * {sqrt2 cos(m phi), 1,
   sqrt2 sin(|m| phi)} for m > 0, m = 0, m < 0, associated Legendre functions
   without the Condon-Shortley phase, N_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!). */
void or_sh_eval(int lmax, double mu, double phi, double *Y)
{
    int L = lmax;
    double *P = (double *)malloc(sizeof(double) * (L + 1) * (L + 1));
    double s = sqrt(fmax(0.0, 1.0 - mu * mu));
    for (int m = 0; m <= L; m++) {
        double pmm = 1.0;
        for (int i = 1; i <= m; i++) pmm *= (2.0 * i - 1.0) * s;
        P[m * (L + 1) + m] = pmm;
        if (m + 1 <= L) P[(m + 1) * (L + 1) + m] = (2.0 * m + 1.0) * mu * pmm;
        for (int l = m + 2; l <= L; l++)
            P[l * (L + 1) + m] = ((2.0 * l - 1.0) * mu * P[(l - 1) * (L + 1) + m]
                                  - (l + m - 1.0) * P[(l - 2) * (L + 1) + m]) / (l - m);
    }
    for (int l = 0; l <= L; l++) {
        for (int m = 0; m <= l; m++) {
            double ratio = 1.0;               /* (l-m)!/(l+m)! */
            for (int i = l - m + 1; i <= l + m; i++) ratio /= (double)i;
            double N = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * ratio);
            double v = N * P[l * (L + 1) + m];
            if (m == 0) {
                Y[l * l + l] = v;
            } else {
                Y[l * l + l + m] = v * sqrt(2.0) * cos(m * phi);
                Y[l * l + l - m] = v * sqrt(2.0) * sin(m * phi);
            }
        }
    }
    free(P);
}

/* Y[k][q] at every ordinate k = a*nphi + b, phi_b = 2 pi b / nphi. */
void or_sh_table(int lmax, int nmu, int nphi, const double *mu, double *Y)
{
    int nl = nlm_of(lmax);
    for (int a = 0; a < nmu; a++)
        for (int b = 0; b < nphi; b++)
            or_sh_eval(lmax, mu[a], 2.0 * M_PI * b / nphi, Y + (long)(a * nphi + b) * nl);
}

static void ordinate_dir(const or_problem *pr, int k, double n[3])
{
    int a = k / pr->nphi, b = k % pr->nphi;
    double mu = pr->mu[a], phi = 2.0 * M_PI * b / pr->nphi;
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    n[0] = st * cos(phi);
    n[1] = st * sin(phi);
    n[2] = mu;
}

static double ordinate_weight(const or_problem *pr, int k)
{
    return pr->wmu[k / pr->nphi] * 2.0 * M_PI / pr->nphi;
}

/* ------------------------------------------------------------------------ */
/* Compton tables, Eqs. 13-14 (Klein-Nishina, electrons at rest)             */
/* ------------------------------------------------------------------------ */

static double legendre_p(int l, double x)
{
    if (l == 0) return 1.0;
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= l; k++) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

/* Klein-Nishina differential cross-section in units of r0^2 for a photon of
   energy x = h nu / (m_e c^2) scattered by angle with cosine mu.  The ratio
   nu1/nu enters squared (Rybicki & Lightman Eq. 7.4); the single power printed
   in Eq. 14 does not integrate to the Klein-Nishina total cross-section. */
static double kn_dsdo(double x, double mu)
{
    double eps = 1.0 / (1.0 + x * (1.0 - mu));
    return 0.5 * eps * eps * (1.0 / eps + eps - (1.0 - mu * mu));
}

/* integral of f(mu) = kn_dsdo(x,mu) * P_l(mu) over [a, b] by 48-point Gauss-Legendre */
static double kn_band_integral(double x, int l, double a, double b, const double *gx, const double *gw, int ng)
{
    double h = 0.5 * (b - a), c = 0.5 * (b + a), s = 0.0;
    for (int i = 0; i < ng; i++) {
        double mu = c + h * gx[i];
        s += gw[i] * kn_dsdo(x, mu) * legendre_p(l, mu);
    }
    return s * h;
}

/* Group-to-group Compton tables for electrons at rest (multi-group treatment
   of the Klein-Nishina kernel, with photons at the bin-centre frequency):
     s[i]        = sigma_KN(nu_i) / sigma_T
     p[l][i][j]  = (2l+1)/2 * integral over mu of p^{i->j}(mu) P_l(mu),
     p^{i->j}(mu) = 4 pi (dsigma/dOmega)(nu_i, mu) / sigma_KN(nu_i) when the
                    scattered frequency nu1(mu) = nu_i / (1 + x (1 - mu)) falls
                    in bin j, else 0.
   mec2 is the electron rest energy in the units of the edges. */
int or_compton_cold(int ng, const double *edges, const double *centres, double mec2,
                    int lmax, double *s, double *p)
{
    const int NQ = 48;
    double gx[48], gw[48];
    or_gauss_legendre(NQ, gx, gw);
    for (int i = 0; i < ng; i++) {
        double nu = centres[i], x = nu / mec2;
        /* total cross-section over 8 equal pieces of [-1, 1] */
        double tot = 0.0;
        for (int piece = 0; piece < 8; piece++)
            tot += kn_band_integral(x, 0, -1.0 + piece * 0.25, -1.0 + (piece + 1) * 0.25, gx, gw, NQ);
        tot *= 2.0 * M_PI;                        /* in r0^2 */
        s[i] = tot / (8.0 * M_PI / 3.0);
        for (int j = 0; j < ng; j++) {
            /* scattering-cosine range mapping into [edges[j], edges[j+1]) */
            double lo, hi;
            double e0 = edges[j], e1 = edges[j + 1];
            lo = (e0 > 0.0) ? 1.0 - (nu / e0 - 1.0) / x : -1.0e300;
            hi = (e1 > 0.0) ? 1.0 - (nu / e1 - 1.0) / x : -1.0e300;
            if (lo < -1.0) lo = -1.0;
            if (hi > 1.0) hi = 1.0;
            for (int l = 0; l <= lmax; l++) {
                double v = 0.0;
                if (hi > lo) {
                    /* split the band in 4 pieces for accuracy */
                    for (int piece = 0; piece < 4; piece++) {
                        double a = lo + (hi - lo) * piece / 4.0, b = lo + (hi - lo) * (piece + 1) / 4.0;
                        v += kn_band_integral(x, l, a, b, gx, gw, NQ);
                    }
                    v *= (2.0 * l + 1.0) / 2.0 * 4.0 * M_PI / tot;
                }
                p[((long)l * ng + i) * ng + j] = v;
            }
        }
    }
    return 0;
}

/* Klein-Nishina total cross-section of a photon of energy x = h nu / (m_e c^2),
   in units of r0^2, by the same 8-piece quadrature as or_compton_cold. */
static double kn_total(double x, const double *gx, const double *gw, int ng)
{
    double tot = 0.0;
    for (int piece = 0; piece < 8; piece++)
        tot += kn_band_integral(x, 0, -1.0 + piece * 0.25, -1.0 + (piece + 1) * 0.25, gx, gw, ng);
    return tot * 2.0 * M_PI;
}

/* Electrons of temperature kT (an isotropic Maxwell-Juttner distribution; not
   part of the paper, whose electrons are at rest).  For an electron of speed
   beta (Lorentz factor gam) moving at cosine mu_e to the incident photon
   (direction z) and the scattered photon going out at (mu1, phi1) in the same
   frame, with x = h nu / (m_e c^2):
     nu1 = nu (1 - beta.Omega) / (1 - beta.Omega1 + (x / gam)(1 - mu1))
   (energy-momentum conservation), and the scattered photons per unit solid
   angle and unit photon path, per electron, are
     R = (1 - beta.Omega) (dsigma/dOmega')_KN (nu1 / nu1')^2
   with the rest-frame frequencies nu' = gam nu (1 - beta.Omega),
   nu1' = gam nu1 (1 - beta.Omega1), the rest-frame scattering angle from the
   invariant nu nu1 (1 - mu1) = nu' nu1' (1 - cos Theta'), the flux factor
   (1 - beta.Omega) and the solid-angle Jacobian (nu1/nu1')^2 of the photon
   aberration. */
typedef struct {
    double nu, x, beta, gam, mue, sine, cphi;
} hot_state;

static double hot_nu1(const hot_state *h, double mu1)
{
    double s1 = sqrt(fmax(0.0, 1.0 - mu1 * mu1));
    double bo1 = h->beta * (h->sine * s1 * h->cphi + h->mue * mu1);
    return h->nu * (1.0 - h->beta * h->mue) / (1.0 - bo1 + h->x / h->gam * (1.0 - mu1));
}

static double hot_rate(const hot_state *h, double mu1)
{
    double s1 = sqrt(fmax(0.0, 1.0 - mu1 * mu1));
    double bo = h->beta * h->mue;
    double bo1 = h->beta * (h->sine * s1 * h->cphi + h->mue * mu1);
    double nu1 = h->nu * (1.0 - bo) / (1.0 - bo1 + h->x / h->gam * (1.0 - mu1));
    double nup = h->gam * h->nu * (1.0 - bo), nu1p = h->gam * nu1 * (1.0 - bo1);
    double omc = h->nu * nu1 * (1.0 - mu1) / (nup * nu1p);          /* 1 - cos Theta' */
    double c = 1.0 - omc;
    double r = nu1p / nup;
    double dsdo = 0.5 * r * r * (1.0 / r + r - (1.0 - c * c));
    double jac = nu1 / nu1p;
    return (1.0 - bo) * dsdo * jac * jac;
}

/* roots in (-1, 1) of a + b mu + c sqrt(1 - mu^2) = 0: with mu = cos psi,
   psi in (0, pi), the equation is R cos(psi - delta) = -a with
   R = sqrt(b^2 + c^2), delta = atan2(c, b); without the square-root term it is
   linear. */
static int hot_roots(double a, double b, double c, double out[2])
{
    int n = 0;
    if (c == 0.0) {
        if (b != 0.0) {
            double m = -a / b;
            if (m > -1.0 && m < 1.0) out[n++] = m;
        }
        return n;
    }
    double R = sqrt(b * b + c * c), y = -a / R;
    if (y < -1.0 || y > 1.0) return 0;
    double delta = atan2(c, b), g = acos(y);
    double cand[2] = {delta - g, delta + g};
    for (int k = 0; k < 2; k++) {
        double psi = cand[k];
        if (psi > M_PI) psi -= 2.0 * M_PI;
        if (psi < -M_PI) psi += 2.0 * M_PI;
        if (psi > 0.0 && psi < M_PI) {
            double m = cos(psi);
            if (m > -1.0 && m < 1.0) out[n++] = m;
        }
    }
    if (n == 2 && out[0] == out[1]) n = 1;
    return n;
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Group-to-group Compton tables for electrons of temperature kT (units of the
   edges; kT = 0: electrons at rest, the paper's kernel), same definitions as
   or_compton_cold with the Klein-Nishina rate averaged over the electrons:
     s[i]       = <R> integrated over all directions / sigma_T
     p[l][i][j] = (2l+1)/2 integral of P_l(mu1) 4 pi <R>(mu1) / (s[i] sigma_T) over
                  the mu1 where the scattered frequency lies in bin j,
   <R>(mu1) the rate averaged over the electrons' momentum and direction and
   over the azimuth of the scattered photon.  The averages are fixed
   quadrature rules: momentum by 16-point Gauss-Legendre in t on [0, 6] with
   (gam - 1) / Theta = t^2 (Theta = kT / m_e c^2; weight p gam t e^{-t^2}),
   the electron's direction cosine by 16-point Gauss-Legendre, the scattered
   azimuth by 12-point Gauss-Legendre on [0, pi] (the rate is even in it);
   along mu1, every interval of [-1, 1] on which the scattered frequency stays
   in one bin (split at the roots of nu1 = edge) takes 4 equal pieces of
   48-point Gauss-Legendre, as the cold tables do.  At kT = 0 the average is
   the single electron at rest.  Parity unpinned beyond the limits the tests
   check (cold limit, normalisation, Thomson limit, mean energy exchange). */
int or_compton_thermal(int ng, const double *edges, const double *centres, double mec2, int lmax, double kT,
                       double *s, double *p)
{
    const int NQ = 48, NT = 16, NE = 16, NF = 12;
    double gx[48], gw[48], tx[16], tw[16], ex[16], ew[16], fx[12], fw[12];
    or_gauss_legendre(NQ, gx, gw);
    or_gauss_legendre(NT, tx, tw);
    or_gauss_legendre(NE, ex, ew);
    or_gauss_legendre(NF, fx, fw);
    double theta = kT / mec2;
    int nt = theta > 0.0 ? NT : 1, ne = theta > 0.0 ? NE : 1, nf = theta > 0.0 ? NF : 1;
    /* momentum nodes and normalised weights */
    double gam_t[16], beta_t[16], wt_t[16], wsum = 0.0;
    for (int a = 0; a < nt; a++) {
        if (theta <= 0.0) { gam_t[a] = 1.0; beta_t[a] = 0.0; wt_t[a] = 1.0; wsum = 1.0; break; }
        double t = 3.0 * (tx[a] + 1.0);                   /* [0, 6] */
        double gam = 1.0 + theta * t * t;
        double pm = sqrt(gam * gam - 1.0);
        gam_t[a] = gam;
        beta_t[a] = pm / gam;
        wt_t[a] = 3.0 * tw[a] * pm * gam * t * exp(-t * t);
        wsum += wt_t[a];
    }
    for (int a = 0; a < nt; a++) wt_t[a] /= wsum;
    int L = lmax;
    #pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < ng; i++) {
        double nu = centres[i], x = nu / mec2;
        double *acc = (double *)calloc((size_t)(L + 1) * ng, sizeof(double));
        double *cut = (double *)malloc(sizeof(double) * (2 * (ng + 1) + 2));
        double *Pl = (double *)malloc(sizeof(double) * (L + 1));
        double sig = 0.0;                                   /* r0^2 units */
        for (int a = 0; a < nt; a++)
            for (int b = 0; b < ne; b++) {
                double mue = theta > 0.0 ? ex[b] : 1.0, wmue = theta > 0.0 ? 0.5 * ew[b] : 1.0;
                double beta = beta_t[a], gam = gam_t[a];
                sig += wt_t[a] * wmue * (1.0 - beta * mue) * kn_total(gam * x * (1.0 - beta * mue), gx, gw, NQ);
                for (int f = 0; f < nf; f++) {
                    double phi = theta > 0.0 ? 0.5 * M_PI * (fx[f] + 1.0) : 0.0;
                    double wphi = theta > 0.0 ? 0.5 * fw[f] : 1.0;      /* mean over [0, pi] */
                    hot_state h = {nu, x, beta, gam, mue, sqrt(fmax(0.0, 1.0 - mue * mue)), cos(phi)};
                    double w = wt_t[a] * wmue * wphi;
                    int nc = 0;
                    cut[nc++] = -1.0;
                    cut[nc++] = 1.0;
                    for (int e = 0; e <= ng; e++) {
                        double E = edges[e];
                        if (E <= 0.0) continue;
                        /* nu1 = E: nu (1 - beta mu_e) = E (1 - beta.Omega1 + (x/gam)(1 - mu1)) */
                        double A = nu * (1.0 - beta * mue) - E * (1.0 + x / gam);
                        double B = E * (x / gam + beta * mue);
                        double C = E * beta * h.sine * h.cphi;
                        nc += hot_roots(A, B, C, cut + nc);
                    }
                    qsort(cut, nc, sizeof(double), cmp_double);
                    for (int c = 0; c + 1 < nc; c++) {
                        double lo = cut[c], hi = cut[c + 1];
                        if (!(hi > lo)) continue;
                        double nm = hot_nu1(&h, 0.5 * (lo + hi));
                        if (nm < edges[0] || nm >= edges[ng]) continue;
                        int j = 0;
                        while (j < ng - 1 && nm >= edges[j + 1]) j++;
                        for (int piece = 0; piece < 4; piece++) {
                            double pa = lo + (hi - lo) * piece / 4.0, pb = lo + (hi - lo) * (piece + 1) / 4.0;
                            double hh = 0.5 * (pb - pa), cc = 0.5 * (pb + pa);
                            for (int q = 0; q < NQ; q++) {
                                double mu1 = cc + hh * gx[q];
                                double v = w * gw[q] * hh * hot_rate(&h, mu1);
                                Pl[0] = 1.0;
                                if (L >= 1) Pl[1] = mu1;
                                for (int l = 2; l <= L; l++)
                                    Pl[l] = ((2.0 * l - 1.0) * mu1 * Pl[l - 1] - (l - 1.0) * Pl[l - 2]) / l;
                                for (int l = 0; l <= L; l++) acc[(long)l * ng + j] += v * Pl[l];
                            }
                        }
                    }
                }
            }
        s[i] = sig / (8.0 * M_PI / 3.0);
        for (int l = 0; l <= L; l++)
            for (int j = 0; j < ng; j++)
                p[((long)l * ng + i) * ng + j] = (2.0 * l + 1.0) / 2.0 * 4.0 * M_PI / sig * acc[(long)l * ng + j];
        free(acc);
        free(cut);
        free(Pl);
    }
    return 0;
}

/* Unbinned averages of the same thermal rate for one photon frequency nu:
   out[0] = s (total / sigma_T), out[1] = mean of nu1/nu - 1 over the scattered
   photons (the rate-weighted mean over all scattered directions). */
int or_compton_thermal_moments(double nu, double mec2, double kT, double *out)
{
    const int NQ = 48, NT = 16, NE = 16, NF = 12;
    double gx[48], gw[48], tx[16], tw[16], ex[16], ew[16], fx[12], fw[12];
    or_gauss_legendre(NQ, gx, gw);
    or_gauss_legendre(NT, tx, tw);
    or_gauss_legendre(NE, ex, ew);
    or_gauss_legendre(NF, fx, fw);
    double theta = kT / mec2, x = nu / mec2;
    int nt = theta > 0.0 ? NT : 1, ne = theta > 0.0 ? NE : 1, nf = theta > 0.0 ? NF : 1;
    double wsum = 0.0, sig = 0.0, tot = 0.0, shift = 0.0;
    for (int a = 0; a < nt; a++) {
        double gam = 1.0, beta = 0.0, wt = 1.0;
        if (theta > 0.0) {
            double t = 3.0 * (tx[a] + 1.0);
            gam = 1.0 + theta * t * t;
            double pm = sqrt(gam * gam - 1.0);
            beta = pm / gam;
            wt = 3.0 * tw[a] * pm * gam * t * exp(-t * t);
        }
        wsum += wt;
        for (int b = 0; b < ne; b++) {
            double mue = theta > 0.0 ? ex[b] : 1.0, wmue = theta > 0.0 ? 0.5 * ew[b] : 1.0;
            sig += wt * wmue * (1.0 - beta * mue) * kn_total(gam * x * (1.0 - beta * mue), gx, gw, NQ);
            for (int f = 0; f < nf; f++) {
                double phi = theta > 0.0 ? 0.5 * M_PI * (fx[f] + 1.0) : 0.0;
                double wphi = theta > 0.0 ? 0.5 * fw[f] : 1.0;
                hot_state h = {nu, x, beta, gam, mue, sqrt(fmax(0.0, 1.0 - mue * mue)), cos(phi)};
                for (int piece = 0; piece < 8; piece++) {
                    double pa = -1.0 + piece * 0.25, pb = pa + 0.25, hh = 0.125, cc = 0.5 * (pa + pb);
                    for (int q = 0; q < NQ; q++) {
                        double mu1 = cc + hh * gx[q];
                        double v = wt * wmue * wphi * gw[q] * hh * hot_rate(&h, mu1) * 2.0 * M_PI;
                        tot += v;
                        shift += v * (hot_nu1(&h, mu1) / nu - 1.0);
                    }
                }
            }
        }
    }
    out[0] = sig / wsum / (8.0 * M_PI / 3.0);
    out[1] = shift / tot;
    out[2] = tot / wsum / (8.0 * M_PI / 3.0);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* S1: source function in SH space (Eqs. 10-12 and the multi-group kernel)   */
/* ------------------------------------------------------------------------ */

/* Electron-temperature bracket of point p: node n and weight w of node n + 1,
   linear in log10 T between nodes and clamped to the node range (n = 0, w = 0
   for electrons at rest). */
static void temp_bracket(const or_problem *pr, long p, int *n, double *w)
{
    *n = 0;
    *w = 0.0;
    if (pr->ntemp < 2 || !pr->kte) return;
    double lt = log10(pr->kte[p]);
    const double *t = pr->lt_nodes;
    int nt = pr->ntemp;
    if (lt <= t[0]) return;
    if (lt >= t[nt - 1]) { *n = nt - 2; *w = 1.0; return; }
    int k = 0;
    while (k < nt - 2 && lt >= t[k + 1]) k++;
    *n = k;
    *w = (lt - t[k]) / (t[k + 1] - t[k]);
}

/* scattering cross-section ratio s_g of point p (interpolated in log10 T) */
static double kn_s_at(const or_problem *pr, long p, int g)
{
    int n;
    double w;
    temp_bracket(pr, p, &n, &w);
    double v = pr->kn_s[(long)n * pr->ng + g];
    if (w > 0.0) v = (1.0 - w) * v + w * pr->kn_s[(long)(n + 1) * pr->ng + g];
    return v;
}

static double chi0_of(const or_problem *pr, long p, int g)
{
    double s = pr->compton ? kn_s_at(pr, p, g) : 1.0;
    return pr->kappa[p * pr->ng + g] + pr->sigma[p] * s;
}

/* S_lm = omega chi_l/(2l+1) I_lm + T_lm with the Thomson Legendre moments
   chi_l = (1, 0, 1/2, 0, ...) of 3/4 (1 + cos^2), or, for Compton,
   S_lm^j = sigma/chi_j sum_i s_i (nu_j dnu_i)/(nu_i dnu_j) p_l^{i->j}/(2l+1) I_lm^i,
   (with a temperature field, s_i p_l^{i->j} interpolated linearly in log10 T
   between the node tables),
   plus the isotropic thermal term T_00 = sqrt(4 pi) kappa B / chi. */
void or_source(const or_problem *pr, const double *I_lm, double *S_lm)
{
    long P = npts(pr);
    int G = pr->ng, NL = nlm_of(pr->lmax);
    #pragma omp parallel for
    for (long p = 0; p < P; p++) {
        for (int j = 0; j < G; j++) {
            double chi = chi0_of(pr, p, j);
            double *S = S_lm + (p * G + j) * NL;
            if (chi <= 0.0) {
                for (int q = 0; q < NL; q++) S[q] = 0.0;
                continue;
            }
            for (int l = 0; l <= pr->lmax; l++) {
                for (int m = -l; m <= l; m++) {
                    int q = l * l + l + m;
                    double v = 0.0;
                    if (!pr->compton) {
                        double chil = (l == 0) ? 1.0 : (l == 2 ? 0.5 : 0.0);
                        v = pr->sigma[p] / chi * chil / (2.0 * l + 1.0) * I_lm[(p * G + j) * NL + q];
                    } else {
                        /* A_l^{ji} at the node temperatures, linear in log10 T between them */
                        int n;
                        double wt;
                        temp_bracket(pr, p, &n, &wt);
                        long LG = (long)(pr->lmax + 1) * G * G;
                        for (int i = 0; i < G; i++) {
                            double dnu_i = pr->edges[i + 1] - pr->edges[i];
                            double dnu_j = pr->edges[j + 1] - pr->edges[j];
                            double f = (pr->centres[j] * dnu_i) / (pr->centres[i] * dnu_j) / (2.0 * l + 1.0);
                            double a0 = pr->kn_s[(long)n * G + i] * pr->kn_p[n * LG + ((long)l * G + i) * G + j];
                            double a = a0;
                            if (wt > 0.0)
                                a = (1.0 - wt) * a0 + wt * pr->kn_s[(long)(n + 1) * G + i]
                                                       * pr->kn_p[(n + 1) * LG + ((long)l * G + i) * G + j];
                            v += f * a * I_lm[(p * G + i) * NL + q];
                        }
                        v *= pr->sigma[p] / chi;
                    }
                    S[q] = v;
                }
            }
            S[0] += sqrt(4.0 * M_PI) * pr->kappa[p * G + j] * pr->bnu[p * G + j] / chi;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* S2 and S6: spherical harmonics <-> discrete ordinates                     */
/* ------------------------------------------------------------------------ */

/* S0(p, g, j) = sum_q Y[j][q] S_q(p, g) */
void or_sh2do(const or_problem *pr, const double *S_lm, double *S0)
{
    long P = npts(pr);
    int G = pr->ng, NL = nlm_of(pr->lmax), K = nord(pr);
    #pragma omp parallel for
    for (long p = 0; p < P; p++)
        for (int g = 0; g < G; g++)
            for (int k = 0; k < K; k++) {
                double v = 0.0;
                for (int q = 0; q < NL; q++) v += pr->Y[(long)k * NL + q] * S_lm[(p * G + g) * NL + q];
                S0[(p * G + g) * K + k] = v;
            }
}

/* I_q(p, g) = sum_j w_j Y[j][q] I0(p, g, j) */
void or_do2sh(const or_problem *pr, const double *I0, double *I_lm)
{
    long P = npts(pr);
    int G = pr->ng, NL = nlm_of(pr->lmax), K = nord(pr);
    #pragma omp parallel for
    for (long p = 0; p < P; p++)
        for (int g = 0; g < G; g++)
            for (int q = 0; q < NL; q++) {
                double v = 0.0;
                for (int k = 0; k < K; k++)
                    v += ordinate_weight(pr, k) * pr->Y[(long)k * NL + q] * I0[(p * G + g) * K + k];
                I_lm[(p * G + g) * NL + q] = v;
            }
}

/* ------------------------------------------------------------------------ */
/* Remap between frames (Eqs. 7-8 and the Lorentz invariants I/nu^3, chi nu) */
/* ------------------------------------------------------------------------ */

/* Bilinear value in (mu, phi) of F given at the ordinates (F[k*stride]).
   Beyond the outermost mu ring the value goes linearly to a pole value at
   mu = -1 or +1, equal to the azimuthal mean of that ring. */
static double angle_interp(const or_problem *pr, const double *F, long stride, const double n[3])
{
    int nmu = pr->nmu, nphi = pr->nphi;
    double mus = n[2];
    if (mus > 1.0) mus = 1.0;
    if (mus < -1.0) mus = -1.0;
    double phis = atan2(n[1], n[0]);
    if (phis < 0.0) phis += 2.0 * M_PI;
    double t = phis / (2.0 * M_PI / nphi);
    double tf = floor(t);
    double fphi = t - tf;
    int b0 = ((int)tf) % nphi;
    if (b0 < 0) b0 += nphi;
    int b1 = (b0 + 1) % nphi;
#define RING(a) ((1.0 - fphi) * F[(long)((a) * nphi + b0) * stride] + fphi * F[(long)((a) * nphi + b1) * stride])
    if (mus < pr->mu[0]) {
        double pole = 0.0;
        for (int b = 0; b < nphi; b++) pole += F[(long)b * stride];
        pole /= nphi;
        double w = (mus + 1.0) / (pr->mu[0] + 1.0);
        return (1.0 - w) * pole + w * RING(0);
    }
    if (mus > pr->mu[nmu - 1]) {
        double pole = 0.0;
        for (int b = 0; b < nphi; b++) pole += F[(long)((nmu - 1) * nphi + b) * stride];
        pole /= nphi;
        double w = (mus - pr->mu[nmu - 1]) / (1.0 - pr->mu[nmu - 1]);
        return (1.0 - w) * RING(nmu - 1) + w * pole;
    }
    int a = 0;
    while (a < nmu - 2 && mus > pr->mu[a + 1]) a++;
    double w = (mus - pr->mu[a]) / (pr->mu[a + 1] - pr->mu[a]);
    return (1.0 - w) * RING(a) + w * RING(a + 1);
#undef RING
}

/* Linear interpolation in ln(nu) of values v[g] given at the group centres.
   zero_outside = 1 (intensity invariants): two ghost centres, the mirror images
   of the outer centres in ln(nu) about the outer edges, carry the value 0 and
   the value is 0 beyond them (when the lowest edge is 0 the lowest value is held
   down to nu = 0).  zero_outside = 0 (opacities): the outer values are held. */
static double freq_interp(const or_problem *pr, const double *v, long stride, double nu, int zero_outside)
{
    int G = pr->ng;
    double x = log(nu);
    double c0 = log(pr->centres[0]), cN = log(pr->centres[G - 1]);
    if (!zero_outside) {
        if (x <= c0) return v[0];
        if (x >= cN) return v[(long)(G - 1) * stride];
    } else {
        if (x < c0) {
            if (pr->edges[0] <= 0.0) return v[0];
            double cg = 2.0 * log(pr->edges[0]) - c0;
            if (x <= cg) return 0.0;
            return v[0] * (x - cg) / (c0 - cg);
        }
        if (x >= cN) {
            double cg = 2.0 * log(pr->edges[G]) - cN;
            if (x >= cg) return 0.0;
            return v[(long)(G - 1) * stride] * (cg - x) / (cg - cN);
        }
    }
    int g = 0;
    while (g < G - 2 && x >= log(pr->centres[g + 1])) g++;
    double cl = log(pr->centres[g]), ch = log(pr->centres[g + 1]);
    double w = (x - cl) / (ch - cl);
    return (1.0 - w) * v[(long)g * stride] + w * v[(long)(g + 1) * stride];
}

static int has_motion(const or_problem *pr, long p)
{
    if (!pr->beta) return 0;
    const double *b = pr->beta + 3 * p;
    return !(b[0] == 0.0 && b[1] == 0.0 && b[2] == 0.0);
}

/* Doppler factor D = nu/nu0 of lab ordinate n at point p and the comoving
   direction n0 of that ray (Eqs. 7-8); D = 1 and n0 = n where the medium is
   at rest. */
static double lab_frame(const or_problem *pr, long p, const double n[3], double n0[3])
{
    n0[0] = n[0]; n0[1] = n[1]; n0[2] = n[2];
    if (!has_motion(pr, p)) return 1.0;
    const double *b = pr->beta + 3 * p;
    double b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    double Gam = 1.0 / sqrt(1.0 - b2);
    double bn = b[0] * n[0] + b[1] * n[1] + b[2] * n[2];
    double D = 1.0 / (Gam * (1.0 - bn));
    double f = Gam * (1.0 - Gam / (Gam + 1.0) * bn);
    for (int c = 0; c < 3; c++) n0[c] = D * (n[c] - f * b[c]);
    return D;
}

/* lab extinction of group g from the comoving extinctions C[G] of the point:
   chi_lab = chi0(nu/D)/D (chi nu invariant), linear in ln nu with the outer
   values held; a grey group takes chi0/D */
static double lab_chi(const or_problem *pr, const double *C, int g, double D, int moving)
{
    if (!moving) return C[g];
    if (pr->grey) return C[g] / D;
    return freq_interp(pr, C, 1, pr->centres[g] / D, 0) / D;
}

/* S3: lab-frame source and extinction on the lab ordinates, plus the implicit
   time terms of Eqs. 5-6:  chi~ = chi_lab + 1/(c dt),
   S~ = (chi_lab S_lab + I_prev/(c dt)) / chi~   (c = 1, inv_cdt = 1/(c dt)).
   Comoving -> lab: nu0 = Gamma nu (1 - beta.n) (Eq. 7), n0 from Eq. 8, and
   S_lab(nu) = nu^3 [S0/nu0^3](n0, nu/D), chi_lab = chi0(nu/D)/D, D = nu/nu0;
   a grey (frequency-integrated) group scales as D^4 instead. */
void or_boost(const or_problem *pr, const double *S0, const double *I_prev, double inv_cdt,
              double *St, double *Xt)
{
    long P = npts(pr);
    int G = pr->ng, K = nord(pr);
    #pragma omp parallel
    {
        double *A = (double *)malloc(sizeof(double) * G);
        double *C = (double *)malloc(sizeof(double) * G);
        #pragma omp for
        for (long p = 0; p < P; p++) {
            for (int g = 0; g < G; g++) C[g] = chi0_of(pr, p, g);
            int moving = has_motion(pr, p);
            for (int k = 0; k < K; k++) {
                double n[3], n0[3];
                ordinate_dir(pr, k, n);
                double D = lab_frame(pr, p, n, n0);
                for (int g = 0; g < G; g++) {
                    double Slab, chil = lab_chi(pr, C, g, D, moving);
                    if (!moving) {
                        Slab = S0[(p * G + g) * K + k];
                    } else if (pr->grey) {
                        Slab = D * D * D * D * angle_interp(pr, S0 + (p * G + g) * K, 1, n0);
                    } else {
                        if (g == 0)
                            for (int gp = 0; gp < G; gp++) {
                                double nc = pr->centres[gp];
                                A[gp] = angle_interp(pr, S0 + (p * G + gp) * K, 1, n0) / (nc * nc * nc);
                            }
                        double nu = pr->centres[g];
                        Slab = nu * nu * nu * freq_interp(pr, A, 1, nu / D, 1);
                    }
                    double ip = I_prev ? I_prev[((long)k * G + g) * P + p] : 0.0;
                    double xt = chil + inv_cdt;
                    long o = ((long)k * G + g) * P + p;
                    Xt[o] = xt;
                    St[o] = (xt > 0.0) ? (chil * Slab + ip * inv_cdt) / xt : 0.0;
                }
            }
        }
        free(A);
        free(C);
    }
}

/* chi~ of S3 for one lab ordinate k and group g at every point: out [P] */
void or_lab_extinction(const or_problem *pr, int k, int g, double inv_cdt, double *out)
{
    long P = npts(pr);
    int G = pr->ng;
    #pragma omp parallel
    {
        double *C = (double *)malloc(sizeof(double) * G);
        #pragma omp for
        for (long p = 0; p < P; p++) {
            for (int gp = 0; gp < G; gp++) C[gp] = chi0_of(pr, p, gp);
            double n[3], n0[3];
            ordinate_dir(pr, k, n);
            double D = lab_frame(pr, p, n, n0);
            out[p] = lab_chi(pr, C, g, D, has_motion(pr, p)) + inv_cdt;
        }
        free(C);
    }
}

/* S5: lab -> comoving on the comoving ordinates.  For comoving ordinate n0 the
   lab direction is n = (nu0/nu)[n0 + Gamma beta (1 + Gamma/(Gamma+1) beta.n0)]
   with nu/nu0 = D' = Gamma (1 + beta.n0), and I0(nu) = nu^3 [I_lab/nu^3](n, D' nu);
   a grey group scales as D'^-4. */
void or_unboost(const or_problem *pr, const double *I_lab, double *I0)
{
    long P = npts(pr);
    int G = pr->ng, K = nord(pr);
    #pragma omp parallel
    {
        double *A = (double *)malloc(sizeof(double) * G);
        #pragma omp for
        for (long p = 0; p < P; p++) {
            int moving = has_motion(pr, p);
            for (int j = 0; j < K; j++) {
                if (!moving) {
                    for (int g = 0; g < G; g++) I0[(p * G + g) * K + j] = I_lab[((long)j * G + g) * P + p];
                    continue;
                }
                double n0[3], n[3];
                ordinate_dir(pr, j, n0);
                const double *b = pr->beta + 3 * p;
                double b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
                double Gam = 1.0 / sqrt(1.0 - b2);
                double bn0 = b[0] * n0[0] + b[1] * n0[1] + b[2] * n0[2];
                double Dp = Gam * (1.0 + bn0);
                double f = Gam * (1.0 + Gam / (Gam + 1.0) * bn0);
                for (int c = 0; c < 3; c++) n[c] = (n0[c] + f * b[c]) / Dp;
                if (pr->grey) {
                    I0[(p * G + 0) * K + j] = angle_interp(pr, I_lab + p, (long)G * P, n) / (Dp * Dp * Dp * Dp);
                    continue;
                }
                for (int gp = 0; gp < G; gp++) {
                    double nc = pr->centres[gp];
                    A[gp] = angle_interp(pr, I_lab + (long)gp * P + p, (long)G * P, n) / (nc * nc * nc);
                }
                for (int g = 0; g < G; g++) {
                    double nu = pr->centres[g];
                    I0[(p * G + g) * K + j] = nu * nu * nu * freq_interp(pr, A, 1, Dp * nu, 1);
                }
            }
        }
        free(A);
    }
}

/* ------------------------------------------------------------------------ */
/* S4: short-characteristic ray trace with the cubic Bezier formal solution  */
/* ------------------------------------------------------------------------ */

/* periodic bilinear value of a plane F[ny][nx] at (i + ox, j + oy) (cell units) */
static double plane_interp(const double *F, int nx, int ny, int i, int j, double ox, double oy)
{
    double xs = i + ox, ys = j + oy;
    double x0 = floor(xs), y0 = floor(ys);
    double fx = xs - x0, fy = ys - y0;
    long i0 = ((long)x0 % nx + nx) % nx, j0 = ((long)y0 % ny + ny) % ny;
    long i1 = (i0 + 1) % nx, j1 = (j0 + 1) % ny;
    return (1.0 - fx) * (1.0 - fy) * F[j0 * nx + i0] + fx * (1.0 - fy) * F[j0 * nx + i1]
         + (1.0 - fx) * fy * F[j1 * nx + i0] + fx * fy * F[j1 * nx + i1];
}

/* Fritsch-Butland weighted harmonic mean of the two one-sided slopes around a
   point, hl and hr being the optical depths of the left and right intervals. */
static double fb_slope(double dl, double dr, double hl, double hr)
{
    if (dl * dr <= 0.0) return 0.0;
    double alpha = (1.0 + hr / (hl + hr)) / 3.0;
    return dl * dr / (alpha * dr + (1.0 - alpha) * dl);
}

static double clampd(double v, double a, double b)
{
    double lo = a < b ? a : b, hi = a < b ? b : a;
    return v < lo ? lo : (v > hi ? hi : v);
}

/* Weights of the cubic Bezier formal solution over optical depth h:
   integral_0^h S(t) e^{-(h-t)} dt = w0 S_u + w1 C_u + w2 C_p + w3 S_p, with
   E_n = h int_0^1 u^n e^{-h u} du.  Series in h for small h. */
static void bezier_weights(double h, double *ex, double w[4])
{
    double E[4];
    if (h < 0.5) {
        for (int n = 0; n < 4; n++) {
            double term = h, sum = 0.0;            /* h * (-h)^m / m! */
            for (int m = 0; m < 60; m++) {
                sum += term / (n + m + 1.0);
                term *= -h / (m + 1.0);
                if (fabs(term) < 1e-30) break;
            }
            E[n] = sum;
        }
        *ex = exp(-h);
    } else {
        double e = exp(-h);
        E[0] = 1.0 - e;
        for (int n = 1; n < 4; n++) E[n] = n / h * E[n - 1] - e;
        *ex = e;
    }
    w[0] = E[3];
    w[1] = 3.0 * (E[2] - E[3]);
    w[2] = 3.0 * (E[1] - 2.0 * E[2] + E[3]);
    w[3] = E[0] - 3.0 * E[1] + 3.0 * E[2] - E[3];
}

/* An upwind displacement within rounding of a whole number of cells is that
   whole number: a ray in a grid plane (n_x = cos(pi/2) evaluates to ~6e-17)
   then interpolates nothing across it.  Otherwise a tap weight of ~1e-15
   would give a vacuum neighbour a depth of ~1e-15 instead of 0, and the
   slope limiter treats zero and positive depths differently. */
static double snap_cells(double o)
{
    double r = nearbyint(o);
    return fabs(o - r) < 1e-9 ? r : o;
}

/* Number of equal pieces into which the path between two neighbouring z
   planes is cut for ordinates of polar cosine mu: enough that no piece moves
   the ray more than one cell horizontally, in any azimuth (a direction with a
   single column is left out: every horizontal offset reaches the same point
   there).  It depends on mu only, so every azimuth of a ring is treated alike. */
static int trace_pieces(const or_problem *pr, double mu)
{
    double h = 0.0;
    if (pr->nx > 1) h = pr->lx / pr->nx;
    if (pr->ny > 1 && (h == 0.0 || pr->ly / pr->ny < h)) h = pr->ly / pr->ny;
    if (h == 0.0) return 1;
    double dz = pr->lz / (pr->nz - 1);
    double c = dz * sqrt(fmax(0.0, 1.0 - mu * mu)) / (fabs(mu) * h);
    int m = (int)ceil(c - 1e-9);
    return m < 1 ? 1 : m;
}

/* Value at the point a fraction f of the way from grid plane A (at the
   horizontal offset (ox, oy) cells from point (i, j)) to grid plane B (same
   offset): bilinear in x and y, linear in z. */
static double path_value(const double *A, const double *B, int nx, int ny, int i, int j, double ox, double oy,
                         double f)
{
    double a = plane_interp(A, nx, ny, i, j, ox, oy);
    if (f == 0.0) return a;
    return (1.0 - f) * a + f * plane_interp(B, nx, ny, i, j, ox, oy);
}

/* For every lab ordinate and group, march the z planes from the inflow face.
   For grid point p on plane m the ray is traced back a distance dz/|mu| to
   the upwind point u on the previous plane, where the intensity I_u is
   bilinear (periodic in x and y).  The path from u to p is cut into np equal
   pieces (trace_pieces) at points q_0 = p, ..., q_np = u, where S~ and chi~
   are bilinear in x and y and linear in z between the grid planes, and the
   intensity is carried along the path piece by piece:
   I(q_j) = I(q_{j+1}) e^{-h} + Bezier integral of S~ over the piece, the
   control points taking their slopes from the neighbouring points q_{j+2}
   and q_{j-1} (which extend one piece beyond u and beyond p when those
   planes exist).  With np = 1 this is the plane-to-plane short
   characteristic. */
/* One lab ordinate k of one group: S, X and Ik are that ordinate's and
   group's [P] planes of S~, chi~ and I, bc its inflow plane [ny*nx] or NULL. */
static void trace_kg(const or_problem *pr, int k, const double *S, const double *X, const double *bc, double *Ik)
{
    int nx = pr->nx, ny = pr->ny, nz = pr->nz;
    long PL = (long)nx * ny;
    double dx = pr->lx / nx, dy = pr->ly / ny, dz = pr->lz / (nz - 1);
    double n[3];
    ordinate_dir(pr, k, n);
    double mu = n[2];
    int np = trace_pieces(pr, mu);
    double ds = dz / fabs(mu) / np;                  /* length of one piece */
    double ox = snap_cells(-ds * n[0] / dx), oy = snap_cells(-ds * n[1] / dy);
    double *qs = (double *)malloc(sizeof(double) * (np + 3));
    double *qx = (double *)malloc(sizeof(double) * (np + 3));
    for (int t = 0; t < nz; t++) {
        int m = (mu > 0.0) ? t : nz - 1 - t;
        int mu_ = (mu > 0.0) ? t - 1 : nz - t;       /* upwind plane          */
        int muu = (mu > 0.0) ? t - 2 : nz + 1 - t;   /* second upwind plane   */
        int md = (mu > 0.0) ? t + 1 : nz - 2 - t;    /* downwind plane        */
        if (t == 0) {
            for (long e = 0; e < PL; e++)
                Ik[m * PL + e] = bc ? bc[e] : 0.0;
            continue;
        }
        int has_d = t <= nz - 2, has_uu = t >= 2;
        for (int j = 0; j < ny; j++) {
            for (int i = 0; i < nx; i++) {
                long e = (long)j * nx + i;
                /* path points q_c, c = -1 .. np + 1, stored at index c + 1 */
                for (int c = -1; c <= np + 1; c++) {
                    double *vs = qs + c + 1, *vx = qx + c + 1;
                    if (c == -1) {
                        if (!has_d) { *vs = *vx = 0.0; continue; }
                        double f = 1.0 / np;
                        *vs = path_value(S + m * PL, S + md * PL, nx, ny, i, j, -ox, -oy, f);
                        *vx = path_value(X + m * PL, X + md * PL, nx, ny, i, j, -ox, -oy, f);
                    } else if (c <= np) {
                        double f = (double)c / np;
                        if (c == np) {          /* on the upwind plane */
                            *vs = plane_interp(S + mu_ * PL, nx, ny, i, j, c * ox, c * oy);
                            *vx = plane_interp(X + mu_ * PL, nx, ny, i, j, c * ox, c * oy);
                        } else {
                            *vs = path_value(S + m * PL, S + mu_ * PL, nx, ny, i, j, c * ox, c * oy, f);
                            *vx = path_value(X + m * PL, X + mu_ * PL, nx, ny, i, j, c * ox, c * oy, f);
                        }
                    } else {
                        if (!has_uu) { *vs = *vx = 0.0; continue; }
                        double f = 1.0 / np;
                        *vs = path_value(S + mu_ * PL, S + muu * PL, nx, ny, i, j, c * ox, c * oy, f);
                        *vx = path_value(X + mu_ * PL, X + muu * PL, nx, ny, i, j, c * ox, c * oy, f);
                    }
                }
                double Iv = plane_interp(Ik + mu_ * PL, nx, ny, i, j, np * ox, np * oy);
                for (int c = np - 1; c >= 0; c--) {
                    /* piece from q_{c+1} (u) to q_c (p); neighbours q_{c+2}, q_{c-1} */
                    double Su = qs[c + 2], Xu = qx[c + 2], Sp = qs[c + 1], Xp = qx[c + 1];
                    int d_ok = c >= 1 || has_d, uu_ok = c + 2 <= np || has_uu;
                    double hu = ds * 0.5 * (Xu + Xp);
                    double dSp = 0.0, dSu = 0.0;
                    if (hu > 0.0) {
                        double d1 = (Sp - Su) / hu;
                        if (d_ok) {
                            double Sd = qs[c], Xd = qx[c];
                            double hd = ds * 0.5 * (Xp + Xd);
                            dSp = (hd > 0.0) ? fb_slope(d1, (Sd - Sp) / hd, hu, hd) : 0.0;
                        } else {
                            dSp = d1;
                        }
                        if (uu_ok) {
                            double Suu = qs[c + 3], Xuu = qx[c + 3];
                            double huu = ds * 0.5 * (Xuu + Xu);
                            dSu = (huu > 0.0) ? fb_slope((Su - Suu) / huu, d1, huu, hu) : 0.0;
                        } else {
                            dSu = d1;
                        }
                    }
                    double Cu = clampd(Su + hu * dSu / 3.0, Su, Sp);
                    double Cp = clampd(Sp - hu * dSp / 3.0, Su, Sp);
                    double ex, w[4];
                    bezier_weights(hu, &ex, w);
                    Iv = Iv * ex + w[0] * Su + w[1] * Cu + w[2] * Cp + w[3] * Sp;
                }
                Ik[m * PL + e] = Iv;
            }
        }
    }
    free(qs); free(qx);
}

void or_trace(const or_problem *pr, const double *St, const double *Xt, double *I)
{
    int G = pr->ng, K = nord(pr);
    long P = npts(pr), PL = (long)pr->nx * pr->ny;
    #pragma omp parallel for collapse(2) schedule(dynamic)
    for (int k = 0; k < K; k++) {
        for (int g = 0; g < G; g++) {
            double n[3];
            ordinate_dir(pr, k, n);
            const double *bc = (n[2] > 0.0) ? pr->bc_bot : pr->bc_top;
            long o = ((long)k * G + g) * P;
            trace_kg(pr, k, St + o, Xt + o, bc ? bc + ((long)k * G + g) * PL : NULL, I + o);
        }
    }
}

/* S4 for the single lab ordinate k and group g: St, Xt and I are [P] */
void or_trace_one(const or_problem *pr, int k, int g, const double *St, const double *Xt, double *I)
{
    long PL = (long)pr->nx * pr->ny;
    double n[3];
    ordinate_dir(pr, k, n);
    const double *bc = (n[2] > 0.0) ? pr->bc_bot : pr->bc_top;
    trace_kg(pr, k, St, Xt, bc ? bc + ((long)k * pr->ng + g) * PL : NULL, I);
}

/* ------------------------------------------------------------------------ */
/* S7 moments (Eddington tensor), S8 residual                                */
/* ------------------------------------------------------------------------ */

/* Lab moments by ordinate quadrature: J = sum w I/4pi, H = sum w n I/4pi,
   K = sum w n n I/4pi, K stored as (xx, yy, zz, xy, xz, yz). */
void or_moments_lab(const or_problem *pr, const double *I_lab, double *J, double *H, double *Kt)
{
    long P = npts(pr);
    int G = pr->ng, K = nord(pr);
    #pragma omp parallel for
    for (long p = 0; p < P; p++)
        for (int g = 0; g < G; g++) {
            double j = 0, h[3] = {0, 0, 0}, kk[6] = {0, 0, 0, 0, 0, 0};
            for (int k = 0; k < K; k++) {
                double n[3];
                ordinate_dir(pr, k, n);
                double v = ordinate_weight(pr, k) * I_lab[((long)k * G + g) * P + p] / (4.0 * M_PI);
                j += v;
                for (int c = 0; c < 3; c++) h[c] += v * n[c];
                kk[0] += v * n[0] * n[0];
                kk[1] += v * n[1] * n[1];
                kk[2] += v * n[2] * n[2];
                kk[3] += v * n[0] * n[1];
                kk[4] += v * n[0] * n[2];
                kk[5] += v * n[1] * n[2];
            }
            J[p * G + g] = j;
            for (int c = 0; c < 3; c++) H[(p * G + g) * 3 + c] = h[c];
            for (int c = 0; c < 6; c++) Kt[(p * G + g) * 6 + c] = kk[c];
        }
}

/* Comoving moments from the l <= 2 SH coefficients of the comoving intensity. */
void or_moments_comoving(const or_problem *pr, const double *I_lm, double *J, double *H, double *Kt)
{
    long P = npts(pr);
    int G = pr->ng, NL = nlm_of(pr->lmax);
    double f4 = 4.0 * M_PI;
    for (long p = 0; p < P; p++)
        for (int g = 0; g < G; g++) {
            const double *c = I_lm + (p * G + g) * NL;
            double i0 = sqrt(f4) * c[0];                                  /* int I dOmega         */
            J[p * G + g] = i0 / f4;
            double hx = 0, hy = 0, hz = 0;
            if (pr->lmax >= 1) {
                hx = sqrt(f4 / 3.0) * c[3];
                hy = sqrt(f4 / 3.0) * c[1];
                hz = sqrt(f4 / 3.0) * c[2];
            }
            H[(p * G + g) * 3 + 0] = hx / f4;
            H[(p * G + g) * 3 + 1] = hy / f4;
            H[(p * G + g) * 3 + 2] = hz / f4;
            double kxx = i0 / 3.0, kyy = i0 / 3.0, kzz = i0 / 3.0, kxy = 0, kxz = 0, kyz = 0;
            if (pr->lmax >= 2) {
                double a20 = sqrt(16.0 * M_PI / 5.0) * c[6];   /* int (3 nz^2 - 1) I  */
                double a22 = sqrt(16.0 * M_PI / 15.0) * c[8];  /* int (nx^2 - ny^2) I */
                kzz = (a20 + i0) / 3.0;
                double sxy = i0 - kzz;                          /* int (nx^2 + ny^2) I */
                kxx = 0.5 * (sxy + a22);
                kyy = 0.5 * (sxy - a22);
                kxy = sqrt(f4 / 15.0) * c[4];
                kxz = sqrt(f4 / 15.0) * c[7];
                kyz = sqrt(f4 / 15.0) * c[5];
            }
            double *k6 = Kt + (p * G + g) * 6;
            k6[0] = kxx / f4; k6[1] = kyy / f4; k6[2] = kzz / f4;
            k6[3] = kxy / f4; k6[4] = kxz / f4; k6[5] = kyz / f4;
        }
}

/* per-group ||S_new - S_old||_2 / ||S_new||_2 over (points, SH terms) */
void or_residual(const or_problem *pr, const double *S_old, const double *S_new, double *r)
{
    long P = npts(pr);
    int G = pr->ng, NL = nlm_of(pr->lmax);
    for (int g = 0; g < G; g++) {
        double dn = 0.0, nn = 0.0;
        for (long p = 0; p < P; p++)
            for (int q = 0; q < NL; q++) {
                double a = S_new[(p * G + g) * NL + q], b = S_old[(p * G + g) * NL + q];
                dn += (a - b) * (a - b);
                nn += a * a;
            }
        r[g] = (nn > 0.0) ? sqrt(dn / nn) : (dn > 0.0 ? INFINITY : 0.0);
    }
}

/* ------------------------------------------------------------------------ */
/* One source iteration: S2, S3, S4, S5, S6, S1, S8                           */
/* ------------------------------------------------------------------------ */

int or_sweep(const or_problem *pr, const double *S_lm, const double *I_prev, double inv_cdt,
             double *I_lab, double *I_lm, double *S_new, double *resid)
{
    long P = npts(pr);
    long ndo = P * pr->ng * nord(pr);
    double *S0 = (double *)malloc(sizeof(double) * ndo);
    double *Xt = (double *)malloc(sizeof(double) * ndo);
    double *St = (double *)malloc(sizeof(double) * ndo);
    if (!S0 || !Xt || !St) { free(S0); free(Xt); free(St); return -2; }
    or_sh2do(pr, S_lm, S0);
    or_boost(pr, S0, I_prev, inv_cdt, St, Xt);
    or_trace(pr, St, Xt, I_lab);
    or_unboost(pr, I_lab, S0);       /* S0 reused as the comoving intensity I0 */
    or_do2sh(pr, S0, I_lm);
    or_source(pr, I_lm, S_new);
    or_residual(pr, S_lm, S_new, resid);
    free(S0); free(Xt); free(St);
    return 0;
}
