// HIP kernels of the source-iteration sweep (gfx950).  Templated on the
// working precision (float or double); geometry of the Lorentz maps is always
// evaluated in double, reductions are accumulated in double.
#include <hip/hip_runtime.h>

#include "rrt_kernels.h"

namespace rrt {

static constexpr double kPiD = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// cubic Bezier formal-solution weights
// ---------------------------------------------------------------------------

// Series coefficients of the four weights as functions of the optical depth h:
// w_i(h) = h sum_m bez_c[i][m] h^m, bez_c[i][m] = (-1)^m/m! * int_0^1 b_i(u) u^m du
// with b_0 = u^3, b_1 = 3u^2(1-u), b_2 = 3u(1-u)^2, b_3 = (1-u)^3.
__constant__ double c_bez64[4][kBezTerms64];
__constant__ float c_bez32[4][kBezTerms32];

void bezier_series_coefficients(double (*c64)[kBezTerms64], float (*c32)[kBezTerms32])
{
    double fact = 1.0;
    for (int m = 0; m < kBezTerms64; ++m) {
        if (m > 0) fact *= m;
        const double sgn = (m % 2) ? -1.0 : 1.0;
        const double a = m + 1.0, b = m + 2.0, c = m + 3.0, d = m + 4.0;
        const double v[4] = {1.0 / d, 3.0 / (c * d), 6.0 / (b * c * d), 6.0 / (a * b * c * d)};
        for (int i = 0; i < 4; ++i) {
            c64[i][m] = sgn / fact * v[i];
            if (m < kBezTerms32) c32[i][m] = (float)(sgn / fact * v[i]);
        }
    }
}

hipError_t upload_bezier_coefficients()
{
    double c64[4][kBezTerms64];
    float c32[4][kBezTerms32];
    bezier_series_coefficients(c64, c32);
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_bez64), c64, sizeof(c64));
    if (e != hipSuccess) return e;
    return hipMemcpyToSymbol(HIP_SYMBOL(c_bez32), c32, sizeof(c32));
}

template <typename real> struct BezTraits;
template <> struct BezTraits<double> {
    static constexpr double hs = 0.5;
    static constexpr int nt = kBezTerms64;
    __device__ static double c(int i, int m) { return c_bez64[i][m]; }
    __device__ static double ex(double h) { return exp(-h); }
};
template <> struct BezTraits<float> {
    static constexpr float hs = 1.0f;
    static constexpr int nt = kBezTerms32;
    __device__ static float c(int i, int m) { return c_bez32[i][m]; }
    __device__ static float ex(float h) { return expf(-h); }
};

// integral over optical depth [0, h] of the Bezier source times e^{-(h - t)}
// = w0 S_u + w1 C_u + w2 C_p + w3 S_p; ex = e^{-h}
template <typename real>
__device__ __forceinline__ void bezier_weights(real h, real &ex, real &w0, real &w1, real &w2, real &w3)
{
    using T = BezTraits<real>;
    ex = T::ex(h);
    if (h < T::hs) {
        real a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
        for (int m = T::nt - 1; m >= 0; --m) {
            a0 = a0 * h + T::c(0, m);
            a1 = a1 * h + T::c(1, m);
            a2 = a2 * h + T::c(2, m);
            a3 = a3 * h + T::c(3, m);
        }
        w0 = h * a0; w1 = h * a1; w2 = h * a2; w3 = h * a3;
    } else {
        const real ih = real(1) / h;
        const real E0 = real(1) - ex;
        const real E1 = E0 * ih - ex;
        const real E2 = real(2) * E1 * ih - ex;
        const real E3 = real(3) * E2 * ih - ex;
        w0 = E3;
        w1 = real(3) * (E2 - E3);
        w2 = real(3) * (E1 - real(2) * E2 + E3);
        w3 = E0 - real(3) * E1 + real(3) * E2 - E3;
    }
}

// Fritsch-Butland weighted harmonic mean of the slopes on the left (dl, over
// optical depth hl) and right (dr, hr) of a point.
template <typename real>
__device__ __forceinline__ real fb_slope(real dl, real dr, real hl, real hr)
{
    if (dl * dr <= real(0)) return real(0);
    const real al = (real(1) + hr / (hl + hr)) * real(1.0 / 3.0);
    return dl * dr / (al * dr + (real(1) - al) * dl);
}

template <typename real>
__device__ __forceinline__ real clamp_between(real v, real a, real b)
{
    const real lo = fmin(a, b), hi = fmax(a, b);
    return fmin(fmax(v, lo), hi);
}

// periodic bilinear value of plane F[ny][nx] at point (i, j) shifted by
// (ix + fx, iy + fy) cells; ix, iy already reduced into [0, nx), [0, ny)
template <typename real>
__device__ __forceinline__ real shifted(const real *__restrict__ F, int i, int j, int nx, int ny,
                                        int ix, int iy, real fx, real fy)
{
    int i0 = i + ix; if (i0 >= nx) i0 -= nx;
    int j0 = j + iy; if (j0 >= ny) j0 -= ny;
    const int i1 = (i0 + 1 == nx) ? 0 : i0 + 1;
    const int j1 = (j0 + 1 == ny) ? 0 : j0 + 1;
    const real a = F[j0 * nx + i0], b = F[j0 * nx + i1], c = F[j1 * nx + i0], d = F[j1 * nx + i1];
    return (real(1) - fy) * ((real(1) - fx) * a + fx * b) + fy * ((real(1) - fx) * c + fx * d);
}

// ---------------------------------------------------------------------------
// S4: ray trace.  One workgroup per (ordinate, group) marches the z planes
// from the inflow face; the previous I plane is kept in LDS.
// ---------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(256) k_trace(TraceArgs<real> a)
{
    extern __shared__ unsigned char smem_raw[];
    real *Ish = reinterpret_cast<real *>(smem_raw);
    const int kg = blockIdx.x;
    const int k = kg / a.G;
    const OrdGeom gm = a.geo[k];
    const int nx = a.nx, ny = a.ny, nz = a.nz, PL = nx * ny;
    const long base = (long)kg * a.P;
    const real *__restrict__ S = a.St + base;
    const real *__restrict__ X = a.Xt + base;
    real *__restrict__ Io = a.I + base;
    const real *__restrict__ bc = gm.up ? a.bc_bot : a.bc_top;
    const real ds = (real)gm.ds;
    const real fxu = (real)gm.fx[1], fyu = (real)gm.fy[1];
    const real fxuu = (real)gm.fx[0], fyuu = (real)gm.fy[0];
    const real fxd = (real)gm.fx[2], fyd = (real)gm.fy[2];
    int cur = 0;
    for (int t = 0; t < nz; ++t) {
        const int m = gm.up ? t : nz - 1 - t;
        const int mu_ = gm.up ? t - 1 : nz - t;
        const int muu = gm.up ? t - 2 : nz + 1 - t;
        const int md = gm.up ? t + 1 : nz - 2 - t;
        real *Icur = Ish + cur * PL;
        const real *Iprv = Ish + (1 - cur) * PL;
        for (int e = threadIdx.x; e < PL; e += blockDim.x) {
            real v;
            if (t == 0) {
                v = bc ? bc[(long)kg * PL + e] : real(0);
            } else {
                const int i = e % nx, j = e / nx;
                const real Sp = S[(long)m * PL + e], Xp = X[(long)m * PL + e];
                const real *Su_pl = S + (long)mu_ * PL, *Xu_pl = X + (long)mu_ * PL;
                const real Su = shifted(Su_pl, i, j, nx, ny, gm.ix[1], gm.iy[1], fxu, fyu);
                const real Xu = shifted(Xu_pl, i, j, nx, ny, gm.ix[1], gm.iy[1], fxu, fyu);
                const real Iu = shifted(Iprv, i, j, nx, ny, gm.ix[1], gm.iy[1], fxu, fyu);
                const real hu = ds * real(0.5) * (Xu + Xp);
                real dSp = 0, dSu = 0;
                if (hu > real(0)) {
                    const real d1 = (Sp - Su) / hu;
                    if (t <= nz - 2) {
                        const real Sd = shifted(S + (long)md * PL, i, j, nx, ny, gm.ix[2], gm.iy[2], fxd, fyd);
                        const real Xd = shifted(X + (long)md * PL, i, j, nx, ny, gm.ix[2], gm.iy[2], fxd, fyd);
                        const real hd = ds * real(0.5) * (Xp + Xd);
                        dSp = (hd > real(0)) ? fb_slope(d1, (Sd - Sp) / hd, hu, hd) : real(0);
                    } else {
                        dSp = d1;
                    }
                    if (t >= 2) {
                        const real Suu = shifted(S + (long)muu * PL, i, j, nx, ny, gm.ix[0], gm.iy[0], fxuu, fyuu);
                        const real Xuu = shifted(X + (long)muu * PL, i, j, nx, ny, gm.ix[0], gm.iy[0], fxuu, fyuu);
                        const real huu = ds * real(0.5) * (Xuu + Xu);
                        dSu = (huu > real(0)) ? fb_slope((Su - Suu) / huu, d1, huu, hu) : real(0);
                    } else {
                        dSu = d1;
                    }
                }
                const real Cu = clamp_between(Su + hu * dSu * real(1.0 / 3.0), Su, Sp);
                const real Cp = clamp_between(Sp - hu * dSp * real(1.0 / 3.0), Su, Sp);
                real ex, w0, w1, w2, w3;
                bezier_weights(hu, ex, w0, w1, w2, w3);
                v = Iu * ex + w0 * Su + w1 * Cu + w2 * Cp + w3 * Sp;
            }
            Icur[e] = v;
            Io[(long)m * PL + e] = v;
        }
        __syncthreads();
        cur ^= 1;
    }
}

// ---------------------------------------------------------------------------
// frame transforms
// ---------------------------------------------------------------------------

struct AngleTaps {
    int a0, a1;      // ring indices; -1 = lower pole, nmu = upper pole
    int b0, b1;
    double wmu, wphi;
};

// bilinear taps of direction n on the Gauss-Legendre x uniform-azimuth mesh
__device__ __forceinline__ AngleTaps angle_taps(const double *__restrict__ mu, int nmu, int nphi, const double n[3])
{
    AngleTaps t;
    double ms = fmin(1.0, fmax(-1.0, n[2]));
    double ph = atan2(n[1], n[0]);
    if (ph < 0.0) ph += 2.0 * kPiD;
    const double s = ph * (nphi / (2.0 * kPiD));
    const double sf = floor(s);
    t.wphi = s - sf;
    int b0 = (int)sf % nphi;
    if (b0 < 0) b0 += nphi;
    t.b0 = b0;
    t.b1 = (b0 + 1 == nphi) ? 0 : b0 + 1;
    if (ms < mu[0]) {
        t.a0 = -1; t.a1 = 0;
        t.wmu = (ms + 1.0) / (mu[0] + 1.0);
    } else if (ms > mu[nmu - 1]) {
        t.a0 = nmu - 1; t.a1 = nmu;
        t.wmu = (ms - mu[nmu - 1]) / (1.0 - mu[nmu - 1]);
    } else {
        int lo = 0, hi = nmu - 1;          // mu[lo] <= ms <= mu[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (ms > mu[mid]) lo = mid; else hi = mid;
        }
        t.a0 = lo; t.a1 = lo + 1;
        t.wmu = (ms - mu[lo]) / (mu[lo + 1] - mu[lo]);
    }
    return t;
}

// value of F (F[k * stride], k = a*nphi + b) at the taps
template <typename real>
__device__ __forceinline__ real angle_value(const real *__restrict__ F, long stride, int nmu, int nphi, const AngleTaps &t)
{
    auto ring = [&](int a) -> real {
        if (a < 0 || a >= nmu) {
            const int ar = (a < 0) ? 0 : nmu - 1;
            real s = 0;
            for (int b = 0; b < nphi; ++b) s += F[(long)(ar * nphi + b) * stride];
            return s / real(nphi);
        }
        const real wp = (real)t.wphi;
        return (real(1) - wp) * F[(long)(a * nphi + t.b0) * stride] + wp * F[(long)(a * nphi + t.b1) * stride];
    };
    const real wm = (real)t.wmu;
    return (real(1) - wm) * ring(t.a0) + wm * ring(t.a1);
}

// frequency bracket in ln(nu): value = wl * v[gl] + wh * v[gh]; gl/gh = -1 means 0
struct FreqTaps { int gl, gh; double wl, wh; };

__device__ __forceinline__ int centre_bracket(const double *__restrict__ lnc, int G, double x)
{
    int lo = 0, hi = G - 1;                   // lnc[lo] <= x < lnc[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (x >= lnc[mid]) lo = mid; else hi = mid;
    }
    return lo;
}

// intensity invariants: zero-valued ghost centres beyond the outer edges
__device__ __forceinline__ FreqTaps freq_taps_zero(const FreqInfo &f, double x)
{
    FreqTaps r{-1, -1, 0.0, 0.0};
    const int G = f.G;
    const double c0 = f.lnc[0], cN = f.lnc[G - 1];
    if (x < c0) {
        if (!f.has_lo_ghost) { r.gl = 0; r.wl = 1.0; return r; }
        if (x <= f.ghost_lo) return r;
        r.gl = 0; r.wl = (x - f.ghost_lo) / (c0 - f.ghost_lo);
        return r;
    }
    if (x >= cN) {
        if (x >= f.ghost_hi) return r;
        r.gl = G - 1; r.wl = (f.ghost_hi - x) / (f.ghost_hi - cN);
        return r;
    }
    const int g = centre_bracket(f.lnc, G, x);
    const double w = (x - f.lnc[g]) / (f.lnc[g + 1] - f.lnc[g]);
    r.gl = g; r.wl = 1.0 - w; r.gh = g + 1; r.wh = w;
    return r;
}

// opacities: outer values held
__device__ __forceinline__ FreqTaps freq_taps_hold(const FreqInfo &f, double x)
{
    FreqTaps r{-1, -1, 0.0, 0.0};
    const int G = f.G;
    if (x <= f.lnc[0]) { r.gl = 0; r.wl = 1.0; return r; }
    if (x >= f.lnc[G - 1]) { r.gl = G - 1; r.wl = 1.0; return r; }
    const int g = centre_bracket(f.lnc, G, x);
    const double w = (x - f.lnc[g]) / (f.lnc[g + 1] - f.lnc[g]);
    r.gl = g; r.wl = 1.0 - w; r.gh = g + 1; r.wh = w;
    return r;
}

template <typename real>
__device__ __forceinline__ bool load_beta(const real *__restrict__ beta, long p, double b[3])
{
    if (!beta) return false;
    b[0] = (double)beta[3 * p]; b[1] = (double)beta[3 * p + 1]; b[2] = (double)beta[3 * p + 2];
    return !(b[0] == 0.0 && b[1] == 0.0 && b[2] == 0.0);
}

// S3: comoving ordinates -> lab ordinates (Eqs. 7-8, invariants S/nu^3 and
// chi nu), plus the implicit time terms (Eqs. 5-6).  Thread per (point, k).
template <typename real>
__global__ void __launch_bounds__(256) k_boost(BoostArgs<real> a)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (p >= a.P) return;
    const int G = a.fi.G, K = a.K;
    double n[3] = {a.dir[4 * k], a.dir[4 * k + 1], a.dir[4 * k + 2]};
    double b[3];
    const bool moving = load_beta(a.beta, p, b);
    const real *__restrict__ S0p = a.S0 + (long)p * G * K;
    const real icdt = a.inv_cdt;
    if (!moving) {
        for (int g = 0; g < G; ++g) {
            const real Sl = S0p[(long)g * K + k];
            const real chil = a.chi0[p * G + g];
            const long o = ((long)k * G + g) * a.P + p;
            const real ip = a.Iprev ? a.Iprev[o] : real(0);
            const real xt = chil + icdt;
            a.Xt[o] = xt;
            a.St[o] = (xt > real(0)) ? (chil * Sl + ip * icdt) / xt : real(0);
        }
        return;
    }
    const double b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    const double gam = 1.0 / sqrt(1.0 - b2);
    const double bn = b[0] * n[0] + b[1] * n[1] + b[2] * n[2];
    const double D = 1.0 / (gam * (1.0 - bn));
    const double f = gam * (1.0 - gam / (gam + 1.0) * bn);
    double n0[3];
    for (int c = 0; c < 3; ++c) n0[c] = D * (n[c] - f * b[c]);
    const AngleTaps at = angle_taps(a.mu, a.nmu, a.nphi, n0);
    const double lnD = log(D);
    for (int g = 0; g < G; ++g) {
        real Sl, chil;
        if (a.fi.grey) {
            const double D2 = D * D;
            Sl = (real)(D2 * D2) * angle_value(S0p, 1, a.nmu, a.nphi, at);
            chil = (real)((double)a.chi0[p * G] / D);
        } else {
            const double x = a.fi.lnc[g] - lnD;
            const FreqTaps ft = freq_taps_zero(a.fi, x);
            double v = 0.0;
            if (ft.gl >= 0) v += ft.wl * (double)angle_value(S0p + (long)ft.gl * K, 1, a.nmu, a.nphi, at) * a.fi.inv_nu3[ft.gl];
            if (ft.gh >= 0) v += ft.wh * (double)angle_value(S0p + (long)ft.gh * K, 1, a.nmu, a.nphi, at) * a.fi.inv_nu3[ft.gh];
            Sl = (real)(a.fi.nu3[g] * v);
            const FreqTaps fc = freq_taps_hold(a.fi, x);
            double c = fc.wl * (double)a.chi0[p * G + fc.gl];
            if (fc.gh >= 0) c += fc.wh * (double)a.chi0[p * G + fc.gh];
            chil = (real)(c / D);
        }
        const long o = ((long)k * G + g) * a.P + p;
        const real ip = a.Iprev ? a.Iprev[o] : real(0);
        const real xt = chil + icdt;
        a.Xt[o] = xt;
        a.St[o] = (xt > real(0)) ? (chil * Sl + ip * icdt) / xt : real(0);
    }
}

// S5: lab ordinates -> comoving ordinates.  Thread per (point, comoving j).
template <typename real>
__global__ void __launch_bounds__(256) k_unboost(UnboostArgs<real> a)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int K = a.K, G = a.fi.G;
    if (idx >= a.P * K) return;
    const long p = idx / K;
    const int j = (int)(idx - p * K);
    double b[3];
    const bool moving = load_beta(a.beta, p, b);
    real *__restrict__ out = a.I0 + (long)p * G * K;
    const long stride = (long)G * a.P;
    if (!moving) {
        for (int g = 0; g < G; ++g) out[(long)g * K + j] = a.Ilab[((long)j * G + g) * a.P + p];
        return;
    }
    const double n0[3] = {a.dir[4 * j], a.dir[4 * j + 1], a.dir[4 * j + 2]};
    const double b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    const double gam = 1.0 / sqrt(1.0 - b2);
    const double bn0 = b[0] * n0[0] + b[1] * n0[1] + b[2] * n0[2];
    const double Dp = gam * (1.0 + bn0);
    const double f = gam * (1.0 + gam / (gam + 1.0) * bn0);
    double n[3];
    for (int c = 0; c < 3; ++c) n[c] = (n0[c] + f * b[c]) / Dp;
    const AngleTaps at = angle_taps(a.mu, a.nmu, a.nphi, n);
    if (a.fi.grey) {
        const double D2 = Dp * Dp;
        out[j] = (real)((double)angle_value(a.Ilab + p, stride, a.nmu, a.nphi, at) / (D2 * D2));
        return;
    }
    const double lnD = log(Dp);
    for (int g = 0; g < G; ++g) {
        const FreqTaps ft = freq_taps_zero(a.fi, a.fi.lnc[g] + lnD);
        double v = 0.0;
        if (ft.gl >= 0) v += ft.wl * (double)angle_value(a.Ilab + (long)ft.gl * a.P + p, stride, a.nmu, a.nphi, at) * a.fi.inv_nu3[ft.gl];
        if (ft.gh >= 0) v += ft.wh * (double)angle_value(a.Ilab + (long)ft.gh * a.P + p, stride, a.nmu, a.nphi, at) * a.fi.inv_nu3[ft.gh];
        out[(long)g * K + j] = (real)(a.fi.nu3[g] * v);
    }
}

// ---------------------------------------------------------------------------
// S2, S6: SH <-> ordinates
// ---------------------------------------------------------------------------

// S0[p][g][k] = sum_q Y[k][q] S[p][g][q]   (Yt stored [q][k])
template <typename real>
__global__ void __launch_bounds__(256) k_sh2do(long PG, int K, int NL, const real *__restrict__ Yt,
                                               const real *__restrict__ S, real *__restrict__ S0)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= PG * K) return;
    const long pg = idx / K;
    const int k = (int)(idx - pg * K);
    const real *s = S + pg * NL;
    real v = 0;
    for (int q = 0; q < NL; ++q) v += Yt[(long)q * K + k] * s[q];
    S0[idx] = v;
}

// I[p][g][q] = sum_k w_k Y[k][q] I0[p][g][k]   (WY stored [k][q])
template <typename real>
__global__ void __launch_bounds__(256) k_do2sh(long PG, int K, int NL, const real *__restrict__ WY,
                                               const real *__restrict__ I0, real *__restrict__ Ilm)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= PG * NL) return;
    const long pg = idx / NL;
    const int q = (int)(idx - pg * NL);
    const real *x = I0 + pg * K;
    real v = 0;
    for (int k = 0; k < K; ++k) v += WY[(long)k * NL + q] * x[k];
    Ilm[idx] = v;
}

// ---------------------------------------------------------------------------
// S1: source function in SH space
// ---------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(256) k_source(SourceArgs<real> a)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int G = a.G, NL = a.NL;
    if (idx >= a.P * G * NL) return;
    const int q = (int)(idx % NL);
    const long pj = idx / NL;
    const int j = (int)(pj % G);
    const long p = pj / G;
    const real chi = a.chi0[pj];
    if (!(chi > real(0))) { a.S[idx] = 0; return; }
    int l = (int)sqrtf((float)q);
    while (l * l > q) --l;
    while ((l + 1) * (l + 1) <= q) ++l;
    const real om = a.sigma[p] / chi;
    real v;
    if (!a.compton) {
        const real cl = (l == 0) ? real(1) : (l == 2 ? real(0.1) : real(0));   // chi_l/(2l+1)
        v = om * cl * a.Ilm[idx];
    } else {
        const real *__restrict__ Arow = a.A + ((long)l * G + j) * G;
        const real *__restrict__ Ip = a.Ilm + (long)p * G * NL + q;
        real s = 0;
        for (int i = 0; i < G; ++i) s += Arow[i] * Ip[(long)i * NL];
        v = om * s;
    }
    if (q == 0) v += real(3.5449077018110318) * a.kappa[pj] * a.bnu[pj] / chi;   // sqrt(4 pi) kappa B / chi
    a.S[idx] = v;
}

// chi0 = kappa + sigma * s_g
template <typename real>
__global__ void k_chi0(long P, int G, const real *__restrict__ kappa, const real *__restrict__ sigma,
                       const real *__restrict__ sg, real *__restrict__ chi0)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P * G) return;
    const long p = idx / G;
    const int g = (int)(idx - p * G);
    chi0[idx] = kappa[idx] + sigma[p] * (sg ? sg[g] : real(1));
}

// ---------------------------------------------------------------------------
// S7: moments
// ---------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(256) k_moments_lab(long P, int G, int K, const double *__restrict__ dir,
                                                     const real *__restrict__ I, double *J, double *H, double *Kt)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P * G) return;
    const int g = (int)(idx / P);
    const long p = idx - (long)g * P;
    double j = 0, h0 = 0, h1 = 0, h2 = 0, k0 = 0, k1 = 0, k2 = 0, k3 = 0, k4 = 0, k5 = 0;
    for (int k = 0; k < K; ++k) {
        const double nx = dir[4 * k], ny = dir[4 * k + 1], nz = dir[4 * k + 2], w = dir[4 * k + 3];
        const double v = w * (double)I[((long)k * G + g) * P + p];
        j += v; h0 += v * nx; h1 += v * ny; h2 += v * nz;
        k0 += v * nx * nx; k1 += v * ny * ny; k2 += v * nz * nz;
        k3 += v * nx * ny; k4 += v * nx * nz; k5 += v * ny * nz;
    }
    const double s = 1.0 / (4.0 * kPiD);
    const long o = p * G + g;
    if (J) J[o] = j * s;
    if (H) { H[3 * o] = h0 * s; H[3 * o + 1] = h1 * s; H[3 * o + 2] = h2 * s; }
    if (Kt) {
        Kt[6 * o] = k0 * s; Kt[6 * o + 1] = k1 * s; Kt[6 * o + 2] = k2 * s;
        Kt[6 * o + 3] = k3 * s; Kt[6 * o + 4] = k4 * s; Kt[6 * o + 5] = k5 * s;
    }
}

template <typename real>
__global__ void k_moments_co(long PG, int NL, int lmax, const real *__restrict__ Ilm, double *J, double *H, double *Kt)
{
    const long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= PG) return;
    const real *c = Ilm + o * NL;
    const double f4 = 4.0 * kPiD;
    const double i0 = sqrt(f4) * (double)c[0];
    double hx = 0, hy = 0, hz = 0;
    if (lmax >= 1) {
        const double s3 = sqrt(f4 / 3.0);
        hx = s3 * (double)c[3]; hy = s3 * (double)c[1]; hz = s3 * (double)c[2];
    }
    double kxx = i0 / 3.0, kyy = i0 / 3.0, kzz = i0 / 3.0, kxy = 0, kxz = 0, kyz = 0;
    if (lmax >= 2) {
        const double a20 = sqrt(16.0 * kPiD / 5.0) * (double)c[6];
        const double a22 = sqrt(16.0 * kPiD / 15.0) * (double)c[8];
        kzz = (a20 + i0) / 3.0;
        const double sxy = i0 - kzz;
        kxx = 0.5 * (sxy + a22);
        kyy = 0.5 * (sxy - a22);
        const double s15 = sqrt(f4 / 15.0);
        kxy = s15 * (double)c[4]; kxz = s15 * (double)c[7]; kyz = s15 * (double)c[5];
    }
    if (J) J[o] = i0 / f4;
    if (H) { H[3 * o] = hx / f4; H[3 * o + 1] = hy / f4; H[3 * o + 2] = hz / f4; }
    if (Kt) {
        Kt[6 * o] = kxx / f4; Kt[6 * o + 1] = kyy / f4; Kt[6 * o + 2] = kzz / f4;
        Kt[6 * o + 3] = kxy / f4; Kt[6 * o + 4] = kxz / f4; Kt[6 * o + 5] = kyz / f4;
    }
}

// ---------------------------------------------------------------------------
// S8: FP64 reductions (deterministic two-pass)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < (unsigned)s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// per block and group: sum (a-b)^2 and sum a^2 over the block's points
template <typename real>
__global__ void __launch_bounds__(256) k_resid_partial(long P, int G, int NL, const real *__restrict__ a,
                                                       const real *__restrict__ b, double *partial)
{
    __shared__ double sh[256];
    const long nthreads = (long)gridDim.x * blockDim.x;
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    for (int g = 0; g < G; ++g) {
        double dd = 0, aa = 0;
        for (long p = tid; p < P; p += nthreads) {
            const real *x = a + (p * G + g) * NL, *y = b + (p * G + g) * NL;
            for (int q = 0; q < NL; ++q) {
                const double u = (double)x[q], d = u - (double)y[q];
                dd += d * d;
                aa += u * u;
            }
        }
        dd = block_sum(dd, sh);
        aa = block_sum(aa, sh);
        if (threadIdx.x == 0) {
            partial[((long)blockIdx.x * G + g) * 2] = dd;
            partial[((long)blockIdx.x * G + g) * 2 + 1] = aa;
        }
    }
}

// five dot products for the Ng extrapolation from the chain s3 (oldest) .. s0
template <typename real>
__global__ void __launch_bounds__(256) k_ng_partial(long n, const real *__restrict__ s0, const real *__restrict__ s1,
                                                    const real *__restrict__ s2, const real *__restrict__ s3, double *partial)
{
    __shared__ double sh[256];
    double a11 = 0, a12 = 0, a22 = 0, b1 = 0, b2 = 0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double x0 = s0[i], x1 = s1[i], x2 = s2[i], x3 = s3[i];
        const double d0 = x0 - x1, d1 = x1 - x2, d2 = x2 - x3;
        const double q1 = d0 - d1, q2 = d0 - d2;
        a11 += q1 * q1; a12 += q1 * q2; a22 += q2 * q2; b1 += d0 * q1; b2 += d0 * q2;
    }
    a11 = block_sum(a11, sh); a12 = block_sum(a12, sh); a22 = block_sum(a22, sh);
    b1 = block_sum(b1, sh); b2 = block_sum(b2, sh);
    if (threadIdx.x == 0) {
        double *o = partial + (long)blockIdx.x * 5;
        o[0] = a11; o[1] = a12; o[2] = a22; o[3] = b1; o[4] = b2;
    }
}

// sum partial[nb][m] over blocks, one block per column m
__global__ void __launch_bounds__(256) k_sum_columns(int nb, int ncol, const double *__restrict__ partial, double *out)
{
    __shared__ double sh[256];
    const int c = blockIdx.x;
    double v = 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) v += partial[(long)b * ncol + c];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) out[c] = v;
}

// out = c0 * x0 + c1 * x1 + c2 * x2
template <typename real>
__global__ void k_combine3(long n, double c0, const real *__restrict__ x0, double c1, const real *__restrict__ x1,
                           double c2, const real *__restrict__ x2, real *__restrict__ out)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = (real)(c0 * (double)x0[i] + c1 * (double)x1[i] + c2 * (double)x2[i]);
}

// ---------------------------------------------------------------------------
// S9: stage combination of the four-stage time scheme (Eqs. A1-A8)
// d = R - Iin; acc = (first ? 0 : acc) + d; Iin = In + coef * d  (or, at the
// last stage, In = In + acc)
// ---------------------------------------------------------------------------
template <typename real>
__global__ void k_rk_stage(long n, const real *__restrict__ R, real *__restrict__ Iin, real *__restrict__ acc,
                           real *__restrict__ In, int first, int last, real coef)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const real d = R[i] - Iin[i];
    const real s = (first ? real(0) : acc[i]) + d;
    if (last) {
        In[i] = In[i] + s;
    } else {
        acc[i] = s;
        Iin[i] = In[i] + coef * d;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename real>
void launch_trace(const TraceArgs<real> &a, hipStream_t st)
{
    const size_t sm = 2 * sizeof(real) * (size_t)a.nx * a.ny;
    hipLaunchKernelGGL(k_trace<real>, dim3(a.K * a.G), dim3(256), sm, st, a);
}
template <typename real>
void launch_boost(const BoostArgs<real> &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_boost<real>, dim3(blocks_for(a.P, 256), a.K), dim3(256), 0, st, a);
}
template <typename real>
void launch_unboost(const UnboostArgs<real> &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_unboost<real>, dim3(blocks_for(a.P * a.K, 256)), dim3(256), 0, st, a);
}
template <typename real>
void launch_sh2do(long PG, int K, int NL, const real *Yt, const real *S, real *S0, hipStream_t st)
{
    hipLaunchKernelGGL(k_sh2do<real>, dim3(blocks_for(PG * K, 256)), dim3(256), 0, st, PG, K, NL, Yt, S, S0);
}
template <typename real>
void launch_do2sh(long PG, int K, int NL, const real *WY, const real *I0, real *Ilm, hipStream_t st)
{
    hipLaunchKernelGGL(k_do2sh<real>, dim3(blocks_for(PG * NL, 256)), dim3(256), 0, st, PG, K, NL, WY, I0, Ilm);
}
template <typename real>
void launch_source(const SourceArgs<real> &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_source<real>, dim3(blocks_for(a.P * a.G * a.NL, 256)), dim3(256), 0, st, a);
}
template <typename real>
void launch_chi0(long P, int G, const real *kappa, const real *sigma, const real *sg, real *chi0, hipStream_t st)
{
    hipLaunchKernelGGL(k_chi0<real>, dim3(blocks_for(P * G, 256)), dim3(256), 0, st, P, G, kappa, sigma, sg, chi0);
}
template <typename real>
void launch_moments_lab(long P, int G, int K, const double *dir, const real *I, double *J, double *H, double *Kt, hipStream_t st)
{
    hipLaunchKernelGGL(k_moments_lab<real>, dim3(blocks_for(P * G, 256)), dim3(256), 0, st, P, G, K, dir, I, J, H, Kt);
}
template <typename real>
void launch_moments_co(long PG, int NL, int lmax, const real *Ilm, double *J, double *H, double *Kt, hipStream_t st)
{
    hipLaunchKernelGGL(k_moments_co<real>, dim3(blocks_for(PG, 256)), dim3(256), 0, st, PG, NL, lmax, Ilm, J, H, Kt);
}
template <typename real>
void launch_resid(long P, int G, int NL, const real *a, const real *b, double *partial, int nblk, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_resid_partial<real>, dim3(nblk), dim3(256), 0, st, P, G, NL, a, b, partial);
    hipLaunchKernelGGL(k_sum_columns, dim3(2 * G), dim3(256), 0, st, nblk, 2 * G, partial, out);
}
template <typename real>
void launch_ng_dots(long n, const real *s0, const real *s1, const real *s2, const real *s3, double *partial, int nblk,
                    double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_ng_partial<real>, dim3(nblk), dim3(256), 0, st, n, s0, s1, s2, s3, partial);
    hipLaunchKernelGGL(k_sum_columns, dim3(5), dim3(256), 0, st, nblk, 5, partial, out);
}
template <typename real>
void launch_combine3(long n, double c0, const real *x0, double c1, const real *x1, double c2, const real *x2, real *out,
                     hipStream_t st)
{
    hipLaunchKernelGGL(k_combine3<real>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, c0, x0, c1, x1, c2, x2, out);
}
template <typename real>
void launch_rk_stage(long n, const real *R, real *Iin, real *acc, real *In, int first, int last, real coef, hipStream_t st)
{
    hipLaunchKernelGGL(k_rk_stage<real>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, R, Iin, acc, In, first, last, coef);
}

hipError_t set_trace_lds_limit(size_t bytes)
{
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_trace<float>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_trace<double>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

#define RRT_INSTANTIATE(real)                                                                                  \
    template void launch_trace<real>(const TraceArgs<real> &, hipStream_t);                                     \
    template void launch_boost<real>(const BoostArgs<real> &, hipStream_t);                                     \
    template void launch_unboost<real>(const UnboostArgs<real> &, hipStream_t);                                 \
    template void launch_sh2do<real>(long, int, int, const real *, const real *, real *, hipStream_t);          \
    template void launch_do2sh<real>(long, int, int, const real *, const real *, real *, hipStream_t);          \
    template void launch_source<real>(const SourceArgs<real> &, hipStream_t);                                   \
    template void launch_chi0<real>(long, int, const real *, const real *, const real *, real *, hipStream_t);  \
    template void launch_moments_lab<real>(long, int, int, const double *, const real *, double *, double *,    \
                                           double *, hipStream_t);                                              \
    template void launch_moments_co<real>(long, int, int, const real *, double *, double *, double *,           \
                                          hipStream_t);                                                         \
    template void launch_resid<real>(long, int, int, const real *, const real *, double *, int, double *,       \
                                     hipStream_t);                                                              \
    template void launch_ng_dots<real>(long, const real *, const real *, const real *, const real *, double *,  \
                                       int, double *, hipStream_t);                                             \
    template void launch_combine3<real>(long, double, const real *, double, const real *, double, const real *, \
                                        real *, hipStream_t);                                                   \
    template void launch_rk_stage<real>(long, const real *, real *, real *, real *, int, int, real, hipStream_t);

RRT_INSTANTIATE(float)
RRT_INSTANTIATE(double)

}  // namespace rrt
