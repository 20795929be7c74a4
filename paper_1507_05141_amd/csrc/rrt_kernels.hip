// HIP kernels of the source-iteration sweep (gfx950).  Templated on the
// working precision (float or double); geometry of the Lorentz maps is always
// evaluated in double, reductions are accumulated in double.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rrt_kernels.h"

namespace rrt {

static constexpr double kPiD = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// cubic Bezier formal-solution weights
// ---------------------------------------------------------------------------

// reciprocal: the hardware v_rcp_f32 (1 ulp) in FP32, exact division in FP64
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }

// With E_n(h) = int_0^h (u/h)^n e^{-u} du (u = optical distance back from the
// downwind point), the downward recurrence E_{n-1} = (h/n)(E_n + e^{-h}) adds
// positive terms only and is stable for every h.  It starts from
// E_3 = (6/h^3) P(4, h), P the regularised lower incomplete gamma function:
// for h < hs by its positive series P(4, h) = h^4 e^{-h} sum_k h^k/(k+4)!, else
// as 1 - e^{-h}(1 + h + h^2/2 + h^3/6) (at most ~4 bits of cancellation).
// The series is evaluated only when some lane of the wave needs it, and then
// selected per lane, so a wave never diverges.
template <typename real> struct BezTraits;
template <> struct BezTraits<double> {
    static constexpr double hs = 1.5;
    static constexpr int nt = 18;      // last term < 1e-16 of the first at h = hs
    // the depth cut of the multi-piece walk: e^-50 ~ 2e-22, under FP64 rounding (1.1e-16)
    // by more than five decades, also for a thousandfold brighter upwind path
    static constexpr double tau_cut = 50.0;
    __device__ static double ex(double h) { return exp(-h); }
};
template <> struct BezTraits<float> {
    static constexpr float hs = 1.5f;
    static constexpr int nt = 10;      // last term < 4e-8 of the first at h = hs
    // e^-25 ~ 1.4e-11, under FP32 rounding (6e-8) by more than three decades, also for a
    // thousandfold brighter upwind path
    static constexpr float tau_cut = 25.0f;
    __device__ static float ex(float h) { return __expf(-h); }
};

// 1/n! as a compile-time constant, and sum_{k=K}^{NT-1} h^(k-K)/(k+4)! by Horner's rule
template <int N> struct InvFact { static constexpr double v = InvFact<N - 1>::v / N; };
template <> struct InvFact<0> { static constexpr double v = 1.0; };
template <typename real, int K, int NT> struct GammaSeries {
    __device__ static real eval(real h) { return real(InvFact<K + 4>::v) + h * GammaSeries<real, K + 1, NT>::eval(h); }
};
template <typename real, int NT> struct GammaSeries<real, NT, NT> {
    __device__ static real eval(real) { return real(0); }
};

// ex = e^{-h} and the moments E_0..E_3 over optical depth [0, h].  The
// integral of the cubic Bezier source (control values S_u, C_u, C_p, S_p)
// times e^{-u} is sum_i w_i S_i with Bernstein weights w_0 = E_3,
// w_1 = 3(E_2 - E_3), w_2 = 3(E_1 - 2E_2 + E_3), w_3 = E_0 - 3E_1 + 3E_2 - E_3;
// bezier_integral regroups it by moments (forward differences of the
// control polygon).
template <typename real>
__device__ __forceinline__ void bezier_moments(real h, real &ex, real &E0, real &E1, real &E2, real &E3)
{
    using T = BezTraits<real>;
    ex = T::ex(h);
    const real ih = fast_rcp(h);
    const real poly = ((h * real(1.0 / 6.0) + real(0.5)) * h + real(1)) * h + real(1);
    E3 = real(6) * (real(1) - ex * poly) * (ih * ih * ih);
    // the series only where some lane of the wave needs it (a wave-uniform
    // branch: optically thick steps, e.g. under a time term, skip it)
    if (__any(h < T::hs)) {
        asm volatile("");       // not speculated: the branch is what saves the work
        const real e3s = real(6) * h * ex * GammaSeries<real, 0, T::nt>::eval(h);
        E3 = (h < T::hs) ? e3s : E3;
    }
    E2 = h * real(1.0 / 3.0) * (E3 + ex);
    E1 = h * real(0.5) * (E2 + ex);
    E0 = h * (E1 + ex);
}

template <typename real>
__device__ __forceinline__ real bezier_integral(real E0, real E1, real E2, real E3, real Su, real Cu, real Cp, real Sp)
{
    const real d1 = Cp - Sp, d2 = (Cu - Cp) - d1, d3 = (Su - Cu) - real(2) * (Cu - Cp) + d1;
    return E0 * Sp + real(3) * (E1 * d1 + E2 * d2) + E3 * d3;
}

// Optical-depth part of one step u -> p, shared by every group with the same
// extinction.  The Fritsch-Butland weighted harmonic-mean slope at a point
// between a left segment (source change dl over optical depth hl) and a right
// one (dr over hr), with alpha = (1 + hr/(hl + hr))/3, is
// (dl/hl)(dr/hr) / (alpha dr/hr + (1 - alpha) dl/hl); times the step depth h it
// equals n dl dr / (a dr + b dl) with a = hl (hl + 2 hr), b = hr (2 hl + hr),
// n = 3 h (hl + hr), and is zero unless dl dr > 0 and hl, hr > 0.
template <typename real>
struct StepDepth {
    real hu;                    // optical depth of the step
    real ap, bp, np;            // slope at p: left = the step, right = p -> d
    real au, bu, nu;            // slope at u: left = uu -> u, right = the step
    bool okp, oku;
    real ex, E0, E1, E2, E3;    // e^{-hu} and the Bezier moments
    real w0, w1, w2, w3;        // the Bernstein weights of S_u, C_u, C_p, S_p they give
};

template <typename real>
__device__ __forceinline__ StepDepth<real> step_depth(real hds, real Xuu, real Xu, real Xp, real Xd, bool has_d,
                                                     bool has_uu)
{
    StepDepth<real> g;
    const real hu = hds * (Xu + Xp);
    g.hu = hu;
    g.ap = g.bp = g.np = g.au = g.bu = g.nu = real(0);
    g.okp = g.oku = false;
    if (has_d) {
        const real hd = hds * (Xp + Xd);
        g.ap = hu * (hu + real(2) * hd);
        g.bp = hd * (real(2) * hu + hd);
        g.np = real(3) * hu * (hu + hd);
        g.okp = hu > real(0) && hd > real(0);
    }
    if (has_uu) {
        const real huu = hds * (Xuu + Xu);
        g.au = huu * (huu + real(2) * hu);
        g.bu = hu * (real(2) * huu + hu);
        g.nu = real(3) * hu * (huu + hu);
        g.oku = huu > real(0) && hu > real(0);
    }
    bezier_moments(hu, g.ex, g.E0, g.E1, g.E2, g.E3);
    g.w0 = g.E3;
    g.w1 = real(3) * (g.E2 - g.E3);
    g.w2 = real(3) * ((g.E1 - g.E2) - (g.E2 - g.E3));
    g.w3 = (g.E0 - g.E3) - real(3) * (g.E1 - g.E2);
    return g;
}

// step depth times the Fritsch-Butland slope from the source changes dl, dr
template <typename real>
__device__ __forceinline__ real fb_slope(real n, real a, real b, bool ok, real dl, real dr)
{
    const real prod = dl * dr;
    const real v = n * prod * fast_rcp(a * dr + b * dl);
    return (ok && prod > real(0)) ? v : real(0);
}

// periodic bilinear value of a plane stored F[(y * nx + x) * ge] (ge values
// per point, F already offset to the wanted one) at point (i, j) shifted by
// (ix + fx, iy + fy) cells; ix, iy already reduced into [0, nx), [0, ny)
template <typename real>
__device__ __forceinline__ real shifted(const real *__restrict__ F, int i, int j, int nx, int ny, int ge, int row,
                                        int ix, int iy, real fx, real fy)
{
    int i0 = i + ix; if (i0 >= nx) i0 -= nx;
    int j0 = j + iy; if (j0 >= ny) j0 -= ny;
    const int i1 = (i0 + 1 == nx) ? 0 : i0 + 1;
    const int j1 = (j0 + 1 == ny) ? 0 : j0 + 1;
    const real a = F[j0 * row + i0 * ge], b = F[j0 * row + i1 * ge], c = F[j1 * row + i0 * ge], d = F[j1 * row + i1 * ge];
    return (real(1) - fy) * ((real(1) - fx) * a + fx * b) + fy * ((real(1) - fx) * c + fx * d);
}

// ---------------------------------------------------------------------------
// launch-order helpers
// ---------------------------------------------------------------------------

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Give each XCD a contiguous range of work items so that neighbours
// (adjacent points, or the groups of one ordinate) share that XCD's L2.
__device__ __forceinline__ long xcd_item(long nitems)
{
    const long per = (nitems + 7) / 8;
    return (long)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

// ---------------------------------------------------------------------------
// frame transforms: shared geometry
// ---------------------------------------------------------------------------

struct AngleTaps {
    int a0, a1;      // ring indices; -1 = lower pole, nmu = upper pole
    int b0, b1;
    double wmu, wphi;
};

// bilinear taps of direction n on the Gauss-Legendre x uniform-azimuth mesh,
// located in precision T (the working precision: the direction itself comes
// from double-precision Lorentz maps)
template <typename T>
__device__ __forceinline__ AngleTaps angle_taps(const double *__restrict__ mu, int nmu, int nphi, const double n[3])
{
    constexpr T two_pi = T(2.0 * kPiD);
    AngleTaps t;
    const T ms = fmin(T(1), fmax(T(-1), (T)n[2]));
    T ph = atan2((T)n[1], (T)n[0]);
    if (ph < T(0)) ph += two_pi;
    const T s = ph * ((T)nphi / two_pi);
    const T sf = floor(s);
    t.wphi = (double)(s - sf);
    int b0 = (int)sf;
    if (b0 >= nphi) b0 -= nphi;
    if (b0 < 0) b0 += nphi;
    t.b0 = b0;
    t.b1 = (b0 + 1 == nphi) ? 0 : b0 + 1;
    const T mlo = (T)mu[0], mhi = (T)mu[nmu - 1];
    if (ms < mlo) {
        t.a0 = -1; t.a1 = 0;
        t.wmu = (double)((ms + T(1)) / (mlo + T(1)));
    } else if (ms > mhi) {
        t.a0 = nmu - 1; t.a1 = nmu;
        t.wmu = (double)((ms - mhi) / (T(1) - mhi));
    } else {
        int lo = 0, hi = nmu - 1;          // mu[lo] <= ms <= mu[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (ms > (T)mu[mid]) lo = mid; else hi = mid;
        }
        t.a0 = lo; t.a1 = lo + 1;
        const T m0 = (T)mu[lo];
        t.wmu = (double)((ms - m0) / ((T)mu[lo + 1] - m0));
    }
    return t;
}

// frequency bracket in ln(nu): value = wl * v[gl] + wh * v[gh]; gl/gh = -1 means 0
struct FreqTaps { int gl, gh; double wl, wh; };

// Group-centre tables staged in LDS.
struct FreqL {
    const double *lnc;      // [G] ln(centre)
    const double *inv_dc;   // [G-1] 1/(lnc[g+1]-lnc[g])
    const double *nu3;      // [G] centre^3
    const double *inv_nu3;  // [G] 1/centre^3
};

__device__ __forceinline__ int centre_bracket(const double *lnc, int G, double x)
{
    int lo = 0, hi = G - 1;                   // lnc[lo] <= x < lnc[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (x >= lnc[mid]) lo = mid; else hi = mid;
    }
    return lo;
}

// intensity invariants: zero-valued ghost centres beyond the outer edges
__device__ __forceinline__ FreqTaps freq_taps_zero(const FreqInfo &f, const FreqL &l, double x)
{
    FreqTaps r{-1, -1, 0.0, 0.0};
    const int G = f.G;
    const double c0 = l.lnc[0], cN = l.lnc[G - 1];
    if (x < c0) {
        if (!f.has_lo_ghost) { r.gl = 0; r.wl = 1.0; return r; }
        if (x <= f.ghost_lo) return r;
        r.gl = 0; r.wl = (x - f.ghost_lo) * f.inv_lo;
        return r;
    }
    if (x >= cN) {
        if (x >= f.ghost_hi) return r;
        r.gl = G - 1; r.wl = (f.ghost_hi - x) * f.inv_hi;
        return r;
    }
    const int g = centre_bracket(l.lnc, G, x);
    const double w = (x - l.lnc[g]) * l.inv_dc[g];
    r.gl = g; r.wl = 1.0 - w; r.gh = g + 1; r.wh = w;
    return r;
}

// opacities: outer values held
__device__ __forceinline__ FreqTaps freq_taps_hold(const FreqInfo &f, const FreqL &l, double x)
{
    FreqTaps r{-1, -1, 0.0, 0.0};
    const int G = f.G;
    if (x <= l.lnc[0]) { r.gl = 0; r.wl = 1.0; return r; }
    if (x >= l.lnc[G - 1]) { r.gl = G - 1; r.wl = 1.0; return r; }
    const int g = centre_bracket(l.lnc, G, x);
    const double w = (x - l.lnc[g]) * l.inv_dc[g];
    r.gl = g; r.wl = 1.0 - w; r.gh = g + 1; r.wh = w;
    return r;
}

// copy the group-centre tables into LDS (4 G doubles)
__device__ __forceinline__ FreqL stage_freq(const FreqInfo &fi, double *buf)
{
    const int G = fi.G;
    for (int g = threadIdx.x; g < G; g += blockDim.x) {
        buf[g] = fi.lnc[g];
        if (g + 1 < G) buf[G + g] = fi.inv_dc[g];
        buf[2 * G + g] = fi.nu3[g];
        buf[3 * G + g] = fi.inv_nu3[g];
    }
    return FreqL{buf, buf + G, buf + 2 * G, buf + 3 * G};
}

__device__ __forceinline__ bool load_beta(const double *__restrict__ beta, long p, double b[3])
{
    if (!beta) return false;
    b[0] = beta[3 * p]; b[1] = beta[3 * p + 1]; b[2] = beta[3 * p + 2];
    return !(b[0] == 0.0 && b[1] == 0.0 && b[2] == 0.0);
}

// lab extinction chi_lab = chi0(nu/D)/D (chi nu invariant), with
// 1/D = nu0/nu = Gamma (1 - beta.n) (Eq. 7); chi0 linear in ln(nu) between
// centres with the outer values held
template <typename real>
__device__ __forceinline__ real chi_lab_of(const real *__restrict__ chi0, long p, int g, const FreqInfo &fi,
                                           const FreqL &fl, int grey_chi, bool moving, double invD)
{
    const int G = fi.G;
    if (!moving) return chi0[p * G + g];
    if (grey_chi || fi.grey) return (real)((double)chi0[p * G + g] * invD);
    const FreqTaps fc = freq_taps_hold(fi, fl, fl.lnc[g] + log(invD));
    double c = fc.wl * (double)chi0[p * G + fc.gl];
    if (fc.gh >= 0) c += fc.wh * (double)chi0[p * G + fc.gh];
    return (real)(c * invD);
}

__device__ __forceinline__ double inv_doppler(const double b[3], double gam, const double n[3])
{
    return gam * (1.0 - (b[0] * n[0] + b[1] * n[1] + b[2] * n[2]));
}

// ---------------------------------------------------------------------------
// S4: ray trace.  One workgroup of kTraceThreads per (ordinate, chunk of GC
// groups) marches the z planes from the inflow face; each thread owns up to
// MAXPT grid points of the plane with their GC groups, which it reads and
// writes as one vector (lab arrays are [k][p][g]), so the tap addresses and a
// grey extinction are shared by the groups.  The source S~ and extinction
// chi~ of the four planes a step touches (second upwind, upwind, current,
// downwind) sit in an LDS ring, the previous intensity plane in LDS
// (overwritten by the new one once every thread has read it); the next plane
// is fetched into registers while the current one is computed.
// LDS planes carry a one-column and one-row periodic halo (row stride nx + 1)
// so that the bilinear taps need no wrap.  chi~ = chi_lab + 1/(c dt) with
// chi_lab precomputed per medium (one value per point when it is grey) or read
// from an array for the stand-alone entry point (XMODE: kChiGrey, kChiGroup,
// kChiArray).  With a grey chi~ the optical depths, slope coefficients and
// Bezier moments of a point are computed once for its GC groups.
// ---------------------------------------------------------------------------
constexpr int kChiGrey = 0, kChiGroup = 1, kChiArray = 2;

template <typename real, int N>
struct alignas(sizeof(real) * N) Pack {
    real v[N];
};
// a store that does not keep its lines in the caches, for lab-frame arrays that the
// next step reads back only after far more data than the caches hold (measured at
// 64^3: the boost's S~ 13.6 -> 13.3 ms, the transpose back to point-major planes 7.0
// -> 6.2 ms, the inverse transform 8.65 -> 8.5 ms; the SH -> ordinate product and
// the ray trace gain nothing or lose)
// a 16-byte load that does not keep its line in the caches, for lab-frame arrays read
// once per step (measured at 64^3: the boost's stage input 13.2 -> 12.5 ms, the inverse
// transform's lab intensities 8.55 -> 8.0 ms, the transposes 0.1 ms each)
template <typename real>
__device__ __forceinline__ Pack<real, 4> load_stream(const real *src)
{
    typedef real v4 __attribute__((ext_vector_type(4)));
    const v4 x = __builtin_nontemporal_load(reinterpret_cast<const v4 *>(src));
    Pack<real, 4> w;
#pragma unroll
    for (int i = 0; i < 4; ++i) w.v[i] = x[i];
    return w;
}
template <typename real, int N>
__device__ __forceinline__ void store_stream(real *dst, const Pack<real, N> &w)
{
    if constexpr (N == 1) {
        __builtin_nontemporal_store(w.v[0], dst);
    } else {
        typedef real vN __attribute__((ext_vector_type(N)));
        vN x;
#pragma unroll
        for (int i = 0; i < N; ++i) x[i] = w.v[i];
        __builtin_nontemporal_store(x, reinterpret_cast<vN *>(dst));
    }
}


template <typename real, int GC, int MAXPT>
struct PlaneRegs {
    Pack<real, GC> s[MAXPT], x[MAXPT];      // x[c].v[0] only when chi~ is grey
};

// (i, j) of plane point pe without an integer division: (pe + 1/2)/nx in FP32
// is within 1e-3 of its exact value for planes up to 2^12 points, far from the
// next integer
__device__ __forceinline__ void plane_ij(int pe, int nx, float rnx, int &i, int &j)
{
    j = (int)(((float)pe + 0.5f) * rnx);
    i = pe - j * nx;
}

struct TraceIdx {
    int nx, ny, PL, RS, PS;     // plane sizes; LDS row stride and plane size (with halo)
    float rnx;                  // 1/nx
};

// global -> registers: S~ and chi (raw) of plane m for this thread's points.
// Threads past the end of the plane load its last point (never stored), so
// the loads are unconditional and stay in flight until the values are stored.
// planes of S~ and chi~ kept in LDS (the stencil's four) and intensity planes.
// (A fifth slot and a second intensity plane, for one barrier per plane instead
// of two, made the 32^3 trace 1.7x slower: 143 KB of LDS against 96 KB.)
constexpr int kRing = 4;
constexpr int kIBuf = 1;

// a thread's points, computed once: plane index e (clamped to the last point, for
// unconditional loads), its offset e ps in a lab plane, its LDS cell and whether it
// also fills the halo column (i = 0) or row (j = 0)
template <int MAXPT>
struct PointSlots {
    int e[MAXPT], eo[MAXPT], cell[MAXPT];
    bool i0[MAXPT], j0[MAXPT], in[MAXPT];
};

// plane m of S~ and chi~ into registers; ps = stride between points (G, or 1 on group-major planes)
template <typename real, int XMODE, int GC, int MAXPT>
__device__ __forceinline__ void trace_fetch(PlaneRegs<real, GC, MAXPT> &r, const real *__restrict__ Sk,
                                            const real *__restrict__ Xk, int ps, int PL, int m,
                                            const PointSlots<MAXPT> &ps_)
{
    using P = Pack<real, GC>;
    const real *__restrict__ Sp = Sk + (long)m * PL * ps;           // the plane's start (uniform)
    const real *__restrict__ Xp = XMODE == kChiGrey ? Xk + (long)m * PL : Xk + (long)m * PL * ps;
#pragma unroll
    for (int c = 0; c < MAXPT; ++c) {
        r.s[c] = *reinterpret_cast<const P *>(Sp + ps_.eo[c]);
        if (XMODE == kChiGrey) r.x[c].v[0] = Xp[ps_.e[c]];
        else r.x[c] = *reinterpret_cast<const P *>(Xp + ps_.eo[c]);
    }
}

// value v of a point into an LDS plane at its cell, and into the periodic halo
// column / row where the point is at i = 0 / j = 0
template <typename T>
__device__ __forceinline__ void lds_put_at(T *pl, const TraceIdx &q, int cell, bool i0, bool j0, const T v)
{
    pl[cell] = v;
    if (i0) pl[cell + q.nx] = v;
    if (j0) {
        pl[cell + q.ny * q.RS] = v;
        if (i0) pl[cell + q.ny * q.RS + q.nx] = v;
    }
}

// registers -> the LDS ring slot of plane t; chi~ = chi + add (the time term)
template <typename real, int XMODE, int GC, int MAXPT>
__device__ __forceinline__ void trace_store(const PlaneRegs<real, GC, MAXPT> &r, real *Sr, real *Xr,
                                            const TraceIdx &q, int t, real add, const PointSlots<MAXPT> &ps_)
{
    constexpr bool xg = XMODE == kChiGrey;
    using P = Pack<real, GC>;
    const int slot = t % kRing;
    P *Sd = reinterpret_cast<P *>(Sr + slot * q.PS * GC);
#pragma unroll
    for (int c = 0; c < MAXPT; ++c) {
        if (ps_.in[c]) {
            lds_put_at(Sd, q, ps_.cell[c], ps_.i0[c], ps_.j0[c], r.s[c]);
            if (xg) {
                lds_put_at(Xr + slot * q.PS, q, ps_.cell[c], ps_.i0[c], ps_.j0[c], r.x[c].v[0] + add);
            } else {
                P x = r.x[c];
#pragma unroll
                for (int n = 0; n < GC; ++n) x.v[n] += add;
                lds_put_at(reinterpret_cast<P *>(Xr + slot * q.PS * GC), q, ps_.cell[c], ps_.i0[c], ps_.j0[c], x);
            }
        }
    }
}

// bilinear value of GC groups from an LDS plane with halo: tap cell, row stride RS
template <typename real, int N>
__device__ __forceinline__ Pack<real, N> bil(const Pack<real, N> *pl, int cell, int RS, const real w[4])
{
    const Pack<real, N> a = pl[cell], b = pl[cell + 1], c = pl[cell + RS], d = pl[cell + RS + 1];
    Pack<real, N> r;
#pragma unroll
    for (int n = 0; n < N; ++n) r.v[n] = w[0] * a.v[n] + w[1] * b.v[n] + w[2] * c.v[n] + w[3] * d.v[n];
    return r;
}

// x clamped to the interval between a and b (one median-of-three in FP32)
__device__ __forceinline__ float clamp_between(float x, float a, float b) { return __builtin_amdgcn_fmed3f(x, a, b); }
__device__ __forceinline__ double clamp_between(double x, double a, double b)
{
    return fmin(fmax(x, fmin(a, b)), fmax(a, b));
}

// LDS cell of the tap of point (i, j) at table offset t (periodic wrap; the
// plane's halo serves the + 1 neighbours)
template <typename T>
__device__ __forceinline__ int tap_cell(const T &t, int i, int j, const TraceIdx &q)
{
    int i0 = i + t.ix; if (i0 >= q.nx) i0 -= q.nx;
    int j0 = j + t.iy; if (j0 >= q.ny) j0 -= q.ny;
    return j0 * q.RS + i0;
}

// value at a path point between grid planes A (the nearer) and B: bilinear
// on each, linear in z, with the eight combined weights of its tap
template <typename real, int N>
__device__ __forceinline__ Pack<real, N> bil2(const Pack<real, N> *A, const Pack<real, N> *B, int cell, int RS,
                                              const real w[8])
{
    const Pack<real, N> a0 = A[cell], a1 = A[cell + 1], a2 = A[cell + RS], a3 = A[cell + RS + 1];
    const Pack<real, N> b0 = B[cell], b1 = B[cell + 1], b2 = B[cell + RS], b3 = B[cell + RS + 1];
    Pack<real, N> r;
#pragma unroll
    for (int n = 0; n < N; ++n)
        r.v[n] = w[0] * a0.v[n] + w[1] * a1.v[n] + w[2] * a2.v[n] + w[3] * a3.v[n] + w[4] * b0.v[n] +
                 w[5] * b1.v[n] + w[6] * b2.v[n] + w[7] * b3.v[n];
    return r;
}

// Fritsch-Butland slope dS/dtau at a path point from its left segment (source
// change dl over optical depth hl) and right segment (dr over hr), with the
// depth coefficients of slope_coef: 3 (hl + hr) dl dr / (a dr + b dl), zero
// unless dl dr > 0 and both depths are positive
template <typename real>
struct SlopeCoef {
    real a, b, n;
    bool ok;
};
template <typename real>
__device__ __forceinline__ SlopeCoef<real> slope_coef(real hl, real hr)
{
    SlopeCoef<real> c;
    c.a = hl * (hl + real(2) * hr);
    c.b = hr * (real(2) * hl + hr);
    c.n = real(3) * (hl + hr);
    c.ok = hl > real(0) && hr > real(0);
    return c;
}
template <typename real>
__device__ __forceinline__ real fb_dtau(const SlopeCoef<real> &c, real dl, real dr)
{
    const real prod = dl * dr;
    const real v = c.n * prod * fast_rcp(c.a * dr + c.b * dl);
    return (c.ok && prod > real(0)) ? v : real(0);
}

// One cubic Bezier step u -> p over every group of the pack: the intensity
// arriving from u is attenuated by e^{-h} and the integral of the source
// added; slopes from the neighbours uu and d where they exist (has_uu,
// has_d), else the secant.
template <typename real, int XMODE, int GC>
__device__ __forceinline__ void bezier_step(Pack<real, GC> &I, real hds, const Pack<real, GC> &Suu,
                                            const Pack<real, GC> &Su, const Pack<real, GC> &Sp,
                                            const Pack<real, GC> &Sd,
                                            const Pack<real, XMODE == kChiGrey ? 1 : GC> &Xuu,
                                            const Pack<real, XMODE == kChiGrey ? 1 : GC> &Xu,
                                            const Pack<real, XMODE == kChiGrey ? 1 : GC> &Xp,
                                            const Pack<real, XMODE == kChiGrey ? 1 : GC> &Xd, bool has_d, bool has_uu)
{
    constexpr bool xg = XMODE == kChiGrey;
    constexpr int XG = xg ? 1 : GC;
    StepDepth<real> gd;
    if (xg) gd = step_depth(hds, Xuu.v[0], Xu.v[0], Xp.v[0], Xd.v[0], has_d, has_uu);
#pragma unroll
    for (int n = 0; n < GC; ++n) {
        if (!xg) gd = step_depth(hds, Xuu.v[n % XG], Xu.v[n % XG], Xp.v[n % XG], Xd.v[n % XG], has_d, has_uu);
        const real sp = Sp.v[n], su = Su.v[n];
        const real dl = sp - su;
        // step depth times the slopes at p and at u (secant where the outer neighbour is missing)
        const real tp = has_d ? fb_slope(gd.np, gd.ap, gd.bp, gd.okp, dl, Sd.v[n] - sp) : dl;
        const real tu = has_uu ? fb_slope(gd.nu, gd.au, gd.bu, gd.oku, su - Suu.v[n], dl) : dl;
        const real Cu = clamp_between(su + tu * real(1.0 / 3.0), su, sp);
        const real Cp = clamp_between(sp - tp * real(1.0 / 3.0), su, sp);
        // a grey extinction shares the step's weights among the groups: the integral is
        // then four products per group; otherwise the moment form (fewer operations
        // for one group)
        I.v[n] = xg ? I.v[n] * gd.ex + gd.w0 * su + gd.w1 * Cu + gd.w2 * Cp + gd.w3 * sp
                    : I.v[n] * gd.ex + bezier_integral(gd.E0, gd.E1, gd.E2, gd.E3, su, Cu, Cp, sp);
    }
}

template <typename real, int XMODE, int GC, int MAXPT, bool MULTI>
__global__ void __launch_bounds__(kTraceThreads) k_trace(TraceArgs<real> a, int rank0, int nrank)
{
    using P = Pack<real, GC>;
    using PX = Pack<real, XMODE == kChiGrey ? 1 : GC>;
    constexpr int T = kTraceThreads;
    constexpr bool xg = XMODE == kChiGrey;
    constexpr int XG = xg ? 1 : GC;
    extern __shared__ unsigned char smem_raw[];
    const int nx = a.nx, ny = a.ny, nz = a.nz, PL = nx * ny, G = a.G;
    const int nch = G / GC;
    // Block b runs on XCD b % 8.  Each XCD takes every eighth ordinate of the
    // list ordered by decreasing cost, and all group chunks of an ordinate in a
    // row (they share the cache lines of its points), so the XCDs get equal work
    // and the longest marches start first.
    const int xcd = blockIdx.x % 8;
    const long slot = blockIdx.x / 8;
    const int rank = 8 * (int)(slot / nch) + xcd;
    if (rank >= nrank) return;
    const int k = a.order[rank0 + rank], g0 = (int)(slot % nch) * GC;
    const TraceIdx q{nx, ny, PL, nx + 1, (nx + 1) * (ny + 1), 1.0f / (float)nx};
    const int XE = q.PS * XG;
    real *Sr = reinterpret_cast<real *>(smem_raw);
    real *Xr = Sr + kRing * q.PS * GC;
    P *Ir = reinterpret_cast<P *>(Xr + kRing * XE);   // kIBuf planes of PS points
    const OrdGeom gm = a.geo[k];
    // tp[c]: path point c = -1 .. npc + 1, read through the constant address
    // space so that the (uniform) taps load into scalar registers
    const __attribute__((address_space(4))) PathTap<real> *tp =
        (const __attribute__((address_space(4))) PathTap<real> *)(a.taps + gm.tap0 + 1);
    const int npc = gm.npc;
    // start of this ordinate's lab slab (+ chunk) and the stride between points
    const long slab = a.gmajor ? ((long)k * G + g0) * a.P : (long)k * a.P * G + g0;
    const int ps = a.gmajor ? 1 : G;
    const real *__restrict__ Sk = a.St + slab;
    const real *__restrict__ Xk = XMODE == kChiArray ? a.Xt + slab
                                : (XMODE == kChiGrey ? a.chilab + (long)k * a.P : a.chilab + slab);
    real *__restrict__ Ik = a.I + slab;
    const int tid = threadIdx.x;
    PlaneRegs<real, GC, MAXPT> rg;

    // plane position of each point, its LDS cell and, for one piece per
    // plane, the cells of its three bilinear taps (second upwind, upwind,
    // downwind): the same on every plane
    int pi[MAXPT], pj[MAXPT], self[MAXPT], cell[MAXPT][3];
    PointSlots<MAXPT> pts;
#pragma unroll
    for (int c = 0; c < MAXPT; ++c) {
        const int e = min(tid + c * T, PL - 1);
        plane_ij(e, nx, q.rnx, pi[c], pj[c]);
        self[c] = pj[c] * q.RS + pi[c];
        cell[c][0] = tap_cell(tp[2], pi[c], pj[c], q);
        cell[c][1] = tap_cell(tp[1], pi[c], pj[c], q);
        cell[c][2] = tap_cell(tp[-1], pi[c], pj[c], q);
        pts.e[c] = e;
        pts.eo[c] = e * ps;
        pts.cell[c] = self[c];
        pts.i0[c] = pi[c] == 0;
        pts.j0[c] = pj[c] == 0;
        pts.in[c] = tid + c * T < PL;
    }

    const real add = XMODE == kChiArray ? real(0) : a.inv_cdt;   // the stand-alone chi~ already holds it
    for (int t = 0; t < nz && t < 3; ++t) {
        trace_fetch<real, XMODE, GC, MAXPT>(rg, Sk, Xk, ps, PL, gm.up ? t : nz - 1 - t, pts);
        trace_store<real, XMODE, GC, MAXPT>(rg, Sr, Xr, q, t, add, pts);
    }
    {
        const int m0 = gm.up ? 0 : nz - 1;
        const real *__restrict__ bc = gm.up ? a.bc_bot : a.bc_top;
#pragma unroll
        for (int c = 0; c < MAXPT; ++c) {
            const int pe = tid + c * T;
            if (pe >= PL) break;
            P v;
            if (bc) {
                v = *reinterpret_cast<const P *>(bc + ((long)k * PL + pe) * G + g0);
            } else {
#pragma unroll
                for (int n = 0; n < GC; ++n) v.v[n] = real(0);
            }
            lds_put_at(Ir, q, pts.cell[c], pts.i0[c], pts.j0[c], v);
            *reinterpret_cast<P *>(Ik + (long)m0 * PL * ps + pts.eo[c]) = v;
        }
    }
    __syncthreads();
    const real hds = real(0.5) * (real)gm.ds;
    // Under a time term every piece is at least 2 hds / (c dt) deep (chi~ >= 1/(c dt)):
    // what enters the path more than tau_cut before p arrives attenuated below
    // e^-tau_cut, under the working precision's resolution, so the walk starts at
    // path point c0, the nearest at least that deep, with I = S~ there (c0 = npc:
    // the whole path).  An extinction array may be thin: no cut.
    int c0 = npc;
    if (MULTI && XMODE != kChiArray && add > real(0)) {
        const real tmin = real(2) * hds * add;
        if (tmin * (real)npc > BezTraits<real>::tau_cut)
            c0 = max(1, min(npc, (int)ceil(BezTraits<real>::tau_cut / tmin)));
    }
    // one piece per plane: second upwind, upwind and downwind taps (each on a grid plane)
    real wts[3][4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        wts[0][n] = tp[2].w[4 + n];
        wts[1][n] = tp[1].w[n];
        wts[2][n] = tp[-1].w[4 + n];
    }
    const int RS = q.RS;
    for (int t = 1; t < nz; ++t) {
        if (t + 2 < nz) trace_fetch<real, XMODE, GC, MAXPT>(rg, Sk, Xk, ps, PL, gm.up ? t + 2 : nz - 3 - t, pts);
        const int m = gm.up ? t : nz - 1 - t;
        real *__restrict__ Iplane = Ik + (long)m * PL * ps;            // this plane's intensities (uniform)
        const bool has_d = t <= nz - 2, has_uu = t >= 2;
        const int sp0 = t % kRing, su0 = (t + kRing - 1) % kRing, suu0 = (t + kRing - 2) % kRing,
                  sd0 = (t + 1) % kRing;
        const P *Spl = reinterpret_cast<const P *>(Sr + sp0 * q.PS * GC);
        const P *Sul = reinterpret_cast<const P *>(Sr + su0 * q.PS * GC);
        const P *Suul = reinterpret_cast<const P *>(Sr + suu0 * q.PS * GC);
        const P *Sdl = reinterpret_cast<const P *>(Sr + sd0 * q.PS * GC);
        const PX *Xpl = reinterpret_cast<const PX *>(Xr + sp0 * XE);
        const PX *Xul = reinterpret_cast<const PX *>(Xr + su0 * XE);
        const PX *Xuul = reinterpret_cast<const PX *>(Xr + suu0 * XE);
        const PX *Xdl = reinterpret_cast<const PX *>(Xr + sd0 * XE);
        const P *Iul = Ir;
        P res[MAXPT];
        if (!MULTI) {
            // one piece: the plane-to-plane step, every tap on a grid plane
#pragma unroll
            for (int c = 0; c < MAXPT; ++c) {
                const int cp = self[c], cu = cell[c][1], cd = cell[c][2], cuu = cell[c][0];
                const P Sp = Spl[cp], Su = bil(Sul, cu, RS, wts[1]);
                P Iu = bil(Iul, cu, RS, wts[1]);
                P Sd, Suu;
                PX Xd, Xuu;
                const PX Xp = Xpl[cp], Xu = bil(Xul, cu, RS, wts[1]);
                if (has_d) {
                    Sd = bil(Sdl, cd, RS, wts[2]);
                    Xd = bil(Xdl, cd, RS, wts[2]);
                }
                if (has_uu) {
                    Suu = bil(Suul, cuu, RS, wts[0]);
                    Xuu = bil(Xuul, cuu, RS, wts[0]);
                }
                bezier_step<real, XMODE, GC>(Iu, hds, Suu, Su, Sp, Sd, Xuu, Xu, Xp, Xd, has_d, has_uu);
                res[c] = Iu;
                if (pts.in[c]) *reinterpret_cast<P *>(Iplane + pts.eo[c]) = res[c];
            }
        } else {
            // npc pieces: the intensity at the upwind point u = path point npc is
            // carried to p = path point 0 piece by piece.  Path point c lies
            // between grid planes (bilinear on each, linear in z); the
            // Fritsch-Butland slope at a path point serves the piece that ends
            // there and the one that starts there.
#pragma unroll
            for (int c = 0; c < MAXPT; ++c) {
                // cells left before the periodic wrap in x and y
                const int rx = nx - pi[c], ry = ny - pj[c];
                P Sup2, Sup, Scur, Sdn;          // path points c + 2, c + 1, c, c - 1 of the walk
                PX Xup2, Xup, Xcur, Xdn;
                real w[8];
                // the tap cell of path point pc: the point's own cell moved by the (uniform)
                // offset, wrapped where it passes the plane's edge (as tap_cell)
                auto taps_of = [&](int pc) {
#pragma unroll
                    for (int n = 0; n < 8; ++n) w[n] = tp[pc].w[n];
                    const int ix = tp[pc].ix, iy = tp[pc].iy;
                    int cl = self[c] + (ix + iy * RS);
                    if (ix >= rx) cl -= nx;
                    if (iy >= ry) cl -= ny * RS;
                    return cl;
                };
                P I;
                if (c0 == npc) {
                    if (has_uu) {                // path point npc + 1: one piece beyond u
                        const int cl = taps_of(npc + 1);
                        Sup2 = bil2(Sul, Suul, cl, RS, w);
                        Xup2 = bil2(Xul, Xuul, cl, RS, w);
                    }
                    const int cl = taps_of(npc);  // path point npc: u on the upwind plane
                    Sup = bil(Sul, cl, RS, w);
                    Xup = bil(Xul, cl, RS, w);
                    I = bil(Iul, cl, RS, w);
                } else {
                    // the walk starts inside the path (c0 < npc): path points c0 + 1 and
                    // c0 between the planes (c0 + 1 on the upwind plane when it is npc)
                    int cl = taps_of(c0 + 1);
                    if (c0 + 1 == npc) {
                        Sup2 = bil(Sul, cl, RS, w);
                        Xup2 = bil(Xul, cl, RS, w);
                    } else {
                        Sup2 = bil2(Spl, Sul, cl, RS, w);
                        Xup2 = bil2(Xpl, Xul, cl, RS, w);
                    }
                    cl = taps_of(c0);
                    Sup = bil2(Spl, Sul, cl, RS, w);
                    Xup = bil2(Xpl, Xul, cl, RS, w);
                    I = Sup;
                }
                if (c0 >= 2) {                   // path point c0 - 1
                    const int cl = taps_of(c0 - 1);
                    Scur = bil2(Spl, Sul, cl, RS, w);
                    Xcur = bil2(Xpl, Xul, cl, RS, w);
                } else {
                    Scur = Spl[self[c]];
                    Xcur = Xpl[self[c]];
                }
                // depths of the piece before u and of the first piece (per group unless grey)
                PX hup, hcur;
#pragma unroll
                for (int n = 0; n < XG; ++n) {
                    hup.v[n] = hds * (Xup2.v[n] + Xup.v[n]);
                    hcur.v[n] = hds * (Xcur.v[n] + Xup.v[n]);
                }
                // slope at u (dS/dtau); unused without the piece before it
                P sup;
                {
                    SlopeCoef<real> sc;
                    if (xg) sc = slope_coef(hup.v[0], hcur.v[0]);
#pragma unroll
                    for (int n = 0; n < GC; ++n) {
                        if (!xg) sc = slope_coef(hup.v[n % XG], hcur.v[n % XG]);
                        sup.v[n] = fb_dtau(sc, Sup.v[n] - Sup2.v[n], Scur.v[n] - Sup.v[n]);
                    }
                }
#pragma unroll 1
                for (int pc = c0 - 1; pc >= 0; --pc) {
                    // piece from path point pc + 1 to pc; the next path point pc - 1
                    const bool pd = pc >= 1 || has_d, puu = pc + 2 <= npc || has_uu;
                    if (pc >= 2) {
                        const int cl = taps_of(pc - 1);
                        Sdn = bil2(Spl, Sul, cl, RS, w);
                        Xdn = bil2(Xpl, Xul, cl, RS, w);
                    } else if (pc == 1) {
                        Sdn = Spl[self[c]];
                        Xdn = Xpl[self[c]];
                    } else if (has_d) {          // path point -1: one piece beyond p
                        const int cl = taps_of(-1);
                        Sdn = bil2(Spl, Sdl, cl, RS, w);
                        Xdn = bil2(Xpl, Xdl, cl, RS, w);
                    }
                    PX hdn;
#pragma unroll
                    for (int n = 0; n < XG; ++n) hdn.v[n] = hds * (Xcur.v[n] + Xdn.v[n]);
                    P scur;                       // slope at path point pc
                    real ex = real(0), E0 = real(0), E1 = real(0), E2 = real(0), E3 = real(0);
                    real bw0 = real(0), bw1 = real(0), bw2 = real(0), bw3 = real(0);
                    SlopeCoef<real> sc;
                    if (xg) {
                        // a grey extinction shares the piece's Bernstein weights among the groups
                        sc = slope_coef(hcur.v[0], hdn.v[0]);
                        bezier_moments(hcur.v[0], ex, E0, E1, E2, E3);
                        bw0 = E3;
                        bw1 = real(3) * (E2 - E3);
                        bw2 = real(3) * ((E1 - E2) - (E2 - E3));
                        bw3 = (E0 - E3) - real(3) * (E1 - E2);
                    }
#pragma unroll
                    for (int n = 0; n < GC; ++n) {
                        if (!xg) {
                            sc = slope_coef(hcur.v[n % XG], hdn.v[n % XG]);
                            bezier_moments(hcur.v[n % XG], ex, E0, E1, E2, E3);
                        }
                        const real h = hcur.v[n % XG];
                        const real su = Sup.v[n], sp = Scur.v[n];
                        const real dl = sp - su;
                        scur.v[n] = fb_dtau(sc, dl, Sdn.v[n] - sp);
                        // step depth times the slopes at p and at u (secant where the outer neighbour is missing)
                        const real tp_ = pd ? h * scur.v[n] : dl;
                        const real tu_ = puu ? h * sup.v[n] : dl;
                        const real Cu = clamp_between(su + tu_ * real(1.0 / 3.0), su, sp);
                        const real Cp = clamp_between(sp - tp_ * real(1.0 / 3.0), su, sp);
                        I.v[n] = xg ? I.v[n] * ex + bw0 * su + bw1 * Cu + bw2 * Cp + bw3 * sp
                                    : I.v[n] * ex + bezier_integral(E0, E1, E2, E3, su, Cu, Cp, sp);
                    }
                    Sup = Scur; Scur = Sdn; sup = scur;
                    Xcur = Xdn; hcur = hdn;
                }
                res[c] = I;
                if (pts.in[c]) *reinterpret_cast<P *>(Iplane + pts.eo[c]) = res[c];
            }
        }
        __syncthreads();
        // every read of plane t - 1 is done: the intensity plane and the slot of
        // plane t - 2 can be overwritten
#pragma unroll
        for (int c = 0; c < MAXPT; ++c)
            if (pts.in[c]) lds_put_at(Ir, q, pts.cell[c], pts.i0[c], pts.j0[c], res[c]);
        if (t + 2 < nz) trace_store<real, XMODE, GC, MAXPT>(rg, Sr, Xr, q, t + 2, add, pts);
        __syncthreads();
    }
}

// Monotone walk of the centre bracket: x increases with g for a fixed ray, so
// the bracket of group g + 1 is found by advancing from that of group g.
struct FreqWalk {
    int lo;
};

// intensity invariants: zero-valued ghost centres beyond the outer edges
__device__ __forceinline__ FreqTaps freq_taps_zero_walk(const FreqInfo &f, const FreqL &l, double x, FreqWalk &w)
{
    FreqTaps r{-1, -1, 0.0, 0.0};
    const int G = f.G;
    const double c0 = l.lnc[0], cN = l.lnc[G - 1];
    if (x < c0) {
        if (!f.has_lo_ghost) { r.gl = 0; r.wl = 1.0; return r; }
        if (x <= f.ghost_lo) return r;
        r.gl = 0; r.wl = (x - f.ghost_lo) * f.inv_lo;
        return r;
    }
    if (x >= cN) {
        if (x >= f.ghost_hi) return r;
        r.gl = G - 1; r.wl = (f.ghost_hi - x) * f.inv_hi;
        return r;
    }
    int g = w.lo;
    while (g + 2 < G && x >= l.lnc[g + 1]) ++g;
    w.lo = g;
    const double wt = (x - l.lnc[g]) * l.inv_dc[g];
    r.gl = g; r.wl = 1.0 - wt; r.gh = g + 1; r.wh = wt;
    return r;
}

// ---------------------------------------------------------------------------
// Frame transforms (S3, S5).  One workgroup per grid point stages that point's
// values in an LDS table F[r][c]: row r = g + 1 for group g, rows 0 and G + 1
// zero (the ghost centres beyond the outer edges); column c < K an ordinate,
// c = K / K + 1 the azimuthal mean of the lowest / highest polar ring (the
// pole values); row stride KS = (K + 2) | 1, odd, so that writing a column
// hits distinct banks.  A direction's bilinear taps become four columns with
// combined weights, the same for every group.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int table_stride(int K) { return (K + 2) | 1; }

template <typename real> struct Taps4 {
    int c[4];
    real w[4];
};

template <typename real>
__device__ __forceinline__ Taps4<real> taps4(const AngleTaps &t, int K, int nmu, int nphi)
{
    auto col = [&](int ring, int b) { return ring < 0 ? K : (ring >= nmu ? K + 1 : ring * nphi + b); };
    Taps4<real> r;
    r.c[0] = col(t.a0, t.b0); r.c[1] = col(t.a0, t.b1);
    r.c[2] = col(t.a1, t.b0); r.c[3] = col(t.a1, t.b1);
    const double um = 1.0 - t.wmu, up = 1.0 - t.wphi;
    r.w[0] = (real)(um * up); r.w[1] = (real)(um * t.wphi);
    r.w[2] = (real)(t.wmu * up); r.w[3] = (real)(t.wmu * t.wphi);
    return r;
}

template <typename real>
__device__ __forceinline__ real tap_row(const real *row, const Taps4<real> &t)
{
    return t.w[0] * row[t.c[0]] + t.w[1] * row[t.c[1]] + t.w[2] * row[t.c[2]] + t.w[3] * row[t.c[3]];
}

// pole columns of rows 1..G: azimuthal means of the lowest and highest ring
template <typename real>
__device__ __forceinline__ void table_poles(real *F, int G, int K, int KS, int nmu, int nphi)
{
    for (int i = threadIdx.x; i < 2 * G; i += blockDim.x) {
        const int g = i >> 1, top = i & 1;
        const real *row = F + (g + 1) * KS + (top ? (nmu - 1) * nphi : 0);
        real s = 0;
        for (int b = 0; b < nphi; ++b) s += row[b];
        F[(g + 1) * KS + K + top] = s / real(nphi);
    }
}

// zero the ghost rows 0 and G + 1
template <typename real>
__device__ __forceinline__ void table_ghosts(real *F, int G, int KS)
{
    for (int i = threadIdx.x; i < KS; i += blockDim.x) {
        F[i] = real(0);
        F[(G + 1) * KS + i] = real(0);
    }
}

// Frequency remap for groups uniform in ln(nu) (spacing delta): the target
// frequency of group g sits at fractional group position g + y for every g, so
// the invariant F/nu^3 is interpolated between groups g + s and g + s + 1
// (s = floor y, weight f = y - s), positions beyond the groups reading the
// zero ghost rows, and nu_g^3 / nu_{g'}^3 = exp(3 delta (g - g')): the value of
// group g is clo A(g + s) + chi A(g + s + 1), A the angle remap of a table row.
// In FP32 the exponent is capped at 80 so that a factor multiplying a ghost
// stays finite (only a group set spanning more than ~12 decades reaches the cap).
template <typename real>
__device__ __forceinline__ void uniform_shift(double y, double delta, int G, int &s, real &clo, real &chi)
{
    const double sf = floor(y);
    if (sf <= -(double)(G + 1) || sf >= (double)G) {      // every position beyond the groups
        s = kAllGhost; clo = real(0); chi = real(0);
        return;
    }
    const real f = (real)(y - sf);
    const real cap = sizeof(real) == 4 ? real(80) : real(700);
    const real e3 = real(-3.0 * delta);
    s = (int)sf;
    clo = (real(1) - f) * exp(fmin(e3 * (real)sf, cap));
    chi = f * exp(fmin(e3 * (real)(sf + 1.0), cap));
}

// remap of every group for non-uniform groups: frequency x = ln(nu_g) + lnD
// bracketed by a monotone walk, invariants F/nu^3 linear in ln(nu)
template <typename real>
__device__ __forceinline__ void general_remap(const real *F, int KS, const FreqInfo &fi, const FreqL &fl,
                                              const Taps4<real> &tp, double lnD, real *out, long ostride)
{
    const int G = fi.G;
    FreqWalk fw{0};
    if (G > 2) fw.lo = centre_bracket(fl.lnc, G, fl.lnc[0] + lnD);
    for (int g = 0; g < G; ++g) {
        const FreqTaps ft = freq_taps_zero_walk(fi, fl, fl.lnc[g] + lnD, fw);
        double v = 0.0;
        if (ft.gl >= 0) v += ft.wl * (double)tap_row(F + (ft.gl + 1) * KS, tp) * fl.inv_nu3[ft.gl];
        if (ft.gh >= 0) v += ft.wh * (double)tap_row(F + (ft.gh + 1) * KS, tp) * fl.inv_nu3[ft.gh];
        out[g * ostride] = (real)(fl.nu3[g] * v);
    }
}

// 2^(y dl2): the frequency factor 1/D of the lab extinction (dl2 = the group spacing in
// log2(nu)); the hardware base-2 exponential in FP32
__device__ __forceinline__ float exp_dl(float y, float dl2) { return __builtin_amdgcn_exp2f(y * dl2); }
__device__ __forceinline__ double exp_dl(double y, double dl2) { return exp2(y * dl2); }

// S~ = (chi S + I_prev/(c dt)) / (chi + 1/(c dt)); in steady state S (or 0 where chi = 0)
__device__ __forceinline__ float time_terms(float chi, float S, float ip, float icdt)
{
    if (icdt == 0.0f) return chi > 0.0f ? S : 0.0f;
    const float xt = chi + icdt;
    return xt > 0.0f ? (chi * S + ip * icdt) * __builtin_amdgcn_rcpf(xt) : 0.0f;
}
__device__ __forceinline__ double time_terms(double chi, double S, double ip, double icdt)
{
    if (icdt == 0.0) return chi > 0.0 ? S : 0.0;
    const double xt = chi + icdt;
    return xt > 0.0 ? (chi * S + ip * icdt) / xt : 0.0;
}

// ---------------------------------------------------------------------------
// Remap plan of a medium: for every (point, ordinate) the taps and frequency
// shift of the boost (lab ordinate k -> comoving direction n0 of Eq. 8 and
// frequency nu/D of Eq. 7) and of the inverse map (comoving ordinate j -> lab
// direction and frequency D' nu, D' = Gamma (1 + beta.n0)).  They depend on
// the velocity field only, so they are computed once per medium.
// ---------------------------------------------------------------------------
template <typename real>
__device__ __forceinline__ RemapEntry<real> remap_entry(const double *mu, int nmu, int nphi, const double nt[3])
{
    const AngleTaps t = angle_taps<real>(mu, nmu, nphi, nt);
    RemapEntry<real> e{};
    e.abs = (t.a0 + 1) | (t.b0 << 10);
    const double um = 1.0 - t.wmu, up = 1.0 - t.wphi;
    e.w[0] = (real)(um * up); e.w[1] = (real)(um * t.wphi);
    e.w[2] = (real)(t.wmu * up); e.w[3] = (real)(t.wmu * t.wphi);
    return e;
}

template <typename real>
__device__ __forceinline__ void entry_freq(RemapEntry<real> &e, const FreqInfo &fi, double D, bool inverse)
{
    if (fi.grey) {
        const double D2 = D * D;
        e.u = (real)(inverse ? 1.0 / (D2 * D2) : D2 * D2);
    } else if (fi.uniform) {
        // positions of the target frequencies nu/D (boost) or D' nu (inverse)
        const double lr = (double)log((real)D) * fi.inv_delta;
        int sh;
        uniform_shift<real>(inverse ? lr : -lr, fi.delta, fi.G, sh, e.u, e.v);
        e.abs |= (sh == kAllGhost ? kPackedGhost : sh) * (1 << 20);
    } else {
        const double x = inverse ? log(D) : -log(D);
        e.u = (real)x;
        e.v = (real)(x - (double)e.u);
    }
}

template <typename real>
__global__ void __launch_bounds__(256) k_remap_plan(PlanArgs<real> a)
{
    const long n = a.P * a.K;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const long p = i / a.K;
        const int k = (int)(i - p * a.K);
        double b[3];
        if (!load_beta(a.beta, p, b)) continue;
        const double gam = a.gam[p];
        const double n[3] = {a.dir[4 * k], a.dir[4 * k + 1], a.dir[4 * k + 2]};
        const double bn = b[0] * n[0] + b[1] * n[1] + b[2] * n[2];
        {
            // lab ordinate k seen from the comoving frame (Eqs. 7-8)
            const double D = 1.0 / inv_doppler(b, gam, n);
            const double f = gam * (1.0 - gam / (gam + 1.0) * bn);
            double n0[3];
            for (int c = 0; c < 3; ++c) n0[c] = D * (n[c] - f * b[c]);
            RemapEntry<real> e = remap_entry<real>(a.mu, a.nmu, a.nphi, n0);
            entry_freq(e, a.fi, D, false);
            if (a.chi_grey) e.kap = a.chilab[(long)k * a.P + p];
            // a per-group extinction on log-uniform groups: the position y = -ln D / dln(nu) of the
            // target frequencies nu/D in group spacings, from which the boost rebuilds chi_lab
            else if (a.fi.uniform) e.kap = (real)(-(double)log((real)D) * a.fi.inv_delta);
            a.boost[i] = e;
        }
        {
            // comoving ordinate k seen from the lab frame (the inverse maps)
            const double Dp = gam * (1.0 + bn);
            const double f = gam * (1.0 + gam / (gam + 1.0) * bn);
            double nl[3];
            for (int c = 0; c < 3; ++c) nl[c] = (n[c] + f * b[c]) / Dp;
            RemapEntry<real> e = remap_entry<real>(a.mu, a.nmu, a.nphi, nl);
            entry_freq(e, a.fi, Dp, true);
            a.unboost[i] = e;
        }
    }
}

// the frequency position shift packed in an entry (kAllGhost: every target beyond the groups)
__device__ __forceinline__ int entry_shift(int abs)
{
    const int sh = abs >> 20;
    return sh == kPackedGhost ? kAllGhost : sh;
}

// the four table columns of an entry's angle taps
template <typename real>
__device__ __forceinline__ Taps4<real> entry_taps(int abs, const real w[4], int K, int nmu, int nphi)
{
    const int a0 = (abs & 1023) - 1, b0 = (abs >> 10) & 1023;
    const int b1 = b0 + 1 == nphi ? 0 : b0 + 1;
    auto col = [&](int ring, int b) { return ring < 0 ? K : (ring >= nmu ? K + 1 : ring * nphi + b); };
    Taps4<real> t;
    t.c[0] = col(a0, b0); t.c[1] = col(a0, b1); t.c[2] = col(a0 + 1, b0); t.c[3] = col(a0 + 1, b1);
    t.w[0] = w[0]; t.w[1] = w[1]; t.w[2] = w[2]; t.w[3] = w[3];
    return t;
}

// x / d for 0 <= x < NPT d with NPT points per workgroup (1 or 2): no integer division
template <int NPT>
__device__ __forceinline__ int point_of(int x, int d)
{
    return NPT == 1 ? 0 : (NPT == 2 ? (int)(x >= d) : x / d);
}

// stage rows [g][j] of a point's ordinate values (n4 runs of four values,
// K4 runs per row) into the table, four 16-byte loads per lane in flight
template <typename real>
__device__ __forceinline__ void stage_rows(const real *__restrict__ src, real *F, int G, int K, int KS)
{
    using P4 = Pack<real, 4>;
    const int T = blockDim.x, tid = threadIdx.x, K4 = K >> 2, n4 = G * K4;
    for (int i0 = tid; i0 < n4; i0 += 4 * T) {
        P4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * T;
            if (i < n4) {
                const int g = i / K4, j = (i - g * K4) * 4;
                v[u] = load_stream(src + (long)g * K + j);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * T;
            if (i < n4) {
                const int g = i / K4, j = (i - g * K4) * 4;
                real *row = F + (g + 1) * KS + j;
                row[0] = v[u].v[0]; row[1] = v[u].v[1]; row[2] = v[u].v[2]; row[3] = v[u].v[3];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// S3: comoving ordinates -> lab ordinates.  The point's comoving source
// S0[g][j] (from the SH -> ordinate product) is staged in the table; the lab
// source of ordinate k is the bilinear (angle) x linear in ln(nu) remap of the
// invariant S0/nu^3 at the comoving direction n0 (Eq. 8) and frequency nu/D
// (Eq. 7) of that ray, times nu^3; then the implicit time terms of Eqs. 5-6
// with the lab extinction chi_lab precomputed per medium.  Output S~[k][p][g].
// A workgroup takes NPT neighbouring points (NPT = 2 where a point's groups
// fill 64 bytes, so that the stage inputs and outputs of one ordinate are read
// and written as whole 128-byte lines; half-line runs scattered over the
// ordinate slabs move at about half the rate).  Each wave takes 64 / NPT
// ordinates: lane l loads the remap entry of ordinate kb + l / NPT at point
// l % NPT, then the lanes run over (ordinate, point, run of W groups) items,
// W = 4 when G allows 16-byte runs, fetching their entry from the lane that
// loaded it; consecutive lanes so write consecutive groups of one ordinate.
// The entries and the time-term inputs of a lane's first four items are
// loaded before the tables are staged.
// ---------------------------------------------------------------------------
template <typename real, int NPT>
__global__ void __launch_bounds__(kRemapThreads, 4) k_boost(BoostArgs<real> a)
{
    using P4 = Pack<real, 4>;
    extern __shared__ unsigned char smem_raw[];
    const long p0 = xcd_item((a.P + NPT - 1) / NPT) * NPT;
    if (p0 >= a.P) return;
    const int G = a.fi.G, K = a.K, T = blockDim.x, tid = threadIdx.x, KS = table_stride(K);
    const int lane = tid & 63, wave = tid >> 6, nwaves = T >> 6;
    const int TS = (G + 2) * KS;                        // one point's table
    double *fbuf = reinterpret_cast<double *>(smem_raw);                // [4G]
    real *F0 = reinterpret_cast<real *>(fbuf + 4 * G);                  // [NPT][G+2][KS]

    const FreqL fl = stage_freq(a.fi, fbuf);
    bool mv[NPT];
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        double b[3];
        mv[q] = p0 + q < a.P && load_beta(a.beta, p0 + q, b);
    }
    const int W = (G & 3) == 0 ? 4 : 1;                // groups per lane item
    const int NC = G / W;                               // items per ordinate and point
    const int IC = NPT * NC;                            // items per ordinate
    const float rIC = 1.0f / (float)IC;
    constexpr int OB = 64 / NPT;                        // ordinates per wave block
    const int kb0 = wave * OB;
    // this lane's entry: ordinate kb + lane / NPT at point p0 + lane % NPT
    const int lq = lane % NPT;
    const long lp = p0 + lq;
    const bool lmv = mv[lq];

    RemapEntry<real> e{};
    real kap = 0;
    P4 pre[4];
    auto fetch_ordinates = [&](int kb) {
        const int km = kb + lane / NPT;
        if (km < K && lp < a.P) {
            if (lmv) e = a.plan[lp * K + km];
            else if (a.chi_grey) kap = a.chilab[(long)km * a.P + lp];
        }
    };
    auto fetch_inputs = [&](int kb, int nit, int base) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int item = base + 64 * u + lane;
            pre[u] = P4{};
            if (a.Iprev && item < nit) {
                // (one point per workgroup: rem < NC, so q = 0 without the division)
                const int kk = (int)(((float)item + 0.5f) * rIC), rem = item - __mul24(kk, IC), q = point_of<NPT>(rem, NC);
                const int g0 = (rem - q * NC) * W;
                if (p0 + q < a.P) {
                    const long o = ((long)(kb + kk) * a.P + p0 + q) * G + g0;
                    if (W == 4) pre[u] = load_stream(a.Iprev + o);
                    else pre[u].v[0] = a.Iprev[o];
                }
            }
        }
    };
    if (kb0 < K) {
        fetch_ordinates(kb0);
        fetch_inputs(kb0, min(OB, K - kb0) * IC, 0);
    }

    // per-group lab extinction rebuilt from the points' comoving one (staged here) and the
    // plan's frequency position: chi_lab = chi0(nu/D)/D, linear in ln(nu), outer values held
    const bool chi_fly = !a.chi_grey && a.fi.uniform && a.chi0 != nullptr;
    real *C0 = F0 + NPT * TS;                           // [NPT][G]
    if (chi_fly)
        for (int i = tid; i < NPT * G; i += T) {
            const int q = i / G;
            C0[i] = p0 + q < a.P ? a.chi0[(p0 + q) * G + (i - q * G)] : real(0);
        }
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        if (p0 + q >= a.P) break;
        const real *__restrict__ src = a.S0 + (p0 + q) * G * K;
        real *F = F0 + q * TS;
        if ((K & 3) == 0) {
            stage_rows(src, F, G, K, KS);
        } else {
            for (int g = 0; g < G; ++g)
                for (int j = tid; j < K; j += T) F[(g + 1) * KS + j] = src[g * K + j];
        }
        if (mv[q]) table_ghosts(F, G, KS);
    }
    __syncthreads();
    bool anymv = false;
#pragma unroll
    for (int q = 0; q < NPT; ++q) anymv = anymv || mv[q];
    if (anymv) {
#pragma unroll
        for (int q = 0; q < NPT; ++q)
            if (mv[q]) table_poles(F0 + q * TS, G, K, KS, a.nmu, a.nphi);
        __syncthreads();
    }
    const real icdt = a.inv_cdt;
    const real dl2 = (real)(a.fi.delta * 1.4426950408889634);   // the group spacing in log2(nu)
    for (int kb = kb0; kb < K; kb += nwaves * OB) {
        const int nk = min(OB, K - kb), nit = nk * IC;
        if (kb != kb0) fetch_ordinates(kb);
        const real kapv = lmv ? e.kap : kap;
        for (int base = 0; base < nit; base += 256) {
            if (kb != kb0 || base != 0) fetch_inputs(kb, nit, base);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int item = base + 64 * u + lane;
                // every lane takes part in the shuffles (their source lanes are all active)
                const int kk = min((int)(((float)item + 0.5f) * rIC), nk - 1), rem = item - __mul24(kk, IC);
                // (items past the last, clamped to the last ordinate, may have rem >= IC: point NPT - 1)
                const int q = min(point_of<NPT>(rem, NC), NPT - 1), g0 = (rem - q * NC) * W;
                const int srcl = kk * NPT + q;
                const real kp = __shfl(kapv, srcl, 64);
                const int ab = __shfl(e.abs, srcl, 64);
                const int sh = entry_shift(ab);
                real w[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) w[i] = __shfl(e.w[i], srcl, 64);
                const real eu = __shfl(e.u, srcl, 64), ev = __shfl(e.v, srcl, 64);
                if (item >= nit || p0 + q >= a.P) continue;
                const real *F = F0 + q * TS;
                const int k = kb + kk;
                const long o = ((long)k * a.P + p0 + q) * G + g0;
                real out[4] = {0, 0, 0, 0};
                if (!mv[q]) {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (i < W) out[i] = F[(g0 + i + 1) * KS + k];
                } else {
                    const Taps4<real> tp = entry_taps(ab, w, K, a.nmu, a.nphi);
                    if (a.fi.grey) {
                        out[0] = eu * tap_row(F + KS, tp);
                    } else if (a.fi.uniform) {
                        if (sh != kAllGhost) {
                            auto A = [&](int gp) -> real {       // row index and stride < 2^24: the full-rate 24-bit product
                                return tap_row(F + __umul24(min(max(gp, -1), G) + 1, KS), tp);
                            };
                            real acur = A(g0 + sh);
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                if (i < W) {
                                    const real anext = A(g0 + i + sh + 1);
                                    out[i] = eu * acur + ev * anext;
                                    acur = anext;
                                }
                            }
                        }
                    } else {
                        const double x = (double)eu + (double)ev;
                        FreqWalk fw{0};
                        if (G > 2) fw.lo = centre_bracket(fl.lnc, G, fl.lnc[g0] + x);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            if (i < W) {
                                const int g = g0 + i;
                                const FreqTaps ft = freq_taps_zero_walk(a.fi, fl, fl.lnc[g] + x, fw);
                                double v = 0.0;
                                if (ft.gl >= 0) v += ft.wl * (double)tap_row(F + (ft.gl + 1) * KS, tp) * fl.inv_nu3[ft.gl];
                                if (ft.gh >= 0) v += ft.wh * (double)tap_row(F + (ft.gh + 1) * KS, tp) * fl.inv_nu3[ft.gh];
                                out[i] = (real)(fl.nu3[g] * v);
                            }
                        }
                    }
                }
                // implicit time terms and the store
                real cx[4];
                if (a.chi_grey) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) cx[i] = kp;
                } else if (chi_fly) {
                    const real *C = C0 + q * G;
                    if (!mv[q]) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) cx[i] = i < W ? C[g0 + i] : real(0);
                    } else {
                        // the W + 1 comoving values the item's groups interpolate between
                        const real sf = floor(kp), f = kp - sf, invD = exp_dl(kp, dl2);
                        const int i0 = g0 + (int)sf;
                        real cv[5];
#pragma unroll
                        for (int i = 0; i < 5; ++i) cv[i] = i <= W ? C[min(max(i0 + i, 0), G - 1)] : real(0);
#pragma unroll
                        for (int i = 0; i < 4; ++i) cx[i] = invD * (cv[i] + f * (cv[i + 1] - cv[i]));
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) cx[i] = i < W ? a.chilab[o + i] : real(0);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (i < W) out[i] = time_terms(cx[i], out[i], pre[u].v[i], icdt);
                if (W == 4) {
                    P4 v;
                    v.v[0] = out[0]; v.v[1] = out[1]; v.v[2] = out[2]; v.v[3] = out[3];
                    store_stream(a.St + o, v);
                } else {
                    a.St[o] = out[0];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// S5: lab ordinates -> comoving ordinates, one thread per comoving ordinate.
// The point's lab intensities I[k][g] are staged in the table (transposed);
// the comoving value of ordinate j is the remap of the invariant I/nu^3 at the
// lab direction and frequency D' nu of that comoving ray.  Output I0[p][g][j].
// ---------------------------------------------------------------------------
// NPT neighbouring points per workgroup (2 where a point's groups fill 64
// bytes: the staging then reads whole 128-byte lines of each ordinate).
template <typename real, int NPT>
__global__ void __launch_bounds__(kRemapThreads, sizeof(real) == 4 ? 8 : 4) k_unboost(UnboostArgs<real> a)
{
    extern __shared__ unsigned char smem_raw[];
    const long p0 = xcd_item((a.P + NPT - 1) / NPT) * NPT;
    if (p0 >= a.P) return;
    const int G = a.fi.G, K = a.K, T = blockDim.x, tid = threadIdx.x, KS = table_stride(K);
    const int TS = (G + 2) * KS;
    double *fbuf = reinterpret_cast<double *>(smem_raw);                // [4G]
    real *F0 = reinterpret_cast<real *>(fbuf + 4 * G);                  // [NPT][G+2][KS]
    const int np = (int)min((long)NPT, a.P - p0);

    const FreqL fl = stage_freq(a.fi, fbuf);
    bool mv[NPT];
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        double b[3];
        mv[q] = q < np && load_beta(a.beta, p0 + q, b);
    }
    // the first (point, ordinate) pair's entry, before staging
    RemapEntry<real> e{};
    {
        const int q = tid / K, j = tid - q * K;
        if (q < np && mv[q]) e = a.plan[(p0 + q) * K + j];
    }
    if ((G & 3) == 0) {
        // 16-byte loads, four groups of one (ordinate, point) per lane, written down a
        // table column; four loads per lane in flight
        using P4 = Pack<real, 4>;
        const int G4 = G >> 2, IC = NPT * G4, n4 = K * IC;
        const float rIC = 1.0f / (float)IC;
        for (int i0 = tid; i0 < n4; i0 += 4 * T) {
            P4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int idx = i0 + u * T;
                const int k = (int)(((float)idx + 0.5f) * rIC), rem = idx - __mul24(k, IC), q = point_of<NPT>(rem, G4);
                if (idx < n4 && q < np) {
                    const int g = (rem - q * G4) * 4;
                    v[u] = load_stream(a.Ilab + ((long)k * a.P + p0 + q) * G + g);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int idx = i0 + u * T;
                const int k = (int)(((float)idx + 0.5f) * rIC), rem = idx - __mul24(k, IC), q = point_of<NPT>(rem, G4);
                if (idx < n4 && q < np) {
                    const int g = (rem - q * G4) * 4;
                    real *F = F0 + q * TS;
                    F[(g + 1) * KS + k] = v[u].v[0];
                    F[(g + 2) * KS + k] = v[u].v[1];
                    F[(g + 3) * KS + k] = v[u].v[2];
                    F[(g + 4) * KS + k] = v[u].v[3];
                }
            }
        }
    } else {
        const int IC = NPT * G;
        const float rIC = 1.0f / (float)IC;
        for (int idx = tid; idx < K * IC; idx += T) {
            const int k = (int)(((float)idx + 0.5f) * rIC), rem = idx - k * IC, q = rem / G, g = rem - q * G;
            if (q < np) F0[q * TS + (g + 1) * KS + k] = a.Ilab[((long)k * a.P + p0 + q) * G + g];
        }
    }
#pragma unroll
    for (int q = 0; q < NPT; ++q)
        if (mv[q]) table_ghosts(F0 + q * TS, G, KS);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NPT; ++q)
        if (mv[q]) table_poles(F0 + q * TS, G, K, KS, a.nmu, a.nphi);
    __syncthreads();
    for (int idx = tid; idx < np * K; idx += T) {
        const int q = point_of<NPT>(idx, K), j = idx - q * K;      // idx < NPT K
        const real *F = F0 + q * TS;
        real *__restrict__ out = a.I0 + (p0 + q) * G * K;
        if (!mv[q]) {
            for (int g = 0; g < G; ++g) out[g * K + j] = F[(g + 1) * KS + j];
            continue;
        }
        if (idx != tid) e = a.plan[(p0 + q) * K + j];
        const Taps4<real> tp = entry_taps(e.abs, e.w, K, a.nmu, a.nphi);
        if (a.fi.grey) {
            out[j] = tap_row(F + KS, tp) * e.u;
        } else if (a.fi.uniform) {
            const int sh = entry_shift(e.abs);
            if (sh == kAllGhost) {
                for (int g = 0; g < G; ++g) out[g * K + j] = real(0);
            } else {
                auto A = [&](int gp) -> real {   // row index and stride < 2^24: the full-rate 24-bit product
                    return tap_row(F + __umul24(min(max(gp, -1), G) + 1, KS), tp);
                };
                real acur = A(sh);
                for (int g = 0; g < G; ++g) {
                    const real anext = A(g + sh + 1);
                    __builtin_nontemporal_store(e.u * acur + e.v * anext, out + g * K + j);
                    acur = anext;
                }
            }
        } else {
            general_remap(F, KS, a.fi, fl, tp, (double)e.u + (double)e.v, out + j, K);
        }
    }
}

// lab extinction chi_lab(k, p[, g]) of the medium (stored [k][p] when chi0 is
// the same for every group, else [k][p][g])
template <typename real>
__global__ void __launch_bounds__(256) k_chilab(ChiLabArgs<real> a)
{
    extern __shared__ unsigned char smem_raw[];
    double *fbuf = reinterpret_cast<double *>(smem_raw);
    const FreqL fl = stage_freq(a.fi, fbuf);
    __syncthreads();
    const int Gn = a.chi_grey ? 1 : a.fi.G;
    const long n = a.P * Gn;
    const int k = blockIdx.y;
    const double nk[3] = {a.dir[4 * k], a.dir[4 * k + 1], a.dir[4 * k + 2]};
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const long p = i / Gn;
        const int g = (int)(i - p * Gn);
        double b[3];
        const bool moving = load_beta(a.beta, p, b);
        const double invD = moving ? inv_doppler(b, a.gam[p], nk) : 1.0;
        a.out[(long)k * n + i] = chi_lab_of(a.chi0, p, g, a.fi, fl, a.chi_grey, moving, invD);
    }
}

// ---------------------------------------------------------------------------
// S6: comoving ordinates -> SH, Ilm[r][q] = sum_j I0[r][j] (w_j Y_q(n_j)) for
// the R = P G rows (point, group), FP32 on the matrix cores
// (v_mfma_f32_16x16x4f32, FP32 accumulation).  A wave owns 16 rows and all NL
// columns (NT tiles of 16); the weight table is staged in LDS per chunk of 64
// ordinates (rows padded by 4 so the B operand reads are conflict-free); the
// rows stream from HBM as 16-byte vectors.  Within a 16-ordinate block lane
// group lg = lane/16 holds ordinates 4 lg .. 4 lg + 3 of its row, and the four
// matrix-core steps take them in that order (the reduction order over j is
// free); the B operand follows the same order.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Dense SH <-> ordinate products on the matrix cores, FP32 and FP64 (Eq. 9
// and its inverse): C[R][N] = A[R][Kd] B[Kd][N], rows R = points x groups.
// A workgroup of W waves owns a panel of 16 W RT rows and a block of 16 NT
// columns (grid.y); each wave keeps RT x NT 16 x 16 accumulator tiles.  B is
// staged in LDS KC rows at a time and shared by the waves; each lane loads
// its rows of A for the chunk as 4-element vectors, so that within a chunk
// the k index of MFMA step (t, s) in lane group g is 16 t + 4 g + s (the same
// permutation on both operands leaves the sum unchanged).  Indices are 64-bit:
// no matrix size limit.
// ---------------------------------------------------------------------------
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <typename real> struct Mfma16;
// Both read A[i][k] from lane i + 16 k and B[k][j] from lane j + 16 k; register r of
// lane l holds row 4 (l / 16) + r (FP32) or l / 16 + 4 r (FP64) of column l % 16
template <> struct Mfma16<float> {
    typedef f32x4 acc;
    __device__ static acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
    __device__ static acc step(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int lg, int r) { return 4 * lg + r; }
};
template <> struct Mfma16<double> {
    typedef f64x4 acc;
    __device__ static acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
    __device__ static acc step(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int lg, int r) { return lg + 4 * r; }
};

// TR (FP32, N a multiple of 4): each 16 x 16 tile is computed transposed (the
// operands swapped), so that a lane holds four consecutive columns of one row
template <typename real, int NT, int RT, int W, int KC, int BV, bool TR>
__global__ void __launch_bounds__(64 * W) k_gemm_panel(long R, int Kd, int N, const real *__restrict__ A,
                                                       const real *__restrict__ B, real *__restrict__ C)
{
    using M = Mfma16<real>;
    typedef real v4 __attribute__((ext_vector_type(4)));
    typedef real vB __attribute__((ext_vector_type(BV)));
    constexpr int NC = 16 * NT, LDB = NC + (sizeof(real) == 4 ? 4 : 2);
    constexpr int T = 64 * W, NBV = KC * NC / BV, BL = (NBV + T - 1) / T;    // B vectors per chunk and per thread
    extern __shared__ unsigned char smem_raw[];
    real *Bs = reinterpret_cast<real *>(smem_raw);                     // two chunks [KC][LDB]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, lr = lane & 15, lg = lane >> 4;
    const long r0 = (long)xcd_item(gridDim.x) * (16 * W * RT) + wave * (16 * RT);
    const int c0 = blockIdx.y * NC;
    const real *Arow[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) Arow[t] = A + min(r0 + 16 * t + lr, R - 1) * (long)Kd;
    const bool avec = (Kd & 3) == 0;
    typename M::acc acc[RT][NT];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[t][c] = M::zero();
    real a[RT][KC / 16][4];
    vB bl[BL];
    // this lane's A values and B vectors of the chunk at kc (zero past Kd and N)
    auto load = [&](int kc) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int t = 0; t < KC / 16; ++t) {
                const int k = kc + 16 * t + 4 * lg;
                if (avec && k + 3 < Kd) {
                    const v4 v = *reinterpret_cast<const v4 *>(Arow[rt] + k);
                    a[rt][t][0] = v.x; a[rt][t][1] = v.y; a[rt][t][2] = v.z; a[rt][t][3] = v.w;
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) a[rt][t][i] = (k + i < Kd) ? Arow[rt][k + i] : real(0);
                }
            }
#pragma unroll
        for (int u = 0; u < BL; ++u) {
            const int i = tid + u * T;
            const int kk = i / (NC / BV), c = (i - kk * (NC / BV)) * BV;
            vB v;
#pragma unroll
            for (int e = 0; e < BV; ++e) v[e] = real(0);
            if (i < NBV && kc + kk < Kd && c0 + c < N) v = *reinterpret_cast<const vB *>(B + (long)(kc + kk) * N + c0 + c);
            bl[u] = v;
        }
    };
    auto stage = [&](int buf) {
        real *Bb = Bs + buf * KC * LDB;
#pragma unroll
        for (int u = 0; u < BL; ++u) {
            const int i = tid + u * T;
            if (i < NBV) {
                const int kk = i / (NC / BV), c = (i - kk * (NC / BV)) * BV;
#pragma unroll
                for (int e = 0; e < BV; ++e) Bb[kk * LDB + c + e] = bl[u][e];
            }
        }
    };
    load(0);
    stage(0);
    __syncthreads();
    int buf = 0;
    for (int kc = 0; kc < Kd; kc += KC) {
        real ac[RT][KC / 16][4];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int t = 0; t < KC / 16; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) ac[rt][t][i] = a[rt][t][i];
        const bool more = kc + KC < Kd;
        if (more) load(kc + KC);                     // the next chunk's loads fly during the products
        const real *Bb = Bs + buf * KC * LDB;
#pragma unroll
        for (int t = 0; t < KC / 16; ++t) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const real *brow = Bb + (16 * t + 4 * lg + s) * LDB + lr;
#pragma unroll
                for (int c = 0; c < NT; ++c) {
                    const real bv = brow[16 * c];
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
                        acc[rt][c] = TR ? M::step(bv, ac[rt][t][s], acc[rt][c]) : M::step(ac[rt][t][s], bv, acc[rt][c]);
                }
            }
        }
        if (more) stage(buf ^ 1);                    // every wave finished the other buffer before the last barrier
        __syncthreads();
        buf ^= 1;
    }
    if (TR) {
        // transposed tiles: lane (lr, lg) holds columns 16 c + 4 lg .. + 3 of row 16 rt + lr,
        // stored as one 16-byte vector (N a multiple of 4)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const long r = r0 + 16 * rt + lr;
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                const int col = c0 + 16 * c + 4 * lg;
                if (r < R && col < N) {
                    v4 v;
                    v.x = acc[rt][c][0]; v.y = acc[rt][c][1]; v.z = acc[rt][c][2]; v.w = acc[rt][c][3];
                    *reinterpret_cast<v4 *>(C + r * N + col) = v;
                }
            }
        }
        return;
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            const int col = c0 + 16 * c + lr;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long r = r0 + 16 * rt + M::row(lg, i);
                if (r < R && col < N) C[r * N + col] = acc[rt][c][i];
            }
        }
}

template <int NT, int RT, int W = 4>
__global__ void __launch_bounds__(64 * W) k_do2sh_f32(long R, int K, int NL, const float *__restrict__ A,
                                                      const float *__restrict__ B, float *__restrict__ C)
{
    constexpr int KC = 64, NC = NT * 16, NLP = NC + 4;
    extern __shared__ unsigned char smem_raw[];
    float *Bs = reinterpret_cast<float *>(smem_raw);                   // [KC][NLP]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lr = lane & 15, lg = lane >> 4;
    const long r0 = (long)xcd_item(gridDim.x) * (16 * W * RT) + wave * (16 * RT);
    const float *Arow[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) Arow[t] = A + min(r0 + 16 * t + lr, R - 1) * (long)K;
    const bool vec = (K & 3) == 0;
    f32x4 acc[RT][NT];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < K; kc += KC) {
        float a[RT][4][4];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int k = kc + 16 * t + 4 * lg;
                if (vec && k + 3 < K) {
                    const f32x4 v = *reinterpret_cast<const f32x4 *>(Arow[rt] + k);
                    a[rt][t][0] = v.x; a[rt][t][1] = v.y; a[rt][t][2] = v.z; a[rt][t][3] = v.w;
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) a[rt][t][i] = (k + i < K) ? Arow[rt][k + i] : 0.f;
                }
            }
        __syncthreads();                                                // the previous chunk's B reads are done
        for (int i = threadIdx.x; i < KC * NC; i += blockDim.x) {
            const int kk = i / NC, c = i - kk * NC;
            Bs[kk * NLP + c] = (kc + kk < K && c < NL) ? B[(long)(kc + kk) * NL + c] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const float *brow = Bs + (16 * t + 4 * lg + s) * NLP + lr;
#pragma unroll
                for (int c = 0; c < NT; ++c) {
                    const float bv = brow[16 * c];
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
                        acc[rt][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt][t][s], bv, acc[rt][c], 0, 0, 0);
                }
            }
        }
    }
    // lane holds rows 4 lg + i, column 16 c + lr of each tile
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            const int col = 16 * c + lr;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long r = r0 + 16 * rt + 4 * lg + i;
                if (r < R && col < NL) C[r * NL + col] = acc[rt][c][i];
            }
        }
}

// The same product with the whole weight table resident in LDS (staged once
// per workgroup, K rounded up to 64 rows of NLP floats): persistent workgroups
// of sixteen waves walk blocks of 16 x 16 RT rows with no barrier inside, each
// wave loading the next 64-ordinate chunk of its rows while the matrix cores
// take the current one.  FULL (K a multiple of 64): every chunk is whole, the
// loads take no branches, the last chunk of a block loads the first chunk of the
// wave's next block, and the block's stores go out after the one wait for it (so
// no load waits for them).
template <int NT, int RT, bool FULL>
__global__ void __launch_bounds__(1024) k_do2sh_f32r(long R, int K, int NL, const float *__restrict__ A,
                                                     const float *__restrict__ B, float *__restrict__ C)
{
    constexpr int W = 16, KC = 64, NC = NT * 16, NLP = NC + 4;
    extern __shared__ unsigned char smem_raw[];
    float *Bs = reinterpret_cast<float *>(smem_raw);                   // [Kr][NLP]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lr = lane & 15, lg = lane >> 4;
    const int Kr = (K + KC - 1) / KC * KC;
    for (int i = threadIdx.x; i < Kr * NC; i += blockDim.x) {
        const int kk = i / NC, c = i - kk * NC;
        Bs[kk * NLP + c] = (kk < K && c < NL) ? B[(long)kk * NL + c] : 0.f;
    }
    __syncthreads();
    const bool vec = (K & 3) == 0;
    const long nblk = (R + 16 * W * RT - 1) / (16 * W * RT);
    if constexpr (FULL) {
        auto rows_of = [&](long blk, const float *(&Ar)[RT]) {
#pragma unroll
            for (int t = 0; t < RT; ++t)
                Ar[t] = A + min(blk * (16 * W * RT) + wave * (16 * RT) + 16 * t + lr, R - 1) * (long)K;
        };
        auto load = [&](f32x4 (&dst)[RT][4], const float *const (&Ar)[RT]) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int t = 0; t < 4; ++t) dst[rt][t] = *reinterpret_cast<const f32x4 *>(Ar[rt] + 16 * t + 4 * lg);
        };
        long blk = blockIdx.x;
        if (blk >= nblk) return;
        const float *Arow[RT], *Anext[RT], *src[RT];
        rows_of(blk, Arow);
        f32x4 a[RT][4], an[RT][4];
        load(a, Arow);
        __builtin_amdgcn_s_waitcnt(0xF70);              // vmcnt(0): the loop starts with no load in flight
        for (; blk < nblk; blk += gridDim.x) {
            // the wave's next block (past its last: the last again, loaded and not used)
            rows_of(min(blk + (long)gridDim.x, nblk - 1), Anext);
            f32x4 acc[RT][NT];
#pragma unroll
            for (int t = 0; t < RT; ++t)
#pragma unroll
                for (int c = 0; c < NT; ++c) acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
            for (int kc = 0; kc < K; kc += KC) {
                const bool last = kc + KC >= K;
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) src[rt] = last ? Anext[rt] : Arow[rt] + kc + KC;
                load(an, src);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const float *brow = Bs + (kc + 16 * t + 4 * lg + s) * NLP + lr;
#pragma unroll
                        for (int c = 0; c < NT; ++c) {
                            const float bv = brow[16 * c];
#pragma unroll
                            for (int rt = 0; rt < RT; ++rt)
                                acc[rt][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt][t][s], bv, acc[rt][c], 0, 0, 0);
                        }
                    }
                }
                if (last) __builtin_amdgcn_s_waitcnt(0xF70);   // vmcnt(0): the next block's rows, not its stores
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int t = 0; t < 4; ++t) a[rt][t] = an[rt][t];
            }
            __builtin_amdgcn_sched_barrier(0);
            const long r0 = blk * (16 * W * RT) + wave * (16 * RT);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int c = 0; c < NT; ++c) {
                    const int col = 16 * c + lr;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const long r = r0 + 16 * rt + 4 * lg + i;
                        if (r < R && col < NL) C[r * NL + col] = acc[rt][c][i];
                    }
                }
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) Arow[rt] = Anext[rt];
        }
        return;
    }
    for (long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const long r0 = blk * (16 * W * RT) + wave * (16 * RT);
        const float *Arow[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) Arow[t] = A + min(r0 + 16 * t + lr, R - 1) * (long)K;
        f32x4 acc[RT][NT];
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int c = 0; c < NT; ++c) acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
        f32x4 a[RT][4], an[RT][4];
        auto load = [&](f32x4 (&dst)[RT][4], int kc) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int k = kc + 16 * t + 4 * lg;
                    if (vec && k + 3 < K) {
                        dst[rt][t] = *reinterpret_cast<const f32x4 *>(Arow[rt] + k);
                    } else {
#pragma unroll
                        for (int i = 0; i < 4; ++i) dst[rt][t][i] = (k + i < K) ? Arow[rt][k + i] : 0.f;
                    }
                }
        };
        load(a, 0);
        for (int kc = 0; kc < K; kc += KC) {
            if (kc + KC < K) load(an, kc + KC);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const float *brow = Bs + (kc + 16 * t + 4 * lg + s) * NLP + lr;
#pragma unroll
                    for (int c = 0; c < NT; ++c) {
                        const float bv = brow[16 * c];
#pragma unroll
                        for (int rt = 0; rt < RT; ++rt)
                            acc[rt][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt][t][s], bv, acc[rt][c], 0, 0, 0);
                    }
                }
            }
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int t = 0; t < 4; ++t) a[rt][t] = an[rt][t];
        }
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                const int col = 16 * c + lr;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const long r = r0 + 16 * rt + 4 * lg + i;
                    if (r < R && col < NL) C[r * NL + col] = acc[rt][c][i];
                }
            }
    }
}

// ---------------------------------------------------------------------------
// Mixed precision: the two SH <-> ordinate products on FP16 matrix cores
// (v_mfma_f32_16x16x32_f16) with FP32 accumulation.  Both operands are split
// into FP16 pairs x = hi + lo (lo the FP16 rounding of the remainder) and a
// block product is hi.hi + lo.hi + hi.lo, about 22 significant bits.  The data
// operand is first brought into FP16 range by a power of two (exact): per row
// (point, group) for the short SH rows of S2, per row and block of 32
// ordinates for S6, whose row maximum is not known before the row has
// streamed by; each block's product is rescaled into the accumulator.  The
// tables (w_j) Y_q(n_j) are stored as FP16 pairs, rows padded by zeros to
// whole 32-element blocks, and staged in LDS per chunk.  Operand layout of the
// 16 x 16 x 32 product: lane group lg = lane/16 holds elements 8 lg .. 8 lg + 7
// of the reduction block for row / column lane % 16 (A and B in the same
// order).
// ---------------------------------------------------------------------------
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// power of two s taking m > 0 into [2^top, 2^(top + 1)) (at top = 14 FP16 keeps
// full precision down to 2^-28 m); m = 0 or tiny gives a bounded scale
__device__ __forceinline__ void fp16_scale(float m, float &s, float &inv, int top = 14)
{
    const int e = max(((__float_as_int(m) >> 23) & 0xff) - 127, -100);
    s = ldexpf(1.0f, top - e);
    inv = ldexpf(1.0f, e - top);
}

// hi + lo FP16 pair of v * s
__device__ __forceinline__ void split_f16x8(const float v[8], float s, f16x8 &hi, f16x8 &lo)
{
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const float x = v[i] * s;
        const _Float16 h = (_Float16)x;
        hi[i] = h;
        lo[i] = (_Float16)(x - (float)h);
    }
}

__device__ __forceinline__ f32x4 mfma3(const f16x8 &ah, const f16x8 &al, const f16x8 &bh, const f16x8 &bl, f32x4 c)
{
    c = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl, c, 0, 0, 0);
}

__device__ __forceinline__ float quad_max(float m)
{
    m = fmaxf(m, __shfl_xor(m, 16, 64));
    return fmaxf(m, __shfl_xor(m, 32, 64));
}

// S6 mixed: Ilm[r][q] = sum_j I0[r][j] WYt[q][j]; WYt = hi, lo FP16 tables [NT*16][Kp], Kp = K up to 32.
// A workgroup of 4 waves takes 64 RT rows (a wave RT tiles of 16 rows); the table is
// staged in LDS per chunk of 64 ordinates ([NT*16][64 + 8] per part).
template <int NT, int RT, int W = 4>
__global__ void __launch_bounds__(64 * W) k_do2sh_f16(long R, int K, int Kp, int NL, const float *__restrict__ A,
                                                   const _Float16 *__restrict__ WYh, const _Float16 *__restrict__ WYl,
                                                   float *__restrict__ C)
{
    constexpr int KC = 64, LS = KC + 8, NC = NT * 16;
    extern __shared__ unsigned char smem_raw[];
    _Float16 *Th = reinterpret_cast<_Float16 *>(smem_raw), *Tl = Th + NC * LS;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lr = lane & 15, lg = lane >> 4;
    const long r0 = (long)xcd_item(gridDim.x) * (16 * W * RT) + wave * (16 * RT);
    const bool vec = (K & 3) == 0;
    const float *Arow[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) Arow[t] = A + min(r0 + 16 * t + lr, R - 1) * (long)K;
    f32x4 acc[RT][NT];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < Kp; kc += KC) {
        __syncthreads();
        // table chunk: columns kc .. kc + 63 of both parts (zero past Kp)
        for (int i = threadIdx.x; i < NC * (KC / 8); i += blockDim.x) {
            const int row = i / (KC / 8), k8 = (i - row * (KC / 8)) * 8;
            f16x8 h = {}, l = {};
            if (kc + k8 < Kp) {
                h = *reinterpret_cast<const f16x8 *>(WYh + (long)row * Kp + kc + k8);
                l = *reinterpret_cast<const f16x8 *>(WYl + (long)row * Kp + kc + k8);
            }
            *reinterpret_cast<f16x8 *>(Th + row * LS + k8) = h;
            *reinterpret_cast<f16x8 *>(Tl + row * LS + k8) = l;
        }
        __syncthreads();
#pragma unroll
        for (int kb = 0; kb < KC; kb += 32) {
            if (kc + kb >= Kp) break;
            const int k = kc + kb + 8 * lg;
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                float v[8];
                if (vec && k + 7 < K) {
                    const f32x4 x = *reinterpret_cast<const f32x4 *>(Arow[t] + k);
                    const f32x4 y = *reinterpret_cast<const f32x4 *>(Arow[t] + k + 4);
                    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w; v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
                } else {
#pragma unroll
                    for (int i = 0; i < 8; ++i) v[i] = (k + i < K) ? Arow[t][k + i] : 0.f;
                }
                float m = 0.f;
#pragma unroll
                for (int i = 0; i < 8; ++i) m = fmaxf(m, fabsf(v[i]));
                float sc, inv;
                fp16_scale(quad_max(m), sc, inv);
                f16x8 ah, al;
                split_f16x8(v, sc, ah, al);
                // inverse scales of the output rows 4 lg + i of this tile
                float ri[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) ri[i] = __shfl(inv, 4 * lg + i, 64);
#pragma unroll
                for (int c = 0; c < NT; ++c) {
                    const int o = (16 * c + lr) * LS + kb + 8 * lg;
                    const f32x4 p = mfma3(ah, al, *reinterpret_cast<const f16x8 *>(Th + o),
                                          *reinterpret_cast<const f16x8 *>(Tl + o), f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc[t][c][i] += p[i] * ri[i];
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            const int col = 16 * c + lr;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long r = r0 + 16 * t + 4 * lg + i;
                if (r < R && col < NL) C[r * NL + col] = acc[t][c][i];
            }
        }
}

// S6 mixed for NT 16-column tiles in one workgroup of W waves (16 W rows): the
// table goes from global memory straight into LDS (global_load_lds, 16 bytes per
// lane) in chunks of 32 ordinates, double buffered, so that the next chunk's table
// and the rows' next 32 values load during the current chunk's products (one
// barrier per chunk).  A chunk is 2 NT blocks of 1 KB (hi, then lo part; column
// tile c): row r of a block (column 16 c + r of the output) at 64 r bytes, its
// ordinates 8 s .. 8 s + 7 in 16-byte slot s ^ ((r >> 2) & 3), so that the 16
// rows a lane group reads fall on distinct banks.  Kp a multiple of 32; the
// tables hold 16 NT rows.  Each row keeps one power-of-two scale that puts its
// largest value so far near 2^8 (FP16 holds up to 65504): a chunk that would pass
// 2^15 under it rescales the row and its sums first, so the products accumulate
// in the matrix-core accumulators and the scale is taken out once at the end.
// What FP16's subnormal floor (2^-24) then drops is below 2^-32 of the row's
// largest value.
template <int NT, int W>
__global__ void __launch_bounds__(64 * W) k_do2sh_f16_dma(long R, int K, int Kp, int NL, const float *__restrict__ A,
                                                       const _Float16 *__restrict__ WYh,
                                                       const _Float16 *__restrict__ WYl, float *__restrict__ C)
{
    constexpr int NB = 2 * NT, BPW = NB / W;                         // 1 KB blocks per chunk, per wave
    static_assert(NB % W == 0, "whole blocks per wave");
    extern __shared__ unsigned char smem_raw[];
    _Float16 *buf = reinterpret_cast<_Float16 *>(smem_raw);         // [2][NB][512]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lr = lane & 15, lg = lane >> 4;
    const long r0 = (long)xcd_item(gridDim.x) * (16 * W) + wave * 16;
    const bool vec = (K & 3) == 0;
    const float *__restrict__ Arow = A + min(r0 + lr, R - 1) * (long)K;
    // the piece this lane moves: row dr of a block, into slot lane & 3 (ordinates 8 ds ..)
    const int dr = lane >> 2, ds = (lane & 3) ^ ((dr >> 2) & 3);
    auto dma = [&](int kc, int b) {
        _Float16 *dst = buf + (size_t)b * NB * 512;
#pragma unroll
        for (int u = 0; u < BPW; ++u) {
            const int blk = wave * BPW + u, part = blk / NT, c = blk - part * NT;
            const _Float16 *src = (part ? WYl : WYh) + (long)(16 * c + dr) * Kp + kc + 8 * ds;
            __builtin_amdgcn_global_load_lds((const void *)src,
                                             (__attribute__((address_space(3))) void *)(dst + blk * 512), 16, 0, 0);
        }
    };
    float nv[8];
    auto load_rows = [&](int kc) {
        const int k = kc + 8 * lg;
        if (vec && k + 7 < K) {
            const f32x4 x = *reinterpret_cast<const f32x4 *>(Arow + k);
            const f32x4 y = *reinterpret_cast<const f32x4 *>(Arow + k + 4);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                nv[i] = x[i];
                nv[4 + i] = y[i];
            }
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) nv[i] = (k + i < K) ? Arow[k + i] : 0.f;
        }
    };
    const int ro = lr * 32 + 8 * (lg ^ ((lr >> 2) & 3));            // this lane's operand slot, in halfs
    f32x4 acc[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nch = Kp / 32;
    float srow = 0.f, irow = 0.f;                       // the row's scale (0 while its values are all 0)
    dma(0, 0);
    load_rows(0);
    for (int ci = 0; ci < nch; ++ci) {
        float v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = nv[i];
        __builtin_amdgcn_s_waitcnt(0);                  // this wave's pieces of the chunk and its values have landed
        __syncthreads();                                // every wave's: the chunk is whole, the other buffer free
        if (ci + 1 < nch) {
            dma(32 * (ci + 1), (ci + 1) & 1);
            load_rows(32 * (ci + 1));
        }
        const _Float16 *Tb = buf + (size_t)(ci & 1) * NB * 512;
        float m = 0.f;
#pragma unroll
        for (int i = 0; i < 8; ++i) m = fmaxf(m, fabsf(v[i]));
        // a row takes a new scale only if one of its four lanes' values asks for it, so
        // the row maximum (two shuffles) is formed only when some lane does
        const bool need = m * srow >= 32768.f || (srow == 0.f && m > 0.f);
        if (__ballot(need) != 0) {                      // wave-uniform: some row of this tile takes a new scale
            m = quad_max(m);
            const bool grow = m * srow >= 32768.f || (srow == 0.f && m > 0.f);
            float f = 1.f;
            if (grow) {
                float sn, in;
                fp16_scale(m, sn, in, 8);
                if (srow != 0.f) f = sn * irow;         // a power of two: the sums rescale exactly
                srow = sn;
                irow = in;
            }
            float fr[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) fr[i] = __shfl(f, 4 * lg + i, 64);
#pragma unroll
            for (int c = 0; c < NT; ++c)
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[c][i] *= fr[i];
        }
        f16x8 ah, al;
        split_f16x8(v, srow, ah, al);
#pragma unroll
        for (int c = 0; c < NT; ++c)
            acc[c] = mfma3(ah, al, *reinterpret_cast<const f16x8 *>(Tb + c * 512 + ro),
                           *reinterpret_cast<const f16x8 *>(Tb + (NT + c) * 512 + ro), acc[c]);
    }
    // inverse scales of the output rows 4 lg + i of this tile
    float ri[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) ri[i] = __shfl(irow, 4 * lg + i, 64);
#pragma unroll
    for (int c = 0; c < NT; ++c) {
        const int col = 16 * c + lr;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const long r = r0 + 4 * lg + i;
            if (r < R && col < NL) C[r * NL + col] = acc[c][i] * ri[i];
        }
    }
}

// S2 mixed: S0[r][j] = sum_q S[r][q] Y[j][q]; Y = hi, lo FP16 tables [Kt][NLp] (Kt = K up to 16,
// NLp = NL up to 32, NB = NLp / 32 blocks); one scale per row.  A workgroup of W waves takes
// 16 W rows; the table is staged in LDS per chunk of 64 ordinates ([64][NLp + 8] per part), the
// next chunk loaded into registers while the current one's products run.
template <int NB, int W = 4>
__global__ void __launch_bounds__(64 * W) k_sh2do_f16(long R, int K, int NL, const float *__restrict__ S,
                                                   const _Float16 *__restrict__ Yh, const _Float16 *__restrict__ Yl,
                                                   float *__restrict__ C)
{
    constexpr int NLp = NB * 32, LS = NLp + 8, JC = 64;
    constexpr int NIT = JC * (NLp / 8), PF = (NIT + 64 * W - 1) / (64 * W);   // 16-byte table pieces
    extern __shared__ unsigned char smem_raw[];
    _Float16 *Th = reinterpret_cast<_Float16 *>(smem_raw), *Tl = Th + JC * LS;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lr = lane & 15, lg = lane >> 4;
    const long r0 = (long)xcd_item(gridDim.x) * (16 * W) + wave * 16;
    const int Kt = (K + 15) / 16 * 16;
    f16x8 ph[PF], pl[PF];
    auto fetch = [&](int jc) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int i = threadIdx.x + u * 64 * W, row = i / (NLp / 8), q8 = (i - row * (NLp / 8)) * 8;
            ph[u] = f16x8{};
            pl[u] = f16x8{};
            if (i < NIT && jc + row < Kt) {
                ph[u] = *reinterpret_cast<const f16x8 *>(Yh + (long)(jc + row) * NLp + q8);
                pl[u] = *reinterpret_cast<const f16x8 *>(Yl + (long)(jc + row) * NLp + q8);
            }
        }
    };
    fetch(0);
    const float *__restrict__ Srow = S + min(r0 + lr, R - 1) * (long)NL;
    float v[NB][8];
    float m = 0.f;
    if ((NL & 7) == 0) {
        // whole 8-value runs (rows 32-byte aligned): two 16-byte loads each
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int q = 32 * b + 8 * lg;
            f32x4 x = {0.f, 0.f, 0.f, 0.f}, y = {0.f, 0.f, 0.f, 0.f};
            if (q < NL) {
                x = *reinterpret_cast<const f32x4 *>(Srow + q);
                y = *reinterpret_cast<const f32x4 *>(Srow + q + 4);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                v[b][i] = x[i];
                v[b][4 + i] = y[i];
            }
        }
    } else {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int q = 32 * b + 8 * lg + i;
                v[b][i] = q < NL ? Srow[q] : 0.f;
            }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 8; ++i) m = fmaxf(m, fabsf(v[b][i]));
    float sc, inv;
    fp16_scale(quad_max(m), sc, inv);
    f16x8 ah[NB], al[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) split_f16x8(v[b], sc, ah[b], al[b]);
    const bool kvec = (K & 3) == 0;
    for (int jc = 0; jc < Kt; jc += JC) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int i = threadIdx.x + u * 64 * W, row = i / (NLp / 8), q8 = (i - row * (NLp / 8)) * 8;
            if (i < NIT) {
                *reinterpret_cast<f16x8 *>(Th + row * LS + q8) = ph[u];
                *reinterpret_cast<f16x8 *>(Tl + row * LS + q8) = pl[u];
            }
        }
        __syncthreads();
        if (jc + JC < Kt) fetch(jc + JC);
#pragma unroll
        for (int c = 0; c < JC / 16; ++c) {
            const int j0 = jc + 16 * c;
            if (j0 >= Kt) break;
            // the tile transposed (table as the first operand): lane (lr, lg) gets ordinates
            // j0 + 4 lg .. + 3 of row r0 + lr, rescaled by that row's own factor and stored
            // as one 16-byte vector
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int o = (16 * c + lr) * LS + 32 * b + 8 * lg;
                acc = mfma3(*reinterpret_cast<const f16x8 *>(Th + o), *reinterpret_cast<const f16x8 *>(Tl + o), ah[b],
                            al[b], acc);
            }
            const int col = j0 + 4 * lg;
            const long r = r0 + lr;
            if (r < R) {
                if (kvec && col + 3 < K) {
                    *reinterpret_cast<f32x4 *>(C + r * K + col) = acc * inv;
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (col + i < K) C[r * K + col + i] = acc[i] * inv;
                }
            }
        }
    }
}

// S2 mixed for NB 32-term SH blocks (NLp = 32 NB) in one workgroup of W waves (16 W rows),
// the table moving from global memory straight into LDS (global_load_lds) in double-
// buffered chunks of 32 ordinates: per part (hi, lo), ordinate tile c (16 ordinates) and
// SH block b one 1 KB block of 16 ordinates x 32 terms, laid out as in k_do2sh_f16_dma
// (ordinate r at 64 r bytes, terms 8 s .. 8 s + 7 in slot s ^ ((r >> 2) & 3)).  The
// tables hold a multiple of 32 ordinates; tiles past Kt (K up to 16) are skipped.
template <int NB, int W>
__global__ void __launch_bounds__(64 * W) k_sh2do_f16_dma(long R, int K, int NL, const float *__restrict__ S,
                                                       const _Float16 *__restrict__ Yh,
                                                       const _Float16 *__restrict__ Yl, float *__restrict__ C)
{
    constexpr int NLp = NB * 32, TPC = 2, NBLK = 2 * TPC * NB, BPW = NBLK / W;
    static_assert(NBLK % W == 0, "whole blocks per wave");
    extern __shared__ unsigned char smem_raw[];
    _Float16 *buf = reinterpret_cast<_Float16 *>(smem_raw);         // [2][NBLK][512]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lr = lane & 15, lg = lane >> 4;
    const long r0 = (long)xcd_item(gridDim.x) * (16 * W) + wave * 16;
    const int Kt = (K + 15) / 16 * 16, nch = (Kt + 31) / 32;
    const int dr = lane >> 2, ds = (lane & 3) ^ ((dr >> 2) & 3);
    auto dma = [&](int jc, int bsel) {
        _Float16 *dst = buf + (size_t)bsel * NBLK * 512;
#pragma unroll
        for (int u = 0; u < BPW; ++u) {
            const int blk = wave * BPW + u, part = blk / (TPC * NB), c = (blk / NB) % TPC, b = blk % NB;
            const _Float16 *src = (part ? Yl : Yh) + (long)(jc + 16 * c + dr) * NLp + 32 * b + 8 * ds;
            __builtin_amdgcn_global_load_lds((const void *)src,
                                             (__attribute__((address_space(3))) void *)(dst + blk * 512), 16, 0, 0);
        }
    };
    dma(0, 0);
    const float *__restrict__ Srow = S + min(r0 + lr, R - 1) * (long)NL;
    float v[NB][8];
    if ((NL & 7) == 0) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int q = 32 * b + 8 * lg;
            f32x4 x = {0.f, 0.f, 0.f, 0.f}, y = {0.f, 0.f, 0.f, 0.f};
            if (q < NL) {
                x = *reinterpret_cast<const f32x4 *>(Srow + q);
                y = *reinterpret_cast<const f32x4 *>(Srow + q + 4);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                v[b][i] = x[i];
                v[b][4 + i] = y[i];
            }
        }
    } else {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int q = 32 * b + 8 * lg + i;
                v[b][i] = q < NL ? Srow[q] : 0.f;
            }
    }
    float m = 0.f;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 8; ++i) m = fmaxf(m, fabsf(v[b][i]));
    float sc, inv;
    fp16_scale(quad_max(m), sc, inv);
    f16x8 ah[NB], al[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) split_f16x8(v[b], sc, ah[b], al[b]);
    const int ro = lr * 32 + 8 * (lg ^ ((lr >> 2) & 3));
    const bool kvec = (K & 3) == 0;
    const long r = r0 + lr;
    for (int ci = 0; ci < nch; ++ci) {
        __builtin_amdgcn_s_waitcnt(0);                  // this wave's pieces of the chunk have landed
        __syncthreads();                                // every wave's: the chunk is whole, the other buffer free
        if (ci + 1 < nch) dma(32 * (ci + 1), (ci + 1) & 1);
        const _Float16 *Tb = buf + (size_t)(ci & 1) * NBLK * 512;
#pragma unroll
        for (int c = 0; c < TPC; ++c) {
            const int j0 = 32 * ci + 16 * c;
            if (j0 >= Kt) break;
            // the tile transposed (table as the first operand): lane (lr, lg) gets ordinates
            // j0 + 4 lg .. + 3 of row r0 + lr, rescaled by that row's own factor
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int b = 0; b < NB; ++b)
                acc = mfma3(*reinterpret_cast<const f16x8 *>(Tb + (c * NB + b) * 512 + ro),
                            *reinterpret_cast<const f16x8 *>(Tb + ((TPC + c) * NB + b) * 512 + ro), ah[b], al[b], acc);
            const int col = j0 + 4 * lg;
            if (r < R) {
                if (kvec && col + 3 < K) {
                    *reinterpret_cast<f32x4 *>(C + r * K + col) = acc * inv;
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (col + i < K) C[r * K + col + i] = acc[i] * inv;
                }
            }
        }
    }
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
    const long p = pj / G;
    const real chi = a.chi0[pj];
    if (!(chi > real(0))) { a.S[idx] = 0; return; }
    int l = (int)sqrtf((float)q);
    while (l * l > q) --l;
    while ((l + 1) * (l + 1) <= q) ++l;
    const real cl = (l == 0) ? real(1) : (l == 2 ? real(0.1) : real(0));   // chi_l/(2l+1), Thomson
    real v = a.sigma[p] / chi * cl * a.Ilm[idx];
    if (q == 0) v += real(3.5449077018110318) * a.kappa[pj] * a.bnu[pj] / chi;   // sqrt(4 pi) kappa B / chi
    a.S[idx] = v;
}

// Thomson source fused with the residual's row sums (NL dividing 64): a wave
// takes 64 / NL (point, group) rows, computes their new source coefficients,
// and reduces sum (S_new - S_old)^2 and sum S_new^2 of each row in FP64 across
// the row's lanes; rows[g P + p] and rows[(G + g) P + p] receive them (the
// per-group totals follow in k_resid_part / k_resid_fin)
template <typename real>
__global__ void __launch_bounds__(256) k_source_resid(SourceArgs<real> a, const real *__restrict__ Sold, double *rows)
{
    const int G = a.G, NL = a.NL, RW = 64 / NL;
    const long PG = a.P * G;
    const int lane = threadIdx.x & 63, sub = lane / NL, q = lane - sub * NL;
    const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long nwaves = ((long)gridDim.x * blockDim.x) >> 6;
    int l = (int)sqrtf((float)q);
    while (l * l > q) --l;
    while ((l + 1) * (l + 1) <= q) ++l;
    const real cl = (l == 0) ? real(1) : (l == 2 ? real(0.1) : real(0));   // chi_l/(2l+1), Thomson
    for (long r0 = wave * RW; r0 < PG; r0 += nwaves * RW) {
        const long r = r0 + sub;
        double dd = 0.0, aa = 0.0;
        if (r < PG) {
            const long idx = r * NL + q, p = r / G;
            const real chi = a.chi0[r];
            real v = 0;
            if (chi > real(0)) {
                v = a.sigma[p] / chi * cl * a.Ilm[idx];
                if (q == 0) v += real(3.5449077018110318) * a.kappa[r] * a.bnu[r] / chi;   // sqrt(4 pi) kappa B / chi
            }
            a.S[idx] = v;
            const double u = (double)v, d = u - (double)Sold[idx];
            dd = d * d;
            aa = u * u;
        }
        for (int off = NL >> 1; off > 0; off >>= 1) {
            dd += __shfl_xor(dd, off, 64);
            aa += __shfl_xor(aa, off, 64);
        }
        if (q == 0 && r < PG) {
            const long pp = r / G, g = r - pp * G;
            rows[g * a.P + pp] = dd;
            rows[(G + g) * a.P + pp] = aa;
        }
    }
}

// sum of x over each row of 16 lanes, left in every lane of the row: four DPP moves
// between registers (lane xor 1 and xor 2 within quads, then the mirrored lane of the
// half row and of the row), no LDS traffic and no waits
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double row16_sum(double x)
{
    x += dpp_move<0xB1>(x);                             // quad_perm [1, 0, 3, 2]
    x += dpp_move<0x4E>(x);                             // quad_perm [2, 3, 0, 1]
    x += dpp_move<0x141>(x);                            // row_half_mirror
    x += dpp_move<0x140>(x);                            // row_mirror
    return x;
}

// the same with four coefficients per lane (16-byte loads and stores; NL a multiple of 4 with
// NL / 4 dividing 64): a wave takes 256 / NL rows
template <typename real>
__global__ void __launch_bounds__(256) k_source_resid4(SourceArgs<real> a, const real *__restrict__ Sold, double *rows)
{
    using P4 = Pack<real, 4>;
    const int G = a.G, NL = a.NL, LR = NL >> 2, RW = 64 / LR;
    const long PG = a.P * G;
    const int lane = threadIdx.x & 63, sub = lane / LR, q0 = (lane - sub * LR) * 4;
    const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long nwaves = ((long)gridDim.x * blockDim.x) >> 6;
    real cl[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int q = q0 + c;
        int l = (int)sqrtf((float)q);
        while (l * l > q) --l;
        while ((l + 1) * (l + 1) <= q) ++l;
        cl[c] = (l == 0) ? real(1) : (l == 2 ? real(0.1) : real(0));   // chi_l/(2l+1), Thomson
    }
    for (long r0 = wave * RW; r0 < PG; r0 += nwaves * RW) {
        const long r = r0 + sub;
        double dd = 0.0, aa = 0.0;
        if (r < PG) {
            const long idx = r * NL + q0, p = r / G;
            const real chi = a.chi0[r];
            const P4 in = *reinterpret_cast<const P4 *>(a.Ilm + idx);
            const P4 old = *reinterpret_cast<const P4 *>(Sold + idx);
            P4 v{};
            if (chi > real(0)) {
                const real f = a.sigma[p] / chi;
#pragma unroll
                for (int c = 0; c < 4; ++c) v.v[c] = f * cl[c] * in.v[c];
                if (q0 == 0) v.v[0] += real(3.5449077018110318) * a.kappa[r] * a.bnu[r] / chi;
            }
            *reinterpret_cast<P4 *>(a.S + idx) = v;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double u = (double)v.v[c], d = u - (double)old.v[c];
                dd += d * d;
                aa += u * u;
            }
        }
        if (LR == 16) {                                    // a row is one DPP row of 16 lanes
            dd = row16_sum(dd);
            aa = row16_sum(aa);
        } else {
            for (int off = LR >> 1; off > 0; off >>= 1) {
                dd += __shfl_xor(dd, off, 64);
                aa += __shfl_xor(aa, off, 64);
            }
        }
        if (q0 == 0 && r < PG) {
            const long pp = r / G, g = r - pp * G;
            rows[g * a.P + pp] = dd;
            rows[(G + g) * a.P + pp] = aa;
        }
    }
}

// Compton: one workgroup per point; its SH intensities I[i][q] (all groups) are
// staged in LDS and S[j][q] = sigma/chi_j sum_i A_l(q)[j][i] I[i][q] + T_q
// SH order of an expansion with nl terms
__device__ __forceinline__ int lmax_of(int nl)
{
    int l = (int)sqrtf((float)nl) - 1;
    while ((l + 1) * (l + 1) < nl) ++l;
    while (l > 0 && l * l >= nl) --l;
    return l;
}

template <typename real>
__global__ void __launch_bounds__(256) k_source_compton(SourceArgs<real> a)
{
    extern __shared__ unsigned char smem_raw[];
    real *sI = reinterpret_cast<real *>(smem_raw);
    const long p = xcd_item(a.P);
    if (p >= a.P) return;
    const int G = a.G, NL = a.NL, T = blockDim.x;
    const real *__restrict__ Ip = a.Ilm + p * G * NL;
    for (int i = threadIdx.x; i < G * NL; i += T) sI[i] = Ip[i];
    __syncthreads();
    const real sig = a.sigma[p];
    const float rNL = 1.0f / (float)NL;
    for (int o = threadIdx.x; o < G * NL; o += T) {
        const int j = (int)(((float)o + 0.5f) * rNL), q = o - j * NL;
        int l = (int)sqrtf((float)q);
        while (l * l > q) --l;
        while ((l + 1) * (l + 1) <= q) ++l;
        const real chi = a.chi0[p * G + j];
        real v = 0;
        if (chi > real(0)) {
            const long LGG = (long)(a.NL > 0 ? lmax_of(a.NL) + 1 : 1) * G * G;
            const long n = a.tnode ? a.tnode[p] : 0;
            const real w = a.tnode ? a.twt[p] : real(0);
            const real *__restrict__ Arow = a.A + n * LGG + ((long)l * G + j) * G;
            real acc = 0;
            if (w > real(0)) {
                const real *__restrict__ Brow = Arow + LGG;
                for (int i = 0; i < G; ++i) acc += ((real(1) - w) * Arow[i] + w * Brow[i]) * sI[i * NL + q];
            } else {
                for (int i = 0; i < G; ++i) acc += Arow[i] * sI[i * NL + q];
            }
            v = sig / chi * acc;
            if (q == 0) v += real(3.5449077018110318) * a.kappa[p * G + j] * a.bnu[p * G + j] / chi;
        }
        a.S[p * G * NL + o] = v;
    }
}

// Compton source on the matrix cores (FP32, G <= 32, L <= 15): for each l the
// group-to-group product S_l = A_l I_l is a 32 x 32 (j x i) by 32 x (2l + 1)
// (i x q) product.  Wave w of eight takes the angular orders l = w and w + 8
// and holds their A_l in registers for the whole launch: order w (at most 15
// columns) as two 16-row v_mfma_f32_16x16x4f32 chains of K = 32 (16 columns),
// order w + 8 as one v_mfma_f32_32x32x2f32 chain (32 columns); the workgroup walks points (persistent), staging a point's
// SH intensities in LDS while the next point's are loaded into registers.  The
// products overwrite the intensities in LDS (a wave writes only the columns of
// its own orders, after it has read them) and leave as 16-byte scaled stores.
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kComptonMfmaThreads = 512;

template <bool TEMP, bool RESID>
__global__ void __launch_bounds__(kComptonMfmaThreads, TEMP ? 2 : 4)
    k_source_compton_mfma(SourceArgs<float> a, int lmax, const float *__restrict__ Sold, double *__restrict__ rows)
{
    typedef float P4 __attribute__((ext_vector_type(4)));
    constexpr int RS = 256;                                // LDS row stride (the largest NL), 32 rows
    extern __shared__ unsigned char smem_raw[];
    const int G = a.G, NL = a.NL, GN = G * NL, GN4 = GN >> 2, NL4 = NL >> 2;
    float *sI = reinterpret_cast<float *>(smem_raw);     // [32][RS] intensities, then products, of the point
    float *sF = sI + 32 * RS;                              // [G] sigma / chi_j (0 where chi_j = 0)
    float *sT = sF + G;                                    // [G] thermal term of q = 0
    float *sO = sF + ((2 * G + 3) & ~3);                   // RESID: [G NL] the point's old source (16-byte aligned)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = lane & 31, kh = lane >> 5;               // B / C column, K half
    // rows G..31 stay zero: they meet zero columns of A
    for (int i = G * RS + tid; i < 32 * RS; i += kComptonMfmaThreads) sI[i] = 0.0f;
    // A_l[m][k] for this wave's orders: for order w + 8 (32 x 32 x 2) lane holds
    // m = n, k = 2 ks + kh in element ks; for order w (16 x 16 x 4) element e holds
    // m = 16 (e / 8) + lane % 16, k = 4 (e % 8) + lane / 16.  With temperature nodes the lane holds the lower node's table (A0) and the
    // difference to the upper one (Ad) of the bracket in use, reloaded when a
    // point's bracket differs (points come in order, and a smooth temperature
    // field changes bracket rarely); a point's table is A0 + w Ad.
    const long LGG = (long)(lmax + 1) * G * G;
    float A0[2][16], Ad[2][TEMP ? 16 : 1];
    int cur = -1;
    float w = 0.0f;
    auto load_tables = [&](int node) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int l = wave + 8 * t;
#pragma unroll
            for (int ks = 0; ks < 16; ++ks) {
                const int m = t ? n : 16 * (ks >> 3) + (lane & 15);
                const int k = t ? 2 * ks + kh : 4 * (ks & 7) + (lane >> 4);
                const bool in = l <= lmax && m < G && k < G;
                const long o = node * LGG + ((long)l * G + m) * G + k;
                A0[t][ks] = in ? a.A[o] : 0.0f;
                if (TEMP) Ad[t][ks] = in ? a.A[o + LGG] - A0[t][ks] : 0.0f;
            }
        }
        cur = node;
    };
    // contiguous points per workgroup; with temperature nodes in the order of
    // their bracket, so that a workgroup reloads its tables rarely
    const long chunk = (a.P + gridDim.x - 1) / gridDim.x;
    const long pbeg = (long)blockIdx.x * chunk, pend = min(a.P, pbeg + chunk);
    constexpr int kPre = 4;                                // 16-byte loads per thread and point (G NL <= 8192)
    P4 pre[kPre], preo[RESID ? kPre : 1];
    float pchi = 0.0f, pkap = 0.0f, pbnu = 0.0f, psig = 0.0f;
    auto point = [&](long idx) -> long { return TEMP ? (long)a.torder[idx] : idx; };
    auto fetch = [&](long idx) {
        const long p = point(idx);
        const P4 *src = reinterpret_cast<const P4 *>(a.Ilm + p * GN);
        const P4 *osrc = reinterpret_cast<const P4 *>(Sold + p * GN);
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
            const int i = tid + u * kComptonMfmaThreads;
            if (i < GN4) {
                pre[u] = src[i];
                if (RESID) preo[u] = osrc[i];
            }
        }
        if (tid < G) {
            pchi = a.chi0[p * G + tid];
            pkap = a.kappa[p * G + tid];
            pbnu = a.bnu[p * G + tid];
            psig = a.sigma[p];
        }
    };
    if (pbeg < pend) fetch(pbeg);
    for (long idx = pbeg; idx < pend; ++idx) {
        const long p = point(idx);
        {
            const int node = TEMP ? a.tnode[p] : 0;
            if (TEMP) w = a.twt[p];
            if (node != cur) load_tables(node);
        }
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
            const int i = tid + u * kComptonMfmaThreads;
            if (i < GN4) {
                const int j = i / NL4, q = (i - j * NL4) * 4;
                *reinterpret_cast<P4 *>(sI + j * RS + q) = pre[u];
                if (RESID) reinterpret_cast<P4 *>(sO)[i] = preo[u];
            }
        }
        if (tid < G) {
            const bool on = pchi > 0.0f;
            sF[tid] = on ? psig / pchi : 0.0f;
            sT[tid] = on ? 3.5449077018110318f * pkap * pbnu / pchi : 0.0f;
        }
        if (idx + 1 < pend) fetch(idx + 1);
        __syncthreads();
        // order w: two 16 x 16 x 4 chains (rows 0-15, 16-31) over 16 columns
        if (wave <= lmax) {
            const int l = wave, q0 = l * l, nq = 2 * l + 1;
            const int cn = lane & 15, kg = lane >> 4;
            const float *col = sI + q0 + min(cn, nq - 1);
            float b[8];
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) b[ks] = col[(4 * ks + kg) * RS];
            asm volatile("" : "+v"(b[0]), "+v"(b[1]), "+v"(b[2]), "+v"(b[3]), "+v"(b[4]), "+v"(b[5]), "+v"(b[6]),
                         "+v"(b[7]));
            f32x4 lo = {0.f, 0.f, 0.f, 0.f}, hi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) {
                lo = __builtin_amdgcn_mfma_f32_16x16x4f32(TEMP ? A0[0][ks] + w * Ad[0][ks % (TEMP ? 16 : 1)] : A0[0][ks],
                                                          b[ks], lo, 0, 0, 0);
                hi = __builtin_amdgcn_mfma_f32_16x16x4f32(
                    TEMP ? A0[0][8 + ks] + w * Ad[0][(8 + ks) % (TEMP ? 16 : 1)] : A0[0][8 + ks], b[ks], hi, 0, 0, 0);
            }
            // register r of lane l holds row 4 (l / 16) + r of column l % 16 (+ 16 for hi)
            if (cn < nq) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = 4 * kg + r;
                    if (m < G) sI[m * RS + q0 + cn] = lo[r];
                    if (m + 16 < G) sI[(m + 16) * RS + q0 + cn] = hi[r];
                }
            }
        }
#pragma unroll
        for (int t = 1; t < 2; ++t) {
            const int l = wave + 8 * t;
            if (l > lmax) break;
            const int q0 = l * l, nq = 2 * l + 1;
            // B operand: columns n >= nq repeat the last column (their outputs are not kept)
            const float *col = sI + kh * RS + q0 + min(n, nq - 1);
            float b[16];
#pragma unroll
            for (int ks = 0; ks < 16; ++ks) b[ks] = col[2 * ks * RS];
            // all sixteen reads issued before the first product (one wait instead of sixteen)
            asm volatile("" : "+v"(b[0]), "+v"(b[1]), "+v"(b[2]), "+v"(b[3]), "+v"(b[4]), "+v"(b[5]), "+v"(b[6]),
                         "+v"(b[7]), "+v"(b[8]), "+v"(b[9]), "+v"(b[10]), "+v"(b[11]), "+v"(b[12]), "+v"(b[13]),
                         "+v"(b[14]), "+v"(b[15]));
            f32x16 acc;
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
            for (int ks = 0; ks < 16; ++ks)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(TEMP ? A0[t][ks] + w * Ad[t][ks % (TEMP ? 16 : 1)] : A0[t][ks],
                                                           b[ks], acc, 0, 0, 0);
            // element (m, n) sits in register r of lane n + 32 ((m / 4) % 2), r = 4 (m / 8) + m % 4;
            // it overwrites the intensity it replaces (this wave's own columns, already read)
            if (n < nq) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int m = 8 * (r >> 2) + 4 * kh + (r & 3);
                    if (m < G) sI[m * RS + q0 + n] = acc[r];
                }
            }
        }
        __syncthreads();
        // S[j][q] = sigma / chi_j (A I)[j][q], plus the thermal term at q = 0; with RESID
        // also each row's sums (S - S_old)^2 and S^2 in FP64, for the residual
        float *dst = a.S + p * GN;
        if (NL4 % kPre == 0) {
            // a row is NL4 / 4 consecutive lanes, each with four of its 16-byte pieces
            // (the lanes of a row store 256-byte runs), so that the row sums take
            // log2(NL4 / 4) cross-lane steps once per point
            const int tpr = NL4 / kPre, j = tid / tpr, t = tid - j * tpr;
            double dd = 0.0, aa = 0.0;
            if (j < G) {
                const float f = sF[j];
#pragma unroll
                for (int u = 0; u < kPre; ++u) {
                    const int q4 = t + tpr * u, i = j * NL4 + q4;
                    P4 v = *reinterpret_cast<const P4 *>(sI + j * RS + 4 * q4);
                    v *= f;
                    if (q4 == 0) v.x += sT[j];
                    reinterpret_cast<P4 *>(dst)[i] = v;
                    if (RESID) {
                        const P4 o = reinterpret_cast<const P4 *>(sO)[i];
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            const double uu = (double)v[c], d = uu - (double)o[c];
                            dd += d * d;
                            aa += uu * uu;
                        }
                    }
                }
            }
            if (RESID) {
                if (tpr == 16) {                           // a row is one DPP row of 16 lanes
                    dd = row16_sum(dd);
                    aa = row16_sum(aa);
                } else {
                    for (int off = tpr >> 1; off > 0; off >>= 1) {
                        dd += __shfl_xor(dd, off, 64);
                        aa += __shfl_xor(aa, off, 64);
                    }
                }
                if (j < G && t == 0) {
                    rows[(long)j * a.P + p] = dd;
                    rows[(long)(G + j) * a.P + p] = aa;
                }
            }
            __syncthreads();                               // the next point overwrites the table and factors
            continue;
        }
        // a row is NL4 consecutive lanes, NL4 dividing 64
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
            const int i = tid + u * kComptonMfmaThreads;
            double dd = 0.0, aa = 0.0;
            if (i < GN4) {
                const int j = i / NL4, q = (i - j * NL4) * 4;
                const float f = sF[j];
                P4 v = *reinterpret_cast<const P4 *>(sI + j * RS + q);
                v *= f;
                if (q == 0) v.x += sT[j];
                reinterpret_cast<P4 *>(dst)[i] = v;
                if (RESID) {
                    const P4 o = reinterpret_cast<const P4 *>(sO)[i];
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const double uu = (double)v[c], d = uu - (double)o[c];
                        dd += d * d;
                        aa += uu * uu;
                    }
                }
            }
            if (RESID) {
                for (int off = NL4 >> 1; off > 0; off >>= 1) {
                    dd += __shfl_xor(dd, off, 64);
                    aa += __shfl_xor(aa, off, 64);
                }
                if (i < GN4 && i % NL4 == 0) {
                    const int j = i / NL4;
                    rows[(long)j * a.P + p] = dd;
                    rows[(long)(G + j) * a.P + p] = aa;
                }
            }
        }
        __syncthreads();                                   // the next point overwrites the table and factors
    }
}

// chi0 = kappa + sigma * s_g
template <typename real>
__global__ void k_chi0(long P, int G, const real *__restrict__ kappa, const real *__restrict__ sigma,
                       const real *__restrict__ sg, const int *__restrict__ tnode, const real *__restrict__ twt,
                       real *__restrict__ chi0)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P * G) return;
    const long p = idx / G;
    const int g = (int)(idx - p * G);
    real s = real(1);
    if (sg) {
        if (tnode) {
            const long n = tnode[p];
            const real w = twt[p];
            s = sg[n * G + g];
            if (w > real(0)) s = (real(1) - w) * s + w * sg[(n + 1) * G + g];
        } else {
            s = sg[g];
        }
    }
    chi0[idx] = kappa[idx] + sigma[p] * s;
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
    const long p = idx / G;
    const int g = (int)(idx - p * G);
    double j = 0, h0 = 0, h1 = 0, h2 = 0, k0 = 0, k1 = 0, k2 = 0, k3 = 0, k4 = 0, k5 = 0;
    for (int k = 0; k < K; ++k) {
        const double nx = dir[4 * k], ny = dir[4 * k + 1], nz = dir[4 * k + 2], w = dir[4 * k + 3];
        const double v = w * (double)I[(long)k * P * G + idx];
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

// per (point, group) row of NL SH terms: sum (a-b)^2 and sum a^2; one wave per
// row (lanes stride the row, then a shuffle reduction), rows strided over waves
template <typename real>
__global__ void __launch_bounds__(256) k_resid_rows(long P, int G, int NL, const real *__restrict__ a,
                                                    const real *__restrict__ b, double *rows)
{
    const int lane = threadIdx.x & 63;
    const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long nwaves = ((long)gridDim.x * blockDim.x) >> 6;
    const long PG = P * G;
    for (long r = wave; r < PG; r += nwaves) {
        const real *x = a + r * NL, *y = b + r * NL;
        double dd = 0, aa = 0;
        for (int q = lane; q < NL; q += 64) {
            const double u = (double)x[q], d = u - (double)y[q];
            dd += d * d;
            aa += u * u;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            dd += __shfl_xor(dd, off, 64);
            aa += __shfl_xor(aa, off, 64);
        }
        if (lane == 0) {
            const long pp = r / G, g = r - pp * G;
            rows[g * P + pp] = dd;
            rows[(G + g) * P + pp] = aa;
        }
    }
}

// Per-group totals of the row sums, out[2g + c] = sum over points of
// rows[(c G + g) P + p], in two passes with a fixed order: block (s, cg) sums
// chunk s of row block cg into part[cg S + s] (two loads in flight per thread),
// then one thread per row block adds its S partial sums in order.
__global__ void __launch_bounds__(256) k_resid_part(long P, int S, const double *__restrict__ rows, double *part)
{
    __shared__ double sh[256];
    const int cg = blockIdx.y, s = blockIdx.x;
    const long chunk = (P + S - 1) / S, b = (long)s * chunk, e = min(P, b + chunk);
    const double *__restrict__ x = rows + (long)cg * P;
    double v0 = 0, v1 = 0;
    long p = b + threadIdx.x;
    for (; p + 256 < e; p += 512) {
        v0 += x[p];
        v1 += x[p + 256];
    }
    if (p < e) v0 += x[p];
    const double v = block_sum(v0 + v1, sh);
    if (threadIdx.x == 0) part[(long)cg * S + s] = v;
}
__global__ void __launch_bounds__(64) k_resid_fin(int G, int S, const double *__restrict__ part, double *out)
{
    const int cg = blockIdx.x * blockDim.x + threadIdx.x;
    if (cg >= 2 * G) return;
    double v = 0;
    for (int s = 0; s < S; ++s) v += part[(long)cg * S + s];
    const int c = cg / G, g = cg - c * G;
    out[2 * g + c] = v;
}
static void launch_group_totals(long P, int G, const double *rows, double *out, hipStream_t st)
{
    // about 1024 blocks over the 2 G row blocks, chunks of at least 512 points
    const long S = std::max<long>(1, std::min<long>({kResidSplit, (1024 + 2 * G - 1) / (2 * G), P / 512}));
    double *part = const_cast<double *>(rows) + 2 * P * G;
    hipLaunchKernelGGL(k_resid_part, dim3((unsigned)S, 2 * G), dim3(256), 0, st, P, (int)S, rows, part);
    hipLaunchKernelGGL(k_resid_fin, dim3((2 * G + 63) / 64), dim3(64), 0, st, G, (int)S, part, out);
}

// five dot products for the Ng extrapolation from the chain s3 (oldest) .. s0
// (arrays [P][G][NL]), each group weighted by 1/||s0_g||^2 taken from the
// per-group sums red[2 g + 1] that the last residual left (floored at floor2
// times the largest, as in the convergence test)
template <typename real>
__global__ void __launch_bounds__(256) k_ng_partial(long n, int G, int NL, const double *__restrict__ red, double floor2,
                                                    const real *__restrict__ s0, const real *__restrict__ s1,
                                                    const real *__restrict__ s2, const real *__restrict__ s3, double *partial)
{
    extern __shared__ unsigned char smem_raw[];
    double *w = reinterpret_cast<double *>(smem_raw);               // [G]
    __shared__ double sh[256];
    double amax = 0;
    for (int g = 0; g < G; ++g) amax = fmax(amax, red[2 * g + 1]);
    for (int g = threadIdx.x; g < G; g += blockDim.x) {
        const double d = fmax(red[2 * g + 1], floor2 * amax);
        w[g] = d > 0 ? 1.0 / d : 1.0;
    }
    __syncthreads();
    double a11 = 0, a12 = 0, a22 = 0, b1 = 0, b2 = 0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double wg = w[(i / NL) % G];
        const double x0 = s0[i], x1 = s1[i], x2 = s2[i], x3 = s3[i];
        const double d0 = x0 - x1, d1 = x1 - x2, d2 = x2 - x3;
        const double q1 = d0 - d1, q2 = d0 - d2;
        a11 += wg * q1 * q1; a12 += wg * q1 * q2; a22 += wg * q2 * q2; b1 += wg * d0 * q1; b2 += wg * d0 * q2;
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

// Ng extrapolation from the FP64 dot products d = (a11, a12, a22, b1, b2) of
// the differences of the last four iterates: (a, b) solve the 2 x 2 normal
// equations and out = (1 - a - b) s3 + a s2 + b s1; nothing is written when
// the system is singular.  Every thread forms the same coefficients, so no
// host round trip is needed.
template <typename real>
__global__ void k_ng_extrapolate(long n, const double *__restrict__ d, const real *__restrict__ s3,
                                 const real *__restrict__ s2, const real *__restrict__ s1, real *__restrict__ out)
{
    const double a11 = d[0], a12 = d[1], a22 = d[2], b1 = d[3], b2 = d[4];
    const double det = a11 * a22 - a12 * a12;
    if (!(det > 1e-14 * a11 * a22) || !isfinite(det)) return;
    const double a = (b1 * a22 - b2 * a12) / det, b = (b2 * a11 - b1 * a12) / det;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = (real)((1.0 - a - b) * (double)s3[i] + a * (double)s2[i] + b * (double)s1[i]);
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
size_t trace_lds(int nx, int ny, int Gc, int chi_per_point)
{
    return sizeof(real) * (size_t)(nx + 1) * (ny + 1) *
           ((kRing + kIBuf) * (size_t)Gc + kRing * (chi_per_point ? 1 : (size_t)Gc));
}
// lab ordinate arrays [k][p][g] <-> [k][g][p], through an LDS tile of 64 points x
// up to 32 groups (both sides read and written in contiguous runs)
template <typename real>
__global__ void __launch_bounds__(256) k_transpose_lab(const real *__restrict__ in, real *__restrict__ out, long P,
                                                       int G, int to_gmajor)
{
    __shared__ real tile[64][33];
    const long k = blockIdx.y, p0 = (long)blockIdx.x * 64;
    const int np = (int)min(64L, P - p0);
    for (int g0 = 0; g0 < G; g0 += 32) {
        const int gn = min(32, G - g0), n = np * gn;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            if (to_gmajor) {
                const int pp = i / gn, gg = i - pp * gn;
                tile[pp][gg] = in[(k * P + p0 + pp) * G + g0 + gg];
            } else {
                const int gg = i / np, pp = i - gg * np;
                tile[pp][gg] = in[(k * G + g0 + gg) * P + p0 + pp];
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            if (to_gmajor) {
                const int gg = i / np, pp = i - gg * np;
                out[(k * G + g0 + gg) * P + p0 + pp] = tile[pp][gg];
            } else {
                const int pp = i / gn, gg = i - pp * gn;
                out[(k * P + p0 + pp) * G + g0 + gg] = tile[pp][gg];
            }
        }
        __syncthreads();
    }
}

// the same with 16-byte loads and stores (G and P multiples of 4): a tile of 128
// points x up to 32 groups, every lane's loads in flight before the LDS writes
template <typename real>
__global__ void __launch_bounds__(256) k_transpose_lab4(const real *__restrict__ in, real *__restrict__ out, long P,
                                                        int G, int to_gmajor)
{
    using P4 = Pack<real, 4>;
    constexpr int TP = 128, TS = 33;
    __shared__ real tile[TP * TS];
    const long k = blockIdx.y, p0 = (long)blockIdx.x * TP;
    const int np = (int)min((long)TP, P - p0);             // a multiple of 4
    for (int g0 = 0; g0 < G; g0 += 32) {
        const int gn = min(32, G - g0), gn4 = gn >> 2, np4 = np >> 2;
        const int n4 = np * gn4;                            // 16-byte pieces of the tile
        P4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int f = threadIdx.x + u * 256;
            if (f < n4) {
                if (to_gmajor) {
                    const int pp = f / gn4, g4 = f - pp * gn4;
                    v[u] = load_stream(in + (k * P + p0 + pp) * G + g0 + 4 * g4);
                } else {
                    const int gg = f / np4, p4 = f - gg * np4;
                    v[u] = load_stream(in + (k * G + g0 + gg) * P + p0 + 4 * p4);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int f = threadIdx.x + u * 256;
            if (f < n4) {
                if (to_gmajor) {
                    const int pp = f / gn4, g4 = f - pp * gn4;
#pragma unroll
                    for (int i = 0; i < 4; ++i) tile[pp * TS + 4 * g4 + i] = v[u].v[i];
                } else {
                    const int gg = f / np4, p4 = f - gg * np4;
#pragma unroll
                    for (int i = 0; i < 4; ++i) tile[(4 * p4 + i) * TS + gg] = v[u].v[i];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int f = threadIdx.x + u * 256;
            if (f < n4) {
                P4 w;
                if (to_gmajor) {
                    const int gg = f / np4, p4 = f - gg * np4;
#pragma unroll
                    for (int i = 0; i < 4; ++i) w.v[i] = tile[(4 * p4 + i) * TS + gg];
                    *reinterpret_cast<P4 *>(out + (k * G + g0 + gg) * P + p0 + 4 * p4) = w;
                } else {
                    const int pp = f / gn4, g4 = f - pp * gn4;
#pragma unroll
                    for (int i = 0; i < 4; ++i) w.v[i] = tile[pp * TS + 4 * g4 + i];
                    store_stream(out + (k * P + p0 + pp) * G + g0 + 4 * g4, w);
                }
            }
        }
        __syncthreads();
    }
}
template <typename real>
void launch_transpose_lab(const real *in, real *out, long P, int G, int K, bool to_gmajor, hipStream_t st)
{
    if (G % 4 == 0 && P % 4 == 0) {
        hipLaunchKernelGGL(k_transpose_lab4<real>, dim3((unsigned)((P + 127) / 128), (unsigned)K), dim3(256), 0, st, in,
                           out, P, G, (int)to_gmajor);
        return;
    }
    hipLaunchKernelGGL(k_transpose_lab<real>, dim3((unsigned)((P + 63) / 64), (unsigned)K), dim3(256), 0, st, in, out,
                       P, G, (int)to_gmajor);
}
template <typename real>
void launch_trace(const TraceArgs<real> &a, bool chi_array, hipStream_t st)
{
    const size_t sm = trace_lds<real>(a.nx, a.ny, a.Gc, !chi_array && a.chi_grey);
    const int nch = a.G / a.Gc;
    const int npt = (a.nx * a.ny + kTraceThreads - 1) / kTraceThreads;
    // ordinates whose path takes several pieces first (a.order lists them first), then
    // the single-piece ones; each launch gives every XCD every eighth ordinate
    const int parts[2][2] = {{0, a.nmulti}, {a.nmulti, a.K - a.nmulti}};
    for (int part = 0; part < 2; ++part) {
        const int r0 = parts[part][0], nr = parts[part][1];
        if (nr <= 0) continue;
        const dim3 grid((unsigned)(8 * ((nr + 7) / 8) * nch)), block(kTraceThreads);
#define RRT_TRACE_CASE(GC, MP)                                                                                   \
        if (a.Gc == GC && npt <= MP) {                                                                           \
            if (part == 0) {                                                                                     \
                if (chi_array) hipLaunchKernelGGL((k_trace<real, kChiArray, GC, MP, true>), grid, block, sm, st, a, r0, nr); \
                else if (a.chi_grey) hipLaunchKernelGGL((k_trace<real, kChiGrey, GC, MP, true>), grid, block, sm, st, a, r0, nr); \
                else hipLaunchKernelGGL((k_trace<real, kChiGroup, GC, MP, true>), grid, block, sm, st, a, r0, nr); \
            } else {                                                                                             \
                if (chi_array) hipLaunchKernelGGL((k_trace<real, kChiArray, GC, MP, false>), grid, block, sm, st, a, r0, nr); \
                else if (a.chi_grey) hipLaunchKernelGGL((k_trace<real, kChiGrey, GC, MP, false>), grid, block, sm, st, a, r0, nr); \
                else hipLaunchKernelGGL((k_trace<real, kChiGroup, GC, MP, false>), grid, block, sm, st, a, r0, nr); \
            }                                                                                                    \
            continue;                                                                                            \
        }
        RRT_TRACE_CASE(1, 1)
        RRT_TRACE_CASE(1, 2)
        RRT_TRACE_CASE(1, 4)
        RRT_TRACE_CASE(2, 1)
        RRT_TRACE_CASE(2, 2)
        RRT_TRACE_CASE(2, 4)
        RRT_TRACE_CASE(4, 1)
        RRT_TRACE_CASE(4, 2)
        RRT_TRACE_CASE(4, 4)
#undef RRT_TRACE_CASE
    }
}
template <typename real>
size_t boost_lds(int K, int G)
{
    return sizeof(double) * 4 * (size_t)G + sizeof(real) * ((G + 2) * (size_t)((K + 2) | 1) + G);
}
template <typename real>
size_t unboost_lds(int K, int G)
{
    return sizeof(double) * 4 * (size_t)G + sizeof(real) * (G + 2) * (size_t)((K + 2) | 1);
}
template <typename real>
void launch_remap_plan(const PlanArgs<real> &a, hipStream_t st)
{
    const long n = a.P * a.K;
    const unsigned nb = (unsigned)std::min<long>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(k_remap_plan<real>, dim3(nb), dim3(256), 0, st, a);
}
template <typename real>
void launch_chilab(const ChiLabArgs<real> &a, hipStream_t st)
{
    const long n = a.P * (a.chi_grey ? 1 : a.fi.G);
    const unsigned nb = (unsigned)std::min<long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_chilab<real>, dim3(nb, a.K), dim3(256), 4 * sizeof(double) * a.fi.G, st, a);
}
template <typename real>
void launch_boost(const BoostArgs<real> &a, hipStream_t st)
{
    // two points per workgroup where a point's groups fill 64 bytes and both tables fit
    const size_t one = boost_lds<real>(a.K, a.fi.G),
                 two = one + sizeof(real) * ((a.fi.G + 2) * (size_t)((a.K + 2) | 1) + a.fi.G);
    if (a.fi.G * sizeof(real) == 64 && two <= 160 * 1024) {
        const long items = (a.P + 1) / 2;
        const unsigned nb = (unsigned)(8 * ((items + 7) / 8));
        hipLaunchKernelGGL((k_boost<real, 2>), dim3(nb), dim3(kRemapThreads), two, st, a);
        return;
    }
    const unsigned nb = (unsigned)(8 * ((a.P + 7) / 8));
    hipLaunchKernelGGL((k_boost<real, 1>), dim3(nb), dim3(kRemapThreads), one, st, a);
}
template <typename real>
void launch_unboost(const UnboostArgs<real> &a, hipStream_t st)
{
    // two points per workgroup where a point's groups fill 64 bytes and both tables fit
    const size_t one = unboost_lds<real>(a.K, a.fi.G), two = one + sizeof(real) * (a.fi.G + 2) * (size_t)((a.K + 2) | 1);
    if (a.fi.G * sizeof(real) == 64 && two <= 160 * 1024) {
        const long items = (a.P + 1) / 2;
        const unsigned nb = (unsigned)(8 * ((items + 7) / 8));
        hipLaunchKernelGGL((k_unboost<real, 2>), dim3(nb), dim3(kRemapThreads), two, st, a);
        return;
    }
    const unsigned nb = (unsigned)(8 * ((a.P + 7) / 8));
    hipLaunchKernelGGL((k_unboost<real, 1>), dim3(nb), dim3(kRemapThreads), one, st, a);
}
size_t do2sh_lds(int NL) { return sizeof(float) * 64 * (size_t)(((NL + 15) / 16) * 16 + 4); }

// FP32 product with a short inner dimension (Kd <= 64, the S2 product of L <= 7):
// the whole table B [Kd][N] (N = 128, 256 or 512) resident in LDS in one
// persistent workgroup of 16 waves per CU.  Wave w computes 16 rows of a block
// and 16 NT columns of group w % CQ (CQ = N / 16 NT); each 16 x 16 tile is
// computed transposed (operands swapped) so that a lane holds four
// consecutive columns of one row and stores them as one 16-byte vector; the
// next block's A rows are loaded during the current products.  KT > 0: Kd = 16 KT,
// so every row piece is a whole 16-byte vector and the loads take no branches.
template <int NT, int KT>
__global__ void __launch_bounds__(1024) k_gemm_short_k(long R, int Kd, int N, const float *__restrict__ A,
                                                       const float *__restrict__ B, float *__restrict__ C)
{
    constexpr int KR = 64, NC = 16 * NT;
    extern __shared__ unsigned char smem_raw[];
    float *Bs = reinterpret_cast<float *>(smem_raw);                   // [KR][N + 4]
    const int NP = N + 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lr = lane & 15, lg = lane >> 4;
    for (int i = threadIdx.x; i < KR * N; i += blockDim.x) {
        const int kk = i / N, c = i - kk * N;
        Bs[kk * NP + c] = kk < Kd ? B[(long)kk * N + c] : 0.f;
    }
    __syncthreads();
    const int CQ = N / NC, RW = 16 / CQ, rq = wave / CQ, cq = wave - rq * CQ;
    const long nblk = (R + 16 * RW - 1) / (16 * RW);
    constexpr int TT = KT > 0 ? KT : 4;                 // 16-wide k tiles
    f32x4 a[TT], an[TT];
    auto load = [&](f32x4 (&dst)[TT], long blk) {
        const float *Ar = A + min(blk * (16 * RW) + rq * 16 + lr, R - 1) * (long)Kd;
        if constexpr (KT > 0) {
#pragma unroll
            for (int t = 0; t < TT; ++t) dst[t] = *reinterpret_cast<const f32x4 *>(Ar + 16 * t + 4 * lg);
        } else {
#pragma unroll
            for (int t = 0; t < TT; ++t) {
                const int k = 16 * t + 4 * lg;
#pragma unroll
                for (int i = 0; i < 4; ++i) dst[t][i] = (k + i < Kd) ? Ar[k + i] : 0.f;
            }
        }
    };
    long blk = blockIdx.x;
    if (blk < nblk) load(a, blk);
    __builtin_amdgcn_s_waitcnt(0xF70);                  // vmcnt(0): the loop starts with no load in flight
    for (; blk < nblk; blk += gridDim.x) {
        // the next block's rows (past the last block: the last block again, not used)
        load(an, min(blk + (long)gridDim.x, nblk - 1));
        __builtin_amdgcn_sched_barrier(0);
        f32x4 acc[NT];
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < TT; ++t) {
            if (KT == 0 && 16 * t >= Kd) break;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const float *brow = Bs + (16 * t + 4 * lg + s) * NP + cq * NC + lr;
#pragma unroll
                for (int c = 0; c < NT; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(brow[16 * c], a[t][s], acc[c], 0, 0, 0);
            }
        }
        // take the next block's rows before this block's stores go out: the wait covers
        // those rows and the stores of the block before, both issued a block of products
        // earlier, and none of this block's stores
        __builtin_amdgcn_s_waitcnt(0xF70);              // vmcnt(0)
#pragma unroll
        for (int t = 0; t < TT; ++t) a[t] = an[t];
        __builtin_amdgcn_sched_barrier(0);
        const long r = blk * (16 * RW) + rq * 16 + lr;
        if (r < R) {
#pragma unroll
            for (int c = 0; c < NT; ++c)
                *reinterpret_cast<f32x4 *>(C + r * N + cq * NC + 16 * c + 4 * lg) = acc[c];
        }
    }
}

// FP32 C[R][N] = A[R][Kd] B[Kd][N] with B given transposed (Bt[N][Kd], k contiguous)
// and Kd a multiple of 16 KS: a wave owns 16 rows and the NT column tiles of the
// workgroup's block (grid.y); B moves from global memory straight into LDS
// (global_load_lds, 16 bytes = four k of one column per lane) in double-buffered
// chunks of 16 KS k, one 1 KB block per 16 k and column tile with column r at 64 r
// bytes and its k 4 s .. 4 s + 3 in slot s ^ ((r >> 2) & 3), so that one 16-byte read
// gives a lane the B values of four matrix-core steps.  One 16-row tile per wave
// keeps the accumulators at 4 NT registers, and four waves fit a SIMD.  TR: the
// tiles computed transposed (a lane holds four consecutive columns of one row; N a
// multiple of 4).
template <int NT, int W, int KS, bool TR>
__global__ void __launch_bounds__(64 * W) k_gemm_dma(long R, int Kd, int N, const float *__restrict__ A,
                                                   const float *__restrict__ Bt, float *__restrict__ C)
{
    constexpr int NC = 16 * NT, KC = 16 * KS, NBK = NT * KS, BPW = (NBK + W - 1) / W;
    extern __shared__ unsigned char smem_raw[];
    float *buf = reinterpret_cast<float *>(smem_raw);                // [2][KS][NT][256]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lr = lane & 15, lg = lane >> 4;
    const long r0 = (long)xcd_item(gridDim.x) * (16 * W) + wave * 16;
    const int c0 = blockIdx.y * NC;
    const float *__restrict__ Arow = A + min(r0 + lr, R - 1) * (long)Kd + 4 * lg;
    const int dc = lane >> 2, ds = (lane & 3) ^ ((dc >> 2) & 3);
    auto dma = [&](int kc, int b) {
#pragma unroll
        for (int u = 0; u < BPW; ++u) {
            const int blk = wave * BPW + u, sub = blk / NT, c = blk - sub * NT;
            if (blk < NBK) {
                const int col = min(c0 + 16 * c + dc, N - 1);
                __builtin_amdgcn_global_load_lds((const void *)(Bt + (long)col * Kd + kc + 16 * sub + 4 * ds),
                                                 (__attribute__((address_space(3))) void *)(buf + (b * NBK + blk) * 256),
                                                 16, 0, 0);
            }
        }
    };
    const int ro = lr * 16 + 4 * (lg ^ ((lr >> 2) & 3));
    f32x4 acc[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nch = Kd / KC;
    dma(0, 0);
    f32x4 an[KS];
#pragma unroll
    for (int u = 0; u < KS; ++u) an[u] = *reinterpret_cast<const f32x4 *>(Arow + 16 * u);
    for (int ci = 0; ci < nch; ++ci) {
        f32x4 a[KS];
#pragma unroll
        for (int u = 0; u < KS; ++u) a[u] = an[u];
        __builtin_amdgcn_s_waitcnt(0);                  // this wave's pieces of the chunk and its A values have landed
        __syncthreads();                                // every wave's: the chunk is whole, the other buffer free
        if (ci + 1 < nch) {
            dma(KC * (ci + 1), (ci + 1) & 1);
#pragma unroll
            for (int u = 0; u < KS; ++u) an[u] = *reinterpret_cast<const f32x4 *>(Arow + KC * (ci + 1) + 16 * u);
        }
        const float *Tb = buf + (ci & 1) * NBK * 256;
#pragma unroll
        for (int u = 0; u < KS; ++u)
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                const f32x4 b = *reinterpret_cast<const f32x4 *>(Tb + (u * NT + c) * 256 + ro);
#pragma unroll
                for (int s2 = 0; s2 < 4; ++s2)
                    acc[c] = TR ? __builtin_amdgcn_mfma_f32_16x16x4f32(b[s2], a[u][s2], acc[c], 0, 0, 0)
                                : __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][s2], b[s2], acc[c], 0, 0, 0);
            }
    }
    if (TR) {
        const long r = r0 + lr;
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            const int col = c0 + 16 * c + 4 * lg;
            if (r < R && col < N) *reinterpret_cast<f32x4 *>(C + r * N + col) = acc[c];
        }
        return;
    }
#pragma unroll
    for (int c = 0; c < NT; ++c) {
        const int col = c0 + 16 * c + lr;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const long r = r0 + 4 * lg + i;
            if (r < R && col < N) C[r * N + col] = acc[c][i];
        }
    }
}
bool launch_gemm_dma(long R, int Kd, int N, const float *A, const float *Bt, float *C, hipStream_t st)
{
    if (!Bt || Kd % 16 || N < 16) return false;
    constexpr int NT = 16;
    const unsigned nby = (unsigned)((N + 16 * NT - 1) / (16 * NT));
    const size_t sm = 2 * sizeof(float) * NT * 256;
    // (measured on MI355X at 2^23 rows: transposed tiles, 512 columns of 256 k, fastest with
    // eight waves; 256 columns of 512 k with sixteen, each chunk of B then serving 256 rows)
    if (N % 4 == 0 && N > Kd) {
        constexpr int W = 8;
        const long nb = (R + 16 * W - 1) / (16 * W);
        if (nb > 0x7fffffffL) return false;
        hipLaunchKernelGGL((k_gemm_dma<NT, W, 1, true>), dim3((unsigned)(8 * ((nb + 7) / 8)), nby), dim3(64 * W), sm,
                           st, R, Kd, N, A, Bt, C);
    } else {
        constexpr int W = 16;
        const long nb = (R + 16 * W - 1) / (16 * W);
        if (nb > 0x7fffffffL) return false;
        hipLaunchKernelGGL((k_gemm_dma<NT, W, 1, false>), dim3((unsigned)(8 * ((nb + 7) / 8)), nby), dim3(64 * W), sm,
                           st, R, Kd, N, A, Bt, C);
    }
    return true;
}

template <typename real>
void launch_gemm(long R, int Kd, int N, const real *A, const real *B, real *C, hipStream_t st)
{
    // columns per workgroup: all of them up to 512 (FP32) / 256 (FP64), so A is read once;
    // B staged through two LDS chunks, as 4-element vectors where the rows allow
#define RRT_GEMM(NT, RT, W, KC)                                                                              \
    {                                                                                                        \
        const long nb = (R + 16 * W * RT - 1) / (16 * W * RT);                                               \
        const unsigned nby = (unsigned)((N + 16 * NT - 1) / (16 * NT));                                       \
        const size_t sm = 2 * sizeof(real) * (size_t)KC * (16 * NT + (sizeof(real) == 4 ? 4 : 2));            \
        const dim3 grid((unsigned)(8 * ((nb + 7) / 8)), nby);                                                \
        if (N % 4 == 0 && sizeof(real) == 4 && N > Kd)                                                       \
            hipLaunchKernelGGL((k_gemm_panel<real, NT, RT, W, KC, 4, true>), grid, dim3(64 * W), sm, st, R, Kd, N, A, \
                               B, C);                                                                        \
        else if (N % 4 == 0)                                                                                 \
            hipLaunchKernelGGL((k_gemm_panel<real, NT, RT, W, KC, 4, false>), grid, dim3(64 * W), sm, st, R, Kd, N, \
                               A, B, C);                                                                     \
        else                                                                                                 \
            hipLaunchKernelGGL((k_gemm_panel<real, NT, RT, W, KC, 1, false>), grid, dim3(64 * W), sm, st, R, Kd, N, A, \
                               B, C);                                                                        \
        return;                                                                                              \
    }
    // (tile shapes: the fastest of a sweep on MI355X at 2^23 rows: 78 % of the FP32
    // matrix peak with 256 columns and 512 inner, 71 % with 512 columns and 256 inner)
    if constexpr (sizeof(real) == 4) {
        if (Kd <= 64 && (N == 128 || N == 256 || N == 512)) {
            const size_t smr = sizeof(float) * 64 * (size_t)(N + 4);
            const long nblk = (R + 16 * (16 / (N / 128)) - 1) / (16 * (16 / (N / 128)));
            const dim3 grid((unsigned)std::min<long>(nblk, 256));
            if (Kd == 64)
                hipLaunchKernelGGL((k_gemm_short_k<8, 4>), grid, dim3(1024), smr, st, R, Kd, N, A, B, C);
            else if (Kd == 16)
                hipLaunchKernelGGL((k_gemm_short_k<8, 1>), grid, dim3(1024), smr, st, R, Kd, N, A, B, C);
            else
                hipLaunchKernelGGL((k_gemm_short_k<8, 0>), grid, dim3(1024), smr, st, R, Kd, N, A, B, C);
            return;
        }
        if (N <= 32) RRT_GEMM(2, 4, 4, 16)
        if (N <= 128) RRT_GEMM(8, 2, 4, 16)
        if (N <= 256) RRT_GEMM(16, 2, 8, 16)
        RRT_GEMM(16, 2, 4, 16)
    } else {
        if (N <= 32) RRT_GEMM(2, 2, 4, 16)
        if (N <= 128) RRT_GEMM(8, 1, 4, 16)
        RRT_GEMM(16, 1, 4, 16)
    }
#undef RRT_GEMM
}

bool launch_do2sh_f32(long R, int K, int NL, const float *A, const float *B, float *C, hipStream_t st, int rt)
{
    const size_t sm = do2sh_lds(NL);
    // NL up to 64 (L <= 7); at L = 15 the library product is faster (measured on MI355X)
    // W waves share each staged table chunk (sixteen where the registers allow)
#define RRT_DO2SH32(NT, RT, W)                                                                                \
    {                                                                                                         \
        const long nb = (R + 16 * W * RT - 1) / (16 * W * RT);                                                \
        if (nb > 0x7fffffffL) return false;                                                                  \
        hipLaunchKernelGGL((k_do2sh_f32<NT, RT, W>), dim3((unsigned)(8 * ((nb + 7) / 8))), dim3(64 * W), sm, st, R, \
                           K, NL, A, B, C);                                                                  \
        return true;                                                                                          \
    }
    // rt 1 and 2 with the whole table resident in LDS where it fits: one persistent
    // workgroup per CU
#define RRT_DO2SH32R(NT, RT)                                                                                  \
    {                                                                                                         \
        const size_t smr = sizeof(float) * (size_t)((K + 63) / 64 * 64) * (NT * 16 + 4);                     \
        if (smr <= 160 * 1024) {                                                                              \
            const long nb = (R + 256 * RT - 1) / (256 * RT);                                                  \
            if (K % 64 == 0)                                                                                  \
                hipLaunchKernelGGL((k_do2sh_f32r<NT, RT, true>), dim3((unsigned)std::min<long>(nb, 256)), dim3(1024), \
                                   smr, st, R, K, NL, A, B, C);                                              \
            else                                                                                              \
                hipLaunchKernelGGL((k_do2sh_f32r<NT, RT, false>), dim3((unsigned)std::min<long>(nb, 256)), dim3(1024), \
                                   smr, st, R, K, NL, A, B, C);                                              \
            return true;                                                                                      \
        }                                                                                                     \
    }
    // (the defaults: resident, one row tile per wave for NL <= 16 and two up to 64, the
    // fastest measured on MI355X at L = 3 and 7)
    if (NL <= 16) {
        if (rt == 0 || rt == 1) RRT_DO2SH32R(1, 1)
        if (rt == 2) RRT_DO2SH32R(1, 2)
        if (rt == 1) RRT_DO2SH32(1, 1, 16)
        if (rt == 2) RRT_DO2SH32(1, 2, 16)
        if (rt == 0 || rt == 4) RRT_DO2SH32(1, 4, 16)
    } else if (NL <= 64) {
        if (rt == 1) RRT_DO2SH32R(4, 1)
        if (rt == 0 || rt == 2) RRT_DO2SH32R(4, 2)
        if (rt == 1) RRT_DO2SH32(4, 1, 16)
        if (rt == 0 || rt == 2) RRT_DO2SH32(4, 2, 16)
        if (rt == 4) RRT_DO2SH32(4, 4, 4)
    }
#undef RRT_DO2SH32R
#undef RRT_DO2SH32
    return false;
}

bool launch_do2sh_f16(long R, int K, int NL, const float *A, const _Float16 *WYh, const _Float16 *WYl, float *C,
                      hipStream_t st, int rt)
{
    const int Kp = (K + 31) / 32 * 32;
    // W waves share each staged table chunk (sixteen where the registers allow)
#define RRT_DO2SH16(NT, RT, W)                                                                               \
    {                                                                                                        \
        const long nb = (R + 16 * W * RT - 1) / (16 * W * RT);                                               \
        if (nb > 0x7fffffffL) return false;                                                                 \
        const size_t sm = 2 * sizeof(_Float16) * (size_t)(NT * 16) * 72;                                    \
        hipLaunchKernelGGL((k_do2sh_f16<NT, RT, W>), dim3((unsigned)(8 * ((nb + 7) / 8))), dim3(64 * W), sm, st, R, \
                           K, Kp, NL, A, WYh, WYl, C);                                                      \
        return true;                                                                                         \
    }
    if (NL <= 16) {
        if (rt == 1) RRT_DO2SH16(1, 1, 16)
        if (rt == 2) RRT_DO2SH16(1, 2, 16)
        if (rt == 0 || rt == 4) RRT_DO2SH16(1, 4, 16)
    } else if (NL <= 64) {
        if (rt == 1) RRT_DO2SH16(4, 1, 16)
        if (rt == 0 || rt == 2) RRT_DO2SH16(4, 2, 16)
        if (rt == 4) RRT_DO2SH16(4, 4, 4)
    } else if (NL <= 256) {
        // eight waves share each staged table chunk
        if (rt == 0 || rt == 1) {
            const long nb = (R + 127) / 128;
            if (nb > 0x7fffffffL) return false;
            const size_t sm = 2 * sizeof(_Float16) * 2 * 16 * 512;          // two chunks of 32 1 KB blocks
            hipLaunchKernelGGL((k_do2sh_f16_dma<16, 8>), dim3((unsigned)(8 * ((nb + 7) / 8))), dim3(512), sm, st, R,
                               K, Kp, NL, A, WYh, WYl, C);
            return true;
        }
    }
#undef RRT_DO2SH16
    return false;
}

bool launch_sh2do_f16(long R, int K, int NL, const float *S, const _Float16 *Yh, const _Float16 *Yl, float *C,
                      hipStream_t st)
{
    const long nb = (R + 63) / 64;
    if (nb > 0x7fffffffL) return false;
    const dim3 grid((unsigned)(8 * ((nb + 7) / 8))), block(256);
    auto sm = [](int NB) { return 2 * sizeof(_Float16) * 64 * (size_t)(NB * 32 + 8); };
    // sixteen waves (256 rows) share each staged table chunk where the rows are short
    const long nb16 = (R + 255) / 256;
    const dim3 grid16((unsigned)(8 * ((nb16 + 7) / 8))), block16(1024);
    if (NL <= 32) hipLaunchKernelGGL((k_sh2do_f16<1, 16>), grid16, block16, sm(1), st, R, K, NL, S, Yh, Yl, C);
    else if (NL <= 64) hipLaunchKernelGGL((k_sh2do_f16<2, 16>), grid16, block16, sm(2), st, R, K, NL, S, Yh, Yl, C);
    else if (NL <= 128) hipLaunchKernelGGL(k_sh2do_f16<4>, grid, block, sm(4), st, R, K, NL, S, Yh, Yl, C);
    else if (NL <= 256) {
        // eight waves share each staged table chunk
        const long nb8 = (R + 127) / 128;
        if (nb8 > 0x7fffffffL) return false;
        hipLaunchKernelGGL((k_sh2do_f16_dma<8, 8>), dim3((unsigned)(8 * ((nb8 + 7) / 8))), dim3(512),
                           2 * sizeof(_Float16) * 32 * 512, st, R, K, NL, S, Yh, Yl, C);
    }
    else return false;
    return true;
}

// the Compton source on the matrix cores: FP32, G <= 32, L <= 15, NL a multiple of 4
template <typename real>
bool compton_mfma_ok(const SourceArgs<real> &a)
{
    int lmax = 0;
    while ((lmax + 1) * (lmax + 1) < a.NL) ++lmax;
    return sizeof(real) == 4 && a.compton && a.G <= 32 && lmax <= 15 && a.NL % 4 == 0;
}
template <typename real>
void launch_compton_mfma(const SourceArgs<real> &a, const real *Sold, double *rows, hipStream_t st)
{
    int lmax = 0;
    while ((lmax + 1) * (lmax + 1) < a.NL) ++lmax;
    const unsigned nb = (unsigned)std::min<long>(a.P, 2048);
    const SourceArgs<float> &af = *reinterpret_cast<const SourceArgs<float> *>(&a);
    const float *so = reinterpret_cast<const float *>(Sold);
    const size_t sm = sizeof(float) * (32 * 256 + 2 * (size_t)a.G + (rows ? 4 + (size_t)a.G * a.NL : 0));
    const dim3 b(kComptonMfmaThreads);
    if (a.tnode) {
        if (rows) hipLaunchKernelGGL((k_source_compton_mfma<true, true>), dim3(nb), b, sm, st, af, lmax, so, rows);
        else hipLaunchKernelGGL((k_source_compton_mfma<true, false>), dim3(nb), b, sm, st, af, lmax, so, rows);
    } else {
        if (rows) hipLaunchKernelGGL((k_source_compton_mfma<false, true>), dim3(nb), b, sm, st, af, lmax, so, rows);
        else hipLaunchKernelGGL((k_source_compton_mfma<false, false>), dim3(nb), b, sm, st, af, lmax, so, rows);
    }
}

template <typename real>
void launch_source(const SourceArgs<real> &a, hipStream_t st)
{
    if (a.compton) {
        int lmax = 0;
        while ((lmax + 1) * (lmax + 1) < a.NL) ++lmax;
        if (compton_mfma_ok(a)) {
            launch_compton_mfma<real>(a, nullptr, nullptr, st);
            return;
        }
        const unsigned nb = (unsigned)(8 * ((a.P + 7) / 8));
        hipLaunchKernelGGL(k_source_compton<real>, dim3(nb), dim3(256), sizeof(real) * (size_t)a.G * a.NL, st, a);
    } else {
        hipLaunchKernelGGL(k_source<real>, dim3(blocks_for(a.P * a.G * a.NL, 256)), dim3(256), 0, st, a);
    }
}
template <typename real>
void launch_chi0(long P, int G, const real *kappa, const real *sigma, const real *sg, const int *tnode, const real *twt,
                 real *chi0, hipStream_t st)
{
    hipLaunchKernelGGL(k_chi0<real>, dim3(blocks_for(P * G, 256)), dim3(256), 0, st, P, G, kappa, sigma, sg, tnode,
                       twt, chi0);
}
template <typename real>
void launch_moments_lab(long P, int G, int K, const double *dir, const real *I, double *J, double *H, double *Kt, hipStream_t st)
{
    hipLaunchKernelGGL(k_moments_lab<real>, dim3(blocks_for(P * G, 256)), dim3(256), 0, st, P, G, K, dir, I, J, H, Kt);
}
// Frequency-integrated moments per point (FP64): X_tot = sum_g dnu_g X_g over the
// per-group J [P][G], H [P][G][3], K [P][G][6], and the Eddington tensor
// f = K_tot / J_tot (0 where J_tot = 0); out [P][16] = J, H (3), K (6), f (6)
__global__ void __launch_bounds__(256) k_moments_integrate(long P, int G, const double *__restrict__ dnu,
                                                           const double *__restrict__ J, const double *__restrict__ H,
                                                           const double *__restrict__ Kt, double *__restrict__ out)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    double j = 0.0, h[3] = {0.0, 0.0, 0.0}, k[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int g = 0; g < G; ++g) {
        const double w = dnu[g];
        const long o = p * G + g;
        j += w * J[o];
        for (int c = 0; c < 3; ++c) h[c] += w * H[3 * o + c];
        for (int c = 0; c < 6; ++c) k[c] += w * Kt[6 * o + c];
    }
    double *r = out + 16 * p;
    r[0] = j;
    for (int c = 0; c < 3; ++c) r[1 + c] = h[c];
    for (int c = 0; c < 6; ++c) r[4 + c] = k[c];
    for (int c = 0; c < 6; ++c) r[10 + c] = j != 0.0 ? k[c] / j : 0.0;
}

void launch_moments_integrate(long P, int G, const double *dnu, const double *J, const double *H, const double *Kt,
                              double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_moments_integrate, dim3(blocks_for(P, 256)), dim3(256), 0, st, P, G, dnu, J, H, Kt, out);
}

template <typename real>
void launch_moments_co(long PG, int NL, int lmax, const real *Ilm, double *J, double *H, double *Kt, hipStream_t st)
{
    hipLaunchKernelGGL(k_moments_co<real>, dim3(blocks_for(PG, 256)), dim3(256), 0, st, PG, NL, lmax, Ilm, J, H, Kt);
}
template <typename real>
bool launch_source_resid(const SourceArgs<real> &a, const real *Sold, double *rows, hipStream_t st)
{
    if (a.compton) {
        // the matrix-core Compton source with the row sums where a row is a power-of-two lane group
        const int nl4 = a.NL / 4;
        if (!compton_mfma_ok(a) || 64 % nl4 != 0) return false;
        launch_compton_mfma(a, Sold, rows, st);
        return true;
    }
    if (a.NL % 4 == 0 && a.NL <= 256 && 256 % a.NL == 0) {
        const int rw = 256 / a.NL;                       // rows per wave
        const long waves = (a.P * a.G + rw - 1) / rw;
        const unsigned nb = (unsigned)std::min<long>((waves + 3) / 4, 16384);
        hipLaunchKernelGGL(k_source_resid4<real>, dim3(nb), dim3(256), 0, st, a, Sold, rows);
        return true;
    }
    if (a.NL > 64 || 64 % a.NL != 0) return false;
    const long waves = (a.P * a.G + 64 / a.NL - 1) / (64 / a.NL);
    const unsigned nb = (unsigned)std::min<long>((waves + 3) / 4, 16384);
    hipLaunchKernelGGL(k_source_resid<real>, dim3(nb), dim3(256), 0, st, a, Sold, rows);
    return true;
}
template <typename real>
void launch_resid_groups(long P, int G, const double *rows, double *out, hipStream_t st)
{
    launch_group_totals(P, G, rows, out, st);
}
template <typename real>
void launch_resid(long P, int G, int NL, const real *a, const real *b, double *rows, int nblk, double *out, hipStream_t st)
{
    (void)nblk;
    const unsigned nb = (unsigned)std::min<long>((P * G + 3) / 4, 8192);   // 4 waves per block, one row each
    hipLaunchKernelGGL(k_resid_rows<real>, dim3(nb), dim3(256), 0, st, P, G, NL, a, b, rows);
    launch_group_totals(P, G, rows, out, st);
}
template <typename real>
void launch_ng_dots(long n, int G, int NL, const double *red, double floor2, const real *s0, const real *s1,
                    const real *s2, const real *s3, double *partial, int nblk, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_ng_partial<real>, dim3(nblk), dim3(256), sizeof(double) * G, st, n, G, NL, red, floor2, s0,
                       s1, s2, s3, partial);
    hipLaunchKernelGGL(k_sum_columns, dim3(5), dim3(256), 0, st, nblk, 5, partial, out);
}
template <typename real>
void launch_ng_extrapolate(long n, const double *dots, const real *s3, const real *s2, const real *s1, real *out,
                           hipStream_t st)
{
    hipLaunchKernelGGL(k_ng_extrapolate<real>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, dots, s3, s2, s1, out);
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

// ---------------------------------------------------------------------------
// Variable-Eddington-tensor hand-off: the frequency-integrated moment equations
// dJ/dt + div H = kappa_E (B - J), dH/dt + div(f J) = -chi_F H closed with the
// transport's Eddington tensor f, advanced by the forward-backward scheme (H
// from J^n, then J from H^{n+1}; the local terms implicit).  Central
// differences, periodic in x and y, one-sided on the z faces; one thread per
// point, neighbours through the caches (each array is streamed once per step).
// ---------------------------------------------------------------------------
struct VetNbr {
    long xp, xm, yp, ym, zp, zm;
    double sz;      // 1/(2 dz) inside, 1/dz on a z face, 0 with one z plane
};
__device__ __forceinline__ VetNbr vet_nbr(const VetArgs &a, long p)
{
    const long PL = (long)a.nx * a.ny;
    const int z = (int)(p / PL);
    const long r = p - (long)z * PL;
    const int y = (int)(r / a.nx), x = (int)(r - (long)y * a.nx);
    VetNbr n;
    n.xp = p + (x + 1 == a.nx ? 1 - a.nx : 1);
    n.xm = p + (x == 0 ? a.nx - 1 : -1);
    n.yp = p + (y + 1 == a.ny ? (long)(1 - a.ny) * a.nx : a.nx);
    n.ym = p + (y == 0 ? (long)(a.ny - 1) * a.nx : -a.nx);
    if (a.nz == 1) {
        n.zp = n.zm = p;
        n.sz = 0.0;
    } else if (z == 0) {
        n.zp = p + PL; n.zm = p; n.sz = a.idz;
    } else if (z == a.nz - 1) {
        n.zp = p; n.zm = p - PL; n.sz = a.idz;
    } else {
        n.zp = p + PL; n.zm = p - PL; n.sz = a.idz2;
    }
    return n;
}

// H^{n+1} and the momentum exchange; f in SoA order [6][P] (xx, yy, zz, xy, xz, yz)
__global__ void __launch_bounds__(256) k_vet_flux(VetArgs a)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.P) return;
    const VetNbr n = vet_nbr(a, p);
    const double *f = a.f;
    const long P = a.P;
    auto fJ = [&](int c, long q) { return f[c * P + q] * a.J[q]; };
    // column of f_ab for row a: (x, y, z) derivative directions
    const int col[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    const double dt = a.dt, den = 1.0 + dt * a.chi[p];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const double div = (fJ(col[r][0], n.xp) - fJ(col[r][0], n.xm)) * a.idx2 +
                           (fJ(col[r][1], n.yp) - fJ(col[r][1], n.ym)) * a.idy2 +
                           (fJ(col[r][2], n.zp) - fJ(col[r][2], n.zm)) * n.sz;
        const double h = (a.H[3 * p + r] - dt * div) / den;
        a.H[3 * p + r] = h;
        a.G[4 * p + 1 + r] += dt * a.chi[p] * h;
    }
}

// J^{n+1} from H^{n+1} and the energy exchange
__global__ void __launch_bounds__(256) k_vet_energy(VetArgs a)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.P) return;
    const VetNbr n = vet_nbr(a, p);
    const double *H = a.H;
    const double divH = (H[3 * n.xp] - H[3 * n.xm]) * a.idx2 + (H[3 * n.yp + 1] - H[3 * n.ym + 1]) * a.idy2 +
                        (H[3 * n.zp + 2] - H[3 * n.zm + 2]) * n.sz;
    const double dt = a.dt, k = a.kap[p], b = a.B[p];
    const double j = (a.J[p] - dt * divH + dt * k * b) / (1.0 + dt * k);
    a.J[p] = j;
    a.G[4 * p] += dt * k * (j - b);
}

// f of the integrated moments ([P][16], columns 10..15) into SoA [6][P]
__global__ void __launch_bounds__(256) k_vet_f(long P, const double *__restrict__ mom, double *__restrict__ f)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
#pragma unroll
    for (int c = 0; c < 6; ++c) f[c * P + p] = mom[16 * p + 10 + c];
}

void launch_vet_f(long P, const double *mom, double *f, hipStream_t st)
{
    hipLaunchKernelGGL(k_vet_f, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, P, mom, f);
}
void launch_vet_flux(const VetArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_vet_flux, dim3((unsigned)((a.P + 255) / 256)), dim3(256), 0, st, a);
}
void launch_vet_energy(const VetArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_vet_energy, dim3((unsigned)((a.P + 255) / 256)), dim3(256), 0, st, a);
}

// number of elements of x[n] that are not finite, or (check_lo) below lo, added to *count
template <typename real>
__global__ void __launch_bounds__(256) k_count_bad(long n, const real *__restrict__ x, real lo, int check_lo,
                                                   unsigned long long *count)
{
    unsigned c = 0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const real v = x[i];
        c += (!isfinite(v) || (check_lo && v < lo)) ? 1u : 0u;
    }
    if (c) atomicAdd(count, (unsigned long long)c);
}
template <typename real>
void launch_count_bad(long n, const real *x, real lo, int check_lo, unsigned long long *count, hipStream_t st)
{
    const unsigned nb = (unsigned)std::max<long>(1, std::min<long>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_count_bad<real>, dim3(nb), dim3(256), 0, st, n, x, lo, check_lo, count);
}

hipError_t set_lds_limits(size_t bytes)
{
    const void *fns[] = {reinterpret_cast<const void *>(&k_trace<float, kChiGrey, 1, 1, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGrey, 1, 1, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGrey, 1, 2, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGrey, 1, 2, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGrey, 1, 4, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGrey, 1, 4, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGrey, 2, 1, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGrey, 2, 1, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGrey, 2, 2, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGrey, 2, 2, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGrey, 2, 4, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGrey, 2, 4, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGrey, 4, 1, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGrey, 4, 1, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGrey, 4, 2, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGrey, 4, 2, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGrey, 4, 4, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGrey, 4, 4, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGroup, 1, 1, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGroup, 1, 1, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGroup, 1, 2, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGroup, 1, 2, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGroup, 1, 4, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGroup, 1, 4, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGroup, 2, 1, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGroup, 2, 1, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGroup, 2, 2, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGroup, 2, 2, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGroup, 2, 4, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGroup, 2, 4, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGroup, 4, 1, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGroup, 4, 1, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGroup, 4, 2, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGroup, 4, 2, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGroup, 4, 4, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiGroup, 4, 4, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiArray, 1, 1, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiArray, 1, 1, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiArray, 1, 2, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiArray, 1, 2, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiArray, 1, 4, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiArray, 1, 4, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiArray, 2, 1, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiArray, 2, 1, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiArray, 2, 2, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiArray, 2, 2, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiArray, 2, 4, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiArray, 2, 4, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiArray, 4, 1, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiArray, 4, 1, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiArray, 4, 2, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiArray, 4, 2, false>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiArray, 4, 4, true>),
                         reinterpret_cast<const void *>(&k_trace<float, kChiArray, 4, 4, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGrey, 1, 1, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGrey, 1, 1, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGrey, 1, 2, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGrey, 1, 2, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGrey, 1, 4, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGrey, 1, 4, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGrey, 2, 1, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGrey, 2, 1, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGrey, 2, 2, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGrey, 2, 2, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGrey, 2, 4, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGrey, 2, 4, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGrey, 4, 1, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGrey, 4, 1, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGrey, 4, 2, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGrey, 4, 2, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGrey, 4, 4, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGrey, 4, 4, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGroup, 1, 1, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGroup, 1, 1, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGroup, 1, 2, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGroup, 1, 2, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGroup, 1, 4, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGroup, 1, 4, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGroup, 2, 1, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGroup, 2, 1, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGroup, 2, 2, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGroup, 2, 2, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGroup, 2, 4, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGroup, 2, 4, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGroup, 4, 1, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGroup, 4, 1, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGroup, 4, 2, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGroup, 4, 2, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGroup, 4, 4, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiGroup, 4, 4, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiArray, 1, 1, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiArray, 1, 1, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiArray, 1, 2, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiArray, 1, 2, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiArray, 1, 4, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiArray, 1, 4, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiArray, 2, 1, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiArray, 2, 1, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiArray, 2, 2, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiArray, 2, 2, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiArray, 2, 4, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiArray, 2, 4, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiArray, 4, 1, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiArray, 4, 1, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiArray, 4, 2, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiArray, 4, 2, false>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiArray, 4, 4, true>),
                         reinterpret_cast<const void *>(&k_trace<double, kChiArray, 4, 4, false>),
                         reinterpret_cast<const void *>(&k_boost<float, 1>),
                         reinterpret_cast<const void *>(&k_boost<float, 2>),
                         reinterpret_cast<const void *>(&k_boost<double, 1>),
                         reinterpret_cast<const void *>(&k_boost<double, 2>),
                         reinterpret_cast<const void *>(&k_unboost<float, 1>),
                         reinterpret_cast<const void *>(&k_unboost<float, 2>),
                         reinterpret_cast<const void *>(&k_unboost<double, 1>),
                         reinterpret_cast<const void *>(&k_unboost<double, 2>),
                         reinterpret_cast<const void *>(&k_source_compton<float>),
                         reinterpret_cast<const void *>(&k_do2sh_f16<1, 1, 16>),
                         reinterpret_cast<const void *>(&k_do2sh_f16<1, 2, 16>),
                         reinterpret_cast<const void *>(&k_do2sh_f16<1, 4, 16>),
                         reinterpret_cast<const void *>(&k_do2sh_f16<4, 1, 16>),
                         reinterpret_cast<const void *>(&k_do2sh_f16<4, 2, 16>),
                         reinterpret_cast<const void *>(&k_do2sh_f16<4, 4, 4>),
                         reinterpret_cast<const void *>(&k_sh2do_f16<1, 16>),
                         reinterpret_cast<const void *>(&k_sh2do_f16<2, 16>),
                         reinterpret_cast<const void *>(&k_sh2do_f16<4>),
                         reinterpret_cast<const void *>(&k_sh2do_f16_dma<8, 8>),
                         reinterpret_cast<const void *>(&k_do2sh_f16_dma<16, 8>),

                         reinterpret_cast<const void *>(&k_source_compton_mfma<false, false>),
                         reinterpret_cast<const void *>(&k_source_compton_mfma<true, false>),
                         reinterpret_cast<const void *>(&k_source_compton_mfma<false, true>),
                         reinterpret_cast<const void *>(&k_source_compton_mfma<true, true>),
                         reinterpret_cast<const void *>(&k_do2sh_f32<1, 1, 16>),
                         reinterpret_cast<const void *>(&k_do2sh_f32<1, 2, 16>),
                         reinterpret_cast<const void *>(&k_do2sh_f32<1, 4, 16>),
                         reinterpret_cast<const void *>(&k_do2sh_f32<4, 1, 16>),
                         reinterpret_cast<const void *>(&k_do2sh_f32<4, 2, 16>),
                         reinterpret_cast<const void *>(&k_do2sh_f32<4, 4, 4>),
                         reinterpret_cast<const void *>(&k_do2sh_f32r<1, 1, false>),
                         reinterpret_cast<const void *>(&k_do2sh_f32r<1, 1, true>),
                         reinterpret_cast<const void *>(&k_do2sh_f32r<1, 2, false>),
                         reinterpret_cast<const void *>(&k_do2sh_f32r<1, 2, true>),
                         reinterpret_cast<const void *>(&k_do2sh_f32r<4, 1, false>),
                         reinterpret_cast<const void *>(&k_do2sh_f32r<4, 1, true>),
                         reinterpret_cast<const void *>(&k_do2sh_f32r<4, 2, false>),
                         reinterpret_cast<const void *>(&k_do2sh_f32r<4, 2, true>),
                         reinterpret_cast<const void *>(&k_gemm_short_k<8, 0>),
                         reinterpret_cast<const void *>(&k_gemm_short_k<8, 1>),
                         reinterpret_cast<const void *>(&k_gemm_short_k<8, 4>),
                         reinterpret_cast<const void *>(&k_source_compton<double>)};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

#define RRT_INSTANTIATE(real)                                                                                  \
    template void launch_trace<real>(const TraceArgs<real> &, bool, hipStream_t);                              \
    template void launch_boost<real>(const BoostArgs<real> &, hipStream_t);                                     \
    template void launch_unboost<real>(const UnboostArgs<real> &, hipStream_t);                                 \
    template size_t trace_lds<real>(int, int, int, int);                                                       \
    template void launch_transpose_lab<real>(const real *, real *, long, int, int, bool, hipStream_t);          \
    template size_t boost_lds<real>(int, int);                                                                 \
    template size_t unboost_lds<real>(int, int);                                                               \
    template void launch_chilab<real>(const ChiLabArgs<real> &, hipStream_t);                                   \
    template void launch_remap_plan<real>(const PlanArgs<real> &, hipStream_t);                                   \
    template void launch_source<real>(const SourceArgs<real> &, hipStream_t);                                   \
    template void launch_gemm<real>(long, int, int, const real *, const real *, real *, hipStream_t);                                   \
    template bool launch_source_resid<real>(const SourceArgs<real> &, const real *, double *, hipStream_t);     \
    template void launch_resid_groups<real>(long, int, const double *, double *, hipStream_t);                  \
    template void launch_chi0<real>(long, int, const real *, const real *, const real *, const int *, const real *,   \
                                    real *, hipStream_t);  \
    template void launch_moments_lab<real>(long, int, int, const double *, const real *, double *, double *,    \
                                           double *, hipStream_t);                                              \
    template void launch_moments_co<real>(long, int, int, const real *, double *, double *, double *,           \
                                          hipStream_t);                                                         \
    template void launch_resid<real>(long, int, int, const real *, const real *, double *, int, double *,       \
                                     hipStream_t);                                                              \
    template void launch_ng_dots<real>(long, int, int, const double *, double, const real *, const real *,     \
                                       const real *, const real *, double *, int, double *, hipStream_t);       \
    template void launch_ng_extrapolate<real>(long, const double *, const real *, const real *, const real *,      \
                                              real *, hipStream_t);                                              \
    template void launch_combine3<real>(long, double, const real *, double, const real *, double, const real *, \
                                        real *, hipStream_t);                                                   \
    template void launch_rk_stage<real>(long, const real *, real *, real *, real *, int, int, real, hipStream_t); \
    template void launch_count_bad<real>(long, const real *, real, int, unsigned long long *, hipStream_t);

RRT_INSTANTIATE(float)
RRT_INSTANTIATE(double)

}  // namespace rrt
