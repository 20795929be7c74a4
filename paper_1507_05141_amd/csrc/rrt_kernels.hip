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

// reciprocal: the hardware v_rcp_f32 (1 ulp) in FP32, exact division in FP64
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }

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
    __device__ static float ex(float h) { return __expf(-h); }
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
        const real ih = fast_rcp(h);
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
    const real al = (real(1) + hr * fast_rcp(hl + hr)) * real(1.0 / 3.0);
    return dl * dr * fast_rcp(al * dr + (real(1) - al) * dl);
}

template <typename real>
__device__ __forceinline__ real clamp_between(real v, real a, real b)
{
    const real lo = fmin(a, b), hi = fmax(a, b);
    return fmin(fmax(v, lo), hi);
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

// taps as kept in LDS, weights in the working precision
template <typename real> struct TapL {
    int a0, a1, b0, b1;
    real wmu, wphi;
};

// value at the taps of a field F[k * sk + g * sg] (k = ordinate) held in LDS;
// pole[g] / pole[G + g] are the azimuthal means of the lowest / highest ring
template <typename real>
__device__ __forceinline__ real tap_value(const real *F, int sk, int sg, int G, int g, int nmu, int nphi,
                                          const TapL<real> &t, const real *pole)
{
    auto ring = [&](int a) -> real {
        if (a < 0) return pole[g];
        if (a >= nmu) return pole[G + g];
        return (real(1) - t.wphi) * F[(a * nphi + t.b0) * sk + g * sg] + t.wphi * F[(a * nphi + t.b1) * sk + g * sg];
    };
    return (real(1) - t.wmu) * ring(t.a0) + t.wmu * ring(t.a1);
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
// MAXPT grid points of the plane with all GC groups.  The source S~ and
// extinction chi~ of the four planes a step touches (second upwind, upwind,
// current, downwind) sit in an LDS ring, the previous intensity plane in LDS
// (overwritten by the new one once every thread has read it); the next plane
// is fetched into registers while the current one is computed.
// LDS planes carry a one-column and one-row periodic halo (row stride nx + 1)
// so that the bilinear taps need no wrap.  chi~ = chi_lab + 1/(c dt) with
// chi_lab precomputed per medium (one value per point when it is grey) or read
// from an array for the stand-alone entry point.  Lab arrays are [k][p][g].
// ---------------------------------------------------------------------------
template <typename real, bool CHI_ARRAY, int GC, int MAXPT>
struct PlaneRegs {
    real s[MAXPT][GC], x[MAXPT][GC];
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

// global -> registers: S~ and chi~ of plane t for this thread's points
template <typename real, bool CHI_ARRAY, int GC, int MAXPT>
__device__ __forceinline__ void trace_fetch(PlaneRegs<real, CHI_ARRAY, GC, MAXPT> &r, const real *__restrict__ Sk,
                                            const real *__restrict__ Xk, const real *__restrict__ Ck, int G, int PL,
                                            int m, real icdt, bool xg)
{
#pragma unroll
    for (int c = 0; c < MAXPT; ++c) {
        const int pe = threadIdx.x + c * kTraceThreads;
        if (pe < PL) {
            const int pidx = m * PL + pe;
            const int o = pidx * G;
#pragma unroll
            for (int gi = 0; gi < GC; ++gi) r.s[c][gi] = Sk[o + gi];
            if (CHI_ARRAY) {
#pragma unroll
                for (int gi = 0; gi < GC; ++gi) r.x[c][gi] = Xk[o + gi];
            } else if (xg) {
                r.x[c][0] = Ck[pidx] + icdt;
            } else {
#pragma unroll
                for (int gi = 0; gi < GC; ++gi) r.x[c][gi] = Xk[o + gi] + icdt;
            }
        }
    }
}

// write value v of point (i, j) into an LDS plane with its periodic halo
template <typename real>
__device__ __forceinline__ void lds_put(real *pl, const TraceIdx &q, int i, int j, int ge, int gi, real v)
{
    pl[(j * q.RS + i) * ge + gi] = v;
    if (i == 0) pl[(j * q.RS + q.nx) * ge + gi] = v;
    if (j == 0) {
        pl[(q.ny * q.RS + i) * ge + gi] = v;
        if (i == 0) pl[(q.ny * q.RS + q.nx) * ge + gi] = v;
    }
}

// registers -> the LDS ring slot of plane t
template <typename real, bool CHI_ARRAY, int GC, int MAXPT>
__device__ __forceinline__ void trace_store(const PlaneRegs<real, CHI_ARRAY, GC, MAXPT> &r, real *Sr, real *Xr,
                                            const TraceIdx &q, int t, bool xg)
{
    const int xge = xg ? 1 : GC;
    real *Sd = Sr + (t & 3) * q.PS * GC, *Xd = Xr + (t & 3) * q.PS * xge;
#pragma unroll
    for (int c = 0; c < MAXPT; ++c) {
        const int pe = threadIdx.x + c * kTraceThreads;
        if (pe < q.PL) {
            int i, j;
            plane_ij(pe, q.nx, q.rnx, i, j);
#pragma unroll
            for (int gi = 0; gi < GC; ++gi) lds_put(Sd, q, i, j, GC, gi, r.s[c][gi]);
            if (xg) {
                lds_put(Xd, q, i, j, 1, 0, r.x[c][0]);
            } else {
#pragma unroll
                for (int gi = 0; gi < GC; ++gi) lds_put(Xd, q, i, j, GC, gi, r.x[c][gi]);
            }
        }
    }
}

// bilinear value from an LDS plane with halo: base = tap (i0, j0), weights w
template <typename real>
__device__ __forceinline__ real bil(const real *pl, int base, int dx, int dy, const real w[4])
{
    return w[0] * pl[base] + w[1] * pl[base + dx] + w[2] * pl[base + dy] + w[3] * pl[base + dx + dy];
}

template <typename real, bool CHI_ARRAY, int GC, int MAXPT>
__global__ void __launch_bounds__(kTraceThreads, (MAXPT <= 2 && sizeof(real) == 4) ? 8 : 1) k_trace(TraceArgs<real> a)
{
    constexpr int T = kTraceThreads;
    extern __shared__ unsigned char smem_raw[];
    const int nx = a.nx, ny = a.ny, nz = a.nz, PL = nx * ny, G = a.G;
    const int nch = G / GC;
    const long item = xcd_item((long)a.K * nch);
    if (item >= (long)a.K * nch) return;
    const int k = (int)(item / nch), g0 = (int)(item - (long)k * nch) * GC;
    const TraceIdx q{nx, ny, PL, nx + 1, (nx + 1) * (ny + 1), 1.0f / (float)nx};
    const int NE = q.PS * GC;
    const bool xg = !CHI_ARRAY && a.chi_grey;        // one chi~ per point
    const int xge = xg ? 1 : GC, XE = q.PS * xge;
    real *Sr = reinterpret_cast<real *>(smem_raw);
    real *Xr = Sr + 4 * NE;
    real *Ir = Xr + 4 * XE;
    const OrdGeom gm = a.geo[k];
    const long slab = (long)k * a.P * G + g0;        // start of this ordinate's lab slab (+ chunk)
    const real *__restrict__ Sk = a.St + slab;
    const real *__restrict__ Xk = CHI_ARRAY ? a.Xt + slab : (xg ? nullptr : a.chilab + slab);
    const real *__restrict__ Ck = xg ? a.chilab + (long)k * a.P : nullptr;
    real *__restrict__ Ik = a.I + slab;
    const int tid = threadIdx.x;
    PlaneRegs<real, CHI_ARRAY, GC, MAXPT> rg;

    for (int t = 0; t < nz && t < 3; ++t) {
        trace_fetch(rg, Sk, Xk, Ck, G, PL, gm.up ? t : nz - 1 - t, a.inv_cdt, xg);
        trace_store(rg, Sr, Xr, q, t, xg);
    }
    {
        const int m0 = gm.up ? 0 : nz - 1;
        const real *__restrict__ bc = gm.up ? a.bc_bot : a.bc_top;
#pragma unroll
        for (int c = 0; c < MAXPT; ++c) {
            const int pe = tid + c * T;
            if (pe >= PL) break;
            int i, j;
            plane_ij(pe, nx, q.rnx, i, j);
#pragma unroll
            for (int gi = 0; gi < GC; ++gi) {
                const real v = bc ? bc[((long)k * PL + pe) * G + g0 + gi] : real(0);
                lds_put(Ir, q, i, j, GC, gi, v);
                Ik[(m0 * PL + pe) * G + gi] = v;
            }
        }
    }
    __syncthreads();
    const real ds = (real)gm.ds;
    real wts[3][4];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const real fx = (real)gm.fx[s], fy = (real)gm.fy[s];
        wts[s][0] = (real(1) - fx) * (real(1) - fy);
        wts[s][1] = fx * (real(1) - fy);
        wts[s][2] = (real(1) - fx) * fy;
        wts[s][3] = fx * fy;
    }
    const int dxS = GC, dyS = q.RS * GC, dxX = xge, dyX = q.RS * xge;
    for (int t = 1; t < nz; ++t) {
        if (t + 2 < nz) trace_fetch(rg, Sk, Xk, Ck, G, PL, gm.up ? t + 2 : nz - 3 - t, a.inv_cdt, xg);
        const int m = gm.up ? t : nz - 1 - t;
        const bool has_d = t <= nz - 2, has_uu = t >= 2;
        const real *Spl = Sr + (t & 3) * NE, *Xpl = Xr + (t & 3) * XE;
        const real *Sul = Sr + ((t - 1) & 3) * NE, *Xul = Xr + ((t - 1) & 3) * XE;
        const real *Suul = Sr + ((t - 2) & 3) * NE, *Xuul = Xr + ((t - 2) & 3) * XE;
        const real *Sdl = Sr + ((t + 1) & 3) * NE, *Xdl = Xr + ((t + 1) & 3) * XE;
        const real *Iprv = Ir;
        real res[MAXPT][GC];
#pragma unroll
        for (int c = 0; c < MAXPT; ++c) {
            const int pe = tid + c * T;
            if (pe >= PL) break;
            int i, j;
            plane_ij(pe, nx, q.rnx, i, j);
            // tap cells of the three shifted points (second upwind, upwind, downwind)
            int cell[3];
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                int i0 = i + gm.ix[s]; if (i0 >= nx) i0 -= nx;
                int j0 = j + gm.iy[s]; if (j0 >= ny) j0 -= ny;
                cell[s] = j0 * q.RS + i0;
            }
            const int self = j * q.RS + i;
            real Xp = 0, Xu = 0, Xd = 0, Xuu = 0;
            if (xg) {
                Xp = Xpl[self];
                Xu = bil(Xul, cell[1], dxX, dyX, wts[1]);
                if (has_d) Xd = bil(Xdl, cell[2], dxX, dyX, wts[2]);
                if (has_uu) Xuu = bil(Xuul, cell[0], dxX, dyX, wts[0]);
            }
            const int og = (m * PL + pe) * G;
#pragma unroll
            for (int gi = 0; gi < GC; ++gi) {
                if (!xg) {
                    Xp = Xpl[self * GC + gi];
                    Xu = bil(Xul + gi, cell[1] * GC, dxX, dyX, wts[1]);
                    if (has_d) Xd = bil(Xdl + gi, cell[2] * GC, dxX, dyX, wts[2]);
                    if (has_uu) Xuu = bil(Xuul + gi, cell[0] * GC, dxX, dyX, wts[0]);
                }
                const real Sp = Spl[self * GC + gi];
                const real Su = bil(Sul + gi, cell[1] * GC, dxS, dyS, wts[1]);
                const real Iu = bil(Iprv + gi, cell[1] * GC, dxS, dyS, wts[1]);
                const real hu = ds * real(0.5) * (Xu + Xp);
                real dSp = 0, dSu = 0;
                if (hu > real(0)) {
                    const real d1 = (Sp - Su) * fast_rcp(hu);
                    if (has_d) {
                        const real Sd = bil(Sdl + gi, cell[2] * GC, dxS, dyS, wts[2]);
                        const real hd = ds * real(0.5) * (Xp + Xd);
                        dSp = (hd > real(0)) ? fb_slope(d1, (Sd - Sp) * fast_rcp(hd), hu, hd) : real(0);
                    } else {
                        dSp = d1;
                    }
                    if (has_uu) {
                        const real Suu = bil(Suul + gi, cell[0] * GC, dxS, dyS, wts[0]);
                        const real huu = ds * real(0.5) * (Xuu + Xu);
                        dSu = (huu > real(0)) ? fb_slope((Su - Suu) * fast_rcp(huu), d1, huu, hu) : real(0);
                    } else {
                        dSu = d1;
                    }
                }
                const real Cu = clamp_between(Su + hu * dSu * real(1.0 / 3.0), Su, Sp);
                const real Cp = clamp_between(Sp - hu * dSp * real(1.0 / 3.0), Su, Sp);
                real ex, w0, w1, w2, w3;
                bezier_weights(hu, ex, w0, w1, w2, w3);
                const real v = Iu * ex + w0 * Su + w1 * Cu + w2 * Cp + w3 * Sp;
                res[c][gi] = v;
                Ik[og + gi] = v;
            }
        }
        __syncthreads();
        // every read of plane t - 1 is done: the intensity plane and the slot of
        // plane t - 2 can be overwritten
#pragma unroll
        for (int c = 0; c < MAXPT; ++c) {
            const int pe = tid + c * T;
            if (pe >= PL) break;
            int i, j;
            plane_ij(pe, nx, q.rnx, i, j);
#pragma unroll
            for (int gi = 0; gi < GC; ++gi) lds_put(Ir, q, i, j, GC, gi, res[c][gi]);
        }
        if (t + 2 < nz) trace_store(rg, Sr, Xr, q, t + 2, xg);
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

// Frequency remap for groups uniform in ln(nu) (spacing delta): the target
// frequency of group g sits at fractional group position g + y for every g, so
// the invariant F/nu^3 is interpolated between groups g + s and g + s + 1
// (s = floor y, weight f = y - s), groups -1 and G being the zero-valued ghost
// centres, and nu_g^3 / nu_{g'}^3 = exp(3 delta (g - g')).  A[g'] are the
// angular remaps of F at the taps; out[g] receives the lab (or comoving) value.
template <typename real>
__device__ __forceinline__ void uniform_remap(const real *F, int sk, int sg, int G, int nmu, int nphi,
                                              const TapL<real> &tp, const real *pole, double y, double delta,
                                              real *out, long ostride = 1)
{
    const double sf = floor(y);
    const double f = y - sf;
    const int s = (int)sf;
    const real clo = (real)((1.0 - f) * exp(-3.0 * delta * sf));
    const real chi = (real)(f * exp(-3.0 * delta * (sf + 1.0)));
    auto A = [&](int gp) -> real {
        return (gp >= 0 && gp < G) ? tap_value(F, sk, sg, G, gp, nmu, nphi, tp, pole) : real(0);
    };
    real acur = A(s);
    for (int g = 0; g < G; ++g) {
        const real anext = A(g + s + 1);
        out[g * ostride] = clo * acur + chi * anext;
        acur = anext;
    }
}

// ---------------------------------------------------------------------------
// S3: comoving ordinates -> lab ordinates, one workgroup per grid point, one
// thread per lab ordinate (all groups).  The point's comoving source S0[g][j]
// (from the SH -> ordinate product) is staged in LDS; the lab source of
// ordinate k is the bilinear (angle) x linear in ln(nu) remap of the invariant
// S0/nu^3 at the comoving direction n0 (Eq. 8) and frequency nu/D (Eq. 7) of
// that ray, times nu^3; then the implicit time terms of Eqs. 5-6 with the lab
// extinction chi_lab precomputed per medium.  Output S~[k][p][g].
// ---------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(kRemapThreads) k_boost(BoostArgs<real> a)
{
    extern __shared__ unsigned char smem_raw[];
    const long p = xcd_item(a.P);
    if (p >= a.P) return;
    const int G = a.fi.G, K = a.K, T = blockDim.x, tid = threadIdx.x, Gp = G + 1;
    double *fbuf = reinterpret_cast<double *>(smem_raw);                // [4G]
    real *sS0 = reinterpret_cast<real *>(fbuf + 4 * G);                 // [G][K]
    real *sPole = sS0 + G * K;                                          // [2][G]
    real *sOut = sPole + 2 * G;                                         // [T][G+1] lab values of a chunk of ordinates

    const FreqL fl = stage_freq(a.fi, fbuf);
    double b[3];
    const bool moving = load_beta(a.beta, p, b);
    const real *__restrict__ src = a.S0 + (long)p * G * K;
    for (int i = tid; i < G * K; i += T) sS0[i] = src[i];
    __syncthreads();
    if (moving) {
        for (int i = tid; i < 2 * G; i += T) {
            const int g = i % G, ring = (i < G) ? 0 : a.nmu - 1;
            real s = 0;
            for (int bb = 0; bb < a.nphi; ++bb) s += sS0[g * K + ring * a.nphi + bb];
            sPole[i] = s / real(a.nphi);
        }
        __syncthreads();
    }
    const real icdt = a.inv_cdt;
    const double gam = moving ? a.gam[p] : 1.0;
    for (int k0 = 0; k0 < K; k0 += T) {
        // lab source of ordinate k = k0 + tid, all groups, into the tile
        const int k = k0 + tid;
        if (k < K) {
            real *outk = sOut + tid * Gp;
            if (!moving) {
                for (int g = 0; g < G; ++g) outk[g] = sS0[g * K + k];
            } else {
                const double n[3] = {a.dir[4 * k], a.dir[4 * k + 1], a.dir[4 * k + 2]};
                const double bn = b[0] * n[0] + b[1] * n[1] + b[2] * n[2];
                const double D = 1.0 / inv_doppler(b, gam, n);
                const double f = gam * (1.0 - gam / (gam + 1.0) * bn);
                double n0[3];
                for (int c = 0; c < 3; ++c) n0[c] = D * (n[c] - f * b[c]);
                const AngleTaps at = angle_taps(a.mu, a.nmu, a.nphi, n0);
                const TapL<real> tp{at.a0, at.a1, at.b0, at.b1, (real)at.wmu, (real)at.wphi};
                if (a.fi.grey) {
                    const double D2 = D * D;
                    outk[0] = (real)(D2 * D2) * tap_value(sS0, 1, K, G, 0, a.nmu, a.nphi, tp, sPole);
                } else if (a.fi.uniform) {
                    uniform_remap(sS0, 1, K, G, a.nmu, a.nphi, tp, sPole, -log(D) * a.fi.inv_delta, a.fi.delta, outk);
                } else {
                    const double lnD = log(D);
                    FreqWalk fw{0};
                    if (G > 2) fw.lo = centre_bracket(fl.lnc, G, fl.lnc[0] - lnD);
                    for (int g = 0; g < G; ++g) {
                        const FreqTaps ft = freq_taps_zero_walk(a.fi, fl, fl.lnc[g] - lnD, fw);
                        double v = 0.0;
                        if (ft.gl >= 0) v += ft.wl * (double)tap_value(sS0, 1, K, G, ft.gl, a.nmu, a.nphi, tp, sPole) * fl.inv_nu3[ft.gl];
                        if (ft.gh >= 0) v += ft.wh * (double)tap_value(sS0, 1, K, G, ft.gh, a.nmu, a.nphi, tp, sPole) * fl.inv_nu3[ft.gh];
                        outk[g] = (real)(fl.nu3[g] * v);
                    }
                }
            }
        }
        __syncthreads();
        // implicit time terms and a coalesced write of the chunk: runs of G values per ordinate
        const int nk = min(T, K - k0);
        const float rG = 1.0f / (float)G;
        for (int idx = tid; idx < nk * G; idx += T) {
            const int kk = (int)(((float)idx + 0.5f) * rG), g = idx - kk * G;
            const long o = ((long)(k0 + kk) * a.P + p) * G + g;
            const real Sl = sOut[kk * Gp + g];
            const real chil = a.chi_grey ? a.chilab[(long)(k0 + kk) * a.P + p] : a.chilab[o];
            const real ip = a.Iprev ? a.Iprev[o] : real(0);
            const real xt = chil + icdt;
            a.St[o] = (xt > real(0)) ? (chil * Sl + ip * icdt) / xt : real(0);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// S5: lab ordinates -> comoving ordinates, one workgroup per grid point, one
// thread per comoving ordinate.  The point's lab intensities I[k][g] are
// staged in LDS; the comoving value of ordinate j is the remap of the
// invariant I/nu^3 at the lab direction and frequency D' nu of that comoving
// ray.  Output I0[p][g][j].
// ---------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(kRemapThreads) k_unboost(UnboostArgs<real> a)
{
    extern __shared__ unsigned char smem_raw[];
    const long p = xcd_item(a.P);
    if (p >= a.P) return;
    const int G = a.fi.G, K = a.K, T = blockDim.x, tid = threadIdx.x, Gp = G + 1;
    double *fbuf = reinterpret_cast<double *>(smem_raw);                // [4G]
    real *sI = reinterpret_cast<real *>(fbuf + 4 * G);                  // [K][G+1] lab (padded rows)
    real *sPole = sI + K * Gp;                                          // [2][G]

    const FreqL fl = stage_freq(a.fi, fbuf);
    double b[3];
    const bool moving = load_beta(a.beta, p, b);
    const float rG = 1.0f / (float)G, rK = 1.0f / (float)K;
    for (int idx = tid; idx < K * G; idx += T) {
        const int k = (int)(((float)idx + 0.5f) * rG), g = idx - k * G;
        sI[k * Gp + g] = a.Ilab[((long)k * a.P + p) * G + g];
    }
    __syncthreads();
    real *__restrict__ out = a.I0 + (long)p * G * K;
    if (!moving) {
        for (int idx = tid; idx < K * G; idx += T) {
            const int g = (int)(((float)idx + 0.5f) * rK), j = idx - g * K;
            out[idx] = sI[j * Gp + g];
        }
        return;
    }
    for (int i = tid; i < 2 * G; i += T) {
        const int g = i % G, ring = (i < G) ? 0 : a.nmu - 1;
        real s = 0;
        for (int bb = 0; bb < a.nphi; ++bb) s += sI[(ring * a.nphi + bb) * Gp + g];
        sPole[i] = s / real(a.nphi);
    }
    __syncthreads();
    const double gam = a.gam[p];
    for (int j = tid; j < K; j += T) {
        const double n0[3] = {a.dir[4 * j], a.dir[4 * j + 1], a.dir[4 * j + 2]};
        const double bn0 = b[0] * n0[0] + b[1] * n0[1] + b[2] * n0[2];
        const double Dp = gam * (1.0 + bn0);
        const double f = gam * (1.0 + gam / (gam + 1.0) * bn0);
        double n[3];
        for (int c = 0; c < 3; ++c) n[c] = (n0[c] + f * b[c]) / Dp;
        const AngleTaps at = angle_taps(a.mu, a.nmu, a.nphi, n);
        const TapL<real> tp{at.a0, at.a1, at.b0, at.b1, (real)at.wmu, (real)at.wphi};
        const double lnD = log(Dp);
        if (!a.fi.grey && a.fi.uniform) {
            uniform_remap(sI, Gp, 1, G, a.nmu, a.nphi, tp, sPole, lnD * a.fi.inv_delta, a.fi.delta, out + j, K);
            continue;
        }
        FreqWalk fw{0};
        if (!a.fi.grey && G > 2) fw.lo = centre_bracket(fl.lnc, G, fl.lnc[0] + lnD);
        for (int g = 0; g < G; ++g) {
            real v;
            if (a.fi.grey) {
                const double D2 = Dp * Dp;
                v = (real)((double)tap_value(sI, Gp, 1, G, g, a.nmu, a.nphi, tp, sPole) / (D2 * D2));
            } else {
                const FreqTaps ft = freq_taps_zero_walk(a.fi, fl, fl.lnc[g] + lnD, fw);
                double s = 0.0;
                if (ft.gl >= 0) s += ft.wl * (double)tap_value(sI, Gp, 1, G, ft.gl, a.nmu, a.nphi, tp, sPole) * fl.inv_nu3[ft.gl];
                if (ft.gh >= 0) s += ft.wh * (double)tap_value(sI, Gp, 1, G, ft.gh, a.nmu, a.nphi, tp, sPole) * fl.inv_nu3[ft.gh];
                v = (real)(fl.nu3[g] * s);
            }
            out[(long)g * K + j] = v;
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

// Compton: one workgroup per point; its SH intensities I[i][q] (all groups) are
// staged in LDS and S[j][q] = sigma/chi_j sum_i A_l(q)[j][i] I[i][q] + T_q
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
            const real *__restrict__ Arow = a.A + ((long)l * G + j) * G;
            real acc = 0;
            for (int i = 0; i < G; ++i) acc += Arow[i] * sI[i * NL + q];
            v = sig / chi * acc;
            if (q == 0) v += real(3.5449077018110318) * a.kappa[p * G + j] * a.bnu[p * G + j] / chi;
        }
        a.S[p * G * NL + o] = v;
    }
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
__global__ void __launch_bounds__(256) k_resid_rows(long PG, int NL, const real *__restrict__ a,
                                                    const real *__restrict__ b, double *rows)
{
    const int lane = threadIdx.x & 63;
    const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long nwaves = ((long)gridDim.x * blockDim.x) >> 6;
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
            rows[2 * r] = dd;
            rows[2 * r + 1] = aa;
        }
    }
}

// out[2g + c] = sum over points of rows[2 (p G + g) + c]; one block per (g, c)
__global__ void __launch_bounds__(256) k_resid_groups(long P, int G, const double *__restrict__ rows, double *out)
{
    __shared__ double sh[256];
    const int g = blockIdx.x >> 1, c = blockIdx.x & 1;
    double v = 0;
    for (long p = threadIdx.x; p < P; p += blockDim.x) v += rows[2 * (p * G + g) + c];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) out[2 * g + c] = v;
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
size_t trace_lds(int nx, int ny, int Gc, int chi_per_point)
{
    return sizeof(real) * (size_t)(nx + 1) * (ny + 1) * (5 * (size_t)Gc + 4 * (chi_per_point ? 1 : (size_t)Gc));
}
template <typename real>
void launch_trace(const TraceArgs<real> &a, bool chi_array, hipStream_t st)
{
    const size_t sm = trace_lds<real>(a.nx, a.ny, a.Gc, !chi_array && a.chi_grey);
    const long items = (long)a.K * (a.G / a.Gc);
    const dim3 grid((unsigned)(8 * ((items + 7) / 8))), block(kTraceThreads);
    const int npt = (a.nx * a.ny + kTraceThreads - 1) / kTraceThreads;
#define RRT_TRACE_CASE(GC, MP)                                                                     \
    if (a.Gc == GC && npt <= MP) {                                                                 \
        if (chi_array) hipLaunchKernelGGL((k_trace<real, true, GC, MP>), grid, block, sm, st, a);  \
        else hipLaunchKernelGGL((k_trace<real, false, GC, MP>), grid, block, sm, st, a);           \
        return;                                                                                    \
    }
    RRT_TRACE_CASE(1, 1)
    RRT_TRACE_CASE(1, 2)
    RRT_TRACE_CASE(1, 8)
    RRT_TRACE_CASE(2, 1)
    RRT_TRACE_CASE(2, 2)
    RRT_TRACE_CASE(2, 8)
#undef RRT_TRACE_CASE
}
template <typename real>
size_t boost_lds(int K, int G)
{
    return 4 * sizeof(double) * G + sizeof(real) * ((size_t)K * (G + 1) + 2 * G + kRemapThreads * (size_t)(G + 1));
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
    const unsigned nb = (unsigned)(8 * ((a.P + 7) / 8));
    hipLaunchKernelGGL(k_boost<real>, dim3(nb), dim3(kRemapThreads), boost_lds<real>(a.K, a.fi.G), st, a);
}
template <typename real>
void launch_unboost(const UnboostArgs<real> &a, hipStream_t st)
{
    const unsigned nb = (unsigned)(8 * ((a.P + 7) / 8));
    hipLaunchKernelGGL(k_unboost<real>, dim3(nb), dim3(kRemapThreads), boost_lds<real>(a.K, a.fi.G), st, a);
}
template <typename real>
void launch_source(const SourceArgs<real> &a, hipStream_t st)
{
    if (a.compton) {
        const unsigned nb = (unsigned)(8 * ((a.P + 7) / 8));
        hipLaunchKernelGGL(k_source_compton<real>, dim3(nb), dim3(256), sizeof(real) * (size_t)a.G * a.NL, st, a);
    } else {
        hipLaunchKernelGGL(k_source<real>, dim3(blocks_for(a.P * a.G * a.NL, 256)), dim3(256), 0, st, a);
    }
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
void launch_resid(long P, int G, int NL, const real *a, const real *b, double *rows, int nblk, double *out, hipStream_t st)
{
    (void)nblk;
    const unsigned nb = (unsigned)std::min<long>((P * G + 3) / 4, 8192);   // 4 waves per block, one row each
    hipLaunchKernelGGL(k_resid_rows<real>, dim3(nb), dim3(256), 0, st, P * G, NL, a, b, rows);
    hipLaunchKernelGGL(k_resid_groups, dim3(2 * G), dim3(256), 0, st, P, G, rows, out);
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

hipError_t set_lds_limits(size_t bytes)
{
    const void *fns[] = {reinterpret_cast<const void *>(&k_trace<float, true, 1, 1>),
                         reinterpret_cast<const void *>(&k_trace<float, true, 1, 2>),
                         reinterpret_cast<const void *>(&k_trace<float, true, 1, 8>),
                         reinterpret_cast<const void *>(&k_trace<float, true, 2, 1>),
                         reinterpret_cast<const void *>(&k_trace<float, true, 2, 2>),
                         reinterpret_cast<const void *>(&k_trace<float, true, 2, 8>),
                         reinterpret_cast<const void *>(&k_trace<float, false, 1, 1>),
                         reinterpret_cast<const void *>(&k_trace<float, false, 1, 2>),
                         reinterpret_cast<const void *>(&k_trace<float, false, 1, 8>),
                         reinterpret_cast<const void *>(&k_trace<float, false, 2, 1>),
                         reinterpret_cast<const void *>(&k_trace<float, false, 2, 2>),
                         reinterpret_cast<const void *>(&k_trace<float, false, 2, 8>),
                         reinterpret_cast<const void *>(&k_trace<double, true, 1, 1>),
                         reinterpret_cast<const void *>(&k_trace<double, true, 1, 2>),
                         reinterpret_cast<const void *>(&k_trace<double, true, 1, 8>),
                         reinterpret_cast<const void *>(&k_trace<double, true, 2, 1>),
                         reinterpret_cast<const void *>(&k_trace<double, true, 2, 2>),
                         reinterpret_cast<const void *>(&k_trace<double, true, 2, 8>),
                         reinterpret_cast<const void *>(&k_trace<double, false, 1, 1>),
                         reinterpret_cast<const void *>(&k_trace<double, false, 1, 2>),
                         reinterpret_cast<const void *>(&k_trace<double, false, 1, 8>),
                         reinterpret_cast<const void *>(&k_trace<double, false, 2, 1>),
                         reinterpret_cast<const void *>(&k_trace<double, false, 2, 2>),
                         reinterpret_cast<const void *>(&k_trace<double, false, 2, 8>),
                         reinterpret_cast<const void *>(&k_boost<float>),
                         reinterpret_cast<const void *>(&k_boost<double>),
                         reinterpret_cast<const void *>(&k_unboost<float>),
                         reinterpret_cast<const void *>(&k_unboost<double>),
                         reinterpret_cast<const void *>(&k_source_compton<float>),
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
    template size_t boost_lds<real>(int, int);                                                                 \
    template void launch_chilab<real>(const ChiLabArgs<real> &, hipStream_t);                                   \
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
