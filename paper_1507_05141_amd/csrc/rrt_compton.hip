// Group-to-group Compton tables on the GPU (FP64), for electrons at rest (the
// paper's Klein-Nishina kernel, Sec. 2.3, Eqs. 13-14) and for a thermal
// (Maxwell-Juttner) electron gas on temperature nodes.
//
// For an electron of speed beta (Lorentz factor gam) whose velocity makes the
// cosine mu_e with the incident photon (taken along z, the velocity in the
// x-z plane), a photon of x = h nu / m_e c^2 scattered into (mu1, phi1) leaves
// with nu1 = nu (1 - beta mu_e) / (1 - beta.Omega1 + (x / gam)(1 - mu1)); the
// scattered photons per unit solid angle and photon path, per electron, are
// R = (1 - beta mu_e) (dsigma/dOmega')_KN (nu1 / nu1')^2, evaluated with the
// rest-frame frequencies nu' = gam nu (1 - beta mu_e), nu1' = gam nu1
// (1 - beta.Omega1) and the rest-frame scattering angle from
// nu nu1 (1 - mu1) = nu' nu1' (1 - cos Theta').  The tables average R over
// the electrons and the scattered azimuth with fixed quadrature rules:
// momentum by 16-point Gauss-Legendre in t on [0, 6], (gam - 1)/Theta = t^2,
// weight p gam t e^{-t^2}; mu_e by 16 points on [-1, 1]; phi1 by 12 points on
// [0, pi]; along mu1, each interval on which nu1 stays in one group (split at
// the roots of nu1 = edge) by 4 equal pieces of 48-point Gauss-Legendre.  At
// kT = 0 the average is the electron at rest.
//   s_i = integral of <R> over directions / sigma_T
//   p_l^{i->j} = (2l+1)/2 int_{nu1 in j} P_l(mu1) 4 pi <R>(mu1) dmu1 / (s_i sigma_T)
//   A_l[j][i] = s_i (nu_j dnu_i)/(nu_i dnu_j) p_l^{i->j} / (2l+1)
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "rrt_internal.h"
#include "rrt_kernels.h"

namespace rrt {

namespace {

constexpr int kNQ = 48, kNT = 16, kNE = 16, kNF = 12, kChunks = 16, kMaxL = 15;
constexpr double kPiC = 3.14159265358979323846;

struct QuadRules {
    double gx[kNQ], gw[kNQ], tx[kNT], tw[kNT], ex[kNE], ew[kNE], fx[kNF], fw[kNF];
};

struct Electron {
    double beta, gam, mue, sine, cphi;
};

__device__ double kn_dsdo(double x, double mu)
{
    const double r = 1.0 / (1.0 + x * (1.0 - mu));
    return 0.5 * r * r * (r + 1.0 / r - (1.0 - mu * mu));
}

// Klein-Nishina total cross-section (r0^2 units) by 8 pieces of 48-point Gauss-Legendre
__device__ double kn_sigma(double x, const QuadRules &q)
{
    double tot = 0.0;
    for (int piece = 0; piece < 8; ++piece) {
        const double c = -1.0 + 0.25 * piece + 0.125;
        double v = 0.0;
        for (int k = 0; k < kNQ; ++k) v += q.gw[k] * kn_dsdo(x, c + 0.125 * q.gx[k]);
        tot += 0.125 * v;
    }
    return 2.0 * kPiC * tot;
}

__device__ double out_freq(double nu, double x, const Electron &e, double mu1)
{
    const double s1 = sqrt(fmax(0.0, 1.0 - mu1 * mu1));
    const double bo1 = e.beta * (e.sine * s1 * e.cphi + e.mue * mu1);
    return nu * (1.0 - e.beta * e.mue) / (1.0 - bo1 + x / e.gam * (1.0 - mu1));
}

__device__ double lab_rate(double nu, double x, const Electron &e, double mu1)
{
    const double s1 = sqrt(fmax(0.0, 1.0 - mu1 * mu1));
    const double bo = e.beta * e.mue;
    const double bo1 = e.beta * (e.sine * s1 * e.cphi + e.mue * mu1);
    const double nu1 = nu * (1.0 - bo) / (1.0 - bo1 + x / e.gam * (1.0 - mu1));
    const double nup = e.gam * nu * (1.0 - bo), nu1p = e.gam * nu1 * (1.0 - bo1);
    const double c = 1.0 - nu * nu1 * (1.0 - mu1) / (nup * nu1p);
    const double r = nu1p / nup;
    const double jac = nu1 / nu1p;
    return (1.0 - bo) * 0.5 * r * r * (1.0 / r + r - (1.0 - c * c)) * jac * jac;
}

// roots in (-1, 1) of a + b mu + c sqrt(1 - mu^2) = 0; appended to r, count returned
__device__ int cut_roots(double a, double b, double c, double *r)
{
    if (c == 0.0) {
        if (b == 0.0) return 0;
        const double m = -a / b;
        if (m > -1.0 && m < 1.0) { r[0] = m; return 1; }
        return 0;
    }
    // mu = cos psi: sqrt(b^2 + c^2) cos(psi - atan2(c, b)) = -a, psi in (0, pi)
    const double R = sqrt(b * b + c * c), y = -a / R;
    if (y < -1.0 || y > 1.0) return 0;
    const double d = atan2(c, b), g = acos(y);
    int n = 0;
    for (int k = 0; k < 2; ++k) {
        double psi = k ? d + g : d - g;
        if (psi > kPiC) psi -= 2.0 * kPiC;
        if (psi < -kPiC) psi += 2.0 * kPiC;
        if (psi > 0.0 && psi < kPiC) {
            const double m = cos(psi);
            if (m > -1.0 && m < 1.0 && !(n == 1 && r[0] == m)) r[n++] = m;
        }
    }
    return n;
}

// momentum node a of temperature theta (kT / m_e c^2): speed, Lorentz factor and
// (unnormalised) weight; theta = 0: the electron at rest
__device__ void momentum_node(double theta, int a, const QuadRules &q, double &beta, double &gam, double &w)
{
    if (theta <= 0.0) { beta = 0.0; gam = 1.0; w = 1.0; return; }
    const double t = 3.0 * (q.tx[a] + 1.0);
    gam = 1.0 + theta * t * t;
    const double pm = sqrt(gam * gam - 1.0);
    beta = pm / gam;
    w = 3.0 * q.tw[a] * pm * gam * t * exp(-t * t);
}

struct TableArgs {
    int G, lmax, nt;
    double mec2;
    const double *edges, *centres, *kT;      // [G+1], [G], [nt]
    const QuadRules *q;
    double *sig_part;                        // [nt][G][kNT * kNE]
    double *band_part;                       // [nt][G][G][kChunks][lmax+1]
};

// the thermal total cross-section, one term per (node, group, momentum node, direction node)
__global__ void __launch_bounds__(256) k_kn_sigma(TableArgs a)
{
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = (long)a.nt * a.G * kNT * kNE;
    if (id >= total) return;
    const int ab = (int)(id % (kNT * kNE));
    const int i = (int)((id / (kNT * kNE)) % a.G), n = (int)(id / ((long)kNT * kNE * a.G));
    const QuadRules &q = *a.q;
    const double theta = a.kT[n] / a.mec2, x = a.centres[i] / a.mec2;
    const int ia = ab / kNE, ib = ab % kNE;
    double v = 0.0;
    if (theta > 0.0 || (ia == 0 && ib == 0)) {
        double beta, gam, w;
        momentum_node(theta, ia, q, beta, gam, w);
        const double mue = theta > 0.0 ? q.ex[ib] : 1.0, wmue = theta > 0.0 ? 0.5 * q.ew[ib] : 1.0;
        v = w * wmue * (1.0 - beta * mue) * kn_sigma(gam * x * (1.0 - beta * mue), q);
    }
    a.sig_part[id] = v;
}

// P_l-weighted integrals of the averaged rate over the scattering cosines that
// land in group j, one thread per (node, group i, group j, chunk of the
// electron / azimuth nodes)
__global__ void __launch_bounds__(128) k_kn_bands(TableArgs a)
{
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int G = a.G, L = a.lmax;
    const long total = (long)a.nt * G * G * kChunks;
    if (id >= total) return;
    const int c = (int)(id % kChunks);
    const int j = (int)((id / kChunks) % G);
    const int i = (int)((id / ((long)kChunks * G)) % G);
    const int n = (int)(id / ((long)kChunks * G * G));
    const QuadRules &q = *a.q;
    const double theta = a.kT[n] / a.mec2, nu = a.centres[i], x = nu / a.mec2;
    const double e0 = a.edges[j], e1 = a.edges[j + 1];
    double acc[kMaxL + 1];
    for (int l = 0; l <= L; ++l) acc[l] = 0.0;
    const int nouter = theta > 0.0 ? kNT * kNE * kNF : 1;
    for (int o = c; o < nouter; o += kChunks) {
        const int ia = o / (kNE * kNF), ib = (o / kNF) % kNE, ifp = o % kNF;
        double beta, gam, wt;
        momentum_node(theta, ia, q, beta, gam, wt);
        const double mue = theta > 0.0 ? q.ex[ib] : 1.0, wmue = theta > 0.0 ? 0.5 * q.ew[ib] : 1.0;
        const double phi = theta > 0.0 ? 0.5 * kPiC * (q.fx[ifp] + 1.0) : 0.0;
        const double wphi = theta > 0.0 ? 0.5 * q.fw[ifp] : 1.0;
        const Electron e{beta, gam, mue, sqrt(fmax(0.0, 1.0 - mue * mue)), cos(phi)};
        const double w = wt * wmue * wphi;
        // cut points: the ends and the roots of nu1 = e0, nu1 = e1
        double cut[6];
        int nc = 0;
        cut[nc++] = -1.0;
        cut[nc++] = 1.0;
        const double edge[2] = {e0, e1};
        for (int k = 0; k < 2; ++k) {
            const double E = edge[k];
            if (!(E > 0.0)) continue;
            // nu1 = E: nu (1 - beta mu_e) = E (1 - beta.Omega1 + (x / gam)(1 - mu1))
            nc += cut_roots(nu * (1.0 - beta * mue) - E * (1.0 + x / gam), E * (x / gam + beta * mue),
                            E * beta * e.sine * e.cphi, cut + nc);
        }
        for (int u = 1; u < nc; ++u)                  // insertion sort of at most six values
            for (int v = u; v > 0 && cut[v - 1] > cut[v]; --v) {
                const double t = cut[v]; cut[v] = cut[v - 1]; cut[v - 1] = t;
            }
        for (int s = 0; s + 1 < nc; ++s) {
            const double lo = cut[s], hi = cut[s + 1];
            if (!(hi > lo)) continue;
            const double nm = out_freq(nu, x, e, 0.5 * (lo + hi));
            if (!(nm >= e0 && nm < e1)) continue;
            for (int piece = 0; piece < 4; ++piece) {
                const double pa = lo + (hi - lo) * piece / 4.0, pb = lo + (hi - lo) * (piece + 1) / 4.0;
                const double hh = 0.5 * (pb - pa), cc = 0.5 * (pb + pa);
                for (int k = 0; k < kNQ; ++k) {
                    const double mu1 = cc + hh * q.gx[k];
                    const double v = w * q.gw[k] * hh * lab_rate(nu, x, e, mu1);
                    double p0 = 1.0, p1 = mu1;
                    acc[0] += v;
                    if (L >= 1) acc[1] += v * mu1;
                    for (int l = 2; l <= L; ++l) {
                        const double p2 = ((2.0 * l - 1.0) * mu1 * p1 - (l - 1.0) * p0) / l;
                        acc[l] += v * p2;
                        p0 = p1;
                        p1 = p2;
                    }
                }
            }
        }
    }
    double *out = a.band_part + id * (L + 1);
    for (int l = 0; l <= L; ++l) out[l] = acc[l];
}

// sums in a fixed order and the final tables: s [nt][G] and p [nt][L+1][G][G] (FP64)
__global__ void __launch_bounds__(256) k_kn_finish(TableArgs a, double *s_out, double *p_out)
{
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int G = a.G, L = a.lmax;
    const long total = (long)a.nt * (L + 1) * G * G;
    if (id >= total) return;
    const int j = (int)(id % G), i = (int)((id / G) % G), l = (int)((id / ((long)G * G)) % (L + 1));
    const int n = (int)(id / ((long)G * G * (L + 1)));
    const double theta = a.kT[n] / a.mec2;
    double wsum = 0.0, sig = 0.0;
    {
        const QuadRules &q = *a.q;
        for (int ia = 0; ia < kNT; ++ia) {
            double beta, gam, w;
            momentum_node(theta, ia, q, beta, gam, w);
            wsum += w;
            if (theta <= 0.0) break;
        }
        const double *sp = a.sig_part + ((long)n * G + i) * kNT * kNE;
        for (int k = 0; k < kNT * kNE; ++k) sig += sp[k];
    }
    double band = 0.0;
    const double *bp = a.band_part + (((long)n * G + i) * G + j) * kChunks * (L + 1);
    for (int c = 0; c < kChunks; ++c) band += bp[(long)c * (L + 1) + l];
    sig /= wsum;
    band /= wsum;
    p_out[id] = (2.0 * l + 1.0) / 2.0 * 4.0 * kPiC / sig * band;
    if (l == 0 && j == 0) s_out[(long)n * G + i] = sig / (8.0 * kPiC / 3.0);
}

}  // namespace

namespace {

// the Gauss-Legendre rules of the table definition (computed once)
const QuadRules &quad_rules()
{
    static QuadRules h{};
    static bool done = false;
    static std::mutex mu;
    std::lock_guard<std::mutex> lock(mu);
    if (!done) {
        gauss_legendre(kNQ, h.gx, h.gw);
        gauss_legendre(kNT, h.tx, h.tw);
        gauss_legendre(kNE, h.ex, h.ew);
        gauss_legendre(kNF, h.fx, h.fw);
        done = true;
    }
    return h;
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

}  // namespace

size_t compton_scratch_bytes(int G, int lmax, int nt)
{
    const size_t nsig = (size_t)nt * G * kNT * kNE, nband = (size_t)nt * G * G * kChunks * (lmax + 1);
    const size_t np = (size_t)nt * (lmax + 1) * G * G;
    return align256(sizeof(QuadRules)) + align256(8 * ((size_t)G + 1)) + align256(8 * (size_t)G) +
           align256(8 * (size_t)nt) + align256(8 * nsig) + align256(8 * nband) + align256(8 * np) +
           align256(8 * (size_t)nt * G);
}

// Tables at the node temperatures kT[0..nt) (units of the edges; 0 = electrons
// at rest) in the scratch buffer buf (device memory of compton_scratch_bytes):
// s [nt][G] and p [nt][lmax+1][G][G] are written to the host arrays s_out,
// p_out in FP64.  Every scratch element is written before it is read.
int compton_tables_in(int G, const double *edges, const double *centres, double mec2, int lmax, int nt,
                      const double *kT, void *scratch_buf, double *s_out, double *p_out, void *stream)
{
    if (lmax > kMaxL) return (int)hipErrorInvalidValue;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const QuadRules &h = quad_rules();
    const size_t nsig = (size_t)nt * G * kNT * kNE, nband = (size_t)nt * G * G * kChunks * (lmax + 1);
    const size_t np = (size_t)nt * (lmax + 1) * G * G;
    char *cur = static_cast<char *>(scratch_buf);
    auto take = [&](size_t n) { char *r = cur; cur += align256(n); return r; };
    QuadRules *d_q = reinterpret_cast<QuadRules *>(take(sizeof(QuadRules)));
    double *d_edges = reinterpret_cast<double *>(take(8 * ((size_t)G + 1)));
    double *d_centres = reinterpret_cast<double *>(take(8 * (size_t)G));
    double *d_kT = reinterpret_cast<double *>(take(8 * (size_t)nt));
    double *d_sig = reinterpret_cast<double *>(take(8 * nsig));
    double *d_band = reinterpret_cast<double *>(take(8 * nband));
    double *d_p = reinterpret_cast<double *>(take(8 * np));
    double *d_s = reinterpret_cast<double *>(take(8 * (size_t)nt * G));
    hipError_t e = hipMemcpyAsync(d_q, &h, sizeof(QuadRules), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_edges, edges, 8 * ((size_t)G + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_centres, centres, 8 * (size_t)G, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_kT, kT, 8 * (size_t)nt, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        TableArgs a{G, lmax, nt, mec2, d_edges, d_centres, d_kT, d_q, d_sig, d_band};
        hipLaunchKernelGGL(k_kn_sigma, dim3((unsigned)((nsig + 255) / 256)), dim3(256), 0, st, a);
        const size_t nthr = (size_t)nt * G * G * kChunks;
        hipLaunchKernelGGL(k_kn_bands, dim3((unsigned)((nthr + 127) / 128)), dim3(128), 0, st, a);
        hipLaunchKernelGGL(k_kn_finish, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, a, d_s, d_p);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(s_out, d_s, 8 * (size_t)nt * G, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(p_out, d_p, 8 * np, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return (int)e;
}

// the same with a scratch buffer allocated for the call
int compton_tables_gpu(int G, const double *edges, const double *centres, double mec2, int lmax, int nt,
                       const double *kT, std::vector<double> &s, std::vector<double> &p, void *stream)
{
    if (lmax > kMaxL) return (int)hipErrorInvalidValue;
    void *buf = nullptr;
    hipError_t e = hipMalloc(&buf, compton_scratch_bytes(G, lmax, nt));
    if (e != hipSuccess) return (int)e;
    s.assign((size_t)nt * G, 0.0);
    p.assign((size_t)nt * (lmax + 1) * G * G, 0.0);
    const int r = compton_tables_in(G, edges, centres, mec2, lmax, nt, kT, buf, s.data(), p.data(), stream);
    (void)hipFree(buf);
    return r;
}

// Scratch of the allocation-free table builder: a file-scope device array, one
// copy per GPU the library runs on, held until the process ends.  Host code
// reaches it only through the address hipGetSymbolAddress returns on each
// device (the array's name is a host-side stand-in there).  Calls on one GPU
// share it: calls that overlap on one GPU race.
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

size_t compton_static_scratch_bytes() { return kStaticScratchBytes; }

namespace {

constexpr int kMaxDevices = 64;

// this device's address of the scratch array, looked up once per device with
// that device current
hipError_t static_scratch(void **out)
{
    static std::mutex mu;
    static void *ptr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[dev] = p;
    }
    *out = ptr[dev];
    return hipSuccess;
}

}  // namespace

int compton_tables_static(int G, const double *edges, const double *centres, double mec2, int lmax, int nt,
                          const double *kT, double *s_out, double *p_out, void *stream)
{
    if (lmax > kMaxL || compton_scratch_bytes(G, lmax, nt) > kStaticScratchBytes) return (int)hipErrorInvalidValue;
    void *buf = nullptr;
    const hipError_t e = static_scratch(&buf);
    if (e != hipSuccess) return (int)e;
    return compton_tables_in(G, edges, centres, mec2, lmax, nt, kT, buf, s_out, p_out, stream);
}

}  // namespace rrt
