// Argument blocks and launchers of the library's HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace rrt {

constexpr int kTraceThreads = 1024;    // threads per ray-trace workgroup
constexpr int kTraceMaxPlane = 4096;   // grid points of an x-y plane (at most): four per ray-trace thread
constexpr int kRemapThreads = 512;  // threads per frame-transform workgroup (one lab ordinate each)

// Per-ordinate geometry of the short characteristic.  The path from the
// previous z plane to a grid point is cut into npc equal pieces of length ds
// (dz/(|mu| npc)), npc being the fewest that move the ray at most one cell
// sideways.  Path point c (0 = the grid point, npc = the upwind point on the
// previous plane, -1 and npc + 1 one piece beyond either end) lies c ds back
// along -n, at the horizontal offset of tap table entry tap0 + c + 1.
struct OrdGeom {
    double ds;
    int up;
    int npc;
    int tap0;
};

// Tap of a path point: the horizontal offset in cells (integer part reduced
// modulo nx, ny) and eight weights, w[0..3] of the (x, y), (x + 1, y),
// (x, y + 1), (x + 1, y + 1) neighbours on the nearer grid plane and w[4..7] of
// the same neighbours on the farther one: the bilinear weights times 1 - f and
// f, f being the path point's fraction of the plane spacing from the nearer
// plane (0 on a grid plane).
template <typename real> struct PathTap {
    int ix, iy;
    real w[8];
};

// Group centres for the ln(nu) interpolation of the frame transforms.
struct FreqInfo {
    int G;
    int grey;
    int has_lo_ghost;        // lowest edge > 0: a zero-valued ghost centre below
    double ghost_lo, ghost_hi;
    double inv_lo, inv_hi;   // 1/(lnc[0]-ghost_lo), 1/(ghost_hi-lnc[G-1])
    int uniform;             // centres uniform in ln(nu) with the ghosts one spacing out
    double delta, inv_delta; // that spacing and its reciprocal
    const double *lnc;       // [G] ln(centre)
    const double *inv_dc;    // [G-1] 1/(lnc[g+1]-lnc[g])
    const double *nu3;       // [G] centre^3
    const double *inv_nu3;   // [G] 1/centre^3
};

// Lab-frame arrays (S~, I, stage inputs) are laid out [k][p][g]: ordinate,
// point, group innermost.  Comoving ordinate arrays are [p][g][j].
template <typename real> struct TraceArgs {
    int nx, ny, nz, G, K, Gc;   // Gc groups per workgroup (divides G)
    long P;
    const OrdGeom *geo;
    const PathTap<real> *taps;  // path taps of every ordinate (OrdGeom::tap0)
    const int *order;           // ordinates by decreasing number of pieces (the costliest start first)
    int nmulti;                 // how many of them take more than one piece
    const double *dir;          // [K][4]
    const real *St;             // S~ [k][p][g]
    const real *Xt;             // chi~ [k][p][g] (stand-alone trace only)
    const real *chilab;         // lab extinction [k][p] (chi_grey) or [k][p][g]
    int chi_grey;
    real inv_cdt;               // 1/(c dt) of the implicit time step, 0 when steady
    const real *bc_bot, *bc_top;  // [k][ny][nx][g] or NULL
    real *I;                    // [k][p][g]
    int gmajor;                 // St, Xt, a per-group chilab and I are [k][g][p] instead (Gc = 1)
};

// Remap of one ordinate at one moving point, fixed by the medium (velocity
// field) and computed once per medium.  Word `abs` packs the four bilinear
// angle taps of the direction in the other frame (ring a0 = (abs & 1023) - 1
// with a1 = a0 + 1, azimuth b0 = (abs >> 10) & 1023 with b1 = b0 + 1 mod nphi;
// rings -1 and nmu are the poles) and, for groups uniform in ln(nu), the
// position shift s = abs >> 20 (signed; kPackedGhost when every target lies
// beyond the groups); w are the tap weights.  Frequency: for a single group
// u = D^4 (to the lab) or D'^-4 (to the comoving frame); for uniform groups the
// two weights u, v with the nu^3 ratios; otherwise the ln(nu) shift u + v split
// into a high and a low part.  kap: the lab extinction of the ordinate at the
// point where it is the same for every group (boost entries only).
template <typename real> struct alignas(16) RemapEntry {
    int abs;
    real kap;
    real w[4];
    real u, v;
};
constexpr int kPackedGhost = -2048;       // s field of abs: every target beyond the groups
constexpr int kAllGhost = -(1 << 30);

template <typename real> struct PlanArgs {
    long P;
    int K, nmu, nphi;
    FreqInfo fi;
    const double *dir, *mu;      // [K][4], [nmu]
    const double *beta, *gam;    // [P][3], [P]
    const real *chilab;          // [k][p] when chi_grey (copied into the boost entries)
    int chi_grey;
    RemapEntry<real> *boost;     // [p][k]: comoving taps of lab ordinate k
    RemapEntry<real> *unboost;   // [p][j]: lab taps of comoving ordinate j
};

template <typename real> struct BoostArgs {
    long P;
    int K, nmu, nphi;
    FreqInfo fi;
    const double *dir, *mu;
    const RemapEntry<real> *plan;  // [p][k]
    const real *S0;             // comoving source on the ordinates [p][g][j]
    const real *Iprev;          // [k][p][g] or NULL
    real inv_cdt;
    const real *chilab;         // [k][p] (chi_grey) or [k][p][g]
    const real *chi0;           // [p][g] comoving extinction (per-group chi on log-uniform groups:
                                // chi_lab rebuilt from the plan's frequency position, chilab unread)
    int chi_grey;
    const double *beta, *gam;
    real *St;                   // [k][p][g]
};

template <typename real> struct ChiLabArgs {
    long P;
    int K;
    FreqInfo fi;
    int chi_grey;               // chi0 the same for every group: output [k][p]
    const double *dir;
    const real *chi0;           // [p][g]
    const double *beta, *gam;
    real *out;
};

template <typename real> struct UnboostArgs {
    long P;
    int K, nmu, nphi;
    FreqInfo fi;
    const double *dir, *mu;
    const RemapEntry<real> *plan;  // [p][j]
    const real *Ilab;           // [k][p][g]
    const double *beta, *gam;
    real *I0;                   // [p][g][j]
};

// Compton source tables A [nt][lmax+1][G][G] (row j, column i) at nt node
// temperatures; with nt > 1 point p interpolates linearly between nodes
// tnode[p] and tnode[p] + 1 with weight twt[p] on the upper one.
template <typename real> struct SourceArgs {
    long P;
    int G, NL, compton;
    const real *chi0, *sigma, *kappa, *bnu, *A, *Ilm;
    real *S;
    const int *tnode;           // [P] or NULL (one table)
    const real *twt;            // [P] or NULL
    const int *torder;          // [P] the points ordered by tnode (with tnode), or NULL
};

template <typename real> void launch_trace(const TraceArgs<real> &a, bool chi_array, hipStream_t st);
// lab ordinate arrays between [k][p][g] (point-major) and [k][g][p] (group-major)
template <typename real> void launch_transpose_lab(const real *in, real *out, long P, int G, int K, bool to_gmajor,
                                                   hipStream_t st);
template <typename real> void launch_boost(const BoostArgs<real> &a, hipStream_t st);
template <typename real> void launch_unboost(const UnboostArgs<real> &a, hipStream_t st);
template <typename real> size_t trace_lds(int nx, int ny, int Gc, int chi_per_point);
template <typename real> size_t boost_lds(int K, int G);
template <typename real> size_t unboost_lds(int K, int G);
template <typename real> void launch_remap_plan(const PlanArgs<real> &a, hipStream_t st);
template <typename real> void launch_chilab(const ChiLabArgs<real> &a, hipStream_t st);
// S6 on the matrix cores (FP32) for NL <= 64; false when the shape is not covered (then use a library
// product).  rt: 16-row tiles per wave (1, 2 or 4; 0 = the default for NL)
// row-major C[R][N] = A[R][Kd] B[Kd][N] on the matrix cores (FP32 or FP64), any sizes
template <typename real> void launch_gemm(long R, int Kd, int N, const real *A, const real *B, real *C, hipStream_t st);
// FP32 C[R][N] = A[R][Kd] B[Kd][N] from B's transpose Bt[N][Kd] (k contiguous) on the matrix
// cores; false (nothing queued) unless Bt is given, Kd is a multiple of 16 and N >= 16
bool launch_gemm_dma(long R, int Kd, int N, const float *A, const float *Bt, float *C, hipStream_t st);
bool launch_do2sh_f32(long R, int K, int NL, const float *A, const float *B, float *C, hipStream_t st, int rt = 0);
size_t do2sh_lds(int NL);
// mixed precision (FP16 matrix cores on hi + lo operand pairs, FP32 accumulation), NL <= 256:
// S6 with the FP16 tables WYt[NL rounded up to 16][K rounded up to 32] and S2 with the FP16
// tables Y[K rounded up to 16][NL rounded up to 32] (hi and lo parts, zero padding); false when
// the shape is not covered
bool launch_do2sh_f16(long R, int K, int NL, const float *A, const _Float16 *WYh, const _Float16 *WYl, float *C,
                      hipStream_t st, int rt = 0);
bool launch_sh2do_f16(long R, int K, int NL, const float *S, const _Float16 *Yh, const _Float16 *Yl, float *C,
                      hipStream_t st);
template <typename real> void launch_source(const SourceArgs<real> &a, hipStream_t st);
// Thomson source with the residual's per-row sums against Sold (rows[g P + p], rows[(G + g) P + p]) in the
// same pass; false (nothing launched) for Compton or NL not dividing 64
template <typename real> bool launch_source_resid(const SourceArgs<real> &a, const real *Sold, double *rows, hipStream_t st);
// rows holds 2 P G row sums followed by room for 2 G kResidSplit partial sums
constexpr int kResidSplit = 64;
template <typename real> void launch_resid_groups(long P, int G, const double *rows, double *out, hipStream_t st);
// chi0 = kappa + sigma s_g, with s [nt][G] interpolated per point as the source tables (tnode / twt NULL: node 0)
template <typename real> void launch_chi0(long P, int G, const real *kappa, const real *sigma, const real *sg,
                                          const int *tnode, const real *twt, real *chi0, hipStream_t st);
template <typename real> void launch_moments_lab(long P, int G, int K, const double *dir, const real *I, double *J, double *H, double *Kt, hipStream_t st);
void launch_moments_integrate(long P, int G, const double *dnu, const double *J, const double *H, const double *Kt,
                              double *out, hipStream_t st);
template <typename real> void launch_moments_co(long PG, int NL, int lmax, const real *Ilm, double *J, double *H, double *Kt, hipStream_t st);
template <typename real> void launch_resid(long P, int G, int NL, const real *a, const real *b, double *partial, int nblk, double *out, hipStream_t st);
// Ng dot products, each group weighted by 1/||s0_g||^2 from the residual sums red (floor2 as there)
template <typename real> void launch_ng_dots(long n, int G, int NL, const double *red, double floor2, const real *s0,
                                             const real *s1, const real *s2, const real *s3, double *partial, int nblk,
                                             double *out, hipStream_t st);
template <typename real> void launch_ng_extrapolate(long n, const double *dots, const real *s3, const real *s2,
                                                    const real *s1, real *out, hipStream_t st);
template <typename real> void launch_combine3(long n, double c0, const real *x0, double c1, const real *x1, double c2, const real *x2, real *out, hipStream_t st);
template <typename real> void launch_rk_stage(long n, const real *R, real *Iin, real *acc, real *In, int first, int last, real coef, hipStream_t st);

// variable-Eddington-tensor hand-off (FP64): one step of the closed moment equations
struct VetArgs {
    int nx, ny, nz;
    long P;
    double idx2, idy2, idz2, idz;       // 1/(2 dx), 1/(2 dy), 1/(2 dz), 1/dz
    double dt;
    const double *f;                    // Eddington tensor, SoA [6][P]: xx, yy, zz, xy, xz, yz
    const double *kap, *chi, *B;        // [P] energy exchange, flux extinction, emission
    double *J, *H, *G;                  // [P], [P][3], [P][4]: updated in place
};
void launch_vet_f(long P, const double *mom, double *f, hipStream_t st);
void launch_vet_flux(const VetArgs &a, hipStream_t st);       // H^{n+1} and the momentum exchange
void launch_vet_energy(const VetArgs &a, hipStream_t st);     // then J^{n+1} and the energy exchange
// elements of x[n] that are not finite or (check_lo) below lo, added to the device counter *count
template <typename real> void launch_count_bad(long n, const real *x, real lo, int check_lo, unsigned long long *count,
                                               hipStream_t st);

hipError_t set_lds_limits(size_t bytes);

}  // namespace rrt
