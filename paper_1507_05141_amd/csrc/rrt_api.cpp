// Host driver and C ABI of librrt (see include/rrt.h): problem set-up, device
// memory, the Lambda iteration with Ng acceleration, the four-stage implicit
// time scheme, and kernel timing.  Every step of the sweep runs in the HIP
// kernels of rrt_kernels.hip; the host only sequences them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <new>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <tuple>
#include <mutex>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "rrt.h"
#include "rrt_internal.h"
#include "rrt_kernels.h"

namespace {

thread_local std::string g_err;

rrt_status fail(rrt_status s, const std::string &m)
{
    g_err = m;
    return s;
}

#define HIPCHK(call)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(RRT_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));  \
    } while (0)

enum KId { KI_TRACE, KI_SH2DO, KI_BOOST, KI_UNBOOST, KI_DO2SH, KI_SOURCE, KI_REDUCE, KI_MOMENTS, KI_RK, KI_VET_FLUX, KI_VET_ENERGY, KI_N };
const char *kNames[KI_N] = {"trace", "sh2do", "boost", "unboost", "do2sh", "source", "reduce", "moments", "rk", "vet_flux", "vet_energy"};

constexpr double kPi = 3.14159265358979323846;
constexpr size_t kMaxLds = 160 * 1024;
constexpr double kResidualFloor = 1e-20;    // of the largest group's source norm
constexpr size_t kMaxGraphs = 16;           // captured sweeps kept per problem
// kernel variants chosen by timing, per problem shape: (groups per trace workgroup, S6 variant)
std::mutex g_tune_mu;
std::map<std::string, std::pair<int, int>> g_tuned;

}  // namespace

struct rrt_problem {
    // sizes
    int nx = 0, ny = 0, nz = 0;
    double lx = 0, ly = 0, lz = 0;
    long P = 0;
    int G = 1, grey = 1, log_centres = 1;
    double mec2 = 0;
    int lmax = 0, NL = 0, nmu = 0, nphi = 0, K = 0;
    rrt_scatter scatter = RRT_THOMSON;
    rrt_precision prec = RRT_FP32;
    size_t esz = 4;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // host tables
    std::vector<double> mu, wmu, edges, centres, Y, dir;
    // Compton tables (FP64 host copies) at the temperature nodes kT_nodes (units of
    // the edges; the single node 0 is the paper's electrons at rest): kn_s [nt][G],
    // kn_A [nt][lmax+1][G][G] (row j, column i)
    std::vector<double> kn_s, kn_A;
    std::vector<double> kT_nodes;
    std::vector<double> lt_nodes;                   // log10 of kT_nodes (temperature field set)
    int *d_tnode = nullptr;                         // per point: lower temperature node
    int *d_torder = nullptr;                        // the points ordered by their lower node
    void *d_twt = nullptr;                          // per point: weight of the upper node
    size_t tab_bytes = 0;                           // bytes of d_A + d_sg
    size_t temp_bytes = 0;                          // bytes of d_tnode + d_twt
    // device tables
    double *d_dir = nullptr, *d_mu = nullptr, *d_lnc = nullptr, *d_nu3 = nullptr, *d_inv_nu3 = nullptr,
           *d_inv_dc = nullptr;
    int Gc = 1;
    int Gc_max = 1;                                 // the most groups per trace workgroup the LDS holds
    rrt::OrdGeom *d_geo = nullptr;
    void *d_taps = nullptr;                         // rrt::PathTap<real> of every ordinate's path points
    int *d_order = nullptr;                         // ordinates by decreasing number of path pieces
    int nmulti = 0;                                 // ordinates whose path takes more than one piece
    void *d_Yt = nullptr, *d_WY = nullptr, *d_A = nullptr, *d_sg = nullptr;
    void *d_Y = nullptr, *d_WYt = nullptr;          // RRT_FP32: the SH tables transposed (the products' k contiguous)
    void *d_Y16 = nullptr, *d_WYt16 = nullptr;     // RRT_MIXED: FP16 SH tables, hi then lo part (zero padded)
    size_t y16_n = 0, wyt16_n = 0;                  // elements per part
    rrt::FreqInfo fi{};
    // fields
    void *d_kappa = nullptr, *d_sigma = nullptr, *d_bnu = nullptr, *d_chi0 = nullptr;
    double *d_beta = nullptr, *d_gam = nullptr;
    void *d_chilab = nullptr;
    void *d_plan = nullptr;                         // remap entries: [p][k] boost, then [p][j] inverse
    void *d_chilabT = nullptr;                      // per-group lab extinction on group-major planes [k][g][p]
    bool gmajor = false;                            // trace on group-major planes (one group per workgroup)
    int grey_chi = 0;
    void *d_bc[2] = {nullptr, nullptr};
    // state and work arrays
    void *d_S = nullptr, *d_Snew = nullptr, *d_Ilm = nullptr;
    void *d_co = nullptr, *d_St = nullptr, *d_Xt = nullptr, *d_Ilab = nullptr, *d_I = nullptr;
    void *d_Iin = nullptr, *d_acc = nullptr;
    void *d_chain[4] = {nullptr, nullptr, nullptr, nullptr};
    double *d_partial = nullptr, *d_red = nullptr;
    unsigned long long *d_count = nullptr;          // counter of invalid elements in borrowed device arrays
    double *d_vet = nullptr;                        // VET hand-off: f [6][P], then kappa, chi, B, J, H [3], G [4] per point
    double *d_mom = nullptr;                        // moments: J, H, K per group, then per point J, H, K, f integrated
    double *d_dnu = nullptr;                        // group widths (1 for a grey group)
    double *h_red = nullptr;                        // pinned host copy of the per-group residual sums
    int nblk_red = 0;
    bool medium_set = false;
    size_t dev_bytes = 0;                           // device memory held by the problem
    // a Lambda iteration in progress: one sweep per round, Ng every fourth chain member
    struct Solve {
        const void *Iprev = nullptr;
        double inv_cdt = 0, tol = 0, r = INFINITY;
        int max_iter = 0, use_ng = 0, it = 0, clen = 0;
        int phase = 0;                              // 0 idle, 1 running, 2 finished
        rrt_status st = RRT_OK;
        std::chrono::steady_clock::time_point t0;
        double seconds = 0;                         // begin to finish
    } sv;
    rrt_batch *batch = nullptr;
    // sweeps captured as HIP graphs, keyed by the source buffer (the two SH
    // buffers alternate), the stage input and 1/(c dt); a key is captured the
    // first time it recurs after two eager sweeps
    struct Captured {
        const void *S, *Iprev;
        double inv_cdt;
        hipGraphExec_t exec;
    };
    std::vector<Captured> graphs;
    bool use_graphs = true;
    bool graphs_failed = false;                     // capture or instantiation refused: eager from then on
    int eager_sweeps = 0;
    // kernel variants: groups per ray-trace workgroup (Gc above) and the S6 product
    // (-1 the default for the shape, 0 the library product, 1/2/4 the matrix-core
    // kernel with that many 16-row tiles per wave); autotuned at the second sweep
    int s6 = -1;
    bool autotune = true, tuned = false;
    bool gc_forced = false;                         // groups per workgroup fixed by the environment
    bool variants_fixed = false;                    // fixed by rrt_set_variants
    size_t lds_lim = 0;
    // kernel timing
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[KI_N];
    std::vector<hipEvent_t> pool;
    double ms[KI_N] = {0};
    int calls[KI_N] = {0};
};

namespace {

size_t sh_elems(const rrt_problem *p) { return (size_t)p->P * p->G * p->NL; }
size_t do_elems(const rrt_problem *p) { return (size_t)p->P * p->G * p->K; }

// Process-wide pool of device blocks that destroyed problems freed (rrt_set_device_pool):
// blocks wait, per (device, size), for a later allocation of the same size.
struct DevPool {
    std::mutex mu;
    size_t max_bytes = 0, held = 0;
    std::map<std::pair<int, size_t>, std::vector<void *>> free;   // (device, bytes) -> blocks
    std::vector<std::tuple<int, size_t, void *>> order;            // pooled blocks, oldest first
    std::map<void *, std::pair<int, size_t>> sizes;                // every block dev_alloc made
};
DevPool &dev_pool()
{
    static DevPool p;
    return p;
}
// take the pooled blocks beyond `keep` bytes (oldest first) out of the pool; the caller frees them
std::vector<void *> pool_take_excess(DevPool &dp, size_t keep)
{
    std::vector<void *> out;
    size_t i = 0;
    for (; i < dp.order.size() && dp.held > keep; ++i) {
        const auto &t = dp.order[i];
        auto &v = dp.free[{std::get<0>(t), std::get<1>(t)}];
        auto it = std::find(v.begin(), v.end(), std::get<2>(t));
        if (it == v.end()) continue;                // already reused
        v.erase(it);
        dp.held -= std::get<1>(t);
        dp.sizes.erase(std::get<2>(t));
        out.push_back(std::get<2>(t));
    }
    dp.order.erase(dp.order.begin(), dp.order.begin() + i);
    return out;
}

rrt_status dev_alloc(void **ptr, size_t bytes)
{
    if (*ptr) return RRT_OK;
    bytes = bytes ? bytes : 1;
    int dev = 0;
    (void)hipGetDevice(&dev);
    DevPool &dp = dev_pool();
    {
        std::lock_guard<std::mutex> lk(dp.mu);
        auto it = dp.free.find({dev, bytes});
        if (it != dp.free.end() && !it->second.empty()) {
            *ptr = it->second.back();
            it->second.pop_back();
            dp.held -= bytes;
            return RRT_OK;
        }
    }
    hipError_t e = hipMalloc(ptr, bytes);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        // the pool may hold what this allocation needs: empty it and try once more
        (void)hipGetLastError();
        std::vector<void *> out;
        {
            std::lock_guard<std::mutex> lk(dp.mu);
            out = pool_take_excess(dp, 0);
        }
        for (void *b : out) (void)hipFree(b);
        if (!out.empty()) e = hipMalloc(ptr, bytes);
    }
    if (e != hipSuccess) {
        *ptr = nullptr;
        return fail(RRT_E_HBM, std::string("hipMalloc of ") + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
    }
    std::lock_guard<std::mutex> lk(dp.mu);
    dp.sizes[*ptr] = {dev, bytes};
    return RRT_OK;
}

// a block whose users have all finished (its problem's stream is idle): into the pool
// while it has room, else freed
void dev_release(void *p)
{
    if (!p) return;
    DevPool &dp = dev_pool();
    std::vector<void *> out;
    {
        std::lock_guard<std::mutex> lk(dp.mu);
        auto it = dp.sizes.find(p);
        if (it != dp.sizes.end() && dp.max_bytes > 0 && it->second.second <= dp.max_bytes) {
            dp.free[it->second].push_back(p);
            dp.order.emplace_back(it->second.first, it->second.second, p);
            dp.held += it->second.second;
            out = pool_take_excess(dp, dp.max_bytes);
            p = nullptr;
        } else if (it != dp.sizes.end()) {
            dp.sizes.erase(it);
        }
    }
    if (p) (void)hipFree(p);
    for (void *b : out) (void)hipFree(b);
}

void dev_free(void *&p)
{
    if (p) {
        {
            DevPool &dp = dev_pool();
            std::lock_guard<std::mutex> lk(dp.mu);
            dp.sizes.erase(p);
        }
        (void)hipFree(p);
    }
    p = nullptr;
}

// allocation owned by the problem (counted in dev_bytes)
rrt_status pr_alloc(rrt_problem *pr, void **ptr, size_t bytes)
{
    if (*ptr) return RRT_OK;
    rrt_status s = dev_alloc(ptr, bytes);
    if (!s) pr->dev_bytes += bytes ? bytes : 1;
    return s;
}

// upload host doubles converted to the working precision
rrt_status upload_real(rrt_problem *pr, void *dst, const double *src, size_t n)
{
    if (pr->prec == RRT_FP64) {
        HIPCHK(hipMemcpyAsync(dst, src, n * 8, hipMemcpyHostToDevice, pr->stream));
        HIPCHK(hipStreamSynchronize(pr->stream));
        return RRT_OK;
    }
    std::vector<float> tmp(n);
    for (size_t i = 0; i < n; ++i) tmp[i] = (float)src[i];
    HIPCHK(hipMemcpyAsync(dst, tmp.data(), n * 4, hipMemcpyHostToDevice, pr->stream));
    HIPCHK(hipStreamSynchronize(pr->stream));
    return RRT_OK;
}

rrt_status download_real(rrt_problem *pr, double *dst, const void *src, size_t n)
{
    if (pr->prec == RRT_FP64) {
        HIPCHK(hipMemcpyAsync(dst, src, n * 8, hipMemcpyDeviceToHost, pr->stream));
        HIPCHK(hipStreamSynchronize(pr->stream));
        return RRT_OK;
    }
    std::vector<float> tmp(n);
    HIPCHK(hipMemcpyAsync(tmp.data(), src, n * 4, hipMemcpyDeviceToHost, pr->stream));
    HIPCHK(hipStreamSynchronize(pr->stream));
    for (size_t i = 0; i < n; ++i) dst[i] = tmp[i];
    return RRT_OK;
}

rrt_status upload_double(rrt_problem *pr, void **dst, const std::vector<double> &v)
{
    rrt_status s = pr_alloc(pr, dst, v.size() * 8);
    if (s) return s;
    HIPCHK(hipMemcpyAsync(*dst, v.data(), v.size() * 8, hipMemcpyHostToDevice, pr->stream));
    HIPCHK(hipStreamSynchronize(pr->stream));
    return RRT_OK;
}

rrt_status alloc_upload_real(rrt_problem *pr, void **dst, const std::vector<double> &v)
{
    rrt_status s = pr_alloc(pr, dst, v.size() * pr->esz);
    if (s) return s;
    return upload_real(pr, *dst, v.data(), v.size());
}

// a caller's pointer that device code may read: device (or managed) memory
rrt_status check_dev_ptr(const void *p, const char *what)
{
    if (!p) return fail(RRT_E_INVALID, std::string(what) + " is NULL");
    hipPointerAttribute_t at{};
    const hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(RRT_E_INVALID, std::string(what) + " is not device memory");
    }
    if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
        return fail(RRT_E_INVALID, std::string(what) + " is not device memory");
    return RRT_OK;
}

// copy between the caller's device memory and the problem's, on the problem's stream;
// returns once the copy is complete (the caller's buffer is borrowed for the call only)
rrt_status copy_dev(rrt_problem *pr, void *dst, const void *src, size_t bytes)
{
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, pr->stream));
    HIPCHK(hipStreamSynchronize(pr->stream));
    return RRT_OK;
}

// elements of a device array (FP64 when fp64, else the working precision) that are not finite
// or (check_lo) below lo
rrt_status count_bad_dev(rrt_problem *pr, const void *x, size_t n, double lo, bool check_lo, unsigned long long *bad,
                         bool fp64 = false)
{
    rrt_status s = pr_alloc(pr, (void **)&pr->d_count, sizeof(unsigned long long));
    if (s) return s;
    HIPCHK(hipMemsetAsync(pr->d_count, 0, sizeof(unsigned long long), pr->stream));
    if (fp64 || pr->prec == RRT_FP64)
        rrt::launch_count_bad<double>((long)n, (const double *)x, lo, check_lo, pr->d_count, pr->stream);
    else
        rrt::launch_count_bad<float>((long)n, (const float *)x, (float)lo, check_lo, pr->d_count, pr->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(bad, pr->d_count, sizeof(unsigned long long), hipMemcpyDeviceToHost, pr->stream));
    HIPCHK(hipStreamSynchronize(pr->stream));
    return RRT_OK;
}

// the caller's device copy of a host-side argument array (doubles), read back for a set-up call
rrt_status read_back(const double *src, size_t n, std::vector<double> &dst)
{
    dst.resize(n);
    HIPCHK(hipMemcpy(dst.data(), src, n * 8, hipMemcpyDeviceToHost));
    return RRT_OK;
}

// drop the captured sweeps (their buffers or kernel choices are about to change)
void clear_graphs(rrt_problem *pr)
{
    if (!pr->graphs.empty() && pr->stream) (void)hipStreamSynchronize(pr->stream);
    for (auto &g : pr->graphs) (void)hipGraphExecDestroy(g.exec);
    pr->graphs.clear();
    pr->eager_sweeps = 0;
}

// --- kernel timing ---------------------------------------------------------
void prof_begin(rrt_problem *pr, int id)
{
    if (!pr->prof) return;
    hipEvent_t a, b;
    if (pr->pool.size() >= 2) {
        a = pr->pool.back(); pr->pool.pop_back();
        b = pr->pool.back(); pr->pool.pop_back();
    } else {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    (void)hipEventRecord(a, pr->stream);
    pr->pending[id].push_back({a, b});
}

void prof_end(rrt_problem *pr, int id)
{
    if (!pr->prof) return;
    (void)hipEventRecord(pr->pending[id].back().second, pr->stream);
}

void prof_collect(rrt_problem *pr)
{
    (void)hipStreamSynchronize(pr->stream);
    for (int i = 0; i < KI_N; ++i) {
        for (auto &e : pr->pending[i]) {
            float t = 0;
            if (hipEventElapsedTime(&t, e.first, e.second) == hipSuccess) {
                pr->ms[i] += t;
                pr->calls[i] += 1;
            }
            pr->pool.push_back(e.first);
            pr->pool.push_back(e.second);
        }
        pr->pending[i].clear();
    }
}

// ---------------------------------------------------------------------------
// the sweep, templated on the working precision
// ---------------------------------------------------------------------------
template <typename real>
struct Engine {
    rrt_problem *pr;

    real *R(void *p) const { return static_cast<real *>(p); }

    rrt_status check_launch()
    {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(RRT_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
        return RRT_OK;
    }

    // row-major C[M][N] = A[M][Kd] . B[Kd][N] on the matrix cores (the library's panel kernel)
    rrt_status gemm(long M, int N, int Kd, const real *A, const real *Bm, real *C, const void *Bt = nullptr)
    {
        if (sizeof(real) == 4 && Kd > 64 &&
            rrt::launch_gemm_dma(M, Kd, N, (const float *)A, (const float *)Bt, (float *)C, pr->stream))
            return check_launch();
        rrt::launch_gemm<real>(M, Kd, N, A, Bm, C, pr->stream);
        return check_launch();
    }

    // S2 + S3: comoving SH source -> comoving ordinates -> lab S~ (with the implicit time terms)
    rrt_status to_lab(const void *S, const void *Iprev, double inv_cdt)
    {
        prof_begin(pr, KI_SH2DO);
        rrt_status s;
        const _Float16 *y16 = (const _Float16 *)pr->d_Y16;
        if (pr->prec == RRT_MIXED && rrt::launch_sh2do_f16(pr->P * pr->G, pr->K, pr->NL, (const float *)S, y16,
                                                           y16 + pr->y16_n, (float *)pr->d_co, pr->stream))
            s = check_launch();
        else
            s = gemm(pr->P * pr->G, pr->K, pr->NL, static_cast<const real *>(S), R(pr->d_Yt), R(pr->d_co), pr->d_Y);
        prof_end(pr, KI_SH2DO);
        if (s) return s;
        rrt::BoostArgs<real> b;
        b.P = pr->P; b.K = pr->K; b.nmu = pr->nmu; b.nphi = pr->nphi; b.fi = pr->fi;
        b.dir = pr->d_dir; b.mu = pr->d_mu; b.plan = plan(0); b.S0 = R(pr->d_co); b.Iprev = static_cast<const real *>(Iprev);
        b.inv_cdt = (real)inv_cdt; b.chilab = R(pr->d_chilab); b.chi0 = R(pr->d_chi0); b.chi_grey = pr->grey_chi;
        b.beta = pr->d_beta; b.gam = pr->d_gam; b.St = R(pr->d_St);
        prof_begin(pr, KI_BOOST);
        rrt::launch_boost<real>(b, pr->stream);
        prof_end(pr, KI_BOOST);
        return check_launch();
    }

    // remap entries of the boost (0) or of the inverse map (1)
    const rrt::RemapEntry<real> *plan(int which) const
    {
        const auto *e = static_cast<const rrt::RemapEntry<real> *>(pr->d_plan);
        return e ? e + (size_t)which * pr->P * pr->K : nullptr;
    }

    // S4 (chi~ from the medium, or from d_Xt when chi_array)
    void trace(const void *St, void *I, double inv_cdt, bool chi_array)
    {
        prof_begin(pr, KI_TRACE);
        trace_launch(St, I, inv_cdt, chi_array, false);
        prof_end(pr, KI_TRACE);
    }
    void trace_launch(const void *St, void *I, double inv_cdt, bool chi_array, bool gmajor)
    {
        rrt::TraceArgs<real> t;
        t.nx = pr->nx; t.ny = pr->ny; t.nz = pr->nz; t.G = pr->G; t.K = pr->K; t.Gc = gmajor ? 1 : pr->Gc; t.P = pr->P;
        t.geo = pr->d_geo; t.taps = static_cast<const rrt::PathTap<real> *>(pr->d_taps); t.order = pr->d_order; t.nmulti = pr->nmulti;
        t.dir = pr->d_dir; t.St = static_cast<const real *>(St); t.Xt = R(pr->d_Xt);
        t.chilab = R(gmajor && !pr->grey_chi ? pr->d_chilabT : pr->d_chilab); t.chi_grey = pr->grey_chi;
        t.inv_cdt = (real)inv_cdt; t.bc_bot = R(pr->d_bc[0]); t.bc_top = R(pr->d_bc[1]); t.I = R(I);
        t.gmajor = gmajor;
        rrt::launch_trace<real>(t, chi_array, pr->stream);
    }
    // S4 on group-major planes: S~ (in d_St) is transposed into d_Ilab, traced into d_St,
    // and the intensity transposed back into d_Ilab (both transposes timed with the trace)
    void trace_gmajor_launch(double inv_cdt)
    {
        rrt::launch_transpose_lab<real>(R(pr->d_St), R(pr->d_Ilab), pr->P, pr->G, pr->K, true, pr->stream);
        trace_launch(pr->d_Ilab, pr->d_St, inv_cdt, false, true);
        rrt::launch_transpose_lab<real>(R(pr->d_St), R(pr->d_Ilab), pr->P, pr->G, pr->K, false, pr->stream);
    }
    bool gmajor_ready() const { return pr->G > 1 && (pr->grey_chi || pr->d_chilabT); }

    // S5 + S6: lab intensity -> comoving ordinates -> comoving SH intensity (into d_Ilm)
    rrt_status fold(const void *Ilab)
    {
        rrt::UnboostArgs<real> u;
        u.P = pr->P; u.K = pr->K; u.nmu = pr->nmu; u.nphi = pr->nphi; u.fi = pr->fi;
        u.dir = pr->d_dir; u.mu = pr->d_mu; u.plan = plan(1); u.Ilab = static_cast<const real *>(Ilab);
        u.beta = pr->d_beta; u.gam = pr->d_gam; u.I0 = R(pr->d_co);
        prof_begin(pr, KI_UNBOOST);
        rrt::launch_unboost<real>(u, pr->stream);
        prof_end(pr, KI_UNBOOST);
        rrt_status s = check_launch();
        if (s) return s;
        prof_begin(pr, KI_DO2SH);
        s = do2sh(pr->s6);
        prof_end(pr, KI_DO2SH);
        return s;
    }
    // S6 with variant v (as rrt_problem::s6)
    rrt_status do2sh(int v)
    {
        const int rt = v > 0 ? v : 0;
        const _Float16 *wy16 = (const _Float16 *)pr->d_WYt16;
        if (pr->prec == RRT_MIXED && rrt::launch_do2sh_f16(pr->P * pr->G, pr->K, pr->NL, (const float *)pr->d_co, wy16,
                                                           wy16 + pr->wyt16_n, (float *)pr->d_Ilm, pr->stream, rt))
            return check_launch();
        if (sizeof(real) == 4 && pr->prec != RRT_MIXED && v != 0 &&
            rrt::launch_do2sh_f32(pr->P * pr->G, pr->K, pr->NL, (const float *)pr->d_co, (const float *)pr->d_WY,
                                  (float *)pr->d_Ilm, pr->stream, rt))
            return check_launch();
        return gemm(pr->P * pr->G, pr->NL, pr->K, R(pr->d_co), R(pr->d_WY), R(pr->d_Ilm), pr->d_WYt);
    }

    // --- autotuning of the kernel variants ---------------------------------
    // Candidates are timed on the problem's own buffers at the start of its second
    // sweep (the first sweep has filled them); the choice is kept per shape for the
    // process, so later problems of the same shape take it without timing.
    std::string tune_key(double inv_cdt) const
    {
        char b[256];
        std::snprintf(b, sizeof b, "%d %d %d %d %d %d %d %d %d %d", pr->nx, pr->ny, pr->nz, pr->G, pr->K, pr->NL,
                      (int)pr->prec, pr->grey_chi, inv_cdt != 0.0, (int)pr->scatter);
        return b;
    }
    // average time (ms) of n launches of f after one untimed launch
    template <class F> float time_ms(F f, int n = 2)
    {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return INFINITY;
        if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return INFINITY; }
        f();
        (void)hipEventRecord(a, pr->stream);
        for (int i = 0; i < n; ++i) f();
        (void)hipEventRecord(b, pr->stream);
        float t = INFINITY;
        if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&t, a, b) != hipSuccess) t = INFINITY;
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return t / n;
    }
    std::vector<int> gc_candidates() const
    {
        std::vector<int> c;
        for (int gc = 4; gc >= 1; gc /= 2) {
            const size_t need = pr->prec == RRT_FP64 ? rrt::trace_lds<double>(pr->nx, pr->ny, gc, 0)
                                                     : rrt::trace_lds<float>(pr->nx, pr->ny, gc, 0);
            if (pr->G % gc == 0 && need <= pr->lds_lim) c.push_back(gc);
        }
        return c;
    }
    std::vector<int> s6_candidates() const
    {
        std::vector<int> c;
        if (pr->prec == RRT_FP64) return c;
        if (pr->NL <= 64) c = {1, 2, 4};
        if (pr->prec == RRT_FP32) c.push_back(0);
        return c;
    }
    rrt_status autotune(double inv_cdt)
    {
        pr->tuned = true;
        const std::string key = tune_key(inv_cdt);
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tuned.find(key);
            if (it != g_tuned.end()) {
                if (!pr->gc_forced) {
                    pr->Gc = it->second.first & 7;
                    pr->gmajor = (it->second.first >> 3) && gmajor_ready();
                    if (pr->gmajor) pr->Gc = 1;
                }
                pr->s6 = it->second.second;
                return RRT_OK;
            }
        }
        const bool try_gm = gmajor_ready() && !pr->gc_forced;
        if (!pr->gc_forced && (gc_candidates().size() > 1 || try_gm)) {
            const auto c = gc_candidates();
            float best = INFINITY;
            int pick = pr->Gc;
            bool pick_gm = false;
            for (int gc : c) {
                pr->Gc = gc;
                const float t = time_ms([&] { trace_launch(pr->d_St, pr->d_Ilab, inv_cdt, false, false); });
                if (t < best) { best = t; pick = gc; }
            }
            if (try_gm) {
                // group-major planes with both transposes (d_St and d_Ilab hold scratch afterwards: the
                // sweep about to run recomputes both)
                const float t = time_ms([&] { trace_gmajor_launch(inv_cdt); });
                if (t < best) { best = t; pick = 1; pick_gm = true; }
            }
            pr->Gc = pick;
            pr->gmajor = pick_gm;
        }
        if (s6_candidates().size() > 1) {
            const auto c = s6_candidates();
            float best = INFINITY;
            int pick = pr->s6;
            for (int v : c) {
                const float t = time_ms([&] { (void)do2sh(v); });
                if (t < best) { best = t; pick = v; }
            }
            pr->s6 = pick;
        }
        rrt_status s = check_launch();
        if (s) return s;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[key] = {pr->Gc + (pr->gmajor ? 8 : 0), pr->s6};
        return RRT_OK;
    }

    // S1: source from d_Ilm into S; with Sold, the residual's row sums against it in the
    // same pass where the kernel allows (returns whether it did)
    bool source(void *S, const void *Sold = nullptr)
    {
        rrt::SourceArgs<real> s;
        s.P = pr->P; s.G = pr->G; s.NL = pr->NL; s.compton = pr->scatter == RRT_COMPTON;
        s.chi0 = R(pr->d_chi0); s.sigma = R(pr->d_sigma); s.kappa = R(pr->d_kappa); s.bnu = R(pr->d_bnu);
        s.A = R(pr->d_A); s.Ilm = R(pr->d_Ilm); s.S = R(S);
        s.tnode = pr->d_tnode; s.twt = R(pr->d_twt); s.torder = pr->d_torder;
        prof_begin(pr, KI_SOURCE);
        const bool fused = Sold && rrt::launch_source_resid<real>(s, static_cast<const real *>(Sold), pr->d_partial,
                                                                  pr->stream);
        if (!fused) rrt::launch_source<real>(s, pr->stream);
        prof_end(pr, KI_SOURCE);
        return fused;
    }

    // S8: max over groups of ||a - b|| / ||a||
    // S8, queued: per-group sums into the pinned host buffer (read after the stream is synchronized)
    // rows_ready: the per-row sums are already in d_partial (fused into the source step)
    rrt_status residual_launch(const void *a, const void *b, bool rows_ready = false)
    {
        prof_begin(pr, KI_REDUCE);
        if (rows_ready)
            rrt::launch_resid_groups<real>(pr->P, pr->G, pr->d_partial, pr->d_red, pr->stream);
        else
            rrt::launch_resid<real>(pr->P, pr->G, pr->NL, static_cast<const real *>(a), static_cast<const real *>(b),
                                    pr->d_partial, pr->nblk_red, pr->d_red, pr->stream);
        prof_end(pr, KI_REDUCE);
        rrt_status s = check_launch();
        if (s) return s;
        HIPCHK(hipMemcpyAsync(pr->h_red, pr->d_red, 2 * (size_t)pr->G * 8, hipMemcpyDeviceToHost, pr->stream));
        return RRT_OK;
    }
    // max over groups of ||a - b|| / ||a|| from the downloaded sums, a group's norm floored
    // at kResidualFloor of the largest group's (relative changes that far down the
    // spectrum carry no weight and are not resolved in single precision)
    double residual_value() const
    {
        double amax = 0.0;
        for (int g = 0; g < pr->G; ++g) amax = std::fmax(amax, pr->h_red[2 * g + 1]);
        const double floor2 = kResidualFloor * kResidualFloor * amax;
        double m = 0.0;
        for (int g = 0; g < pr->G; ++g) {
            const double dd = pr->h_red[2 * g], aa = std::fmax(pr->h_red[2 * g + 1], floor2);
            const double rg = (aa > 0.0) ? std::sqrt(dd / aa) : (dd > 0.0 ? INFINITY : 0.0);
            if (!(rg <= m)) m = rg;
        }
        return m;
    }
    rrt_status residual(const void *a, const void *b, double *r)
    {
        rrt_status s = residual_launch(a, b);
        if (s) return s;
        HIPCHK(hipStreamSynchronize(pr->stream));
        *r = residual_value();
        return RRT_OK;
    }

    // one source iteration from d_S (Iprev/inv_cdt: implicit time terms), queued on the
    // stream; the residual sums arrive in h_red.  Once a (source buffer, stage input,
    // 1/(c dt)) key has run eagerly, later sweeps with that key replay a captured graph.
    rrt_status sweep_launch(const void *Iprev, double inv_cdt)
    {
        const bool graphs = pr->use_graphs && !pr->graphs_failed && !pr->prof;
        if (graphs) {
            for (const auto &g : pr->graphs)
                if (g.S == pr->d_S && g.Iprev == Iprev && g.inv_cdt == inv_cdt) {
                    HIPCHK(hipGraphLaunch(g.exec, pr->stream));
                    std::swap(pr->d_S, pr->d_Snew);
                    return RRT_OK;
                }
            if (pr->eager_sweeps >= 2 && pr->graphs.size() < kMaxGraphs) {
                rrt_status s = capture_sweep(Iprev, inv_cdt);
                if (s != RRT_E_STATE) return s;
            }
        }
        if (pr->eager_sweeps == 1 && pr->autotune && !pr->tuned) {
            rrt_status s = autotune(inv_cdt);
            if (s) return s;
        }
        ++pr->eager_sweeps;
        return sweep_queue(Iprev, inv_cdt);
    }
    // capture one sweep into a graph and launch it; RRT_E_STATE when the runtime
    // refuses (nothing queued then: the caller runs the sweep eagerly)
    rrt_status capture_sweep(const void *Iprev, double inv_cdt)
    {
        const void *S0 = pr->d_S;
        auto refuse = [&]() {
            (void)hipGetLastError();
            if (pr->d_S != S0) std::swap(pr->d_S, pr->d_Snew);
            pr->graphs_failed = true;
            return RRT_E_STATE;
        };
        if (hipStreamBeginCapture(pr->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return refuse();
        rrt_status s = sweep_queue(Iprev, inv_cdt);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(pr->stream, &graph);
        if (s || e != hipSuccess || !graph) {
            if (graph) (void)hipGraphDestroy(graph);
            return refuse();
        }
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess || !exec) return refuse();
        pr->graphs.push_back({S0, Iprev, inv_cdt, exec});
        HIPCHK(hipGraphLaunch(exec, pr->stream));
        return RRT_OK;
    }
    rrt_status sweep_queue(const void *Iprev, double inv_cdt)
    {
        rrt_status s = to_lab(pr->d_S, Iprev, inv_cdt);
        if (s) return s;
        if (pr->gmajor) {
            prof_begin(pr, KI_TRACE);
            trace_gmajor_launch(inv_cdt);
            prof_end(pr, KI_TRACE);
        } else {
            trace(pr->d_St, pr->d_Ilab, inv_cdt, false);
        }
        if ((s = fold(pr->d_Ilab))) return s;
        const bool fused = source(pr->d_Snew, pr->d_S);
        if ((s = check_launch())) return s;
        s = residual_launch(pr->d_Snew, pr->d_S, fused);
        if (s) return s;
        std::swap(pr->d_S, pr->d_Snew);
        return RRT_OK;
    }
    rrt_status sweep(const void *Iprev, double inv_cdt, double *resid)
    {
        rrt_status s = sweep_launch(Iprev, inv_cdt);
        if (s) return s;
        HIPCHK(hipStreamSynchronize(pr->stream));
        *resid = residual_value();
        return RRT_OK;
    }

    // initial source: S = source(fold(I)) (thermal only when I = 0)
    rrt_status initial_source(const void *I)
    {
        rrt_status s = fold(I);
        if (s) return s;
        source(pr->d_S);
        return check_launch();
    }

    // Ng extrapolation of the chain (chain[3] newest) into d_S, queued (coefficients on the device);
    // the dot products weight each group by the inverse square of its norm in chain[3]
    rrt_status ng_step()
    {
        const size_t n = sh_elems(pr);
        prof_begin(pr, KI_REDUCE);
        // d_red still holds the last residual's per-group sums, ||chain[3]_g||^2 among them
        rrt::launch_ng_dots<real>((long)n, pr->G, pr->NL, pr->d_red, kResidualFloor * kResidualFloor,
                                  R(pr->d_chain[3]), R(pr->d_chain[2]), R(pr->d_chain[1]), R(pr->d_chain[0]),
                                  pr->d_partial, pr->nblk_red, pr->d_red, pr->stream);
        rrt::launch_ng_extrapolate<real>((long)n, pr->d_red, R(pr->d_chain[3]), R(pr->d_chain[2]), R(pr->d_chain[1]),
                                         R(pr->d_S), pr->stream);
        prof_end(pr, KI_REDUCE);
        return check_launch();
    }

    // Lambda iteration in rounds: solve_begin queues the initial source; each round
    // queues one sweep (round_launch) and, once the stream has been synchronized,
    // reads its residual and queues the Ng bookkeeping (round_finish).  The lab
    // intensity of the last sweep is left in d_Ilab.
    rrt_status solve_begin(const void *Iprev, double inv_cdt, const void *Iinit, double tol, int max_iter, int use_ng)
    {
        auto &v = pr->sv;
        v = rrt_problem::Solve{};
        v.Iprev = Iprev; v.inv_cdt = inv_cdt; v.tol = tol; v.max_iter = max_iter; v.use_ng = use_ng;
        v.t0 = std::chrono::steady_clock::now();
        const size_t shb = sh_elems(pr) * pr->esz;
        rrt_status s = initial_source(Iinit);
        if (s) return s;
        if (use_ng) {
            for (int c = 0; c < 4; ++c)
                if ((s = pr_alloc(pr, &pr->d_chain[c], shb))) return s;
            HIPCHK(hipMemcpyAsync(pr->d_chain[0], pr->d_S, shb, hipMemcpyDeviceToDevice, pr->stream));
            v.clen = 1;
        }
        v.phase = 1;
        return RRT_OK;
    }
    rrt_status round_launch()
    {
        ++pr->sv.it;
        return sweep_launch(pr->sv.Iprev, pr->sv.inv_cdt);
    }
    rrt_status round_finish()
    {
        auto &v = pr->sv;
        v.r = residual_value();
        if (v.r < v.tol) {
            v.phase = 2;
            v.st = RRT_OK;
            return RRT_OK;
        }
        if (v.use_ng) {
            const size_t shb = sh_elems(pr) * pr->esz;
            HIPCHK(hipMemcpyAsync(pr->d_chain[v.clen], pr->d_S, shb, hipMemcpyDeviceToDevice, pr->stream));
            if (++v.clen == 4) {
                rrt_status s = ng_step();
                if (s) return s;
                HIPCHK(hipMemcpyAsync(pr->d_chain[0], pr->d_S, shb, hipMemcpyDeviceToDevice, pr->stream));
                v.clen = 1;
            }
        }
        if (v.it >= v.max_iter) {
            v.phase = 2;
            v.st = RRT_E_NOT_CONVERGED;
        }
        return RRT_OK;
    }
    rrt_status solve(const void *Iprev, double inv_cdt, const void *Iinit, double tol, int max_iter, int use_ng,
                     int *iters, double *res)
    {
        rrt_status s = solve_begin(Iprev, inv_cdt, Iinit, tol, max_iter, use_ng);
        while (!s && pr->sv.phase == 1) {
            if ((s = round_launch())) break;
            if (hipStreamSynchronize(pr->stream) != hipSuccess) {
                s = fail(RRT_E_DEVICE, "stream synchronize");
                break;
            }
            s = round_finish();
        }
        pr->sv.phase = 0;
        *iters = pr->sv.it;
        *res = pr->sv.r;
        return s ? s : pr->sv.st;
    }

    // moments of the lab intensity state or the comoving SH intensity into the problem's
    // moment buffer (per group J, H, K, then the frequency-integrated ones)
    rrt_status moments_launch(rrt_frame frame)
    {
        const size_t pg = (size_t)pr->P * pr->G;
        double *dJ = pr->d_mom, *dH = dJ + pg, *dK = dH + 3 * pg;
        prof_begin(pr, KI_MOMENTS);
        if (frame == RRT_FRAME_LAB)
            rrt::launch_moments_lab<real>(pr->P, pr->G, pr->K, pr->d_dir, R(pr->d_I), dJ, dH, dK, pr->stream);
        else
            rrt::launch_moments_co<real>((long)pg, pr->NL, pr->lmax, R(pr->d_Ilm), dJ, dH, dK, pr->stream);
        rrt::launch_moments_integrate(pr->P, pr->G, pr->d_dnu, dJ, dH, dK, dK + 6 * pg, pr->stream);
        prof_end(pr, KI_MOMENTS);
        return check_launch();
    }
    rrt_status moments(rrt_frame frame, double *J, double *H, double *Kt)
    {
        const size_t pg = (size_t)pr->P * pr->G;
        rrt_status s = moments_launch(frame);
        if (s) return s;
        const double *dJ = pr->d_mom, *dH = dJ + pg, *dK = dH + 3 * pg;
        hipError_t e = hipSuccess;
        if (J && e == hipSuccess) e = hipMemcpyAsync(J, dJ, pg * 8, hipMemcpyDeviceToHost, pr->stream);
        if (H && e == hipSuccess) e = hipMemcpyAsync(H, dH, pg * 24, hipMemcpyDeviceToHost, pr->stream);
        if (Kt && e == hipSuccess) e = hipMemcpyAsync(Kt, dK, pg * 48, hipMemcpyDeviceToHost, pr->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(pr->stream);
        if (e != hipSuccess) return fail(RRT_E_DEVICE, std::string("moments download: ") + hipGetErrorString(e));
        return RRT_OK;
    }
    rrt_status moments_integrated(rrt_frame frame, double *out)
    {
        const size_t pg = (size_t)pr->P * pr->G;
        rrt_status s = moments_launch(frame);
        if (s) return s;
        hipError_t e = hipMemcpyAsync(out, pr->d_mom + 10 * pg, (size_t)pr->P * 16 * 8, hipMemcpyDeviceToHost, pr->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(pr->stream);
        if (e != hipSuccess) return fail(RRT_E_DEVICE, std::string("moments download: ") + hipGetErrorString(e));
        return RRT_OK;
    }

    rrt_status advance(double dt, int nsteps, int scheme, double tol, int max_iter, int use_ng, int *iters, double *res)
    {
        const size_t n = do_elems(pr);
        const size_t b = n * pr->esz;
        rrt_status s;
        if ((s = pr_alloc(pr, &pr->d_Iin, b)) || (s = pr_alloc(pr, &pr->d_acc, b))) return s;
        int total = 0;
        double rmax = 0;
        for (int step = 0; step < nsteps; ++step) {
            if (scheme == RRT_SCHEME_EULER) {
                int it = 0;
                double r = 0;
                s = solve(pr->d_I, 1.0 / dt, pr->d_I, tol, max_iter, use_ng, &it, &r);
                total += it;
                rmax = std::fmax(rmax, r);
                if (s && s != RRT_E_NOT_CONVERGED) return s;
                HIPCHK(hipMemcpyAsync(pr->d_I, pr->d_Ilab, b, hipMemcpyDeviceToDevice, pr->stream));
                if (s) return s;
                continue;
            }
            HIPCHK(hipMemcpyAsync(pr->d_Iin, pr->d_I, b, hipMemcpyDeviceToDevice, pr->stream));
            const double frac[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
            const double coef[4] = {3.0, 1.5, 3.0, 0.0};
            for (int st = 0; st < 4; ++st) {
                int it = 0;
                double r = 0;
                s = solve(pr->d_Iin, 1.0 / (frac[st] * dt), pr->d_Iin, tol, max_iter, use_ng, &it, &r);
                total += it;
                rmax = std::fmax(rmax, r);
                if (s && s != RRT_E_NOT_CONVERGED) return s;
                if (s) return s;
                prof_begin(pr, KI_RK);
                rrt::launch_rk_stage<real>((long)n, R(pr->d_Ilab), R(pr->d_Iin), R(pr->d_acc), R(pr->d_I), st == 0,
                                           st == 3, (real)coef[st], pr->stream);
                prof_end(pr, KI_RK);
                if ((s = check_launch())) return s;
            }
        }
        // comoving SH intensity of the final state, for the comoving moments
        if ((s = fold(pr->d_I))) return s;
        *iters = total;
        *res = rmax;
        return check_launch();
    }
};

template <typename F>
rrt_status dispatch(rrt_problem *pr, F &&f)
{
    if (pr->prec == RRT_FP64) {
        Engine<double> e{pr};
        return f(e);
    }
    Engine<float> e{pr};
    return f(e);
}

// the per-group lab extinction transposed for group-major ray traces (allocated on first
// need, recomputed with every medium); nothing to do for an extinction shared by all groups
rrt_status ensure_chilab_gmajor(rrt_problem *pr)
{
    if (pr->grey_chi || pr->G < 2) return RRT_OK;
    rrt_status s = pr_alloc(pr, &pr->d_chilabT, (size_t)pr->K * pr->P * pr->G * pr->esz);
    if (s) return s;
    if (pr->prec == RRT_FP64)
        rrt::launch_transpose_lab<double>((const double *)pr->d_chilab, (double *)pr->d_chilabT, pr->P, pr->G, pr->K,
                                          true, pr->stream);
    else
        rrt::launch_transpose_lab<float>((const float *)pr->d_chilab, (float *)pr->d_chilabT, pr->P, pr->G, pr->K,
                                         true, pr->stream);
    HIPCHK(hipGetLastError());
    return RRT_OK;
}

rrt_status check_sizes(const rrt_grid *g, const rrt_groups *gr, const rrt_angles *a, rrt_scatter sc, int prec)
{
    if (!g || !gr || !a) return fail(RRT_E_INVALID, "NULL grid/groups/angles");
    if (g->nx < 1 || g->ny < 1 || g->nz < 2) return fail(RRT_E_INVALID, "grid needs nx, ny >= 1 and nz >= 2");
    if (!(g->lx > 0) || !(g->ly > 0) || !(g->lz > 0)) return fail(RRT_E_INVALID, "domain lengths must be > 0");
    if (a->lmax < 0 || a->n_mu < 2 || a->n_phi < 1) return fail(RRT_E_INVALID, "bad angular sizes");
    if (a->n_mu % 2) return fail(RRT_E_INVALID, "n_mu must be even (no horizontal ordinate)");
    if ((long)a->n_mu * a->n_phi > 65535) return fail(RRT_E_INVALID, "at most 65535 ordinates");
    // the remap plan packs the ring (10 bits), azimuth (10 bits) and group shift (12 bits) in one word
    if (a->n_mu > 1022 || a->n_phi > 1024) return fail(RRT_E_INVALID, "at most 1022 polar and 1024 azimuthal nodes");
    if (gr->ngroups > 2046) return fail(RRT_E_INVALID, "at most 2046 groups");
    if (a->n_mu < a->lmax + 1 || a->n_phi < 2 * a->lmax + 1)
        return fail(RRT_E_INVALID, "ordinate mesh too coarse for lmax (need n_mu >= lmax+1, n_phi >= 2 lmax+1)");
    if (prec != RRT_FP64 && prec != RRT_FP32 && prec != RRT_MIXED) return fail(RRT_E_INVALID, "unknown precision");
    if (prec == RRT_MIXED && (a->lmax + 1) * (a->lmax + 1) > 256)
        return fail(RRT_E_INVALID, "mixed precision supports (lmax + 1)^2 <= 256");
    if (sc != RRT_THOMSON && sc != RRT_COMPTON) return fail(RRT_E_INVALID, "unknown scattering kernel");
    if (!gr->edges) {
        if (gr->ngroups != 1) return fail(RRT_E_INVALID, "a grey problem has exactly one group");
        if (sc == RRT_COMPTON) return fail(RRT_E_INVALID, "Compton scattering needs frequency groups");
    } else {
        if (gr->ngroups < 1) return fail(RRT_E_INVALID, "ngroups must be >= 1");
        for (int i = 0; i <= gr->ngroups; ++i)
            if (!std::isfinite(gr->edges[i]) || gr->edges[i] < 0) return fail(RRT_E_INVALID, "edges must be finite and >= 0");
        for (int i = 0; i < gr->ngroups; ++i)
            if (!(gr->edges[i + 1] > gr->edges[i])) return fail(RRT_E_INVALID, "edges must ascend");
        if (gr->log_centres && !(gr->edges[0] > 0)) return fail(RRT_E_INVALID, "log centres need edges > 0");
        if (sc == RRT_COMPTON && !(gr->mec2 > 0)) return fail(RRT_E_INVALID, "Compton scattering needs mec2 > 0");
    }
    (void)prec;
    return RRT_OK;
}

size_t footprint(const rrt_grid *g, const rrt_groups *gr, const rrt_angles *a, int prec, int time_dep, int use_ng)
{
    const size_t esz = prec == RRT_FP64 ? 8 : 4;
    const size_t P = (size_t)g->nx * g->ny * g->nz, G = gr->ngroups, K = (size_t)a->n_mu * a->n_phi;
    const size_t NL = (size_t)(a->lmax + 1) * (a->lmax + 1);
    size_t sh = P * G * NL * esz, dob = P * G * K * esz;
    size_t total = 3 * sh + 4 * dob;                 // S, Snew, Ilm; comoving ordinates, St, Ilab, I
    total += dob;                                    // lab extinction (per group: an upper bound)
    // its group-major copy, where the ray trace's planes leave LDS for one group per workgroup
    const size_t tl2 = (prec == RRT_FP64 ? rrt::trace_lds<double>(g->nx, g->ny, 2, 0)
                                          : rrt::trace_lds<float>(g->nx, g->ny, 2, 0));
    if (G >= 8 && tl2 > kMaxLds) total += dob;
    if (time_dep) total += 2 * dob;                  // stage input, accumulator
    if (use_ng) total += 4 * sh;                     // Ng chain
    total += P * (3 * G + 1) * esz + 4 * P * 8;     // fields, chi0, beta, Gamma
    total += 2 * P * K * 8 * esz;                    // remap plan of a moving medium (two entries per point and ordinate)
    total += 2 * (size_t)g->nx * g->ny * K * G * esz;  // boundaries
    total += 16 * P * G + 16 * G * rrt::kResidSplit + (1 << 20);   // residual row and partial sums, tables
    total += P * (8 + esz) + 25 * (size_t)(a->lmax + 1) * G * G * esz;  // electron-temperature brackets, node tables
    total += (P * G * 10 + P * 16) * 8;              // moment buffer
    return total;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *rrt_last_error(void) { return g_err.c_str(); }

size_t rrt_footprint_bytes(const rrt_grid *grid, const rrt_groups *groups, const rrt_angles *angles,
                           rrt_precision precision, int time_dependent, int use_ng)
{
    if (check_sizes(grid, groups, angles, RRT_THOMSON, precision) != RRT_OK) return 0;
    return footprint(grid, groups, angles, precision, time_dependent, use_ng);
}

// Compton tables at the node temperatures kT (units of the edges; {0}: electrons at
// rest), built on the GPU in FP64; the source tables A = s_i (nu_j dnu_i)/(nu_i dnu_j)
// p_l^{i->j}/(2l+1) and s are uploaded in the working precision
// Compton tables already built in this process, keyed by everything they depend on
// (groups, centres, rest energy, order, node temperatures): problems of a served
// mix share group sets and node grids, and a table build costs tens of ms
struct TableKey {
    int G, L;
    double mec2;
    std::vector<double> edges, centres, kT;
    bool operator<(const TableKey &o) const
    {
        return std::tie(G, L, mec2, edges, centres, kT) < std::tie(o.G, o.L, o.mec2, o.edges, o.centres, o.kT);
    }
};
static std::mutex g_tab_mu;
static std::map<TableKey, std::pair<std::vector<double>, std::vector<double>>> g_tables;
constexpr size_t kMaxCachedTables = 64;

static rrt_status build_compton_tables(rrt_problem *pr, const std::vector<double> &kT)
{
    if (pr->kT_nodes == kT && pr->d_A) return RRT_OK;
    const int G = pr->G, L = pr->lmax, nt = (int)kT.size();
    std::vector<double> sv, pv;
    const TableKey key{G, L, pr->mec2, pr->edges, pr->centres, kT};
    bool hit = false;
    {
        std::lock_guard<std::mutex> lk(g_tab_mu);
        auto it = g_tables.find(key);
        if (it != g_tables.end()) {
            sv = it->second.first;
            pv = it->second.second;
            hit = true;
        }
    }
    if (!hit) {
        const int e = rrt::compton_tables_gpu(G, pr->edges.data(), pr->centres.data(), pr->mec2, L, nt, kT.data(), sv,
                                              pv, pr->stream);
        if (e != 0) return fail(RRT_E_DEVICE, std::string("Compton tables: ") + hipGetErrorString((hipError_t)e));
        std::lock_guard<std::mutex> lk(g_tab_mu);
        if (g_tables.size() >= kMaxCachedTables) g_tables.clear();
        g_tables[key] = {sv, pv};
    }
    std::vector<double> A((size_t)nt * (L + 1) * G * G, 0.0);
    for (int n = 0; n < nt; ++n)
        for (int l = 0; l <= L; ++l)
            for (int i = 0; i < G; ++i)
                for (int j = 0; j < G; ++j) {
                    const double dnu_i = pr->edges[i + 1] - pr->edges[i], dnu_j = pr->edges[j + 1] - pr->edges[j];
                    const double pl = pv[(((size_t)n * (L + 1) + l) * G + i) * G + j];
                    A[(((size_t)n * (L + 1) + l) * G + j) * G + i] =
                        sv[(size_t)n * G + i] * (pr->centres[j] * dnu_i) / (pr->centres[i] * dnu_j) * pl / (2.0 * l + 1.0);
                }
    // replace the device tables
    pr->dev_bytes -= std::min(pr->dev_bytes, pr->tab_bytes);
    dev_free(pr->d_A);
    dev_free(pr->d_sg);
    pr->tab_bytes = 0;
    rrt_status s;
    if ((s = alloc_upload_real(pr, &pr->d_A, A)) || (s = alloc_upload_real(pr, &pr->d_sg, sv))) return s;
    pr->tab_bytes = (A.size() + sv.size()) * pr->esz;
    pr->kn_s = sv;
    pr->kn_A = A;
    pr->kT_nodes = kT;
    return RRT_OK;
}

void rrt_destroy(rrt_problem *pr)
{
    if (!pr) return;
    if (pr->batch) (void)rrt_batch_remove(pr->batch, pr);
    if (pr->stream) (void)hipStreamSynchronize(pr->stream);
    clear_graphs(pr);
    if (pr->h_red) (void)hipHostFree(pr->h_red);
    void *bufs[] = {pr->d_dir, pr->d_mu, pr->d_lnc, pr->d_nu3, pr->d_inv_nu3, pr->d_inv_dc, pr->d_geo, pr->d_taps, pr->d_order, pr->d_Yt, pr->d_WY, pr->d_Y, pr->d_WYt,
                    pr->d_Y16, pr->d_WYt16,
                    pr->d_A, pr->d_sg, pr->d_tnode, pr->d_twt, pr->d_torder, pr->d_kappa, pr->d_sigma, pr->d_bnu, pr->d_beta, pr->d_gam, pr->d_chi0, pr->d_chilab, pr->d_plan, pr->d_chilabT, pr->d_bc[0], pr->d_bc[1],
                    pr->d_S, pr->d_Snew, pr->d_Ilm, pr->d_co, pr->d_St, pr->d_Xt, pr->d_Ilab, pr->d_I, pr->d_Iin,
                    pr->d_acc, pr->d_chain[0], pr->d_chain[1], pr->d_chain[2], pr->d_chain[3], pr->d_partial, pr->d_red, pr->d_count, pr->d_vet, pr->d_mom, pr->d_dnu};
    for (void *b : bufs) dev_release(b);          // the stream is idle (synchronised above)
    for (int i = 0; i < KI_N; ++i)
        for (auto &e : pr->pending[i]) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    for (auto e : pr->pool) (void)hipEventDestroy(e);
    if (pr->own_stream && pr->stream) (void)hipStreamDestroy(pr->stream);
    delete pr;
}

// arguments of the stand-alone table builder; centres from the edges
static rrt_status table_args(int ngroups, const double *edges, int log_centres, double mec2, int lmax, int ntemp,
                             const double *kT, double *centres)
{
    if (ngroups < 1 || !edges || !kT || ntemp < 1 || lmax < 0 || lmax > 15)
        return fail(RRT_E_INVALID, "need ngroups >= 1, edges, 0 <= lmax <= 15 and ntemp >= 1 temperatures");
    if (!(mec2 > 0.0) || !std::isfinite(mec2)) return fail(RRT_E_INVALID, "mec2 must be finite and > 0");
    for (int g = 0; g < ngroups; ++g)
        if (!std::isfinite(edges[g]) || !std::isfinite(edges[g + 1]) || !(edges[g + 1] > edges[g]) || edges[0] < 0.0 ||
            (log_centres && !(edges[0] > 0.0)))
            return fail(RRT_E_INVALID, "edges must be finite and ascending (positive for log centres)");
    for (int n = 0; n < ntemp; ++n)
        if (!std::isfinite(kT[n]) || kT[n] < 0.0) return fail(RRT_E_INVALID, "temperatures must be finite and >= 0");
    for (int g = 0; g < ngroups; ++g)
        centres[g] = log_centres ? std::sqrt(edges[g] * edges[g + 1]) : 0.5 * (edges[g] + edges[g + 1]);
    return RRT_OK;
}

rrt_status rrt_compton_tables(int ngroups, const double *edges, int log_centres, double mec2, int lmax, int ntemp,
                              const double *kT, double *s, double *p, void *hip_stream)
{
    std::vector<double> c(std::max(ngroups, 1));
    rrt_status st = table_args(ngroups, edges, log_centres, mec2, lmax, ntemp, kT, c.data());
    if (st) return st;
    if (!s || !p) return fail(RRT_E_INVALID, "s and p are required");
    std::vector<double> sv, pv;
    const int e = rrt::compton_tables_gpu(ngroups, edges, c.data(), mec2, lmax, ntemp, kT, sv, pv, hip_stream);
    if (e != 0) return fail(RRT_E_DEVICE, std::string("Compton tables: ") + hipGetErrorString((hipError_t)e));
    std::copy(sv.begin(), sv.end(), s);
    std::copy(pv.begin(), pv.end(), p);
    return RRT_OK;
}

rrt_status rrt_compton_tables_noalloc(int ngroups, const double *edges, int log_centres, double mec2, int lmax,
                                      int ntemp, const double *kT, double *s, double *p, void *hip_stream)
{
    constexpr int kMaxGroups = 1024;
    double c[kMaxGroups];
    if (ngroups > kMaxGroups) return fail(RRT_E_INVALID, "at most 1024 groups");
    rrt_status st = table_args(ngroups, edges, log_centres, mec2, lmax, ntemp, kT, c);
    if (st) return st;
    if (!s || !p) return fail(RRT_E_INVALID, "s and p are required");
    const size_t need = rrt::compton_scratch_bytes(ngroups, lmax, ntemp), have = rrt::compton_static_scratch_bytes();
    if (need > have)
        return fail(RRT_E_INVALID, "tables of " + std::to_string(ngroups) + " groups, lmax " + std::to_string(lmax) +
                                       " at " + std::to_string(ntemp) + " temperatures need " + std::to_string(need) +
                                       " bytes of scratch; the allocation-free builder has " + std::to_string(have));
    const int e = rrt::compton_tables_static(ngroups, edges, c, mec2, lmax, ntemp, kT, s, p, hip_stream);
    if (e != 0) return fail(RRT_E_DEVICE, std::string("Compton tables: ") + hipGetErrorString((hipError_t)e));
    return RRT_OK;
}

rrt_status rrt_get_compton_tables(const rrt_problem *pr, int *ntemp, double *kT_nodes, double *s, double *A)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    if (pr->scatter != RRT_COMPTON) return fail(RRT_E_STATE, "not a Compton problem");
    const size_t nt = pr->kT_nodes.size();
    if (ntemp) *ntemp = (int)nt;
    if (kT_nodes) std::copy(pr->kT_nodes.begin(), pr->kT_nodes.end(), kT_nodes);
    if (s) std::copy(pr->kn_s.begin(), pr->kn_s.end(), s);
    if (A) std::copy(pr->kn_A.begin(), pr->kn_A.end(), A);
    return RRT_OK;
}

rrt_status rrt_create(const rrt_grid *grid, const rrt_groups *groups, const rrt_angles *angles, rrt_scatter scatter,
                      rrt_precision precision, void *hip_stream, rrt_problem **out)
{
    if (!out) return fail(RRT_E_INVALID, "out is NULL");
    *out = nullptr;
    rrt_status s = check_sizes(grid, groups, angles, scatter, precision);
    if (s) return s;
    rrt_problem *pr = new (std::nothrow) rrt_problem();
    if (!pr) return fail(RRT_E_HOST_OOM, "problem allocation");
    pr->nx = grid->nx; pr->ny = grid->ny; pr->nz = grid->nz;
    pr->lx = grid->lx; pr->ly = grid->ly; pr->lz = grid->lz;
    pr->P = (long)pr->nx * pr->ny * pr->nz;
    pr->grey = groups->edges == nullptr;
    pr->G = groups->ngroups;
    pr->log_centres = groups->log_centres;
    pr->mec2 = groups->mec2;
    pr->lmax = angles->lmax; pr->NL = (pr->lmax + 1) * (pr->lmax + 1);
    pr->nmu = angles->n_mu; pr->nphi = angles->n_phi; pr->K = pr->nmu * pr->nphi;
    pr->scatter = scatter;
    pr->prec = precision;
    pr->esz = precision == RRT_FP64 ? 8 : 4;
    auto bail = [&](rrt_status st) { rrt_destroy(pr); return st; };
    if (hip_stream) {
        pr->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        hipError_t e = hipStreamCreateWithFlags(&pr->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(fail(RRT_E_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e)));
        pr->own_stream = true;
    }
    {
        int dev = 0, lds = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        const size_t lim = std::min(kMaxLds, (size_t)lds);
        if (e == hipSuccess) e = rrt::set_lds_limits(lim);
        if (e != hipSuccess) return bail(fail(RRT_E_DEVICE, std::string("kernel set-up: ") + hipGetErrorString(e)));
        // sized for a chi~ per group, which also covers the grey and stand-alone cases
        auto tl = [&](int gc) {
            return pr->prec == RRT_FP64 ? rrt::trace_lds<double>(pr->nx, pr->ny, gc, 0)
                                        : rrt::trace_lds<float>(pr->nx, pr->ny, gc, 0);
        };
        // groups per ray-trace workgroup: the largest of 4, 2, 1 that divides G and
        // fits the LDS (a thread reads and writes the groups of a point as one
        // vector, and shares the tap addresses and a grey extinction among them)
        const long plane = (long)pr->nx * pr->ny;
        auto fits = [&](int gc) { return gc >= 1 && pr->G % gc == 0 && tl(gc) <= lim; };
        pr->Gc = 0;
        const char *env = std::getenv("RRT_TRACE_GC");
        const int want = env ? std::atoi(env) : 0;
        pr->lds_lim = lim;
        if ((want == 1 || want == 2 || want == 4) && fits(want)) {
            pr->Gc = want;
            pr->gc_forced = true;
        }
        for (int gc = 4; !pr->Gc && gc >= 1; gc /= 2)
            if (fits(gc)) pr->Gc = gc;
        pr->Gc_max = 0;
        for (int gc = 4; !pr->Gc_max && gc >= 1; gc /= 2)
            if (fits(gc)) pr->Gc_max = gc;
        const size_t need_boost = pr->prec == RRT_FP64 ? rrt::boost_lds<double>(pr->K, pr->G)
                                                       : rrt::boost_lds<float>(pr->K, pr->G);
        if (!pr->Gc || plane > rrt::kTraceMaxPlane)
            return bail(fail(RRT_E_INVALID, "an x-y plane is too large for the ray-trace kernel on this device"));
        if (scatter == RRT_COMPTON && pr->esz * (size_t)pr->G * pr->NL > lim)
            return bail(fail(RRT_E_INVALID, "groups x SH terms per point too large for the Compton source kernel"));
        if (need_boost > lim)
            return bail(fail(RRT_E_INVALID, "ordinates x groups per point too large for the frame-transform "
                                            "kernels' LDS in this precision"));
    }
    // ordinates and SH tables
    rrt::gauss_legendre(pr->nmu, pr->mu, pr->wmu);
    const int K = pr->K, NL = pr->NL;
    pr->dir.resize(4 * (size_t)K);
    pr->Y.resize((size_t)K * NL);
    for (int a = 0; a < pr->nmu; ++a)
        for (int b = 0; b < pr->nphi; ++b) {
            const int k = a * pr->nphi + b;
            const double m = pr->mu[a], ph = 2.0 * kPi * b / pr->nphi, st = std::sqrt(std::fmax(0.0, 1.0 - m * m));
            pr->dir[4 * k] = st * std::cos(ph);
            pr->dir[4 * k + 1] = st * std::sin(ph);
            pr->dir[4 * k + 2] = m;
            pr->dir[4 * k + 3] = pr->wmu[a] * 2.0 * kPi / pr->nphi;
            rrt::real_sh(pr->lmax, m, ph, &pr->Y[(size_t)k * NL]);
        }
    std::vector<double> Yt((size_t)NL * K), WY((size_t)K * NL);
    for (int k = 0; k < K; ++k)
        for (int q = 0; q < NL; ++q) {
            Yt[(size_t)q * K + k] = pr->Y[(size_t)k * NL + q];
            WY[(size_t)k * NL + q] = pr->dir[4 * k + 3] * pr->Y[(size_t)k * NL + q];
        }
    if ((s = upload_double(pr, (void **)&pr->d_dir, pr->dir)) || (s = upload_double(pr, (void **)&pr->d_mu, pr->mu)) ||
        (s = alloc_upload_real(pr, &pr->d_Yt, Yt)) || (s = alloc_upload_real(pr, &pr->d_WY, WY)))
        return bail(s);
    if (pr->prec == RRT_FP32) {
        // Y[k][q] (the forward product's B transposed) and WYt[q][k] (the backward one's)
        std::vector<double> WYt((size_t)NL * K);
        for (int k = 0; k < K; ++k)
            for (int q = 0; q < NL; ++q) WYt[(size_t)q * K + k] = WY[(size_t)k * NL + q];
        if ((s = alloc_upload_real(pr, &pr->d_Y, pr->Y)) || (s = alloc_upload_real(pr, &pr->d_WYt, WYt))) return bail(s);
    }
    if (pr->prec == RRT_MIXED) {
        // FP16 hi + lo tables in the layouts of the matrix-core operands: Y16[K up to 32][NL up
        // to the forward kernel's row width: 32, 64, 128 or 256] and WYt16[NL up to the backward
        // kernel's column count: 16, 64 or 256][K up to 32], zero padded
        const int Kt = (K + 31) / 32 * 32, Kp = (K + 31) / 32 * 32;
        const int NLp = NL <= 32 ? 32 : NL <= 64 ? 64 : NL <= 128 ? 128 : 256;
        const int NLr = NL <= 16 ? 16 : NL <= 64 ? 64 : 256;
        pr->y16_n = (size_t)Kt * NLp;
        pr->wyt16_n = (size_t)NLr * Kp;
        std::vector<_Float16> y16(2 * pr->y16_n, (_Float16)0.0f), wyt16(2 * pr->wyt16_n, (_Float16)0.0f);
        auto put = [](std::vector<_Float16> &t, size_t n, size_t i, double v) {
            const _Float16 h = (_Float16)v;
            t[i] = h;
            t[n + i] = (_Float16)(v - (double)h);
        };
        for (int k = 0; k < K; ++k)
            for (int q = 0; q < NL; ++q) {
                put(y16, pr->y16_n, (size_t)k * NLp + q, pr->Y[(size_t)k * NL + q]);
                put(wyt16, pr->wyt16_n, (size_t)q * Kp + k, WY[(size_t)k * NL + q]);
            }
        hipError_t e = hipMalloc(&pr->d_Y16, y16.size() * sizeof(_Float16));
        if (e == hipSuccess) e = hipMalloc(&pr->d_WYt16, wyt16.size() * sizeof(_Float16));
        if (e == hipSuccess) e = hipMemcpy(pr->d_Y16, y16.data(), y16.size() * sizeof(_Float16), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(pr->d_WYt16, wyt16.data(), wyt16.size() * sizeof(_Float16), hipMemcpyHostToDevice);
        if (e != hipSuccess) return bail(fail(RRT_E_HBM, std::string("mixed-precision tables: ") + hipGetErrorString(e)));
    }
    // ray-trace geometry per ordinate: the path from the previous z plane is cut
    // into the fewest equal pieces that move the ray at most one cell sideways
    // (a single column or row in x or y is left out: every offset reaches the
    // same point there); the count depends on mu only
    {
        const double dx = pr->lx / pr->nx, dy = pr->ly / pr->ny, dz = pr->lz / (pr->nz - 1);
        double hmin = 0.0;
        if (pr->nx > 1) hmin = dx;
        if (pr->ny > 1 && (hmin == 0.0 || dy < hmin)) hmin = dy;
        std::vector<rrt::OrdGeom> geo(K);
        std::vector<double> tix, tiy, tw;          // per tap: integer shift and eight weights
        for (int k = 0; k < K; ++k) {
            const double *n = &pr->dir[4 * k];
            rrt::OrdGeom &gm = geo[k];
            const double amu = std::fabs(n[2]);
            int npc = 1;
            if (hmin > 0.0) {
                const double cells = dz * std::sqrt(std::max(0.0, 1.0 - n[2] * n[2])) / (amu * hmin);
                npc = std::max(1, (int)std::ceil(cells - 1e-9));
            }
            gm.npc = npc;
            gm.ds = dz / amu / npc;
            gm.up = n[2] > 0 ? 1 : 0;
            gm.tap0 = (int)tix.size();
            // a displacement within rounding of whole cells (a ray in a grid plane,
            // n_x = cos(pi/2) ~ 6e-17) is taken as whole: no tap weight of ~1e-15
            // gives a vacuum neighbour a positive depth, which the slope limiter
            // would treat differently from zero
            auto snap = [](double o) { const double r = std::nearbyint(o); return std::fabs(o - r) < 1e-9 ? r : o; };
            const double ox = snap(-gm.ds * n[0] / dx), oy = snap(-gm.ds * n[1] / dy);
            for (int c = -1; c <= npc + 1; ++c) {
                const double sx = c * ox, sy = c * oy;
                const double fx0 = std::floor(sx), fy0 = std::floor(sy);
                const double fx = sx - fx0, fy = sy - fy0;
                long ix = (long)fx0 % pr->nx, iy = (long)fy0 % pr->ny;
                if (ix < 0) ix += pr->nx;
                if (iy < 0) iy += pr->ny;
                tix.push_back((double)ix);
                tiy.push_back((double)iy);
                // fraction of the plane spacing from the nearer plane: c / npc between
                // the grid point's plane and the upwind one, 1 / npc one piece beyond
                // either end, 0 on a grid plane
                const double f = (c == -1 || c == npc + 1) ? 1.0 / npc : (c == 0 || c == npc) ? 0.0 : (double)c / npc;
                const double w4[4] = {(1.0 - fx) * (1.0 - fy), fx * (1.0 - fy), (1.0 - fx) * fy, fx * fy};
                for (int w = 0; w < 4; ++w) tw.push_back((1.0 - f) * w4[w]);
                for (int w = 0; w < 4; ++w) tw.push_back(f * w4[w]);
            }
        }
        std::vector<int> order(K);
        for (int k = 0; k < K; ++k) order[k] = k;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return geo[x].npc > geo[y].npc; });
        pr->nmulti = 0;
        for (int k = 0; k < K; ++k) pr->nmulti += geo[k].npc > 1;
        s = pr_alloc(pr, (void **)&pr->d_geo, sizeof(rrt::OrdGeom) * K);
        if (s) return bail(s);
        s = pr_alloc(pr, (void **)&pr->d_order, sizeof(int) * K);
        if (s) return bail(s);
        const size_t nt = tix.size();
        auto fill_taps = [&](auto *tag, size_t esz) -> rrt_status {
            using real = std::remove_pointer_t<decltype(tag)>;
            std::vector<rrt::PathTap<real>> taps(nt);
            for (size_t i = 0; i < nt; ++i) {
                taps[i].ix = (int)tix[i];
                taps[i].iy = (int)tiy[i];
                for (int w = 0; w < 8; ++w) taps[i].w[w] = (real)tw[8 * i + w];
            }
            rrt_status st = pr_alloc(pr, &pr->d_taps, esz * nt);
            if (st) return st;
            if (hipMemcpy(pr->d_taps, taps.data(), esz * nt, hipMemcpyHostToDevice) != hipSuccess)
                return fail(RRT_E_DEVICE, "geometry upload");
            return RRT_OK;
        };
        s = pr->prec == RRT_FP64 ? fill_taps((double *)nullptr, sizeof(rrt::PathTap<double>))
                                 : fill_taps((float *)nullptr, sizeof(rrt::PathTap<float>));
        if (s) return bail(s);
        hipError_t e = hipMemcpy(pr->d_geo, geo.data(), sizeof(rrt::OrdGeom) * K, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(pr->d_order, order.data(), sizeof(int) * K, hipMemcpyHostToDevice);
        if (e != hipSuccess) return bail(fail(RRT_E_DEVICE, "geometry upload"));
    }
    // groups
    const int G = pr->G;
    if (pr->grey) {
        pr->edges = {0.0, 1.0};
        pr->centres = {1.0};
    } else {
        pr->edges.assign(groups->edges, groups->edges + G + 1);
        pr->centres.resize(G);
        for (int g = 0; g < G; ++g)
            pr->centres[g] = pr->log_centres ? std::sqrt(pr->edges[g] * pr->edges[g + 1]) : 0.5 * (pr->edges[g] + pr->edges[g + 1]);
    }
    {
        std::vector<double> lnc(G), nu3(G), inu3(G), idc(std::max(1, G - 1), 0.0);
        for (int g = 0; g < G; ++g) {
            lnc[g] = std::log(pr->centres[g]);
            nu3[g] = pr->centres[g] * pr->centres[g] * pr->centres[g];
            inu3[g] = 1.0 / nu3[g];
        }
        for (int g = 0; g + 1 < G; ++g) idc[g] = 1.0 / (lnc[g + 1] - lnc[g]);
        if ((s = upload_double(pr, (void **)&pr->d_lnc, lnc)) || (s = upload_double(pr, (void **)&pr->d_nu3, nu3)) ||
            (s = upload_double(pr, (void **)&pr->d_inv_nu3, inu3)) || (s = upload_double(pr, (void **)&pr->d_inv_dc, idc)))
            return bail(s);
        pr->fi.G = G;
        pr->fi.grey = pr->grey;
        pr->fi.has_lo_ghost = pr->edges[0] > 0.0;
        pr->fi.ghost_lo = pr->edges[0] > 0.0 ? 2.0 * std::log(pr->edges[0]) - lnc[0] : -INFINITY;
        pr->fi.ghost_hi = 2.0 * std::log(pr->edges[G]) - lnc[G - 1];
        pr->fi.inv_lo = pr->edges[0] > 0.0 ? 1.0 / (lnc[0] - pr->fi.ghost_lo) : 0.0;
        pr->fi.inv_hi = 1.0 / (pr->fi.ghost_hi - lnc[G - 1]);
        pr->fi.inv_dc = pr->d_inv_dc;
        // groups uniform in ln(nu): constant ln spacing of the edges (then the ghost
        // centres sit one spacing beyond the outer centres)
        pr->fi.uniform = 0;
        if (!pr->grey && G >= 2 && pr->log_centres && pr->edges[0] > 0.0) {
            const double d = std::log(pr->edges[1] / pr->edges[0]);
            bool uni = d > 0.0;
            for (int g = 1; g < G && uni; ++g)
                if (std::fabs(std::log(pr->edges[g + 1] / pr->edges[g]) - d) > 1e-12 * d) uni = false;
            if (uni) {
                pr->fi.uniform = 1;
                pr->fi.delta = d;
                pr->fi.inv_delta = 1.0 / d;
            }
        }
        pr->fi.lnc = pr->d_lnc;
        pr->fi.nu3 = pr->d_nu3;
        pr->fi.inv_nu3 = pr->d_inv_nu3;
    }
    if (scatter == RRT_COMPTON) {
        s = build_compton_tables(pr, std::vector<double>{0.0});
        if (s) return bail(s);
    }
    // state arrays
    const size_t shb = sh_elems(pr) * pr->esz, dob = do_elems(pr) * pr->esz;
    if ((s = pr_alloc(pr, &pr->d_S, shb)) || (s = pr_alloc(pr, &pr->d_Snew, shb)) || (s = pr_alloc(pr, &pr->d_Ilm, shb)) ||
        (s = pr_alloc(pr, &pr->d_co, dob)) || (s = pr_alloc(pr, &pr->d_St, dob)) || (s = pr_alloc(pr, &pr->d_Ilab, dob)) ||
        (s = pr_alloc(pr, &pr->d_I, dob)))
        return bail(s);
    {
        hipError_t e = hipMemsetAsync(pr->d_I, 0, dob, pr->stream);
        if (e == hipSuccess) e = hipMemsetAsync(pr->d_S, 0, shb, pr->stream);
        if (e == hipSuccess) e = hipMemsetAsync(pr->d_Ilm, 0, shb, pr->stream);
        if (e == hipSuccess) e = hipMemsetAsync(pr->d_Ilab, 0, dob, pr->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(pr->stream);
        if (e != hipSuccess) return bail(fail(RRT_E_DEVICE, "initial clear"));
    }
    pr->nblk_red = 1024;
    if ((s = pr_alloc(pr, (void **)&pr->d_partial,
                       std::max((size_t)pr->nblk_red * std::max(2 * G, 5),
                                2 * (size_t)pr->P * G + 2 * (size_t)G * rrt::kResidSplit) * 8)) ||
        (s = pr_alloc(pr, (void **)&pr->d_red, (size_t)std::max(2 * G, 5) * 8)) ||
        (s = pr_alloc(pr, (void **)&pr->d_mom, ((size_t)pr->P * G * 10 + (size_t)pr->P * 16) * 8)))
        return bail(s);
    {
        std::vector<double> dnu(G, 1.0);
        if (!pr->grey)
            for (int g = 0; g < G; ++g) dnu[g] = pr->edges[g + 1] - pr->edges[g];
        if ((s = upload_double(pr, (void **)&pr->d_dnu, dnu))) return bail(s);
    }
    if (hipHostMalloc((void **)&pr->h_red, (size_t)std::max(2 * G, 5) * 8, hipHostMallocDefault) != hipSuccess) {
        pr->h_red = nullptr;
        return bail(fail(RRT_E_HOST_OOM, "pinned residual buffer"));
    }
    *out = pr;
    g_err.clear();
    return RRT_OK;
}

rrt_status rrt_set_medium(rrt_problem *pr, const double *kappa, const double *sigma, const double *bnu,
                          const double *beta, const double *kte)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    if (!kappa || !sigma || !bnu) return fail(RRT_E_INVALID, "kappa, sigma and bnu are required");
    const size_t P = pr->P, G = pr->G;
    if (kte && pr->scatter != RRT_COMPTON)
        return fail(RRT_E_INVALID, "an electron temperature field applies to Compton scattering only");
    if (kte)
        for (size_t i = 0; i < P; ++i)
            if (!std::isfinite(kte[i]) || !(kte[i] > 0.0)) return fail(RRT_E_INVALID, "kte must be finite and > 0");
    clear_graphs(pr);
    for (size_t i = 0; i < P * G; ++i) {
        if (!std::isfinite(kappa[i]) || kappa[i] < 0) return fail(RRT_E_INVALID, "kappa must be finite and >= 0");
        if (!std::isfinite(bnu[i])) return fail(RRT_E_INVALID, "bnu must be finite");
    }
    for (size_t i = 0; i < P; ++i)
        if (!std::isfinite(sigma[i]) || sigma[i] < 0) return fail(RRT_E_INVALID, "sigma must be finite and >= 0");
    if (beta)
        for (size_t i = 0; i < P; ++i) {
            const double b2 = beta[3 * i] * beta[3 * i] + beta[3 * i + 1] * beta[3 * i + 1] + beta[3 * i + 2] * beta[3 * i + 2];
            if (!std::isfinite(b2) || !(b2 < 1.0)) return fail(RRT_E_INVALID, "|beta| must be < 1");
        }
    rrt_status s;
    if ((s = pr_alloc(pr, &pr->d_kappa, P * G * pr->esz)) || (s = pr_alloc(pr, &pr->d_sigma, P * pr->esz)) ||
        (s = pr_alloc(pr, &pr->d_bnu, P * G * pr->esz)) || (s = pr_alloc(pr, &pr->d_chi0, P * G * pr->esz)))
        return s;
    if ((s = upload_real(pr, pr->d_kappa, kappa, P * G)) || (s = upload_real(pr, pr->d_sigma, sigma, P)) ||
        (s = upload_real(pr, pr->d_bnu, bnu, P * G)))
        return s;
    if (beta) {
        std::vector<double> gam(P);
        for (size_t i = 0; i < P; ++i) {
            const double b2 = beta[3 * i] * beta[3 * i] + beta[3 * i + 1] * beta[3 * i + 1] + beta[3 * i + 2] * beta[3 * i + 2];
            gam[i] = 1.0 / std::sqrt(1.0 - b2);
        }
        if ((s = pr_alloc(pr, (void **)&pr->d_beta, P * 3 * 8)) || (s = pr_alloc(pr, (void **)&pr->d_gam, P * 8))) return s;
        HIPCHK(hipMemcpyAsync(pr->d_beta, beta, P * 3 * 8, hipMemcpyHostToDevice, pr->stream));
        HIPCHK(hipMemcpyAsync(pr->d_gam, gam.data(), P * 8, hipMemcpyHostToDevice, pr->stream));
        HIPCHK(hipStreamSynchronize(pr->stream));
    } else {
        void *b = pr->d_beta;
        dev_free(b);
        pr->d_beta = nullptr;
        void *gm = pr->d_gam;
        dev_free(gm);
        pr->d_gam = nullptr;
    }
    // extinction independent of frequency: Thomson with the same kappa in every group
    pr->grey_chi = 1;
    if (pr->scatter == RRT_COMPTON) pr->grey_chi = 0;
    for (size_t p = 0; p < P && pr->grey_chi; ++p)
        for (size_t g = 1; g < G; ++g)
            if (kappa[p * G + g] != kappa[p * G]) { pr->grey_chi = 0; break; }
    // lab extinction per (ordinate, point[, group]) of this medium
    {
        const size_t nchi = (size_t)pr->K * P * (pr->grey_chi ? 1 : G);
        void *c = pr->d_chilab;
        dev_free(c);
        pr->d_chilab = nullptr;
        if ((s = pr_alloc(pr, &pr->d_chilab, nchi * pr->esz))) return s;
    }
    // electron temperature: tables on log10 T nodes 1/8 decade apart covering the field,
    // each point between two nodes (linear in log10 T)
    if (pr->scatter == RRT_COMPTON) {
        std::vector<double> nodes{0.0};
        std::vector<double> lt;
        if (kte) {
            double lo = INFINITY, hi = -INFINITY;
            for (size_t i = 0; i < P; ++i) {
                const double v = std::log10(kte[i]);
                lo = std::min(lo, v);
                hi = std::max(hi, v);
            }
            const double a = std::floor(8.0 * lo + 1e-9) / 8.0, b = std::ceil(8.0 * hi - 1e-9) / 8.0;
            const int nt = (int)std::lround((b - a) * 8.0) + 1;
            nodes.assign(nt, 0.0);
            lt.assign(nt, 0.0);
            for (int n = 0; n < nt; ++n) {
                lt[n] = a + n / 8.0;
                nodes[n] = std::pow(10.0, lt[n]);
            }
        }
        if ((s = build_compton_tables(pr, nodes))) return s;
        pr->lt_nodes = lt;
        dev_free(*reinterpret_cast<void **>(&pr->d_tnode));
        dev_free(*reinterpret_cast<void **>(&pr->d_torder));
        dev_free(pr->d_twt);
        pr->dev_bytes -= std::min(pr->dev_bytes, pr->temp_bytes);
        pr->temp_bytes = 0;
        if (kte && lt.size() >= 2) {
            const int nt = (int)lt.size();
            std::vector<int> tn(P);
            std::vector<double> tw(P);
            for (size_t i = 0; i < P; ++i) {
                const double v = std::log10(kte[i]);
                int n = 0;
                double w = 0.0;
                if (v >= lt[nt - 1]) {
                    n = nt - 2;
                    w = 1.0;
                } else if (v > lt[0]) {
                    while (n < nt - 2 && v >= lt[n + 1]) ++n;
                    w = (v - lt[n]) / (lt[n + 1] - lt[n]);
                }
                tn[i] = n;
                tw[i] = w;
            }
            // the points ordered by bracket (counting sort, stable)
            std::vector<int> order(P), start(nt + 1, 0);
            for (size_t i = 0; i < P; ++i) ++start[tn[i] + 1];
            for (int n = 0; n < nt; ++n) start[n + 1] += start[n];
            for (size_t i = 0; i < P; ++i) order[start[tn[i]]++] = (int)i;
            if ((s = dev_alloc((void **)&pr->d_tnode, P * sizeof(int))) || (s = dev_alloc(&pr->d_twt, P * pr->esz)) ||
                (s = dev_alloc((void **)&pr->d_torder, P * sizeof(int))))
                return s;
            pr->temp_bytes = P * (2 * sizeof(int) + pr->esz);
            pr->dev_bytes += pr->temp_bytes;
            HIPCHK(hipMemcpyAsync(pr->d_tnode, tn.data(), P * sizeof(int), hipMemcpyHostToDevice, pr->stream));
            HIPCHK(hipMemcpyAsync(pr->d_torder, order.data(), P * sizeof(int), hipMemcpyHostToDevice, pr->stream));
            if ((s = upload_real(pr, pr->d_twt, tw.data(), P))) return s;
        }
    }
    auto chilab = [&](auto tag) {
        using real = decltype(tag);
        rrt::launch_chi0<real>((long)P, (int)G, (const real *)pr->d_kappa, (const real *)pr->d_sigma,
                               (const real *)pr->d_sg, pr->d_tnode, (const real *)pr->d_twt, (real *)pr->d_chi0,
                               pr->stream);
        rrt::ChiLabArgs<real> c;
        c.P = (long)P; c.K = pr->K; c.fi = pr->fi; c.chi_grey = pr->grey_chi; c.dir = pr->d_dir;
        c.chi0 = (const real *)pr->d_chi0; c.beta = pr->d_beta; c.gam = pr->d_gam; c.out = (real *)pr->d_chilab;
        rrt::launch_chilab<real>(c, pr->stream);
    };
    if (pr->prec == RRT_FP64) chilab(0.0); else chilab(0.0f);
    // group-major copy of a per-group extinction where the trace may use it: planes that
    // leave LDS for one group per workgroup only, or a copy kept from an earlier medium
    // default groups per trace workgroup for this medium: with a per-group extinction, four
    // spill registers (1024-thread workgroups hold 128 per lane) and are slower than two on
    // planes of 32 x 32 points and more, and than one on smaller planes (more workgroups);
    // the autotuner may revise it
    if (!pr->variants_fixed && !pr->gc_forced && !pr->tuned) {
        int gc = pr->Gc_max;
        if (!pr->grey_chi && pr->G > 1) gc = std::min(gc, (long)pr->nx * pr->ny >= 1024 ? 2 : 1);
        pr->Gc = gc;
    }
    if (!pr->grey_chi && pr->G > 1 && (pr->Gc_max == 1 || pr->d_chilabT || pr->gmajor))
        if ((s = ensure_chilab_gmajor(pr))) return s;
    // default: group-major planes where one group per workgroup is all the LDS holds and a
    // point's groups span whole 32-byte sectors (G >= 8); the autotuner may revise it
    if (!pr->variants_fixed && !pr->gc_forced) pr->gmajor = pr->Gc_max == 1 && pr->G >= 8;
    // remap plan of the velocity field
    if (beta) {
        const size_t esz = pr->prec == RRT_FP64 ? sizeof(rrt::RemapEntry<double>) : sizeof(rrt::RemapEntry<float>);
        if ((s = pr_alloc(pr, &pr->d_plan, 2 * P * pr->K * esz))) return s;
        auto plan = [&](auto tag) {
            using real = decltype(tag);
            rrt::PlanArgs<real> a;
            a.P = (long)P; a.K = pr->K; a.nmu = pr->nmu; a.nphi = pr->nphi; a.fi = pr->fi;
            a.dir = pr->d_dir; a.mu = pr->d_mu; a.beta = pr->d_beta; a.gam = pr->d_gam;
            a.chilab = static_cast<const real *>(pr->d_chilab); a.chi_grey = pr->grey_chi;
            a.boost = static_cast<rrt::RemapEntry<real> *>(pr->d_plan);
            a.unboost = a.boost + P * pr->K;
            rrt::launch_remap_plan<real>(a, pr->stream);
        };
        if (pr->prec == RRT_FP64) plan(0.0); else plan(0.0f);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(pr->stream));
    pr->medium_set = true;
    return RRT_OK;
}

rrt_status rrt_set_boundary(rrt_problem *pr, int face, const double *I_in)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    if (face != 0 && face != 1) return fail(RRT_E_INVALID, "face must be 0 (z = 0) or 1 (z = lz)");
    clear_graphs(pr);
    if (!I_in) {
        dev_free(pr->d_bc[face]);
        return RRT_OK;
    }
    const size_t n = (size_t)pr->K * pr->G * pr->nx * pr->ny;
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(I_in[i])) return fail(RRT_E_INVALID, "boundary intensity must be finite");
    rrt_status s = pr_alloc(pr, &pr->d_bc[face], n * pr->esz);
    if (s) return s;
    return upload_real(pr, pr->d_bc[face], I_in, n);
}

rrt_status rrt_set_intensity(rrt_problem *pr, const double *I_lab)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    const size_t n = do_elems(pr);
    if (!I_lab) {
        HIPCHK(hipMemsetAsync(pr->d_I, 0, n * pr->esz, pr->stream));
        HIPCHK(hipStreamSynchronize(pr->stream));
        return RRT_OK;
    }
    return upload_real(pr, pr->d_I, I_lab, n);
}

rrt_status rrt_set_source_sh(rrt_problem *pr, const double *S_lm)
{
    if (!pr || !S_lm) return fail(RRT_E_INVALID, "NULL argument");
    return upload_real(pr, pr->d_S, S_lm, sh_elems(pr));
}

rrt_status rrt_sweep(rrt_problem *pr, double dt_stage, rrt_info *info)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    if (!pr->medium_set) return fail(RRT_E_STATE, "rrt_set_medium must come first");
    if (!(dt_stage >= 0) || !std::isfinite(dt_stage)) return fail(RRT_E_INVALID, "dt_stage must be >= 0");
    auto t0 = std::chrono::steady_clock::now();
    double r = 0;
    rrt_status s = dispatch(pr, [&](auto &e) {
        return e.sweep(dt_stage > 0 ? pr->d_I : nullptr, dt_stage > 0 ? 1.0 / dt_stage : 0.0, &r);
    });
    if (info) {
        info->iters = 1;
        info->residual = r;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        info->updates = (long long)do_elems(pr);
    }
    return s;
}

rrt_status rrt_solve(rrt_problem *pr, double tol, int max_iter, int use_ng, rrt_info *info)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    if (pr->batch) return fail(RRT_E_STATE, "the problem is in a batch: remove it first");
    if (!pr->medium_set) return fail(RRT_E_STATE, "rrt_set_medium must come first");
    if (max_iter < 1 || !(tol >= 0)) return fail(RRT_E_INVALID, "need max_iter >= 1 and tol >= 0");
    auto t0 = std::chrono::steady_clock::now();
    int it = 0;
    double r = 0;
    rrt_status s = dispatch(pr, [&](auto &e) { return e.solve(nullptr, 0.0, pr->d_I, tol, max_iter, use_ng, &it, &r); });
    if (s == RRT_OK || s == RRT_E_NOT_CONVERGED) {
        hipError_t e = hipMemcpyAsync(pr->d_I, pr->d_Ilab, do_elems(pr) * pr->esz, hipMemcpyDeviceToDevice, pr->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(pr->stream);
        if (e != hipSuccess) s = fail(RRT_E_DEVICE, "state copy");
        if (s == RRT_E_NOT_CONVERGED) fail(s, "source iteration did not converge within max_iter");
    }
    if (info) {
        info->iters = it;
        info->residual = r;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        info->updates = (long long)it * (long long)do_elems(pr);
    }
    return s;
}

rrt_status rrt_advance(rrt_problem *pr, double dt, int nsteps, int scheme, double tol, int max_iter, int use_ng,
                       rrt_info *info)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    if (pr->batch) return fail(RRT_E_STATE, "the problem is in a batch: remove it first");
    if (!pr->medium_set) return fail(RRT_E_STATE, "rrt_set_medium must come first");
    if (!(dt > 0) || nsteps < 0 || max_iter < 1 || !(tol >= 0)) return fail(RRT_E_INVALID, "bad time-step arguments");
    if (scheme != RRT_SCHEME_RK4 && scheme != RRT_SCHEME_EULER) return fail(RRT_E_INVALID, "unknown scheme");
    auto t0 = std::chrono::steady_clock::now();
    int it = 0;
    double r = 0;
    rrt_status s = dispatch(pr, [&](auto &e) { return e.advance(dt, nsteps, scheme, tol, max_iter, use_ng, &it, &r); });
    if (s == RRT_E_NOT_CONVERGED) fail(s, "a stage did not converge within max_iter");
    if (info) {
        info->iters = it;
        info->residual = r;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        info->updates = (long long)it * (long long)do_elems(pr);
    }
    return s;
}

rrt_status rrt_get_moments(rrt_problem *pr, rrt_frame frame, double *J, double *H, double *K)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    if (frame != RRT_FRAME_LAB && frame != RRT_FRAME_COMOVING) return fail(RRT_E_INVALID, "unknown frame");
    return dispatch(pr, [&](auto &e) { return e.moments(frame, J, H, K); });
}

rrt_status rrt_get_moments_integrated(rrt_problem *pr, rrt_frame frame, double *out)
{
    if (!pr || !out) return fail(RRT_E_INVALID, "NULL argument");
    if (frame != RRT_FRAME_LAB && frame != RRT_FRAME_COMOVING) return fail(RRT_E_INVALID, "unknown frame");
    return dispatch(pr, [&](auto &e) { return e.moments_integrated(frame, out); });
}

rrt_status rrt_get_source_sh(rrt_problem *pr, double *S_lm)
{
    if (!pr || !S_lm) return fail(RRT_E_INVALID, "NULL argument");
    return download_real(pr, S_lm, pr->d_S, sh_elems(pr));
}

rrt_status rrt_get_intensity_sh(rrt_problem *pr, double *I_lm)
{
    if (!pr || !I_lm) return fail(RRT_E_INVALID, "NULL argument");
    return download_real(pr, I_lm, pr->d_Ilm, sh_elems(pr));
}

rrt_status rrt_get_intensity(rrt_problem *pr, double *I_lab)
{
    if (!pr || !I_lab) return fail(RRT_E_INVALID, "NULL argument");
    return download_real(pr, I_lab, pr->d_I, do_elems(pr));
}

rrt_status rrt_get_sweep_intensity(rrt_problem *pr, double *I_lab)
{
    if (!pr || !I_lab) return fail(RRT_E_INVALID, "NULL argument");
    return download_real(pr, I_lab, pr->d_Ilab, do_elems(pr));
}

rrt_status rrt_ray_trace(rrt_problem *pr, const double *S_tilde, const double *chi_tilde, double *I_lab)
{
    if (!pr || !S_tilde || !chi_tilde || !I_lab) return fail(RRT_E_INVALID, "NULL argument");
    const size_t n = do_elems(pr);
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(S_tilde[i]) || !std::isfinite(chi_tilde[i]) || chi_tilde[i] < 0)
            return fail(RRT_E_INVALID, "S~ must be finite and chi~ finite and >= 0");
    rrt_status s;
    if ((s = pr_alloc(pr, &pr->d_Xt, n * pr->esz))) return s;
    if ((s = upload_real(pr, pr->d_St, S_tilde, n)) || (s = upload_real(pr, pr->d_Xt, chi_tilde, n))) return s;
    s = dispatch(pr, [&](auto &e) {
        e.trace(pr->d_St, pr->d_Ilab, 0.0, true);
        return e.check_launch();
    });
    if (s) return s;
    return download_real(pr, I_lab, pr->d_Ilab, n);
}

rrt_status rrt_get_lab_source(rrt_problem *pr, double dt_stage, double *S_tilde)
{
    if (!pr || !S_tilde) return fail(RRT_E_INVALID, "NULL argument");
    if (!pr->medium_set) return fail(RRT_E_STATE, "rrt_set_medium must come first");
    if (!(dt_stage >= 0) || !std::isfinite(dt_stage)) return fail(RRT_E_INVALID, "dt_stage must be >= 0");
    rrt_status s = dispatch(pr, [&](auto &e) {
        return e.to_lab(pr->d_S, dt_stage > 0 ? pr->d_I : nullptr, dt_stage > 0 ? 1.0 / dt_stage : 0.0);
    });
    if (s) return s;
    return download_real(pr, S_tilde, pr->d_St, do_elems(pr));
}

// ---- device-pointer variants ----------------------------------------------

rrt_status rrt_set_medium_dev(rrt_problem *pr, const double *kappa, const double *sigma, const double *bnu,
                              const double *beta, const double *kte)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    rrt_status s;
    if ((s = check_dev_ptr(kappa, "kappa")) || (s = check_dev_ptr(sigma, "sigma")) || (s = check_dev_ptr(bnu, "bnu")))
        return s;
    if ((beta && (s = check_dev_ptr(beta, "beta"))) || (kte && (s = check_dev_ptr(kte, "kte")))) return s;
    const size_t P = (size_t)pr->P, G = (size_t)pr->G;
    std::vector<double> k, sg, b, v, t;
    if ((s = read_back(kappa, P * G, k)) || (s = read_back(sigma, P, sg)) || (s = read_back(bnu, P * G, b))) return s;
    if ((beta && (s = read_back(beta, P * 3, v))) || (kte && (s = read_back(kte, P, t)))) return s;
    return rrt_set_medium(pr, k.data(), sg.data(), b.data(), beta ? v.data() : nullptr, kte ? t.data() : nullptr);
}

rrt_status rrt_set_intensity_dev(rrt_problem *pr, const void *I_lab)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    rrt_status s = check_dev_ptr(I_lab, "I_lab");
    if (s) return s;
    return copy_dev(pr, pr->d_I, I_lab, do_elems(pr) * pr->esz);
}

rrt_status rrt_set_source_sh_dev(rrt_problem *pr, const void *S_lm)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    rrt_status s = check_dev_ptr(S_lm, "S_lm");
    if (s) return s;
    return copy_dev(pr, pr->d_S, S_lm, sh_elems(pr) * pr->esz);
}

rrt_status rrt_get_source_sh_dev(rrt_problem *pr, void *S_lm)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    rrt_status s = check_dev_ptr(S_lm, "S_lm");
    if (s) return s;
    return copy_dev(pr, S_lm, pr->d_S, sh_elems(pr) * pr->esz);
}

rrt_status rrt_get_intensity_sh_dev(rrt_problem *pr, void *I_lm)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    rrt_status s = check_dev_ptr(I_lm, "I_lm");
    if (s) return s;
    return copy_dev(pr, I_lm, pr->d_Ilm, sh_elems(pr) * pr->esz);
}

rrt_status rrt_get_intensity_dev(rrt_problem *pr, void *I_lab)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    rrt_status s = check_dev_ptr(I_lab, "I_lab");
    if (s) return s;
    return copy_dev(pr, I_lab, pr->d_I, do_elems(pr) * pr->esz);
}

rrt_status rrt_get_sweep_intensity_dev(rrt_problem *pr, void *I_lab)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    rrt_status s = check_dev_ptr(I_lab, "I_lab");
    if (s) return s;
    return copy_dev(pr, I_lab, pr->d_Ilab, do_elems(pr) * pr->esz);
}

rrt_status rrt_get_lab_source_dev(rrt_problem *pr, double dt_stage, void *S_tilde)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    rrt_status s = check_dev_ptr(S_tilde, "S_tilde");
    if (s) return s;
    if (!pr->medium_set) return fail(RRT_E_STATE, "rrt_set_medium must come first");
    if (!(dt_stage >= 0) || !std::isfinite(dt_stage)) return fail(RRT_E_INVALID, "dt_stage must be >= 0");
    s = dispatch(pr, [&](auto &e) {
        return e.to_lab(pr->d_S, dt_stage > 0 ? pr->d_I : nullptr, dt_stage > 0 ? 1.0 / dt_stage : 0.0);
    });
    if (s) return s;
    return copy_dev(pr, S_tilde, pr->d_St, do_elems(pr) * pr->esz);
}

rrt_status rrt_get_moments_dev(rrt_problem *pr, rrt_frame frame, double *J, double *H, double *K)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    if (frame != RRT_FRAME_LAB && frame != RRT_FRAME_COMOVING) return fail(RRT_E_INVALID, "unknown frame");
    rrt_status s;
    if ((J && (s = check_dev_ptr(J, "J"))) || (H && (s = check_dev_ptr(H, "H"))) || (K && (s = check_dev_ptr(K, "K"))))
        return s;
    s = dispatch(pr, [&](auto &e) { return e.moments_launch(frame); });
    if (s) return s;
    const size_t pg = (size_t)pr->P * pr->G;
    const double *dJ = pr->d_mom, *dH = dJ + pg, *dK = dH + 3 * pg;
    if (J) HIPCHK(hipMemcpyAsync(J, dJ, pg * 8, hipMemcpyDeviceToDevice, pr->stream));
    if (H) HIPCHK(hipMemcpyAsync(H, dH, pg * 24, hipMemcpyDeviceToDevice, pr->stream));
    if (K) HIPCHK(hipMemcpyAsync(K, dK, pg * 48, hipMemcpyDeviceToDevice, pr->stream));
    HIPCHK(hipStreamSynchronize(pr->stream));
    return RRT_OK;
}

rrt_status rrt_get_moments_integrated_dev(rrt_problem *pr, rrt_frame frame, double *out)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    if (frame != RRT_FRAME_LAB && frame != RRT_FRAME_COMOVING) return fail(RRT_E_INVALID, "unknown frame");
    rrt_status s = check_dev_ptr(out, "out");
    if (s) return s;
    s = dispatch(pr, [&](auto &e) { return e.moments_launch(frame); });
    if (s) return s;
    const size_t pg = (size_t)pr->P * pr->G;
    return copy_dev(pr, out, pr->d_mom + 10 * pg, (size_t)pr->P * 16 * 8);
}

rrt_status rrt_ray_trace_dev(rrt_problem *pr, const void *S_tilde, const void *chi_tilde, void *I_lab)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    rrt_status s;
    if ((s = check_dev_ptr(S_tilde, "S_tilde")) || (s = check_dev_ptr(chi_tilde, "chi_tilde")) ||
        (s = check_dev_ptr(I_lab, "I_lab")))
        return s;
    const size_t n = do_elems(pr);
    unsigned long long bad_s = 0, bad_x = 0;
    if ((s = count_bad_dev(pr, S_tilde, n, 0.0, false, &bad_s)) || (s = count_bad_dev(pr, chi_tilde, n, 0.0, true, &bad_x)))
        return s;
    if (bad_s || bad_x) return fail(RRT_E_INVALID, "S~ must be finite and chi~ finite and >= 0");
    if ((s = pr_alloc(pr, &pr->d_Xt, n * pr->esz))) return s;
    if ((s = copy_dev(pr, pr->d_St, S_tilde, n * pr->esz)) || (s = copy_dev(pr, pr->d_Xt, chi_tilde, n * pr->esz)))
        return s;
    s = dispatch(pr, [&](auto &e) {
        e.trace(pr->d_St, pr->d_Ilab, 0.0, true);
        return e.check_launch();
    });
    if (s) return s;
    return copy_dev(pr, I_lab, pr->d_Ilab, n * pr->esz);
}

// ---- variable-Eddington-tensor hand-off --------------------------------------

// Eddington tensor of the lab intensity state into d_vet, then nsteps steps on the
// device arrays (G zeroed first); returns after the stream completes
static rrt_status vet_run(rrt_problem *pr, double dt, int nsteps, const double *kap, const double *chi,
                          const double *B, double *J, double *H, double *G)
{
    const long P = pr->P;
    rrt_status s = dispatch(pr, [&](auto &e) { return e.moments_launch(RRT_FRAME_LAB); });
    if (s) return s;
    rrt::launch_vet_f(P, pr->d_mom + (size_t)10 * P * pr->G, pr->d_vet, pr->stream);
    HIPCHK(hipMemsetAsync(G, 0, (size_t)P * 4 * 8, pr->stream));
    rrt::VetArgs a;
    a.nx = pr->nx; a.ny = pr->ny; a.nz = pr->nz; a.P = P;
    const double dx = pr->lx / pr->nx, dy = pr->ly / pr->ny, dz = pr->nz > 1 ? pr->lz / (pr->nz - 1) : 1.0;
    a.idx2 = 0.5 / dx; a.idy2 = 0.5 / dy; a.idz2 = 0.5 / dz; a.idz = 1.0 / dz;
    a.dt = dt; a.f = pr->d_vet; a.kap = kap; a.chi = chi; a.B = B; a.J = J; a.H = H; a.G = G;
    for (int n = 0; n < nsteps; ++n) {
        prof_begin(pr, KI_VET_FLUX);
        rrt::launch_vet_flux(a, pr->stream);
        prof_end(pr, KI_VET_FLUX);
        prof_begin(pr, KI_VET_ENERGY);
        rrt::launch_vet_energy(a, pr->stream);
        prof_end(pr, KI_VET_ENERGY);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(pr->stream));
    return RRT_OK;
}

static rrt_status vet_args(rrt_problem *pr, double dt, int nsteps)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    if (!pr->medium_set) return fail(RRT_E_STATE, "rrt_set_medium must come first");
    if (!(dt > 0) || !std::isfinite(dt) || nsteps < 0) return fail(RRT_E_INVALID, "need dt > 0 and nsteps >= 0");
    return pr_alloc(pr, (void **)&pr->d_vet, (size_t)pr->P * 17 * 8);
}

rrt_status rrt_vet_step(rrt_problem *pr, double dt, int nsteps, const double *kappa_E, const double *chi_F,
                        const double *B, double *J, double *H, double *G)
{
    rrt_status s = vet_args(pr, dt, nsteps);
    if (s) return s;
    if (!kappa_E || !chi_F || !B || !J || !H) return fail(RRT_E_INVALID, "NULL argument");
    const size_t P = (size_t)pr->P;
    for (size_t p = 0; p < P; ++p) {
        if (!(kappa_E[p] >= 0) || !std::isfinite(kappa_E[p]) || !(chi_F[p] >= 0) || !std::isfinite(chi_F[p]))
            return fail(RRT_E_INVALID, "kappa_E and chi_F must be finite and >= 0");
        if (!std::isfinite(B[p]) || !std::isfinite(J[p]) || !std::isfinite(H[3 * p]) || !std::isfinite(H[3 * p + 1]) ||
            !std::isfinite(H[3 * p + 2]))
            return fail(RRT_E_INVALID, "B, J and H must be finite");
    }
    double *dk = pr->d_vet + 6 * P, *dc = dk + P, *db = dc + P, *dj = db + P, *dh = dj + P, *dg = dh + 3 * P;
    HIPCHK(hipMemcpyAsync(dk, kappa_E, P * 8, hipMemcpyHostToDevice, pr->stream));
    HIPCHK(hipMemcpyAsync(dc, chi_F, P * 8, hipMemcpyHostToDevice, pr->stream));
    HIPCHK(hipMemcpyAsync(db, B, P * 8, hipMemcpyHostToDevice, pr->stream));
    HIPCHK(hipMemcpyAsync(dj, J, P * 8, hipMemcpyHostToDevice, pr->stream));
    HIPCHK(hipMemcpyAsync(dh, H, P * 24, hipMemcpyHostToDevice, pr->stream));
    if ((s = vet_run(pr, dt, nsteps, dk, dc, db, dj, dh, dg))) return s;
    HIPCHK(hipMemcpyAsync(J, dj, P * 8, hipMemcpyDeviceToHost, pr->stream));
    HIPCHK(hipMemcpyAsync(H, dh, P * 24, hipMemcpyDeviceToHost, pr->stream));
    if (G) HIPCHK(hipMemcpyAsync(G, dg, P * 32, hipMemcpyDeviceToHost, pr->stream));
    HIPCHK(hipStreamSynchronize(pr->stream));
    return RRT_OK;
}

rrt_status rrt_vet_step_dev(rrt_problem *pr, double dt, int nsteps, const double *kappa_E, const double *chi_F,
                            const double *B, double *J, double *H, double *G)
{
    rrt_status s = vet_args(pr, dt, nsteps);
    if (s) return s;
    if ((s = check_dev_ptr(kappa_E, "kappa_E")) || (s = check_dev_ptr(chi_F, "chi_F")) || (s = check_dev_ptr(B, "B")) ||
        (s = check_dev_ptr(J, "J")) || (s = check_dev_ptr(H, "H")) || (G && (s = check_dev_ptr(G, "G"))))
        return s;
    const size_t P = (size_t)pr->P;
    unsigned long long bad[5] = {0, 0, 0, 0, 0};
    if ((s = count_bad_dev(pr, kappa_E, P, 0.0, true, &bad[0], true)) ||
        (s = count_bad_dev(pr, chi_F, P, 0.0, true, &bad[1], true)) ||
        (s = count_bad_dev(pr, B, P, 0.0, false, &bad[2], true)) ||
        (s = count_bad_dev(pr, J, P, 0.0, false, &bad[3], true)) ||
        (s = count_bad_dev(pr, H, 3 * P, 0.0, false, &bad[4], true)))
        return s;
    if (bad[0] || bad[1]) return fail(RRT_E_INVALID, "kappa_E and chi_F must be finite and >= 0");
    if (bad[2] || bad[3] || bad[4]) return fail(RRT_E_INVALID, "B, J and H must be finite");
    return vet_run(pr, dt, nsteps, kappa_E, chi_F, B, J, H, G ? G : pr->d_vet + 13 * P);
}

rrt_status rrt_set_autotune(rrt_problem *pr, int enable)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    pr->autotune = enable != 0;
    return RRT_OK;
}

rrt_status rrt_set_variants(rrt_problem *pr, int trace_groups, int s6_variant)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    bool ok_gc = trace_groups == 0;
    dispatch(pr, [&](auto &e) {
        for (int gc : e.gc_candidates()) ok_gc = ok_gc || gc == trace_groups || (trace_groups == -1 && gc == 1);
        return RRT_OK;
    });
    if (trace_groups == -1 && pr->G < 2) ok_gc = false;
    if (!ok_gc)
        return fail(RRT_E_INVALID, "groups per ray-trace workgroup must divide G and fit the LDS (1, 2 or 4; -1: one "
                                   "group on group-major planes, G > 1)");
    if (trace_groups == -1 && pr->medium_set) {
        rrt_status s = ensure_chilab_gmajor(pr);
        if (s) return s;
    }
    bool ok_s6 = s6_variant == -1;
    dispatch(pr, [&](auto &e) {
        for (int v : e.s6_candidates()) ok_s6 = ok_s6 || v == s6_variant;
        return RRT_OK;
    });
    if (!ok_s6) return fail(RRT_E_INVALID, "S6 variant not available for this shape and precision");
    clear_graphs(pr);
    if (trace_groups) {
        pr->gmajor = trace_groups == -1;
        pr->Gc = pr->gmajor ? 1 : trace_groups;
    }
    pr->s6 = s6_variant;
    pr->autotune = false;
    pr->variants_fixed = true;
    return RRT_OK;
}

rrt_status rrt_get_variants(const rrt_problem *pr, int *trace_groups, int *s6_variant, int *tuned)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    if (trace_groups) *trace_groups = pr->gmajor ? -1 : pr->Gc;
    if (s6_variant) *s6_variant = pr->s6;
    if (tuned) *tuned = pr->tuned ? 1 : 0;
    return RRT_OK;
}

rrt_status rrt_set_graphs(rrt_problem *pr, int enable)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    if (!enable) clear_graphs(pr);
    pr->use_graphs = enable != 0;
    return RRT_OK;
}

rrt_status rrt_graph_count(const rrt_problem *pr, int *count)
{
    if (!pr || !count) return fail(RRT_E_INVALID, "problem and count are required");
    *count = pr->graphs_failed ? -1 : (int)pr->graphs.size();
    return RRT_OK;
}

rrt_status rrt_set_profiling(rrt_problem *pr, int enable)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    prof_collect(pr);
    for (int i = 0; i < KI_N; ++i) {
        pr->ms[i] = 0;
        pr->calls[i] = 0;
    }
    pr->prof = enable != 0;
    return RRT_OK;
}

rrt_status rrt_kernel_time(rrt_problem *pr, const char *kernel, int *launches, double *ms)
{
    if (!pr || !kernel) return fail(RRT_E_INVALID, "NULL argument");
    prof_collect(pr);
    for (int i = 0; i < KI_N; ++i)
        if (std::strcmp(kernel, kNames[i]) == 0) {
            if (launches) *launches = pr->calls[i];
            if (ms) *ms = pr->ms[i];
            return RRT_OK;
        }
    return fail(RRT_E_INVALID, std::string("unknown kernel name ") + kernel);
}

rrt_status rrt_synchronize(rrt_problem *pr)
{
    if (!pr) return fail(RRT_E_INVALID, "problem is NULL");
    HIPCHK(hipStreamSynchronize(pr->stream));
    return RRT_OK;
}


// ---------------------------------------------------------------------------
// Batches: concurrent steady-state solves of independent problems
// ---------------------------------------------------------------------------
}  // extern "C"

struct rrt_batch {
    size_t budget = 0, used = 0;
    std::vector<rrt_problem *> items;
    std::vector<size_t> share;                      // bytes each admitted problem counts against the budget
};

namespace {

// a finished solve leaves its lab intensity as the problem's state, as rrt_solve does
void batch_finish(rrt_problem *pr)
{
    auto &v = pr->sv;
    v.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - v.t0).count();
    if (v.st == RRT_OK || v.st == RRT_E_NOT_CONVERGED) {
        hipError_t e = hipMemcpyAsync(pr->d_I, pr->d_Ilab, do_elems(pr) * pr->esz, hipMemcpyDeviceToDevice, pr->stream);
        if (e != hipSuccess) v.st = RRT_E_DEVICE;
    }
}

}  // namespace

extern "C" {

rrt_status rrt_set_device_pool(size_t max_bytes, size_t *held)
{
    DevPool &dp = dev_pool();
    std::vector<void *> out;
    {
        std::lock_guard<std::mutex> lk(dp.mu);
        dp.max_bytes = max_bytes;
        out = pool_take_excess(dp, max_bytes);
        if (held) *held = dp.held;
    }
    for (void *b : out) (void)hipFree(b);
    return RRT_OK;
}

size_t rrt_device_bytes(const rrt_problem *pr) { return pr ? pr->dev_bytes : 0; }

rrt_status rrt_batch_create(size_t max_hbm_bytes, rrt_batch **out)
{
    if (!out) return fail(RRT_E_INVALID, "out is NULL");
    *out = nullptr;
    rrt_batch *b = new (std::nothrow) rrt_batch();
    if (!b) return fail(RRT_E_HOST_OOM, "batch allocation");
    b->budget = max_hbm_bytes;
    *out = b;
    return RRT_OK;
}

rrt_status rrt_batch_admit(rrt_batch *b, rrt_problem *pr, double tol, int max_iter, int use_ng)
{
    if (!b || !pr) return fail(RRT_E_INVALID, "batch or problem is NULL");
    if (!pr->medium_set) return fail(RRT_E_STATE, "rrt_set_medium must come first");
    if (pr->batch) return fail(RRT_E_STATE, "the problem is already in a batch");
    if (max_iter < 1 || !(tol >= 0)) return fail(RRT_E_INVALID, "need max_iter >= 1 and tol >= 0");
    const size_t shb = sh_elems(pr) * pr->esz;
    const size_t need = pr->dev_bytes + ((use_ng && !pr->d_chain[0]) ? 4 * shb : 0);
    if (b->used + need > b->budget)
        return fail(RRT_E_HBM, "the batch's device-memory budget has no room for this problem");
    rrt_status s = dispatch(pr, [&](auto &e) { return e.solve_begin(nullptr, 0.0, pr->d_I, tol, max_iter, use_ng); });
    if (s) {
        pr->sv.phase = 0;
        return s;
    }
    pr->batch = b;
    b->items.push_back(pr);
    b->share.push_back(pr->dev_bytes);
    b->used += pr->dev_bytes;
    return RRT_OK;
}

rrt_status rrt_batch_step(rrt_batch *b, int rounds, int *active)
{
    if (!b || rounds < 0) return fail(RRT_E_INVALID, "batch is NULL or rounds < 0");
    for (int r = 0; r < rounds; ++r) {
        int n = 0;
        // queue one iteration of every running solve on its own stream, then collect them
        for (rrt_problem *pr : b->items) {
            if (pr->sv.phase != 1) continue;
            rrt_status s = dispatch(pr, [&](auto &e) { return e.round_launch(); });
            if (s) {
                pr->sv.st = s;
                pr->sv.phase = 2;
                batch_finish(pr);
            } else {
                ++n;
            }
        }
        if (!n) break;
        for (rrt_problem *pr : b->items) {
            if (pr->sv.phase != 1) continue;
            rrt_status s = hipStreamSynchronize(pr->stream) == hipSuccess
                               ? dispatch(pr, [&](auto &e) { return e.round_finish(); })
                               : fail(RRT_E_DEVICE, "stream synchronize");
            if (s) {
                pr->sv.st = s;
                pr->sv.phase = 2;
            }
            if (pr->sv.phase == 2) batch_finish(pr);
        }
    }
    if (active) {
        int n = 0;
        for (rrt_problem *pr : b->items) n += pr->sv.phase == 1;
        *active = n;
    }
    return RRT_OK;
}

rrt_status rrt_batch_poll(rrt_batch *b, const rrt_problem *pr, int *done, rrt_info *info)
{
    if (!b || !pr || !done) return fail(RRT_E_INVALID, "batch, problem or done is NULL");
    if (pr->batch != b) return fail(RRT_E_STATE, "the problem is not in this batch");
    const auto &v = pr->sv;
    *done = v.phase == 2;
    if (info) {
        info->iters = v.it;
        info->residual = v.r;
        info->seconds = v.phase == 2 ? v.seconds
                                     : std::chrono::duration<double>(std::chrono::steady_clock::now() - v.t0).count();
        info->updates = (long long)v.it * (long long)do_elems(pr);
    }
    if (v.phase == 2 && v.st != RRT_OK) {
        if (v.st == RRT_E_NOT_CONVERGED) fail(v.st, "source iteration did not converge within max_iter");
        return v.st;
    }
    return RRT_OK;
}

rrt_status rrt_batch_remove(rrt_batch *b, rrt_problem *pr)
{
    if (!b || !pr) return fail(RRT_E_INVALID, "batch or problem is NULL");
    for (size_t i = 0; i < b->items.size(); ++i) {
        if (b->items[i] != pr) continue;
        if (hipStreamSynchronize(pr->stream) != hipSuccess) return fail(RRT_E_DEVICE, "stream synchronize");
        b->used -= b->share[i];
        b->items.erase(b->items.begin() + i);
        b->share.erase(b->share.begin() + i);
        pr->batch = nullptr;
        pr->sv.phase = 0;
        return RRT_OK;
    }
    return fail(RRT_E_STATE, "the problem is not in this batch");
}

void rrt_batch_destroy(rrt_batch *b)
{
    if (!b) return;
    while (!b->items.empty()) (void)rrt_batch_remove(b, b->items.back());
    delete b;
}

}  // extern "C"
