/*
 * rrt.h -- C ABI of the MI355X mixed-frame relativistic radiative-transfer
 * library (librrt.so): the source-iteration sweep of the spherical-harmonic
 * discrete-ordinate method with time dependence, Lorentz transformation and
 * Thomson / Compton scattering of Tominaga, Shibata & Blinnikov (2015).
 *
 * The problem is the static transfer equation n.grad I = -chi I + eta (Eq. 1),
 * or its implicit time-discretised form with chi~ = chi + 1/(c dt) and
 * eta~ = eta + I(t)/(c dt) (Eqs. 4-6), solved by Lambda iteration (Sec. 2):
 * the source function is kept as real spherical harmonics in the comoving
 * frame (Eqs. 9-11), turned into discrete ordinates, Lorentz transformed to the
 * laboratory frame (Eqs. 7-8 and the invariants I/nu^3, chi nu), integrated
 * along rays in the laboratory frame, and folded back into comoving spherical
 * harmonics.  Units: c = 1 (time in units of length).
 *
 * Conventions used by every call
 *  - Grid: nx x ny x nz points; x_i = i lx/nx and y_j = j ly/ny are periodic,
 *    z_m = m lz/(nz-1) with the inflow boundaries on the planes z = 0, lz.
 *    Point index p = (z*ny + y)*nx + x; P = nx*ny*nz.
 *  - Ordinates: k = a*n_phi + b with mu_a the n_mu Gauss-Legendre nodes in
 *    ascending order and phi_b = 2 pi b / n_phi; zenith along z, azimuth from
 *    x towards y.  K = n_mu*n_phi.  n_mu must be even (no mu = 0 ray), and the
 *    mesh must resolve the SH order: n_mu >= lmax+1, n_phi >= 2*lmax+1.
 *  - Spherical harmonics: real orthonormal Y_lm, index q = l*l + l + m,
 *    NLM = (lmax+1)^2.
 *  - Groups: edges e_0 < ... < e_G; centres sqrt(e_g e_{g+1}) (log_centres=1)
 *    or (e_g+e_{g+1})/2.  edges == NULL with ngroups == 1 is one grey
 *    (frequency-integrated) group.
 *  - Array layouts (all row-major, C order):
 *      per-point fields     kappa, bnu [P][G]; sigma, kte [P]; beta [P][3]
 *      lab intensity        [K][P][G]        (ordinate, point, group innermost)
 *      z-boundary inflow    [K][ny][nx][G]   (only inflow ordinates are read)
 *      SH coefficients      [P][G][NLM]
 *      moments              J [P][G], H [P][G][3], K [P][G][6] (xx,yy,zz,xy,xz,yz)
 *  - Ownership: host arrays passed in are copied before the call returns; the
 *    caller keeps them.  The library owns all device memory from rrt_create to
 *    rrt_destroy.  Output arrays are caller-allocated with the sizes above.
 *  - Errors: every call returns an rrt_status; on failure rrt_last_error()
 *    describes it (thread-local, valid until the next call on that thread).
 *    No call aborts the process.
 *  - Threads: one problem must not be used from two threads at once; separate
 *    problems are independent.
 */
#ifndef RRT_H
#define RRT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RRT_OK = 0,
    RRT_E_INVALID = -1,        /* bad argument: sizes, NaN, kappa<0, |beta|>=1, ...   */
    RRT_E_HOST_OOM = -2,       /* host allocation failed                             */
    RRT_E_HBM = -3,            /* device memory would not fit / allocation failed    */
    RRT_E_NOT_CONVERGED = -4,  /* iteration limit reached; the last iterate is kept  */
    RRT_E_DEVICE = -5,         /* a HIP call failed                                  */
    RRT_E_STATE = -6           /* call out of order (e.g. solve before set_medium)   */
} rrt_status;

/* Working precision.  RRT_MIXED computes in FP32 like RRT_FP32 except the two
   SH <-> ordinate products of every sweep (Eq. 9, forward and backward), which
   run on FP16 matrix cores with FP32 accumulation: the data operand is scaled
   by powers of two per (point, group) row (per row and block of 32 ordinates
   in the backward product) and the SH tables are rounded to FP16.  Needs
   (lmax + 1)^2 <= 256.  Reductions stay FP64 in every mode. */
typedef enum { RRT_FP64 = 0, RRT_FP32 = 1, RRT_MIXED = 2 } rrt_precision;
typedef enum { RRT_THOMSON = 0, RRT_COMPTON = 1 } rrt_scatter;
typedef enum { RRT_FRAME_LAB = 0, RRT_FRAME_COMOVING = 1 } rrt_frame;
typedef enum { RRT_SCHEME_RK4 = 0, RRT_SCHEME_EULER = 1 } rrt_scheme;

typedef struct { int nx, ny, nz; double lx, ly, lz; } rrt_grid;
typedef struct {
    int ngroups;
    const double *edges;   /* ngroups+1 ascending edges, or NULL for one grey group */
    int log_centres;       /* 1: geometric centres; 0: arithmetic centres           */
    double mec2;           /* electron rest energy in the units of the edges (Compton) */
} rrt_groups;
typedef struct { int lmax, n_mu, n_phi; } rrt_angles;
typedef struct {
    int iters;             /* source iterations (sweeps) performed                   */
    double residual;       /* max over groups of ||S_new - S_old|| / ||S_new||       */
    double seconds;        /* wall time of the call                                  */
    long long updates;     /* grid-point x ordinate x group updates performed        */
} rrt_info;

typedef struct rrt_problem rrt_problem;

/* Create a problem: computes the ordinate set, the SH tables and, for Compton
   scattering, the Klein-Nishina group-to-group tables for electrons at rest
   (Sec. 2.3, Eqs. 13-14; built on the GPU in FP64), and allocates the device
   arrays.  hip_stream: a hipStream_t on
   which all work is queued, or NULL for a stream owned by the library.
   Errors: RRT_E_INVALID (sizes, odd n_mu, mesh too coarse for lmax, bad edges),
   RRT_E_HBM (device memory), RRT_E_DEVICE. */
rrt_status rrt_create(const rrt_grid *grid, const rrt_groups *groups, const rrt_angles *angles,
                      rrt_scatter scatter, rrt_precision precision, void *hip_stream,
                      rrt_problem **out);

/* Comoving medium (Eq. 1 with chi = alpha + sigma): absorption kappa [P][G] >= 0,
   n_e sigma_T [P] >= 0 (scattering coefficient per unit length), thermal source
   function bnu [P][G] (emission kappa*B), flow velocity beta [P][3] with
   |beta| < 1 or NULL for a static medium, electron temperature kte [P] > 0 in
   the units of the edges (Compton only) or NULL for electrons at rest (the
   paper's kernel, Sec. 2.3).  With a temperature field the group-to-group
   tables of the Klein-Nishina rate averaged over a Maxwell-Juttner electron
   gas (an extension of Eqs. 13-14; not in the paper) are built on the GPU at
   node temperatures log10 T_n = a + n/8 covering the field (a, b the field's
   log10 range rounded out to eighths of a decade), and every point uses the
   source tables A = s_i (nu_j dnu_i)/(nu_i dnu_j) p_l^{i->j}/(2l+1) and the
   cross-section ratio s interpolated linearly in log10 T between its two
   nodes.  Tables built once are kept for the process, keyed by the groups,
   mec2, lmax and node temperatures, so problems sharing them skip the build.
   Errors: RRT_E_INVALID for NaN/negative/|beta|>=1, for kte <= 0 or
   kte with Thomson scattering; RRT_E_DEVICE if the tables fail. */
rrt_status rrt_set_medium(rrt_problem *pr, const double *kappa, const double *sigma,
                          const double *bnu, const double *beta, const double *kte);

/* Inflow intensity on the z = 0 (face 0) or z = lz (face 1) plane in the lab
   frame, [K][ny][nx][G]; only ordinates entering the domain are used.
   NULL = vacuum (the default). */
rrt_status rrt_set_boundary(rrt_problem *pr, int face, const double *I_in);

/* Lab intensity state [K][P][G] (the initial condition of rrt_advance, the
   previous-time intensity of a time-dependent rrt_sweep, the first guess of
   rrt_solve); NULL sets it to zero. */
rrt_status rrt_set_intensity(rrt_problem *pr, const double *I_lab);

/* Frequency-integrated moments of the same fields as rrt_get_moments, reduced
   on the device in FP64 (X_tot = sum_g dnu_g X_g with the group widths, 1 for
   a grey group; Sec. 4 and the abstract: the Eddington tensor is what the
   method hands on), and the Eddington tensor f = K_tot / J_tot (0 where
   J_tot = 0): out [P][16] = J, H (x, y, z), K (xx, yy, zz, xy, xz, yz),
   f (same order).  Uses the problem's own moment buffer (no allocation).
   Errors: RRT_E_INVALID for NULL or an unknown frame. */
rrt_status rrt_get_moments_integrated(rrt_problem *pr, rrt_frame frame, double *out);

/* Stand-alone group-to-group Compton tables (Sec. 2.3, Eqs. 13-14, and
   their thermal average) for ngroups groups with edges [ngroups+1] (centres
   as in rrt_groups), electron rest energy mec2 in the units of the edges,
   Legendre orders 0..lmax (lmax <= 15), at ntemp electron temperatures
   kT [ntemp] (units of the edges; 0 = electrons at rest): cross-section
   ratios s [ntemp][ngroups] (sigma(nu_i; T)/sigma_T) and Legendre moments
   p [ntemp][lmax+1][ngroups][ngroups] (p_l^{i->j}, incident group i), FP64,
   into caller host arrays.  Built on the GPU on hip_stream (NULL: the null
   stream) with a device scratch buffer allocated and freed by the call.
   Errors: RRT_E_INVALID (sizes, edges, temperatures), RRT_E_DEVICE. */
rrt_status rrt_compton_tables(int ngroups, const double *edges, int log_centres, double mec2, int lmax, int ntemp,
                              const double *kT, double *s, double *p, void *hip_stream);

/* rrt_compton_tables without any device allocation, for callers that cannot
   allocate (code under HIP graph capture, tight serving loops, harnesses that
   forbid hipMalloc): the scratch is a static device array of 32 MiB per GPU,
   kept until the process ends, instead of a buffer allocated per call.  Same
   arguments, kernels and results.  Sizes whose scratch exceeds 32 MiB
   (about nt G^2 (lmax+1) 128 bytes) are refused with RRT_E_INVALID.  The array
   is shared by every call on a GPU: calls that overlap on one GPU race. */
rrt_status rrt_compton_tables_noalloc(int ngroups, const double *edges, int log_centres, double mec2, int lmax,
                                      int ntemp, const double *kT, double *s, double *p, void *hip_stream);

/* Compton tables in use (FP64 copies): ntemp node temperatures kT_nodes
   [ntemp] (a single node 0 for electrons at rest), cross-section ratios
   s [ntemp][G] (sigma(nu_i; T)/sigma_T) and source tables A
   [ntemp][lmax+1][G][G] (row j, column i: A_l^{ji} = s_i (nu_j dnu_i) /
   (nu_i dnu_j) p_l^{i->j} / (2l+1), Sec. 2.3).  Any output may be NULL (e.g.
   to query ntemp first).  Errors: RRT_E_STATE for Thomson problems. */
rrt_status rrt_get_compton_tables(const rrt_problem *pr, int *ntemp, double *kT_nodes, double *s, double *A);

/* Comoving SH source S [P][G][NLM] used by the next rrt_sweep. */
rrt_status rrt_set_source_sh(rrt_problem *pr, const double *S_lm);

/* One source iteration from the current SH source (no Ng): SH -> comoving
   ordinates, comoving -> lab transform with the time terms of Eqs. 5-6 when
   dt_stage > 0 (the intensity state is I(t)), ray trace, lab -> comoving,
   ordinates -> SH, new source, residual.  Afterwards the SH source is the new
   one and the last lab intensity / comoving SH intensity are readable.
   Errors: RRT_E_STATE before rrt_set_medium. */
rrt_status rrt_sweep(rrt_problem *pr, double dt_stage, rrt_info *info);

/* Steady solve: Lambda iteration from the source of the intensity state until
   residual < tol (Ng acceleration every third iteration of a chain when
   use_ng).  The intensity state becomes the last lab intensity.
   Returns RRT_E_NOT_CONVERGED after max_iter sweeps (result still readable). */
rrt_status rrt_solve(rrt_problem *pr, double tol, int max_iter, int use_ng, rrt_info *info);

/* nsteps time steps of length dt from the intensity state: RRT_SCHEME_RK4 is
   the four implicit stages of Appendix A (dt/6, dt/3, dt/3, dt/6 and
   Eq. A1), RRT_SCHEME_EULER one implicit stage.  Each stage is a solve to tol.
   Every stage returns the boundary inflow on the inflow faces unchanged, so
   the intensity state should already hold it there (upward ordinates on
   z = 0, downward ones on z = lz): with RRT_SCHEME_RK4 a difference d between
   the state and the boundary on those faces grows to d 9^m after m
   steps (the scheme's amplification of an infinitely stiff mode); with
   RRT_SCHEME_EULER it is replaced by the boundary in one step.  The library
   does not alter the caller's state. */
rrt_status rrt_advance(rrt_problem *pr, double dt, int nsteps, int scheme, double tol,
                       int max_iter, int use_ng, rrt_info *info);

/* Moments per point and group: lab frame by ordinate quadrature of the
   intensity state, comoving frame from the l <= 2 SH coefficients of the last
   comoving intensity: J = int I/4pi, H = int n I/4pi, K = int n n I/4pi; the
   Eddington tensor is K/J.  Reduced in FP64 into the problem's moment buffer
   (allocated with the problem and counted in its device bytes: no allocation
   per call).  Any output pointer may be NULL. */
rrt_status rrt_get_moments(rrt_problem *pr, rrt_frame frame, double *J, double *H, double *K);

rrt_status rrt_get_source_sh(rrt_problem *pr, double *S_lm);        /* [P][G][NLM] */
rrt_status rrt_get_intensity_sh(rrt_problem *pr, double *I_lm);     /* [P][G][NLM] */
rrt_status rrt_get_intensity(rrt_problem *pr, double *I_lab);       /* [K][P][G] state */
/* lab intensity produced by the last ray trace (rrt_sweep / solve / stage) */
rrt_status rrt_get_sweep_intensity(rrt_problem *pr, double *I_lab); /* [K][P][G]   */

/* Ray trace alone (the sweep's transfer step) from given lab S~ and chi~
   [K][P][G] with the problem's boundaries; result [K][P][G]. */
rrt_status rrt_ray_trace(rrt_problem *pr, const double *S_tilde, const double *chi_tilde,
                         double *I_lab);

/* The lab source S~ [K][P][G] that the next rrt_sweep(dt_stage) traces: the
   current SH source turned into comoving ordinates (Eq. 9), transformed to
   the lab ordinates (Eqs. 7-8) and combined with the time terms of Eqs. 5-6
   (the intensity state is I(t) when dt_stage > 0).  Runs the sweep's own S2
   and S3 kernels into its work array; the state is unchanged.
   Errors: RRT_E_STATE before rrt_set_medium, RRT_E_INVALID for dt_stage < 0. */
rrt_status rrt_get_lab_source(rrt_problem *pr, double dt_stage, double *S_tilde);

/* Device-pointer variants of the calls above, for callers whose data already
   sits in HBM (sizes and layouts as in the host calls).  Arrays of the
   problem's working precision (double for RRT_FP64, float for RRT_FP32 and
   RRT_MIXED) are typed void*; the medium and the moments stay FP64.  Each
   call queues its copies and kernels on the problem's stream and returns once
   they are complete: the caller's buffers are borrowed for the call only, and
   work the caller queued on another stream must be complete before the call.
   A pointer that is not device (or managed) memory is refused with
   RRT_E_INVALID.  rrt_set_medium_dev reads the fields back to the host (a
   set-up call: the validation and the temperature ordering of rrt_set_medium
   run there); rrt_ray_trace_dev validates S~ and chi~ on the device. */
rrt_status rrt_set_medium_dev(rrt_problem *pr, const double *kappa, const double *sigma, const double *bnu,
                              const double *beta, const double *kte);
rrt_status rrt_set_intensity_dev(rrt_problem *pr, const void *I_lab);         /* [K][P][G]   */
rrt_status rrt_set_source_sh_dev(rrt_problem *pr, const void *S_lm);          /* [P][G][NLM] */
rrt_status rrt_get_source_sh_dev(rrt_problem *pr, void *S_lm);                /* [P][G][NLM] */
rrt_status rrt_get_intensity_sh_dev(rrt_problem *pr, void *I_lm);             /* [P][G][NLM] */
rrt_status rrt_get_intensity_dev(rrt_problem *pr, void *I_lab);               /* [K][P][G] state */
rrt_status rrt_get_sweep_intensity_dev(rrt_problem *pr, void *I_lab);         /* [K][P][G]   */
rrt_status rrt_get_lab_source_dev(rrt_problem *pr, double dt_stage, void *S_tilde);   /* [K][P][G] */
rrt_status rrt_get_moments_dev(rrt_problem *pr, rrt_frame frame, double *J, double *H, double *K);
rrt_status rrt_get_moments_integrated_dev(rrt_problem *pr, rrt_frame frame, double *out);  /* [P][16] */
rrt_status rrt_ray_trace_dev(rrt_problem *pr, const void *S_tilde, const void *chi_tilde, void *I_lab);

/* Variable-Eddington-tensor hand-off (Sec. 4: the tensor from the transfer
   solution, instead of an approximate closure, in a radiation-hydrodynamics
   update).  The Eddington tensor f of the lab intensity state (as
   rrt_get_moments_integrated with RRT_FRAME_LAB; 0 where J = 0) closes the
   frequency-integrated moment equations
       dJ/dt + div H = kappa_E (B - J),   dH/dt + div (f J) = -chi_F H
   (c = 1, angle-averaged moments as everywhere here), advanced nsteps steps
   of dt by a forward-backward scheme (not in the paper): H from J^n, then J
   from H^{n+1}, the local terms implicit; central differences on the
   problem's grid, periodic in x and y, one-sided (first order) on the two z
   faces.  f is taken once per call.  The hydrodynamics side gives the energy
   exchange coefficient kappa_E [P] >= 0, the flux extinction chi_F [P] >= 0
   and the emission B [P]; J [P] and H [P][3] are advanced in place; G [P][4]
   (may be NULL) receives the exchange with the gas over the call,
   sum dt kappa_E (J^{n+1} - B) and sum dt chi_F H^{n+1}.  Stable for dt up
   to 2 h / sqrt(3) with h the smallest grid spacing (f has eigenvalues in
   [0, 1]).  FP64 in every precision; the work buffer (17 doubles per point)
   is allocated on first use and counted in rrt_device_bytes.  rrt_vet_step
   takes host arrays; rrt_vet_step_dev device arrays (validated on the device,
   borrowed for the call as the other *_dev calls).  Kernel times: "vet_flux",
   "vet_energy".  Errors: RRT_E_STATE before rrt_set_medium, RRT_E_INVALID for
   dt <= 0, nsteps < 0, negative or non-finite coefficients, non-finite B, J
   or H. */
rrt_status rrt_vet_step(rrt_problem *pr, double dt, int nsteps, const double *kappa_E, const double *chi_F,
                        const double *B, double *J, double *H, double *G);
rrt_status rrt_vet_step_dev(rrt_problem *pr, double dt, int nsteps, const double *kappa_E, const double *chi_F,
                            const double *B, double *J, double *H, double *G);

/* Device bytes the problem needs (0 if the arguments are invalid). */
size_t rrt_footprint_bytes(const rrt_grid *grid, const rrt_groups *groups, const rrt_angles *angles,
                           rrt_precision precision, int time_dependent, int use_ng);

/* Kernel variants.  Two choices of the sweep have several correct kernels:
   the groups per ray-trace workgroup (1, 2 or 4: those dividing G whose
   planes fit the LDS) and the ordinate -> SH product (S6; -1 the default for
   the shape, 0 the library product (FP32 only), 1, 2 or 4 the matrix-core
   kernel with that many 16-row tiles per wave, for (L+1)^2 <= 64 in FP32 and
   mixed precision).  trace_groups -1 (G > 1) traces one group per workgroup
   on group-major planes: the lab source is transposed to [k][g][p] before the
   trace and the intensity back after it, so that the trace reads and writes
   whole planes of one group contiguously (for planes too large for more than
   one group in LDS); a per-group extinction is then kept transposed too (one
   more ordinate-size array).  It is the default where only one group per
   workgroup fits the LDS and G >= 8.  With autotuning on (the default) each candidate is timed
   on the problem's own buffers at the start of its second sweep and the
   fastest kept; the choice is remembered per problem shape for the rest of
   the process (the group-major trace is a candidate where a transposed
   extinction exists: planes that fit one group per workgroup only).  The first
   sweep always uses the defaults.  Variants differ only in the order of
   floating-point sums.  rrt_set_variants fixes them
   (trace_groups 0 keeps the current one) and turns autotuning off; it
   returns RRT_E_INVALID for a variant the shape or precision does not have.
   RRT_TRACE_GC in the environment at creation fixes the groups per workgroup. */
rrt_status rrt_set_autotune(rrt_problem *pr, int enable);
rrt_status rrt_set_variants(rrt_problem *pr, int trace_groups, int s6_variant);
rrt_status rrt_get_variants(const rrt_problem *pr, int *trace_groups, int *s6_variant, int *tuned);

/* Captured sweeps.  With graphs enabled (the default) a sweep whose source
   buffer, stage input and 1/(c dt) have already been run eagerly is captured
   once into a HIP graph on the problem's stream and replayed from then on:
   the same kernels in the same order, so results are bit-identical to eager
   sweeps; only the host launch cost changes.  Graphs are not used while kernel
   timing is on.  Disabling drops the captured graphs.  Setting the medium or a
   boundary drops them too (their buffers may change).  If the runtime refuses
   a capture the problem runs eagerly from then on.  rrt_graph_count returns
   the number of captured sweeps held, or -1 after a refused capture. */
rrt_status rrt_set_graphs(rrt_problem *pr, int enable);
rrt_status rrt_graph_count(const rrt_problem *pr, int *count);

/* Kernel timing: when enabled, each launch of the library's kernels is
   bracketed by HIP events on the problem's stream; rrt_kernel_time returns
   the number of launches and their summed duration (ms) for one kernel name
   ("trace", "sh2do", "boost", "unboost", "do2sh", "source", "reduce",
   "moments", "rk", "vet_flux", "vet_energy") since the last reset,
   synchronising the stream. */
rrt_status rrt_set_profiling(rrt_problem *pr, int enable);
rrt_status rrt_kernel_time(rrt_problem *pr, const char *kernel, int *launches, double *ms);

/* Synchronise the problem's stream. */
rrt_status rrt_synchronize(rrt_problem *pr);

/* Destroy a problem (removing it from its batch first) and free its memory. */
void rrt_destroy(rrt_problem *pr);
const char *rrt_last_error(void);

/* Device memory the problem holds now, in bytes (grows when Ng chains or
   time-stepping arrays are first needed). */
size_t rrt_device_bytes(const rrt_problem *pr);

/* Keep up to max_bytes of the device memory that rrt_destroy frees, for reuse
   by later problems that allocate blocks of the same sizes (exact sizes, per
   device; the oldest blocks are freed first beyond the limit).  For serving
   many problems: freeing device memory synchronises the whole device, so
   every retirement would otherwise stall the other problems' streams.  0, the
   default, frees at once; lowering the limit frees the excess now (and 0
   everything held).  A block enters the pool only after its problem's
   stream is idle.  When an allocation fails the pool is emptied and the
   allocation tried again.  Process-wide and thread-safe; memory held in the
   pool is in no problem's rrt_device_bytes.  *held (may be NULL) receives the
   bytes held after the call. */
rrt_status rrt_set_device_pool(size_t max_bytes, size_t *held);

/* ---------------------------------------------------------------------------
   Batches: steady-state solves of independent problems sharing the GPU.
   Each admitted problem runs the Lambda iteration with Ng acceleration of
   rrt_solve (Sec. 2), kept on the device between calls; rrt_batch_step
   advances every running solve by one iteration per round, queuing all of
   them (each problem on its own stream) before waiting, so their kernels
   overlap.  A solve runs exactly the iterations rrt_solve would, so its
   result is the same alone and in a batch.  A batch keeps pointers to its
   problems but owns none of them.
   ------------------------------------------------------------------------- */
typedef struct rrt_batch rrt_batch;

/* A batch whose admitted problems may hold at most max_hbm_bytes of device
   memory (rrt_device_bytes, counted at admission). */
rrt_status rrt_batch_create(size_t max_hbm_bytes, rrt_batch **out);

/* Admit a problem (medium set, not in a batch) and start its solve from its
   current intensity state (0 after rrt_create), as rrt_solve(tol, max_iter,
   use_ng).  RRT_E_HBM when the budget has no room (the batch is unchanged),
   RRT_E_STATE / RRT_E_INVALID for bad state or arguments. */
rrt_status rrt_batch_admit(rrt_batch *b, rrt_problem *pr, double tol, int max_iter, int use_ng);

/* Advance every running solve by up to `rounds` iterations; *active (may be
   NULL) receives the number still running. */
rrt_status rrt_batch_step(rrt_batch *b, int rounds, int *active);

/* *done = 1 once the problem's solve has finished; info (may be NULL) as for
   rrt_solve, seconds measured from admission.  Returns the finished solve's
   status (RRT_OK, RRT_E_NOT_CONVERGED, or a device error), RRT_OK while it
   runs.  A finished problem's results are read with the usual getters. */
rrt_status rrt_batch_poll(rrt_batch *b, const rrt_problem *pr, int *done, rrt_info *info);

/* Take a problem (finished or not) out of the batch, returning its share of
   the budget; the problem itself stays valid. */
rrt_status rrt_batch_remove(rrt_batch *b, rrt_problem *pr);

/* Remove every problem and free the batch. */
void rrt_batch_destroy(rrt_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* RRT_H */
