/*
 * rte_romsad.h -- C ABI of the MI355X (gfx950) library for the steady one-group
 * radiative transfer equation solved by flexible GMRES with the ROMSAD
 * preconditioner (Peng, arXiv 2410.08735).
 *
 * Conventions shared by every call
 *  - Return value: 0 (RTE_OK) on success, < 0 on error, > 0 a warning
 *    (RTE_WNOTCONV: a solve stopped before its tolerance; its outputs and
 *    statistics are still written).  rte_status_string() names a code.
 *  - Arrays marked "device" are caller-owned device pointers (for example the
 *    storage of a torch tensor), contiguous, FP64 unless stated.  Arrays marked
 *    "host" are caller-owned host memory.  The library never frees or keeps
 *    caller memory beyond the call.
 *  - Every call that takes `stream` enqueues its work on that HIP stream (a
 *    hipStream_t passed as void*; NULL = the null stream).  Calls that return
 *    host-visible results (statistics, reports, ranks) synchronise the stream
 *    before returning.
 *  - Invalid arguments are rejected with RTE_EINVAL before any kernel launch.
 *    The solvers (fgmres_solve, si_solve, romsad_build_greedy,
 *    rte_mlp_snapshots) also read the cross sections on the host and reject
 *    a sigma_t that is not finite and > 0 or a sigma_s that is not finite and
 *    >= 0; the operator-level calls (rte_sweep, rte_apply_A, rte_rhs,
 *    rte_dsa_apply, romsad_apply) stay asynchronous and do not read them.
 *  - Opaque handles (rte_batch, rte_rom, rte_mlp) are library-owned and are
 *    released with their destroy call.
 *
 * Discretisation and layout (sections 2.1-2.3 of the paper)
 *  - S_N ordinates Omega_j with normalised weights w_j (sum w_j = 1); the scalar
 *    flux is phi = sum_j w_j psi_j.
 *  - Upwind DG with degree 1: P1 in slab geometry (2 dofs per cell), Q1 in X-Y
 *    geometry (4 dofs per cell), on a uniform nx x ny grid of a box.
 *  - Per cell the orthonormal tensor Legendre basis e_p(x) e_q(y),
 *    e_0 = 1/sqrt(h), e_1 = sqrt(3) s/sqrt(h), s the local coordinate in [-1, 1].
 *  - Instance vector layout: dof = cell * nloc + p + 2 q, cell = k * nx + i.
 *    A batch vector packs the instances one after another; rte_batch_offset()
 *    gives where an instance starts.  Angular fluxes are [n_ord][ndof] per
 *    instance, packed likewise (rte_batch_psi_offset()).
 *  - Cross sections are piecewise constant on regions: sigma_t and sigma_s
 *    arguments are device arrays [n_inst][max_regions] (row stride
 *    rte_batch_max_regions()); the cell -> region map is fixed at batch creation.
 *  - Inflow (section 2, the boundary condition): an isotropic constant value on
 *    each side of the domain, device array [n_inst][4] = (left, right, bottom,
 *    top) (slab: left, right, unused, unused); a side's value enters for the
 *    directions pointing into the domain there.  NULL = zero inflow.
 */
#ifndef RTE_ROMSAD_H
#define RTE_ROMSAD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  RTE_OK = 0,
  RTE_EINVAL = -1,      /* invalid argument (shape, pointer, value)           */
  RTE_EHIP = -2,        /* a HIP runtime call failed                          */
  RTE_ENOMEM = -3,      /* device allocation failed                           */
  RTE_EBREAKDOWN = -4,  /* Krylov breakdown with a singular least squares     */
  RTE_ESINGULAR = -5,   /* singular reduced operator                          */
  RTE_EIO = -6,         /* file read/write failed                             */
  RTE_ENONFINITE = -7,  /* a non-finite (NaN / Inf) value reached a norm      */
  RTE_WNOTCONV = 1      /* not converged within the iteration limits          */
};

enum { RTE_F64 = 0, RTE_F32 = 1, RTE_BF16 = 2 };

enum { RTE_PC_NONE = 0, RTE_PC_DSA = 1, RTE_PC_ROMSAD = 2, RTE_PC_MLP = 3 };

/* DSA variants (App. A): fully consistent, or partially consistent (the
 * first-moment rows keep only the central-flux part of the advection, the
 * jump part D_J is dropped there).                                           */
enum { RTE_DSA_FC = 0, RTE_DSA_PC = 1 };

typedef struct rte_batch rte_batch;
typedef struct rte_rom rte_rom;
typedef struct rte_mlp rte_mlp;

const char* rte_status_string(int status);

/* ---------------------------------------------------------------- quadrature
 * Chebyshev-Legendre rule CL(n_theta, n_z) of section 2.1: theta_j1 =
 * (2 j1 - 1) pi / n_theta with weight 1/n_theta, times the normalised n_z-point
 * Gauss-Legendre rule in Omega_z; ordinate j = (j2 - 1) n_theta + j1.
 * folded != 0 keeps only the Omega_z > 0 nodes with doubled weights (exact in
 * X-Y geometry, where the operator depends on Omega_x, Omega_y only).
 * Outputs (host) have n_theta * n_z (folded: n_theta * n_z / 2) entries.      */
int rte_quadrature_cl(int n_theta, int n_z, int folded, double* ox, double* oy, double* w);
/* Slab S_n: Gauss-Legendre nodes mu_j (ox), oy = 0, weights w_j / 2 (App. A). */
int rte_quadrature_gl(int n, double* ox, double* oy, double* w);

/* ---------------------------------------------------------------- batches
 * One parameter instance: geometry, ordinates (host arrays copied at
 * creation) and the cell -> region map.  dim = 1: ny must be 1 and omega_y is
 * ignored.                                                                    */
typedef struct {
  int32_t dim, nx, ny;
  double x0, x1, y0, y1;
  int32_t n_ord;
  const double* omega_x; /* host [n_ord] */
  const double* omega_y; /* host [n_ord] */
  const double* weight;  /* host [n_ord], sum 1 */
  const int32_t* region; /* host [nx*ny] values in [0, n_regions) */
  int32_t n_regions;
} rte_instance_desc;

int rte_batch_create(const rte_instance_desc* inst, int n_inst, rte_batch** out);
void rte_batch_destroy(rte_batch* b);
int rte_batch_size(const rte_batch* b);
int64_t rte_batch_ndof(const rte_batch* b, int inst);
int64_t rte_batch_offset(const rte_batch* b, int inst);
int64_t rte_batch_total_dof(const rte_batch* b);
int64_t rte_batch_psi_offset(const rte_batch* b, int inst);
int64_t rte_batch_total_psi(const rte_batch* b);
int rte_batch_max_regions(const rte_batch* b);
/* The 2D sweep's launch plan per precision (dtype RTE_F64 / RTE_F32): kernel
 * variant (0: work-group slots follow the wavefront diagonal; 1: each slot
 * owns fixed rows and prefetches their next source values; 2: one wave per
 * work item, one lane per row, y traces passed between lanes, no barrier:
 * for batches of a few instances), G lanes per cell
 * group, opl ordinates per lane (a work group sweeps G * opl ordinates of one
 * quadrant) and threads per work group.  The first sweep of a batch times
 * every admissible plan and keeps the fastest (the autotuner); setting a plan
 * fixes it.  set: RTE_EINVAL for a plan the batch cannot run (G in
 * {1,2,4,8,16,32}; opl 1, 2 with G in {4,8,16}, 4 with G in {4,8}, or 8
 * with G = 4; threads a multiple of 64 and of G, up to 512; LDS within 64 KB;
 * variant 1 needs ceil(max_ny / (threads / G)) <= 8 rows per slot and at
 * most 256 regions, and takes up to 1024 threads when that is one row per
 * slot, except in FP64 with opl 8; variant 2 needs G = 1, threads = 64,
 * opl 1, 2 or 4, max_ny <= 256 and at most 256 regions).
 * Setting a plan resets the work-item order to 0.
 * get: out[6] = {variant, G, opl, threads, tuned, order}.                   */
int rte_batch_set_sweep_plan(rte_batch* b, int dtype, int variant, int G, int opl, int threads);
/* The order in which a sweep's work items start (0: instance by instance,
 * each XCD a contiguous run, so an instance's ordinate blocks share one L2;
 * 1: by decreasing cell-ordinates, dealt round robin over the XCDs, so that
 * in a batch of unequal instances the largest start first).  The autotuner
 * times both on its best plans for such batches.  RTE_EINVAL for another
 * value.                                                                   */
int rte_batch_set_sweep_order(rte_batch* b, int dtype, int order);

/* Cross sections that vary inside the cells (the variable-scattering problem
 * of section 5.3): sigma_t(x) = sum_f theta_t,f s_f(x) and sigma_s(x) =
 * sum_f theta_s,f s_f(x) with n_fields shape functions s_f, given by their
 * values at the nq x nq Gauss-Legendre points of every cell (host
 * [n_fields][ncell][nq * nq], point index gy * nq + gx with gx, gy the
 * ascending nodes along x and y, cell = k * nx + i).  The library forms every
 * cell's 4 x 4 mass block int_T s_f e_a e_b with the same rule; from then on
 * the per-instance sigma_t / sigma_s arrays hold the coefficients theta
 * ([n_inst][max_regions], first n_fields entries) and the region map is not
 * used.  Needs an X-Y batch whose instances share one grid, rule and region
 * map, with n_regions >= n_fields each (RTE_EINVAL otherwise).  Supported
 * afterwards:
 * rte_sweep, rte_rhs, rte_apply_A (the sweep's local matrices use the full
 * blocks), rte_dsa_apply and the DSA inside the solvers with restart >= 1
 * on reflection-symmetric rules (the multigrid hierarchy works with the cell
 * averages, the GMRES around it with the full blocks), romsad_apply,
 * fgmres_solve (preconditioners none, DSA, ROMSAD), romsad_build_greedy with
 * hf_dsa_tol > 0; si_solve, the learned correction and rte_mlp_snapshots
 * return RTE_EINVAL.  The sweep plan's variant is reset to 0 (the row-slot
 * kernel needs region-wise cross sections).                                 */
int rte_batch_set_fields(rte_batch* b, int n_fields, int nq, const double* values);
int rte_batch_sweep_plan(const rte_batch* b, int dtype, int32_t* out);

/* ---------------------------------------------------------------- transport
 * rte_sweep: the transport sweep of section 3.1 for every ordinate of every
 * instance, psi_j = (D_j + Sigma_t)^{-1} (q + g_j^(bc)), and its quadrature
 * reduction phi = sum_j w_j psi_j (the operator T of the memory-efficient
 * formulation, section 3.1).  q (device, packed [total_dof]) is isotropic.
 * phi_out (device, packed) and psi_out (device, [total_psi]) are each optional
 * (NULL) but not both.  dtype selects the arithmetic (RTE_F32 / RTE_F64);
 * inputs and outputs are FP64 either way.                                     */
int rte_sweep(const rte_batch* b, const double* sigma_t, const double* q, const double* inflow,
              double* phi_out, double* psi_out, int dtype, void* stream);

/* rte_sweep_noalloc: rte_sweep with phi_out only (psi is not stored), for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  It allocates
 * nothing: the partial scalar fluxes go to a static 64 MiB device array that
 * each GPU the library runs on holds until the process ends, and it does not
 * autotune (it launches the batch's current plan: the default one, one set
 * with rte_batch_set_sweep_plan, or one an earlier rte_sweep tuned).
 * RTE_EINVAL (nothing launched, a message on stderr) when the plan's partial
 * fluxes exceed 64 MiB (entries = sum over instances of ndof times the
 * ordinate blocks of the plan; FP64 8 B, FP32 4 B each).  Every call
 * overwrites the part of the array it uses before reading it; calls that
 * overlap on one GPU (other streams or threads) share the array and race.   */
int rte_sweep_noalloc(const rte_batch* b, const double* sigma_t, const double* q, const double* inflow,
                      double* phi_out, int dtype, void* stream);

/* rte_scalar_flux: phi = sum_j w_j psi_j for stored angular fluxes (the
 * discrete integration operator Q of section 2.3).                            */
int rte_scalar_flux(const rte_batch* b, const double* psi, double* phi_out, void* stream);

/* rte_apply_A: y = (I - T Sigma_s) x, the memory-efficient operator A~ of
 * section 3.2 (zero inflow), one sweep; dtype as in rte_sweep.               */
int rte_apply_A(const rte_batch* b, const double* sigma_t, const double* sigma_s, const double* x,
                double* y, int dtype, void* stream);

/* rte_rhs: b~ = sum_j w_j (D_j + Sigma_t)^{-1} (G + g_j^(bc)) (section 3.1).   */
int rte_rhs(const rte_batch* b, const double* sigma_t, const double* G, const double* inflow,
            double* b_out, int dtype, void* stream);

/* ---------------------------------------------------------------- DSA
 * rte_dsa_apply: z = M_DSA^{-1} v = v + dphi, where (dphi, dJ) solves the fully
 * consistent P1 moment system of App. A (zeroth and first angular moments of
 * the upwind correction equation under delta psi_j = dphi + 3 Omega_j.dJ,
 * written for X-Y geometry with the same two steps) with right-hand side
 * Sigma_s v; variant RTE_DSA_PC solves the partially consistent system of the
 * same appendix instead (no D_J terms in the first-moment rows).  restart >= 1: restarted GMRES (Krylov dimension `restart`)
 * preconditioned with one geometric-multigrid V-cycle per step (2 x 2 cell
 * agglomeration, red-black block Gauss-Seidel smoothing with exact cell-block
 * solves), in FP64, until the relative residual is <= inner_tol or inner_max
 * iterations.  restart = 0: inner_max stationary V-cycle iterations from zero
 * (inner_tol unused); when every instance has a reflection-symmetric rule the
 * hierarchy then runs in FP32 (a preconditioner, not an exact solve).
 * stats_iters (host [n_inst], nullable) receives the iterations used.
 * Errors: RTE_EINVAL for null pointers, inner_max < 1, restart outside
 * [0, 500], a negative / NaN inner_tol, an unknown variant, or RTE_DSA_PC with
 * restart = 0 (the block smoother does not converge on the PC system: PC
 * solves always run the preconditioned GMRES).                              */
int rte_dsa_apply(const rte_batch* b, const double* sigma_t, const double* sigma_s, const double* v,
                  double* z, double inner_tol, int inner_max, int restart, int variant,
                  int32_t* stats_iters, void* stream);

/* ---------------------------------------------------------------- FGMRES
 * fgmres_solve: Alg. 1 (flexible GMRES) for A~ phi = b~ on every instance,
 * zero initial guess, restarted every m iterations from the FP64 true
 * residual.  Per iteration j of a cycle the preconditioner is
 *   RTE_PC_NONE  z = v,
 *   RTE_PC_DSA   z = M_DSA^{-1} v,
 *   RTE_PC_ROMSAD  M_ROM^{-1} for j <= window, M_DSA^{-1} after (eq. of the
 *                  ROMSAD preconditioner); with window_cycles = k >= 1 only
 *                  the first k cycles open a window,
 *   RTE_PC_MLP   the learned reduced correction for j <= window with the ROMSAD
 *                correction as fallback and DSA after the window.
 * Stopping: Givens estimate <= rtol * ||b~|| ends a cycle; the FP64 true
 * residual ||b~ - A~ phi|| / ||b~|| <= rtol ends the solve.  A breakdown
 * H_{j+1,j} <= breakdown_tol * ||H(:, j)|| also ends the cycle (Alg. 1 stops
 * there): it is lucky when the rotated diagonal entry of column j is larger
 * than breakdown_tol * ||H(:, j)|| (the j-column least squares is solved and
 * the solve continues from its iterate), unhappy otherwise (the least squares
 * is singular: column j is dropped, the instance stops with status
 * RTE_EBREAKDOWN).  sweep_dtype sets
 * the arithmetic of the inner A~ applies.  True residuals are FP64, formed
 * as T (G~ + Sigma_s phi) - phi with RTE_F32 (whose b~, which starts the first
 * cycle and scales the stopping test, comes from an FP32 sweep) and as
 * b~ - A~ phi with an FP64 b~ with RTE_F64.
 * phi (device, packed) receives the solution.  stats (host [n_inst]).
 * Failure conventions (per instance; they never abort the batch):
 *  - every region's sigma_t must be finite and > 0 and sigma_s finite and
 *    >= 0: RTE_EINVAL otherwise, before phi is written (checked on the host
 *    before a call that tunes the sweep plans, else by a kernel whose result
 *    is read with ||b~||);
 *  - a non-finite ||b~|| or true residual norm stops that instance with
 *    status RTE_ENONFINITE (its phi is then unspecified); a non-finite Givens
 *    estimate ends its cycle early;
 *  - an unhappy breakdown stops it with status RTE_EBREAKDOWN (phi = the
 *    iterate before the singular column);
 *  - a singular reduced operator A_r(mu) (pivot below 1e-14 max |A_r|, found
 *    once per solve) makes that instance use DSA wherever it would use the
 *    ROM solve, with rom_singular = 1;
 * the call then returns RTE_WNOTCONV (outputs and statistics written).     */
typedef struct {
  int32_t precond;       /* RTE_PC_*                                         */
  int32_t m;             /* Krylov dimension per cycle                       */
  int32_t max_cycles;
  int32_t sweep_dtype;   /* RTE_F32 or RTE_F64                               */
  double rtol;
  int32_t window;        /* ROMSAD window (iterations per cycle using the ROM)*/
  int32_t dsa_inner_max; /* DSA inner GMRES iterations                       */
  int32_t dsa_restart;
  double dsa_inner_tol;
  int32_t keep_krylov;   /* internal use by the offline builders: 0           */
  int32_t window_cycles; /* restart cycles whose first `window` iterations use
                            the ROM / learned correction: 0 = every cycle,
                            k >= 1 = the first k cycles only                 */
  int32_t use_graph;     /* nonzero: each Krylov index's operator application
                            (batched sweep + reduction) is captured once into a
                            HIP graph and replayed; needs a created stream (on
                            the null stream the operator runs eagerly)       */
  int32_t dsa_variant;   /* RTE_DSA_FC or RTE_DSA_PC for every DSA application
                            (the DSA preconditioner and ROMSAD after the
                            window); RTE_DSA_PC needs dsa_restart >= 1      */
  double breakdown_tol;  /* relative breakdown threshold (above); 0 = 1e-14 */
} rte_solve_opts;

typedef struct {
  int32_t iterations;    /* Arnoldi steps over all cycles                     */
  int32_t cycles;
  int32_t sweeps_f32;    /* transport sweeps by precision (b~ included)       */
  int32_t sweeps_f64;
  int32_t pc_rom, pc_dsa, pc_mlp, pc_fallback; /* preconditioner uses        */
  int32_t status;        /* 0 converged, RTE_WNOTCONV, RTE_EBREAKDOWN,
                            RTE_ENONFINITE                                   */
  double true_relres;    /* final FP64 ||b~ - A~ phi|| / ||b~||              */
  double est_relres;     /* last Givens estimate / ||b~||                     */
  int32_t rom_singular;  /* 1: A_r(mu) singular, DSA ran in place of the ROM  */
  int32_t pad;
  double mlp_rom_diff;   /* RTE_PC_MLP: mean over the network's steps of
                            ||W_w (c_MLP - c_ROM)|| / ||W_w c_ROM||, the
                            learned correction against the ROM solve; else 0 */
} rte_solve_stats;

int fgmres_solve(const rte_batch* b, const double* sigma_t, const double* sigma_s, const double* G,
                 const double* inflow, const rte_solve_opts* opts, const rte_rom* rom,
                 const rte_mlp* mlp, const double* mu, int mu_dim, double* phi,
                 rte_solve_stats* stats, void* stream);

/* si_solve: source iteration with synthetic acceleration (section 3), the
 * left-preconditioned Richardson iteration phi <- phi + M_l^{-1} (b~ - A~ phi)
 * from phi = 0, one batched sweep per iteration.  opts->precond: RTE_PC_NONE
 * (plain SI), RTE_PC_DSA, or RTE_PC_ROMSAD (M_ROM for the first `window`
 * iterations, M_DSA after them; rom required).  An instance stops when
 * ||b~ - A~ phi|| <= rtol ||b~|| (the residual of the iterate it returns);
 * opts->max_cycles bounds the iterations; m, window_cycles, use_graph and
 * keep_krylov are ignored.  stats: iterations = preconditioner applications,
 * true_relres = last residual (computed with sweep_dtype sweeps), status 0 or
 * RTE_WNOTCONV (also returned when any instance did not converge).          */
int si_solve(const rte_batch* b, const double* sigma_t, const double* sigma_s, const double* G,
             const double* inflow, const rte_solve_opts* opts, const rte_rom* rom, double* phi,
             rte_solve_stats* stats, void* stream);

/* ---------------------------------------------------------------- ROMSAD
 * A ROM holds the orthonormal psi-space basis U_r ([r][n_ord][ndof], section
 * 4.3) of one grid/quadrature (instance 0 of the batch it was built on), the
 * two sums W_1 = sum_j U_{r,j}, W_w = sum_j w_j U_{r,j}, and the affine
 * pieces of U_r^T A(mu) U_r for region-wise constant cross sections
 * (eq. of the affine assumption):
 *   U^T A U = A_D + sum_R sigma_t,R G_R - sum_R sigma_s,R S_R,
 *   A_D = sum_j U_j^T D_j U_j, G_R = sum_j U_j^T M_R U_j, S_R = W_1^T M_R W_w.
 *
 * romsad_build_greedy: the greedy algorithm of section 4.4.2 on the training
 * instances of `train` (all with the same grid, ordinates and region map):
 * step 1 b~ and eta0 = Sigma_s b~ for all; step 2(a) FP64 FGMRES-DSA solve of
 * the sampled instance to hf_rtol and the xi recurrence; 2(b) window
 * psi-storing sweeps; 2(c) MGS with truncation (App. B, eps_qr) and the
 * reduced operators; step 3 the residual indicator R_mu on every unsampled
 * instance and its argmax (ties: lowest index), until max R_mu < eps_rom or
 * n_giter sampled parameters.  hf_dsa_tol selects the DSA of the 2(a) solves:
 * 0 = one multigrid V-cycle per application, > 0 = V-cycle-preconditioned
 * GMRES to that relative tolerance.  report (host, nullable).               */
typedef struct {
  int32_t n_sampled;
  int32_t sampled[256];      /* training indices in sampling order            */
  double max_residual[256];  /* max R_mu after each greedy iteration          */
  int32_t rank;
  int32_t truncated;
  double seconds_step[5];    /* step 1, 2a, 2b, 2c, 3 wall time               */
} rte_greedy_report;

int romsad_build_greedy(const rte_batch* train, const double* sigma_t, const double* sigma_s,
                        const double* G, const double* inflow, int window, int mu1_index,
                        double eps_rom, int n_giter, double eps_qr, double hf_rtol,
                        double hf_dsa_tol, rte_rom** out, rte_greedy_report* report,
                        void* stream);

/* rte_rom_from_basis: a ROM from a given orthonormal basis U (device
 * [r][n_ord][ndof] of instance 0 of `b`); computes W_1, W_w and the affine
 * pieces on the device.                                                       */
int rte_rom_from_basis(const rte_batch* b, const double* U, int r, rte_rom** out, void* stream);

/* romsad_apply: z = M_ROM^{-1} v = v + W_w (U^T A(mu) U)^{-1} W_1^T Sigma_s v
 * (eq. of the ROM-based SA preconditioner) for every instance of `b`, whose
 * instances must share the ROM's grid, ordinates and region map; mu enters
 * through the per-region cross sections.  A singular reduced operator leaves
 * z = v for that instance and returns RTE_ESINGULAR.                         */
int romsad_apply(const rte_rom* rom, const rte_batch* b, const double* sigma_t,
                 const double* sigma_s, const double* v, double* z, void* stream);

/* A ROM set serves a batch whose instances have different grids or
 * quadratures (the uneven-batch pattern): instance k uses
 * roms[rom_of_instance[k]] (host array [n_inst of b]), which must match its
 * grid, ordinates and region map (RTE_EINVAL otherwise).  The set is accepted
 * wherever fgmres_solve / romsad_apply take a ROM for RTE_PC_ROMSAD (not for
 * the learned correction, export or save); it does not own the member ROMs,
 * which must outlive it.  Destroy with rte_rom_destroy.                     */
int rte_rom_set_create(const rte_batch* b, const rte_rom* const* roms, int n_roms,
                       const int32_t* rom_of_instance, rte_rom** out);
/* Basis size (the largest member's for a set). */
int rte_rom_rank(const rte_rom* rom);
/* Host copies of the ROM's arrays (each pointer nullable): U [r][n_ord][ndof],
 * W1, Ww [r][ndof], AD [r][r], G, S [n_regions][r][r].                        */
int rte_rom_export(const rte_rom* rom, double* U, double* W1, double* Ww, double* AD, double* G,
                   double* S);
int rte_rom_save(const rte_rom* rom, const char* path);
int rte_rom_load(const char* path, rte_rom** out);
void rte_rom_destroy(rte_rom* rom);

/* ---------------------------------------------------------------- learned preconditioner
 * A GELU MLP (n_in -> width x depth -> n_out) mapping the normalised
 * parameter and the normalised reduced residual coefficients g / ||g||,
 * g = W_1^T Sigma_s v, to reduced correction coefficients c / ||g||; inside
 * fgmres_solve (RTE_PC_MLP) the correction is z = v + W_w c for the first
 * `window` iterations of a cycle.  Flexible GMRES admits any such nonlinear
 * preconditioner (section 4.2).  Parameters are FP32, flat, per layer W [out][in]
 * then b [out]; network outputs are y * scale + shift (output standardisation).
 * dtype RTE_BF16: products on the matrix cores with bfloat16 operands and FP32
 * accumulation; RTE_F32: FP32 arithmetic throughout.  All X, Y, T are device
 * arrays of row-major FP32 rows.                                              */
int rte_mlp_create(int n_in, int width, int depth, int n_out, rte_mlp** out);
void rte_mlp_destroy(rte_mlp* m);
/* Glorot-uniform weights from a SplitMix64 stream seeded by `seed`, zero biases,
 * output scale 1 and shift 0, Adam moments cleared (a new network starts at
 * zero and must be initialised or given parameters before training).  Blocking. */
int rte_mlp_init(rte_mlp* m, uint64_t seed);
int64_t rte_mlp_num_params(const rte_mlp* m);
int rte_mlp_set_params(rte_mlp* m, const float* host_params, const float* host_scale,
                       const float* host_shift);
int rte_mlp_get_params(const rte_mlp* m, float* host_params, float* host_scale, float* host_shift);
/* Y [rows][n_out] = network(X [rows][n_in]).                                   */
int rte_mlp_forward(rte_mlp* m, const float* X, float* Y, int rows, int dtype, void* stream);
/* Gradient (device [num_params]) and value (host, nullable) of the mean squared
 * error between network(X) and T over all rows * n_out entries.              */
int rte_mlp_grad(rte_mlp* m, const float* X, const float* T, int rows, int dtype, float* loss,
                 float* grad, void* stream);
/* Adam (lr, 0.9, 0.999, 1e-8) on BF16-matrix-core gradients for `epochs` passes over
 * n rows in shuffled minibatches (SplitMix64-seeded Fisher-Yates).  standardize != 0
 * first sets the output shift/scale to T's column mean and standard deviation.
 * loss_hist (host [epochs], nullable) receives the mean minibatch loss.      */
/* One Adam step (Kingma and Ba; lr, 0.9, 0.999, 1e-8, bias-corrected with the
 * network's own step count, which it increments) on the parameters with the
 * given gradient (device [num_params] FP32), e.g. one from rte_mlp_grad; the
 * moments are the network's (cleared by init / set_params).                  */
int rte_mlp_adam_step(rte_mlp* m, const float* grad, float lr, void* stream);
int rte_mlp_train(rte_mlp* m, const float* X, const float* T, int n, int epochs, int batch,
                  float lr, uint64_t seed, int standardize, float* loss_hist, void* stream);
/* Training data from FGMRES runs (section 4.4.1): solve every instance with
 * `opts`, recover xi^(l) = A~^{-1} v^(l), l < window, from the first cycle (the
 * xi recurrence), and emit rows X = [mu, g/||g||] with g = W_1^T Sigma_s v^(l) and
 * targets T = c_opt / ||g||, c_opt the least-squares coefficients of
 * xi^(l) - v^(l) (the ideal scalar-flux correction) in span(W_w).  mu: device [n_inst][mu_dim]
 * (FP64, already normalised).  X: [n_inst*window][mu_dim + r], T:
 * [n_inst*window][r], valid: device int32 [n_inst*window] (row usable).     */
int rte_mlp_snapshots(const rte_batch* b, const double* sigma_t, const double* sigma_s,
                      const double* G, const double* inflow, const rte_rom* rom,
                      const rte_solve_opts* opts, const double* mu, int mu_dim, float* X,
                      float* T, int32_t* valid, void* stream);

/* ---------------------------------------------------------------- profiling
 * HIP-event timing of the library's hot kernels for benchmarking.
 * rte_prof_enable(1) starts recording (and clears earlier records); every
 * launch of a profiled kernel is bracketed by two events on its stream.
 * rte_prof_read synchronises on the recorded events and returns, for one
 * slot, the number of launches, their summed duration in milliseconds and
 * the summed work units (sweeps: cell-ordinates processed).  A launch that
 * found every instance already converged (FGMRES enqueues a step before it
 * knows the outcome of the previous one) is not counted.
 * Slots: 0 FP64 sweep, 1 FP32 sweep, 2 DSA operator, 3 Arnoldi MGS, 4 ROM.  */
int rte_prof_enable(int on);
int rte_prof_read(int slot, int64_t* launches, double* total_ms, double* total_units);
/* Enqueues an empty kernel (rte::k_region_marker, argument id) on `stream`, so
 * that an external kernel trace can locate a region between two marks.      */
int rte_prof_mark(int id, void* stream);
/* Operator applications captured into HIP graphs by fgmres_solve (use_graph)
 * since the library was loaded: a new capture is made whenever a cached graph
 * would refer to reallocated buffers (a new sweep plan, grown partial buffers)
 * or to other arguments.                                                     */
int64_t rte_graph_captures(void);

#ifdef __cplusplus
}
#endif
#endif
