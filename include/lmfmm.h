/*
 * lmfmm.h -- C ABI of the layered-media dyadic fast multipole library
 * (MI355X / gfx950, fp64).
 *
 * The library evaluates, for current elements J_j at source points x_j and
 * target points y_i in a horizontally layered medium,
 *
 *     A(y_i) = sum_j G(y_i, x_j) J_j ,
 *
 * where G is the layered electric dyadic Green's function: the free-space
 * dyadic (I + grad grad / k^2) e^{ikR}/(4 pi R) when source and target share a
 * layer (skipped for coincident points), plus the interface reaction field
 * (all pairs).  The operation is the layered sum of the paper's Sec. 3.3
 * (problem statement of the FMM in layered media) in the standard
 * orientation: target first, source second (Sec. 3.1).  The reaction field is
 * evaluated by one FMM per reaction component (Sec. 3.3), with M2L tables
 * from Chebyshev-expanded associated Legendre functions and Sommerfeld
 * quadrature on a deformed contour (Sec. 3.4); the free-space part by a
 * Helmholtz FMM with the dyadic operator applied to the local expansion
 * (Sec. 2).
 *
 * Medium: layers 0..n-1 from top to bottom, interfaces z = d[0] > d[1] > ...
 * (n-1 values), real wavenumbers k[l] > 0, relative permeabilities mu[l] > 0
 * (default 1) and eps proportional to k^2 / mu (only ratios enter the
 * interface conditions of the paper's two 1-D problems, Sec. 3.1).
 * A point with d[l] < z < d[l-1] lies in layer l.  Time convention: outgoing
 * e^{+ikR}, Im k_z >= 0.
 *
 * Errors: every function returns an int status, LM_OK (0) on success or a
 * negative code; lm_last_error() describes the last failure on a context.
 * On LM_EINVAL, LM_EDOMAIN and LM_ESTATE no output is touched.  Nothing
 * throws across the ABI.  One context must not be used from two host
 * threads at once; distinct contexts are independent.  The evaluations of
 * one context share its work buffers and the work-queue counters of its
 * persistent launches, so they must not overlap on the device either: issue
 * them on one stream, or order their streams.
 *
 * Ownership: the caller owns every array it passes.  Positions are host
 * arrays, copied by lm_build.  Currents and outputs are device arrays of
 * interleaved complex128 (re, im) values, 16-byte aligned; the library never
 * keeps them.  The context owns its device tables and work buffers until
 * lm_destroy (or the next lm_build / lm_set_layers / lm_set_params).
 */
#ifndef LMFMM_H
#define LMFMM_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LM_OK 0
#define LM_EINVAL (-1)   /* invalid argument (null pointer, size, range)            */
#define LM_EDOMAIN (-2)  /* invalid medium or geometry (interfaces, k, point on an  */
                         /* interface, points too close to an interface)            */
#define LM_ESTATE (-3)   /* wrong call order                                        */
#define LM_ENOMEM (-4)   /* device allocation failed                                */
#define LM_EHIP (-5)     /* HIP runtime error (message carries hipGetErrorString)   */
#define LM_EACCURACY (-6) /* a quadrature rule of the build cannot reach the         */
                          /* accuracy requested in lm_params.tol                     */

#define LM_PMAX_ORDER 20

typedef struct lm_ctx lm_ctx;

typedef struct {
  int p;              /* reaction-field expansion order, 1..20                      */
  int p_free;         /* free-space expansion order, 0 => p                          */
  int free_depth;     /* free-space octree leaf level, 0 => chosen by a cost model   */
  int max_depth;      /* cap of the reaction-tree refinement next to interfaces      */
  int gamma1_panels;  /* Gauss-Legendre panels (16 nodes each) on the contour piece  */
                      /* from 0 to a in the fourth quadrant (Sec. 3.4); default 4;   */
                      /* the direct near field uses at most 2 within the series     */
                      /* range of its Bessel functions                              */
  double contour_a;   /* end point a of that piece on the real axis, 0 => 1.5 max k  */
  double tail_digits; /* the real tail [a, kcut] of the Sommerfeld integrals ends at */
                      /* kcut = a + (3p + tail_digits) / dz_min                       */
  int components;     /* bit 0: free-space part, bit 1: reaction field (3 = both)    */
  int m2l_adapt;      /* 1: each M2L offset uses the least order whose truncation   */
                      /* bound (separation ratio^(p+1)) does not exceed that of the */
                      /* instance's worst admissible pair, lowered by m2l_margin   */
                      /* decades; 0: order p everywhere                            */
  double m2l_margin;  /* see m2l_adapt (default 3)                                  */
  int react_s2t;      /* 0: reaction trees are refined next to the gap between      */
                      /* images and effective locations until no source and        */
                      /* target leaves are adjacent (every reaction interaction   */
                      /* is an M2L).  1 (default): a tree stops one level earlier */
                      /* where a cost model finds the direct near field cheaper   */
                      /* than that level's M2L work; 2: always one level earlier; */
                      /* 3: every reaction pair direct (single-box reaction trees:*/
                      /* the decomposition of Sec. 3.1 without expansions).       */
                      /* Leaves that stay adjacent interact directly through the  */
                      /* component's Sommerfeld integral (S2T, Sec. 3.3/3.4).     */
  int m2l_variant;    /* tile shape of the M2L GEMM kernel: -1 (default) tunes each */
                      /* launch of the schedule on its first eager evaluation and  */
                      /* keeps the fastest; 0..LM_M2L_VARIANTS-1 fixes one (64-row  */
                      /* tiles; 0: 8 values of k per LDS chunk; 1: 4 values,       */
                      /* double-buffered; 2: 8 values, double-buffered).  All      */
                      /* variants give bitwise equal results.                      */
  double tol;         /* requested relative accuracy, 0 (default): no check.  With  */
                      /* tol > 0, lm_build returns LM_EACCURACY when a quadrature   */
                      /* rule of the plan is coarser than tol: the real tail of the*/
                      /* M2L tables' Sommerfeld integrals (cut where the integrand */
                      /* has decayed by e^-tail_digits beyond the growth of the     */
                      /* Legendre products), the direct reaction pairs (tail cut at*/
                      /* 28 e-folds and two panels on the first contour piece,     */
                      /* about 2.5e-9 of a pair's field), or fewer than three      */
                      /* panels on that piece (about 2e-9).  The expansions'       */
                      /* truncation error is not bounded a priori: it is set by p  */
                      /* (recorded errors per order: see the tests).                */
  int host_trees;     /* 0 (default): lm_build keys and sorts the records of every */
                      /* octree and forms its boxes on the device (Morton keys,    */
                      /* radix sort, box starts per level); 1: on the host.  Both  */
                      /* give the same plan (the interaction lists and tables are  */
                      /* built on the host).                                       */
} lm_params;

#define LM_M2L_VARIANTS 3

/* Fills *prm with the defaults (p = 12, p_free = p, automatic depths, m2l_adapt = 1,
 * m2l_margin = 3, gamma1_panels = 4, react_s2t = 1, m2l_variant = -1, tol = 0,
 * host_trees = 0). */
int lm_default_params(lm_params* prm);

/* Creates a context bound to HIP device `hip_device`.  *out is owned by the
 * caller and released with lm_destroy.  LM_EHIP if the device does not exist. */
int lm_create(lm_ctx** out, int hip_device);

/* Releases the context and every device buffer it owns. */
int lm_destroy(lm_ctx* ctx);

/* Message of the last failure on ctx (valid until the next call on ctx). */
const char* lm_last_error(const lm_ctx* ctx);

/* Sets the layered medium (Sec. 3.1).  d_host: n_layers-1 interfaces,
 * strictly decreasing; k_host: n_layers wavenumbers, finite and > 0; mu_host:
 * NULL (all 1) or n_layers relative permeabilities, finite and > 0 (they
 * enter the TE and TM interface conditions and scale the TM part of the
 * reaction field by mu_target / mu_source).  Host arrays, copied.  LM_EDOMAIN
 * for an invalid value.  Invalidates a previous lm_build. */
int lm_set_layers(lm_ctx* ctx, int n_layers, const double* d_host, const double* k_host,
                  const double* mu_host);

/* Sets the method parameters (copied).  Invalidates a previous lm_build. */
int lm_set_params(lm_ctx* ctx, const lm_params* prm);

/* Builds trees, interaction lists and every translation table for the
 * given points: src_xyz [n_src][3] and tgt_xyz [n_tgt][3] are HOST arrays of
 * fp64 coordinates (may be the same array).  Runs the table kernels on
 * `stream` (a hipStream_t, NULL = default stream) and synchronises it once
 * before returning.  LM_EDOMAIN if a point lies on an interface
 * (|z - d| <= 1e-12 max(1,|d|)) or closer to one than the refinement cap
 * allows; LM_ESTATE if no medium was set; LM_EACCURACY if lm_params.tol is
 * set and a quadrature rule of the plan cannot reach it. */
int lm_build(lm_ctx* ctx, int64_t n_src, const double* src_xyz, int64_t n_tgt,
             const double* tgt_xyz, void* stream);

/* Builds several independent geometries into one plan, so that every later
 * lm_evaluate / lm_evaluate_adjoint / lm_grad_src_xyz processes all of them
 * together: each pass launches once for all geometries (the leaf passes once
 * per group of instances that share no target point: free space, and each
 * reaction component type), so many small problems run at the occupancy of
 * one large one.  Geometry g owns the sources src_off[g] .. src_off[g+1]-1 and
 * the targets tgt_off[g] .. tgt_off[g+1]-1 of the concatenated HOST arrays
 * src_xyz / tgt_xyz; only sources and targets of the same geometry interact
 * (each geometry is the sum of Sec. 3.3 on its own points, with its own
 * trees).  src_off, tgt_off: HOST int64 [n_geom+1], starting at 0,
 * non-decreasing; J and A of the evaluations are the concatenations in the
 * same order.  Otherwise as lm_build.  LM_EINVAL for bad offsets. */
int lm_build_batch(lm_ctx* ctx, int n_geom, const int64_t* src_off, const double* src_xyz,
                   const int64_t* tgt_off, const double* tgt_xyz, void* stream);

/* Evaluates A = G J for n_rhs right-hand sides on the built geometry.
 * J: DEVICE complex128 [n_rhs][n_src][3]; A: DEVICE complex128
 * [n_rhs][n_tgt][3], overwritten.  All work is enqueued on `stream`
 * (asynchronous: the call returns before the results are ready).  The
 * summation order is fixed, so repeated calls give bitwise equal results. */
int lm_evaluate(lm_ctx* ctx, int n_rhs, const void* J, void* A, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as lm_evaluate, A = G J, with every work buffer of the
 * evaluation (multipole and local expansions, P2M partials, M2L outputs) in
 * a static device array of the library, LM_NOALLOC_SCRATCH_BYTES per GPU,
 * held from the library's load until the process ends.  The call allocates
 * nothing (no hipMalloc, hipFree, events or library allocations); the plan
 * and its tables are allocated by lm_build as for lm_evaluate, which also
 * prepares this call's single-right-hand-side M2L schedule.  Right-hand
 * sides are evaluated one after the other, each bitwise equal to
 * lm_evaluate's column.  M2L tile shapes are not autotuned here (the
 * m2l_variant parameter if fixed, else variant 0; all give the same bits).
 * J: DEVICE complex128 [n_rhs][n_src][3]; A: DEVICE complex128
 * [n_rhs][n_tgt][3], overwritten; asynchronous on `stream`.  All calls on
 * one GPU share its array: calls that overlap in time on one GPU (from
 * several host threads or streams) race and give wrong results.  LM_ENOMEM,
 * with nothing written, when the build's work buffers for one right-hand
 * side exceed the array (lm_last_error gives the bytes needed); LM_EHIP if
 * the array's device address could not be obtained (lm_create looks it up
 * once per device); otherwise errors as lm_evaluate. */
#define LM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int lm_evaluate_noalloc(lm_ctx* ctx, int n_rhs, const void* J, void* A, void* stream);

/* Magnetic field of the same currents: H = G_H J with the magnetic dyadic of
 * Sec. 3.1 (the J6..J9 form), normalised as G_H(x, y) = (1/mu(x)) curl_x
 * G(x, y) (Faraday's law; in free space curl (g I) q = grad g x q, the
 * paper's free-space G_H without its constant i/(omega mu_0) factor).
 * Evaluated as the curl of the electric field on the same plan: the far
 * field by exact derivatives of the local expansions (ladder relations of
 * the regular wave functions), the free-space near field in closed form,
 * and the directly evaluated reaction pairs by the Sommerfeld integrals of
 * the J6..J9 form.  J: DEVICE complex128 [n_rhs][n_src][3]; H: DEVICE
 * complex128 [n_rhs][n_tgt][3], overwritten.  Asynchronous, errors and
 * determinism as lm_evaluate. */
int lm_evaluate_h(lm_ctx* ctx, int n_rhs, const void* J, void* H, void* stream);

/* Adjoint evaluation (the conjugate transpose of lm_evaluate's operator):
 *     gJ_j = sum_i G(x_i, x_j)^H gA_i      (x_i targets, x_j sources),
 * for n_rhs vectors.  gA: DEVICE complex128 [n_rhs][n_tgt][3]; gJ: DEVICE
 * complex128 [n_rhs][n_src][3], overwritten.  Computed through the
 * reciprocity of the layered Green's function, G(x, y) mu(y) = G(y, x)^T mu(x)
 * (Sec. 3.3; mu(x) the permeability of x's layer): gJ_j = conj(G~ conj(mu gA))_j
 * / mu_j with G~ the forward sum with sources and targets exchanged.  When the source and target arrays given to lm_build
 * are the same point set this is the built FMM itself; otherwise a second
 * FMM with the roles exchanged is built on the first call (which then
 * synchronises `stream` once and allocates; later calls reuse it).  The
 * result equals G^H gA to the FMM's accuracy (it is the adjoint of the exact
 * operator, not the exact transpose of the discrete FMM).  Asynchronous on
 * `stream` otherwise; errors as lm_evaluate. */
int lm_evaluate_adjoint(lm_ctx* ctx, int n_rhs, const void* gA, void* gJ, void* stream);

/* Gradient with respect to the source positions (targets fixed) of a real
 * loss L whose gradient with respect to A is gA (gA = dL/dRe A + i dL/dIm A,
 * the convention of complex autograd):
 *     gX_j = sum_r Re sum_i gA_{r,i}^H (d/dx_j G(x_i, x_j)) J_{r,j},
 * summed over the n_rhs right-hand sides.  J: DEVICE complex128
 * [n_rhs][n_src][3] (the currents of the forward evaluation); gA: DEVICE
 * complex128 [n_rhs][n_tgt][3]; gX: DEVICE fp64 [n_src][3], overwritten.
 * Uses the same reciprocity as lm_evaluate_adjoint: the field of the
 * currents mu conj(gA) placed at the targets is differentiated at the source
 * points (ladder relations of the regular wave functions on the local
 * expansions, closed-form derivative of the free-space dyadic in the near
 * field, Bessel-ladder and d/dz derivatives inside the Sommerfeld integrals
 * of the directly evaluated reaction pairs), contracted with J and divided
 * by mu of the source's layer.  Build, stream and error behaviour as
 * lm_evaluate_adjoint. */
int lm_grad_src_xyz(lm_ctx* ctx, int n_rhs, const void* J, const void* gA, double* gX, void* stream);

/* Phase timing.  lm_set_timing(ctx, 1) (re)starts recording HIP events on
 * the evaluation stream between the phases of every following lm_evaluate
 * and around every launch of the M2L GEMM kernel, the M2L reduction and the
 * near-field kernels; lm_timings() waits for the recorded events and writes
 * up to n values, summed over the timed evaluations: the milliseconds of
 * each phase (indices LM_PHASE_*), the number of timed evaluations (index
 * LM_PHASES), and for each of those kernels the milliseconds spent in it and
 * the number of its launches (LM_TIMING_*_MS, LM_TIMING_*_LAUNCHES; the M2L
 * GEMM and reduction are parts of LM_PHASE_M2L, the near-field kernels of
 * LM_PHASE_P2P). */
int lm_set_timing(lm_ctx* ctx, int enable);
int lm_timings(lm_ctx* ctx, double* out_host, int n);

#define LM_PHASE_CLEAR 0   /* zeroing of A and of the local expansions           */
#define LM_PHASE_P2M 1
#define LM_PHASE_M2M 2
#define LM_PHASE_M2L 3     /* M2L GEMM launches and the per-target reductions    */
#define LM_PHASE_L2L 4
#define LM_PHASE_L2P 5
#define LM_PHASE_P2P 6     /* near field: free-space P2P and reaction S2T         */
#define LM_PHASES 7
#define LM_TIMING_M2L_GEMM_MS (LM_PHASES + 1)
#define LM_TIMING_M2L_GEMM_LAUNCHES (LM_PHASES + 2)
#define LM_TIMING_M2L_REDUCE_MS (LM_PHASES + 3)      /* per-target sums of the M2L outputs  */
#define LM_TIMING_M2L_REDUCE_LAUNCHES (LM_PHASES + 4)
#define LM_TIMING_P2P_MS (LM_PHASES + 5)             /* free-space near field                */
#define LM_TIMING_P2P_LAUNCHES (LM_PHASES + 6)
#define LM_TIMING_S2T_MS (LM_PHASES + 7)             /* direct reaction pairs               */
#define LM_TIMING_S2T_LAUNCHES (LM_PHASES + 8)
#define LM_TIMINGS_COUNT (LM_PHASES + 9)

/* The M2L GEMM variant of each launch of the evaluation schedule for n_rhs
 * right-hand sides (one launch per chunk, in evaluation order).  HOST arrays:
 * variant_host [cap] receives the chosen variant (-1: not tuned yet),
 * ms_host [cap * LM_M2L_VARIANTS] the autotuner's time of each variant in
 * milliseconds (negative: not measured).  Returns the number of launches
 * (0 when no evaluation with n_rhs has run yet) or a negative error. */
int lm_m2l_variants(const lm_ctx* ctx, int n_rhs, int* variant_host, double* ms_host, int cap);

/* Statistics of the current build (host array of n doubles, indices below). */
int lm_stats(const lm_ctx* ctx, double* out_host, int n);

#define LM_STAT_N_FREE_INST 0
#define LM_STAT_N_REACT_INST 1
#define LM_STAT_M2L_PAIRS_FREE 2
#define LM_STAT_M2L_PAIRS_REACT 3
#define LM_STAT_P2P_PAIRS 4          /* free-space near-field point pairs          */
#define LM_STAT_N_CASES 5            /* reaction M2L table cases                   */
#define LM_STAT_N_NODES 6            /* Sommerfeld quadrature nodes                */
#define LM_STAT_MAT_BYTES 7
#define LM_STAT_ME_BYTES_PER_RHS 8
#define LM_STAT_LE_BYTES_PER_RHS 9
#define LM_STAT_T_PLAN_MS 10
#define LM_STAT_T_UPLOAD_MS 11
#define LM_STAT_T_TABLES_MS 12
#define LM_STAT_N_SRC_BOXES 13
#define LM_STAT_N_TGT_BOXES 14
#define LM_STAT_N_M2L_CLASSES 15
#define LM_STAT_N_M2L_TILES_1RHS 16
#define LM_STAT_M2L_CMAC_USEFUL 17   /* complex multiply-adds of the M2L per rhs   */
                                     /* (reaction: the even and odd blocks of the  */
                                     /* mirror-adapted tensor)                     */
#define LM_STAT_M2L_CMAC_EXEC 18     /* same, rows padded to 64-row GEMM tiles     */
#define LM_STAT_N_LEAVES_P2M 19
#define LM_STAT_FREE_DEPTH 20
#define LM_STAT_S2T_PAIRS 21         /* reaction near-field (S2T) point pairs        */
#define LM_STAT_M2L_FLOP_EXEC 22     /* MFMA flops the M2L GEMM executes per rhs (16x16 */
                                     /* tiles inside the orders and pair counts, k padded */
                                     /* to 16, three real MFMAs per complex step)        */
#define LM_STAT_P2M_FLOPS 23         /* algorithmic flops per rhs: 8 per complex          */
#define LM_STAT_M2M_FLOPS 24         /* multiply-add of the expansion sums (P2M, L2P)     */
#define LM_STAT_L2L_FLOPS 25         /* and the dense translations (M2M, L2L)             */
#define LM_STAT_L2P_FLOPS 26
#define LM_STAT_REDUCE_BYTES 27      /* bytes the M2L reduction must move per rhs         */
#define LM_STAT_S2T_NODE_EVALS 28    /* quadrature nodes summed over the direct reaction  */
                                     /* pairs (each pair stops at its own cut)            */
#define LM_STAT_M2L_CMAC_DENSE 29    /* complex multiply-adds of the same M2L per rhs in  */
                                     /* the dense spin-basis form (three P x 3P products  */
                                     /* per reaction pair, Sec. 3.3)                      */
#define LM_STAT_P2P_KERNEL_EVALS 30  /* free-space near field: evaluations of the pair    */
                                     /* kernel (when the targets are the sources, one per */
                                     /* unordered pair of different leaves, and every     */
                                     /* ordered pair inside a leaf; else P2P_PAIRS)       */
#define LM_STAT_TREE_RECORDS 31      /* records of every octree (points of each tree) */
#define LM_STAT_TREE_SORT_MS 32      /* device time of their keys and sort (0 when    */
                                     /* sorted on the host)                           */
#define LM_STAT_PLAN_DIGEST_HI 33    /* 64-bit hash of the plan (trees, lists, M2L    */
#define LM_STAT_PLAN_DIGEST_LO 34    /* schedule, table cases, nodes), its two halves:*/
                                     /* equal plans give equal values                 */
#define LM_STATS_COUNT 35

/* ---- iterative solve over the evaluation ---- */

/* Restarted GMRES for the coupled-dipole system on the built point set
 *     (D - G) X = B,      D = diag(d_j) on the three components of point j,
 * with G the layered sum that lm_evaluate applies: the matrix-vector product
 * of an integral-equation solver, the use the paper's introduction gives for
 * the layered sum (Sec. 3.3 writes the sum over the first argument with
 * method-of-moments solvers in view; by the reciprocity stated there it is
 * the same operator).  Each right-hand side is solved to its own stopping test,
 * in lockstep with the others, so that every operator application is one
 * batched lm_evaluate of all n_rhs vectors.
 *
 * The build must have the same point array as sources and targets (LM_ESTATE
 * otherwise).  diag: DEVICE complex128 [n] or NULL (D = 0); B: DEVICE
 * complex128 [n_rhs][n][3]; X: DEVICE complex128 [n_rhs][n][3], the initial
 * guess on entry (zero it for the usual start), the last iterate on return;
 * X must not overlap B or diag (B and diag are only read).
 * Stopping test per column: ||B - (D - G) X|| <= tol ||B|| (2-norm), checked
 * on the true residual at the end of each restart cycle; a column with B = 0
 * returns X = 0.  restart: Krylov dimension per cycle, 1..LM_SOLVE_MAX_RESTART;
 * max_iter: total Arnoldi steps (operator applications not counting residual
 * checks), >= 1.  relres_host: NULL or host double [n_rhs], the final true
 * relative residuals; info: NULL or host struct, filled.  Orthogonalisation is
 * classical Gram-Schmidt applied twice, by deterministic reductions, so the
 * result is bitwise repeatable.  The call synchronises `stream` several times
 * per iteration (host decisions) and allocates the Krylov basis, (restart + 1)
 * n_rhs n 48 bytes, on first use or growth (kept until the next build).
 * Returns LM_OK also when max_iter ends the iteration before the stopping
 * test holds (info->converged = 0); errors as lm_evaluate. */
#define LM_SOLVE_MAX_RESTART 64

typedef struct {
  int iters;          /* Arnoldi steps taken                                     */
  int matvecs;        /* operator applications, residual checks included          */
  int cycles;         /* restart cycles                                          */
  int converged;      /* 1 if every column met the stopping test                   */
  double ms_total;    /* time of the call on `stream` (HIP events)                 */
  double ms_matvec;   /* time of the operator applications within it               */
  double ms_krylov;   /* time of the vector kernels (products, updates, norms)     */
  double krylov_bytes;/* bytes those kernels must move (each vector read or written once per pass) */
} lm_solve_info;

int lm_solve(lm_ctx* ctx, int n_rhs, const void* diag, const void* B, void* X, double tol, int restart,
             int max_iter, double* relres_host, lm_solve_info* info, void* stream);

/* Self-test of the device arithmetic used by the near field (no context):
 * for each x_dev[i] writes out_dev[6i..6i+5] = sin x, cos x (the reduced-range
 * routine of the near field), 1/sqrt(x^2 + 1e-300) (refined estimate), the
 * same by the library's sqrt and division, and J0(|x|), J1(|x|) (the
 * polynomial forms used on the real tail of the direct reaction near field).
 * DEVICE arrays x [n], out [6n]; enqueued on `stream`.  For tests. */
int lm_selftest_math(int64_t n, const double* x_dev, double* out_dev, void* stream);

/* ---- host-only helpers (no GPU needed), for tests of the host logic ---- */

/* Reaction components of a medium (Sec. 3.1): returns their count and writes
 * up to `cap` records of 8 ints: target layer, source layer, arrives-up,
 * leaves-up, sign s, target map slope (+1 identity / -1 reflection), source
 * map slope, 0. */
int lm_host_components(int n_layers, const double* d, const double* k, int* out, int cap);

/* Appendix A: C[j][s] with T_j(a x + b) = sum_s C[j][s] T_s(x), j,s <= jmax,
 * written row-major with stride jmax+1 into out[(jmax+1)^2]. */
int lm_host_cheb_affine(int jmax, double a, double b, double* out);

/* Appendix B: B[tri(n,m)][k] with P^m_n(cos t) = tau_nm(t) sum_k B^k T_k(cos 2t)
 * for 0 <= m <= n <= p (orthonormal Legendre functions, Condon-Shortley
 * phase); tri(n,m) = n(n+1)/2 + m; *stride receives the row stride. */
int lm_host_legendre_cheb(int p, double* out, int* stride);

/* The host logic of lm_solve (Arnoldi with Gram-Schmidt applied twice, Givens
 * least squares, restarts, per-column stopping tests, right-hand sides in
 * lockstep) on a dense complex system A X = B of order n held in host
 * memory: A row-major complex128 [n][n], B and X complex128 [n_rhs][n]
 * (X: initial guess in, solution out).  Same arguments and results as
 * lm_solve; *iters receives the Arnoldi steps and relres [n_rhs] the final
 * true relative residuals (LM_OK also when max_iter ends the iteration
 * first: compare relres with tol).  LM_EINVAL, with nothing written, for
 * n < 1, n_rhs outside 1..4096, a null A, b or x, restart outside
 * 1..LM_SOLVE_MAX_RESTART, max_iter < 1, or tol not finite and > 0. */
int lm_host_gmres_dense(int n, int n_rhs, const double* A, const double* b, double* x, double tol, int restart,
                        int max_iter, int* iters, double* relres);

/* Plans a build on the host only (trees, lists, tables sizes) and returns
 * lm_stats-style statistics; errbuf receives the planner's message on failure. */
int lm_host_plan_stats(int n_layers, const double* d, const double* k, const lm_params* prm,
                       int64_t n_src, const double* src_xyz, int64_t n_tgt, const double* tgt_xyz,
                       double* out, int n, char* errbuf, int errlen);

/* For tests of the planner's external-sort route (the one lm_build takes
 * with the octree sort on the device), on the host only: plans the
 * geometries (offsets as lm_build_batch) with the octree records keyed and
 * sorted outside the planner by a plain host implementation of that
 * route's contract (Morton keys of the lattice cells, a stable sort per
 * tree), and with the planner's own sort, and writes both plans' 64-bit
 * digests (as lm_stats PLAN_DIGEST) to digest[0] and digest[1].  Errors as
 * lm_host_plan_stats. */
int lm_host_plan_digests(int n_layers, const double* d, const double* k, const lm_params* prm, int n_geom,
                         const int64_t* src_off, const double* src_xyz, const int64_t* tgt_off,
                         const double* tgt_xyz, uint64_t* digest, char* errbuf, int errlen);

#ifdef __cplusplus
}
#endif
#endif /* LMFMM_H */
