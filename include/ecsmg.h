/*
 * ecsmg.h -- C ABI of the MI355X (gfx950) multigrid-preconditioned Krylov
 * solver for the exterior-complex-scaled (ECS) Helmholtz problem
 *
 *     (-Lap - k^2(x)) u = f      on a box, u = 0 at the end of every contour,
 *
 * following bin Zubair, Reps and Vanroose, "A preconditioned iterative solver
 * for the scattering solutions of the Schroedinger equation" (model problem
 * of Sec. 2, discretisation of Sec. 3, preconditioners and multigrid of
 * Sec. 4, Krylov outer solve of Sec. 5).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Grids are node based.  nodes[a] counts the nodes of axis a INCLUDING the
 *    two Dirichlet end nodes; 2D problems use axes 0 (x) and 1 (y) and ignore
 *    nodes[2].  Real node coordinates are x_i = lo + i (hi - lo)/(nodes - 1).
 *  - Arrays are device pointers, contiguous, node-major with x fastest:
 *    index = (k * nodes[1] + j) * nodes[0] + i.  Complex arrays are
 *    interleaved (re, im): complex128 (16 B/node) unless stated otherwise.
 *    Boundary entries of inputs are ignored; boundary entries of outputs are
 *    written as zero.
 *  - All device memory is owned by the caller.  The library keeps only host
 *    metadata; its device scratch lives in the workspace the caller hands to
 *    ecs_set_workspace().  k^2 is borrowed until the next ecs_set_k2() or
 *    ecs_destroy().
 *  - Work is enqueued on the HIP stream given to ecs_create().  Calls that
 *    return results to the host (solves, stats) synchronise that stream.
 *  - A context is not thread safe; use one per problem and thread.
 *  - Every call returns an ecs_status; on failure ecs_last_error() gives a
 *    message.  No call aborts the process.
 */
#ifndef ECSMG_H
#define ECSMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ECS_OK = 0,
  ECS_NOT_CONVERGED = 1,  /* maxit reached; x holds the last iterate, stats valid  */
  ECS_EINVAL = -1,        /* bad argument (size, dtype, order, parameter range)   */
  ECS_ENOMEM = -2,        /* workspace too small                                  */
  ECS_EDEVICE = -3,       /* HIP runtime error (message in ecs_last_error)        */
  ECS_EBREAKDOWN = -4,    /* Krylov breakdown or NaN/Inf in the iteration         */
  ECS_ESTATE = -5         /* call-order violation (e.g. solve before workspace)   */
} ecs_status;

typedef struct ecs_ctx ecs_ctx;

enum { ECS_F64 = 0, ECS_F32 = 1 };
enum { ECS_SIDE_LO = 0, ECS_SIDE_HI = 1 };
enum { ECS_BC_DIRICHLET = 0, ECS_BC_ECS = 1 };
/* preconditioner operators of Sec. 5 */
enum { ECS_PREC_NONE = 0, ECS_PREC_LAPLACE = 1, ECS_PREC_CSL = 2, ECS_PREC_CSG = 3, ECS_PREC_QD = 4 };
enum { ECS_SMOOTH_JACOBI = 0, ECS_SMOOTH_RBGS = 1 };
enum { ECS_KRYLOV_GMRES = 0, ECS_KRYLOV_FGMRES = 1, ECS_KRYLOV_BICGSTAB = 2 };
enum { ECS_OP_A = 0, ECS_OP_AT = 1, ECS_OP_M = 2 };
/* Gram-Schmidt of the GMRES / FGMRES Arnoldi step (see ecs_solve_desc) */
enum { ECS_ORTH_DCGS2 = 0, ECS_ORTH_CGS2 = 1, ECS_ORTH_CGS1 = 2, ECS_ORTH_CGS2_SELECTIVE = 3 };

/* Preconditioner M and the multigrid cycle that approximately inverts it
 * (Sec. 4.2, Algorithm 1; operators of Sec. 5):
 *   LAPLACE  M = -Lap
 *   CSL      M = -Lap + (beta1 + i beta2) k^2
 *   CSG      M = Z on the grid rotated by e^{i theta_alpha}
 *   QD       M = (1 - i) I + Z / |Re lambda0| with |Re lambda0| =
 *            |re_lambda0| (Sec. 5 quotes Re lambda0 as negative numbers);
 *            re_lambda0 = 0 selects max k^2 (the rough rule of Sec. 5)
 *   NONE     no preconditioner (Krylov on A alone)
 * smoother: omega-Jacobi or red-black SOR ("omega-red-black Jacobi"),
 * red = nodes with i+j(+k) even first.  gamma_f = gamma_c = 1 is the V cycle.
 * coarsest_nodes: nodes per axis of the coarsest grid (>= 3); every axis must
 * satisfy (nodes - 1) = (coarsest_nodes - 1) * 2^(levels - 1).
 * vcycle_dtype: ECS_F64 or ECS_F32 (the whole cycle in complex FP32). */
typedef struct {
  int kind;
  double beta1, beta2;
  double theta_alpha;
  double re_lambda0;
  int smoother;
  double omega;
  int nu1, nu2;
  int gamma_f, gamma_c;
  int coarsest_nodes;
  int vcycle_dtype;
} ecs_prec_desc;

/* Krylov settings (Sec. 5).  Right preconditioning, x0 = 0 unless
 * x_is_guess, Hermitian inner products, stop when the TRUE relative residual
 * ||b - A x||_2 / ||b||_2 <= rtol (interior nodes).
 *   GMRES(restart):  x = x0 + M^{-1} V y
 *   FGMRES(restart): x = x0 + Z y, z_j = M^{-1} v_j stored in vcycle_dtype;
 *                    inner > 0 makes the preconditioner `inner` iterations of
 *                    Bi-CGSTAB (from zero, on A, right-preconditioned by the
 *                    cycle) in the cycle's dtype: the nested mixed form with
 *                    vcycle_dtype = ECS_F32, the same algorithm in FP64
 *                    with ECS_F64.
 *   BICGSTAB:        van der Vorst's method, shadow residual r^ = r0.
 * maxit counts outer iterations (Arnoldi steps / Bi-CGSTAB iterations).
 * history: optional host array of history_len doubles receiving the
 * estimated relative residual after each iteration.
 * orth: the Arnoldi step's Gram-Schmidt (GMRES, FGMRES; Hermitian inner
 * products): classical Gram-Schmidt with a second pass -- delayed by one step
 * (ECS_ORTH_DCGS2, the default 0: the newest basis vector is
 * reorthogonalised in the same two passes over the basis that orthogonalise
 * the next direction, so every vector gets two passes for the memory traffic
 * of one; the rotated Hessenberg column is not corrected for the delayed
 * pass, a change of the size of the first pass's rounding error, and the
 * preconditioner sees the vector before its second pass), always
 * (ECS_ORTH_CGS2), when the first pass leaves less than 1/sqrt(2) of the new
 * vector's norm (ECS_ORTH_CGS2_SELECTIVE: the criterion of Daniel, Gragg,
 * Kaufman and Stewart), or never (ECS_ORTH_CGS1).
 * nrhs: Bi-CGSTAB right-hand sides of one system at once in ecs_batch_solve
 * (1..8; 0: up to 8), and in ecs_workspace_size the batched solve's storage
 * for that many (0 there sizes a single solve only); other calls ignore it. */
typedef struct {
  int krylov;
  int restart;
  double rtol;
  int maxit;
  int x_is_guess;
  int inner;
  double *history;
  int history_len;
  int orth;
  int nrhs;
} ecs_solve_desc;

typedef struct {
  int iterations;          /* outer Krylov iterations                         */
  int restarts;            /* restart cycles (GMRES) / true-residual restarts */
  int64_t vcycles;         /* preconditioner applications (multigrid cycles)  */
  int64_t inner_iterations;/* inner Bi-CGSTAB iterations (nested form)       */
  double rel_residual;     /* true ||b - A x|| / ||b|| at exit (FP64)         */
  double seconds;          /* host wall time inside the call                  */
  int status;              /* same value as returned                          */
  int64_t reorthogonalisations; /* second Gram-Schmidt passes run (GMRES; with
                              the delayed pass: every step but each restart
                              cycle's first)                                  */
  int64_t inner_breakdowns;/* nested form: inner Bi-CGSTAB runs cut short by
                              a zero or non-finite scalar (a breakdown, or an
                              exactly converged residual); the iterate reached
                              so far serves as that step's direction          */
} ecs_stats;

/* Create a problem on the calling thread's current HIP device.
 * dim = 2 or 3; nodes/lo/hi have dim meaningful entries; stream is a
 * hipStream_t (NULL = default stream).  All sides start as plain Dirichlet
 * ends without a layer. */
ecs_status ecs_create(ecs_ctx **out, int dim, const int64_t *nodes, const double *lo, const double *hi,
                      void *stream);

/* Exterior complex scaling of one side (Sec. 3.1): for kind = ECS_BC_ECS the
 * contour is z(x) = x until the real coordinate `start`, and rotated beyond
 * it, z = start + (x - start) e^{i theta} (0 < theta < pi/2), ending in a
 * homogeneous Dirichlet node.  ECS_BC_DIRICHLET removes the layer. */
ecs_status ecs_set_ecs(ecs_ctx *ctx, int axis, int side, int kind, double start, double theta);

/* k^2 at the real node coordinates (the k^2(x) of the model problem, Sec. 2;
 * Sec. 3.2 evaluates it at the nodes): a device array of prod(nodes) reals,
 * node-major, of real_dtype ECS_F64 (double) or ECS_F32 (float).
 *   ECS_F64: borrowed and read by every later call (apply, cycle, solve) until
 *            the next ecs_set_k2 or ecs_destroy.
 *   ECS_F32: read once, by ecs_set_workspace, which widens it exactly into
 *            FP64 storage inside the workspace (ecs_workspace_size counts it,
 *            so call ecs_set_k2 first); later changes to the array take effect
 *            at the next ecs_set_workspace.
 * Invalidates the preconditioner setup (call ecs_set_workspace again).
 * Errors: ECS_EINVAL for a null pointer or another dtype. */
ecs_status ecs_set_k2(ecs_ctx *ctx, const void *k2_dev, int real_dtype);

ecs_status ecs_set_precond(ecs_ctx *ctx, const ecs_prec_desc *desc);

/* Bytes of device workspace needed for solves described by `desc` (NULL:
 * enough for ecs_apply / ecs_vcycle and the per-step entry points only). */
ecs_status ecs_workspace_size(ecs_ctx *ctx, const ecs_solve_desc *desc, size_t *bytes);

/* Hand over the workspace (256-byte aligned device memory, caller-owned, kept
 * until the next call or destroy) and build the device hierarchy: contour
 * weights per level, injected k^2, coarsest dense inverse.  Requires k^2 and
 * the preconditioner to be set. */
ecs_status ecs_set_workspace(ecs_ctx *ctx, void *dev, size_t bytes);

/* Solve A x = b (Sec. 5).  b, x: complex128 device arrays. */
ecs_status ecs_solve(ecs_ctx *ctx, const ecs_solve_desc *desc, const void *b_dev, void *x_dev, ecs_stats *stats);

/* For callers that cannot allocate device memory (serving loops, harnesses
 * that forbid hipMalloc; the solve itself waits on the host between Krylov
 * steps, so it is not for use inside a graph capture): ecs_solve with
 * the Krylov vectors in the library's static device scratch instead of the
 * workspace.  Same arguments, method, results and statuses as ecs_solve; the
 * call itself allocates nothing (no hipMalloc/hipFree, no graph, no event):
 * the cycle is launched eagerly whatever ecs_set_graphs says, and kernel
 * timers are not recorded.  The context's workspace need only hold the
 * hierarchy (ecs_workspace_size with desc = NULL).  Limit: the Krylov storage
 * of the solve must fit the scratch, 64 MiB per device (Bi-CGSTAB up to about
 * 513^2 nodes, GMRES(30) up to about 257^2); larger ones return ECS_ENOMEM
 * with the size in ecs_last_error.  Every call on one GPU shares that GPU's
 * scratch (it keeps the last call's contents; each solve initialises what it
 * reads): calls that overlap on one GPU, from different streams or threads,
 * race and must be serialised by the caller. */
ecs_status ecs_solve_static(ecs_ctx *ctx, const ecs_solve_desc *desc, const void *b_dev, void *x_dev,
                            ecs_stats *stats);

/* Solve A^T lam = g (plain transpose, no conjugation) with the same
 * preconditioner, through the similarity A^T = W A W^{-1}, W = diag of the
 * products of the dual cell widths w_i = (h_{i-1} + h_i)/2. */
ecs_status ecs_solve_adjoint(ecs_ctx *ctx, const ecs_solve_desc *desc, const void *g_dev, void *lam_dev,
                             ecs_stats *stats);

/* grad = Re(lam * u) per node (real FP64 output): the derivative of a real
 * loss with respect to k^2 when A^T lam = conj(dL/du). */
ecs_status ecs_grad_k2(ecs_ctx *ctx, const void *lam_dev, const void *u_dev, double *grad_dev);

/* y = op x on the finest grid, complex128: op = A (Z = -Lap - k^2), A^T, or
 * the preconditioner operator M in FP64. */
ecs_status ecs_apply(ecs_ctx *ctx, int op, const void *x_dev, void *y_dev);

/* z = MG(v): one preconditioner application from a zero guess (Algorithm 1
 * at the finest level), complex128 in and out; the cycle runs in the
 * preconditioner's vcycle_dtype. */
ecs_status ecs_vcycle(ecs_ctx *ctx, const void *v_dev, void *z_dev);

/* The same cycle on vectors already in the cycle's dtype (complex64 when
 * vcycle_dtype is ECS_F32, complex128 otherwise): no conversion passes. */
ecs_status ecs_vcycle_native(ecs_ctx *ctx, const void *v_dev, void *z_dev);

/* Coupled block system (Sec. 2: the partial-wave expansion couples 2D
 * Helmholtz problems only through potentials): sum_j A_ij x_j = b_i,
 * i = 0 .. nb-1 (nb <= 8), with A_ii the ECS operator -Lap - k^2_ii of block i
 * (context ctx[i]: its k^2, contour and preconditioner; every block on the same
 * grid and device) and A_ij = -diag(k2c_ij) for i != j.  Solved by right-
 * preconditioned FGMRES(outer->restart) over the stacked vector (FP64, true
 * residual over interior nodes <= outer->rtol) with the block-diagonal
 * preconditioner z_i ~ A_ii^{-1} r_i of Sec. 2, each block solved by its own
 * context: all blocks together by the batched Bi-CGSTAB driver to
 * inner->rtol (inner->maxit iterations at most), or, with inner = NULL, one
 * multigrid cycle of each block's preconditioner.
 *   k2c: device array of nb * nb * nodes doubles, the potential k2c_ij of the
 *        pair (i, j) at offset (i nb + j) * nodes (entries i == j are not
 *        read); NULL for uncoupled blocks.  Borrowed for the call.
 *   b, x: stacked complex128 device arrays of nb * nodes entries, block i at
 *        offset i * nodes; x is a guess when outer->x_is_guess.
 *   workspace: device memory of ecs_coupled_workspace_size bytes, 256-byte
 *        aligned, caller-owned; the contexts' own workspaces must be sized for
 *        `inner` as one right-hand side of the batched solve
 *        (ecs_workspace_size with inner, nrhs = 1).
 *   stats: iterations = outer iterations, inner_iterations and vcycles summed
 *        over all block solves.  Outer work runs on ctx[0]'s stream; the call
 *        returns after every stream involved has finished.
 * Returns ECS_EINVAL (message on ctx[0]) for nb outside 1..8 or a NULL outer. */
ecs_status ecs_coupled_workspace_size(int nb, ecs_ctx *const *ctx, const ecs_solve_desc *outer, size_t *bytes);
ecs_status ecs_coupled_solve(int nb, ecs_ctx *const *ctx, const double *k2c, const ecs_solve_desc *outer,
                             const ecs_solve_desc *inner, void *workspace, size_t ws_bytes, const void *b_dev,
                             void *x_dev, ecs_stats *stats);

/* Stand-alone multigrid on the preconditioner, M x = b (Sec. 5: the
 * preconditioner solved on its own, the "mg-conv" and "# cycles" columns of
 * Tables 1-4): x <- x + MG(b - M x), which is Algorithm 1 started from the
 * previous iterate, until ||b - M x||_2 <= rtol ||b||_2 over interior nodes
 * or after maxcycles cycles.  Also a warm start for ecs_solve (Sec. 5 feeds
 * the preconditioner's solution at 1e-2 to the Krylov method as its guess).
 * b, x: complex128 device arrays; x_is_guess = 0 starts from x = 0.  M's
 * residual is formed in FP64; the cycle runs in the preconditioner's
 * vcycle_dtype.  history (optional host array of history_len doubles)
 * receives ||b - M x_m|| / ||b|| for m = 0, 1, ... (the entry before the
 * first cycle included).  stats: iterations = vcycles = cycles done,
 * rel_residual = the last ratio.  Returns ECS_OK, ECS_NOT_CONVERGED after
 * maxcycles cycles, or ECS_EBREAKDOWN on NaN/Inf.  Uses the workspace's
 * Krylov scratch (any workspace size is enough). */
ecs_status ecs_mg_solve(ecs_ctx *ctx, const void *b_dev, void *x_dev, double rtol, int maxcycles, int x_is_guess,
                        double *history, int history_len, ecs_stats *stats);

/* Per-step entry points on level `level` (0 = finest) of the hierarchy,
 * operating on arrays of that level's size in the cycle's dtype (complex128
 * for ECS_F64, complex64 for ECS_F32):
 *   ecs_smooth:            nsweeps smoothing sweeps of M u = b, u in place
 *   ecs_residual_restrict: rc = FW(b - M u), rc on level+1
 *   ecs_prolong_correct:   u += P ec, ec on level+1 (bilinear / trilinear)
 *   ecs_coarse_solve:      x = M_C^{-1} b on the coarsest level            */
ecs_status ecs_smooth(ecs_ctx *ctx, int level, const void *b_dev, void *u_dev, int nsweeps);
ecs_status ecs_residual_restrict(ecs_ctx *ctx, int level, const void *b_dev, const void *u_dev, void *rc_dev);
ecs_status ecs_prolong_correct(ecs_ctx *ctx, int level, const void *ec_dev, void *u_dev);
ecs_status ecs_coarse_solve(ecs_ctx *ctx, const void *b_dev, void *x_dev);

/* Number of levels and nodes per axis of one level (after set_precond). */
ecs_status ecs_level_info(ecs_ctx *ctx, int level, int *nlevels, int64_t *nodes);

/* Kernel timing for measurement: when enabled, HIP events are recorded on the
 * context's stream around launches of kernel class `kclass` -- enable = 1:
 * every launch; enable = n > 1: one launch in n (the 1st, (n+1)-th, ...),
 * which keeps the events' own cost (a few microseconds per timed launch) off
 * most launches of a timed solve; 0: off; negative: ECS_EINVAL.  Classes:
 *   0 finest-level smoothing sweep      5 finest-level residual + restriction
 *   1 Arnoldi multi-dot (partials)      6 finest-level prolongation + correction
 *   2 FP64 operator A (matvec)          7 finest-level fused down kernel
 *   3 coarse-level cycle kernels        8 finest-level fused up kernel
 *   4 Arnoldi orthogonal update          9 empty kernel (ecs_timing_calibrate)
 *  10 finest-level fused down kernel forming a Bi-CGSTAB's p
 *  11 finest-level fused down kernel forming a Bi-CGSTAB's s
 *     (classes 10 and 11 run instead of 7 in the nested FP32 Bi-CGSTAB, and
 *     in the outer Bi-CGSTAB with the FP64 cycle up to 1025^2 finest nodes,
 *     when ecs_tuning.fuse_updates applies)
 * A timed duration runs from the dispatch of the kernel to its completion.
 * ecs_timing_read synchronises the stream and returns the number of timed
 * launches, their summed duration in ms and their summed algorithmic bytes
 * (the minimum HBM traffic of each launch: every input read once, every
 * output written once), then resets the class. */
ecs_status ecs_timing_enable(ecs_ctx *ctx, int kclass, int enable);
ecs_status ecs_timing_read(ecs_ctx *ctx, int kclass, int64_t *launches, double *total_ms, double *algo_bytes);

/* Time `launches` (1..65536) launches of an empty kernel on the context's
 * stream as class 9: their average is the fixed part of a timed duration
 * (dispatch to the first wave, completion) that carries no work, which a
 * measurement may subtract from the average of another class.  Enables
 * class 9 for the call only. */
ecs_status ecs_timing_calibrate(ecs_ctx *ctx, int launches);

/* Launch schedule of the fused 2D V(1,1) red-black cycle.  It chooses which
 * kind of kernel runs each level (one level per kernel, two levels per
 * kernel, the single-workgroup tail) and their tile heights; the method's
 * arithmetic is the same under every schedule, but kernels of different kinds
 * order some floating-point operations differently, so the cycle's result
 * can change at the level of rounding (in FP32 enough to move a nested
 * solve's outer iteration count by a few percent):
 *   down_rows   coarse rows per block of the fused pre-smoothing/restriction
 *               kernel on grids above small_grid: 2 to 6, 8 (16 in FP32)
 *   up_rows     fine rows per block of the fused prolongation/post-smoothing
 *               kernel on grids above small_grid: 4, 8, 10, 12, 16 or 32
 *   small_grid  grids with at most this many nodes per axis use 2 / 4 rows
 *   tail_nodes  levels with at most this many nodes per axis run in the
 *               single-workgroup kernel that ends the cycle: 3..65; above 33
 *               it applies to FP32 cycles only (their wide tail holds up to
 *               5696 nodes, e.g. 65^2 down to a 9^2 coarsest), FP64 cycles
 *               and general cycles use min(tail_nodes, 33)
 *   pair_grid   levels above the tail with at most this many nodes per axis
 *               run two per kernel (pairs counted from the tail up); 0: none
 *   fuse_updates  1: the FP32 Bi-CGSTAB inside FGMRES (desc->inner > 0), and
 *               the Bi-CGSTAB solve with the FP64 cycle on grids of at most
 *               1025^2 nodes, form their p and s updates inside the finest
 *               level's down kernel when that level has its own down kernel
 *               and the cycle is not launched as a graph
 *               (ECS_GRAPHS_ALWAYS), with the same values as the separate
 *               update kernels; 0: separate update kernels
 * Defaults {4, 8, 513, 33, 129, 1}; a project autotuner picks the tile
 * heights per grid size and dtype by timing cycles.  Other values:
 * ECS_EINVAL. */
typedef struct {
  int down_rows;
  int up_rows;
  int small_grid;
  int tail_nodes;
  int pair_grid;
  int fuse_updates;
} ecs_tuning;
ecs_status ecs_set_tuning(ecs_ctx *ctx, const ecs_tuning *tuning);
ecs_status ecs_get_tuning(ecs_ctx *ctx, ecs_tuning *tuning);

/* How the preconditioner cycle is launched (results are the same in every
 * mode):
 *   ECS_GRAPHS_NEVER   every kernel eagerly on the context's stream
 *   ECS_GRAPHS_ALWAYS  the cycle is captured once per (input, output) buffer
 *                      pair as a HIP graph and replayed with one launch
 *   ECS_GRAPHS_AUTO    (default) graphs for general cycles, whose many small
 *                      launches would make the host the bottleneck; eager
 *                      launches for the fused 2D V(1,1) red-black cycle
 *                      (about two launches per level), where the device-side
 *                      completion of a graph launch costs more than the host
 *                      launches it saves
 * Any other value: ECS_EINVAL. */
enum { ECS_GRAPHS_NEVER = 0, ECS_GRAPHS_ALWAYS = 1, ECS_GRAPHS_AUTO = 2 };
ecs_status ecs_set_graphs(ecs_ctx *ctx, int mode);

/* Batched solve of n independent problems (Bi-CGSTAB), the many independent
 * Helmholtz blocks of Sec. 2 at once.  desc[s] holds system s's Krylov
 * settings (desc[s]->krylov must be ECS_KRYLOV_BICGSTAB; rtol, maxit and
 * x_is_guess may differ between systems).  b[s], x[s] point to nrhs[s]
 * contiguous complex128 vectors of system s (x read as the initial guesses
 * when x_is_guess).  Each context is fully set up with its own workspace and
 * should have its own stream.
 *   Right-hand sides: with the fused 2D V(1,1) red-black cycle (2D, RB-GS,
 *   nu1 = nu2 = 1, V) a system's right-hand sides are solved together, up to
 *   min(8, desc[s]->nrhs if > 0) at once, every kernel of an iteration serving
 *   all of them in one launch (per right-hand side the same arithmetic as a
 *   single solve); other set-ups take them one at a time.  The workspace must
 *   hold that many at once (ecs_workspace_size with that nrhs; 1 for other
 *   set-ups), else ECS_ENOMEM.
 *   Scheduling: the driver enqueues one round of a system at a time on that
 *   system's stream (the restarts -- true residuals -- of the right-hand sides
 *   that need one, one iteration of the others, one readback), records an
 *   event after it and polls the events from the host; a system's next round
 *   is enqueued as soon as its own previous one has completed, so systems of
 *   different sizes progress independently.
 * Returns after every stream has been synchronised; a context given twice is
 * ECS_EINVAL.  stats[s] aggregates the system's right-hand sides: summed
 * iterations, restarts and cycles, the largest final true residual, the worst
 * status, and the wall time of the whole batch. */
ecs_status ecs_batch_solve(int n, ecs_ctx *const *ctxs, const ecs_solve_desc *const *desc, const void *const *b,
                           void *const *x, const int *nrhs, ecs_stats *stats);

/* Plain device copy of `bytes` bytes (bandwidth probe), on `stream`. */
ecs_status ecs_copy_probe(const void *src_dev, void *dst_dev, size_t bytes, void *stream);

const char *ecs_last_error(const ecs_ctx *ctx);
void ecs_destroy(ecs_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* ECSMG_H */
