/*
 * hipsso -- differentiable linear-static structural FEA on one MI355X (gfx950).
 *
 * C ABI of the hot path: element stiffness of 12-DOF space-frame members and 4-node flat
 * shells, deterministic assembly into a sparse K, the support-constrained solve K u = f with
 * block-Jacobi preconditioned conjugate gradients, objectives, and the adjoint sensitivity of an
 * objective with respect to nodal coordinates, shell thickness and per-element stiffness scale.
 *
 * Paper: Wu, "JAX-SSO: Differentiable Finite Element Analysis Solver for Structural
 * Optimization and Seamless Integration with Neural Networks" (arXiv 2407.20026).
 *   Sec. 2.2.1  K u = f (Eq. 1); element-to-global index maps; vectorised assembly of all element
 *               matrices into a sparse K; supports through Lagrange multipliers (Eqs. 2-3);
 *               the model-building API (nodes, 6-flag supports, 6-component nodal loads,
 *               beam-columns with E, G, Iy, Iz, J, A; MITC-4 quads with x, y, z of 4 nodes,
 *               t, E, nu, kx, ky).
 *   Sec. 2.2.2  solving the constrained system (the paper uses direct solvers; this library
 *               uses preconditioned conjugate gradients on the masked system).
 *   Sec. 2.3.1  adjoint equation K^T lambda = dg/du^T (Eq. 5) and adjoint sensitivity
 *               dg/dp = dg/dp|explicit - lambda^T (dK/dp u - df/dp) (Eq. 6); node parameters
 *               (coordinate of a node) and objectives ("strain energy" f^T u / 2).
 *   Sec. 3.3-3.4 thickness as a design variable; SIMP stiffness scaling E = rho^P E0 (Eq. 13).
 *
 * Conventions shared by every entry point:
 *   - Global DOF d = 6 * node + c, c in (ux, uy, uz, rx, ry, rz).  SI units.
 *   - Every array pointer is a DEVICE pointer (memory the caller allocated on the GPU the
 *     problem runs on), row-major, densely packed.  Exceptions are marked "host".
 *   - Input arrays are borrowed for the duration of the call; the library copies what it keeps.
 *   - Outputs go to caller-allocated device buffers.
 *   - Work is enqueued on the stream given at creation.  sso_problem_create, sso_solve,
 *     sso_objective and sso_adjoint synchronise that stream before returning (they report
 *     convergence, errors and host scalars); sso_problem_update only enqueues.  A solve
 *     cannot return at enqueue and still report its outcome, because its stopping test reads
 *     the iteration state back between chunks of iterations.  The asynchronous form is
 *     sso_solve_begin, then sso_batch_launch (returns at once) and sso_batch_wait (waits for
 *     the states only), then sso_solve_end; sso_problem_set_stream moves a problem between
 *     streams.
 *   - A problem is not thread-safe: use one problem per host thread.
 *   - Every function returns SSO_OK (0) or a negative status; sso_strerror gives the text.
 *     On error, outputs are left unspecified and the problem stays usable (except after
 *     SSO_EHIP, which reports a failed HIP runtime call).
 */
#ifndef HIPSSO_H
#define HIPSSO_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SSO_OK = 0,
  SSO_EINVAL = -1,      /* bad argument, index out of range, degenerate element           */
  SSO_ENOMEM = -2,      /* device allocation failed                                       */
  SSO_EHIP = -3,        /* a HIP runtime call failed                                      */
  SSO_ENOTCONV = -4,    /* PCG reached max_it before the residual target (stats filled)   */
  SSO_EBREAKDOWN = -5,  /* p^T K p <= 0 or not finite: K not positive definite (e.g. an
                           unsupported rigid-body mode); stats filled                     */
  SSO_ESIZE = -6        /* problem larger than the static scratch of
                           sso_size_objective_noalloc (SSO_NOALLOC_MAX_QUADS)              */
};

enum {
  SSO_OBJ_COMPLIANCE = 0,     /* g = f^T u                      (loss of Sec. 3.6)      */
  SSO_OBJ_STRAIN_ENERGY = 1,  /* g = f^T u / 2                  (Sec. 2.2.3, 2.3.2)     */
  SSO_OBJ_LINEAR = 2,         /* g = a^T u, a given                                        */
  SSO_OBJ_USER = 3            /* caller supplies dg/du; dg/dp omits explicit dependence    */
};

/* Precision.  AUTO picks, per problem, mixed precision when the FP64 K alone holds at least
 * SSO_AUTO_MIXED_K_BYTES (128 MiB) -- from there K no longer stays in the 256 MB Infinity Cache
 * between iterations and the FP32 inner iterations' halved bytes pay for the extra iterations
 * of the restarted inner solves -- and, for a tolerance of SSO_AUTO_TIGHT_RTOL (1e-9) or tighter,
 * at least SSO_AUTO_MIXED_TIGHT_K_BYTES (256 MiB): there the restarts cost more outer steps.
 * FP64 otherwise.  Measured on single shells, forward solve, FP64 against mixed with inner
 * solves capped at 30: rtol 1e-8, 250 x 250 (K 162 MB) 297 against 264 ms, 300 x 300 (234 MB)
 * 515 against 493, 400 x 400 (417 MB) 1,368 against 1,067; rtol 1e-10, 250 x 250 342 against
 * 349, 300 x 300 529-560 against 576-597, 400 x 400 1,517 against 1,243.  In AUTO's mixed
 * precision an inner_max_it of 0 means 30 (the best of the measured caps) and the outer step
 * limit is at least max_it / 30. */
enum { SSO_PREC_FP64 = 0, SSO_PREC_MIXED = 1, SSO_PREC_AUTO = 2 };
#define SSO_AUTO_MIXED_K_BYTES (128.0 * 1024.0 * 1024.0)
#define SSO_AUTO_MIXED_TIGHT_K_BYTES (256.0 * 1024.0 * 1024.0)
#define SSO_AUTO_TIGHT_RTOL 1e-9

/* PCG recurrences.  STANDARD: Hestenes-Stiefel CG, two kernels and two reductions per
 * iteration.  FUSED: the single-reduction form of Chronopoulos & Gear (one kernel and one
 * reduction per iteration; keeps B = K M, M the block-Jacobi inverse, beside K: one more array
 * of K's size).  AUTO: sso_solve takes WG for FP64 problems resident in one workgroup's LDS
 * (at most 144 nodes; measured 3.07 against 4.39 ms on the 121-node grid-shell), FUSED up to
 * 8,192 nodes (latency-bound sizes; 13.4 against 20.2 ms on a 60 x 60 shell, equal on 90 x 90,
 * 88 against 63 ms on 120 x 120) and STANDARD above; sso_solve_begin (multi-problem launches)
 * takes WG for the same LDS-resident problems and STANDARD for the others.
 * WG: the standard recurrences with one workgroup per problem, every iteration inside one launch
 * (workgroup barriers between the phases, no grid-wide synchronisation; a single solve is one
 * launch up to 16,384 iterations, a multi-problem launch gives such a problem 16 times the
 * iterations asked for, in a kernel of its own beside the other kinds).  A problem of at most
 * 144 nodes whose vectors, pattern and packed inverses fit 60 KiB runs resident in LDS (only K
 * read from memory each iteration); larger ones read everything from memory and are slower than
 * the other recurrences.  FP64 only (with SSO_PREC_MIXED: SSO_EINVAL; AUTO precision resolves to
 * FP64).  Its rounding differs from STANDARD's in the order of the reductions only. */
enum { SSO_SOLVER_AUTO = 0, SSO_SOLVER_STANDARD = 1, SSO_SOLVER_FUSED = 2, SSO_SOLVER_WG = 3 };

/* Structure description.  Sec. 2.2.1 model-building API. */
typedef struct {
  int32_t n_nodes;
  const double* xyz;          /* [n_nodes][3] nodal coordinates (add_node)                    */
  const uint8_t* fixed;       /* [n_nodes][6] 1 = DOF fixed, 0 = free (add_support flags)    */
  const double* f_nodal;      /* [n_nodes][6] nodal forces and moments (add_nodal_load)      */
  int32_t n_beams;
  const int32_t* beam_nodes;  /* [n_beams][2] end nodes i, j (add_beamcol)                   */
  const double* beam_prop;    /* [n_beams][6] E, G, A, Iy, Iz, J                             */
  int32_t n_quads;
  const int32_t* quad_nodes;  /* [n_quads][4] corner nodes, counter-clockwise about the
                                 element normal                                             */
  const double* quad_prop;    /* [n_quads][5] t, E, nu, kx, ky (kx = ky = 1 required)        */
  const double* quad_scale;   /* [n_quads] stiffness scale s_e (e.g. rho^3), or NULL = 1     */
  double unit_weight;         /* self-weight of quads along -Z, N/m^3 (0 = none)             */
  double surface_load;        /* uniform pressure on quads along -Z, N/m^2 (0 = none)        */
  const double* u_prescribed; /* [n_nodes][6] prescribed displacements b of Eq. 3, read at the
                                 fixed DOFs (the rest is ignored), or NULL = all zero        */
} sso_mesh;

typedef struct {
  int32_t precision;          /* SSO_PREC_FP64, SSO_PREC_AUTO (above), or SSO_PREC_MIXED:
                                 FP64 flexible CG (one
                                 stored direction) whose preconditioner is an FP32 PCG solve
                                 (FP32 K, vectors, SpMV and dot accumulation); element
                                 stiffness, the outer products with K, the step lengths and
                                 the updates of u stay FP64                                  */
  double rtol;                /* stop when ||f - K u||_2 <= rtol ||f||_2 (recursive residual;
                                 the reported residual is recomputed)                       */
  int32_t max_it;             /* PCG iteration limit per solve                               */
  int32_t refine_steps;       /* mixed precision: maximum outer (FP64) steps                 */
  int32_t profile_every;      /* 0 = off; n > 0: time every n-th PCG iteration with HIP
                                 events on the problem's stream (stats.spmv_us)              */
  double inner_rtol;          /* mixed precision: relative tolerance of each FP32 inner PCG
                                 solve (0 = 1e-5)                                           */
  int32_t solver;             /* SSO_SOLVER_*: PCG recurrences (also of the FP32 inner solves) */
  int32_t inner_max_it;       /* mixed precision: iteration cap of each FP32 inner solve
                                 (0 = none: each inner solve runs to its tolerance)          */
} sso_options;

typedef struct {
  int32_t iters;              /* PCG iterations of the last solve (all inner solves)         */
  double rel_residual;        /* ||f - K u||_2 / ||f||_2 recomputed after the solve, the row
                                 sums of K u in double-double (compensated) arithmetic       */
  double t_elem_us;           /* element stiffness + loads                                   */
  double t_asm_us;            /* assembly + masking + block-Jacobi                           */
  double t_solve_us;          /* PCG                                                         */
  double t_adj_us;            /* adjoint solve + element contraction + gather (sso_adjoint)  */
  double bytes_moved;         /* algorithmic HBM bytes of the PCG iterations                 */
  double spmv_us;             /* mean duration of one PCG iteration, from samples of 8
                                 back-to-back iterations (profile_every; dispatch gaps
                                 included): k_spmv_dir_single (reading K's upper triangle
                                 when sym_products) + k_update_single of the standard
                                 recurrences, k_cg1_iter1 of the single-reduction ones       */
  int32_t spmv_samples;       /* number of sampled iterations                                */
  double spmv_bytes;          /* algorithmic bytes of one iteration                          */
  int32_t refine_steps;       /* mixed precision: outer steps (FP32 inner solves) run        */
  int32_t solver;             /* SSO_SOLVER_STANDARD, _FUSED or _WG: recurrences that ran    */
  int32_t sym_products;       /* 1: the standard recurrences' products read only K's upper
                                 triangle, each block below the diagonal as the transpose of
                                 its mirror (single FP64 solves of a K of 128 MiB or more; the
                                 same sums, bitwise, as reading all of K); spmv_bytes counts
                                 that triangle.  Multi-problem launches do the same when their
                                 problems' K take 128 MiB together; sso_solve_end reports 0
                                 and counts all of K for them                                */
} sso_stats;

typedef struct sso_problem sso_problem;

/* Create a problem: copies the mesh into device buffers owned by the problem and builds, once
 * per topology, the sparse pattern of K, the sort permutation of the element contribution list
 * and the node-to-element incidence (Sec. 2.2.1, element index maps and sparse storage).
 * mesh: host struct whose array members are device pointers.  opts: host struct, or NULL for
 * defaults (FP64, rtol 1e-8, max_it 200000, refine_steps 20).  stream: HIP stream for all work
 * of this problem (0 = null stream).  *out receives the handle.
 * Errors: SSO_EINVAL for negative counts, n_nodes == 0, a node index outside [0, n_nodes) or
 * an element that repeats a node; SSO_ENOMEM; SSO_EHIP. */
int sso_problem_create(const sso_mesh* mesh, const sso_options* opts, hipStream_t stream,
                       sso_problem** out);

/* The same as sso_problem_create for a structure of the same topology as `like` (an existing
 * problem on the current device): same node, member and quad counts and the same connectivity
 * (beam_nodes, quad_nodes); coordinates, supports, loads and properties may all differ.  The
 * pattern of K, the sort permutation and the padded rows are not rebuilt but shared with `like`
 * (reference-counted: they live until the last problem that uses them is destroyed, whichever
 * order the problems are destroyed in), so creation skips the pattern build and its
 * synchronisations; results are bitwise those of sso_problem_create.  For request loops that
 * see the same structure sizes again and again.  Sharing problems may run on different streams;
 * destroying two of them at the same time from two threads is safe.  Errors: SSO_EINVAL (counts
 * differ, connectivity differs -- checked on the device before the call returns --, `like` on
 * another device, and as sso_problem_create), SSO_ENOMEM, SSO_EHIP.  sso_problem_bytes of the
 * new problem does not count the shared pattern. */
int sso_problem_create_like(const sso_problem* like, const sso_mesh* mesh,
                            const sso_options* opts, hipStream_t stream, sso_problem** out);

/* Replace design inputs without changing the topology: the design parameters p of the
 * optimisation problem (Sec. 2.3.1, Eq. (4); updated between steps as in Eq. (7)) -- nodal
 * coordinates (node parameters, Sec. 2.3.1), shell thickness (Sec. 3.3) and the per-element
 * stiffness scale (SIMP, Sec. 3.4 Eq. (13)).  Device pointers, each may be NULL to keep the
 * current values: xyz [n_nodes][3]; quad_t [n_quads] thickness; quad_scale [n_quads] stiffness
 * scale.  Enqueued on the problem's stream; invalidates the last solution. */
int sso_problem_update(sso_problem* p, const double* xyz, const double* quad_t,
                       const double* quad_scale);

/* Replace solver options (host struct).  A change of precision or solver invalidates the last
 * solution (sso_objective / sso_adjoint need a new sso_solve).  Errors: SSO_EINVAL for values
 * outside their ranges or while a begun solve (sso_solve_begin) is not yet ended. */
int sso_set_options(sso_problem* p, const sso_options* opts);

/* Forward analysis: element stiffness (beams: K = s T^T k T; quads: flat shell, K = s T^T W^T k
 * W T), loads (nodal + self-weight + surface load lumped to corners), deterministic assembly
 * K[slot] = sum of the slot's element entries in ascending element order, support masking
 * (constrained d: K[d,:] = K[:,d] = 0, K[d,d] = 1, f[d] = 0; with prescribed values b a
 * free row's load loses K(row, d) b[d] and u[d] = b[d] is set after the solve -- identical in
 * u to the Lagrange system of Eqs. 2-3 with V u = b), block-Jacobi preconditioner, PCG; the
 * relative residual is that of the free equations.  u_out: [n_nodes][6] device output (may be NULL).  stats: host struct
 * or NULL.  Errors: SSO_EINVAL (degenerate element: zero-length beam, det J <= 0, zero quad
 * area, non-positive t/E/A/I/J, nu outside (-1, 0.5), kx or ky != 1; a diagonal 6x6 block that
 * is not positive definite), SSO_ENOTCONV (u_out then holds the last iterate, and
 * sso_objective / sso_adjoint may still be called), SSO_EBREAKDOWN, SSO_EHIP. */
int sso_solve(sso_problem* p, double* u_out, sso_stats* stats);

/* Forward analysis split for multi-problem launches: sso_solve_begin runs everything up to the
 * first PCG iteration (elements, loads, assembly, masking, block-Jacobi, PCG initialisation),
 * FP64 or mixed precision, either recurrence (SSO_SOLVER_AUTO picks STANDARD here: the faster
 * form when many problems share the launches); sso_batch_iterate then advances many begun
 * problems together (mixed precision: including the FP64 outer steps between FP32 inner
 * solves); sso_solve_end finishes one (FP64 correction of the true residual, u_out as in
 * sso_solve, stats) once its iteration has stopped.  With the same precision and recurrence,
 * results are bitwise the same as sso_solve's. */
int sso_solve_begin(sso_problem* p);
int sso_solve_end(sso_problem* p, double* u_out, sso_stats* stats);

/* A multi-problem launcher bound to one stream.  Problems iterated together must have been
 * created on that stream.  Callers: a request loop that keeps many problems in flight. */
typedef struct sso_batch sso_batch;
int sso_batch_create(hipStream_t stream, sso_batch** out);
/* Launch n_iter PCG iterations for every problem of ps[0..n) whose iteration has not stopped,
 * all problems of one recurrence kind (sso_options.solver at sso_solve_begin) in one launch per
 * kernel, then read back their states: done[i] (host, may be NULL) = 1 when problem i's
 * iteration has stopped (converged, limit or breakdown).  Errors: SSO_EINVAL (problem not
 * begun, on another stream, or listed twice), SSO_EHIP. */
int sso_batch_iterate(sso_batch* b, sso_problem* const* ps, int n, int n_iter, int32_t* done);
/* sso_batch_iterate in two halves, so that the host can work while the GPU iterates:
 * sso_batch_launch enqueues the n_iter iterations and the copy of the problems' states to pinned
 * host memory and returns at once; sso_batch_wait(b, ps, n, done) waits for them, then does what
 * sso_batch_iterate does after its launches (mixed precision's outer steps, done flags).  The
 * wait must list the same problems in the same order as the launch; between the two, the listed
 * problems may not be iterated, ended, moved to another stream or destroyed, and a batch holds at
 * most one pending launch.  Errors: SSO_EINVAL (as sso_batch_iterate; a launch while one is
 * pending; a wait without a launch or with another list), SSO_EHIP. */
int sso_batch_launch(sso_batch* b, sso_problem* const* ps, int n, int n_iter);
int sso_batch_wait(sso_batch* b, sso_problem* const* ps, int n, int32_t* done);
/* Timing samples of the multi-problem FP64 standard iterations (the product kernel over all of
 * K or its upper triangle, then k_update; Sec. 2.2.1 Eq. (1) solved by PCG, the same kernels as
 * without sampling), for measurement.  every > 0: of the launches (sso_batch_launch or
 * sso_batch_iterate) whose problems all run FP64 standard recurrences -- one-workgroup problems
 * may run beside them on the batch's second stream -- every every-th brackets its first
 * min(span, n_iter) iterations with HIP events on the batch stream; every = 0 stops sampling.
 * Resets the sums.  Errors: SSO_EINVAL (NULL batch, every or span negative, span 0 with every
 * > 0, a launch pending), SSO_EHIP (event creation). */
int sso_batch_profile(sso_batch* b, int every, int span);
/* The sums since sso_batch_profile: us = the sampled spans' event time in microseconds,
 * iters = iterations in those spans (each one launch of each kernel over all listed problems),
 * bytes = algorithmic bytes of the problem-iterations done inside the spans with all of K
 * counted (a problem's iterations there from its next-iteration index before and after the
 * launch, at most the span), bytes_read = the same with K counted as the launch's product read
 * it (its upper triangle when the problems' K take 128 MiB together).  Outputs are host
 * pointers, each may be NULL.  Errors: SSO_EINVAL (NULL batch). */
int sso_batch_timing(const sso_batch* b, double* us, int64_t* iters, double* bytes,
                     double* bytes_read);
void sso_batch_destroy(sso_batch* b);

/* Move a problem's work to another stream (e.g. between a stream that admits and finishes
 * requests and the stream of a multi-problem launcher): the new stream is ordered after all work
 * already enqueued for the problem on its old stream (an event), and every later call enqueues on
 * the new one.  Errors: SSO_EINVAL (NULL problem, or listed in a pending sso_batch_launch),
 * SSO_EHIP. */
int sso_problem_set_stream(sso_problem* p, hipStream_t stream);

/* Objective value g(u) of the last solve (the objective of Sec. 2.3.1, Eq. (4)) into *g_host
 * (host): compliance f^T u (the loss of the network example, Sec. 3.6), strain energy f^T u / 2
 * (Sec. 2.2.3, 2.3.2; f: the applied load on the free DOFs), or a^T u for SSO_OBJ_LINEAR (a:
 * device [n_nodes][6]).  SSO_OBJ_USER: SSO_EINVAL.
 * Errors: SSO_EINVAL without a previous successful solve. */
int sso_objective(sso_problem* p, int kind, const double* a, double* g_host);

/* Adjoint sensitivity of the last solve (Eqs. 5-6).  kind selects g:
 *   COMPLIANCE / STRAIN_ENERGY: lambda = u exactly (K lambda = f), no second solve -- unless
 *   displacements are prescribed (then lambda solves the masked K lambda = f);
 *   LINEAR: dg_du = a; USER: dg_du = dg/du supplied by the caller ([n_nodes][6] device), and
 *   lambda solves the masked K lambda = dg/du with the same K and preconditioner.
 * Outputs (device, caller-allocated): dg_dxyz [n_nodes][3] (required); dg_dt [n_quads] and
 * dg_dscale [n_quads] (each may be NULL).  Per element e and parameter p the contribution
 * c_lam (lambda_e^T df_e/dp - lambda_e^T dK_e/dp u_e) + c_u u_e^T df_e/dp (u_e taken as 0 at
 * constrained DOFs in the last term) is formed exactly
 * (forward-mode dual numbers), then summed per node over incident elements in ascending
 * element order.  stats: host or NULL (t_adj_us; iters of the adjoint solve if one ran).
 * Errors: SSO_EINVAL (no solve, bad kind, NULL dg_du for LINEAR/USER), SSO_ENOTCONV,
 * SSO_EBREAKDOWN, SSO_EHIP. */
int sso_adjoint(sso_problem* p, int kind, const double* dg_du, double* dg_dxyz,
                double* dg_dt, double* dg_dscale, sso_stats* stats);

/* Penalised material volume of the size optimisation example (Sec. 3.3) on the last solve:
 *   g = (1 + eps1 c) W,  c = sum over nodes j of max(0, |u_jz| / u_max - 1),
 *   W = sum over quads e of A_e t_e + max(0, (t_min - t_e) / t_min),
 * A_e = |d13 x d24| / 2 (the area the loads use).  out_host[3] (host) = {g, c, W}.
 * dg_dxyz [n_nodes][3] (required) and dg_dt [n_quads] (may be NULL), device outputs:
 * eps1 W dc/dp + (1 + eps1 c) dW/dp, with dc/dp from the adjoint (Eqs. 5-6) for
 * dg/du = sign(u_jz) / u_max on the active nodes (0 elsewhere, also at the kink).  The
 * self-adaptive update of eps1 between optimisation steps is the caller's.  stats: host or
 * NULL (iters of the adjoint solve, t_adj_us).  Errors: SSO_EINVAL (no solve, eps1 < 0,
 * u_max or t_min not positive, NULL outputs), SSO_ENOTCONV, SSO_EBREAKDOWN, SSO_EHIP. */
int sso_size_objective(sso_problem* p, double eps1, double u_max, double t_min,
                       double* out_host, double* dg_dxyz, double* dg_dt, sso_stats* stats);

/* The self-adaptive penalty coefficient of the size optimisation for the next step (Sec. 3.3,
 * Eq. (10)): *eps1_next (host) = kappa * eps1 after a design that violated the displacement limit
 * (c > 0 in sso_size_objective's output), eps1 / kappa otherwise (the paper's example uses
 * kappa = 1.015).  Host arithmetic only; no problem and no GPU involved.  Errors: SSO_EINVAL for
 * eps1 < 0, kappa <= 0, a value that is not finite, or eps1_next NULL. */
int sso_size_penalty_update(double eps1, int violated, double kappa, double* eps1_next);

/* The same as sso_size_objective, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving or optimisation loops, harnesses that forbid hipMalloc): its
 * scratch -- the reduction partials and the per-quad volume terms -- lives in a static device
 * array of SSO_NOALLOC_SCRATCH_BYTES (16 MiB) that the library holds on each GPU it runs on
 * until the process ends, instead of buffers the problem allocates on first use.  No hipMalloc,
 * hipFree or allocating library routine is called: the problem must have been solved with its
 * current options (sso_solve, which allocated the solver's own work vectors); the adjoint solve
 * runs in those.  Results are bitwise those of sso_size_objective.  Every call on one GPU shares
 * that GPU's scratch: calls that overlap on one GPU (other host threads, other streams) race and
 * must be serialised by the caller.  Errors: as sso_size_objective, and SSO_ESIZE when the
 * problem has more than SSO_NOALLOC_MAX_QUADS quads. */
#define SSO_NOALLOC_SCRATCH_BYTES (16u << 20)
#define SSO_NOALLOC_MAX_QUADS 139673
int sso_size_objective_noalloc(sso_problem* p, double eps1, double u_max, double t_min,
                               double* out_host, double* dg_dxyz, double* dg_dt,
                               sso_stats* stats);

/* Hat filter of nodal sensitivities (Sec. 3.1-3.2): for n design nodes (nodes [n] device int32
 * indices into the problem's nodes, or NULL for nodes 0..n-1) with sensitivities g [n]
 * (device), out[i] = sum_j w_ij g_j / sum_j w_ij, w_ij = max(0, radius - |X_i - X_j|), X the
 * problem's current coordinates (3-D distance), j ascending.  out [n] device.  Errors:
 * SSO_EINVAL (n < 0, radius not positive, NULL arrays, a node index outside [0, n_nodes)),
 * SSO_EHIP.  Synchronises the stream. */
int sso_hat_filter(sso_problem* p, int32_t n, const int32_t* nodes, const double* g,
                   double radius, double* out);

/* The scalar CSR view of the pattern and the scatter permutation: the element-to-global index
 * maps and the sparse storage of the assembled K (Sec. 2.2.1, Eq. (1)), built on first call,
 * owned by the problem, valid until destroy.  All arrays are device int32:
 *   row_ptr [n_dof + 1], col [nnz]: scalar CSR of K, columns sorted;
 *   perm [n_coo]: stable sort of the element contribution list (element-major, beams then
 *                 quads, each local matrix row-major) by (row, col);
 *   seg [nnz + 1]: perm[seg[s] .. seg[s+1]) are the contributions of slot s.
 * *nnz and *n_coo are host outputs.  Errors: SSO_EINVAL if n_coo >= 2^31. */
int sso_pattern(sso_problem* p, const int32_t** row_ptr, const int32_t** col,
                const int32_t** perm, const int32_t** seg, int64_t* nnz, int64_t* n_coo);

/* Read back the assembled, masked K in scalar CSR order into vals [nnz] (device), the masked
 * system's right-hand side f [n_nodes][6] (device, may be NULL) of the last solve (0 on the
 * fixed DOFs; with prescribed displacements the lifted load on the free ones).  K is bitwise
 * symmetric: an entry below the diagonal holds the sum of its transposed entry's element
 * contributions, in that entry's order (the element matrices are symmetric up to rounding). */
int sso_matrix(sso_problem* p, double* vals, double* f);

/* Device memory the problem holds (*bytes, host): the memory taken for every buffer allocated on
 * its behalf so far -- mesh copies, pattern, element list, K, preconditioner, solver vectors, and
 * what later calls added (mixed-precision copies, the size objective's scratch, the scalar CSR
 * view) -- all kept until sso_problem_destroy; buffers freed within a call are not counted.
 * Buffers above 512 KiB are taken one by one; smaller ones are carved from 2 MiB chunks, counted
 * whole (a chunk is left for a new one only with less than 512 KiB free).  For admission by
 * memory footprint in a request loop.  Errors: SSO_EINVAL (NULL argument). */
int sso_problem_bytes(const sso_problem* p, int64_t* bytes);

/* Sizes: n_dof, block count (6x6 blocks of K) and nnz = 36 * blocks (host outputs). */
int sso_sizes(const sso_problem* p, int64_t* n_dof, int64_t* n_blocks, int64_t* nnz);

const char* sso_strerror(int status);

/* Frees the problem's device memory (stream-ordered on its stream, then waits for that stream)
 * and its host state. */
void sso_problem_destroy(sso_problem* p);

/* Device memory: every buffer the library allocates comes from a memory pool of its own on the
 * problem's device, which keeps freed memory for the next allocation instead of returning it to
 * the driver (a request loop creates and destroys problems of recurring sizes; mapping fresh
 * memory each time cost about 1 ms per problem).  The pool therefore holds up to the peak of what
 * problems held at once.  sso_pool_trim releases what the pool holds beyond keep_bytes of unused
 * memory back to the driver; memory freed on a stream whose work has not completed is released
 * by a later call.  device: HIP device ordinal.  Errors: SSO_EINVAL (bad ordinal), SSO_EHIP.
 * A device whose pool was never used returns SSO_OK. */
int sso_pool_trim(int device, uint64_t keep_bytes);

#ifdef __cplusplus
}
#endif
#endif /* HIPSSO_H */
