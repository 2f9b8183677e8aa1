/*
 * bddc.h - C ABI of the MI355X (gfx950) adaptive BDDC library.
 *
 * The library solves the assembled problem R^T A R u = R^T f of a
 * substructured finite element discretization (Sec. 2, eq. (assembled)) by
 * PCG preconditioned with BDDC in the algebraic form of Algorithm 2 (Sec. 5),
 * with corner, edge-average and adaptively selected face constraints
 * (Sec. 3, Algorithm 1).  Constraints are imposed by the generalized change
 * of variables of Sec. 5 (QR with column pivoting, eq. (T)); every
 * substructure matrix is then factored by dense Cholesky on the GPU.
 *
 * Conventions
 * - Meshes are Q1 hexahedra.  Degrees of freedom are node-major,
 *   component-minor (dpn = 1 for the scalar problem, 3 for elasticity).  The
 *   *global* numbering skips Dirichlet dofs and keeps that order; every
 *   vector passed to apply / solve uses it (length n_glob, see bddc_info).
 * - Ownership: the caller owns every array it passes.  bddc_setup copies
 *   what it needs and keeps no caller pointer.  Vectors passed to
 *   bddc_apply / bddc_pcg_solve are DEVICE pointers (e.g. a torch tensor's
 *   data_ptr()) on the context's device, caller-allocated, used on the
 *   context's stream; the call returns after the result is complete.
 * - Call order: create -> setup -> [adapt] -> factor -> apply / pcg_solve.
 *   adapt changes the constraints and invalidates the factors.  A call out of
 *   order returns BDDC_ERR_STATE.
 * - Errors: no exception crosses the ABI.  Every function returns a status;
 *   bddc_last_error() gives a message for the last failing call on a context.
 * - Threads: one context per host thread.
 */
#ifndef BDDC_H
#define BDDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bddc_ctx bddc_ctx;

typedef enum {
  BDDC_OK = 0,
  BDDC_ERR_ARG = 1,                 /* invalid argument (null pointer, size) */
  BDDC_ERR_STATE = 2,               /* call out of order */
  BDDC_ERR_OOM = 3,                 /* device or host allocation failed */
  BDDC_ERR_NOT_SPD = 4,             /* non-positive pivot in a substructure factor */
  BDDC_ERR_SINGULAR_COARSE = 5,     /* non-positive pivot in the coarse factor */
  BDDC_ERR_NO_CONVERGENCE = 6,      /* PCG hit maxit, or a NaN / breakdown */
  BDDC_ERR_INSUFFICIENT_CORNERS = 7,/* Assumption 1 or 2 cannot hold */
  BDDC_ERR_DEVICE = 8               /* HIP runtime error */
} bddc_status;

/* Library-wide options.  Zero-initialize and set what you need. */
typedef struct {
  int device;                        /* HIP device ordinal; < 0: host-only context
                                        (setup analysis and inspection only; factor,
                                        adapt, apply and solve return BDDC_ERR_STATE) */
  void *hip_stream;                  /* hipStream_t to run on; NULL: library stream */
  int factor_precision;              /* 64 (default, 0 means 64) or 32: the constrained
                                        substructure factor L_rr is kept in FP32 and
                                        the preconditioner's local triangular solves
                                        run in FP32; the factorizations, Phi, the
                                        coarse problem, averaging, Schur operator
                                        and PCG stay FP64 */
  /* optional device allocator (e.g. a framework's caching allocator);
     NULL: hipMalloc / hipFree */
  void *(*alloc)(size_t bytes, void *user);
  void (*free)(void *ptr, void *user);
  void *alloc_user;
  int verbose;                       /* nonzero: per-phase timings on stderr */
  int autotune;                      /* nonzero: the first batched GEMM of each shape
                                        (element type, transposes, batch size, largest
                                        M, N, K) times every tile shape whose result is
                                        bitwise the default one's and keeps the fastest
                                        for the rest of the process; the trials save
                                        and restore the product's output, so results
                                        do not depend on this switch.  The first call
                                        of a shape costs a few extra products. */
  int per_substructure_launches;     /* nonzero: the unbatched baseline.  Every
                                        batched dense operation (Cholesky, TRSM,
                                        GEMM of the interior fronts, the pair
                                        eliminations, reduced pair matrices, K_rr,
                                        Phi, S_pi) runs one launch sequence per
                                        entry; the interior fronts of one
                                        substructure at a time (those of a depth
                                        batched), LOBPCG one face pair per
                                        launch, the PCG's Schur products and
                                        local triangular solves one substructure
                                        per launch.  Data-movement kernels stay
                                        batched.  Results agree with the batched
                                        ones to rounding (tile shapes follow the
                                        batch); the GEMM tuner is not used */
  int chol_launch;                   /* the batched Cholesky factorizations (K_rr, the
                                        coarse matrix, the interior fronts, the pair
                                        eliminations): 0 (default) picks per call,
                                        1 runs one launch per step of the blocked
                                        factorization (block-column update,
                                        diagonal factor, panel solve, trailing
                                        update), 2 always runs the fused launch: one
                                        launch walks every step of every
                                        substructure, tasks taken from a ticket
                                        counter and waiting on device-side
                                        per-entry counters (Sec. 4: the local
                                        factorizations are independent).  0 fuses
                                        batches of up to 40,000 tile tasks, where
                                        that measured faster.  Every setting gives
                                        the same factor, bit for bit */
} bddc_options;

/* Q1 hexahedral mesh (Sec. 2: substructure matrices are subassembled from
   element matrices).  Host pointers. */
typedef struct {
  int kind;                  /* 0: scalar Poisson (1 dof/node), 1: elasticity (3) */
  int64_t n_nodes;
  const double *xyz;         /* n_nodes x 3, row-major */
  int64_t n_elems;
  const int64_t *hex8;       /* n_elems x 8; nodes (0,0,0)(1,0,0)(1,1,0)(0,1,0)
                                (0,0,1)(1,0,1)(1,1,1)(0,1,1) of the element */
  const double *coef;        /* n_elems: conductivity k or Young's modulus E */
  double nu;                 /* Poisson ratio (elasticity) */
  const uint8_t *dirichlet;  /* n_nodes*dpn: 1 = dof fixed to zero */
} bddc_mesh;

/* Nonoverlapping decomposition into substructures (Sec. 2). */
typedef struct {
  int32_t n_sub;
  const int32_t *elem_sub;   /* n_elems, values in [0, n_sub) */
} bddc_partition;

/* Coarse degrees of freedom (Sec. 2 and 7): corners, plus arithmetic averages
   over edges (mode >= 1) and faces (mode >= 2). */
typedef struct {
  int mode;                  /* 0: c, 1: c+e, 2: c+e+f, 3: every glob dof constrained */
  int augment_corners;       /* nonzero: add face nodes as corners until each face
                                pair sees 1 (scalar) / 3 non-collinear (elasticity)
                                corners in its closure (Assumptions 1 and 2) */
  double qr_drop_tol;        /* rows of U with |U_kk| <= tol*|U_11| are dropped
                                (Sec. 5 after eq. (T)); 0 means 1e-10 */
  int adaptive_edges;        /* 0: bddc_adapt keeps only the face part of each
                                adaptive row, as in the paper's computations
                                (Remark after Proposition 1); nonzero: each row d
                                is split into its face part and one row per edge
                                of the face's closure (Sec. 3 after Proposition 1),
                                and the edge rows are added to those edges'
                                constraints, so that every pair problem re-solved
                                on the new constraints stays below tau.  An edge
                                part whose largest entry is at most 1e-8 times the
                                largest entry of d is rounding residue and dropped. */
} bddc_constraints;

typedef struct {
  double rtol;               /* stop when ||r_k||_2 <= rtol ||r_0||_2; 0 means 1e-8 */
  int maxit;                 /* 0 means 1000 */
} bddc_pcg_params;

typedef struct {
  int iters;                 /* PCG iterations (operator applications) */
  int converged;             /* the stopping test ||r_k|| <= rtol ||r_0|| was met */
  double relres;             /* ||r_k|| / ||r_0|| at exit (PCG's own residual) */
  double kappa, lmin, lmax;  /* Lanczos estimates from the CG coefficients */
  double seconds;            /* wall time of the call */
  double true_relres;        /* ||R^T f - R^T A R u|| / ||r_0|| of the returned u, from
                                the substructure matrices A_i (eq. (assembled)) */
  int refinements;           /* correction solves run because true_relres exceeded
                                both rtol and twice residual_floor after the main
                                solve (at most 3, stopping when the true residual
                                stops halving; each solves A d = f - A u with the
                                same preconditioner) */
  int refine_iters;          /* PCG iterations of those correction solves (not in
                                iters, which counts the main solve only) */
  double residual_floor;     /* eps || |A| |u| || / ||r_0||: the rounding scale of
                                evaluating the product A u in FP64; true_relres
                                cannot be shown below about this level */
} bddc_pcg_info;

typedef struct {
  double omega;              /* condition number indicator (eq. (cond-ind)): the
                                largest eigenvalue not selected, over all pairs */
  int64_t nc;                /* rows of D after adaptation */
  int64_t n_added;           /* adaptive face rows added by this call */
  int64_t n_pairs;           /* face pairs solved */
  int64_t lobpcg_iters;      /* total LOBPCG iterations over all pairs */
  int64_t unconverged;       /* pairs whose LOBPCG did not converge */
  double seconds;
  int64_t n_added_edge;      /* adaptive edge rows added (adaptive_edges only; before
                                the QR drops dependent rows) */
} bddc_adapt_info;

typedef struct {
  int64_t n_glob;            /* global dofs (Dirichlet dofs removed) */
  int64_t n_sub;
  int64_t n_corners, n_edges, n_faces;
  int64_t nc;                /* rows of D = sum over globs of m_g (k_g - 1) */
  int64_t n_coarse;          /* coarse unknowns: corner dofs + explicit averages */
  int64_t n_iface_total;     /* sum of substructure interface sizes */
  int64_t max_interior, max_iface;
  double factor_flops;       /* flops of the last bddc_factor (dense, executed) */
  double factor_seconds;
  double apply_bytes;        /* bytes the PCG-internal apply streams per RHS */
  double pcg_iter_bytes;     /* bytes one PCG iteration streams per RHS */
  size_t device_bytes;       /* device memory held by the context */
  int64_t autotune_entries;  /* GEMM shapes tuned so far in this process */
  int64_t fp32_fallbacks;    /* factor_precision 32: substructures whose FP32 local
                                factorization met a non-positive pivot and were
                                factored again in FP64 (stored rounded to FP32) */
} bddc_info;

bddc_status bddc_create(const bddc_options *opt, bddc_ctx **ctx);

/* Sec. 2 (the substructure matrices A_i assembled from the elements of each
   substructure, the restriction R, the globs: faces, edges and corners,
   Assumptions 1 and 2), Sec. 5 (constraint rows H^avg per glob, QR with
   column pivoting, the change of variables T of eq. (T)) and Sec. 7 (weights
   of E from the diagonals of A_i, arithmetic edge averages).  Builds all of
   these on the host from the caller's mesh, partition and constraint choice
   (all host arrays, copied before the call returns; nothing is retained) and
   uploads the substructure matrices to the device.  Dirichlet dofs (mesh
   dirichlet flags) are eliminated after the globs are classified.  Errors:
   BDDC_ERR_ARG for inconsistent inputs (sizes, out-of-range substructure or
   node ids), BDDC_ERR_INSUFFICIENT_CORNERS when augment_corners = 0 and a
   pair of adjacent substructures with a floating member sees fewer than one
   (scalar) or three non-collinear (elasticity) corners (Assumption 2),
   BDDC_ERR_OOM / BDDC_ERR_DEVICE from the upload.  Invalidates earlier
   adaptation and factors. */
bddc_status bddc_setup(bddc_ctx *ctx, const bddc_mesh *mesh, const bddc_partition *part,
                       const bddc_constraints *cons);

/* Algorithm 1: solve the face-pair eigenproblems on the GPU and add, on every
   face, the rows of the eigenvectors with lambda >= tau (edge parts dropped)
   to the constraints chosen at bddc_setup.  Adaptive rows of an earlier call
   are replaced, so the call may be repeated (e.g. for several tau).
   Requires a prior bddc_setup; invalidates factors.  The Dirichlet factors
   and Schur complements it computes are reused by the next bddc_factor. */
bddc_status bddc_adapt(bddc_ctx *ctx, double tau, bddc_adapt_info *info);

/* The "3eigv" variant of Sec. 7: as bddc_adapt, but every face takes the rows
   of its rows_per_face dominant eigenvectors (all of them if the face's pair
   problem has fewer), whatever their eigenvalues; omega is then the largest
   eigenvalue not taken.  rows_per_face >= 1, else BDDC_ERR_ARG.  With three
   rows per face in elasticity the count equals that of the face averages. */
bddc_status bddc_adapt_count(bddc_ctx *ctx, int rows_per_face, bddc_adapt_info *info);

/* The factorization steps of Algorithm 2 (Sec. 5, with the primal assembly
   of the coarse problem of the Remark after it): Dirichlet factors A_II and
   Schur complements S_i (reused from bddc_adapt when it ran last), T_i^T
   S_i T_i split into the remaining (r) and coarse (pi) dofs, the constrained
   local factor K_rr = L L^T, the coarse basis Phi_i = -K_rr^-1 K_r,pi, S_pi^i,
   the assembled coarse matrix and its Cholesky factor; all substructures in
   each batched launch.  Requires bddc_setup; device memory is the
   context's.  Errors: BDDC_ERR_STATE before setup, BDDC_ERR_NOT_SPD naming
   the substructure and pivot of a non-positive pivot in A_II or K_rr,
   BDDC_ERR_SINGULAR_COARSE for the coarse factor, BDDC_ERR_OOM /
   BDDC_ERR_DEVICE. */
bddc_status bddc_factor(bddc_ctx *ctx);

/* z = M_BDDC r (Algorithm 2) for nrhs columns.  r, z: device, n_glob x nrhs,
   column-major with leading dimensions ldr, ldz >= n_glob.  The columns are
   applied in blocks of up to 8: within a block every factor (interior
   fronts, K_rr, Phi, coarse factor) is read once for all its columns.  A
   column's result has the same bits whatever nrhs is. */
bddc_status bddc_apply(bddc_ctx *ctx, int nrhs, const double *r, int64_t ldr, double *z,
                       int64_t ldz);

/* bddc_apply for callers that cannot allocate device memory (code under HIP
   graph capture, tight serving loops, harnesses that forbid hipMalloc): the
   same kernels and results, but the work vectors of the application (local
   stacks, coarse vector, front updates of the interior solves, triangular
   solve counters) live in one static device array of 64 MiB per device
   instead of the context's buffers, and the call allocates nothing (no
   hipMalloc, hipFree or allocating library routine).  Arguments as
   bddc_apply (device vectors owned by the caller; the context must be
   factored).  The call only enqueues work on the context's stream and
   returns before it completes.  A problem whose work vectors exceed the
   array is rejected with BDDC_ERR_ARG and a message giving both sizes.  All
   calls on one device share the array (each clears the part it uses first):
   calls that overlap on one device race. */
bddc_status bddc_apply_noalloc(bddc_ctx *ctx, int nrhs, const double *r, int64_t ldr, double *z,
                               int64_t ldz);

/* Solve R^T A R u = f (Sec. 2, eq. (assembled)) by PCG on the reduced problem
   with the BDDC preconditioner of Algorithm 2 (Sec. 2: zero interface start
   with interior Dirichlet solves, so (I - P)^T is not needed; Sec. 7: stop
   at ||r_k||_2 <= rtol ||r_0||_2, condition number from the Lanczos
   coefficients of CG).  f, u: device, n_glob x nrhs column-major, owned by
   the caller (u written); each column is an independent solve.  Columns are
   solved in blocks of up to 8 by a block PCG in lock step: every
   application of the Schur operator and of the preconditioner reads each
   factor once for the whole block, every column keeps its own scalars and
   stop test, and a column that has stopped is left untouched while the
   others go on.  A column's result (solution, iterations, history, kappa)
   has the same bits whatever nrhs is.  After the stop the true residual of
   the assembled system is computed with the A_i, column by column
   (bddc_pcg_info.true_relres, residual_floor, refinements).  params may be
   NULL (rtol 1e-8, maxit 1000).  info may be NULL, else nrhs entries.
   Errors: BDDC_ERR_STATE before bddc_factor, BDDC_ERR_ARG for bad vectors or
   leading dimensions, BDDC_ERR_NO_CONVERGENCE when a column stops at maxit or
   on a breakdown (its info entry still filled), BDDC_ERR_DEVICE. */
bddc_status bddc_pcg_solve(bddc_ctx *ctx, int nrhs, const double *f, int64_t ldf, double *u,
                           int64_t ldu, const bddc_pcg_params *params, bddc_pcg_info *info);

bddc_status bddc_get_info(const bddc_ctx *ctx, bddc_info *info);

/* Adaptive rows of one face glob (after bddc_adapt), for inspection:
   face index f in [0, n_faces).  Writes up to max_rows rows of n_dofs
   entries (row-major, face dofs in ascending global order), and the face's
   global dof ids if dofs != NULL.  Returns the counts through *rows, *n_dofs
   and the face's two substructures through subs[2]. */
bddc_status bddc_get_face_rows(const bddc_ctx *ctx, int64_t f, int64_t max_rows, double *out,
                               int64_t *dofs, int64_t *rows, int64_t *n_dofs, int32_t *subs);

/* Adaptive rows of one edge glob (after bddc_adapt with adaptive_edges), for
   inspection: edge index e in [0, n_edges).  Rows of n_dofs entries
   (row-major, edge dofs in ascending global order), ordered by face, then by
   eigenvalue (largest first); the edge's global dof ids if dofs != NULL. */
bddc_status bddc_get_edge_rows(const bddc_ctx *ctx, int64_t e, int64_t max_rows, double *out,
                               int64_t *dofs, int64_t *rows, int64_t *n_dofs);

/* Eigenvalues of the last bddc_adapt for face f, descending (up to max). */
bddc_status bddc_get_face_eigs(const bddc_ctx *ctx, int64_t f, int64_t max, double *out,
                               int64_t *count);

/* Relative residual history ||r_k||_2 / ||r_0||_2, k = 0..iters, of the last
   right-hand side solved by bddc_pcg_solve on this context. */
bddc_status bddc_pcg_history(const bddc_ctx *ctx, int64_t max, double *out, int64_t *count);

/* Substructure s as built by bddc_setup: n local dofs (interior first, then
   interface, each ascending in the global numbering), the CSR matrix A_s of
   the subassembled element matrices (Sec. 2) and the weights of the averaging
   operator E on the n - n_interior interface dofs.  Pass NULL arrays to query
   n, n_interior and nnz first; otherwise gdof[n], rowptr[n+1], col[nnz],
   val[nnz], weights[n - n_interior] are written. */
bddc_status bddc_get_substructure(const bddc_ctx *ctx, int32_t s, int64_t *n, int64_t *n_interior,
                                  int64_t *nnz, int64_t *gdof, int64_t *rowptr, int32_t *col,
                                  double *val, double *weights);

/* Kernel timing with HIP events on the context's stream.
   mode 1: phases of factor / apply / PCG (e.g. "factor_trsm_interior", which
           spans many kernel launches) are timed as categories;
   mode 2: every launch of the main kernels is timed under its kernel name
           (e.g. "chol_update_kernel"), so that per-launch averages can be set
           beside a profiler's;
   mode 0: off.
   Every entry keeps the summed time, the number of timed intervals and the
   algorithmic bytes and flops they must move / perform (from the operand
   sizes: one pass over a dense matrix counts its stored entries once).
   Setting a mode clears the statistics.  Timing serializes nothing but adds
   two event records per timed interval. */
typedef struct {
  char name[32];
  double ms;                 /* summed over launches */
  int64_t launches;
  double bytes;              /* summed algorithmic bytes */
  double flops;              /* summed algorithmic flops */
} bddc_kernel_stat;

bddc_status bddc_set_timing(bddc_ctx *ctx, int mode);
/* Writes up to max entries; *count receives the number of categories. */
bddc_status bddc_get_timing(const bddc_ctx *ctx, int max, bddc_kernel_stat *out, int *count);

const char *bddc_last_error(const bddc_ctx *ctx);
void bddc_destroy(bddc_ctx *ctx);

/* ---------------------------------------------------------------------------
   Request server: many independent solves (each a full setup -> adapt ->
   factor -> PCG of the hot path above, on its own mesh) served with
   continuous admission.  Requests are queued in arrival order; the head of
   the queue is admitted as soon as a worker is free and its device-memory
   footprint estimate fits beside those of the requests in flight (a request
   larger than the whole budget runs alone).  Each admitted request runs on
   its worker's own non-blocking stream with stream-ordered allocations, so
   the device work of the requests in flight overlaps, and its memory returns
   to the pool when it finishes.  Results do not depend on what else runs:
   every kernel is deterministic and no reduction crosses requests.

   Footprint estimate (bytes, from the mesh and partition before any
   allocation): 8 * sum over substructures of 6 n_G^2 (Schur complement and
   its work copy, the interface factor and its transpose, the top fronts'
   contribution blocks) plus 6 n_G^2 more when tau > 0 (the face-pair Schur
   complements held during adaptation), plus the CSR matrices and vectors,
   times 1.15.  n_G counts a substructure's non-Dirichlet dofs on nodes it
   shares with another substructure.

   All calls are thread-safe.  Errors of a request (bad input, OOM, non-SPD)
   are reported in its bddc_request_info; the call that returns them
   succeeds. */
typedef struct bddc_server bddc_server;

typedef struct {
  int device;                 /* HIP device ordinal */
  int factor_precision;       /* 64 or 32 (0 means 64), for every request */
  int max_active;             /* requests in flight at once (0 means 4) */
  double hbm_budget_bytes;    /* admission limit on the summed footprint
                                 estimates (0: 80% of the device's free memory) */
  double resident_bytes;      /* > 0: resident factors.  The factored context of
                                 a finished request stays on the device (its
                                 footprint counts in the budget); a later request
                                 on the same problem (mesh, partition,
                                 constraints, tau and load length equal byte for
                                 byte; any load values) skips setup, adaptation
                                 and factorization, and up to 16 queued requests
                                 on it are taken by one worker.  A queue head
                                 whose problem is resident but in use waits for
                                 it (the requests behind it wait too).  Idle
                                 contexts beyond this many bytes of footprint, or
                                 in the way of a new request, are destroyed least
                                 recently used first; their footprints count until
                                 their memory is freed.  The requests taken on
                                 one context are solved as blocks: those with
                                 equal PCG parameters, up to 8 per block, in one
                                 bddc_pcg_solve call with nrhs > 1 (each
                                 request's result has the same bits as when
                                 solved alone); each block's results are
                                 published when it finishes.  0: every request
                                 builds and frees its own context. */
} bddc_server_options;

typedef struct {
  int64_t id;
  int state;                  /* 0 queued, 1 running, 2 done, 3 failed */
  int status;                 /* bddc_status of a failed request, else 0 */
  double submit_s, start_s, done_s;  /* seconds since the server was created */
  double footprint_bytes;     /* the admission estimate */
  int64_t n_glob;
  double omega;               /* adaptation indicator (0 without adaptation) */
  int64_t nc;                 /* rows of D used by the solve */
  bddc_pcg_info pcg;
  char error[160];            /* message of a failed request */
  int reused;                 /* 1: served by a resident factorization */
  int batch;                  /* right-hand sides of the block PCG that solved it */
} bddc_request_info;

bddc_status bddc_server_create(const bddc_server_options *opt, bddc_server **out);
/* Queues one request.  All arrays are host pointers, copied before the call
   returns.  tau > 0 runs bddc_adapt(tau) before the factorization, tau <= 0
   solves with the given constraints only.  f: the load in the global
   numbering of the mesh's non-Dirichlet dofs (ascending node, then
   component); its length n_glob must match the mesh (checked at setup: a
   mismatch fails the request).  params may be NULL (defaults of
   bddc_pcg_solve).  *id receives the request id.  Returns BDDC_ERR_OOM,
   queueing nothing, when the request's footprint estimate alone exceeds the
   admission budget (it could never be admitted). */
bddc_status bddc_server_submit(bddc_server *srv, const bddc_mesh *mesh, const bddc_partition *part,
                               const bddc_constraints *cons, double tau, const double *f,
                               int64_t n_glob, const bddc_pcg_params *params, int64_t *id);
/* Blocks until request id has finished; copies the solution (n_glob host
   doubles) to u when u != NULL and fills info (may be NULL).  The request's
   record is kept until bddc_server_release. */
bddc_status bddc_server_wait(bddc_server *srv, int64_t id, double *u, bddc_request_info *info);
/* Non-blocking state of request id. */
bddc_status bddc_server_query(bddc_server *srv, int64_t id, bddc_request_info *info);
/* Forgets a finished request (its host copy of the solution). */
bddc_status bddc_server_release(bddc_server *srv, int64_t id);
/* Finishes every queued request, then stops the workers and frees the
   server. */
void bddc_server_destroy(bddc_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* BDDC_H */
