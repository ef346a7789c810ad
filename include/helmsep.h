/*
 * helmsep.h -- C ABI of the MI355X separable Helmholtz block solver.
 *
 * Druskin & Zaslavsky, "Fast finite-difference convolution for 3D problems in
 * layered media" (arXiv:1909.01299), Sec. 2.  The library solves
 *
 *     A u = f,   A = S (Dx (x) I (x) I + I (x) Dy (x) I) + I (x) I (x) (Dz - diag k^2(z)),
 *
 * the 7-point finite-volume operator of eqs. (2)-(3) divided by its diagonal
 * mass matrices and with the sign chosen so that D_d = M_d^{-1} K_d is positive
 * on a uniform grid, the constant lambda replaced by a layered k^2(z), S =
 * diag(sigma(z)) at the nodes and Dz the flux form with sigma(z) at the z
 * steps (sigma = 1 unless given).  Per axis d with n interior nodes and steps h[0..n] (complex in a
 * PML), node i lies between h[i] and h[i+1], hhat_i = (h[i] + h[i+1]) / 2 and
 * (K u)_i = (u_i - u_{i-1}) / h[i] - (u_{i+1} - u_i) / h[i+1]; the walls carry
 * homogeneous Dirichlet data.
 *
 * The grid may be split by separator planes x = s (s in sep_x) and y = t into
 * Cartesian blocks S^ij = S^i_x x S^j_y x S_z (Sec. 2, eq. (4)); a solve then
 * runs the two-level cyclic reduction of Sec. 2 (block solves, interface
 * residual, global interface solve of eq. (6), local correction of eq. (7)).
 * Without separators it is one separable block solve (eq. (5)): transform x
 * and y by the generalized eigenvectors W^{-1} (a sine transform on a uniform
 * axis), one tridiagonal solve in z per (kx, ky) mode, transform back by W.
 *
 * Conventions for every entry point:
 *  - Arrays f, u, g, a, r are device pointers to contiguous complex128
 *    (interleaved re, im doubles) of shape [nrhs][nz][ny][nx], x fastest.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream); all
 *    device work is enqueued asynchronously on it.  Host arrays are copied
 *    before the call returns.
 *  - The caller owns every array and the workspace; the plan owns its device
 *    tables.  Solve-type calls never allocate device memory.
 *  - Errors are returned as hs_status; the text of the last error on the
 *    calling thread is available from hs_last_error().  Argument errors are
 *    detected on the host before any device work is enqueued.
 *  - One plan may be used by one stream at a time.
 */
#ifndef HELMSEP_H
#define HELMSEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HS_OK = 0,
  HS_ERR_ARG = 1,       /* invalid argument (sizes, steps, separators, pointers) */
  HS_ERR_ALLOC = 2,     /* device allocation for plan tables failed              */
  HS_ERR_DEVICE = 3,    /* no usable device, or a HIP call failed                */
  HS_ERR_SINGULAR = 4,  /* eigen tables or z pivots numerically unusable         */
  HS_ERR_NOCONV = 5,    /* refinement did not reach its tolerance                */
  HS_ERR_STATE = 6      /* call out of order (e.g. no workspace bound)           */
} hs_status;

typedef enum {
  HS_C128 = 0,          /* every transform and sweep in complex128               */
  HS_C64_REFINE = 1     /* complex64 transforms and sweeps, FP64 residual and
                           iterative refinement (not in the paper)               */
} hs_precision;

typedef struct hs_plan_s* hs_plan;
typedef struct hs_batch_s* hs_batch;

/* Grid description (paper Sec. 2: tensor grid with per-axis steps).
 * hx: 2*(nx+1) doubles, complex steps (re, im) h_0..h_nx; likewise hy.
 * hz: nz+1 real steps.  layer_of_z: nz entries in [0, nlayers).
 * k2: 2*nlayers doubles, complex k^2 per layer.
 * sigma_node, sigma_step: the coefficient sigma(z) of eqs. (1)-(2), real and
 * positive, at the nz nodes (it scales the x and y terms of row k) and at
 * the nz+1 z steps (step k joins node k-1 and node k; the z term is the
 * difference of the fluxes sigma u_z through the two steps of a node); both
 * NULL for sigma = 1, both or neither given.  All host pointers. */
typedef struct {
  int32_t nx, ny, nz;
  const double* hx;
  const double* hy;
  const double* hz;
  int32_t nlayers;
  const int32_t* layer_of_z;
  const double* k2;
  const double* sigma_node;
  const double* sigma_step;
} hs_grid;

/* Separator planes (0-based interior indices, strictly increasing, at least
 * one node between neighbours and between a separator and a wall).  A block
 * is a maximal run of nodes between separators (Sec. 2, eq. (4)).  Zero
 * separators = one block.  Any count: the second gridding of Sec. 2 (about
 * sqrt(n) blocks of about sqrt(n) nodes per axis) is the intended use of
 * many.  Up to 4 separators per axis enter the global z solve as low-rank
 * terms; with more, their lines are first expanded into a dense spectral
 * right-hand side (one more write and read of the global grid).  A block
 * side may not exceed 512 nodes. */
typedef struct {
  int32_t nsep_x;
  const int32_t* sep_x;
  int32_t nsep_y;
  const int32_t* sep_y;
} hs_blocks;

typedef struct {
  hs_precision prec;
  int32_t refine_steps;   /* HS_C64_REFINE: correction steps, at most 16 (default 2
                             when 0; a negative value: none, one complex64 pass) */
  int32_t max_rhs;        /* largest nrhs a solve will be called with (>= 1)       */
  int32_t flags;          /* bit 0: force the dense transform on uniform axes;
                             bits 1-2: z-line chunks per mode (0 auto, 1: 8, 2: 16,
                             3: 32; must hold nz within 16 rows per chunk);
                             bit 3: expand the right-hand side of the global
                             interface solve densely (the path taken anyway
                             with more than 4 separators on an axis)            */
  double tol;             /* > 0: every solve ends with the FP64 residual of the u
                             it returns (one more read of f and u, nothing written)
                             and hs_get_info reports HS_ERR_NOCONV when
                             |f - A u| / |f| exceeds tol for some right-hand side;
                             0: no final check (residuals are still recorded for
                             the iterates a refinement step corrects)          */
} hs_options;

typedef struct {
  int32_t nblocks;
  int32_t refine_steps;
  int32_t n_dense_axes;     /* block axes using the dense eigenvector transform */
  int32_t n_sine_axes;      /* block axes using the sine transform              */
  double kappa_max;         /* largest condition number estimate of a W table   */
  double eig_resid_max;     /* max ||D W - W Lambda|| / (||D|| ||W||)            */
  double inv_resid_max;     /* max |W^{-1} W - I|                               */
  double min_pivot;         /* smallest |z pivot| over all modes (FP64 scan)    */
  double plan_seconds;      /* host time spent building the plan               */
  size_t table_bytes;       /* device bytes held by the plan                   */
  int64_t n_fp64_modes;     /* HS_C64_REFINE: modes near resonance (Re(lam_x +
                               lam_y) <= 1.25 max Re k^2) whose z solves run in
                               FP64 with the workgroup that holds them        */
  int32_t z_chunks;         /* z-line chunks per mode in use (hs_plan_tune)   */
  int32_t sine_lines;       /* sine-transform lines per workgroup (0 = default) */
  int32_t z_fixed_rows;     /* 1: z solves in instances with a fixed row count
                               per chunk (chosen by hs_plan_tune)            */
  int32_t global_dense;     /* decomposed grids: 1 when the global interface
                               solve's right-hand side is expanded densely
                               before its z solve, 0 when its separator lines
                               enter the z solve as low-rank terms          */
  int32_t fp64_stream;      /* HS_C64_REFINE: 1 when the FP64 z solves of the
                               near-resonance workgroups run on a second stream
                               beside the FP32 launch, 0 when they run first on
                               the solve's stream (chosen by hs_plan_tune)    */
  int32_t n_split_fp16;     /* HS_C64_REFINE: axes whose dense tables run on fp16
                               matrix cores as two-term splits (n <= 256, or
                               n <= 512 for real sine tables)                */
  /* Convergence record of the last solve (read after its stream has been
   * synchronized).  Every FP64 residual r = f - A u that a solve evaluates
   * (the one each refinement step corrects, and the final one when tol > 0)
   * also yields |r|, |f| and |u| per right-hand side, reduced on the device
   * in a fixed order into the plan workspace. */
  double tol;               /* the plan's hs_options.tol                        */
  double resid_first;       /* max over RHS of |f - A u_0| / |f| for the first
                               pass u_0 (-1: not evaluated)                   */
  double resid_final;       /* the same for the returned u (-1: not evaluated,
                               i.e. tol == 0)                                 */
  int32_t resid_evals;      /* residuals recorded by the last solve            */
  int32_t converged;        /* 1: resid_final <= tol; 0: not (hs_get_info then
                               returns HS_ERR_NOCONV); -1: not checked         */
} hs_info;

/* Build a plan: validates the grid and blocks (HS_ERR_ARG), computes the 1D
 * generalized eigen tables of every block axis and of the global axes in FP64
 * on the host (Sec. 2, A_d W = M_d W Lambda with W = 0 on the block walls),
 * scans the z pivots of every mode, and uploads the tables to the current
 * device (HS_ERR_DEVICE without one).  `blocks` and `opts` may be NULL.
 * Size limits (HS_ERR_ARG beyond them): nx ny nz <= 2^34, nx ny <= 2^28,
 * nz <= 512, every block side <= 512. */
hs_status hs_plan_create(const hs_grid* grid, const hs_blocks* blocks,
                         const hs_options* opts, hs_plan* out);
void hs_plan_destroy(hs_plan plan);

/* Device workspace the caller must bind before solving nrhs right-hand sides. */
size_t hs_plan_workspace_bytes(hs_plan plan, int32_t nrhs);
/* Bind caller-owned device memory of at least hs_plan_workspace_bytes(plan,
 * max_rhs) bytes, 256-byte aligned.  The plan keeps the pointer, not a copy. */
hs_status hs_plan_bind_workspace(hs_plan plan, void* dev_ptr, size_t bytes);

/* Replace the layer values k^2 (2*nlayers host doubles).  Waits for all work
 * on the device (solves in flight read the tables), rebuilds the z tables and
 * re-scans the pivots; synchronous. */
hs_status hs_set_k2(hs_plan plan, const double* k2);

/* u = A^{-1} f for nrhs right-hand sides (Sec. 2, the seven-step algorithm,
 * or eq. (5) for one block).  u may alias f in both precisions (the mixed
 * path then first copies f into the workspace, since its residuals read f
 * after u has been written). */
hs_status hs_solve(hs_plan plan, const void* f, void* u, int32_t nrhs, void* stream);

/* a = A^{-H} g.  Uses the symmetry of the finite-volume matrix M A of eq. (3):
 * A^{-H} g = conj(M A^{-1} M^{-1} conj(g)), so the forward kernels are reused.
 * a may alias g. */
hs_status hs_solve_adjoint(hs_plan plan, const void* g, void* a, int32_t nrhs, void* stream);

/* grad[r][l] = sum over (x, y) and z in layer l of a * conj(u) (complex128,
 * device, nrhs*nlayers entries): the gradient of a real misfit with respect to
 * k^2_l in torch's convention when a = A^{-H} dJ/du. */
hs_status hs_grad_k2(hs_plan plan, const void* u, const void* a, void* grad,
                     int32_t nrhs, void* stream);

/* hs_grad_k2 for callers that cannot allocate device memory at the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same result, bit for bit, with no bound workspace; the
 * partial sums live in a static device array of the library (65536 complex128
 * values, 1 MiB per device, held until the process ends), so nrhs * nz must
 * not exceed 65536 (HS_ERR_ARG otherwise).  Every call on one device shares
 * that array: calls that overlap on one device (different streams, or other
 * threads) race and must be serialized by the caller. */
hs_status hs_grad_k2_noalloc(hs_plan plan, const void* u, const void* a, void* grad, int32_t nrhs,
                             void* stream);

/* r = f - A u in FP64 by the 7-point stencil on the whole grid (eq. (2)). */
hs_status hs_residual(hs_plan plan, const void* f, const void* u, void* r,
                      int32_t nrhs, void* stream);

/* out = A u in FP64 by the same stencil (eqs. (2)-(3)). */
hs_status hs_apply(hs_plan plan, const void* u, void* out, int32_t nrhs, void* stream);

/* Plan statistics and the convergence record of the last solve.  Reads the
 * record from the workspace (synchronous copy; call after the solve's stream
 * has been synchronized).  Returns HS_ERR_NOCONV, with *info filled, when the
 * last solve's final residual exceeded a positive tol. */
hs_status hs_get_info(hs_plan plan, hs_info* info);

/* The relative residuals |f - A u_k| / |f| recorded by the last solve, as
 * rel[k * nrhs + r] for evaluation k (k = 0: the first pass; k = refine
 * steps: the returned u, when tol > 0) and right-hand side r.  max_entries
 * bounds what is written; *n_evals and *nrhs receive the counts.
 * HS_ERR_STATE when no solve has recorded residuals.  Synchronous copy. */
hs_status hs_get_residuals(hs_plan plan, double* rel, int32_t max_entries, int32_t* n_evals,
                           int32_t* nrhs);

/* Autotune the plan's launch shapes for nrhs right-hand sides: every usable
 * combination of z-line chunks per mode in {8, 16, 32}, sine-transform lines
 * per workgroup in {4, 8, 16}, (where nz fills the chunks exactly) z-solve
 * instances with a fixed row count per chunk or not, and (decomposed grids
 * with at most 4 separators per axis) the global right-hand side expanded
 * densely or as low-rank terms, and (HS_C64_REFINE with near-resonance
 * modes) the stream of the FP64 z solves is timed with hipEvents on `stream` on
 * scratch data (each combination's time: its fastest single solve over two
 * passes of three) and the fastest is kept in the plan.  cache_path (may be
 * NULL) names a JSON-lines file keyed by device architecture and plan shape:
 * a hit skips the timing, a miss appends the result.  Needs a bound workspace;
 * allocates and frees two scratch arrays; synchronizes the stream. */
hs_status hs_plan_tune(hs_plan plan, int32_t nrhs, const char* cache_path, void* stream);

/* Nested partitions (Sec. 2, the remark on multi-level cyclic reduction):
 * the interface problem of `plan` (Alg. step 5: A w = r with r on its
 * separator planes) is solved by the cyclic reduction of `coarse` instead of
 * the global eigenvector basis.  coarse: a plan of the same grid (steps,
 * layers, k^2, sigma), precision and device, with max_rhs at least plan's,
 * whose separators are a subset of plan's (it may have none, or a coarser
 * plan of its own: any depth).  The residual on the separators is scattered
 * onto a grid array, solved by coarse's own pass (no refinement of its own)
 * and read back on the separators; the rest of the solve is unchanged.  The
 * plan keeps the pointer: coarse must outlive it, keep a bound workspace and
 * not be used concurrently with it.  hs_set_k2 on plan also sets coarse's
 * k^2.  NULL detaches.  Waits for the device; the workspace layout changes
 * (hs_plan_workspace_bytes grows by two grid arrays per right-hand side) and
 * the bound workspace is released: bind one again before solving.
 * HS_ERR_ARG when coarse does not fit (another grid, precision or device, a
 * separator not in plan's, max_rhs too small, a cycle, a single-block plan). */
hs_status hs_plan_set_coarse(hs_plan plan, hs_plan coarse);

/* Set the launch shapes directly (as hs_plan_tune would store them), e.g. to
 * reuse one plan's tuning on another plan of the same shapes: z_chunks in
 * {0 (default for nz), 8, 16, 32}, sine_lines in {0 (default), 4, 8, 16},
 * z_fixed_rows in {0, 1} (1 is used only where nz fills the chunks exactly),
 * global_dense in {-1 (keep), 0, 1} (ignored on a single block; 0 is refused
 * where more than 4 separators on an axis, or flag bit 3, require the dense
 * expansion), fp64_stream in {-1 (keep), 0, 1} (see hs_info).  Changing global_dense waits for the device and rewrites the
 * plan's descriptors.  HS_ERR_ARG for a value outside these sets or one the
 * plan cannot use (a z chunking that cannot hold nz, sine lines whose LDS
 * does not fit). */
hs_status hs_plan_set_launch(hs_plan plan, int32_t z_chunks, int32_t sine_lines, int32_t z_fixed_rows,
                             int32_t global_dense, int32_t fp64_stream);

/* Per-stage timing.  While enabled, every stage of a solve is bracketed by
 * hipEvents recorded on the solve's stream (events come from a pool created
 * here, so solves still allocate nothing).  hs_profile_read synchronizes on
 * the recorded events and returns, per stage, the accumulated milliseconds,
 * the number of launches and the algorithmic bytes and flops of one launch
 * (compulsory reads and writes of the stage's inputs and outputs; 8 flops per
 * complex multiply-add of a dense transform, the Thomas count of a z sweep).
 * Reading resets the accumulators. */
typedef struct {
  char name[32];
  double ms;
  int64_t launches;
  double bytes_per_launch;
  double flops_per_launch;
} hs_stage_time;

hs_status hs_profile_enable(hs_plan plan, int32_t on);
/* Restrict the events of enabled profiling to the stage named `stage` (a name
 * hs_profile_read reports; other stages then record nothing and add no
 * events to the stream), or record every stage again (stage = NULL).  Names
 * of 32 or more characters are HS_ERR_ARG; an unknown name records nothing. */
hs_status hs_profile_only(hs_plan plan, const char* stage);
hs_status hs_profile_read(hs_plan plan, hs_stage_time* out, int32_t max_out, int32_t* n_out);

/* Batched solve of many independent plans (one block each, any sizes) and
 * right-hand sides, enqueued as one captured HIP graph per call.
 * nrhs[i] right-hand sides for plans[i]; the plans must outlive the batch and
 * share one precision.  The batch copies the plans' tables when it is created:
 * later hs_set_k2 calls on a plan do not reach it (create a new batch).  Its
 * launch shapes start as those of plans[0] and are the batch's own after
 * hs_batch_tune.  Errors: HS_ERR_ARG (decomposed plans, mixed precisions or devices,
 * nrhs outside [1, 4096]), HS_ERR_ALLOC, HS_ERR_DEVICE. */
hs_status hs_batch_create(const hs_plan* plans, int32_t nplans, const int32_t* nrhs,
                          hs_batch* out);
size_t hs_batch_workspace_bytes(hs_batch batch);
hs_status hs_batch_bind_workspace(hs_batch batch, void* dev_ptr, size_t bytes);
/* f[i], u[i]: device arrays of plans[i] with nrhs[i] right-hand sides.  New
 * array pointers make the batch capture its graph again (after waiting for
 * the device, since the previous graph's descriptors are rewritten).  The
 * complex64 path needs u[i] distinct from f[i]. */
hs_status hs_batch_solve(hs_batch batch, const void* const* f, void* const* u, void* stream);
/* Autotune the batch's own launch shapes (z-line chunks, sine lines per
 * workgroup, fixed z-solve rows; as hs_plan_tune, but timed on the whole
 * captured graph of the batch, the fastest of two replays per combination)
 * with the caller's arrays: u is overwritten.
 * cache_path (may be NULL): JSON-lines cache keyed by device, precision and
 * the plans' shapes.  Synchronizes the stream. */
hs_status hs_batch_tune(hs_batch batch, const void* const* f, void* const* u, const char* cache_path,
                        void* stream);
void hs_batch_destroy(hs_batch batch);

/* Host-only 1D generalized eigensolver used by the plan (no device needed):
 * K W = M W diag(lam) for one axis with n interior nodes and complex steps
 * h (2*(n+1) doubles).  Outputs (caller-allocated host arrays): lam 2*n
 * doubles; W and Winv 2*n*n doubles, row-major, W[i][m] = component i of
 * eigenvector m.  stats (may be NULL): [kappa, eig_resid, inv_resid]. */
hs_status hs_axis_eig(int32_t n, const double* h, double* lam, double* W, double* Winv,
                      double* stats);

const char* hs_status_str(hs_status s);
const char* hs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HELMSEP_H */
