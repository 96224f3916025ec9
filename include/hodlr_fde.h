/* hodlr_fde.h -- C ABI of the MI355X (gfx950) HODLR solver for space-fractional
 * diffusion equations (Massei, Mazza, Robol: "Fast solvers for two-dimensional
 * fractional diffusion equations using rank structured matrices").
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Return value: hodlr_status, 0 == HODLR_OK.  Negative values are
 *   host-detected errors (nothing was enqueued); positive values are
 *   numerical conditions reported by the device (valid after the call
 *   returns, since every entry point that reports them synchronises its
 *   stream before returning).
 * - No C++ exception crosses this boundary.
 * - Pointers documented "device" must point to device memory of the current
 *   HIP device (e.g. a torch tensor's data_ptr()).  Pointers documented
 *   "host" are ordinary host memory.
 * - Matrices are column-major, 0-based.  A "batch" is a set of independent
 *   problems whose vectors are concatenated: problem i owns rows
 *   offsets[i] .. offsets[i+1]-1 of every vector argument.
 * - Ownership: the caller owns every buffer it passes.  A matrix built by
 *   hodlr_build_ws lives entirely in the caller's workspace (sized by
 *   hodlr_workspace_size); the library allocates no device memory for it.
 *   A matrix built by hodlr_build, and the other handles, own the device
 *   memory they allocate (tree plan, compressed operator, factors, scratch),
 *   released by the matching *_destroy.  *_destroy(NULL) is a no-op.
 * - Streams: a context wraps one hipStream_t supplied by the caller (NULL =
 *   the legacy default stream); all work is enqueued on it.  One context
 *   must not be used from two host threads at once.
 */
#ifndef HODLR_FDE_H
#define HODLR_FDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HODLR_OK = 0,
  HODLR_EINVAL = -1,     /* bad argument; hodlr_last_arg() names it (1-based) */
  HODLR_ENOMEM = -2,     /* device allocation failed */
  HODLR_EHIP = -3,       /* a HIP runtime call failed */
  HODLR_EWORKSPACE = -4, /* a matrix in a caller workspace needs more of it (a factorisation
                            schedule at launch shapes hodlr_workspace_size did not size) */
  HODLR_ESTATE = -5,     /* call out of order (e.g. solve before factor) */
  HODLR_ESINGULAR = 1,   /* zero or non-finite pivot in a leaf LU */
  HODLR_ENOCONV = 2,     /* refinement missed rtol; the FP64 fallback result is returned */
  HODLR_ERANK = 3        /* a rank cap truncated above the tolerance */
} hodlr_status;

typedef enum {
  HODLR_FP64 = 0,        /* factors stored and applied in FP64 */
  HODLR_MIXED_FP32 = 1,  /* low-rank factors + leaf inverses stored in FP32, FP64 refinement */
  HODLR_MIXED_BF16 = 2   /* low-rank factors in BF16, leaf inverses FP32, FP64 refinement */
} hodlr_precision;

typedef struct hodlr_ctx_s* hodlr_ctx;
typedef struct hodlr_mat_s* hodlr_mat;
typedef struct fde2d_plan_s* fde2d_plan;

/* Space discretisations of an operator. */
typedef enum {
  FDE_FD = 0,   /* shifted Grunwald-Letnikov finite differences (Sec. 2.2.1) */
  FDE_FE = 1    /* P1 (hat-function) finite elements on the uniform grid (Sec. 2.2.2) */
} fde_discretization;

/* One 1D operator.
 * FDE_FD (Sec. 2.2.1, eq. (system_FD)):
 *   M = shift*I + nu*(D+ T_alpha + D- T_alpha^T),   nu = dt / dx^alpha,
 * with T_alpha the lower Hessenberg Toeplitz matrix of Grunwald-Letnikov
 * weights (eq. (toeplitz_FD)).
 * FDE_FE (Sec. 2.2.2, Sec. 3.4.3):
 *   M = shift*E + nu*(D+ T + D- T^T),   E = tridiag(1/6, 2/3, 1/6),
 * the Galerkin matrix shift*Mass - dt (D+ K+ + D- K-) of hat functions of
 * height 1 divided by dx, where K+_ij = <phi_i, d^alpha_+ phi_j> (eq.
 * (fe-int)) = -dx^(1-alpha) T_ij, T_ij = -w_{i-j+1} with
 *   w_m = (1/Gamma(4-alpha)) sum_{t=-2..2} c_t (m-1+t)_+^(3-alpha),
 *   c = (1, -4, 6, -4, 1),
 * and K- = K+^T.  d+- are applied as row scalings (samples at the nodes):
 * with constant coefficients, the case of the paper's finite-element
 * experiment, that is the Galerkin matrix exactly.
 * shift = 1 for the 1D implicit Euler step; shift = 1/2 (+ an ADI shift)
 * for the coefficients of the 2D Sylvester step (eq. (sylv-timestepping),
 * eq. (sylv-timestepping-fe)). */
typedef struct {
  int64_t n;              /* interior grid points, 1 <= N < 2^23 (eq. (part)) */
  double alpha;           /* fractional order, 1 <= alpha <= 2 */
  double dt, dx;          /* time step and grid spacing; nu = dt/dx^alpha */
  double shift;           /* shift s > 0 of the identity (FD) or of the mass matrix E (FE) */
  const double* d_plus;   /* device, n samples d+(x_i) >= 0 */
  const double* d_minus;  /* device, n samples d-(x_i) >= 0 */
  int discretization;     /* fde_discretization; 0 (FDE_FD) in a zero-initialised struct */
} fde_operator;

typedef struct {
  int leaf;               /* maximal leaf size b, 16 <= b <= 64 ("minimal dimension", Sec. 3.4.1) */
  double tol;             /* truncation tolerance eps: blocks are truncated at eps*||M||_2 (Sec. 3.4.1) */
  int prec;               /* hodlr_precision used by hodlr_solve */
  int max_rank;           /* cap on every off-diagonal rank, <= 32 */
  int refine_max;         /* max FP64 refinement sweeps per solve (any precision; 0 = plain solve) */
  double rtol;            /* refinement target ||d||_2 / ||x||_2 for the last correction d */
  int gmres_m;            /* 0: each refinement sweep is d = M_low^{-1} r, x += d; 1..16: each sweep is a
                             cycle of gmres_m GMRES iterations on M d = r, right-preconditioned by the solve
                             with the stored (reduced-precision) factors (GMRES-IR), x += d */
} hodlr_opts;

typedef struct {
  int status;             /* worst hodlr_status seen by the device */
  int refine_iters;       /* refinement sweeps taken (max over problems) */
  double rel_residual;    /* max over problems of ||b - M x||_2/||b||_2 after the call (mixed modes) */
  int max_rank;           /* largest off-diagonal rank of the factors */
  int leaf;               /* problem index of a singular leaf (ESINGULAR), else -1 */
  int row;                /* leaf index of that leaf, else -1 */
  int used_fallback;      /* 1 if any problem fell back to the FP64 factors */
  double rel_correction;  /* max over problems of ||d||_2/||x||_2, d = last refinement correction
                             (estimates the forward error; 0 without refinement) */
  double backward_error;  /* 2D step: ||R||_F / ((a + b) ||X||_F + ||C||_F), R = C - A X - X B^T, with
                             a <= ||A||_2, b <= ||B||_2 the largest diagonal entries of A and B, so an upper
                             bound of the normwise backward error; 0 in 1D */
  double guess_residual;  /* 2D step with a first guess X0: ||C - A X0 - X0 B^T||_F / ||C||_F, the figure
                             its acceptance test reads; 0 otherwise */
} hodlr_info;

typedef struct {
  int batch;              /* number of operators */
  int leaf;               /* leaf size b */
  int max_levels;         /* deepest tree */
  int64_t total_n;        /* sum of n */
  int max_rank_A;         /* rank of the compressed off-diagonal blocks of M */
  int max_rank_factors;   /* rank of the LU factor blocks (0 before hodlr_factor) */
  size_t bytes_factors;   /* bytes read by one single-RHS solve at the chosen precision */
  size_t bytes_device;    /* device memory held by the handle */
  double factor_flops;    /* algorithmic FP64 flops of hodlr_factor (model from the final ranks) */
  double core_flops;      /* part of factor_flops in the small recompression cores (k x k Gram work) of
                             the nodes factored by the split kernels */
  double gram_flops;      /* part of factor_flops in forming Gram matrices of tall factors (split kernels) */
  double leaf_flops;      /* part of factor_flops in the dense leaves (update, LU, inverses) */
  double node_rec_flops;  /* part in the fused node kernels' first launch (Grams, cores, forms of S12, S21) */
  double node_pend_flops; /* part in the fused node kernels' last launch (C, W, pending recompression) */
  double sp_expand_flops; /* part in the subtree products' expansions (leaf blocks and half the level
                             products of U~12, V~21 and the inverse blocks) */
  double sp_project_flops;/* part in the subtree products' projections (the other half of the levels) */
} hodlr_mat_info;

/* ---- context ------------------------------------------------------------ */
hodlr_status hodlr_ctx_create(hodlr_ctx* ctx, void* hip_stream);
void hodlr_ctx_destroy(hodlr_ctx ctx);
int hodlr_last_arg(hodlr_ctx ctx);

/* Per-kernel timing, for measurement runs (the caller that needs kernel
 * durations, e.g. a roofline report or an autotuner).  With timing on, every
 * kernel the library launches for calls made through ctx is bracketed by two
 * HIP events on ctx's stream, and each entry point waits for its kernels
 * before returning; captured time-step graphs are replaced by direct launches.
 * Launch counts and summed durations accumulate per kernel (named by its
 * launch expression) until hodlr_ctx_timing_reset.  Timing perturbs the
 * timings of the calls it brackets only by the event records between launches.
 * hodlr_ctx_timing_entry: i in [0, hodlr_ctx_timing_count); name points into
 * ctx and stays valid until the next reset or ctx destruction. */
hodlr_status hodlr_ctx_set_timing(hodlr_ctx ctx, int enable);
int hodlr_ctx_timing_count(hodlr_ctx ctx);
hodlr_status hodlr_ctx_timing_entry(hodlr_ctx ctx, int i, const char** name, int64_t* launches,
                                    double* total_ms);
void hodlr_ctx_timing_reset(hodlr_ctx ctx);
const char* hodlr_status_string(hodlr_status s);
hodlr_status hodlr_default_opts(hodlr_opts* opts);

/* ---- 1D: build, factor, solve (Sec. 3.4, Sec. 3.5) ----------------------
 * hodlr_build compresses each operator into HODLR form: the Grunwald-
 * Letnikov weights g_k (recursion of Sec. 3.4.2), an ACA of the top-level
 * subdiagonal Toeplitz block (diagonally pivoted, which is a partial
 * Cholesky because that block reversed is a PSD Hankel matrix, Lemma
 * hadamard-product), every other off-diagonal block by restriction and
 * diagonal scaling (Sec. 3.4.2), dense leaves straight from g.
 * ops: host array of `batch` descriptors (their d+/d- pointers are device).
 * The operators are copied; the caller may free d+/d- after the call.   */
hodlr_status hodlr_build(hodlr_ctx ctx, const fde_operator* ops, int batch,
                         const hodlr_opts* opts, hodlr_mat* out);

/* Device memory, in bytes, that hodlr_build_ws needs for these operators and
 * options (ops as for hodlr_build; their d+/d- pointers are not read and may be
 * NULL): the compressed operator of eq. (system_FD) in HODLR form, its LU and
 * inverse factors (Sec. 3.5) with the reduced-precision copies opts->prec
 * asks for, the solve and refinement scratch, and the factorisation schedule
 * at every launch shape hodlr_autotune tries (or that the process has tuned
 * for this tree).  Host-only: no device work.  HODLR_EINVAL (argument 1-4)
 * for arguments hodlr_build would refuse. */
hodlr_status hodlr_workspace_size(const fde_operator* ops, int batch, const hodlr_opts* opts,
                                  size_t* bytes);

/* hodlr_build into caller-owned device memory: every device buffer of the
 * matrix is carved from `workspace` (device, ws_bytes >= hodlr_workspace_size
 * of the same arguments, any alignment), so no later call on the matrix
 * allocates device memory either.  The caller keeps the workspace alive until
 * hodlr_destroy(m) and frees it afterwards; hodlr_destroy releases nothing of
 * it.  HODLR_EINVAL with hodlr_last_arg() == 6 if ws_bytes is too small, 5 if
 * workspace is NULL.  Launch shapes set later by hodlr_set_tuning that
 * hodlr_workspace_size did not size make hodlr_factor return
 * HODLR_EWORKSPACE. */
hodlr_status hodlr_build_ws(hodlr_ctx ctx, const fde_operator* ops, int batch,
                            const hodlr_opts* opts, void* workspace, size_t ws_bytes,
                            hodlr_mat* out);

/* Time-dependent coefficients d+(x, t), d-(x, t) (the paper assumes them
 * constant in time, Sec. 2.2.1, which lets one LU serve every step; with
 * coefficients that change, the matrix of eq. (system_FD) changes every
 * step).  Replaces the d+/d- samples of every problem of m by those of ops
 * (host array of m's batch size; n, alpha, dt, dx and shift must equal the
 * values m was built with, else HODLR_EINVAL with argument 3) and rebuilds
 * the compressed operator in place: truncation tolerances from the new
 * coefficients, the Hankel compression and the assembly of all blocks and
 * leaves.  The weights, the exact-residual tables, the tree and the
 * factorisation schedule are kept.  m must be factored again before it is
 * solved with (HODLR_ESTATE otherwise). */
hodlr_status hodlr_update_coefficients(hodlr_ctx ctx, hodlr_mat m, const fde_operator* ops);
/* Releases m.  Waits for the device to be idle, then frees the device memory
 * hodlr_build allocated for m (a matrix of hodlr_build_ws holds none).  With
 * the environment variable HODLR_POOL=1 the blocks go to a process-wide pool
 * instead (per device, at most 160 GB), from which a later matrix that needs
 * blocks of exactly the same sizes takes them; an allocation that fails then
 * releases the pool and is retried. */
void hodlr_destroy(hodlr_mat m);
hodlr_status hodlr_get_info(hodlr_mat m, hodlr_mat_info* info);

/* The generator the library computed for problem `item` of the batch:
 * g_0 .. g_{count-1}, count <= n + 3, copied to host memory `out` (the
 * call waits for the context's stream).  FDE_FD: the Grunwald-Letnikov
 * weights of eq. (Grun) by the recursion of Sec. 3.4.2; FDE_FE: the P1
 * stiffness generator w_m of eq. (fe-int) (see fde_operator), each evaluated
 * in double-double arithmetic and rounded once.  Errors: HODLR_EINVAL for a
 * null handle (2), item out of range (3), null out (4), count out of range (5). */
hodlr_status hodlr_get_weights(hodlr_ctx ctx, hodlr_mat m, int item, double* out, int64_t count);

/* y = M_H x with the compressed HODLR operator (Sec. 3.4.1).  x, y device,
 * concatenated over the batch, nrhs columns with leading dimension ld. */
hodlr_status hodlr_matvec(hodlr_ctx ctx, hodlr_mat m, const double* x, double* y,
                          int nrhs, int64_t ld);

/* y = M x exactly (up to FFT rounding) through circulant embedding of the
 * Toeplitz matrices (the FFT matrix-vector product of Sec. 3.4.2); the near
 * band, the shift term and the finite-element mass matrix are summed in
 * double-double.  Used as the refinement residual.  Same layout as
 * hodlr_matvec. */
hodlr_status hodlr_toeplitz_matvec(hodlr_ctx ctx, hodlr_mat m, const double* x, double* y,
                                   int nrhs, int64_t ld);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): the product of
 * hodlr_toeplitz_matvec, same arguments, same results, with its transform
 * scratch in a static device array of the library (16 MiB per GPU, held until
 * the process ends) instead of the handle's own scratch; columns go one at a
 * time.  Allocates nothing.  The matrix must need at most 16 MiB of packed
 * scratch (2 M complex doubles per problem, M the power of two >= 2n - 1: for
 * example two problems of 65536 rows, or one of 262144), else HODLR_EINVAL
 * (argument 2) and a
 * message on stderr.  All calls on one GPU share its array: calls that overlap
 * on one GPU (two streams, two host threads) race and must be serialised by
 * the caller. */
hodlr_status hodlr_toeplitz_matvec_noalloc(hodlr_ctx ctx, hodlr_mat m, const double* x, double* y,
                                           int nrhs, int64_t ld);

/* HODLR LU of every operator (Sec. 3.5): block LU with leaf partial pivoting,
 * low-rank Schur-complement updates recompressed to the truncation
 * tolerance, plus the HODLR inverses of both triangular factors. */
hodlr_status hodlr_factor(hodlr_ctx ctx, hodlr_mat m, hodlr_info* info);

/* Launch-shape autotuner of the factorisation (a production pattern, not part
 * of the paper).  Times the factorisation kernels of m (HIP events, best of two
 * runs) in a coordinate search over: the largest child size (rows) of a node
 * whose phase A runs as fused single-work-group kernels (0, 128, 256, 512,
 * 1024; 0 = never), rows per Gram partial of the other nodes (128, 256, 512),
 * and the work-group size of the leaves (256 or 512 threads; the
 * recompression cores always run with 256).  Keeps the fastest for m and for every matrix of the same
 * tree signature (batch, total rows, depth, leaf size) built later in the
 * process.  The trial runs overwrite m's factors: call hodlr_factor afterwards.
 * best (may be NULL): the chosen shapes and their factorisation time. */
typedef struct {
  int core_threads;
  int leaf_threads;
  int gram_rows;
  int fuse_rows;
  double factor_ms;
} hodlr_tuning;
hodlr_status hodlr_autotune(hodlr_ctx ctx, hodlr_mat m, hodlr_tuning* best);

/* Sets m's factorisation launch shapes (core_threads: 256; leaf_threads: 256
 * or 512; gram_rows: 32 .. 65536, a multiple of 32; fuse_rows >= 0; factor_ms is
 * ignored), for instance ones found by hodlr_autotune on another matrix.  Any
 * other value: HODLR_EINVAL (argument 3).  The factors computed with any valid
 * shape agree up to the rounding order of the Gram sums. */
hodlr_status hodlr_set_tuning(hodlr_ctx ctx, hodlr_mat m, const hodlr_tuning* t);

/* x <- M^{-1} x for every problem and column (Sec. 3.5 back substitution,
 * applied through the HODLR inverses of the triangular factors).  With
 * opts.refine_max > 0 the solve is followed by FP64 iterative refinement whose
 * residual is hodlr_toeplitz_matvec, until the correction satisfies
 * ||d||_2 <= rtol ||x||_2 (the residual of a stiff M floors near u ||M|| ||x||); a
 * mixed-precision solve that stalls falls back to the FP64 factors (status
 * HODLR_ENOCONV, info->used_fallback = 1).  x: device, ld >= total n.
 * info: host, may be NULL. */
hodlr_status hodlr_solve(hodlr_ctx ctx, hodlr_mat m, double* x, int nrhs, int64_t ld,
                         hodlr_info* info);

/* Implicit Euler time stepping (eq. (system_FD)):  u <- M^{-1}(u + fscale*f),
 * `steps` times, for every problem of the batch at once (fscale = dt for the
 * scheme of eq. (system_FD) with a time-independent source).  u, f device
 * (concatenated, one column); f may be NULL (f = 0).  The per-step kernel
 * sequence (right-hand side, solve at the stored precision, refine_max FP64
 * refinement sweeps with the exact residual) is captured once into a HIP graph
 * and replayed.  With refine_max > 0 every step's last correction d is checked
 * on the device: the steps run in groups of 32, each group from a copy of u and
 * ending with one read-back of the worst ||d||_2/||u||_2 of its steps; a group
 * in which any step of any problem missed opts.rtol (or went non-finite) is
 * restored and redone step by step on the FP64 factors, each step refined until
 * it converges or stalls (info->used_fallback = 1).  Returns HODLR_ENOCONV
 * (with or without info) if a step still missed rtol.  info->rel_correction:
 * the worst ||d||_2/||u||_2 over all steps and problems (0 without refinement);
 * info->rel_residual: the last step's ||b - M u||_2/||b||_2. */
hodlr_status hodlr_time_steps(hodlr_ctx ctx, hodlr_mat m, double* u, const double* f,
                              double fscale, int steps, hodlr_info* info);

/* ---- 2D: per-step Sylvester equation (Sec. 4.2-4.3) ----------------------
 * A U + U B^T = C with A = 1/2 I + nu_x(D1+ T + D1- T^T) (x direction),
 * B = 1/2 I + nu_y(...) (y direction), C = U_m + dt F (eq. (sylv-timestepping)).
 * Solved by factored ADI with shifted HODLR solves: the plan builds and
 * factors A + q_j I and B + p_j I for J shift pairs chosen from the spectral
 * intervals (FP64).  Low-rank matrices are X = Z W^T, device, column-major. */
typedef struct {
  int64_t rows;           /* rows of Z (nx) -- W has ny rows */
  int rank;               /* columns in use */
  int capacity;           /* allocated columns (outputs: max rank accepted) */
  int64_t ldz, ldw;       /* leading dimensions */
  double* Z;              /* device */
  double* W;              /* device */
} lr_matrix;

typedef struct {
  double tol;             /* target relative accuracy of each step (see fde2d_sylvester_step) */
  int max_shifts;         /* cap on J, the number of shift pairs (<= 64) */
  int max_rank;           /* cap on the rank of the solution factors (<= 32) */
} fde2d_opts;

/* Plan for one 2D problem: opx, opy are the 1D operators of the x and y
 * directions with shift 1/2 (the split of the identity in Sec. 4.2).  The
 * spectral intervals [s, s + 2 nu alpha max(d+ + d-)] (Gershgorin, strict
 * diagonal dominance of Sec. 2.2.1) fix J and the shifts (Zolotarev problem,
 * elliptic functions); A + q_j I and B + p_j I are built as one batched HODLR
 * operator and factored with hopts (prec selects the factor precision). */
hodlr_status fde2d_plan_create(hodlr_ctx ctx, const fde_operator* opx, const fde_operator* opy,
                               const hodlr_opts* hopts, const fde2d_opts* opts, fde2d_plan* out);
/* Device memory, in bytes, that fde2d_plan_create_ws needs for these
 * arguments: the shifted factor sets (2J HODLR operators, J fixed from the
 * spectral intervals as fde2d_plan_create fixes it, which reads the d+/d-
 * samples), the unshifted A and B for the exact residual, and the sweeps'
 * low-rank work arrays.  No device memory is allocated. */
hodlr_status fde2d_plan_workspace_size(hodlr_ctx ctx, const fde_operator* opx, const fde_operator* opy,
                                       const hodlr_opts* hopts, const fde2d_opts* opts, size_t* bytes);
/* fde2d_plan_create into caller-owned device memory (workspace: device,
 * ws_bytes >= fde2d_plan_workspace_size of the same arguments, any alignment):
 * the plan's HODLR batches and work arrays are carved from it and the library
 * allocates no device memory for the plan.  Keep the workspace alive until
 * fde2d_plan_destroy.  HODLR_EINVAL with hodlr_last_arg() == 7 if ws_bytes is
 * too small, 6 if workspace is NULL. */
hodlr_status fde2d_plan_create_ws(hodlr_ctx ctx, const fde_operator* opx, const fde_operator* opy,
                                  const hodlr_opts* hopts, const fde2d_opts* opts, void* workspace,
                                  size_t ws_bytes, fde2d_plan* out);
/* Work counters of a plan, for measurement (a roofline report): values[0] the
 * algorithmic flops of the low-rank recompression cores run so far (a model of
 * each core on R concatenated columns with output rank r: 2R^2 + 4R^3/3 +
 * 4R^2(r+1) + 4R^2 r), values[1] the flops of the dense residual sums
 * (2 nx ny K for K columns), values[2] the bytes one single-column solve of all
 * shifted operators reads (hodlr_mat_info.bytes_factors of the shifted batch),
 * values[3] J, values[4] the largest factor rank, values[5] the shift pairs of
 * the extended Krylov solver's projected equation (0 before its first use),
 * values[6] the flops of its dense products (2 M N K per k_ek_gemm launch,
 * N before clipping to a device-held width, so an upper bound); up to count
 * values.  Waits for the device.  reset != 0 clears the three flop counters. */
hodlr_status fde2d_plan_counters(fde2d_plan p, double* values, int count, int reset);
void fde2d_plan_destroy(fde2d_plan p);
int fde2d_plan_shifts(fde2d_plan p, double* p_shifts, double* q_shifts, int cap);

/* One implicit Euler step of eq. (sylv-timestepping): U_next solves
 *   A X + X B^T = C,  C = U_m + dt F,
 * with every matrix in low-rank form.  With finite-element operators
 * (FDE_FE) the step is that of eq. (sylv-timestepping-fe),
 *   A X E_y + E_x X B^T = C,  C = E_x (U_m + dt F) E_y,
 * E the mass matrices, solved by the same sweeps in generalized form: the
 * shifted solves use A + q_j E_x and B + p_j E_y, the fADI residual factors
 * are updated through E, and no inverse of E is formed; A X, X B^T below read
 * A X E_y, E_x X B^T and ||A|| + ||B|| reads ||A|| ||E_y|| + ||E_x|| ||B||.  U_m: input, at most 64 columns; F: at
 * most 32 (rank 0 allowed).  C, recompressed, is the right-hand side of a
 * first factored ADI sweep with the plan's shifted HODLR solves, run until the
 * fADI residual G_J H_J^T is below opts.tol * ||C||_F; its result (recompressed
 * at opts.tol / 10) is the main term X_main of the solution.  The residual
 * R = C - A X - X B^T of the current solution is then formed entry by entry
 * from the factors (C from the caller's U_m and F, A Z and B W by the exact
 * Toeplitz products), which resolves ||R||_F to about u times the size of its
 * terms, and while the normwise backward error info->backward_error exceeds
 * opts.tol, or (reduced-precision factors) while the forward-error estimate
 * of iterative refinement |D_k|^2 / (|D_{k-1}| |X_main|) (D_0 = X_main; at
 * least one correction; BF16 factors, whose late corrections shrink slowly and
 * unsteadily: |D_k| / |X_main|) exceeds opts.tol (at most 6 times), a correction
 * sweep solves A D + D B^T = R (R
 * compressed by a randomized range finder on its factors) and D joins the
 * correction term X_corr (recompressed so that its truncation changes the
 * backward error by at most opts.tol / 10).  The two terms are kept apart
 * because a recompression of a sum resolves its smaller term only to about
 * sqrt(u) times the larger one.
 * U_next = [Z_main, Z_corr][W_main, W_corr]^T: caller-allocated factors with
 * `capacity` (>= the rank used, <= 64) columns; on return U_next->rank is the
 * rank used.  HODLR_ENOCONV if the backward error (or, reduced precision, the
 * forward-error estimate) is still above opts.tol after the corrections, HODLR_ERANK
 * if the correction term hit its rank cap.
 * info->rel_residual: ||R||_F / ||C||_F of the returned solution;
 * info->rel_correction: the last correction relative to ||X_main||_F;
 * info->refine_iters: ADI steps taken in total; info->max_rank: U_next->rank. */
hodlr_status fde2d_sylvester_step(hodlr_ctx ctx, fde2d_plan p, const lr_matrix* U_m,
                                  const lr_matrix* F, double dt, lr_matrix* U_next,
                                  hodlr_info* info);
/* fde2d_sylvester_step with the extended Krylov subspace method of Sec. 4.3
 * in place of each fADI sweep (the first solve and every correction): the
 * orthonormal bases U of EK(A, G) = span{G, A^-1 G, A G, A^-2 G, ...} and V
 * of EK(B, H), for the right-hand side G H^T of the solve, grow by an operator
 * block and an inverse block per iteration (two extended block Arnoldi
 * processes: A, B by the exact Toeplitz products, A^-1, B^-1 by plain HODLR
 * solves with the unshifted factors of A and B, which the first call
 * factors with the plan's hopts and keeps); a new block is orthogonalised
 * against its basis and loses its directions below 1e-10 of its norm
 * (deflation).  The projected equation (U^T A U) Y + Y (V^T B V)^T =
 * (U^T G)(V^T H)^T, at most 640 x 640, is solved on the device by factored ADI
 * on explicit inverses (LU with partial
 * pivoting) of the shifted projected matrices, until the residual of U Y V^T
 * (formed from three orthogonal terms) is at most the solve's target; the
 * solve's result U Y V^T is then compressed to at most 32 columns.
 * HODLR_ESINGULAR if a shifted projected matrix has an exactly zero pivot.
 * Finite elements: the same on E_x^-1 A D + D (E_y^-1 B)^T = (E_x^-1 G)(E_y^-1 H)^T
 * (the operator products followed by tridiagonal mass solves, the inverses
 * as A^-1 E; its residual bounds the generalized one, E's eigenvalues being
 * below 1).  Arguments, outputs and stopping as fde2d_sylvester_step, except
 * that info->refine_iters counts extended Krylov iterations.
 * The solver's arrays (bases, projected matrices and their 2 x J shifted
 * inverses, at most 640 x 640 each) are allocated on the first call; a plan
 * made by fde2d_plan_create_ws takes them from the workspace given by
 * fde2d_ek_attach_workspace instead, and without one returns
 * HODLR_EWORKSPACE.  The plan's shifted factor sets are not used: the
 * projected equation takes its own Zolotarev shift pairs on the plan's
 * spectral intervals, as many as opts.tol / 10 needs (at most 64), so a plan
 * made for this entry point alone may set max_shifts = 1. */
hodlr_status fde2d_sylvester_step_ek(hodlr_ctx ctx, fde2d_plan p, const lr_matrix* U_m,
                                     const lr_matrix* F, double dt, lr_matrix* U_next,
                                     hodlr_info* info);
/* Device bytes of the extended Krylov solver's arrays for plan p
 * (fde2d_sylvester_step_ek), including the alignment slack of a workspace
 * that fde2d_ek_attach_workspace takes.  Allocates nothing. */
hodlr_status fde2d_ek_workspace_size(hodlr_ctx ctx, fde2d_plan p, size_t* bytes);
/* Give a plan made by fde2d_plan_create_ws the caller-owned device memory
 * for the extended Krylov solver's arrays (workspace: device, ws_bytes >=
 * fde2d_ek_workspace_size, any alignment; keep it alive until
 * fde2d_plan_destroy).  Once per plan: HODLR_ESTATE for a plan without a
 * workspace or with one already attached; HODLR_EINVAL with hodlr_last_arg()
 * == 4 if ws_bytes is too small, 3 if workspace is NULL. */
hodlr_status fde2d_ek_attach_workspace(hodlr_ctx ctx, fde2d_plan p, void* workspace, size_t ws_bytes);

/* As fde2d_sylvester_step, starting from a first guess X0 of the solution
 * (low-rank, rank <= opts.max_rank; NULL or rank 0: no guess).  The exact
 * residual R = C - A X0 - X0 B^T becomes the right-hand side of the first
 * sweep, whose result corrects X0.  The J shift pairs of the plan reduce a
 * residual by about (0.1 opts.tol)^(1/J) per shift; if ||R||_F / ||C||_F
 * exceeds (0.1 opts.tol)^(4/J) (the guess would save less than one block of
 * four shifts), or R needs more than 31 columns to meet its tolerance, the
 * guess is dropped and the plain step runs (info->used_fallback = 1).  The ADI sweeps apply the
 * shift pairs in an interleaved order and stop once the fADI residual is below
 * opts.tol * ||C||_F, so a guess with a small residual takes fewer ADI steps
 * (info->refine_iters).  Argument 7 is U_next.  The learned warm start of the
 * 2D time stepper (a network's prediction of U^{m+1}, compressed by
 * fde2d_compress_field) is what this entry point is for. */
hodlr_status fde2d_sylvester_step_guess(hodlr_ctx ctx, fde2d_plan p, const lr_matrix* U_m,
                                        const lr_matrix* F, double dt, const lr_matrix* X0,
                                        lr_matrix* U_next, hodlr_info* info);

/* Dense field out[i + j nx] = (X)(i, j) for X = Z W^T (FP32, device, nx x ny
 * column-major, nx, ny of the plan). */
hodlr_status fde2d_field_from_lr(hodlr_ctx ctx, fde2d_plan p, const lr_matrix* X, float* out);

/* Low-rank approximation of a dense field (FP32, device, nx x ny column-major)
 * by a randomized range finder: a 32-column sketch X Om with uniform random Om
 * (counter-based generator, `seed`), two orthonormalising passes, then X^T Q,
 * truncated at tol ||X||_F and at min(out->capacity, opts.max_rank) columns.
 * out: caller-allocated factors; out->rank is set. */
hodlr_status fde2d_compress_field(hodlr_ctx ctx, fde2d_plan p, const float* X, double tol,
                                  uint64_t seed, lr_matrix* out);

/* ---- learned warm start: the network --------------------------------------
 * Not part of the paper: a four-layer 3x3 convolutional network predicts
 * u_{k+1} ~ u + net(u) from u = u_k on the 2D grid (zero padding = the
 * absorbing boundary); channels 1 -> 32 -> 32 -> 32 -> 1, ReLU after the first
 * three layers.  Parameters (FP32, fde_net_param_count() of them, in this
 * order): w1[32][1][3][3], b1[32], w2[32][32][3][3], b2[32], w3[32][32][3][3],
 * b3[32], w4[1][32][3][3], b4[1]; w[o][c][p][q] multiplies input channel c at
 * the neighbour (i + p - 1, j + q - 1) for output channel o.  Hidden
 * activations are stored in BF16 (act_bf16 = 1: the 32 -> 32 layers run on
 * BF16 matrix cores with FP32 accumulation) or FP32 (act_bf16 = 0); weights,
 * gradients and Adam state are FP32.  Images: n x h x w row-major FP32, device;
 * n*h*w <= max_pixels. */
typedef struct fde_net_s* fde_net;
int fde_net_param_count(void);
hodlr_status fde_net_create(hodlr_ctx ctx, int act_bf16, int64_t max_pixels, fde_net* out);
void fde_net_destroy(fde_net net);
/* host arrays of fde_net_param_count() floats; set_params also clears the Adam state */
hodlr_status fde_net_set_params(hodlr_ctx ctx, fde_net net, const float* params, int count);
hodlr_status fde_net_get_params(hodlr_ctx ctx, fde_net net, float* params, int count);
/* gradients of the last fde_net_train_step */
hodlr_status fde_net_get_grads(hodlr_ctx ctx, fde_net net, float* grads, int count);
/* pred = u + net(u) */
hodlr_status fde_net_forward(hodlr_ctx ctx, fde_net net, const float* u, int n, int h, int w,
                             float* pred);
/* One step on the batch: loss = mean over the interior (margin pixels left out
 * on every side) of (pred - target)^2, its gradients, and, if update != 0, an
 * Adam step (beta1 = 0.9, beta2 = 0.999, eps = 1e-8) with learning rate lr.
 * loss (host, may be NULL) is written after the device work completes. */
hodlr_status fde_net_train_step(hodlr_ctx ctx, fde_net net, const float* u, const float* target,
                                int n, int h, int w, int margin, float lr, int update,
                                double* loss);

#ifdef __cplusplus
}
#endif
#endif /* HODLR_FDE_H */
