/*
 * cta.h -- C ABI of the MI355X (gfx950) tensor-equation solver.
 *
 * The library solves the regularised tensor equation
 *
 *     N(X) = X x_1 G_1 ... x_N G_N + lambda * sum_k X x_k R_k = B,
 *     G_k = A_k^T A_k,  R_k = D_k^T D_k,  B = Y x_1 A_1^T ... x_N A_N^T,
 *
 * built from the paper's separable transformation (Sec. 2.1, eq.
 * separable_transf), its tensor equation (Sec. 3, eq. TensorEq), the
 * normal-equation pattern A^T A of tensor transposition (App. A.7) and the
 * Kronecker-sum regulariser of the discrete Poisson equation (Sec. 4.1), with
 * the tensor conjugate gradients of Fig. Tensor_CG.  The operator is never
 * formed: it is applied as a chain of mode products (Sec. 4.1: sequential
 * separable transformations along individual dimensions).
 *
 * Conventions for every call:
 *  - Tensors are dense, row-major (C order): mode 1 varies slowest, mode N is
 *    contiguous.  Matrices are row-major.  A mode product X x_k M contracts
 *    the column index of M with index k of X and puts the row index of M at
 *    position k (ordered spaces, Sec. 2.1).
 *  - Pointers named host_* are host memory; every other data pointer is
 *    device memory on the current HIP device.  Tensor pointers must be
 *    aligned to 16 bytes.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is enqueued on that stream.  Calls marked "asynchronous" return
 *    after enqueueing; the caller synchronises before reading results.
 *  - The caller allocates and owns every tensor it passes.  Handles own only
 *    their factor copies and workspace and release them in *_destroy.
 *  - Errors are reported by status code only; no call aborts or throws.
 *    cta_last_error() returns a thread-local message for the last non-OK
 *    status returned on the calling thread.
 *  - One handle is used from one host thread and one stream at a time.
 */
#ifndef CTA_H
#define CTA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CTA_OK = 0,
    CTA_NOT_CONVERGED = 1,   /* result written, tolerance not reached */
    CTA_ERR_ARG = -1,        /* null pointer, bad count, bad option value */
    CTA_ERR_SHAPE = -2,      /* extents inconsistent or above the limits */
    CTA_ERR_DTYPE = -3,      /* dtype combination not supported */
    CTA_ERR_HIP = -4,        /* a HIP runtime call failed */
    CTA_ERR_NOMEM = -5,      /* device allocation failed */
    CTA_ERR_BREAKDOWN = -6,  /* CG breakdown: <p, N p> <= 0 or non-finite */
    CTA_ERR_UNSUPPORTED = -7 /* valid request outside what this build handles */
} cta_status;

typedef enum { CTA_F64 = 0, CTA_F32 = 1, CTA_BF16 = 2 } cta_dtype;

/* Arithmetic of the operator chain inside a solve or an operator apply.
 *  CTA_PREC_F64        FP64 tensors, FP64 MFMA, FP64 dots.
 *  CTA_PREC_F32        FP32 tensors, FP32 MFMA, FP64 dots.
 *  CTA_PREC_BF16       FP32 vectors; chain inputs and intermediates rounded to
 *                      BF16 (nearest-even), BF16 MFMA with FP32 accumulation;
 *                      regulariser in FP32; FP64 dots.
 *  CTA_PREC_BF16_REFINE  (solves only) FP64 outer iterative refinement with an
 *                      FP64 residual recomputation, inner CG in CTA_PREC_BF16
 *                      restarted from zero at every outer step.
 *  CTA_PREC_BF16_RELIABLE  (solves only) one CG in CTA_PREC_BF16 with reliable
 *                      updates: whenever the recursive residual has dropped by
 *                      inner_rtol since the last update, the FP32 correction is
 *                      added to the FP64 solution, the residual is replaced by
 *                      the FP64 true residual and the iteration continues with
 *                      the same search direction (beta rescaled by
 *                      rho_true / rho_recursive). */
typedef enum {
    CTA_PREC_F64 = 0,
    CTA_PREC_F32 = 1,
    CTA_PREC_BF16 = 2,
    CTA_PREC_BF16_REFINE = 3,
    CTA_PREC_BF16_RELIABLE = 4
} cta_precision;

/* Largest extent of any mode (rows or columns of any factor). */
#define CTA_MAX_EXTENT 256
/* Largest tensor order. */
#define CTA_MAX_ORDER 8

const char* cta_last_error(void);
/* Library version string, e.g. "cta 0.1.0 gfx950". */
const char* cta_version(void);

/* ------------------------------------------------------------------------
 * General multi-mode product (Sec. 2.1, eq. separable_transf; Sec. 2, eq.
 * first_product restricted to separable operators).
 *
 * Y = X x_{k in mode_mask} op_k(M_k), op_k(M) = M, or M^T when bit k of
 * trans_mask is set.  M_k is stored row-major with m_rows[k] x m_cols[k]
 * entries; op_k(M_k) must have as many columns as X has extent on mode k, and
 * its row count is the extent of Y on mode k.  Modes outside mode_mask are
 * copied unchanged.  The evaluation order is chosen by the library to
 * minimise flops (products on distinct modes commute, Sec. 2.1).  Arrays
 * x_dims, M, m_rows, m_cols have `order` entries (entries of modes outside
 * mode_mask are ignored).  Inputs and outputs may be F64, F32 or BF16 in any
 * combination; `compute` fixes the MFMA arithmetic and the storage type of
 * intermediates.  Workspace: device memory of at least
 * cta_ttm_workspace_bytes(...) bytes, owned by the caller, not retained.
 * Asynchronous.  X and Y must not overlap.
 * ---------------------------------------------------------------------- */
size_t cta_ttm_workspace_bytes(int order, const int64_t* x_dims, uint32_t mode_mask,
                               uint32_t trans_mask, const int64_t* m_rows,
                               const int64_t* m_cols, cta_dtype compute);
cta_status cta_ttm(int order, const int64_t* x_dims, const void* X, cta_dtype x_dtype,
                   uint32_t mode_mask, uint32_t trans_mask, const void* const* M,
                   const int64_t* m_rows, const int64_t* m_cols, cta_dtype m_dtype,
                   cta_dtype compute, void* Y, cta_dtype y_dtype, void* workspace,
                   size_t workspace_bytes, void* stream);

/* cta_ttm without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The workspace (padded factor copies and
 * the chain intermediates, the bytes cta_ttm_workspace_bytes reports) comes
 * from a fixed array of CTA_TTM_SCRATCH_BYTES in the library's device memory,
 * one per GPU, held until the process ends; products that need more return
 * CTA_ERR_SHAPE.  No call allocates or frees memory.  Every call on one GPU
 * uses that GPU's array, so calls that overlap on one GPU (two streams, two
 * host threads) race and must be serialised by the caller; the array keeps
 * the last call's contents, which no later call reads before writing.
 * Arguments, results and errors otherwise as cta_ttm; asynchronous. */
#define CTA_TTM_SCRATCH_BYTES (32u << 20)
cta_status cta_ttm_noalloc(int order, const int64_t* x_dims, const void* X, cta_dtype x_dtype,
                           uint32_t mode_mask, uint32_t trans_mask, const void* const* M,
                           const int64_t* m_rows, const int64_t* m_cols, cta_dtype m_dtype,
                           cta_dtype compute, void* Y, cta_dtype y_dtype, void* stream);

/* ------------------------------------------------------------------------
 * Operator handle: the per-mode factors of one tensor equation.
 *
 * order N in [2, CTA_MAX_ORDER]; n[k] unknown extents; m[k] sample extents;
 * host_A[k]: A_k, row-major m[k] x n[k], FP64 host memory.  host_D may be
 * NULL (no regulariser); otherwise host_D[k] is D_k, row-major p[k] x n[k]
 * (p[k] may be 0 for "no regulariser on mode k").  lambda >= 0 is expected
 * (a negative value is accepted; CG then reports CTA_ERR_BREAKDOWN if the
 * operator is not positive definite).  The handle computes G_k and R_k in
 * FP64 on the host (App. A.7), stores them on the device in FP64, FP32 and
 * BF16, and allocates its solver workspace (about 12 tensors of n's size).
 * Synchronous with respect to `stream`.
 * ---------------------------------------------------------------------- */
typedef struct cta_op_s* cta_op;

cta_status cta_op_create(cta_op* out, int order, const int64_t* n, const int64_t* m,
                         const double* const* host_A, const double* const* host_D,
                         const int64_t* p, double lambda, void* stream);
cta_status cta_op_destroy(cta_op op);
/* Device bytes owned by the handle. */
size_t cta_op_device_bytes(cta_op op);

/* Y = X x_1 A_1 ... x_N A_N (forward model; X has extents n, Y extents m).
 * Asynchronous.  Uses the handle's workspace (not reentrant per handle). */
cta_status cta_forward(cta_op op, const void* X, cta_dtype x_dtype, void* Y,
                       cta_dtype y_dtype, cta_precision chain, void* stream);

/* B = Y x_1 A_1^T ... x_N A_N^T (App. A.7).  Y has extents m, B extents n.
 * The chain runs in `chain` precision (CTA_PREC_F64 or CTA_PREC_F32).
 * Asynchronous. */
cta_status cta_rhs(cta_op op, const void* Y, cta_dtype y_dtype, void* B, cta_dtype b_dtype,
                   cta_precision chain, void* stream);

/* Q = N(P) with P, Q of extents n and dtype `dtype` (F64 for CTA_PREC_F64,
 * F32 for CTA_PREC_F32 and CTA_PREC_BF16).  If `dot` is not NULL the FP64
 * inner product <P, Q> (App. A.6) is written to the device double *dot.
 * Asynchronous.  P and Q must not overlap. */
cta_status cta_apply_normal_op(cta_op op, const void* P, void* Q, cta_dtype dtype,
                               cta_precision chain, double* dot, void* stream);

/* Autotuner of one operator: times every tile-shape variant combination of
 * the chain passes of N in `chain` precision (median of `reps` applies on the
 * handle's own workspace, which it overwrites), rejects any variant whose
 * output is not bit-identical to the default shapes', and keeps the fastest
 * in the handle for later applies and solves.  Synchronous. */
cta_status cta_tune_op(cta_op op, cta_precision chain, int reps, void* stream);
/* The variants chosen for `chain` (tail, middle, last pass) into host_variants3;
 * cta_op_set_tuning sets them: tail 0 or 1 (blocks per workgroup) or 2
 * (persistent workgroups with both factors in LDS that load the next group's
 * vectors while computing the current one; BF16 chains inside CG with the
 * last two extents <= 128 and <= 32, else as 0), middle 0 or 1 (tile
 * shape) or 2 (persistent workgroups with the factor in LDS that load the next
 * 64-column tile while computing the current one, BF16 chains with
 * n_k <= 128 and the trailing extent a multiple of 64, else as 1), last
 * 0..8 (0, 1: tile shape; 2, 3: the narrow shape with its tiles walked
 * along the second mode first, in groups of 8 planes or all planes; 4: row
 * blocks of 32 with the whole stencil staged on chip, F32/BF16 chains of
 * order 3 or 4, else as 2; 5: persistent workgroups that load the next
 * tile while computing the current one, BF16 chains with 96 < n_1 <= 128,
 * else as 2; 6: as 5 with zero rows around the LDS window, vector reads
 * of the band coefficients and each XCD's workgroups sweeping one range of
 * tiles; 7: as 6 with workgroups of 512 threads, two per CU; 8: one
 * 1024-thread workgroup per CU sweeping a run of tiles along one plane of
 * the second mode with P in an on-chip ring, order 4 with n_N <= 24, else
 * as 6). */
cta_status cta_op_get_tuning(cta_op op, cta_precision chain, int* host_variants3);
cta_status cta_op_set_tuning(cta_op op, cta_precision chain, const int* host_variants3);

/* Band-aware applies.  Cubic B-spline collocation factors give Gram matrices
 * G_k with half-bandwidth 3 (Sec. 6: each sample touches 4 basis functions
 * per mode), so a mode product with G_k is a short stencil along mode k.
 * cta_op_create records the largest half-bandwidth w of the G_k
 * (cta_op_band_width); when w <= 4 it keeps the bands in FP64 and FP32 and
 * turns the banded applies on.  Then every F64 or F32 application of N that
 * is not part of an inner CG iteration (cta_apply_normal_op with those
 * chains, the residual updates of the mixed-precision solves, the final
 * FP64 residual check) runs as N streaming passes: modes N .. 2 as banded
 * mode products, mode 1 with the regulariser and <P, Q> fused, every sum over
 * the 2w + 1 taps in ascending offset.  The result equals the dense chain's
 * up to rounding.  cta_op_set_banded(op, 0) restores the dense passes;
 * enabling fails with CTA_ERR_ARG when w > 4.  Returns of cta_op_band_width:
 * w, or -1 for a NULL handle. */
cta_status cta_op_set_banded(cta_op op, int enable);
int cta_op_band_width(cta_op op);

/* Tensor-inverse preconditioner (Sec. 3: a separable operator is inverted
 * mode by mode).  The separable part of N with each G_k replaced by
 * G_k + c R_k is inverted per mode:
 *     M^-1(R) = R x_1 (G_1 + c R_1)^-1 ... x_N (G_N + c R_N)^-1,
 * exact for lambda = 0 and c = 0.  The inverses are formed on the host in
 * FP64 (Cholesky; CTA_ERR_ARG if some G_k + c R_k is not positive definite)
 * and kept on the device in F64, F32 and BF16; a later call replaces them,
 * c < 0 removes the preconditioner.  Synchronous. */
cta_status cta_op_set_preconditioner(cta_op op, double c);
/* Z = M^-1(R) in `chain` precision (F64 tensors for CTA_PREC_F64, F32
 * otherwise); optional FP64 <R, Z> written to the device double *dot.
 * Asynchronous. */
cta_status cta_apply_precond(cta_op op, const void* R, void* Z, cta_dtype dtype, cta_precision chain,
                             double* dot, void* stream);


/* ------------------------------------------------------------------------
 * Conjugate-gradient solve (Fig. Tensor_CG) of N(X) = B.
 *
 * Stopping test: ||r||_2 <= rtol * ||B||_2 on the recursive residual (the
 * printed "until rho > threshold" is read as rho <= threshold, as in the
 * Jacobi solver of Fig. Tensor_Jacobi); on exit the true residual is
 * recomputed in FP64.
 * Precision / dtype of B and X:
 *   CTA_PREC_F64          B, X F64
 *   CTA_PREC_F32          B, X F32
 *   CTA_PREC_BF16         B, X F32  (inner arithmetic only; rarely reaches 1e-8)
 *   CTA_PREC_BF16_REFINE  B, X F64  (outer FP64 refinement to rtol, inner CG
 *                                    in CTA_PREC_BF16 to inner_rtol)
 *   CTA_PREC_BF16_RELIABLE B, X F64 (BF16-chain CG with FP64 reliable updates
 *                                    every inner_rtol reduction; max_refine
 *                                    bounds the updates, max_iter the
 *                                    iterations between two updates)
 * X is read as the starting tensor when x0_given != 0, else overwritten.
 * With fallback_zero != 0 a starting tensor whose residual is not smaller than
 * ||B|| is replaced by zero.  The call synchronises `stream` and fills
 * *host_info.  Returns CTA_OK, CTA_NOT_CONVERGED (max_iter or max_refine hit;
 * the last X is written) or an error.
 * ---------------------------------------------------------------------- */
typedef struct {
    cta_precision precision;
    double rtol;        /* relative residual target, e.g. 1e-8 */
    int max_iter;       /* CG iterations (for refinement: per inner solve) */
    int x0_given;       /* 1: X holds the starting tensor */
    int fallback_zero;  /* 1: use zero if the start is worse than zero */
    double inner_rtol;  /* refinement: inner relative tolerance (e.g. 1e-2) */
    int max_refine;     /* refinement: outer steps */
    int check_every;    /* host reads the convergence flag every this many iterations
                           (reliable updates: the first read of a group after as many
                           iterations as the previous group took, then every
                           max(1, check_every / 4)) */
    int precond;        /* preconditioned CG (not for cta_solve_batched): the
                           iteration uses z = M^-1 r for the search direction and
                           <r, z> for the step lengths, the stopping test stays
                           ||r|| <= rtol ||B||.  0: none; 1: the tensor-inverse
                           preconditioner (cta_op_set_preconditioner); 2: the
                           diagonal of N (tensor Jacobi, Fig. Tensor_Jacobi);
                           3: one tensor multigrid V-cycle (Fig. TMG,
                           cta_op_set_multigrid) */
} cta_cg_opts;

typedef struct {
    int status;               /* cta_status of this solve */
    int iters;                /* total CG iterations (all inner solves) */
    int refine_steps;         /* outer refinement steps or reliable updates (0 without) */
    double rel_res_recursive; /* ||r_rec|| / ||B|| at exit */
    double rel_res_true;      /* ||B - N(X)|| / ||B|| recomputed in FP64 */
    double seconds;           /* wall time of the solve (host clock) */
} cta_cg_info;

/* Defaults: F32, rtol 1e-6, max_iter 10000, no start, inner_rtol 1e-2,
 * max_refine 30, check_every 16, no preconditioner. */
void cta_cg_opts_default(cta_cg_opts* opts);

cta_status cta_cg_solve(cta_op op, const void* B, void* X, cta_dtype dtype,
                        const cta_cg_opts* opts, cta_cg_info* host_info, void* stream);
/* Autotuner of the preconditioner strength: solves N(X) = B once per
 * candidate c (host_c[0..count)) with `opts` (precond forced to 1, X
 * overwritten) and keeps the preconditioner of the fastest solve that
 * converged; its c goes to *best_c (host).  CTA_NOT_CONVERGED if no candidate
 * converged (the preconditioner is then removed).  Synchronous. */
cta_status cta_tune_preconditioner(cta_op op, const void* B, void* X, cta_dtype dtype,
                                   const cta_cg_opts* opts, const double* host_c, int count,
                                   double* best_c, void* stream);

/* ------------------------------------------------------------------------
 * Tensor Jacobi (Fig. Tensor_Jacobi, Sec. 4.1).  The main diagonal of N at
 * multi-index i is d[i] = prod_k G_k[i_k, i_k] + lambda sum_k R_k[i_k, i_k]
 * (the diagonal of a Kronecker product is the product of the factors'
 * diagonals, and a Kronecker-sum term contributes R_k's diagonal); the
 * handle keeps the per-mode diagonals and forms d on the fly, never as a
 * tensor.  Flat tensor sizes must stay below 2^31.
 *
 * cta_apply_jacobi: Z = omega * R / d elementwise (R, Z device tensors of
 * extents n, both F64 or both F32); optional FP64 <R, Z> to the device
 * double *dot.  Asynchronous.
 *
 * cta_jacobi_solve: the stationary iteration of Fig. Tensor_Jacobi,
 * U <- U + omega (B - N U) / d, from U = 0 (or X when opts->x0_given) until
 * ||B - N U|| <= rtol ||B|| (tested before every sweep, as the figure's loop
 * does) or opts->max_iter sweeps.  The printed iteration is omega = 1; it
 * converges only when 2 diag(N) - N is positive definite, which Gram products
 * of B-spline collocation are not, so omega < 2 / lambda_max(diag(N)^-1 N)
 * is needed there (a diverging iteration ends with CTA_ERR_BREAKDOWN once the
 * residual is not finite, or CTA_NOT_CONVERGED).  opts: precision
 * CTA_PREC_F64 (B, X F64) or CTA_PREC_F32 (B, X F32), rtol, max_iter,
 * x0_given, check_every; info->iters counts sweeps, rel_res_recursive is the
 * last tested residual, rel_res_true the FP64 recomputation.  Synchronises
 * `stream`.
 * ---------------------------------------------------------------------- */
cta_status cta_apply_jacobi(cta_op op, const void* R, void* Z, cta_dtype dtype, double omega, double* dot,
                            void* stream);
cta_status cta_jacobi_solve(cta_op op, const void* B, void* X, cta_dtype dtype, const cta_cg_opts* opts,
                            double omega, cta_cg_info* host_info, void* stream);

/* ------------------------------------------------------------------------
 * Tensor multigrid (Fig. TMG, Sec. 4.2): a V-cycle over a hierarchy of
 * scales with separable restriction and prolongation (one matrix per mode),
 * damped-Jacobi smoothing and a direct solve on the last scale, used as a CG
 * preconditioner (cta_cg_opts.precond = 3) or applied alone.
 *
 * cta_op_set_multigrid builds the hierarchy (GetScale) on the host in FP64:
 *  - mode k of a scale is coarsened to ceil(n_k / 2) while n_k >= 8 (else
 *    kept); prolongation P_k (n_k x nc_k) is linear interpolation from nc_k
 *    uniform points over the same index interval, restriction is P_k^T;
 *  - the next scale's operator has the same form: G_k' = P_k^T G_k P_k (the
 *    exact Galerkin image of the data term) and R_k' = s_k^2 P_k^T R_k P_k
 *    with s_k^2 = prod_{l != k} n_l / nc_l (the regulariser's identity
 *    factors become P_l^T P_l, lumped to (n_l / nc_l) I);
 *  - scales are added while the current one has more than coarse_max
 *    unknowns and a mode can be coarsened, up to max_levels scales in all;
 *    the last one must have at most 4096 unknowns (CTA_ERR_ARG otherwise);
 *  - every scale but the last is smoothed by nu sweeps of damped Jacobi
 *    before and after the coarse-grid correction, with omega = omega_scale /
 *    b and b = max(prod_k lmax(g_k^-1/2 G_k g_k^-1/2), max_k lmax(r_k^-1/2
 *    R_k r_k^-1/2)) >= lambda_max(diag(N)^-1 N) (g_k, r_k the diagonals of
 *    G_k, R_k); omega_scale in (0, 2);
 *  - the last scale is solved with the inverse of its assembled matrix.
 * max_levels < 2 removes the hierarchy.  The handle owns the coarse scales'
 * operators, transfer matrices and vectors.  Synchronous.
 *
 * cta_op_multigrid_info: number of scales to *host_levels; for the first
 * `capacity` scales their extents (user order, row-major [scale][mode]) and
 * smoother weights omega (either array may be NULL).
 *
 * cta_apply_multigrid: Z = V(R), one V-cycle from zero on R, in `chain`
 * precision (F64 tensors for CTA_PREC_F64, F32 for CTA_PREC_F32 and
 * CTA_PREC_BF16); optional FP64 <R, Z> to the device double *dot.
 * Asynchronous; uses the handle's work vectors (not reentrant per handle).
 * ---------------------------------------------------------------------- */
cta_status cta_op_set_multigrid(cta_op op, int max_levels, int64_t coarse_max, int nu, double omega_scale);
cta_status cta_op_multigrid_info(cta_op op, int* host_levels, int64_t* host_extents, double* host_omega,
                                 int capacity);
cta_status cta_apply_multigrid(cta_op op, const void* R, void* Z, cta_dtype dtype, cta_precision chain,
                               double* dot, void* stream);

/* ------------------------------------------------------------------------
 * Batched solve: `count` independent problems of order 3 in one persistent
 * launch.  ops[i] is the handle of problem i (each with its own shapes and
 * lambda), B[i] and X[i] its device tensors (dtype F32, CTA_PREC_F32 only).
 * Work is ordered largest problem first; each problem is solved by a team of
 * workgroups that synchronise through device-memory barriers; the kernel's
 * tile shapes come from the autotuner cache (cta_tune_batched) when present.
 * Synchronises `stream` and fills host_infos[count].
 * ---------------------------------------------------------------------- */
cta_status cta_solve_batched(int count, const cta_op* ops, const void* const* B,
                             void* const* X, cta_dtype dtype, const cta_cg_opts* opts,
                             cta_cg_info* host_infos, void* stream);

/* Autotuner: times every candidate tile configuration of the batched solver
 * for each distinct problem shape among ops[0..count) on `stream`, validates
 * each candidate's operator output against the reference configuration,
 * and stores the fastest median per shape in the process-wide cache, which
 * cta_solve_batched reads.  When `cache_path` is not NULL the cache is also
 * written there as JSON (and read back by cta_tune_load). */
cta_status cta_tune_batched(int count, const cta_op* ops, int reps, const char* cache_path,
                            void* stream);
cta_status cta_tune_load(const char* cache_path);
/* Copy a JSON description of the current cache into host_buf (NUL
 * terminated, truncated to bytes); returns the full length via *needed. */
cta_status cta_tune_dump(char* host_buf, size_t bytes, size_t* needed);

/* ------------------------------------------------------------------------
 * Learned warm start: a separable network (per-mode 1-D convolutions, the
 * convolution row of Table 1) mapping B to a starting tensor X0.
 *
 * Architecture (order 4 tensors only), with s = RMS of B (||B|| / sqrt(size)):
 *   h0 = lw * (B / s) + lb                  pointwise lift 1 -> C channels
 *   `blocks` residual blocks: four convolutions of width `width` along modes
 *   1..4 (zero padding, C -> C channels, bias), ReLU after the first three,
 *   the fourth added to the block input
 *   X0 = s * (pw . h + pb)                  pointwise projection C -> 1
 * s depends on B only, so no gradient flows through it.  FP32 master
 * parameters and Adam state; BF16 copies of the convolution weights and of
 * the activations, FP32 accumulation on MFMA.  C must be 32 and width 5.
 *
 * Flat FP32 parameter layout (cta_ws_params): lw[C], lb[C]; for each block
 * and each mode k: W_k[(co*C + ci)*width + w] (C*C*width entries), then the
 * bias c_k[C]; then pw[C], pb.  Memory: (blocks*4 + 4) activation tensors of
 * 64 bytes per entry are allocated at creation.
 * ---------------------------------------------------------------------- */
typedef struct cta_ws_s* cta_ws;

cta_status cta_ws_create(cta_ws* out, int order, const int64_t* n, int channels, int width,
                         int blocks, uint64_t seed, void* stream);
cta_status cta_ws_destroy(cta_ws w);
/* Number of FP32 parameters. */
int64_t cta_ws_num_params(cta_ws w);
/* X0 = s * f(B / s) for one F32 tensor B (extents n, row-major), X0 F32.
 * The activations are always kept for cta_ws_backward (`training` is
 * accepted for interface stability).  Asynchronous. */
cta_status cta_ws_forward(cta_ws w, const void* B, void* X0, int training, void* stream);
/* Given dL/dX0 (F32, extents n) of the last training forward, accumulate the
 * parameter gradient.  Asynchronous. */
cta_status cta_ws_backward(cta_ws w, const void* dX0, void* stream);
/* Scale-free mean-squared error of the last forward output X0 against the
 * target T (F32): L = mean(((X0 - T) / s)^2).  Writes dL/dX0 to dX0 and L to
 * the DEVICE double *loss (may be NULL).  Asynchronous. */
cta_status cta_ws_mse(cta_ws w, const void* X0, const void* T, void* dX0, double* loss,
                      void* stream);
/* Zero the accumulated gradient.  Asynchronous. */
cta_status cta_ws_zero_grad(cta_ws w, void* stream);
/* One Adam step on the FP32 master weights with the accumulated gradient
 * (step counter kept in the handle), then refresh the BF16 copies.
 * Asynchronous. */
cta_status cta_ws_adam_step(cta_ws w, float lr, float beta1, float beta2, float eps,
                            void* stream);
/* Copy the FP32 master parameters (set == 0) or the accumulated FP32
 * gradient (set == 2) to host_buf, or load parameters from it (set == 1).
 * `bytes` must equal 4 * cta_ws_num_params.  Synchronous. */
cta_status cta_ws_params(cta_ws w, void* host_buf, size_t bytes, int set, void* stream);

/* ------------------------------------------------------------------------
 * Scattered-measurement operator (Sec. 6, the paper's application): the
 * coefficients X (order N in [2, 4], extents n_k >= 4, row-major) of a cubic
 * B-spline field (clamped uniform knots on [0, 1], n_k functions per mode)
 * are observed at `count` scattered sites t^i in [0, 1]^N.  Row i of the
 * system is the Khatri-Rao product a_i = b^i_1 (x) ... (x) b^i_N of the basis
 * rows of its coordinates (the repeated-index product of Sec. 2.2), so
 *   forward:  y_i = <a_i, X>,            adjoint:  B = sum_i y_i a_i,
 *   normal:   N(X) = sum_i a_i <a_i, X> + lam * sum_k X x_k (D_k^T D_k),
 * the CANDECOMP sum of Sec. 6 plus the Kronecker-sum regulariser.  Neither N
 * nor its CP factors are stored: the kernels evaluate the basis from the
 * sites.  Sites are sorted into bricks of knot-span cells at creation; each
 * brick's coefficient tile is worked on in LDS and written to a scratch slot
 * of its own, and a second pass sums the slots covering each coefficient in a
 * fixed order (no global atomics; the order of the LDS additions within a
 * tile is not fixed, so results may differ between calls by rounding).
 *
 * cta_sop_create: host_coords (host, float32, mode-major: coordinate k of
 * site i at [k * count + i]) must lie in [0, 1] (CTA_ERR_ARG otherwise);
 * host_D[k] (host, row-major d_rows[k] x n[k], FP64) is the regulariser
 * factor of mode k, or NULL / host_D NULL for none; D_k^T D_k must have
 * half-bandwidth <= 2 (second differences; CTA_ERR_UNSUPPORTED otherwise).
 * count may be 0 (then N is the regulariser alone).  Synchronous; the
 * handle owns its device memory (sites, permutation, bricks, bands and, on
 * first use per dtype, the tile scratch and CG vectors).
 * Device arrays: X, B, P, Q of n_1 * .. * n_N elements, y of `count`
 * elements in the caller's site order, all of dtype CTA_F64 or CTA_F32 (the
 * arithmetic precision).  dot (device, FP64, or NULL) receives <P, Q>.
 * Calls are enqueued on `stream`; one handle must not be used from two
 * streams at once (the scratch tiles are shared).
 * ---------------------------------------------------------------------- */
typedef struct cta_sop_s* cta_sop;

cta_status cta_sop_create(cta_sop* out, int order, const int64_t* n, int64_t count,
                          const float* host_coords, const double* const* host_D,
                          const int64_t* d_rows, double lam);
cta_status cta_sop_destroy(cta_sop op);
/* host_out8: brick cells per mode (4 entries, 0 past the order), tile
 * elements, chunks (workgroups of the brick pass), bricks, device bytes. */
cta_status cta_sop_layout(cta_sop op, int64_t* host_out8);
cta_status cta_sop_forward(cta_sop op, const void* X, void* y, cta_dtype dtype, void* stream);
cta_status cta_sop_adjoint(cta_sop op, const void* y, void* B, cta_dtype dtype, void* stream);
cta_status cta_sop_apply_normal(cta_sop op, const void* P, void* Q, cta_dtype dtype, double* dot,
                                void* stream);
/* Tensor CG (Fig. Tensor_CG) on the scattered normal operator in the dtype's
 * precision (F64 or F32 vectors, FP64 dots).  opts: rtol, max_iter,
 * x0_given (X holds the start), fallback_zero (a start whose residual is
 * not below ||B|| is replaced by zero), check_every (the host reads the flag
 * every this many iterations); precision is taken from dtype and precond
 * must be 0.  Stops when ||r|| <= rtol ||B|| (recursive residual); the true
 * residual is then recomputed in the dtype's precision, and when it misses
 * rtol the iteration restarts once from it.  Fills *host_info; returns
 * CTA_OK only when the true residual meets rtol, else CTA_NOT_CONVERGED
 * (the last X written) or an error.  Synchronises `stream`. */
cta_status cta_sop_cg_solve(cta_sop op, const void* B, void* X, cta_dtype dtype, const cta_cg_opts* opts,
                            cta_cg_info* host_info, void* stream);

/* ------------------------------------------------------------------------
 * Kernel timing tracer.  When enabled, every kernel the library launches is
 * bracketed by two HIP events recorded on the launch's stream (so the timing
 * is of the kernel as it ran inside the caller's work).  cta_prof_read
 * synchronises the recorded events and writes a JSON object
 * {"<kernel>": {"count", "total_ms", "min_ms", "max_ms", "active_count",
 * "active_ms"}, ...} into host_buf (NUL terminated, truncated to bytes; the
 * full length is returned in *needed).  The active figures cover the
 * launches that ran at least a tenth of the kernel's 90th-percentile
 * duration: the iterations a solver enqueues past convergence exit at once on
 * the device-side converged flag, and they are left out there.  cta_prof_reset drops the records (called
 * with the tracer off it also destroys the tracer's HIP events).  Process-wide; not meant for
 * concurrent use from several threads.
 * ---------------------------------------------------------------------- */
cta_status cta_prof_enable(int on);
cta_status cta_prof_reset(void);
cta_status cta_prof_read(char* host_buf, size_t bytes, size_t* needed);

#ifdef __cplusplus
}
#endif

#endif /* CTA_H */
