// Host-side launchers of the gfx950 kernels (internal interface of libcta).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cta {

enum DT { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2 };

inline int dt_size(int dt) { return dt == DT_F64 ? 8 : (dt == DT_F32 ? 4 : 2); }
// K granularity of the MFMA instruction used for a compute type
inline int dt_kstep(int dt) { return dt == DT_F64 ? 8 : (dt == DT_F32 ? 16 : 32); }

// A factor matrix on the device in one compute type, zero padded to
// rows_st = roundup(rows, 64), ld = roundup(cols, 32).
struct Mat {
    const void* p = nullptr;
    int ld = 0;
    int rows = 0, cols = 0;
};

// Device scalars of one CG solve (FP64).
struct CgScalars {
    double rho;        // <r, r> of the current residual
    double pq;         // <p, N p>
    double alpha, beta;
    double threshold;  // (rtol * ||B||)^2
    double bnorm2;     // ||B||^2
    double rho0;
    double dot;        // result slot of stand-alone dots
    int iters;
    int done;          // 0 running, 1 converged, 2 breakdown, 3 iteration limit
    int max_iter;
    int pad0;
    int nblk;          // number of partials written by the last reduction kernel
    int precond;       // 1: preconditioned CG (alpha, beta from <r, z>)
    double rz;         // <r, z>, z = M^-1 r (preconditioned CG)
    double dot2;       // second result slot of stand-alone dots
};

enum { DONE_RUNNING = 0, DONE_CONVERGED = 1, DONE_BREAKDOWN = 2, DONE_MAXITER = 3 };

// Multiply-high division by a constant (Granlund and Montgomery, "Division by
// invariant integers using multiplication", 1994): with l = ceil(log2 d) and
// mul = floor(2^32 (2^l - d) / d) + 1, floor(n / d) = (mulhi(mul, n) + n) >> l
// for every n < 2^31 (the sum cannot overflow 32 bits).
__host__ __device__ inline void fastdiv_init(uint32_t d, uint32_t* mul, int* shift) {
    int l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    *shift = l;
    *mul = (uint32_t)(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
}

// Banded regulariser of the normal operator (half-bandwidth <= 2).
struct StencilDesc {
    const void* P;
    const void* rband[8];
    int64_t ext[8];
    int64_t stride[8];
    int order;
    double lam;
};

// What the finalize kernel does with the reduced total.
enum {
    POST_NONE = 0,   // nothing
    POST_DOT = 1,    // *out = total
    POST_ALPHA = 2,  // pq = total; alpha = rho / pq (breakdown if pq <= 0)
    POST_RHO = 3,    // rho1 = total; beta = rho1 / rho; rho = rho1; iters++; convergence test
                     // (preconditioned: rho = total; iters++; convergence test only)
    POST_RZ = 4      // preconditioned: rz1 = total; beta = rz1 / rz; rz = rz1
};

// Maximum grid of the reducing kernels (and size of the partials array).
constexpr int kMaxGrid = 16384;

// Sum partials[0..n) in index order and apply `post` (one workgroup).
hipError_t launch_finalize(const double* partials, int n, CgScalars* scal, int post, double* out,
                           hipStream_t s);

// ---- TTM passes ----
// `variant` selects a tile shape (0 = default; see kernels_ttm.hip); the
// autotuner times the variants of every pass of an operator.
hipError_t launch_strided(int tc, const void* X, void* Y, const Mat& M, int64_t lead, int K, int J,
                          int64_t trail, const int* done, hipStream_t s, int variant = 0);
hipError_t launch_contig(int tc, const void* X, void* Y, const Mat& M, int64_t rows, int K, int J,
                         const int* done, hipStream_t s);
bool tail_fits(int tc, int K1, int J2);
// With Pvec: the chain input is p = X + beta p (X is r), written back to Pvec;
// with Xsol as well: Xsol += alpha p (p before its update) on the same pass.
hipError_t launch_tail(int tin, int tout, int tc, const void* X, void* Y, const Mat& M1,
                       const Mat& M2, int64_t nblk, int K1, int K2, int J1, int J2, void* Pvec,
                       const double* beta, const int* done, hipStream_t s, int variant = 0,
                       void* Xsol = nullptr, const double* alpha = nullptr);
// Last pass of the normal operator: Q = X x_1 M (mode 1 of a (K, trail)
// tensor) + banded regulariser of P, with the FP64 <P, Q> reduced on device.
hipError_t launch_normal_last(int tmid, int tvec, int tc, const void* X, void* Q, const Mat& M,
                              int K, int J, int64_t trail, const StencilDesc& st,
                              double* partials, CgScalars* scal, int post, double* dot_out,
                              const int* done, hipStream_t s, int variant = 0);

// Preconditioner tail pass (BF16 chain) with r = r - alpha q fused: R is read
// and written, the chain input is the new r, and <r, r> is finalized with
// POST_RHO (convergence test of the preconditioned iteration).
hipError_t launch_tail_r(void* R, const void* Q, void* Y, const Mat& M1, const Mat& M2, int64_t nblk, int K1,
                         int K2, int J1, int J2, const double* alpha, const int* done, double* partials,
                         CgScalars* scal, hipStream_t s, int variant = 0);

// Last pass without regulariser (the preconditioner's), BF16 chain, pipelined:
// Z = X x_1 M (FP32) and <R, Z>; hipErrorNotSupported when the shape does not fit.
hipError_t launch_last_nr(const void* X, void* Z, const void* R, const Mat& M, int K, int64_t trail,
                          double* partials, CgScalars* scal, int post, double* dot_out, const int* done,
                          hipStream_t s);

// ---- band-aware normal operator (F64 or F32; half-bandwidth w <= 4) ----
// Y = X x_k G on the (lead, K, trail) view with gb[j * (2w+1) + d + w] = G[j][j+d].
hipError_t launch_band_mode(int dt, const void* X, void* Y, const void* gb, int w, int64_t lead, int K,
                            int64_t trail, hipStream_t s);
// Q = X x_1 G_1 (banded) + lam * regulariser(P) and <P, Q> partials (then `post`).
hipError_t launch_band_last(int dt, const void* X, void* Q, const void* gb, int w, int K, int64_t trail,
                            const StencilDesc& st, double* partials, CgScalars* scal, int post,
                            double* dot_out, hipStream_t s);

// Y = X x_k M for a matrix whose row j has its nonzeros in columns lo[j] ..
// lo[j] + w - 1 (coef[j * w + c] = M[j][lo[j] + c], w in {4, 6, 8}).
hipError_t launch_rect_band(int dt, const void* X, void* Y, const int* lo, const void* coef, int w,
                            int64_t lead, int K, int J, int64_t trail, hipStream_t s);

// ---- vector kernels (Tv = F32 or F64) ----
hipError_t launch_cast(int tin, int tout, const void* x, void* y, int64_t n, hipStream_t s);
hipError_t launch_fill_zero(void* x, int64_t bytes, hipStream_t s);
// y = a*x + b*y in type tv
hipError_t launch_axpby(int tv, double a, const void* x, double b, void* y, int64_t n,
                        hipStream_t s);
// r = B - Q (tb: dtype of B and Q; tr: dtype of r); returns <r, r> into scal->rho via reduction
hipError_t launch_residual(int tb, int tr, const void* B, const void* Q, void* r, int64_t n,
                           double* partials, CgScalars* scal, double* out, hipStream_t s);
// r = B - Q for FP64 B and FP32 Q, r in FP32; <r, r> into *out
hipError_t launch_residual_mixed(const double* B, const float* Q, float* r, int64_t n, double* partials,
                                 CgScalars* scal, double* out, hipStream_t s);
// out = <x, y> (FP64, deterministic two-stage reduction)
hipError_t launch_dot(int tv, const void* x, const void* y, int64_t n, double* partials,
                      CgScalars* scal, double* out, hipStream_t s);
// x += alpha p (skipped when x is NULL: the tail pass applies it); r -= alpha q;
// rho1 = <r, r>; beta, convergence test (CG step)
hipError_t launch_cg_update(int tv, void* x, void* r, const void* p, const void* q, int64_t n,
                            double* partials, CgScalars* scal, hipStream_t s);
// x += alpha p with the device alpha, whatever the done flag: applies the step
// that the fused tail pass has not applied yet when an iteration loop ends
hipError_t launch_x_flush(int tv, void* x, const void* p, int64_t n, const CgScalars* scal,
                          hipStream_t s);
// CG setup from device dots: threshold, rho, beta = 0, done flag; precond = 1
// for the preconditioned iteration (scal->rz already holds <r, M^-1 r>)
hipError_t launch_cg_setup(CgScalars* scal, double rtol2, int max_iter, hipStream_t s,
                           int precond = 0);
// start of an iteration group after a reliable update (true <r, r> in scal->dot,
// and for the preconditioned iteration the true <r, z> in scal->dot2)
hipError_t launch_cg_group(CgScalars* scal, double threshold, int max_iter, int keep_dir,
                           hipStream_t s, int precond = 0);
// padded copy of a (possibly transposed) device matrix in another dtype
hipError_t launch_pad_matrix(int tin, int tout, const void* src, int rows, int cols, int trans,
                             void* dst, int rows_st, int ld, hipStream_t s);
// deterministic test pattern in [-0.5, 0.5) (hash of the index)
hipError_t launch_fill_pattern(int tv, void* x, int64_t n, hipStream_t s);
// X64 += (double) d32
hipError_t launch_add_f64(double* X, const void* d, int td, int64_t n, hipStream_t s);

// ---------------------------------------------------------------- diagonal and multigrid
// Main diagonal of the normal operator from per-mode diagonals:
// d[i] = prod_k g[k][i_k] + lam * sum_k r[k][i_k] (r[k] may be NULL); fmul/fsh
// are the multiply-high division constants of ext[k] (fastdiv_init).  Flat
// indices must stay below 2^31.
struct DiagDesc {
    const double* g[8];
    const double* r[8];
    int ext[8];
    uint32_t fmul[8];
    int fsh[8];
    int order;
    double lam;
};
// z = omega r / d; with post != POST_NONE also <r, z> (finalized with `post`).
// Skipped entirely when *gate is set (gate may be NULL).
hipError_t launch_jacobi_apply(int tv, const void* r, void* z, int64_t n, const DiagDesc& d, double omega,
                               double* partials, CgScalars* scal, int post, double* out, const int* gate,
                               hipStream_t s);
// Preconditioned CG step with the diagonal: r -= alpha q, z = r / d; <r, r>
// finalized with POST_RHO (stopping test) and <r, z> with POST_RZ (beta).
hipError_t launch_jacobi_update(int tv, void* r, const void* q, void* z, int64_t n, const DiagDesc& d,
                                double* partials, double* partials2, CgScalars* scal, hipStream_t s);
// Cout = C + omega (B - Q) / d with Q = N(C) (Cout may be C); dotmode 1:
// ||B - Q||^2, 2: <B, C_new> (finalized with `post`), 0: no reduction.
// Gated like launch_jacobi_apply.
hipError_t launch_jacobi_correct(int tv, const void* C, void* Cout, const void* B, const void* Q, int64_t n,
                                 const DiagDesc& d, double omega, int dotmode, double* partials,
                                 CgScalars* scal, int post, double* out, const int* gate, hipStream_t s);
// t = b - t and c += t (gated)
hipError_t launch_mg_sub(int tv, void* t, const void* b, int64_t n, const int* gate, hipStream_t s);
hipError_t launch_mg_add(int tv, void* c, const void* t, int64_t n, const int* gate, hipStream_t s);
// y = M x for a row-major n x n matrix (gated)
hipError_t launch_dense_matvec(int tv, const void* M, const void* x, void* y, int n, const int* gate,
                               hipStream_t s);

// ---------------------------------------------------------------- scattered operator
// Brick geometry of the scattered-measurement operator (order N <= 4).  A
// cell is one knot span per mode (C_k = n_k - 3 spans); a brick holds bc_k
// cells per mode and touches a tile of te_k = bc_k + 3 coefficients per mode
// (row-major, strides ts, tile = prod te).  gs: row-major strides of the
// coefficient tensor; roff: first row of mode k in the regulariser band table.
struct SopGeom {
    int N;
    int n[4], C[4], bc[4], nb[4], te[4], ts[4], roff[4];
    int64_t gs[4];
    int tile;
    int64_t ncoef;
};
enum { SOP_FWD = 0, SOP_ADJ = 1, SOP_NRM = 2 };

// One workgroup per chunk: y = A X (FWD, y in the caller's site order), or the
// chunk's tile of A^T y (ADJ) or A^T A X (NRM) into tiles[chunk].
hipError_t launch_sop_brick(int dt, int mode, const SopGeom& g, const float* coords, int64_t S,
                            const int* perm, const int* cstart, const int* cbrick, int nchunks,
                            const void* X, const void* yin, void* yout, void* tiles,
                            const CgScalars* scal, hipStream_t s);
// Q = sum of covering tiles (+ lam * regulariser(P) and <P, Q> partials when P
// is given; the finalize kernel then applies `post`).
hipError_t launch_sop_gather(int dt, const SopGeom& g, const void* tiles, const int* bchunk0, const void* P,
                             const void* rb, double lam, void* Q, double* partials, CgScalars* scal, int post,
                             double* out, hipStream_t s);
// x += alpha p; p = r + beta p (scalars on the device; skipped once done)
hipError_t launch_sop_pstep(int dt, void* x, void* p, const void* r, int64_t n, const CgScalars* scal,
                            hipStream_t s);

}  // namespace cta
