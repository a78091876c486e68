// Internal definitions shared by the host-side translation units of libcta.
#pragma once

#include <stdint.h>

#include <vector>

#include "../../include/cta.h"
#include "launch.hpp"

struct cta_op_s;

// One scale of the tensor multigrid hierarchy (Fig. TMG).  Scale 0 is the
// handle itself; scale l > 0 is an operator of the same form built from the
// Galerkin images of the factors (owned).  P/Pt: prolongation from scale
// l + 1 (n_k x nc_k) and restriction (its transpose), F64 and F32 copies.
struct cta_mg_scale {
    cta_op_s* op = nullptr;
    bool owned = false;
    cta::Mat P[2][CTA_MAX_ORDER];
    cta::Mat Pt[2][CTA_MAX_ORDER];
    double omega = 0.0;     // Jacobi damping of the smoother
    void* C = nullptr;      // this scale's correction (scales > 0), 8 bytes per unknown
    void* B = nullptr;      // this scale's right-hand side (scales > 0)
    void* T = nullptr;      // N(C), then the residual, then the prolonged correction
};

// Operator handle: per-mode factors on the device and the solver workspace.
struct cta_op_s {
    int order = 0;       // internal order (order 2 is lifted to 3)
    int user_order = 0;
    int lift = 0;        // leading unit modes added
    int64_t n[CTA_MAX_ORDER] = {0};
    int64_t m[CTA_MAX_ORDER] = {0};
    double lam = 0.0;
    int64_t N = 0;       // unknowns
    int64_t Msamp = 0;   // samples
    int64_t big = 0;     // prod_k max(n_k, m_k): bound of chain intermediates
    cta::Mat G[3][CTA_MAX_ORDER];   // G_k = A_k^T A_k per compute dtype
    cta::Mat A[2][CTA_MAX_ORDER];   // A_k   (F64, F32)
    cta::Mat At[2][CTA_MAX_ORDER];  // A_k^T (F64, F32)
    void* rband[2][CTA_MAX_ORDER] = {{nullptr}};  // R_k bands (F64, F32)
    void* T1 = nullptr;  // chain intermediates (N x 8 bytes each)
    void* T2 = nullptr;
    void* vx = nullptr;  // CG vectors (N x 8 bytes each)
    void* vr = nullptr;
    void* vp = nullptr;
    void* vq = nullptr;
    void* vaux = nullptr;
    void* rw0 = nullptr;  // forward / rhs work buffers (big x 8 bytes each, lazy)
    void* rw1 = nullptr;
    cta::CgScalars* scal = nullptr;
    cta::CgScalars* hscal = nullptr;  // pinned host mirror
    double* partials = nullptr;
    std::vector<void*> allocs;
    size_t dev_bytes = 0;
    // tile-shape variants of the normal-operator passes, per compute dtype
    // (F64, F32, BF16); set by cta_tune_op, 0 = default shapes
    int var_tail[3] = {0, 0, 0};
    int var_mid[3] = {0, 0, 0};
    int var_last[3] = {0, 0, 0};
    // host FP64 copies of G_k and R_k (R_k empty: no regulariser on mode k)
    std::vector<double> hG[CTA_MAX_ORDER], hR[CTA_MAX_ORDER];
    // tensor-inverse preconditioner: (G_k + c R_k)^-1 per compute dtype
    cta::Mat Pinv[3][CTA_MAX_ORDER];
    bool has_pc = false;
    double pc_c = 0.0;
    // banded Grams: half-bandwidth band_w <= 4 of every G_k, bands per dtype
    // (F64, F32); use_band routes the F64/F32 applies without fused CG
    // updates through the banded passes
    bool band_ok = false;
    bool use_band = false;
    int band_w = -1;
    void* gband[2][CTA_MAX_ORDER] = {{nullptr}};
    // banded rows of A_k (direction 0, forward model) and A_k^T (direction 1,
    // right-hand side): first column and w coefficients per row, per dtype
    bool cb_ok[2] = {false, false};
    int cb_w[2] = {0, 0};
    int* cb_lo[2][CTA_MAX_ORDER] = {{nullptr}};
    void* cb_coef[2][2][CTA_MAX_ORDER] = {{{nullptr}}};
    // false for the coarse scales of the multigrid hierarchy, which are built
    // from G_k and R_k alone (no forward model or right-hand side)
    bool has_A = true;
    // per-mode diagonals of G_k and R_k (FP64; drm[k] NULL without regulariser)
    double* dgm[CTA_MAX_ORDER] = {nullptr};
    double* drm[CTA_MAX_ORDER] = {nullptr};
    double* partials2 = nullptr;  // second partials array (two dots in one pass)
    // tensor multigrid preconditioner (cta_op_set_multigrid); empty: none
    std::vector<cta_mg_scale> mg;
    std::vector<void*> mg_allocs;
    int mg_nu = 1;
    int mg_ncoarse = 0;               // unknowns of the coarsest scale
    void* mg_inv[2] = {nullptr, nullptr};  // its inverse matrix (F64, F32), row-major
    // device copy of the batched solver's schedule when this handle is the
    // first problem of a batch (reused by later calls, freed with the handle)
    void* batch_buf = nullptr;
    size_t batch_bytes = 0;
};

namespace cta {
cta_status fail(cta_status st, const char* fmt, ...);
// Banded factors of a rectangular chain: per mode, the first column of each
// row and w coefficients per row (device pointers).
struct ChainBand {
    int w = 0;
    const int* lo[CTA_MAX_ORDER] = {nullptr};
    const void* coef[CTA_MAX_ORDER] = {nullptr};
};
std::vector<int> plan_order(int N, const int64_t* in_ext, const int64_t* out_ext,
                            const std::vector<int>& modes, int64_t* max_elems);
// Y = X x_k M_k over `order` (mode products on modes in that order); with
// `band`, each pass uses the banded rows instead of the dense M_k.
cta_status run_chain(int N, const int64_t* in_ext, const int64_t* out_ext, const Mat* mats,
                     const std::vector<int>& order, const void* X, int tin, void* Y, int tout,
                     int tc, void* w0, void* w1, hipStream_t s, const ChainBand* band = nullptr,
                     const int* gate = nullptr);
// Q = N(P).  fuse_update: the chain input is p = r + beta p (op->vr, op->vp),
// and with xsol the previous CG step's xsol += alpha p is applied on the
// same pass.
// gate: a done flag every pass checks (exits when set); without it the passes
// are gated only when fuse_update is set (on op's own flag).  A gated apply
// always takes the dense passes.
cta_status apply_normal(cta_op_s* op, const void* P, void* Q, int prec, int post, double* dot_out,
                        bool fuse_update, hipStream_t s, void* xsol = nullptr,
                        const void* fuse_src = nullptr, const int* gate = nullptr);
// Z = M^-1(R) (the tensor-inverse preconditioner) with <R, Z> reduced on the
// device and handled by `post`; gated: every kernel exits when the solve's
// done flag is set.
// fuse_r (BF16 chain, inside the preconditioned iteration): R is the residual
// r, updated as r -= alpha q (q = op->vq) by the first pass, which also forms
// <r, r> and the stopping test (POST_RHO) before the rest of the chain.
cta_status apply_precond(cta_op_s* op, const void* R, void* Z, int prec, int post, double* dot_out,
                         bool gated, hipStream_t s, bool fuse_r = false);
// Build the device side of a handle from its FP64 factors (cta_abi.cpp).
cta_status op_build(cta_op_s* op, std::vector<std::vector<double>>& G, std::vector<std::vector<double>>& R,
                    const std::vector<bool>& has_reg, const std::vector<std::vector<double>>* A);
cta_status dev_alloc(void** p, size_t bytes, std::vector<void*>& allocs, size_t& acc);
cta_status upload_mat(const double* host, int rows, int cols, bool trans, int dt, Mat* out,
                      std::vector<void*>& allocs, size_t& acc);
// Inverse of a symmetric positive definite n x n matrix (row-major) by
// Cholesky factorisation; false when a pivot is not positive.
bool spd_inverse(const std::vector<double>& A, int n, std::vector<double>& inv);
// Preconditioner kinds of cta_cg_opts.precond.
enum { PC_NONE = 0, PC_TENSOR_INV = 1, PC_JACOBI = 2, PC_MULTIGRID = 3 };
// Diagonal descriptor of a handle's operator (diagonal of N from per-mode parts).
DiagDesc diag_desc(const cta_op_s* op);
// z = M^-1 r for the preconditioner `kind` with <r, z> handled by `post`
// (gated: kernels exit when the solve's done flag is set).
cta_status precond_apply(cta_op_s* op, int kind, const void* R, void* Z, int prec, int post, double* dot_out,
                         bool gated, hipStream_t s);
// The preconditioned CG step after q = N(p) and alpha: r -= alpha q with the
// stopping test, then z = M^-1 r and beta = <r, z>_new / <r, z>_old.
cta_status precond_step(cta_op_s* op, int kind, int prec, hipStream_t s);
// One V-cycle z = V(r) of the multigrid preconditioner (Fig. TMG).
cta_status mg_vcycle(cta_op_s* op, const void* R, void* Z, int prec, int post, double* dot_out, bool gated,
                     hipStream_t s);
void mg_release(cta_op_s* op);
}  // namespace cta
