// Host side of the tensor Jacobi iteration (Fig. Tensor_Jacobi) and of the
// tensor multigrid V-cycle (Fig. TMG, Sec. 4.2) as a stationary solver and as
// preconditioners of the tensor CG.
//
// The multigrid hierarchy is built on the host in FP64 (GetScale):
//  * per mode, prolongation P_k (n_k x nc_k) is linear interpolation from a
//    uniform coarse grid over the same index interval (fine index i at coarse
//    coordinate i (nc_k - 1) / (n_k - 1)); a mode is coarsened to
//    ceil(n_k / 2) while n_k >= 8, else kept; restriction is P_k^T;
//  * the next scale's operator has G_k' = P_k^T G_k P_k (the exact Galerkin
//    image of the data term, which is a Kronecker product) and
//    R_k' = s_k^2 P_k^T R_k P_k with s_k^2 = prod_{l != k} n_l / nc_l: the
//    identity factors of the Kronecker-sum regulariser become P_l^T P_l, whose
//    rows sum to n_l / nc_l on average (P_l 1 = 1), and are lumped to that
//    multiple of I, so every scale is an operator of the same form and runs
//    the same passes;
//  * the smoother is damped Jacobi with omega = omega_scale / b, b the bound
//    max(prod_k lmax(g_k^-1/2 G_k g_k^-1/2), max_k lmax(r_k^-1/2 R_k r_k^-1/2))
//    of the largest eigenvalue of diag(N)^-1 N (g_k, r_k the diagonals);
//  * the coarsest scale is solved with its assembled matrix's inverse
//    (Cholesky), applied as a dense matrix-vector product.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/cta.h"
#include "abi_internal.hpp"
#include "launch.hpp"

using namespace cta;

#define PC_TRY(x)                      \
    do {                               \
        cta_status st_ = (x);          \
        if (st_ != CTA_OK) return st_; \
    } while (0)
#define PC_HIP(x)                                                                             \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) return fail(CTA_ERR_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

namespace {

int vec_type(int prec) { return prec == CTA_PREC_F64 ? DT_F64 : DT_F32; }
int mat_slot(int prec) { return prec == CTA_PREC_F64 ? 0 : 1; }

// Largest eigenvalue of diag(M)^-1/2 M diag(M)^-1/2 over the rows with a
// positive diagonal (M symmetric, row-major n x n), by cyclic Jacobi rotations
// until the off-diagonal mass is at rounding level.
double scaled_lambda_max(const std::vector<double>& M, int n) {
    std::vector<int> keep;
    for (int i = 0; i < n; ++i)
        if (M[(size_t)i * n + i] > 0.0) keep.push_back(i);
    const int m = (int)keep.size();
    if (m == 0) return 0.0;
    std::vector<double> S((size_t)m * m);
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            const int i = keep[a], j = keep[b];
            S[(size_t)a * m + b] = M[(size_t)i * n + j] / std::sqrt(M[(size_t)i * n + i] * M[(size_t)j * n + j]);
        }
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) {
                const double v = S[(size_t)a * m + b] * S[(size_t)a * m + b];
                tot += v;
                if (a != b) off += v;
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < m - 1; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = S[(size_t)p * m + q];
                if (apq == 0.0) continue;
                const double app = S[(size_t)p * m + p], aqq = S[(size_t)q * m + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < m; ++k) {  // rotate columns p, q
                    const double skp = S[(size_t)k * m + p], skq = S[(size_t)k * m + q];
                    S[(size_t)k * m + p] = c * skp - sn * skq;
                    S[(size_t)k * m + q] = sn * skp + c * skq;
                }
                for (int k = 0; k < m; ++k) {  // rotate rows p, q
                    const double spk = S[(size_t)p * m + k], sqk = S[(size_t)q * m + k];
                    S[(size_t)p * m + k] = c * spk - sn * sqk;
                    S[(size_t)q * m + k] = sn * spk + c * sqk;
                }
            }
    }
    double best = S[0];
    for (int a = 1; a < m; ++a) best = std::max(best, S[(size_t)a * m + a]);
    return best;
}

double smoother_bound(const cta_op_s* op) {
    double data = 1.0;
    for (int k = 0; k < op->order; ++k) data *= scaled_lambda_max(op->hG[k], (int)op->n[k]);
    double reg = 0.0;
    if (op->lam > 0)
        for (int k = 0; k < op->order; ++k)
            if (!op->hR[k].empty()) reg = std::max(reg, scaled_lambda_max(op->hR[k], (int)op->n[k]));
    return std::max(data, reg);
}

// Linear interpolation (n x nc, row-major) from nc uniform coarse points.
std::vector<double> interpolation(int n, int nc) {
    std::vector<double> P((size_t)n * nc, 0.0);
    if (nc == n) {
        for (int i = 0; i < n; ++i) P[(size_t)i * nc + i] = 1.0;
        return P;
    }
    for (int i = 0; i < n; ++i) {
        const double x = (double)i * (nc - 1) / (n - 1);
        const int J = std::min((int)std::floor(x), nc - 2);
        const double w = x - J;
        P[(size_t)i * nc + J] += 1.0 - w;
        P[(size_t)i * nc + J + 1] += w;
    }
    return P;
}

// P^T M P (M n x n, P n x nc)
std::vector<double> galerkin(const std::vector<double>& M, const std::vector<double>& P, int n, int nc) {
    std::vector<double> MP((size_t)n * nc, 0.0), out((size_t)nc * nc, 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            const double m = M[(size_t)i * n + k];
            if (m == 0.0) continue;
            for (int j = 0; j < nc; ++j) MP[(size_t)i * nc + j] += m * P[(size_t)k * nc + j];
        }
    for (int a = 0; a < n; ++a)
        for (int i = 0; i < nc; ++i) {
            const double p = P[(size_t)a * nc + i];
            if (p == 0.0) continue;
            for (int j = 0; j < nc; ++j) out[(size_t)i * nc + j] += p * MP[(size_t)a * nc + j];
        }
    return out;
}

// Dense matrix of N on a small scale (row-major multi-index order):
// N[i][j] = prod_k G_k[i_k][j_k] + lam sum_k R_k[i_k][j_k] prod_{l != k} [i_l == j_l].
std::vector<double> assemble(const cta_op_s* op) {
    const int N = op->order;
    const int64_t tot = op->N;
    std::vector<double> M((size_t)tot * tot, 0.0);
    std::vector<int> ii(N), jj(N);
    for (int64_t i = 0; i < tot; ++i) {
        int64_t r = i;
        for (int k = N - 1; k >= 0; --k) {
            ii[k] = (int)(r % op->n[k]);
            r /= op->n[k];
        }
        for (int64_t j = 0; j < tot; ++j) {
            int64_t c = j;
            int differ = 0, which = -1;
            for (int k = N - 1; k >= 0; --k) {
                jj[k] = (int)(c % op->n[k]);
                c /= op->n[k];
                if (jj[k] != ii[k]) {
                    ++differ;
                    which = k;
                }
            }
            double v = 1.0;
            for (int k = 0; k < N; ++k) v *= op->hG[k][(size_t)ii[k] * op->n[k] + jj[k]];
            if (op->lam != 0.0) {
                if (differ == 0) {
                    for (int k = 0; k < N; ++k)
                        if (!op->hR[k].empty()) v += op->lam * op->hR[k][(size_t)ii[k] * op->n[k] + ii[k]];
                } else if (differ == 1 && !op->hR[which].empty()) {
                    v += op->lam * op->hR[which][(size_t)ii[which] * op->n[which] + jj[which]];
                }
            }
            M[(size_t)i * tot + j] = v;
        }
    }
    return M;
}

cta_status check_vec_dtype(cta_dtype dtype, int prec) {
    const int want = vec_type(prec);
    if ((int)dtype != want)
        return fail(CTA_ERR_DTYPE, "tensors must be %s for this precision", want == DT_F64 ? "CTA_F64" : "CTA_F32");
    return CTA_OK;
}

// One V-cycle on scale l for N_l(C) = B (C overwritten).  On scale 0 with
// post != POST_NONE, <B, C> is reduced by the last smoothing sweep.
cta_status vcycle_at(cta_op_s* fine, int l, const void* B, void* C, int prec, int post, double* dot,
                     const int* gate, hipStream_t s) {
    cta_mg_scale& sc = fine->mg[l];
    cta_op_s* op = sc.op;
    const int tv = vec_type(prec);
    const int64_t n = op->N;
    if (l + 1 == (int)fine->mg.size()) {  // DirectSolve
        PC_HIP(launch_dense_matvec(tv, fine->mg_inv[mat_slot(prec)], B, C, (int)n, gate, s));
        return CTA_OK;
    }
    const DiagDesc d = diag_desc(op);
    const int N = op->order;
    cta_mg_scale& nx = fine->mg[l + 1];
    const int64_t* ext = op->n;
    const int64_t* cext = nx.op->n;
    std::vector<int> modes;  // coarsened modes (the others have P_k = I)
    for (int k = 0; k < N; ++k)
        if (cext[k] != ext[k]) modes.push_back(k);
    // Presmooth from a zero start: the first sweep is C = omega B / d
    PC_HIP(launch_jacobi_apply(tv, B, C, n, d, sc.omega, nullptr, nullptr, POST_NONE, nullptr, gate, s));
    for (int it = 1; it < fine->mg_nu; ++it) {
        PC_TRY(apply_normal(op, C, sc.T, prec, POST_NONE, nullptr, false, s, nullptr, nullptr, gate));
        PC_HIP(launch_jacobi_correct(tv, C, C, B, sc.T, n, d, sc.omega, 0, nullptr, nullptr, POST_NONE, nullptr,
                                     gate, s));
    }
    // separable restriction of the residual B - N(C)
    PC_TRY(apply_normal(op, C, sc.T, prec, POST_NONE, nullptr, false, s, nullptr, nullptr, gate));
    PC_HIP(launch_mg_sub(tv, sc.T, B, n, gate, s));
    std::vector<int> rorder = plan_order(N, ext, cext, modes, nullptr);
    PC_TRY(run_chain(N, ext, cext, sc.Pt[mat_slot(prec)], rorder, sc.T, tv, nx.B, tv, tv, op->T1, op->T2, s,
                     nullptr, gate));
    // V-cycle on the next scale from zero
    PC_TRY(vcycle_at(fine, l + 1, nx.B, nx.C, prec, POST_NONE, nullptr, gate, s));
    // coarse-grid correction: C += P C_next
    std::vector<int> porder = plan_order(N, cext, ext, modes, nullptr);
    PC_TRY(run_chain(N, cext, ext, sc.P[mat_slot(prec)], porder, nx.C, tv, sc.T, tv, tv, op->T1, op->T2, s,
                     nullptr, gate));
    PC_HIP(launch_mg_add(tv, C, sc.T, n, gate, s));
    // Postsmooth
    for (int it = 0; it < fine->mg_nu; ++it) {
        PC_TRY(apply_normal(op, C, sc.T, prec, POST_NONE, nullptr, false, s, nullptr, nullptr, gate));
        const bool reduce = l == 0 && post != POST_NONE && it + 1 == fine->mg_nu;
        PC_HIP(launch_jacobi_correct(tv, C, C, B, sc.T, n, d, sc.omega, reduce ? 2 : 0, fine->partials, fine->scal,
                                     reduce ? post : POST_NONE, dot, gate, s));
    }
    return CTA_OK;
}

}  // namespace

namespace cta {

DiagDesc diag_desc(const cta_op_s* op) {
    DiagDesc d{};
    d.order = op->order;
    d.lam = op->lam;
    for (int k = 0; k < op->order; ++k) {
        d.g[k] = op->dgm[k];
        d.r[k] = op->drm[k];
        d.ext[k] = (int)op->n[k];
        fastdiv_init((uint32_t)op->n[k], &d.fmul[k], &d.fsh[k]);
    }
    return d;
}

cta_status mg_vcycle(cta_op_s* op, const void* R, void* Z, int prec, int post, double* dot_out, bool gated,
                     hipStream_t s) {
    if (op->mg.size() < 2) return fail(CTA_ERR_ARG, "no multigrid hierarchy: call cta_op_set_multigrid first");
    return vcycle_at(op, 0, R, Z, prec, post, dot_out, gated ? &op->scal->done : nullptr, s);
}

cta_status precond_apply(cta_op_s* op, int kind, const void* R, void* Z, int prec, int post, double* dot_out,
                         bool gated, hipStream_t s) {
    switch (kind) {
    case PC_TENSOR_INV:
        return apply_precond(op, R, Z, prec, post, dot_out, gated, s);
    case PC_JACOBI: {
        const DiagDesc d = diag_desc(op);
        PC_HIP(launch_jacobi_apply(vec_type(prec), R, Z, op->N, d, 1.0, op->partials, op->scal, post, dot_out,
                                   gated ? &op->scal->done : nullptr, s));
        return CTA_OK;
    }
    case PC_MULTIGRID:
        return mg_vcycle(op, R, Z, prec, post, dot_out, gated, s);
    default:
        return fail(CTA_ERR_ARG, "unknown preconditioner %d", kind);
    }
}

cta_status precond_step(cta_op_s* op, int kind, int prec, hipStream_t s) {
    const int tv = vec_type(prec);
    if (kind == PC_TENSOR_INV && prec == CTA_PREC_BF16)  // r -= alpha q fused into the first pass
        return apply_precond(op, op->vr, op->vaux, prec, POST_RZ, nullptr, true, s, true);
    if (kind == PC_JACOBI) {
        const DiagDesc d = diag_desc(op);
        PC_HIP(launch_jacobi_update(tv, op->vr, op->vq, op->vaux, op->N, d, op->partials, op->partials2, op->scal,
                                    s));
        return CTA_OK;
    }
    PC_HIP(launch_cg_update(tv, nullptr, op->vr, op->vp, op->vq, op->N, op->partials, op->scal, s));
    return precond_apply(op, kind, op->vr, op->vaux, prec, POST_RZ, nullptr, true, s);
}

void mg_release(cta_op_s* op) {
    if (op->mg.empty() && op->mg_allocs.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto& sc : op->mg)
        if (sc.owned) cta_op_destroy(sc.op);
    op->mg.clear();
    for (void* p : op->mg_allocs) (void)hipFree(p);
    op->mg_allocs.clear();
    op->mg_inv[0] = op->mg_inv[1] = nullptr;
    op->mg_ncoarse = 0;
}

}  // namespace cta

// ---------------------------------------------------------------------------
extern "C" cta_status cta_apply_jacobi(cta_op op, const void* R, void* Z, cta_dtype dtype, double omega,
                                       double* dot, void* stream) {
    if (!op || !R || !Z) return fail(CTA_ERR_ARG, "NULL argument");
    if (dtype != CTA_F64 && dtype != CTA_F32) return fail(CTA_ERR_DTYPE, "R and Z must be CTA_F64 or CTA_F32");
    if (!std::isfinite(omega)) return fail(CTA_ERR_ARG, "omega must be finite");
    const DiagDesc d = diag_desc(op);
    PC_HIP(launch_jacobi_apply(dtype == CTA_F64 ? DT_F64 : DT_F32, R, Z, op->N, d, omega, op->partials, op->scal,
                               dot ? POST_DOT : POST_NONE, dot, nullptr, (hipStream_t)stream));
    return CTA_OK;
}

extern "C" cta_status cta_jacobi_solve(cta_op op, const void* B, void* X, cta_dtype dtype, const cta_cg_opts* opts,
                                       double omega, cta_cg_info* info, void* stream) {
    if (!op || !B || !X || !opts || !info) return fail(CTA_ERR_ARG, "NULL argument");
    std::memset(info, 0, sizeof *info);
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    const int prec = opts->precision;
    if (prec != CTA_PREC_F64 && prec != CTA_PREC_F32)
        return fail(CTA_ERR_ARG, "the Jacobi solver runs in CTA_PREC_F64 or CTA_PREC_F32");
    PC_TRY(check_vec_dtype(dtype, prec));
    if (!(opts->rtol >= 0) || opts->max_iter < 0) return fail(CTA_ERR_ARG, "bad rtol or max_iter");
    if (!(omega > 0) || !std::isfinite(omega)) return fail(CTA_ERR_ARG, "omega must be positive and finite");
    if (B == X) return fail(CTA_ERR_ARG, "B and X must not overlap");
    if (!tail_fits(prec == CTA_PREC_F64 ? DT_F64 : DT_F32, (int)op->n[op->order - 2], (int)op->n[op->order - 1]))
        return fail(CTA_ERR_UNSUPPORTED, "last two extents too large for the fused tail in this precision");
    const int tv = vec_type(prec);
    const int64_t n = op->N;
    const size_t vb = (size_t)n * dt_size(tv);
    const int check = opts->check_every > 0 ? opts->check_every : 16;
    const DiagDesc d = diag_desc(op);
    if (!opts->x0_given) PC_HIP(launch_fill_zero(X, vb, s));
    // device scalars: the residual test runs in the finalize of each sweep
    // (POST_RHO of the preconditioned form: rho = ||B - N U||^2, iters++, test)
    PC_HIP(launch_dot(tv, B, B, n, op->partials, op->scal, &op->scal->bnorm2, s));
    PC_HIP(launch_dot(tv, B, B, n, op->partials, op->scal, &op->scal->rho, s));
    PC_HIP(launch_cg_setup(op->scal, opts->rtol * opts->rtol, opts->max_iter + 1, s, 1));
    // sweep k reads U_k from buf[k % 2] and writes U_{k+1} to buf[(k+1) % 2];
    // its finalize tests ||B - N U_k||, so on exit the answer is U_{iters-1}
    void* buf[2] = {X, op->vx};
    const int* gate = &op->scal->done;
    int64_t launched = 0;
    for (;;) {
        for (int c = 0; c < check; ++c, ++launched) {
            void* cur = buf[launched & 1];
            void* nxt = buf[(launched + 1) & 1];
            PC_TRY(apply_normal(op, cur, op->vq, prec, POST_NONE, nullptr, false, s, nullptr, nullptr, gate));
            PC_HIP(launch_jacobi_correct(tv, cur, nxt, B, op->vq, n, d, omega, 1, op->partials, op->scal, POST_RHO,
                                         nullptr, gate, s));
        }
        if (hipMemcpyAsync(op->hscal, op->scal, sizeof(CgScalars), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(CTA_ERR_HIP, "scalar readback failed");
        if (op->hscal->done != DONE_RUNNING) break;
    }
    const int done = op->hscal->done;
    const int tests = op->hscal->iters;  // finalizes run: U_0 .. U_{tests-1} were tested
    const int sweeps = std::max(0, tests - 1);
    if (tests > 0 && ((tests - 1) & 1)) PC_HIP(launch_cast(tv, tv, op->vx, X, n, s));
    const double bn2 = op->hscal->bnorm2;
    const double rho = op->hscal->rho;
    // the FP64 judge of the answer
    double rel_true = 0;
    {
        const void* X64 = X;
        const void* B64 = B;
        if (tv != DT_F64) {
            PC_HIP(launch_cast(tv, DT_F64, X, op->vaux, n, s));
            PC_HIP(launch_cast(tv, DT_F64, B, op->vr, n, s));
            X64 = op->vaux;
            B64 = op->vr;
        }
        PC_TRY(apply_normal(op, X64, op->vq, CTA_PREC_F64, POST_NONE, nullptr, false, s));
        PC_HIP(launch_residual(DT_F64, DT_F64, B64, op->vq, op->vp, n, op->partials, op->scal, &op->scal->dot, s));
        if (hipMemcpyAsync(op->hscal, op->scal, sizeof(CgScalars), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(CTA_ERR_HIP, "scalar readback failed");
        rel_true = bn2 > 0 ? std::sqrt(op->hscal->dot / bn2) : std::sqrt(op->hscal->dot);
    }
    info->iters = sweeps;
    info->refine_steps = 0;
    info->rel_res_recursive = bn2 > 0 ? std::sqrt(std::max(rho, 0.0) / bn2) : 0.0;
    info->rel_res_true = rel_true;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    cta_status st;
    if (done == DONE_CONVERGED)
        st = CTA_OK;
    else if (done == DONE_BREAKDOWN)
        st = fail(CTA_ERR_BREAKDOWN, "Jacobi iteration diverged (non-finite residual)");
    else
        st = fail(CTA_NOT_CONVERGED, "tolerance not reached within the iteration limit");
    info->status = st;
    return st;
}

extern "C" cta_status cta_op_set_multigrid(cta_op op, int max_levels, int64_t coarse_max, int nu,
                                           double omega_scale) {
    if (!op) return fail(CTA_ERR_ARG, "op is NULL");
    mg_release(op);
    if (max_levels < 2) return CTA_OK;
    if (nu < 1 || nu > 8) return fail(CTA_ERR_ARG, "nu must be in [1, 8]");
    if (!(omega_scale > 0) || !(omega_scale < 2)) return fail(CTA_ERR_ARG, "omega_scale must be in (0, 2)");
    if (coarse_max < 1 || coarse_max > 4096) return fail(CTA_ERR_ARG, "coarse_max must be in [1, 4096]");
    const int N = op->order;
    op->mg_nu = nu;
    cta_mg_scale top;
    top.op = op;
    top.owned = false;
    top.omega = omega_scale / smoother_bound(op);
    op->mg.push_back(top);
    size_t& acc = op->dev_bytes;
    cta_status st = CTA_OK;
    for (;;) {
        cta_op_s* cur = op->mg.back().op;
        int64_t nc[CTA_MAX_ORDER];
        bool any = false;
        for (int k = 0; k < N; ++k) {
            nc[k] = cur->n[k] >= 8 ? (cur->n[k] + 1) / 2 : cur->n[k];
            any = any || nc[k] != cur->n[k];
        }
        if ((int)op->mg.size() == max_levels || cur->N <= coarse_max || !any) break;
        // GetScale: the next scale's operator and the transfer matrices
        cta_op_s* co = new cta_op_s();
        co->order = N;
        co->user_order = op->user_order;
        co->lift = op->lift;
        co->lam = op->lam;
        std::vector<std::vector<double>> G(N), R(N), P(N);
        std::vector<bool> has_reg(N, false);
        for (int k = 0; k < N; ++k) {
            co->n[k] = co->m[k] = nc[k];
            const int n_k = (int)cur->n[k], c_k = (int)nc[k];
            P[k] = interpolation(n_k, c_k);
            G[k] = galerkin(cur->hG[k], P[k], n_k, c_k);
            if (!cur->hR[k].empty()) {
                double s2 = 1.0;
                for (int l = 0; l < N; ++l)
                    if (l != k) s2 *= (double)cur->n[l] / (double)nc[l];
                R[k] = galerkin(cur->hR[k], P[k], n_k, c_k);
                for (double& v : R[k]) v *= s2;
                has_reg[k] = true;
            }
        }
        st = op_build(co, G, R, has_reg, nullptr);
        cta_mg_scale& fsc = op->mg.back();
        for (int k = 0; k < N && st == CTA_OK; ++k)
            for (int dt = 0; dt < 2 && st == CTA_OK; ++dt) {
                st = upload_mat(P[k].data(), (int)cur->n[k], (int)nc[k], false, dt, &fsc.P[dt][k], op->mg_allocs, acc);
                if (st == CTA_OK)
                    st = upload_mat(P[k].data(), (int)cur->n[k], (int)nc[k], true, dt, &fsc.Pt[dt][k], op->mg_allocs,
                                    acc);
            }
        if (st == CTA_OK && !fsc.T) st = dev_alloc(&fsc.T, (size_t)cur->N * 8, op->mg_allocs, acc);
        cta_mg_scale sc;
        sc.op = co;
        sc.owned = true;
        if (st == CTA_OK) {
            sc.omega = omega_scale / smoother_bound(co);
            st = dev_alloc(&sc.C, (size_t)co->N * 8, op->mg_allocs, acc);
        }
        if (st == CTA_OK) st = dev_alloc(&sc.B, (size_t)co->N * 8, op->mg_allocs, acc);
        if (st == CTA_OK) st = dev_alloc(&sc.T, (size_t)co->N * 8, op->mg_allocs, acc);
        if (st != CTA_OK) {
            std::string keep = cta_last_error();
            cta_op_destroy(co);
            mg_release(op);
            return fail(st, "%s", keep.c_str());
        }
        op->mg.push_back(sc);
    }
    if (op->mg.size() < 2) {
        mg_release(op);
        return fail(CTA_ERR_ARG, "the operator is already at or below coarse_max: no coarser scale");
    }
    const cta_op_s* last = op->mg.back().op;
    if (last->N > 4096) {
        const int64_t nn = last->N;
        mg_release(op);
        return fail(CTA_ERR_ARG, "the coarsest scale has %lld unknowns (more than 4096): raise max_levels",
                    (long long)nn);
    }
    // DirectSolve: the inverse of the coarsest assembled matrix
    const int nco = (int)last->N;
    std::vector<double> M = assemble(last), inv;
    if (!spd_inverse(M, nco, inv)) {
        mg_release(op);
        return fail(CTA_ERR_ARG, "the coarsest scale's matrix is not positive definite");
    }
    std::vector<float> inv32(inv.begin(), inv.end());
    st = dev_alloc(&op->mg_inv[0], inv.size() * 8, op->mg_allocs, acc);
    if (st == CTA_OK) st = dev_alloc(&op->mg_inv[1], inv.size() * 4, op->mg_allocs, acc);
    if (st == CTA_OK && (hipMemcpy(op->mg_inv[0], inv.data(), inv.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
                         hipMemcpy(op->mg_inv[1], inv32.data(), inv32.size() * 4, hipMemcpyHostToDevice) != hipSuccess))
        st = fail(CTA_ERR_HIP, "copy of the coarsest inverse failed");
    if (st != CTA_OK) {
        mg_release(op);
        return st;
    }
    op->mg_ncoarse = nco;
    return CTA_OK;
}

extern "C" cta_status cta_op_multigrid_info(cta_op op, int* host_levels, int64_t* host_extents,
                                            double* host_omega, int capacity) {
    if (!op || !host_levels) return fail(CTA_ERR_ARG, "NULL argument");
    *host_levels = (int)op->mg.size();
    const int N = op->user_order;
    for (int l = 0; l < (int)op->mg.size() && l < capacity; ++l) {
        if (host_extents)
            for (int k = 0; k < N; ++k) host_extents[(size_t)l * N + k] = op->mg[l].op->n[k + op->lift];
        if (host_omega) host_omega[l] = op->mg[l].omega;
    }
    return CTA_OK;
}

extern "C" cta_status cta_apply_multigrid(cta_op op, const void* R, void* Z, cta_dtype dtype, cta_precision chain,
                                          double* dot, void* stream) {
    if (!op || !R || !Z) return fail(CTA_ERR_ARG, "NULL argument");
    if (chain != CTA_PREC_F64 && chain != CTA_PREC_F32 && chain != CTA_PREC_BF16)
        return fail(CTA_ERR_ARG, "chain precision must be F64, F32 or BF16");
    PC_TRY(check_vec_dtype(dtype, chain));
    if (R == Z) return fail(CTA_ERR_ARG, "R and Z must not overlap");
    for (const auto& sc : op->mg)
        if (!tail_fits(chain == CTA_PREC_F64 ? DT_F64 : (chain == CTA_PREC_F32 ? DT_F32 : DT_BF16),
                       (int)sc.op->n[sc.op->order - 2], (int)sc.op->n[sc.op->order - 1]))
            return fail(CTA_ERR_UNSUPPORTED, "a scale's last two extents are too large for this precision");
    return mg_vcycle(op, R, Z, chain, dot ? POST_DOT : POST_NONE, dot, false, (hipStream_t)stream);
}
