// Host side of the C ABI: argument validation, factor setup (App. A.7),
// mode-order planning (Sec. 2.1), the CG driver (Fig. Tensor_CG) and the
// FP64 iterative refinement around a BF16 inner solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/cta.h"
#include "abi_internal.hpp"
#include "launch.hpp"

using namespace cta;

// ---------------------------------------------------------------------------
// errors
static thread_local std::string g_err;

namespace cta {
cta_status fail(cta_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}
}  // namespace cta

extern "C" const char* cta_last_error(void) { return g_err.c_str(); }
extern "C" const char* cta_version(void) { return "cta 0.1.0 gfx950"; }

// ---------------------------------------------------------------------------
// host helpers
namespace cta {

static uint16_t host_bf16(double x) {
    // double -> float (nearest) -> bf16 (nearest even), as the device does
    const float f = (float)x;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

static int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Upload a rows x cols row-major FP64 host matrix (optionally transposed) as a
// zero-padded device copy in dtype dt.
cta_status upload_mat(const double* host, int rows, int cols, bool trans, int dt, Mat* out,
                      std::vector<void*>& allocs, size_t& bytes_acc) {
    const int R = trans ? cols : rows, C = trans ? rows : cols;
    const int rs = (int)round_up(R, 64), ld = (int)round_up(C, 32);
    const size_t es = dt_size(dt);
    std::vector<unsigned char> buf((size_t)rs * ld * es, 0);
    for (int i = 0; i < R; ++i)
        for (int j = 0; j < C; ++j) {
            const double v = trans ? host[(size_t)j * cols + i] : host[(size_t)i * cols + j];
            unsigned char* dst = buf.data() + ((size_t)i * ld + j) * es;
            if (dt == DT_F64) {
                std::memcpy(dst, &v, 8);
            } else if (dt == DT_F32) {
                const float f = (float)v;
                std::memcpy(dst, &f, 4);
            } else {
                const uint16_t h = host_bf16(v);
                std::memcpy(dst, &h, 2);
            }
        }
    void* p = nullptr;
    if (hipMalloc(&p, buf.size()) != hipSuccess) return fail(CTA_ERR_NOMEM, "hipMalloc of a factor failed");
    allocs.push_back(p);
    bytes_acc += buf.size();
    if (hipMemcpy(p, buf.data(), buf.size(), hipMemcpyHostToDevice) != hipSuccess)
        return fail(CTA_ERR_HIP, "copy of a factor to the device failed");
    out->p = p;
    out->ld = ld;
    out->rows = R;
    out->cols = C;
    return CTA_OK;
}

cta_status dev_alloc(void** p, size_t bytes, std::vector<void*>& allocs, size_t& acc) {
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        return fail(CTA_ERR_NOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    allocs.push_back(*p);
    acc += bytes;
    return CTA_OK;
}

static int prec_tc(int prec) {
    return prec == CTA_PREC_F64 ? DT_F64 : (prec == CTA_PREC_F32 ? DT_F32 : DT_BF16);
}
static int prec_tvec(int prec) { return prec == CTA_PREC_F64 ? DT_F64 : DT_F32; }

// ---------------------------------------------------------------------------
// normal operator: Q = N(P)
//   pass A: tail on modes (N-2, N-1) of P (optionally fused with p = r + beta p)
//   middle: strided passes on modes N-3 .. 1
//   last  : mode 0 with the banded regulariser of P and <P, Q>
// Q = N(P) through the banded passes (F64 or F32, no fused CG update).
static cta_status apply_normal_band(cta_op_s* op, const void* P, void* Q, int prec, int post,
                                    double* dot_out, hipStream_t s) {
    const int N = op->order;
    const int dt = prec == CTA_PREC_F64 ? DT_F64 : DT_F32;
    const int bi = dt == DT_F64 ? 0 : 1;
    const void* cur = P;
    void* outs[2] = {op->T1, op->T2};
    int o = 0;
    for (int k = N - 1; k >= 1; --k) {
        int64_t lead = 1, trail = 1;
        for (int l = 0; l < k; ++l) lead *= op->n[l];
        for (int l = k + 1; l < N; ++l) trail *= op->n[l];
        hipError_t e = launch_band_mode(dt, cur, outs[o], op->gband[bi][k], op->band_w, lead, (int)op->n[k],
                                        trail, s);
        if (e != hipSuccess) return fail(CTA_ERR_HIP, "banded mode pass launch: %s", hipGetErrorString(e));
        cur = outs[o];
        o ^= 1;
    }
    StencilDesc st{};
    st.P = P;
    st.order = N;
    st.lam = op->lam;
    int64_t stride = 1;
    for (int k = N - 1; k >= 0; --k) {
        st.ext[k] = op->n[k];
        st.stride[k] = stride;
        stride *= op->n[k];
        st.rband[k] = op->rband[bi][k];
    }
    hipError_t e = launch_band_last(dt, cur, Q, op->gband[bi][0], op->band_w, (int)op->n[0], op->N / op->n[0],
                                    st, op->partials, op->scal, post, dot_out, s);
    if (e != hipSuccess) return fail(CTA_ERR_HIP, "banded last pass launch: %s", hipGetErrorString(e));
    return CTA_OK;
}

cta_status apply_normal(cta_op_s* op, const void* P, void* Q, int prec, int post,
                        double* dot_out, bool fuse_update, hipStream_t s, void* xsol,
                        const void* fuse_src, const int* gate) {
    if (op->use_band && !fuse_update && !gate && (prec == CTA_PREC_F64 || prec == CTA_PREC_F32) &&
        (post == POST_NONE || post == POST_DOT))
        return apply_normal_band(op, P, Q, prec, post, dot_out, s);
    const int N = op->order;
    const int tc = prec_tc(prec), tv = prec_tvec(prec);
    const int* done = gate ? gate : (fuse_update ? &op->scal->done : nullptr);
    const int a = N - 2, b = N - 1;
    const int64_t nblk = op->N / (op->n[a] * op->n[b]);
    if (!tail_fits(tc, (int)op->n[a], (int)op->n[b]))
        return fail(CTA_ERR_UNSUPPORTED,
                    "last two extents (%lld, %lld) exceed the fused-tail LDS budget for this precision",
                    (long long)op->n[a], (long long)op->n[b]);
    const void* Pin = P;
    void* pvec = nullptr;
    if (fuse_update) {
        Pin = fuse_src ? fuse_src : op->vr;   // chain input is r (or z) + beta p, written to p
        pvec = op->vp;
        P = op->vp;
    }
    hipError_t e = launch_tail(tv, tc, tc, Pin, op->T1, op->G[tc][a], op->G[tc][b], nblk,
                               (int)op->n[a], (int)op->n[b], (int)op->n[a], (int)op->n[b], pvec,
                               &op->scal->beta, done, s, op->var_tail[tc],
                               fuse_update ? xsol : nullptr, &op->scal->alpha);
    if (e != hipSuccess) return fail(CTA_ERR_HIP, "tail pass launch: %s", hipGetErrorString(e));
    void* cur = op->T1;
    void* nxt = op->T2;
    for (int k = N - 3; k >= 1; --k) {
        int64_t lead = 1, trail = 1;
        for (int l = 0; l < k; ++l) lead *= op->n[l];
        for (int l = k + 1; l < N; ++l) trail *= op->n[l];
        e = launch_strided(tc, cur, nxt, op->G[tc][k], lead, (int)op->n[k], (int)op->n[k], trail,
                           done, s, op->var_mid[tc]);
        if (e != hipSuccess) return fail(CTA_ERR_HIP, "mode pass launch: %s", hipGetErrorString(e));
        std::swap(cur, nxt);
    }
    StencilDesc st{};
    st.P = P;
    st.order = N;
    st.lam = op->lam;
    int64_t stride = 1;
    for (int k = N - 1; k >= 0; --k) {
        st.ext[k] = op->n[k];
        st.stride[k] = stride;
        stride *= op->n[k];
        st.rband[k] = op->rband[tv == DT_F64 ? 0 : 1][k];
    }
    e = launch_normal_last(tc, tv, tc, cur, Q, op->G[tc][0], (int)op->n[0], (int)op->n[0],
                           op->N / op->n[0], st, op->partials, op->scal, post, dot_out, done, s,
                           op->var_last[tc]);
    if (e != hipSuccess) return fail(CTA_ERR_HIP, "last pass launch: %s", hipGetErrorString(e));
    return CTA_OK;
}

// Z = M^-1(R): mode products of R with (G_k + c R_k)^-1, the same passes as
// the normal operator (fused tail, strided middle modes, last pass) with no
// regulariser in the last pass, whose FP64 dot gives <R, Z>.
cta_status apply_precond(cta_op_s* op, const void* R, void* Z, int prec, int post, double* dot_out,
                         bool gated, hipStream_t s, bool fuse_r) {
    if (!op->has_pc) return fail(CTA_ERR_ARG, "no preconditioner: call cta_op_set_preconditioner first");
    const int N = op->order;
    const int tc = prec_tc(prec), tv = prec_tvec(prec);
    const int* done = gated ? &op->scal->done : nullptr;
    const int a = N - 2, b = N - 1;
    const int64_t nblk = op->N / (op->n[a] * op->n[b]);
    hipError_t e;
    if (fuse_r) {
        // R is the residual: r -= alpha q (q in op->vq), <r, r> and the
        // stopping test in the same pass (BF16 chain)
        if (tc != DT_BF16) return fail(CTA_ERR_ARG, "the fused residual update needs the BF16 chain");
        e = launch_tail_r(const_cast<void*>(R), op->vq, op->T1, op->Pinv[tc][a], op->Pinv[tc][b], nblk,
                          (int)op->n[a], (int)op->n[b], (int)op->n[a], (int)op->n[b], &op->scal->alpha, done,
                          op->partials, op->scal, s, op->var_tail[tc]);
    } else {
        e = launch_tail(tv, tc, tc, R, op->T1, op->Pinv[tc][a], op->Pinv[tc][b], nblk, (int)op->n[a],
                        (int)op->n[b], (int)op->n[a], (int)op->n[b], nullptr, nullptr, done, s,
                        op->var_tail[tc]);
    }
    if (e != hipSuccess) return fail(CTA_ERR_HIP, "preconditioner tail launch: %s", hipGetErrorString(e));
    void* cur = op->T1;
    void* nxt = op->T2;
    for (int k = N - 3; k >= 1; --k) {
        int64_t lead = 1, trail = 1;
        for (int l = 0; l < k; ++l) lead *= op->n[l];
        for (int l = k + 1; l < N; ++l) trail *= op->n[l];
        e = launch_strided(tc, cur, nxt, op->Pinv[tc][k], lead, (int)op->n[k], (int)op->n[k], trail, done, s,
                           op->var_mid[tc]);
        if (e != hipSuccess) return fail(CTA_ERR_HIP, "preconditioner mode pass: %s", hipGetErrorString(e));
        std::swap(cur, nxt);
    }
    StencilDesc st{};
    st.P = R;
    st.order = N;
    st.lam = 0.0;
    int64_t stride = 1;
    for (int k = N - 1; k >= 0; --k) {
        st.ext[k] = op->n[k];
        st.stride[k] = stride;
        stride *= op->n[k];
        st.rband[k] = nullptr;
    }
    e = hipErrorNotSupported;
    if (tc == DT_BF16 && tv == DT_F32)
        e = launch_last_nr(cur, Z, R, op->Pinv[tc][0], (int)op->n[0], op->N / op->n[0], op->partials, op->scal,
                           post, dot_out, done, s);
    if (e == hipErrorNotSupported)
        e = launch_normal_last(tc, tv, tc, cur, Z, op->Pinv[tc][0], (int)op->n[0], (int)op->n[0],
                               op->N / op->n[0], st, op->partials, op->scal, post, dot_out, done, s,
                               op->var_last[tc]);
    if (e != hipSuccess) return fail(CTA_ERR_HIP, "preconditioner last pass: %s", hipGetErrorString(e));
    return CTA_OK;
}

// ---------------------------------------------------------------------------
// rectangular chain for forward / rhs / general TTM: planner + passes
// Choose the order of the mode products minimising flops (products on
// distinct modes commute, Sec. 2.1; Sec. 2.1 also motivates picking the order
// that gives the least work and the smallest intermediates).
std::vector<int> plan_order(int N, const int64_t* in_ext, const int64_t* out_ext,
                            const std::vector<int>& modes, int64_t* max_elems) {
    std::vector<int> perm(modes);
    std::sort(perm.begin(), perm.end());
    std::vector<int> best = perm;
    double best_cost = -1;
    int64_t best_max = 0;
    do {
        int64_t cur[CTA_MAX_ORDER];
        for (int k = 0; k < N; ++k) cur[k] = in_ext[k];
        double cost = 0;
        int64_t tot = 1, mx = 0;
        for (int k = 0; k < N; ++k) tot *= cur[k];
        mx = tot;
        for (int k : perm) {
            cost += 2.0 * (double)(tot / cur[k]) * (double)out_ext[k] * (double)cur[k];
            tot = tot / cur[k] * out_ext[k];
            cur[k] = out_ext[k];
            mx = std::max(mx, tot);
        }
        if (best_cost < 0 || cost < best_cost || (cost == best_cost && mx < best_max)) {
            best_cost = cost;
            best = perm;
            best_max = mx;
        }
    } while (std::next_permutation(perm.begin(), perm.end()));
    if (max_elems) *max_elems = best_max;
    return best;
}

// Run the chain: X (in dtype tin) -> Y (dtype tout) using compute type tc and
// the two work buffers (each >= max intermediate elements * size(tc)).
cta_status run_chain(int N, const int64_t* in_ext, const int64_t* out_ext, const Mat* mats,
                     const std::vector<int>& order, const void* X, int tin, void* Y, int tout,
                     int tc, void* w0, void* w1, hipStream_t s, const ChainBand* band, const int* gate) {
    int64_t cur[CTA_MAX_ORDER];
    int64_t tot = 1;
    for (int k = 0; k < N; ++k) {
        cur[k] = in_ext[k];
        tot *= cur[k];
    }
    const void* src = X;
    hipError_t e;
    if (tin != tc || order.empty()) {
        e = launch_cast(tin, tc, X, w0, tot, s);
        if (e != hipSuccess) return fail(CTA_ERR_HIP, "cast launch: %s", hipGetErrorString(e));
        src = w0;
    }
    if (order.empty()) {
        e = launch_cast(tc, tout, w0, Y, tot, s);
        if (e != hipSuccess) return fail(CTA_ERR_HIP, "cast launch: %s", hipGetErrorString(e));
        return CTA_OK;
    }
    for (size_t i = 0; i < order.size(); ++i) {
        const int k = order[i];
        const bool last = i + 1 == order.size();
        void* dst = (last && tout == tc) ? Y : (src == w0 ? w1 : w0);
        int64_t lead = 1, trail = 1;
        for (int l = 0; l < k; ++l) lead *= cur[l];
        for (int l = k + 1; l < N; ++l) trail *= cur[l];
        const int K = (int)cur[k], J = (int)out_ext[k];
        // the contiguous mode keeps the MFMA pass, which is faster there than
        // the banded one (rows of K contiguous elements are MFMA operands as
        // loaded)
        if (band && trail > 1)
            e = launch_rect_band(tc, src, dst, band->lo[k], band->coef[k], band->w, lead, K, J, trail, s);
        else if (trail == 1)
            e = launch_contig(tc, src, dst, mats[k], lead, K, J, gate, s);
        else
            e = launch_strided(tc, src, dst, mats[k], lead, K, J, trail, gate, s);
        if (e != hipSuccess) return fail(CTA_ERR_HIP, "mode %d pass launch: %s", k, hipGetErrorString(e));
        tot = tot / cur[k] * J;
        cur[k] = J;
        src = dst;
    }
    if (src != Y) {
        e = launch_cast(tc, tout, src, Y, tot, s);
        if (e != hipSuccess) return fail(CTA_ERR_HIP, "cast launch: %s", hipGetErrorString(e));
    }
    return CTA_OK;
}

}  // namespace cta

namespace cta {
// Everything of a handle that follows from G_k, R_k (and, when Ah is given,
// the collocation factors A_k): device copies, bands, work vectors, scalars.
// op->order, n, m, lam, lift and user_order must be set; on failure the
// caller destroys the handle.
cta_status op_build(cta_op_s* op, std::vector<std::vector<double>>& G, std::vector<std::vector<double>>& R,
                    const std::vector<bool>& has_reg, const std::vector<std::vector<double>>* Ah) {
    std::vector<std::vector<double>> none;
    const std::vector<std::vector<double>>& A = Ah ? *Ah : none;
    op->has_A = Ah != nullptr;
    op->N = 1;
    op->Msamp = 1;
    int64_t big = 1;
    for (int k = 0; k < op->order; ++k) {
        op->N *= op->n[k];
        op->Msamp *= op->m[k];
        big *= std::max(op->n[k], op->m[k]);
    }
    op->big = big;
    for (int k = 0; k < op->order; ++k) {
        op->hG[k] = G[k];
        op->hR[k] = R[k];
    }
    cta_status st = CTA_OK;
    auto& al = op->allocs;
    size_t& acc = op->dev_bytes;
    for (int k = 0; k < op->order && st == CTA_OK; ++k) {
        const int nk = (int)op->n[k], mk = (int)op->m[k];
        for (int dt = 0; dt < 3 && st == CTA_OK; ++dt)
            st = upload_mat(G[k].data(), nk, nk, false, dt, &op->G[dt][k], al, acc);
        for (int dt = 0; dt < 2 && st == CTA_OK && Ah; ++dt) {
            st = upload_mat(A[k].data(), mk, nk, false, dt, &op->A[dt][k], al, acc);
            if (st == CTA_OK) st = upload_mat(A[k].data(), mk, nk, true, dt, &op->At[dt][k], al, acc);
        }
        if (st == CTA_OK && has_reg[k]) {
            std::vector<double> band64(nk * 5, 0.0);
            std::vector<float> band32(nk * 5, 0.f);
            for (int i = 0; i < nk; ++i)
                for (int d = -2; d <= 2; ++d)
                    if (i + d >= 0 && i + d < nk) {
                        band64[i * 5 + d + 2] = R[k][(size_t)i * nk + i + d];
                        band32[i * 5 + d + 2] = (float)R[k][(size_t)i * nk + i + d];
                    }
            st = dev_alloc(&op->rband[0][k], band64.size() * 8, al, acc);
            if (st == CTA_OK) st = dev_alloc(&op->rband[1][k], band32.size() * 4, al, acc);
            if (st == CTA_OK &&
                (hipMemcpy(op->rband[0][k], band64.data(), band64.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
                 hipMemcpy(op->rband[1][k], band32.data(), band32.size() * 4, hipMemcpyHostToDevice) != hipSuccess))
                st = fail(CTA_ERR_HIP, "copy of regulariser bands failed");
        }
    }
    // banded Grams (B-spline collocation gives half-bandwidth 3): the band of
    // every G_k when all are within half-bandwidth kBandMax
    if (st == CTA_OK) {
        constexpr int kBandMax = 4;
        int w = 0;
        for (int k = 0; k < op->order; ++k) {
            const int nk = (int)op->n[k];
            for (int i = 0; i < nk; ++i)
                for (int j = 0; j < nk; ++j)
                    if (G[k][(size_t)i * nk + j] != 0.0) w = std::max(w, std::abs(i - j));
        }
        op->band_w = w;
        if (w <= kBandMax) {
            const int wd = 2 * w + 1;
            for (int k = 0; k < op->order && st == CTA_OK; ++k) {
                const int nk = (int)op->n[k];
                std::vector<double> b64((size_t)nk * wd, 0.0);
                std::vector<float> b32((size_t)nk * wd, 0.f);
                for (int i = 0; i < nk; ++i)
                    for (int d = -w; d <= w; ++d)
                        if (i + d >= 0 && i + d < nk) {
                            b64[(size_t)i * wd + d + w] = G[k][(size_t)i * nk + i + d];
                            b32[(size_t)i * wd + d + w] = (float)G[k][(size_t)i * nk + i + d];
                        }
                st = dev_alloc(&op->gband[0][k], b64.size() * 8, al, acc);
                if (st == CTA_OK) st = dev_alloc(&op->gband[1][k], b32.size() * 4, al, acc);
                if (st == CTA_OK &&
                    (hipMemcpy(op->gband[0][k], b64.data(), b64.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
                     hipMemcpy(op->gband[1][k], b32.data(), b32.size() * 4, hipMemcpyHostToDevice) != hipSuccess))
                    st = fail(CTA_ERR_HIP, "copy of the Gram bands failed");
            }
            op->band_ok = op->use_band = st == CTA_OK && op->N < ((int64_t)1 << 30);
        }
    }
    // banded rows of A_k and A_k^T for the forward and right-hand-side chains:
    // the span of each row's nonzeros, rounded up to 4, 6 or 8 columns
    for (int dir = 0; dir < 2 && st == CTA_OK && op->band_ok && Ah; ++dir) {
        int wmax = 0;
        std::vector<std::vector<int>> los(op->order);
        for (int k = 0; k < op->order; ++k) {
            const int nk = (int)op->n[k], mk = (int)op->m[k];
            const int rows = dir == 0 ? mk : nk, cols = dir == 0 ? nk : mk;
            los[k].assign(rows, 0);
            for (int r = 0; r < rows; ++r) {
                int first = -1, last = -1;
                for (int c = 0; c < cols; ++c) {
                    const double v = dir == 0 ? A[k][(size_t)r * nk + c] : A[k][(size_t)c * nk + r];
                    if (v != 0.0) {
                        if (first < 0) first = c;
                        last = c;
                    }
                }
                los[k][r] = first < 0 ? 0 : first;
                wmax = std::max(wmax, first < 0 ? 0 : last - first + 1);
            }
        }
        if (wmax > 8) continue;
        const int w = wmax <= 4 ? 4 : wmax <= 6 ? 6 : 8;
        for (int k = 0; k < op->order && st == CTA_OK; ++k) {
            const int nk = (int)op->n[k], mk = (int)op->m[k];
            const int rows = dir == 0 ? mk : nk, cols = dir == 0 ? nk : mk;
            std::vector<double> c64((size_t)rows * w, 0.0);
            std::vector<float> c32((size_t)rows * w, 0.f);
            for (int r = 0; r < rows; ++r)
                for (int c = 0; c < w; ++c) {
                    const int col = los[k][r] + c;
                    if (col >= cols) continue;
                    const double v = dir == 0 ? A[k][(size_t)r * nk + col] : A[k][(size_t)col * nk + r];
                    c64[(size_t)r * w + c] = v;
                    c32[(size_t)r * w + c] = (float)v;
                }
            st = dev_alloc((void**)&op->cb_lo[dir][k], (size_t)rows * 4, al, acc);
            if (st == CTA_OK) st = dev_alloc(&op->cb_coef[dir][0][k], c64.size() * 8, al, acc);
            if (st == CTA_OK) st = dev_alloc(&op->cb_coef[dir][1][k], c32.size() * 4, al, acc);
            if (st == CTA_OK &&
                (hipMemcpy(op->cb_lo[dir][k], los[k].data(), (size_t)rows * 4, hipMemcpyHostToDevice) != hipSuccess ||
                 hipMemcpy(op->cb_coef[dir][0][k], c64.data(), c64.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
                 hipMemcpy(op->cb_coef[dir][1][k], c32.data(), c32.size() * 4, hipMemcpyHostToDevice) != hipSuccess))
                st = fail(CTA_ERR_HIP, "copy of the factor bands failed");
        }
        if (st == CTA_OK) {
            op->cb_ok[dir] = true;
            op->cb_w[dir] = w;
        }
    }
    const size_t vb = (size_t)op->N * 8;
    void** vecs[] = {&op->T1, &op->T2, &op->vx, &op->vr, &op->vp, &op->vq, &op->vaux};
    for (void** v : vecs)
        if (st == CTA_OK) st = dev_alloc(v, vb, al, acc);
    if (st == CTA_OK) st = dev_alloc((void**)&op->scal, sizeof(CgScalars), al, acc);
    if (st == CTA_OK) st = dev_alloc((void**)&op->partials, kMaxGrid * sizeof(double), al, acc);
    if (st == CTA_OK) st = dev_alloc((void**)&op->partials2, kMaxGrid * sizeof(double), al, acc);
    // per-mode diagonals of G_k and R_k: the main diagonal of N is formed from
    // them on the fly (Jacobi steps of Fig. Tensor_Jacobi)
    for (int k = 0; k < op->order && st == CTA_OK; ++k) {
        const int nk = (int)op->n[k];
        std::vector<double> dg(nk), dr(nk);
        for (int i = 0; i < nk; ++i) {
            dg[i] = G[k][(size_t)i * nk + i];
            dr[i] = has_reg[k] ? R[k][(size_t)i * nk + i] : 0.0;
        }
        st = dev_alloc((void**)&op->dgm[k], (size_t)nk * 8, al, acc);
        if (st == CTA_OK && has_reg[k]) st = dev_alloc((void**)&op->drm[k], (size_t)nk * 8, al, acc);
        if (st == CTA_OK && hipMemcpy(op->dgm[k], dg.data(), (size_t)nk * 8, hipMemcpyHostToDevice) != hipSuccess)
            st = fail(CTA_ERR_HIP, "copy of the diagonal of G_k failed");
        if (st == CTA_OK && has_reg[k] &&
            hipMemcpy(op->drm[k], dr.data(), (size_t)nk * 8, hipMemcpyHostToDevice) != hipSuccess)
            st = fail(CTA_ERR_HIP, "copy of the diagonal of R_k failed");
    }
    if (st == CTA_OK && hipMemset(op->scal, 0, sizeof(CgScalars)) != hipSuccess)
        st = fail(CTA_ERR_HIP, "hipMemset of the scalars failed");
    if (st == CTA_OK && hipHostMalloc((void**)&op->hscal, sizeof(CgScalars), hipHostMallocDefault) != hipSuccess)
        st = fail(CTA_ERR_NOMEM, "hipHostMalloc of the scalar mirror failed");
    return st;
}
}  // namespace cta

// ---------------------------------------------------------------------------
// operator handle
extern "C" cta_status cta_op_create(cta_op* out, int order, const int64_t* n, const int64_t* m,
                                    const double* const* host_A, const double* const* host_D,
                                    const int64_t* p, double lambda, void* stream) {
    (void)stream;
    if (!out) return fail(CTA_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (order < 2 || order > CTA_MAX_ORDER) return fail(CTA_ERR_ARG, "order %d outside [2, %d]", order, CTA_MAX_ORDER);
    if (!n || !m || !host_A) return fail(CTA_ERR_ARG, "n, m and host_A are required");
    if (host_D && !p) return fail(CTA_ERR_ARG, "host_D given without p");
    if (!std::isfinite(lambda)) return fail(CTA_ERR_ARG, "lambda is not finite");
    for (int k = 0; k < order; ++k) {
        if (n[k] < 1 || m[k] < 1 || n[k] > CTA_MAX_EXTENT || m[k] > CTA_MAX_EXTENT)
            return fail(CTA_ERR_SHAPE, "mode %d: extents n=%lld m=%lld outside [1, %d]", k,
                        (long long)n[k], (long long)m[k], CTA_MAX_EXTENT);
        if (!host_A[k]) return fail(CTA_ERR_ARG, "host_A[%d] is NULL", k);
        if (host_D && p[k] < 0) return fail(CTA_ERR_SHAPE, "p[%d] < 0", k);
        if (host_D && p[k] > 0 && !host_D[k]) return fail(CTA_ERR_ARG, "host_D[%d] is NULL", k);
    }
    cta_op_s* op = new cta_op_s();
    // order 2 is lifted to order 3 with a leading unit mode (G = 1, no regulariser)
    const int lift = order == 2 ? 1 : 0;
    op->lift = lift;
    op->user_order = order;
    op->order = order + lift;
    op->lam = lambda;
    std::vector<std::vector<double>> G(op->order), A(op->order), R(op->order);
    std::vector<bool> has_reg(op->order, false);
    for (int k = 0; k < op->order; ++k) {
        const int uk = k - lift;
        if (uk < 0) {
            op->n[k] = 1;
            op->m[k] = 1;
            G[k] = {1.0};
            A[k] = {1.0};
            continue;
        }
        const int64_t nk = n[uk], mk = m[uk];
        op->n[k] = nk;
        op->m[k] = mk;
        A[k].assign(host_A[uk], host_A[uk] + nk * mk);
        G[k].assign(nk * nk, 0.0);
        for (int64_t i = 0; i < nk; ++i)
            for (int64_t j = 0; j < nk; ++j) {
                double sacc = 0;
                for (int64_t r = 0; r < mk; ++r) sacc += A[k][r * nk + i] * A[k][r * nk + j];
                G[k][i * nk + j] = sacc;
            }
        if (host_D && p[uk] > 0) {
            const int64_t pk = p[uk];
            const double* D = host_D[uk];
            R[k].assign(nk * nk, 0.0);
            for (int64_t i = 0; i < nk; ++i)
                for (int64_t j = 0; j < nk; ++j) {
                    double sacc = 0;
                    for (int64_t r = 0; r < pk; ++r) sacc += D[r * nk + i] * D[r * nk + j];
                    R[k][i * nk + j] = sacc;
                }
            for (int64_t i = 0; i < nk; ++i)
                for (int64_t j = 0; j < nk; ++j)
                    if (std::llabs(i - j) > 2 && R[k][i * nk + j] != 0.0) {
                        delete op;
                        return fail(CTA_ERR_UNSUPPORTED,
                                    "mode %d: D_k^T D_k has half-bandwidth > 2 (only banded regularisers "
                                    "with half-bandwidth <= 2 are supported)", uk);
                    }
            has_reg[k] = true;
        }
    }
    cta_status st = cta::op_build(op, G, R, has_reg, &A);
    if (st != CTA_OK) {
        std::string keep = g_err;
        cta_op_destroy(op);
        g_err = keep;
        return st;
    }
    *out = op;
    return CTA_OK;
}

extern "C" cta_status cta_op_destroy(cta_op op) {
    if (!op) return CTA_OK;
    (void)hipDeviceSynchronize();
    cta::mg_release(op);
    if (op->batch_buf) (void)hipFree(op->batch_buf);
    for (void* p : op->allocs) (void)hipFree(p);
    if (op->hscal) (void)hipHostFree(op->hscal);
    delete op;
    return CTA_OK;
}

extern "C" size_t cta_op_device_bytes(cta_op op) { return op ? op->dev_bytes : 0; }

namespace cta {
cta_status ensure_chain_ws(cta_op_s* op) {
    if (op->rw0) return CTA_OK;
    cta_status st = dev_alloc(&op->rw0, (size_t)op->big * 8, op->allocs, op->dev_bytes);
    if (st == CTA_OK) st = dev_alloc(&op->rw1, (size_t)op->big * 8, op->allocs, op->dev_bytes);
    return st;
}
}  // namespace cta

static cta_status check_dtype(cta_dtype d) {
    if (d != CTA_F64 && d != CTA_F32 && d != CTA_BF16) return fail(CTA_ERR_DTYPE, "unknown dtype %d", (int)d);
    return CTA_OK;
}

static cta_status op_chain(cta_op op, const void* X, cta_dtype xd, void* Y, cta_dtype yd,
                           cta_precision chain, bool forward, void* stream) {
    if (!op || !X || !Y) return fail(CTA_ERR_ARG, "NULL argument");
    cta_status st = check_dtype(xd);
    if (st == CTA_OK) st = check_dtype(yd);
    if (st != CTA_OK) return st;
    if (chain != CTA_PREC_F64 && chain != CTA_PREC_F32)
        return fail(CTA_ERR_ARG, "forward/rhs chains run in CTA_PREC_F64 or CTA_PREC_F32");
    if (!op->has_A) return fail(CTA_ERR_ARG, "this handle has no collocation factors");
    st = ensure_chain_ws(op);
    if (st != CTA_OK) return st;
    const int tc = prec_tc(chain);
    const int N = op->order;
    std::vector<int> modes;
    for (int k = op->lift; k < N; ++k) modes.push_back(k);
    const int64_t* in_ext = forward ? op->n : op->m;
    const int64_t* out_ext = forward ? op->m : op->n;
    std::vector<int> order = plan_order(N, in_ext, out_ext, modes, nullptr);
    const Mat* mats = forward ? op->A[tc == DT_F64 ? 0 : 1] : op->At[tc == DT_F64 ? 0 : 1];
    // banded factors (B-spline collocation): streaming banded passes
    const int dir = forward ? 0 : 1;
    ChainBand band{};
    const bool banded = op->use_band && op->cb_ok[dir];
    if (banded) {
        band.w = op->cb_w[dir];
        for (int k = 0; k < N; ++k) {
            band.lo[k] = op->cb_lo[dir][k];
            band.coef[k] = op->cb_coef[dir][tc == DT_F64 ? 0 : 1][k];
        }
    }
    return run_chain(N, in_ext, out_ext, mats, order, X, (int)xd, Y, (int)yd, tc, op->rw0, op->rw1,
                     (hipStream_t)stream, banded ? &band : nullptr);
}

extern "C" cta_status cta_forward(cta_op op, const void* X, cta_dtype x_dtype, void* Y,
                                  cta_dtype y_dtype, cta_precision chain, void* stream) {
    return op_chain(op, X, x_dtype, Y, y_dtype, chain, true, stream);
}

extern "C" cta_status cta_rhs(cta_op op, const void* Y, cta_dtype y_dtype, void* B,
                              cta_dtype b_dtype, cta_precision chain, void* stream) {
    return op_chain(op, Y, y_dtype, B, b_dtype, chain, false, stream);
}

extern "C" cta_status cta_apply_normal_op(cta_op op, const void* P, void* Q, cta_dtype dtype,
                                          cta_precision chain, double* dot, void* stream) {
    if (!op || !P || !Q) return fail(CTA_ERR_ARG, "NULL argument");
    if (chain != CTA_PREC_F64 && chain != CTA_PREC_F32 && chain != CTA_PREC_BF16)
        return fail(CTA_ERR_ARG, "chain precision must be F64, F32 or BF16");
    const int tv = prec_tvec(chain);
    if ((int)dtype != tv)
        return fail(CTA_ERR_DTYPE, "P/Q dtype must be %s for this chain precision",
                    tv == DT_F64 ? "CTA_F64" : "CTA_F32");
    if (P == Q) return fail(CTA_ERR_ARG, "P and Q must not overlap");
    return apply_normal(op, P, Q, chain, dot ? POST_DOT : POST_NONE, dot, false, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// CG driver
extern "C" void cta_cg_opts_default(cta_cg_opts* o) {
    if (!o) return;
    o->precision = CTA_PREC_F32;
    o->rtol = 1e-6;
    o->max_iter = 10000;
    o->x0_given = 0;
    o->fallback_zero = 0;
    o->precond = 0;
    o->inner_rtol = 1e-2;
    o->max_refine = 30;
    o->check_every = 16;
}

namespace cta {

static cta_status read_scal(cta_op_s* op, hipStream_t s) {
    if (hipMemcpyAsync(op->hscal, op->scal, sizeof(CgScalars), hipMemcpyDeviceToHost, s) != hipSuccess)
        return fail(CTA_ERR_HIP, "scalar readback failed");
    if (hipStreamSynchronize(s) != hipSuccess) return fail(CTA_ERR_HIP, "stream synchronize failed");
    return CTA_OK;
}

#define CTA_TRY(x)                          \
    do {                                    \
        cta_status st_ = (x);               \
        if (st_ != CTA_OK) return st_;      \
    } while (0)
#define CTA_HIP(x)                                                                  \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) return fail(CTA_ERR_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

// Inner CG loop on the handle's vectors: x (vx or the user's X), r = vr, p = vp,
// q = vq, with scal->rho and scal->bnorm2 already set.  Returns the final done flag.
cta_status cg_loop(cta_op_s* op, void* x, int prec, double rtol, int max_iter, int check_every,
                   hipStream_t s, int* done_out, int* iters_out, int pc) {
    const int tv = prec_tvec(prec);
    const size_t vb = (size_t)op->N * dt_size(tv);
    CTA_HIP(launch_fill_zero(op->vp, vb, s));
    // preconditioned: z = M^-1 r in vaux and <r, z> before the first step
    if (pc) CTA_TRY(precond_apply(op, pc, op->vr, op->vaux, prec, POST_DOT, &op->scal->rz, false, s));
    CTA_HIP(launch_cg_setup(op->scal, rtol * rtol, max_iter, s, pc ? 1 : 0));
    if (check_every < 1) check_every = 1;
    // x += alpha p of each step is applied by the next step's tail pass (which
    // reads p anyway); the last step's is flushed when the loop ends
    for (;;) {
        for (int c = 0; c < check_every; ++c) {
            CTA_TRY(apply_normal(op, nullptr, op->vq, prec, POST_ALPHA, nullptr, true, s, x,
                                 pc ? op->vaux : nullptr));
            if (pc)
                CTA_TRY(precond_step(op, pc, prec, s));
            else
                CTA_HIP(launch_cg_update(tv, nullptr, op->vr, op->vp, op->vq, op->N, op->partials, op->scal, s));
        }
        CTA_TRY(read_scal(op, s));
        if (op->hscal->done != DONE_RUNNING) break;
    }
    CTA_HIP(launch_x_flush(tv, x, op->vp, op->N, op->scal, s));
    *done_out = op->hscal->done;
    *iters_out = op->hscal->iters;
    return CTA_OK;
}

// FP64 residual norm ||B - N(X)||_2 for X and B of dtype tx; uses vaux, vq
// and vr as FP64 scratch.  NaN when the FP64 chain does not fit.
cta_status true_residual(cta_op_s* op, const void* B, const void* X, int tx, hipStream_t s,
                         double* res) {
    if (!tail_fits(DT_F64, (int)op->n[op->order - 2], (int)op->n[op->order - 1])) {
        *res = NAN;
        return CTA_OK;
    }
    const void* X64 = X;
    if (tx != DT_F64) {
        CTA_HIP(launch_cast(tx, DT_F64, X, op->vaux, op->N, s));
        X64 = op->vaux;
    }
    CTA_TRY(apply_normal(op, X64, op->vq, CTA_PREC_F64, POST_NONE, nullptr, false, s));
    const void* B64 = B;
    if (tx != DT_F64) {
        CTA_HIP(launch_cast(tx, DT_F64, B, op->vr, op->N, s));
        B64 = op->vr;
    }
    CTA_HIP(launch_residual(DT_F64, DT_F64, B64, op->vq, op->vr, op->N, op->partials, op->scal,
                            &op->scal->dot, s));
    CTA_TRY(read_scal(op, s));
    *res = std::sqrt(op->hscal->dot);
    return CTA_OK;
}

}  // namespace cta

extern "C" cta_status cta_cg_solve(cta_op op, const void* B, void* X, cta_dtype dtype,
                                   const cta_cg_opts* opts, cta_cg_info* info, void* stream) {
    if (!op || !B || !X || !opts || !info) return fail(CTA_ERR_ARG, "NULL argument");
    std::memset(info, 0, sizeof *info);
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    const int prec = opts->precision;
    if (prec < CTA_PREC_F64 || prec > CTA_PREC_BF16_RELIABLE) return fail(CTA_ERR_ARG, "bad precision");
    const bool mixed = prec == CTA_PREC_BF16_REFINE || prec == CTA_PREC_BF16_RELIABLE;
    const int pc = opts->precond;
    if (pc < PC_NONE || pc > PC_MULTIGRID) return fail(CTA_ERR_ARG, "precond must be 0, 1, 2 or 3");
    if (pc == PC_TENSOR_INV && !op->has_pc) return fail(CTA_ERR_ARG, "precond = 1 but no preconditioner was set");
    if (pc == PC_MULTIGRID && op->mg.empty())
        return fail(CTA_ERR_ARG, "precond = 3 but no multigrid hierarchy was set (cta_op_set_multigrid)");
    if (!(opts->rtol >= 0) || opts->max_iter < 0) return fail(CTA_ERR_ARG, "bad rtol or max_iter");
    const int want = (prec == CTA_PREC_F64 || mixed) ? DT_F64 : DT_F32;
    if ((int)dtype != want)
        return fail(CTA_ERR_DTYPE, "B and X must be %s for this precision", want == DT_F64 ? "CTA_F64" : "CTA_F32");
    if (B == X) return fail(CTA_ERR_ARG, "B and X must not overlap");
    const int N = op->order;
    if (!tail_fits(prec_tc(mixed ? CTA_PREC_F64 : prec), (int)op->n[N - 2], (int)op->n[N - 1]))
        return fail(CTA_ERR_UNSUPPORTED, "last two extents too large for the fused tail in this precision");
    const int check = opts->check_every > 0 ? opts->check_every : 16;
    const int64_t n = op->N;
    int done = 0, iters = 0;

    if (!mixed) {
        const int tv = prec_tvec(prec);
        const size_t vb = (size_t)n * dt_size(tv);
        CTA_HIP(launch_dot(tv, B, B, n, op->partials, op->scal, &op->scal->bnorm2, s));
        if (opts->x0_given) {
            CTA_TRY(apply_normal(op, X, op->vq, prec, POST_NONE, nullptr, false, s));
            CTA_HIP(launch_residual(tv, tv, B, op->vq, op->vr, n, op->partials, op->scal, &op->scal->rho, s));
            if (opts->fallback_zero) {
                CTA_TRY(read_scal(op, s));
                if (!(op->hscal->rho < op->hscal->bnorm2)) {
                    CTA_HIP(launch_fill_zero(X, vb, s));
                    CTA_HIP(launch_cast(tv, tv, B, op->vr, n, s));
                    CTA_HIP(launch_dot(tv, B, B, n, op->partials, op->scal, &op->scal->rho, s));
                }
            }
        } else {
            CTA_HIP(launch_fill_zero(X, vb, s));
            CTA_HIP(launch_cast(tv, tv, B, op->vr, n, s));
            CTA_HIP(launch_dot(tv, B, B, n, op->partials, op->scal, &op->scal->rho, s));
        }
        CTA_TRY(cg_loop(op, X, prec, opts->rtol, opts->max_iter, check, s, &done, &iters, pc));
        int total = iters;
        double rel_rec = std::sqrt(std::max(0.0, op->hscal->rho) / std::max(op->hscal->bnorm2, 1e-300));
        double bn2 = op->hscal->bnorm2;
        double rel_true = 0;
        CTA_TRY(true_residual(op, B, X, tv, s, &rel_true));
        rel_true = bn2 > 0 ? rel_true / std::sqrt(bn2) : rel_true;
        // one restart from the recomputed residual when the recursive residual
        // met the tolerance but the true one did not
        if (done == DONE_CONVERGED && rel_true > opts->rtol && total < opts->max_iter) {
            CTA_TRY(apply_normal(op, X, op->vq, prec, POST_NONE, nullptr, false, s));
            CTA_HIP(launch_residual(tv, tv, B, op->vq, op->vr, n, op->partials, op->scal, &op->scal->rho, s));
            CTA_HIP(launch_dot(tv, B, B, n, op->partials, op->scal, &op->scal->bnorm2, s));
            CTA_TRY(cg_loop(op, X, prec, opts->rtol, opts->max_iter - total, check, s, &done, &iters, pc));
            total += iters;
            rel_rec = std::sqrt(std::max(0.0, op->hscal->rho) / std::max(op->hscal->bnorm2, 1e-300));
            CTA_TRY(true_residual(op, B, X, tv, s, &rel_true));
            rel_true = bn2 > 0 ? rel_true / std::sqrt(bn2) : rel_true;
        }
        // the recursive test passed but the recomputed residual is still above
        // the tolerance after the restart: report it as not converged
        if (done == DONE_CONVERGED && std::isfinite(rel_true) && rel_true > opts->rtol)
            done = DONE_MAXITER;
        info->iters = total;
        info->refine_steps = 0;
        info->rel_res_recursive = rel_rec;
        info->rel_res_true = rel_true;
    } else {
        // FP64 iterative refinement; the inner solves use the BF16 chain
        const double rtol = opts->rtol;
        const double eta = opts->inner_rtol > 0 ? opts->inner_rtol : 1e-2;
        CTA_HIP(launch_dot(DT_F64, B, B, n, op->partials, op->scal, &op->scal->bnorm2, s));
        CTA_TRY(read_scal(op, s));
        const double bn2 = op->hscal->bnorm2;
        if (!opts->x0_given) CTA_HIP(launch_fill_zero(X, (size_t)n * 8, s));
        auto outer_residual = [&](double* rr) -> cta_status {
            CTA_TRY(apply_normal(op, X, op->vq, CTA_PREC_F64, POST_NONE, nullptr, false, s));
            CTA_HIP(launch_residual(DT_F64, DT_F32, B, op->vq, op->vr, n, op->partials, op->scal,
                                    &op->scal->rho, s));
            CTA_TRY(read_scal(op, s));
            *rr = op->hscal->rho;
            return CTA_OK;
        };
        double rr = 0;
        CTA_TRY(outer_residual(&rr));
        if (opts->x0_given && opts->fallback_zero && !(rr < bn2)) {
            CTA_HIP(launch_fill_zero(X, (size_t)n * 8, s));
            CTA_TRY(outer_residual(&rr));
        }
        int steps = 0, total = 0;
        done = DONE_RUNNING;
        if (prec == CTA_PREC_BF16_RELIABLE) {
            // One CG over the BF16 chain; vx holds the FP32 correction since the
            // last reliable update, vp the search direction kept across updates.
            const double target = rtol * rtol * bn2;
            const bool f32_ok = tail_fits(DT_F32, (int)op->n[N - 2], (int)op->n[N - 1]);
            CTA_HIP(launch_fill_zero(op->vx, (size_t)n * 4, s));
            CTA_HIP(launch_fill_zero(op->vp, (size_t)n * 4, s));
            // Every group cuts the residual by the same factor eta, so groups take
            // similar iteration counts: the first check of a group comes after as
            // many iterations as the previous group took, later ones every
            // check/4.  Iterations launched past convergence exit at once, but
            // each still costs a dispatch.
            int first_chunk = check;
            const int later_chunk = std::max(1, check / 4);
            while (true) {
                if (!std::isfinite(rr)) {
                    done = DONE_BREAKDOWN;
                    break;
                }
                if (rr <= target) {
                    done = DONE_CONVERGED;
                    break;
                }
                if (steps >= opts->max_refine) {
                    done = DONE_MAXITER;
                    break;
                }
                // iterate until the recursive residual has dropped by eta since this
                // update (or a little below the target, which the true residual then checks)
                const double thr = std::max(eta * eta * rr, 0.25 * target);
                if (pc)
                    CTA_TRY(precond_apply(op, pc, op->vr, op->vaux, CTA_PREC_BF16, POST_DOT, &op->scal->dot2, false,
                                          s));
                CTA_HIP(launch_cg_group(op->scal, thr, opts->max_iter, steps > 0 ? 1 : 0, s, pc ? 1 : 0));
                int gdone = DONE_RUNNING;
                for (int chunk = first_chunk;; chunk = later_chunk) {
                    for (int c = 0; c < chunk; ++c) {
                        CTA_TRY(apply_normal(op, nullptr, op->vq, CTA_PREC_BF16, POST_ALPHA, nullptr, true, s,
                                             op->vx, pc ? op->vaux : nullptr));
                        if (pc) {
                            CTA_TRY(precond_step(op, pc, CTA_PREC_BF16, s));
                        } else {
                            CTA_HIP(launch_cg_update(DT_F32, nullptr, op->vr, op->vp, op->vq, n, op->partials,
                                                     op->scal, s));
                        }
                    }
                    CTA_TRY(read_scal(op, s));
                    gdone = op->hscal->done;
                    if (gdone != DONE_RUNNING) break;
                }
                CTA_HIP(launch_x_flush(DT_F32, op->vx, op->vp, n, op->scal, s));
                total += op->hscal->iters;
                first_chunk = std::max(1, std::min(op->hscal->iters, 4 * check));
                if (gdone == DONE_BREAKDOWN && op->hscal->iters == 0) {
                    done = DONE_BREAKDOWN;
                    break;
                }
                // reliable update: X64 += vx, vx = 0, r = B - N(X64).  While the new
                // residual is expected above 1e-4 ||B|| (eta^2 times the last one), the
                // FP32 chain's error (~1e-6 ||B||) is below 1% of it and N(X) is formed
                // in FP32; the updates close to the tolerance use the FP64 chain.
                CTA_HIP(launch_add_f64((double*)X, op->vx, DT_F32, n, s));
                ++steps;
                const bool f32_update = eta * eta * rr > 1e-8 * bn2 && f32_ok;
                if (f32_update) {
                    CTA_HIP(launch_cast(DT_F64, DT_F32, X, op->vx, n, s));
                    CTA_TRY(apply_normal(op, op->vx, op->vq, CTA_PREC_F32, POST_NONE, nullptr, false, s));
                    CTA_HIP(launch_residual_mixed((const double*)B, (const float*)op->vq, (float*)op->vr, n,
                                                  op->partials, op->scal, &op->scal->dot, s));
                    CTA_HIP(launch_fill_zero(op->vx, (size_t)n * 4, s));
                } else {
                    CTA_HIP(launch_fill_zero(op->vx, (size_t)n * 4, s));
                    CTA_TRY(apply_normal(op, X, op->vq, CTA_PREC_F64, POST_NONE, nullptr, false, s));
                    CTA_HIP(launch_residual(DT_F64, DT_F32, B, op->vq, op->vr, n, op->partials, op->scal,
                                            &op->scal->dot, s));
                }
                CTA_TRY(read_scal(op, s));
                rr = op->hscal->dot;
                if (gdone == DONE_BREAKDOWN) {
                    done = rr <= target ? DONE_CONVERGED : DONE_BREAKDOWN;
                    break;
                }
            }
        }
        while (prec == CTA_PREC_BF16_REFINE) {
            if (!std::isfinite(rr)) {
                done = DONE_BREAKDOWN;
                break;
            }
            if (rr <= rtol * rtol * bn2) {
                done = DONE_CONVERGED;
                break;
            }
            if (steps >= opts->max_refine) {
                done = DONE_MAXITER;
                break;
            }
            // inner solve N_bf16 d = r (r in vr as FP32, rho = ||r||^2 already set)
            CTA_HIP(launch_fill_zero(op->vx, (size_t)n * 4, s));
            CTA_HIP(launch_dot(DT_F32, op->vr, op->vr, n, op->partials, op->scal, &op->scal->bnorm2, s));
            int idone = 0, iit = 0;
            CTA_TRY(cg_loop(op, op->vx, CTA_PREC_BF16, eta, opts->max_iter, check, s, &idone, &iit, pc));
            total += iit;
            if (idone == DONE_BREAKDOWN && iit == 0) {
                done = DONE_BREAKDOWN;
                break;
            }
            CTA_HIP(launch_add_f64((double*)X, op->vx, DT_F32, n, s));
            ++steps;
            CTA_TRY(outer_residual(&rr));
        }
        info->iters = total;
        info->refine_steps = steps;
        info->rel_res_recursive = std::sqrt(std::max(0.0, rr) / std::max(bn2, 1e-300));
        info->rel_res_true = info->rel_res_recursive;  // the outer residual is recomputed in FP64
    }
    if (hipStreamSynchronize(s) != hipSuccess) return fail(CTA_ERR_HIP, "stream synchronize failed");
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    cta_status st;
    if (done == DONE_CONVERGED)
        st = CTA_OK;
    else if (done == DONE_BREAKDOWN)
        st = fail(CTA_ERR_BREAKDOWN, "CG breakdown: <p, N p> <= 0 or a non-finite scalar");
    else
        st = fail(CTA_NOT_CONVERGED, "tolerance not reached within the iteration limit");
    info->status = st;
    return st;
}

// ---------------------------------------------------------------------------
// Autotuner of one operator's chain: every combination of pass variants is
// timed on the handle's workspace (median of `reps` applies) and validated
// against the default combination (the difference must be exactly zero: the
// variants change tiling only, not the order of any sum).
extern "C" cta_status cta_tune_op(cta_op op, cta_precision chain, int reps, void* stream) {
    if (!op) return fail(CTA_ERR_ARG, "op is NULL");
    if (chain != CTA_PREC_F64 && chain != CTA_PREC_F32 && chain != CTA_PREC_BF16)
        return fail(CTA_ERR_ARG, "chain precision must be F64, F32 or BF16");
    if (reps < 1) reps = 5;
    hipStream_t s = (hipStream_t)stream;
    const int tc = prec_tc(chain), tv = prec_tvec(chain);
    if (!tail_fits(tc, (int)op->n[op->order - 2], (int)op->n[op->order - 1]))
        return fail(CTA_ERR_UNSUPPORTED, "operator chain not supported in this precision");
    CTA_HIP(launch_fill_pattern(tv, op->vp, op->N, s));
    hipEvent_t e0, e1;
    CTA_HIP(hipEventCreate(&e0));
    CTA_HIP(hipEventCreate(&e1));
    int best[3] = {0, 0, 0};
    float best_ms = 1e30f;
    // the dense passes are what is tuned: banded applies are off meanwhile
    const bool use_band = op->use_band;
    op->use_band = false;
    // tail pass: 2 block counts; middle passes: 2 tile shapes and the
    // persistent pipelined form; last pass: 9 (two tile shapes, two
    // plane-grouped tile orders of the narrow one, row blocks with the whole
    // stencil in LDS, the persistent pipelined form with its two epilogues,
    // the second also with 512-thread workgroups, and plane sweeps with P in
    // an LDS ring)
    for (int combo = 0; combo < 54; ++combo) {
        op->var_tail[tc] = combo % 2;
        op->var_mid[tc] = (combo / 2) % 3;
        op->var_last[tc] = combo / 6;
        void* out = combo == 0 ? op->vaux : op->vq;
        cta_status st = apply_normal(op, op->vp, out, chain, POST_NONE, nullptr, false, s);
        if (st != CTA_OK) {
            op->use_band = use_band;
            return st;
        }
        if (combo != 0) {
            CTA_HIP(launch_residual(tv, tv, op->vaux, op->vq, op->vx, op->N, op->partials, op->scal,
                                    &op->scal->dot, s));
            CTA_TRY(read_scal(op, s));
            if (op->hscal->dot != 0.0) continue;  // not identical: never chosen
        }
        std::vector<float> ms;
        for (int r = 0; r < reps; ++r) {
            CTA_HIP(hipEventRecord(e0, s));
            st = apply_normal(op, op->vp, op->vq, chain, POST_NONE, nullptr, false, s);
            if (st != CTA_OK) {
                op->use_band = use_band;
                return st;
            }
            CTA_HIP(hipEventRecord(e1, s));
            CTA_HIP(hipEventSynchronize(e1));
            float t = 0;
            CTA_HIP(hipEventElapsedTime(&t, e0, e1));
            ms.push_back(t);
        }
        std::sort(ms.begin(), ms.end());
        const float med = ms[ms.size() / 2];
        if (med < best_ms) {
            best_ms = med;
            best[0] = combo % 2;
            best[1] = (combo / 2) % 3;
            best[2] = combo / 6;
        }
    }
    op->use_band = use_band;
    if (tc == DT_BF16 && best_ms < 1e30f) {
        // The tail pass inside CG also applies x += alpha p and p = r + beta p;
        // its persistent pipelined form (tail variant 2) is timed against the
        // chosen one on that fused pass, with alpha = beta = 0 so that every
        // apply sees the same input, and must give the identical output.
        op->var_mid[tc] = best[1];
        op->var_last[tc] = best[2];
        CgScalars hs{};
        hs.rho = 1.0;
        hs.bnorm2 = 1.0;
        hs.done = DONE_RUNNING;
        CTA_HIP(hipMemcpy(op->scal, &hs, sizeof hs, hipMemcpyHostToDevice));
        CTA_HIP(launch_fill_pattern(DT_F32, op->vr, op->N, s));
        const int cand[2] = {best[0], 2};
        float med2[2] = {1e30f, 1e30f};
        bool same = true;
        for (int c = 0; c < 2; ++c) {
            op->var_tail[tc] = cand[c];
            CTA_TRY(apply_normal(op, nullptr, c == 0 ? op->vaux : op->vq, chain, POST_NONE, nullptr, true, s,
                                 op->vx, nullptr));
            if (c == 1) {
                CTA_HIP(launch_residual(tv, tv, op->vaux, op->vq, op->vx, op->N, op->partials, op->scal,
                                        &op->scal->dot, s));
                CTA_TRY(read_scal(op, s));
                same = op->hscal->dot == 0.0;
            }
            std::vector<float> ms;
            for (int r = 0; r < reps; ++r) {
                CTA_HIP(hipEventRecord(e0, s));
                CTA_TRY(apply_normal(op, nullptr, op->vq, chain, POST_NONE, nullptr, true, s, op->vx, nullptr));
                CTA_HIP(hipEventRecord(e1, s));
                CTA_HIP(hipEventSynchronize(e1));
                float t = 0;
                CTA_HIP(hipEventElapsedTime(&t, e0, e1));
                ms.push_back(t);
            }
            std::sort(ms.begin(), ms.end());
            med2[c] = ms[ms.size() / 2];
        }
        if (same && med2[1] < med2[0]) best[0] = 2;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    op->var_tail[tc] = best[0];
    op->var_mid[tc] = best[1];
    op->var_last[tc] = best[2];
    return CTA_OK;
}

extern "C" cta_status cta_op_get_tuning(cta_op op, cta_precision chain, int* host_variants3) {
    if (!op || !host_variants3) return fail(CTA_ERR_ARG, "NULL argument");
    const int tc = prec_tc(chain);
    host_variants3[0] = op->var_tail[tc];
    host_variants3[1] = op->var_mid[tc];
    host_variants3[2] = op->var_last[tc];
    return CTA_OK;
}

extern "C" cta_status cta_op_set_tuning(cta_op op, cta_precision chain, const int* host_variants3) {
    if (!op || !host_variants3) return fail(CTA_ERR_ARG, "NULL argument");
    for (int i = 0; i < 3; ++i)
        if (host_variants3[i] < 0 || host_variants3[i] > (i == 2 ? 8 : 2))
            return fail(CTA_ERR_ARG, "variants must be 0..2 (tail, middle) and 0..8 (last)");
    const int tc = prec_tc(chain);
    op->var_tail[tc] = host_variants3[0];
    op->var_mid[tc] = host_variants3[1];
    op->var_last[tc] = host_variants3[2];
    return CTA_OK;
}

extern "C" cta_status cta_op_set_banded(cta_op op, int enable) {
    if (!op) return fail(CTA_ERR_ARG, "NULL operator");
    if (enable && !op->band_ok)
        return fail(CTA_ERR_ARG, "the Gram factors are not banded (half-bandwidth %d > 4)", op->band_w);
    op->use_band = enable != 0;
    return CTA_OK;
}

extern "C" int cta_op_band_width(cta_op op) { return op ? op->band_w : -1; }

// ---------------------------------------------------------------------------
// Tensor-inverse preconditioner: (G_k + c R_k)^-1 per mode, by Cholesky
// factorisation and forward / back substitution of the unit vectors (FP64).
namespace cta {
bool spd_inverse(const std::vector<double>& A, int n, std::vector<double>& inv) {
    std::vector<double> L((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double d = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(d > 0.0)) return false;
        const double ljj = std::sqrt(d);
        L[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double v = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) v -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = v / ljj;
        }
    }
    inv.assign((size_t)n * n, 0.0);
    std::vector<double> y(n);
    for (int c = 0; c < n; ++c) {
        for (int i = 0; i < n; ++i) {  // L y = e_c
            double v = i == c ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) v -= L[(size_t)i * n + k] * y[k];
            y[i] = v / L[(size_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {  // L^T x = y
            double v = y[i];
            for (int k = i + 1; k < n; ++k) v -= L[(size_t)k * n + i] * inv[(size_t)k * n + c];
            inv[(size_t)i * n + c] = v / L[(size_t)i * n + i];
        }
    }
    return true;
}
}  // namespace cta

namespace {
void release_mat(cta_op_s* op, Mat& m) {
    if (!m.p) return;
    void* p = const_cast<void*>(m.p);
    auto it = std::find(op->allocs.begin(), op->allocs.end(), p);
    if (it != op->allocs.end()) op->allocs.erase(it);
    (void)hipFree(p);
    m = Mat{};
}
}  // namespace

extern "C" cta_status cta_op_set_preconditioner(cta_op op, double c) {
    if (!op) return fail(CTA_ERR_ARG, "op is NULL");
    if (!std::isfinite(c)) return fail(CTA_ERR_ARG, "c must be finite");
    if (hipDeviceSynchronize() != hipSuccess) return fail(CTA_ERR_HIP, "synchronize failed");
    for (int dt = 0; dt < 3; ++dt)
        for (int k = 0; k < op->order; ++k) release_mat(op, op->Pinv[dt][k]);
    op->has_pc = false;
    if (c < 0) return CTA_OK;
    size_t acc = 0;
    for (int k = 0; k < op->order; ++k) {
        const int nk = (int)op->n[k];
        std::vector<double> M = op->hG[k], inv;
        if (!op->hR[k].empty())
            for (size_t i = 0; i < M.size(); ++i) M[i] += c * op->hR[k][i];
        if (!spd_inverse(M, nk, inv))
            return fail(CTA_ERR_ARG, "G_%d + c R_%d is not positive definite", k - op->lift, k - op->lift);
        for (int dt = 0; dt < 3; ++dt) {
            cta_status st = upload_mat(inv.data(), nk, nk, false, dt, &op->Pinv[dt][k], op->allocs, acc);
            if (st != CTA_OK) return st;
        }
    }
    op->dev_bytes += acc;
    op->has_pc = true;
    op->pc_c = c;
    return CTA_OK;
}

extern "C" cta_status cta_apply_precond(cta_op op, const void* R, void* Z, cta_dtype dtype,
                                        cta_precision chain, double* dot, void* stream) {
    if (!op || !R || !Z) return fail(CTA_ERR_ARG, "NULL argument");
    if (chain != CTA_PREC_F64 && chain != CTA_PREC_F32 && chain != CTA_PREC_BF16)
        return fail(CTA_ERR_ARG, "chain precision must be F64, F32 or BF16");
    const int want = chain == CTA_PREC_F64 ? CTA_F64 : CTA_F32;
    if ((int)dtype != want) return fail(CTA_ERR_DTYPE, "R and Z must be %s", want == CTA_F64 ? "CTA_F64" : "CTA_F32");
    if (R == Z) return fail(CTA_ERR_ARG, "R and Z must not overlap");
    if (!tail_fits(prec_tc(chain), (int)op->n[op->order - 2], (int)op->n[op->order - 1]))
        return fail(CTA_ERR_UNSUPPORTED, "operator chain not supported in this precision");
    return apply_precond(op, R, Z, chain, dot ? POST_DOT : POST_NONE, dot, false, (hipStream_t)stream);
}

extern "C" cta_status cta_tune_preconditioner(cta_op op, const void* B, void* X, cta_dtype dtype,
                                              const cta_cg_opts* opts, const double* host_c, int count,
                                              double* best_c, void* stream) {
    if (!op || !B || !X || !opts || !host_c || !best_c) return fail(CTA_ERR_ARG, "NULL argument");
    if (count < 1) return fail(CTA_ERR_ARG, "no candidates");
    cta_cg_opts o = *opts;
    o.precond = 1;
    o.x0_given = 0;
    double best = -1.0, best_s = 1e300;
    for (int i = 0; i < count; ++i) {
        if (!(host_c[i] >= 0)) return fail(CTA_ERR_ARG, "candidate %d is negative", i);
        CTA_TRY(cta_op_set_preconditioner(op, host_c[i]));
        cta_cg_info info;
        const cta_status st = cta_cg_solve(op, B, X, dtype, &o, &info, stream);
        if (st < 0 && st != CTA_ERR_BREAKDOWN) return st;
        if (st == CTA_OK && info.seconds < best_s) {
            best_s = info.seconds;
            best = host_c[i];
        }
    }
    *best_c = best;
    if (best < 0) {
        CTA_TRY(cta_op_set_preconditioner(op, -1.0));
        return fail(CTA_NOT_CONVERGED, "no candidate strength converged");
    }
    return cta_op_set_preconditioner(op, best);
}
