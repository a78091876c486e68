// gfx950 vector kernels of the tensor CG (Fig. Tensor_CG): elementwise
// updates (App. A.4) fused with FP64 inner products (App. A.6).
#include <algorithm>

#include "launch.hpp"
#include "prof.hpp"
#include "reduce.hpp"

namespace cta {

namespace {

constexpr int kItems = 4;  // elements per thread per sweep

int red_grid(int64_t n) {
    const int64_t per = (int64_t)CTA_WG * kItems;
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, kMaxGrid));
}

int plain_grid(int64_t n) {
    const int64_t per = (int64_t)CTA_WG * kItems;
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, 65536));
}

template <typename T> struct V4 { typedef T __attribute__((ext_vector_type(4))) type; };

// Visit elements [i, i+4) of every sweep; full groups of 4 use 16/32-byte
// accesses when the arrays are 4-element aligned (n % 4 == 0 suffices for
// device allocations), the ragged end is done element by element.
#define CTA_SWEEP(n, BODY4, BODY1)                                                   \
    for (int64_t i = ((int64_t)blockIdx.x * CTA_WG + threadIdx.x) * kItems; i < (n); \
         i += (int64_t)gridDim.x * CTA_WG * kItems) {                               \
        if (i + kItems <= (n) && ((n) % kItems) == 0) {                              \
            BODY4                                                                   \
        } else {                                                                    \
            for (int64_t e = i; e < std::min<int64_t>(i + kItems, (n)); ++e) {       \
                BODY1                                                               \
            }                                                                       \
        }                                                                           \
    }

}  // namespace

// ------------------------------------------------------------------ cast
template <typename Ti, typename To>
__global__ __launch_bounds__(CTA_WG) void k_cast(const Ti* __restrict__ x, To* __restrict__ y,
                                                 int64_t n) {
    CTA_SWEEP(n,
              {
                  for (int u = 0; u < kItems; ++u) y[i + u] = cvt<To>(x[i + u]);
              },
              { y[e] = cvt<To>(x[e]); })
}

hipError_t launch_cast(int tin, int tout, const void* x, void* y, int64_t n, hipStream_t s) {
    const int g = plain_grid(n);
    ProfScope ps("cast", s);
#define CTA_CAST(TI, TO, A, B)                                                              \
    if (tin == A && tout == B) {                                                            \
        k_cast<TI, TO><<<g, CTA_WG, 0, s>>>((const TI*)x, (TO*)y, n);                      \
        return hipGetLastError();                                                           \
    }
    CTA_CAST(double, float, DT_F64, DT_F32)
    CTA_CAST(float, double, DT_F32, DT_F64)
    CTA_CAST(double, bf16, DT_F64, DT_BF16)
    CTA_CAST(bf16, double, DT_BF16, DT_F64)
    CTA_CAST(float, bf16, DT_F32, DT_BF16)
    CTA_CAST(bf16, float, DT_BF16, DT_F32)
    CTA_CAST(double, double, DT_F64, DT_F64)
    CTA_CAST(float, float, DT_F32, DT_F32)
    CTA_CAST(bf16, bf16, DT_BF16, DT_BF16)
#undef CTA_CAST
    return hipErrorInvalidValue;
}

__global__ __launch_bounds__(CTA_WG) void k_zero(unsigned char* p, int64_t bytes) {
    for (int64_t i = ((int64_t)blockIdx.x * CTA_WG + threadIdx.x) * 16; i < bytes;
         i += (int64_t)gridDim.x * CTA_WG * 16) {
        if (i + 16 <= bytes) {
            *reinterpret_cast<uint4*>(p + i) = make_uint4(0, 0, 0, 0);
        } else {
            for (int64_t e = i; e < bytes; ++e) p[e] = 0;
        }
    }
}

hipError_t launch_fill_zero(void* x, int64_t bytes, hipStream_t s) {
    if (bytes <= 0) return hipSuccess;
    if ((reinterpret_cast<uintptr_t>(x) & 15) != 0) return hipErrorInvalidValue;
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((bytes + 4095) / 4096, 65536));
    ProfScope ps("fill_zero", s);
    k_zero<<<g, CTA_WG, 0, s>>>(reinterpret_cast<unsigned char*>(x), bytes);
    return hipGetLastError();
}

// ------------------------------------------------------------------ axpby
template <typename T>
__global__ __launch_bounds__(CTA_WG) void k_axpby(T a, const T* __restrict__ x, T b,
                                                  T* __restrict__ y, int64_t n) {
    typedef typename V4<T>::type v4;
    CTA_SWEEP(n,
              {
                  v4 xv = *reinterpret_cast<const v4*>(x + i);
                  v4 yv = *reinterpret_cast<v4*>(y + i);
                  *reinterpret_cast<v4*>(y + i) = a * xv + b * yv;
              },
              { y[e] = a * x[e] + b * y[e]; })
}

hipError_t launch_axpby(int tv, double a, const void* x, double b, void* y, int64_t n,
                        hipStream_t s) {
    const int g = plain_grid(n);
    ProfScope ps("axpby", s);
    if (tv == DT_F64) {
        k_axpby<double><<<g, CTA_WG, 0, s>>>(a, (const double*)x, b, (double*)y, n);
    } else if (tv == DT_F32) {
        k_axpby<float><<<g, CTA_WG, 0, s>>>((float)a, (const float*)x, (float)b, (float*)y, n);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ finalize
// One workgroup: total = sum of partials in index order, then the scalar step.
__global__ __launch_bounds__(1024) void k_finalize(const double* __restrict__ partials, int n,
                                                   CgScalars* scal, int post, double* out) {
    if ((post == POST_ALPHA || post == POST_RHO || post == POST_RZ) && scal->done) return;
    __shared__ double red[16];
    // thread i sums partials i, i+1024, i+2048, ... (loads issued four at a time)
    double acc = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * 1024 < n; i += 4 * 1024) {
        const double a0 = partials[i], a1 = partials[i + 1024];
        const double a2 = partials[i + 2048], a3 = partials[i + 3072];
        acc += a0;
        acc += a1;
        acc += a2;
        acc += a3;
    }
    for (; i < n; i += 1024) acc += partials[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x != 0) return;
    double total = 0.0;
    for (int w = 0; w < 16; ++w) total += red[w];
    if (post == POST_DOT) {
        *out = total;
    } else if (post == POST_ALPHA) {
        scal->pq = total;
        if (!(total > 0.0) || !__builtin_isfinite(total)) {
            scal->done = DONE_BREAKDOWN;
            scal->alpha = 0.0;  // no step: the pending x update of the fused tail is void
        } else {
            scal->alpha = (scal->precond ? scal->rz : scal->rho) / total;
        }
    } else if (post == POST_RHO) {
        const double rho = scal->rho;
        if (!scal->precond) scal->beta = total / rho;
        scal->rho = total;
        scal->iters += 1;
        if (!__builtin_isfinite(total))
            scal->done = DONE_BREAKDOWN;
        else if (total <= scal->threshold)
            scal->done = DONE_CONVERGED;
        else if (scal->iters >= scal->max_iter)
            scal->done = DONE_MAXITER;
    } else if (post == POST_RZ) {
        if (!(total > 0.0) || !__builtin_isfinite(total)) {
            scal->done = DONE_BREAKDOWN;  // the preconditioner is not positive definite
        } else {
            scal->beta = total / scal->rz;
            scal->rz = total;
        }
    }
}

hipError_t launch_finalize(const double* partials, int n, CgScalars* scal, int post, double* out,
                           hipStream_t s) {
    ProfScope ps("finalize", s);
    k_finalize<<<1, 1024, 0, s>>>(partials, n, scal, post, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ residual r = B - Q, <r, r>
template <typename Tb, typename Tr, typename Tq = Tb>
__global__ __launch_bounds__(CTA_WG) void k_residual(const Tb* __restrict__ B,
                                                     const Tq* __restrict__ Q, Tr* __restrict__ r,
                                                     int64_t n, double* partials) {
    __shared__ double red[4];
    double acc = 0.0;
    CTA_SWEEP(n,
              {
                  for (int u = 0; u < kItems; ++u) {
                      const Tr v = cvt<Tr>(B[i + u] - (Tb)Q[i + u]);
                      r[i + u] = v;
                      acc += (double)v * (double)v;
                  }
              },
              {
                  const Tr v = cvt<Tr>(B[e] - (Tb)Q[e]);
                  r[e] = v;
                  acc += (double)v * (double)v;
              })
    block_partial(acc, partials, red);
}

hipError_t launch_residual(int tb, int tr, const void* B, const void* Q, void* r, int64_t n,
                           double* partials, CgScalars* scal, double* out, hipStream_t s) {
    const int g = red_grid(n);
    {
        ProfScope ps(tb == DT_F64 ? (tr == DT_F64 ? "residual.f64" : "residual.f64_f32") : "residual.f32", s);
        if (tb == DT_F64 && tr == DT_F64)
            k_residual<double, double><<<g, CTA_WG, 0, s>>>((const double*)B, (const double*)Q,
                                                            (double*)r, n, partials);
        else if (tb == DT_F64 && tr == DT_F32)
            k_residual<double, float><<<g, CTA_WG, 0, s>>>((const double*)B, (const double*)Q,
                                                           (float*)r, n, partials);
        else if (tb == DT_F32 && tr == DT_F32)
            k_residual<float, float><<<g, CTA_WG, 0, s>>>((const float*)B, (const float*)Q,
                                                          (float*)r, n, partials);
        else
            return hipErrorInvalidValue;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_finalize(partials, g, scal, POST_DOT, out, s);
}

// r = B - Q with B in FP64 and Q in FP32, r stored in FP32, <r, r> reduced
hipError_t launch_residual_mixed(const double* B, const float* Q, float* r, int64_t n, double* partials,
                                 CgScalars* scal, double* out, hipStream_t s) {
    const int g = red_grid(n);
    {
        ProfScope ps("residual.f64_f32q", s);
        k_residual<double, float, float><<<g, CTA_WG, 0, s>>>(B, Q, r, n, partials);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_finalize(partials, g, scal, POST_DOT, out, s);
}

// ------------------------------------------------------------------ dot
template <typename T>
__global__ __launch_bounds__(CTA_WG) void k_dot(const T* __restrict__ x, const T* __restrict__ y,
                                                int64_t n, double* partials) {
    __shared__ double red[4];
    double acc = 0.0;
    CTA_SWEEP(n,
              {
                  for (int u = 0; u < kItems; ++u) acc += (double)x[i + u] * (double)y[i + u];
              },
              { acc += (double)x[e] * (double)y[e]; })
    block_partial(acc, partials, red);
}

hipError_t launch_dot(int tv, const void* x, const void* y, int64_t n, double* partials,
                      CgScalars* scal, double* out, hipStream_t s) {
    const int g = red_grid(n);
    {
        ProfScope ps(tv == DT_F64 ? "dot.f64" : "dot.f32", s);
        if (tv == DT_F64)
            k_dot<double><<<g, CTA_WG, 0, s>>>((const double*)x, (const double*)y, n, partials);
        else if (tv == DT_F32)
            k_dot<float><<<g, CTA_WG, 0, s>>>((const float*)x, (const float*)y, n, partials);
        else
            return hipErrorInvalidValue;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_finalize(partials, g, scal, POST_DOT, out, s);
}

// ------------------------------------------------------------------ CG step
// C += alpha P; R -= alpha Q; partial of rho1 = <R, R>.  The finalize kernel
// forms beta and the convergence test; P = R + beta P is fused into the first
// pass of the next operator application.
template <typename T, bool WITH_X>
__global__ __launch_bounds__(CTA_WG) void k_cg_update(T* __restrict__ x, T* __restrict__ r,
                                                      const T* __restrict__ p,
                                                      const T* __restrict__ q, int64_t n,
                                                      double* partials, const CgScalars* scal) {
    if (scal->done) return;
    __shared__ double red[4];
    typedef typename V4<T>::type v4;
    const T alpha = (T)scal->alpha;
    double acc = 0.0;
    CTA_SWEEP(n,
              {
                  if constexpr (WITH_X) {
                      v4 xv = *reinterpret_cast<v4*>(x + i);
                      const v4 pv = *reinterpret_cast<const v4*>(p + i);
                      xv = xv + alpha * pv;
                      *reinterpret_cast<v4*>(x + i) = xv;
                  }
                  // r's old value and q are dead after these reads: non-temporal
                  v4 rv = __builtin_nontemporal_load(reinterpret_cast<v4*>(r + i));
                  const v4 qv = __builtin_nontemporal_load(reinterpret_cast<const v4*>(q + i));
                  rv = rv - alpha * qv;
                  // the new r streams out too: the next pass reads it non-temporally,
                  // and kept out of the caches it leaves them to p, T and X
                  __builtin_nontemporal_store(rv, reinterpret_cast<v4*>(r + i));
                  for (int u = 0; u < kItems; ++u) acc += (double)rv[u] * (double)rv[u];
              },
              {
                  if constexpr (WITH_X) x[e] = x[e] + alpha * p[e];
                  const T rv = r[e] - alpha * q[e];
                  r[e] = rv;
                  acc += (double)rv * (double)rv;
              })
    block_partial(acc, partials, red);
}

template <typename T>
__global__ __launch_bounds__(CTA_WG) void k_x_flush(T* __restrict__ x, const T* __restrict__ p,
                                                    int64_t n, const CgScalars* scal) {
    const T alpha = (T)scal->alpha;
    for (int64_t i = (int64_t)blockIdx.x * CTA_WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * CTA_WG)
        x[i] = x[i] + alpha * p[i];
}

hipError_t launch_x_flush(int tv, void* x, const void* p, int64_t n, const CgScalars* scal,
                          hipStream_t s) {
    ProfScope ps("x_flush", s);
    const int g = plain_grid(n);
    if (tv == DT_F64)
        k_x_flush<double><<<g, CTA_WG, 0, s>>>((double*)x, (const double*)p, n, scal);
    else if (tv == DT_F32)
        k_x_flush<float><<<g, CTA_WG, 0, s>>>((float*)x, (const float*)p, n, scal);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_cg_update(int tv, void* x, void* r, const void* p, const void* q, int64_t n,
                            double* partials, CgScalars* scal, hipStream_t s) {
    const int g = red_grid(n);
    {
        ProfScope ps(x ? (tv == DT_F64 ? "cg_update.f64" : "cg_update.f32")
                       : (tv == DT_F64 ? "cg_update_r.f64" : "cg_update_r.f32"), s);
        if (tv == DT_F64 && x)
            k_cg_update<double, true><<<g, CTA_WG, 0, s>>>((double*)x, (double*)r, (const double*)p,
                                                           (const double*)q, n, partials, scal);
        else if (tv == DT_F64)
            k_cg_update<double, false><<<g, CTA_WG, 0, s>>>(nullptr, (double*)r, nullptr,
                                                            (const double*)q, n, partials, scal);
        else if (tv == DT_F32 && x)
            k_cg_update<float, true><<<g, CTA_WG, 0, s>>>((float*)x, (float*)r, (const float*)p,
                                                          (const float*)q, n, partials, scal);
        else if (tv == DT_F32)
            k_cg_update<float, false><<<g, CTA_WG, 0, s>>>(nullptr, (float*)r, nullptr,
                                                           (const float*)q, n, partials, scal);
        else
            return hipErrorInvalidValue;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_finalize(partials, g, scal, POST_RHO, nullptr, s);
}

__global__ void k_cg_setup(CgScalars* scal, double rtol2, int max_iter, int precond) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    scal->precond = precond;
    scal->threshold = rtol2 * scal->bnorm2;
    scal->rho0 = scal->rho;
    scal->beta = 0.0;
    scal->alpha = 0.0;
    scal->iters = 0;
    scal->max_iter = max_iter;
    if (!__builtin_isfinite(scal->rho) || !__builtin_isfinite(scal->bnorm2))
        scal->done = DONE_BREAKDOWN;
    else if (scal->rho <= scal->threshold)
        scal->done = DONE_CONVERGED;
    else if (max_iter <= 0)
        scal->done = DONE_MAXITER;
    else
        scal->done = DONE_RUNNING;
}

// Start of a group of CG iterations.  keep_dir = 0: a fresh start from the
// residual whose <r, r> is in scal->rho (beta = 0, the search direction is
// rebuilt from r).  keep_dir = 1: after a reliable update, the true
// residual's <r, r> is in scal->dot; the search direction is kept and
// beta = rho_true / rho_k, where rho_k = rho / beta is the residual norm
// before the last CG step.
__global__ void k_cg_group(CgScalars* scal, double threshold, int max_iter, int keep_dir,
                           int precond) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double rt = keep_dir ? scal->dot : scal->rho;
    double beta = 0.0;
    scal->precond = precond;
    if (precond) {
        // the same rescaling with <r, z>: beta = <r, z>_true / <r, z>_k
        const double zt = scal->dot2;
        if (keep_dir && scal->rz > 0.0) beta = scal->beta * zt / scal->rz;
        scal->rz = zt;
    } else if (keep_dir && scal->rho > 0.0) {
        beta = scal->beta * rt / scal->rho;
    }
    scal->beta = beta;
    scal->rho = rt;
    scal->rho0 = rt;
    scal->alpha = 0.0;
    scal->threshold = threshold;
    scal->iters = 0;
    scal->max_iter = max_iter;
    if (!__builtin_isfinite(rt) || !__builtin_isfinite(beta))
        scal->done = DONE_BREAKDOWN;
    else if (rt <= threshold)
        scal->done = DONE_CONVERGED;
    else if (max_iter <= 0)
        scal->done = DONE_MAXITER;
    else
        scal->done = DONE_RUNNING;
}

hipError_t launch_cg_group(CgScalars* scal, double threshold, int max_iter, int keep_dir, hipStream_t s,
                           int precond) {
    ProfScope ps("cg_group", s);
    k_cg_group<<<1, 64, 0, s>>>(scal, threshold, max_iter, keep_dir, precond);
    return hipGetLastError();
}

hipError_t launch_cg_setup(CgScalars* scal, double rtol2, int max_iter, hipStream_t s, int precond) {
    ProfScope ps("cg_setup", s);
    k_cg_setup<<<1, 64, 0, s>>>(scal, rtol2, max_iter, precond);
    return hipGetLastError();
}

// ------------------------------------------------------------------ test pattern
template <typename T>
__global__ __launch_bounds__(CTA_WG) void k_fill_pattern(T* x, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * CTA_WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * CTA_WG) {
        const uint32_t h = (uint32_t)(i * 2654435761ull) ^ (uint32_t)(i >> 32);
        x[i] = (T)((double)(h >> 8) * (1.0 / 16777216.0) - 0.5);
    }
}

hipError_t launch_fill_pattern(int tv, void* x, int64_t n, hipStream_t s) {
    const int g = plain_grid(n);
    if (tv == DT_F64)
        k_fill_pattern<double><<<g, CTA_WG, 0, s>>>((double*)x, n);
    else if (tv == DT_F32)
        k_fill_pattern<float><<<g, CTA_WG, 0, s>>>((float*)x, n);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ------------------------------------------------------------------ X64 += d
template <typename Td>
__global__ __launch_bounds__(CTA_WG) void k_add_f64(double* __restrict__ X,
                                                    const Td* __restrict__ d, int64_t n) {
    CTA_SWEEP(n,
              {
                  for (int u = 0; u < kItems; ++u) X[i + u] += (double)d[i + u];
              },
              { X[e] += (double)d[e]; })
}

hipError_t launch_add_f64(double* X, const void* d, int td, int64_t n, hipStream_t s) {
    const int g = plain_grid(n);
    ProfScope ps("add_f64", s);
    if (td == DT_F32)
        k_add_f64<float><<<g, CTA_WG, 0, s>>>(X, (const float*)d, n);
    else if (td == DT_F64)
        k_add_f64<double><<<g, CTA_WG, 0, s>>>(X, (const double*)d, n);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace cta

namespace cta {

// ------------------------------------------------------------------ factor padding
// dst[i][j] (rows_st x ld, dtype To) = op(src)[i][j] for i < R, j < C, else 0,
// where op(src) = src (rows x cols) or its transpose.
template <typename Ti, typename To>
__global__ __launch_bounds__(CTA_WG) void k_pad_matrix(const Ti* __restrict__ src, int rows,
                                                       int cols, int trans, To* __restrict__ dst,
                                                       int rows_st, int ld) {
    const int R = trans ? cols : rows, C = trans ? rows : cols;
    const int64_t total = (int64_t)rows_st * ld;
    for (int64_t e = (int64_t)blockIdx.x * CTA_WG + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * CTA_WG) {
        const int i = (int)(e / ld), j = (int)(e % ld);
        To v = cvt<To>(0.f);
        if (i < R && j < C) v = cvt<To>(trans ? src[(int64_t)j * cols + i] : src[(int64_t)i * cols + j]);
        dst[e] = v;
    }
}

hipError_t launch_pad_matrix(int tin, int tout, const void* src, int rows, int cols, int trans,
                             void* dst, int rows_st, int ld, hipStream_t s) {
    const int64_t total = (int64_t)rows_st * ld;
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((total + CTA_WG - 1) / CTA_WG, 4096));
    ProfScope ps("pad_matrix", s);
#define CTA_PAD(TI, TO, A, B)                                                                 \
    if (tin == A && tout == B) {                                                              \
        k_pad_matrix<TI, TO><<<g, CTA_WG, 0, s>>>((const TI*)src, rows, cols, trans, (TO*)dst, \
                                                  rows_st, ld);                               \
        return hipGetLastError();                                                             \
    }
    CTA_PAD(double, double, DT_F64, DT_F64)
    CTA_PAD(double, float, DT_F64, DT_F32)
    CTA_PAD(double, bf16, DT_F64, DT_BF16)
    CTA_PAD(float, double, DT_F32, DT_F64)
    CTA_PAD(float, float, DT_F32, DT_F32)
    CTA_PAD(float, bf16, DT_F32, DT_BF16)
    CTA_PAD(bf16, double, DT_BF16, DT_F64)
    CTA_PAD(bf16, float, DT_BF16, DT_F32)
    CTA_PAD(bf16, bf16, DT_BF16, DT_BF16)
#undef CTA_PAD
    return hipErrorInvalidValue;
}

}  // namespace cta
