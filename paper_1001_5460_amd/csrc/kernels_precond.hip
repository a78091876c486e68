// gfx950 kernels of the tensor Jacobi iteration (Fig. Tensor_Jacobi) and of
// the tensor multigrid V-cycle (Fig. TMG): the diagonal of the normal
// operator formed on the fly from per-mode diagonals, the Jacobi smoothing
// and preconditioning steps fused with their FP64 inner products, the
// V-cycle's vector updates, and the dense solve of the coarsest scale.
//
// The main diagonal of N(X) = X x_1 G_1 ... x_N G_N + lam sum_k X x_k R_k at
// multi-index i is prod_k G_k[i_k, i_k] + lam sum_k R_k[i_k, i_k]; it is
// never stored as a tensor.  A thread handles 4 consecutive elements; when the
// contiguous extent is a multiple of 4 they share all leading indices, so the
// product and sum over the leading modes are formed once per group.
#include <algorithm>

#include "launch.hpp"
#include "prof.hpp"
#include "reduce.hpp"

namespace cta {

namespace {

constexpr int kPer = 4;  // elements per thread per sweep

int grid_for(int64_t n, int cap) {
    const int64_t per = (int64_t)CTA_WG * kPer;
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, cap));
}

__device__ __forceinline__ uint32_t fdiv(uint32_t v, uint32_t mul, int sh) {
    return (__umulhi(mul, v) + v) >> sh;
}

// Leading-mode terms of the diagonal for the row `lead` (flat index divided by
// the contiguous extent): prod_{k<N-1} g_k[i_k] and sum_{k<N-1} r_k[i_k], both
// accumulated in ascending mode order.
__device__ __forceinline__ void lead_terms(const DiagDesc& d, uint32_t lead, double& prod, double& sum) {
    uint32_t idx[8];
    for (int k = d.order - 2; k >= 0; --k) {
        const uint32_t q = fdiv(lead, d.fmul[k], d.fsh[k]);
        idx[k] = lead - q * (uint32_t)d.ext[k];
        lead = q;
    }
    prod = 1.0;
    sum = 0.0;
    for (int k = 0; k < d.order - 1; ++k) {
        prod *= d.g[k][idx[k]];
        if (d.r[k]) sum += d.r[k][idx[k]];
    }
}

__device__ __forceinline__ double diag_at(const DiagDesc& d, double prod, double sum, uint32_t j) {
    const int L = d.order - 1;
    const double rl = d.r[L] ? d.r[L][j] : 0.0;
    return prod * d.g[L][j] + d.lam * (sum + rl);
}

// Visit groups of 4 elements [i, i+4): FAST when the group shares its
// leading indices (n and the contiguous extent are multiples of 4), else
// element by element.  `dg[u]` is the diagonal of element i+u.
#define CTA_DIAG_SWEEP(n, d, BODY)                                                        \
    for (int64_t i = ((int64_t)blockIdx.x * CTA_WG + threadIdx.x) * kPer; i < (n);        \
         i += (int64_t)gridDim.x * CTA_WG * kPer) {                                      \
        const int L_ = (d).order - 1;                                                     \
        const int cnt = (int)std::min<int64_t>(kPer, (n) - i);                            \
        double dg[kPer] = {1.0, 1.0, 1.0, 1.0};                                          \
        if (cnt == kPer && ((d).ext[L_] % kPer) == 0) {                                   \
            const uint32_t lead = fdiv((uint32_t)i, (d).fmul[L_], (d).fsh[L_]);           \
            double pr, sm;                                                                \
            lead_terms((d), lead, pr, sm);                                                \
            const uint32_t j0 = (uint32_t)i - lead * (uint32_t)(d).ext[L_];               \
            for (int u = 0; u < kPer; ++u) dg[u] = diag_at((d), pr, sm, j0 + u);          \
        } else {                                                                          \
            for (int u = 0; u < cnt; ++u) {                                               \
                const uint32_t e = (uint32_t)(i + u);                                     \
                const uint32_t lead = fdiv(e, (d).fmul[L_], (d).fsh[L_]);                 \
                double pr, sm;                                                            \
                lead_terms((d), lead, pr, sm);                                            \
                dg[u] = diag_at((d), pr, sm, e - lead * (uint32_t)(d).ext[L_]);           \
            }                                                                             \
        }                                                                                 \
        BODY                                                                              \
    }

template <typename T> struct V4 { typedef T __attribute__((ext_vector_type(4))) type; };

// 4 consecutive elements as one vector access when FULL (16 or 32 bytes,
// aligned: i is a multiple of 4 and the arrays are allocation-aligned), else
// element by element for the first cnt.
template <typename T>
__device__ __forceinline__ typename V4<T>::type ld4(const T* p, bool full, int cnt) {
    typename V4<T>::type v;
    if (full) return *reinterpret_cast<const typename V4<T>::type*>(p);
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = u < cnt ? p[u] : T(0);
    return v;
}
template <typename T>
__device__ __forceinline__ void st4(T* p, const typename V4<T>::type& v, bool full, int cnt) {
    if (full) {
        *reinterpret_cast<typename V4<T>::type*>(p) = v;
        return;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (u < cnt) p[u] = v[u];
}

}  // namespace

// ------------------------------------------------------------------ z = omega r / d
template <typename T>
__global__ __launch_bounds__(CTA_WG) void k_jacobi_apply(const T* __restrict__ r, T* __restrict__ z,
                                                         int64_t n, DiagDesc d, double omega,
                                                         double* partials, const int* gate) {
    if (gate && *gate) return;
    __shared__ double red[4];
    double acc = 0.0;
    const bool vec = (n % 4) == 0;
    CTA_DIAG_SWEEP(n, d, {
        const bool full = vec && cnt == kPer;
        const typename V4<T>::type rv = ld4(r + i, full, cnt);
        typename V4<T>::type zv;
        for (int u = 0; u < kPer; ++u) {
            zv[u] = (T)(omega * (double)rv[u] / dg[u]);
            if (u < cnt) acc += (double)rv[u] * (double)zv[u];
        }
        st4(z + i, zv, full, cnt);
    })
    if (partials) block_partial(acc, partials, red);
}

hipError_t launch_jacobi_apply(int tv, const void* r, void* z, int64_t n, const DiagDesc& d, double omega,
                               double* partials, CgScalars* scal, int post, double* out, const int* gate,
                               hipStream_t s) {
    if (n >= ((int64_t)1 << 31)) return hipErrorNotSupported;
    const int g = grid_for(n, kMaxGrid);
    double* part = post == POST_NONE ? nullptr : partials;
    {
        ProfScope ps(tv == DT_F64 ? "jacobi_apply.f64" : "jacobi_apply.f32", s);
        if (tv == DT_F64)
            k_jacobi_apply<double><<<g, CTA_WG, 0, s>>>((const double*)r, (double*)z, n, d, omega, part, gate);
        else if (tv == DT_F32)
            k_jacobi_apply<float><<<g, CTA_WG, 0, s>>>((const float*)r, (float*)z, n, d, omega, part, gate);
        else
            return hipErrorInvalidValue;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return post == POST_NONE ? hipSuccess : launch_finalize(partials, g, scal, post, out, s);
}

// ------------------------------------------------------------------ r -= alpha q; z = r / d
// The preconditioned CG step with the diagonal preconditioner: the residual
// update, <r, r> (stopping test) and <r, z> (next conjugation ratio) in one
// pass over r and q.
template <typename T>
__global__ __launch_bounds__(CTA_WG) void k_jacobi_update(T* __restrict__ r, const T* __restrict__ q,
                                                          T* __restrict__ z, int64_t n, DiagDesc d,
                                                          double* partials, double* partials2,
                                                          const CgScalars* scal) {
    if (scal->done) return;
    __shared__ double red[4];
    const T alpha = (T)scal->alpha;
    double rr = 0.0, rz = 0.0;
    const bool vec = (n % 4) == 0;
    CTA_DIAG_SWEEP(n, d, {
        const bool full = vec && cnt == kPer;
        typename V4<T>::type rv = ld4(r + i, full, cnt);
        const typename V4<T>::type qv = ld4(q + i, full, cnt);
        typename V4<T>::type zv;
        for (int u = 0; u < kPer; ++u) {
            rv[u] = rv[u] - alpha * qv[u];
            zv[u] = (T)((double)rv[u] / dg[u]);
            if (u < cnt) {
                rr += (double)rv[u] * (double)rv[u];
                rz += (double)rv[u] * (double)zv[u];
            }
        }
        st4(r + i, rv, full, cnt);
        st4(z + i, zv, full, cnt);
    })
    block_partial(rr, partials, red);
    block_partial(rz, partials2, red);
}

hipError_t launch_jacobi_update(int tv, void* r, const void* q, void* z, int64_t n, const DiagDesc& d,
                                double* partials, double* partials2, CgScalars* scal, hipStream_t s) {
    if (n >= ((int64_t)1 << 31)) return hipErrorNotSupported;
    const int g = grid_for(n, kMaxGrid);
    {
        ProfScope ps(tv == DT_F64 ? "jacobi_update.f64" : "jacobi_update.f32", s);
        if (tv == DT_F64)
            k_jacobi_update<double><<<g, CTA_WG, 0, s>>>((double*)r, (const double*)q, (double*)z, n, d,
                                                         partials, partials2, scal);
        else if (tv == DT_F32)
            k_jacobi_update<float><<<g, CTA_WG, 0, s>>>((float*)r, (const float*)q, (float*)z, n, d, partials,
                                                        partials2, scal);
        else
            return hipErrorInvalidValue;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipError_t e = launch_finalize(partials, g, scal, POST_RHO, nullptr, s);
    if (e != hipSuccess) return e;
    return launch_finalize(partials2, g, scal, POST_RZ, nullptr, s);
}

// ------------------------------------------------------------------ C' = C + omega (B - Q) / d
// One damped Jacobi sweep with Q = N(C) given, written to Cout (which may be
// C itself).  dotmode 1 reduces ||B - Q||^2 (the residual of the C the sweep
// starts from: the stationary iteration's test), dotmode 2 reduces
// <B, C_new> (the V-cycle's <r, z>).
template <typename T>
__global__ __launch_bounds__(CTA_WG) void k_jacobi_correct(const T* C, T* Cout, const T* __restrict__ B,
                                                           const T* __restrict__ Q, int64_t n, DiagDesc d,
                                                           double omega, int dotmode, double* partials,
                                                           const int* gate) {
    if (gate && *gate) return;
    __shared__ double red[4];
    double acc = 0.0;
    const bool vec = (n % 4) == 0;
    CTA_DIAG_SWEEP(n, d, {
        const bool full = vec && cnt == kPer;
        const typename V4<T>::type bv = ld4(B + i, full, cnt);
        const typename V4<T>::type qv = ld4(Q + i, full, cnt);
        const typename V4<T>::type cv0 = ld4(C + i, full, cnt);
        typename V4<T>::type cv;
        for (int u = 0; u < kPer; ++u) {
            const double b = (double)bv[u];
            const double res = b - (double)qv[u];
            cv[u] = (T)((double)cv0[u] + omega * res / dg[u]);
            if (u < cnt) acc += dotmode == 1 ? res * res : b * (double)cv[u];
        }
        st4(Cout + i, cv, full, cnt);
    })
    if (dotmode) block_partial(acc, partials, red);
}

hipError_t launch_jacobi_correct(int tv, const void* C, void* Cout, const void* B, const void* Q, int64_t n,
                                 const DiagDesc& d, double omega, int dotmode, double* partials,
                                 CgScalars* scal, int post, double* out, const int* gate, hipStream_t s) {
    if (n >= ((int64_t)1 << 31)) return hipErrorNotSupported;
    const int g = grid_for(n, kMaxGrid);
    {
        ProfScope ps(tv == DT_F64 ? "jacobi_correct.f64" : "jacobi_correct.f32", s);
        if (tv == DT_F64)
            k_jacobi_correct<double><<<g, CTA_WG, 0, s>>>((const double*)C, (double*)Cout, (const double*)B,
                                                          (const double*)Q, n, d, omega, dotmode, partials,
                                                          gate);
        else if (tv == DT_F32)
            k_jacobi_correct<float><<<g, CTA_WG, 0, s>>>((const float*)C, (float*)Cout, (const float*)B,
                                                         (const float*)Q, n, d, omega, dotmode, partials,
                                                         gate);
        else
            return hipErrorInvalidValue;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return dotmode ? launch_finalize(partials, g, scal, post, out, s) : hipSuccess;
}

// ------------------------------------------------------------------ V-cycle vector steps
// t = b - t (the residual from t = N(C)), or c += t (the coarse correction);
// skipped when the gate (a solve's done flag) is set.
template <typename T, bool SUB>
__global__ __launch_bounds__(CTA_WG) void k_mg_vec(T* __restrict__ y, const T* __restrict__ x, int64_t n,
                                                   const int* gate) {
    if (gate && *gate) return;
    for (int64_t i = (int64_t)blockIdx.x * CTA_WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * CTA_WG)
        y[i] = SUB ? x[i] - y[i] : y[i] + x[i];
}

static hipError_t launch_mg_vec(int tv, bool sub, void* y, const void* x, int64_t n, const int* gate,
                                hipStream_t s) {
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((n + CTA_WG - 1) / CTA_WG, 65536));
    ProfScope ps(sub ? "mg_residual" : "mg_correct", s);
    if (tv == DT_F64 && sub)
        k_mg_vec<double, true><<<g, CTA_WG, 0, s>>>((double*)y, (const double*)x, n, gate);
    else if (tv == DT_F64)
        k_mg_vec<double, false><<<g, CTA_WG, 0, s>>>((double*)y, (const double*)x, n, gate);
    else if (tv == DT_F32 && sub)
        k_mg_vec<float, true><<<g, CTA_WG, 0, s>>>((float*)y, (const float*)x, n, gate);
    else if (tv == DT_F32)
        k_mg_vec<float, false><<<g, CTA_WG, 0, s>>>((float*)y, (const float*)x, n, gate);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_mg_sub(int tv, void* t, const void* b, int64_t n, const int* gate, hipStream_t s) {
    return launch_mg_vec(tv, true, t, b, n, gate, s);
}

hipError_t launch_mg_add(int tv, void* c, const void* t, int64_t n, const int* gate, hipStream_t s) {
    return launch_mg_vec(tv, false, c, t, n, gate, s);
}

// ------------------------------------------------------------------ coarsest scale: y = M x
// M is the n x n inverse of the coarsest system (row-major); one wave per
// row, each lane summing a strided part of the row in FP64, then a wave sum.
template <typename T>
__global__ __launch_bounds__(CTA_WG) void k_dense_matvec(const T* __restrict__ M, const T* __restrict__ x,
                                                         T* __restrict__ y, int n, const int* gate) {
    if (gate && *gate) return;
    const int row = blockIdx.x * CTA_WAVES + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const T* m = M + (int64_t)row * n;
    double acc = 0.0;
    for (int j = lane; j < n; j += 64) acc += (double)m[j] * (double)x[j];
    acc = wave_sum(acc);
    if (lane == 0) y[row] = (T)acc;
}

hipError_t launch_dense_matvec(int tv, const void* M, const void* x, void* y, int n, const int* gate,
                               hipStream_t s) {
    const int g = (n + CTA_WAVES - 1) / CTA_WAVES;
    ProfScope ps("mg_coarse_solve", s);
    if (tv == DT_F64)
        k_dense_matvec<double><<<g, CTA_WG, 0, s>>>((const double*)M, (const double*)x, (double*)y, n, gate);
    else if (tv == DT_F32)
        k_dense_matvec<float><<<g, CTA_WG, 0, s>>>((const float*)M, (const float*)x, (float*)y, n, gate);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace cta
