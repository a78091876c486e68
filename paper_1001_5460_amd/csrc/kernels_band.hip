// Band-aware normal operator for banded Gram factors (NEXT-4 of the scope:
// cubic B-spline collocation gives G_k = A_k^T A_k with half-bandwidth 3,
// Sec. 6, so a mode product with G_k is a 7-tap stencil along mode k).
//
// Q = P x_N G_N ... x_1 G_1 + lam sum_k P x_k R_k (the normal operator of
// Sec. 2.1 in normal-equation form) is applied as N streaming passes: modes
// N .. 2 as banded mode products T_out[b, j, t] = sum_d G_k[j, j+d] T_in[b,
// j+d, t], then mode 1 with the regulariser's 17-point stencil and the FP64
// partial sums of <P, Q> fused into the same pass.  Each pass reads and writes
// every element once (neighbour taps come from the caches), so a pass is
// bound by HBM bandwidth instead of the dense MFMA contraction, which does
// n_k / (2w + 1) times the flops.  Every sum runs over the taps in ascending
// offset; taps outside the tensor have zero coefficients and clamped
// addresses.
#include <algorithm>
#include <type_traits>

#include "launch.hpp"
#include "prof.hpp"
#include "reduce.hpp"
#include "ttm.hpp"

namespace cta {

template <typename T, int V>
struct VecT;
template <> struct VecT<double, 1> { typedef double type; };
template <> struct VecT<double, 2> { typedef double __attribute__((ext_vector_type(2))) type; };
template <> struct VecT<float, 1> { typedef float type; };
template <> struct VecT<float, 4> { typedef float __attribute__((ext_vector_type(4))) type; };

template <typename T, int V>
__device__ __forceinline__ typename VecT<T, V>::type ldv(const T* p) {
    return *reinterpret_cast<const typename VecT<T, V>::type*>(p);
}
template <typename T, int V>
__device__ __forceinline__ void stv(T* p, typename VecT<T, V>::type v) {
    *reinterpret_cast<typename VecT<T, V>::type*>(p) = v;
}

// ---------------------------------------------------------------------------
// Banded mode product on the (lead, K, trail) view.  A unit is JB consecutive
// rows j of V consecutive t of one b: the thread loads the JB + 2W input rows
// of its column strip once and forms the JB outputs from that window, so each
// input element is read (JB + 2W) / JB times instead of 2W + 1 times.
// gb[j * (2W + 1) + d + W] = G[j][j + d] (zero off the matrix).
constexpr int BAND_JB = 8;
constexpr int BAND_JB_LAST = 4;

struct BandModeArgs {
    const void* X;
    void* Y;
    const void* gb;
    int K, njb;          // rows and row blocks
    int64_t trail;
    int64_t nunit;       // lead * njb * trail / V  (< 2^30)
    uint32_t tmul, kmul;
    int tshift, kshift;  // division by trail / V and by njb
};

template <typename T, int W, int V, int JB>
__global__ __launch_bounds__(CTA_WG) void k_band_mode(BandModeArgs a) {
    typedef typename VecT<T, V>::type vt;
    const T* __restrict__ X = reinterpret_cast<const T*>(a.X);
    T* __restrict__ Y = reinterpret_cast<T*>(a.Y);
    const T* __restrict__ gb = reinterpret_cast<const T*>(a.gb);
    const int ntv = (int)(a.trail / V);
    for (int u = blockIdx.x * CTA_WG + threadIdx.x; u < (int)a.nunit; u += gridDim.x * CTA_WG) {
        const int q = fast_div(u, a.tmul, a.tshift);      // b * njb + row block
        const int tv = u - q * ntv;
        const int b = fast_div(q, a.kmul, a.kshift);
        const int j0 = (q - b * a.njb) * JB;
        const int64_t off = ((int64_t)b * a.K) * a.trail + (int64_t)tv * V;
        const T* __restrict__ xb = X + off;
        vt win[JB + 2 * W];
#pragma unroll
        for (int r = 0; r < JB + 2 * W; ++r) {
            const int jj = min(max(j0 - W + r, 0), a.K - 1);
            win[r] = ldv<T, V>(xb + (int64_t)jj * a.trail);
        }
#pragma unroll
        for (int i = 0; i < JB; ++i) {
            const int j = j0 + i;
            if (j >= a.K) break;
            const T* __restrict__ g = gb + j * (2 * W + 1);
            vt acc = vt(0);
#pragma unroll
            for (int d = -W; d <= W; ++d) acc += g[d + W] * win[i + d + W];
            stv<T, V>(Y + off + (int64_t)j * a.trail, acc);
        }
    }
}

template <typename T, int W>
static hipError_t band_mode_T(BandModeArgs a, int64_t lead, hipStream_t s) {
    constexpr int V = 16 / sizeof(T);
    constexpr int JB = BAND_JB;
    const bool vec = a.trail % V == 0;
    const int v = vec ? V : 1;
    a.njb = (a.K + JB - 1) / JB;
    a.nunit = lead * a.njb * (a.trail / v);
    if (a.nunit >= ((int64_t)1 << 30) || lead * a.K * a.trail >= ((int64_t)1 << 31))
        return hipErrorInvalidValue;  // int indices with headroom
    fastdiv_init((uint32_t)(a.trail / v), &a.tmul, &a.tshift);
    fastdiv_init((uint32_t)a.njb, &a.kmul, &a.kshift);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((a.nunit + CTA_WG - 1) / CTA_WG, 65536));
    if (vec)
        k_band_mode<T, W, V, JB><<<grid, CTA_WG, 0, s>>>(a);
    else
        k_band_mode<T, W, 1, JB><<<grid, CTA_WG, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_band_mode(int dt, const void* X, void* Y, const void* gb, int w, int64_t lead, int K,
                            int64_t trail, hipStream_t s) {
    BandModeArgs a{};
    a.X = X; a.Y = Y; a.gb = gb; a.K = K; a.trail = trail;
    ProfScope ps(dt == DT_F64 ? "band_mode.f64" : "band_mode.f32", s);
#define CTA_BAND_W(TT)                                                   \
    switch (w) {                                                         \
        case 0: return band_mode_T<TT, 0>(a, lead, s);                   \
        case 1: return band_mode_T<TT, 1>(a, lead, s);                   \
        case 2: return band_mode_T<TT, 2>(a, lead, s);                   \
        case 3: return band_mode_T<TT, 3>(a, lead, s);                   \
        case 4: return band_mode_T<TT, 4>(a, lead, s);                   \
    }
    if (dt == DT_F64) CTA_BAND_W(double)
    if (dt == DT_F32) CTA_BAND_W(float)
#undef CTA_BAND_W
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Mode-1 banded product + lam * 17-point regulariser + FP64 partials of
// <P, Q>, on the (K, trail) view (lead 1).  A unit is JB consecutive rows j of
// V consecutive t; the mode-1 taps of the chain input and of P come from
// windows of rows held in registers.  The regulariser sums mode 1, then modes 2 .. N-1, then mode N (taps
// in ascending offset); rband[k][i * 5 + d + 2] = R_k[i][i + d].
template <typename T>
struct BandLastArgs {
    const T* X;       // chain input (modes 2..N applied)
    const T* P;
    T* Q;
    const T* gb;      // G_1 band
    const T* rband[8];
    int64_t ext[8], stride[8];
    uint32_t smul[8], emul[8];
    int sshift[8], eshift[8];
    int order, K;
    int64_t trail, total;
    int64_t nunit;
    uint32_t tmul;
    int tshift;
    double lam;
    double* partials;
};

template <typename T, int W, int V, int JB>
__global__ __launch_bounds__(CTA_WG) void k_band_last(BandLastArgs<T> a) {
    typedef typename VecT<T, V>::type vt;
    __shared__ double red[CTA_WAVES];
    double dot = 0.0;
    const int N = a.order;
    const int ntv = (int)(a.trail / V);
    const T lam = (T)a.lam;
    const int nN = (int)a.ext[N - 1];
    const bool has1 = a.rband[0] != nullptr;
    const T* __restrict__ rbN = a.rband[N - 1];
    for (int u = blockIdx.x * CTA_WG + threadIdx.x; u < (int)a.nunit; u += gridDim.x * CTA_WG) {
        const int jb = fast_div(u, a.tmul, a.tshift);
        const int t = (u - jb * ntv) * V;
        const int j0 = jb * JB;
        // the rows j0 - W .. j0 + JB - 1 + W of the chain input and j0 - 2 ..
        // j0 + JB + 1 of P in this thread's column strip
        vt xw[JB + 2 * W], pw[JB + 4];
#pragma unroll
        for (int r = 0; r < JB + 2 * W; ++r) {
            const int jj = min(max(j0 - W + r, 0), a.K - 1);
            xw[r] = ldv<T, V>(a.X + (int64_t)jj * a.trail + t);
        }
#pragma unroll
        for (int r = 0; r < JB + 4; ++r) {
            const int jj = min(max(j0 - 2 + r, 0), a.K - 1);
            pw[r] = ldv<T, V>(a.P + (int64_t)jj * a.trail + t);
        }
        // positions along the other modes depend on t only
        const int i0 = t - fast_div(t, a.emul[N - 1], a.eshift[N - 1]) * nN;
#pragma unroll
        for (int i = 0; i < JB; ++i) {
            const int j = j0 + i;
            if (j >= a.K) break;
            const int64_t base = (int64_t)j * a.trail + t;
            // chain part: mode-1 banded product
            const T* __restrict__ g = a.gb + j * (2 * W + 1);
            vt acc = vt(0);
#pragma unroll
            for (int d = -W; d <= W; ++d) acc += g[d + W] * xw[i + d + W];
            // regulariser: mode 1, modes 2 .. N-1, mode N
            vt reg = vt(0);
            if (has1) {
                const T* __restrict__ br = a.rband[0] + j * 5;
#pragma unroll
                for (int d = -2; d <= 2; ++d) reg += br[d + 2] * pw[i + d + 2];
            }
            const vt pc = pw[i + 2];
            for (int k = 1; k < N - 1; ++k) {
                const T* __restrict__ rb = a.rband[k];
                if (!rb) continue;
                const int sk = (int)a.stride[k], nk = (int)a.ext[k];
                const int uk = fast_div(t, a.smul[k], a.sshift[k]);
                const int ik = uk - fast_div(uk, a.emul[k], a.eshift[k]) * nk;
                const T* __restrict__ br = rb + ik * 5;
#pragma unroll
                for (int d = -2; d <= 2; ++d) {
                    if (d == 0) {
                        reg += br[2] * pc;
                    } else {
                        const int dd = (ik + d >= 0 && ik + d < nk) ? d : 0;
                        reg += br[d + 2] * ldv<T, V>(a.P + base + (int64_t)dd * sk);
                    }
                }
            }
            if (rbN) {
                // contiguous mode: per-element band rows, taps at +-1, +-2,
                // read as the vectors before, at and after the unit (clamped
                // at the ends of the tensor, where the coefficients are zero)
                constexpr int L = V >= 2 ? V : 2;
                T w[3 * L];
                if constexpr (V >= 2) {
                    const vt pl = ldv<T, V>(a.P + max(base - V, (int64_t)0));
                    const vt pr = ldv<T, V>(a.P + min(base + V, a.total - V));
#pragma unroll
                    for (int e = 0; e < V; ++e) {
                        w[e] = pl[e];
                        w[L + e] = pc[e];
                        w[2 * L + e] = pr[e];
                    }
                } else {
#pragma unroll
                    for (int d = -2; d <= 3; ++d) w[L + d] = a.P[min(max(base + d, (int64_t)0), a.total - 1)];
                }
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    int ie = i0 + e;
                    if (ie >= nN) ie -= nN;
                    const T* __restrict__ br = rbN + ie * 5;
                    T sum = T(0);
#pragma unroll
                    for (int d = -2; d <= 2; ++d) sum += br[d + 2] * w[L + e + d];
                    if constexpr (V == 1)
                        reg += sum;
                    else
                        reg[e] += sum;
                }
            }
            const vt qv = acc + lam * reg;
            stv<T, V>(a.Q + base, qv);
            if constexpr (V == 1) {
                dot += (double)pc * (double)qv;
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) dot += (double)pc[e] * (double)qv[e];
            }
        }
    }
    block_partial(dot, a.partials, red);
}

template <typename T, int W>
static hipError_t band_last_T(BandLastArgs<T> a, int* grid_out, hipStream_t s) {
    constexpr int V = 16 / sizeof(T);
    const int N = a.order;
    bool vec = a.trail % V == 0 && a.ext[N - 1] % V == 0;
    for (int k = 1; k < N - 1; ++k) vec = vec && a.stride[k] % V == 0;
    const int v = vec ? V : 1;
    constexpr int JB = BAND_JB_LAST;
    a.nunit = (int64_t)((a.K + JB - 1) / JB) * (a.trail / v);
    if (a.total >= ((int64_t)1 << 30)) return hipErrorInvalidValue;  // int indices with headroom
    fastdiv_init((uint32_t)(a.trail / v), &a.tmul, &a.tshift);
    for (int k = 1; k < N; ++k) {
        fastdiv_init((uint32_t)a.stride[k], &a.smul[k], &a.sshift[k]);
        fastdiv_init((uint32_t)a.ext[k], &a.emul[k], &a.eshift[k]);
    }
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((a.nunit + CTA_WG - 1) / CTA_WG, kMaxGrid));
    *grid_out = grid;
    if (vec)
        k_band_last<T, W, V, JB><<<grid, CTA_WG, 0, s>>>(a);
    else
        k_band_last<T, W, 1, JB><<<grid, CTA_WG, 0, s>>>(a);
    return hipGetLastError();
}

template <typename T>
static hipError_t band_last_dispatch(const BandLastArgs<T>& a, int w, int* grid, hipStream_t s) {
    switch (w) {
        case 0: return band_last_T<T, 0>(a, grid, s);
        case 1: return band_last_T<T, 1>(a, grid, s);
        case 2: return band_last_T<T, 2>(a, grid, s);
        case 3: return band_last_T<T, 3>(a, grid, s);
        case 4: return band_last_T<T, 4>(a, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_band_last(int dt, const void* X, void* Q, const void* gb, int w, int K, int64_t trail,
                            const StencilDesc& st, double* partials, CgScalars* scal, int post,
                            double* dot_out, hipStream_t s) {
    int grid = 0;
    hipError_t e = hipErrorInvalidValue;
    {
        ProfScope ps(dt == DT_F64 ? "band_last.f64" : "band_last.f32", s);
        if (dt == DT_F64 || dt == DT_F32) {
            auto fill = [&](auto& a) {
                typedef std::remove_const_t<std::remove_reference_t<decltype(*a.P)>> TT;
                a.X = reinterpret_cast<const TT*>(X);
                a.P = reinterpret_cast<const TT*>(st.P);
                a.Q = reinterpret_cast<TT*>(Q);
                a.gb = reinterpret_cast<const TT*>(gb);
                for (int k = 0; k < st.order; ++k) {
                    a.rband[k] = reinterpret_cast<const TT*>(st.rband[k]);
                    a.ext[k] = st.ext[k];
                    a.stride[k] = st.stride[k];
                }
                a.order = st.order;
                a.K = K;
                a.trail = trail;
                a.total = (int64_t)K * trail;
                a.lam = st.lam;
                a.partials = partials;
            };
            if (dt == DT_F64) {
                BandLastArgs<double> a{};
                fill(a);
                e = band_last_dispatch(a, w, &grid, s);
            } else {
                BandLastArgs<float> a{};
                fill(a);
                e = band_last_dispatch(a, w, &grid, s);
            }
        }
    }
    if (e != hipSuccess || post == POST_NONE) return e;
    return launch_finalize(partials, grid, scal, post, dot_out, s);
}

}  // namespace cta

namespace cta {

// ---------------------------------------------------------------------------
// Banded rectangular mode product for the forward model and the right-hand
// side (Sec. 6: a sample touches 4 consecutive B-spline basis functions per
// mode, and a basis function a short run of consecutive samples):
// Y[b, j, t] = sum_{c < W} coef[j * W + c] * X[b, lo[j] + c, t] on the
// (lead, K -> J, trail) view.  Rows past K have zero coefficients and clamped
// addresses.  A unit is V consecutive t of one (b, j).
struct RectBandArgs {
    const void* X;
    void* Y;
    const int* lo;
    const void* coef;
    int K, J;
    int64_t trail;
    int64_t nunit;       // lead * J * trail / V  (< 2^30)
    uint32_t tmul, jmul;
    int tshift, jshift;  // division by trail / V and by J
};

template <typename T, int W, int V>
__global__ __launch_bounds__(CTA_WG) void k_rect_band(RectBandArgs a) {
    typedef typename VecT<T, V>::type vt;
    const T* __restrict__ X = reinterpret_cast<const T*>(a.X);
    T* __restrict__ Y = reinterpret_cast<T*>(a.Y);
    const T* __restrict__ cf = reinterpret_cast<const T*>(a.coef);
    const int ntv = (int)(a.trail / V);
    for (int u = blockIdx.x * CTA_WG + threadIdx.x; u < (int)a.nunit; u += gridDim.x * CTA_WG) {
        const int q = fast_div(u, a.tmul, a.tshift);      // b * J + j
        const int tv = u - q * ntv;
        const int b = fast_div(q, a.jmul, a.jshift);
        const int j = q - b * a.J;
        const int lo = a.lo[j];
        const T* __restrict__ xb = X + ((int64_t)b * a.K) * a.trail + (int64_t)tv * V;
        const T* __restrict__ c = cf + j * W;
        vt acc = vt(0);
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const int k = min(lo + i, a.K - 1);
            acc += c[i] * ldv<T, V>(xb + (int64_t)k * a.trail);
        }
        stv<T, V>(Y + (int64_t)q * a.trail + (int64_t)tv * V, acc);
    }
}

template <typename T, int W>
static hipError_t rect_band_T(RectBandArgs a, int64_t lead, hipStream_t s) {
    constexpr int V = 16 / sizeof(T);
    const bool vec = a.trail % V == 0;
    const int v = vec ? V : 1;
    a.nunit = lead * a.J * (a.trail / v);
    if (a.nunit >= ((int64_t)1 << 30) || lead * a.K * a.trail >= ((int64_t)1 << 31))
        return hipErrorInvalidValue;
    fastdiv_init((uint32_t)(a.trail / v), &a.tmul, &a.tshift);
    fastdiv_init((uint32_t)a.J, &a.jmul, &a.jshift);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((a.nunit + CTA_WG - 1) / CTA_WG, 65536));
    if (vec)
        k_rect_band<T, W, V><<<grid, CTA_WG, 0, s>>>(a);
    else
        k_rect_band<T, W, 1><<<grid, CTA_WG, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_rect_band(int dt, const void* X, void* Y, const int* lo, const void* coef, int w,
                            int64_t lead, int K, int J, int64_t trail, hipStream_t s) {
    RectBandArgs a{};
    a.X = X; a.Y = Y; a.lo = lo; a.coef = coef; a.K = K; a.J = J; a.trail = trail;
    ProfScope ps(dt == DT_F64 ? "rect_band.f64" : "rect_band.f32", s);
#define CTA_RECT_W(TT)                                                   \
    switch (w) {                                                         \
        case 4: return rect_band_T<TT, 4>(a, lead, s);                   \
        case 6: return rect_band_T<TT, 6>(a, lead, s);                   \
        case 8: return rect_band_T<TT, 8>(a, lead, s);                   \
    }
    if (dt == DT_F64) CTA_RECT_W(double)
    if (dt == DT_F32) CTA_RECT_W(float)
#undef CTA_RECT_W
    return hipErrorInvalidValue;
}

}  // namespace cta
