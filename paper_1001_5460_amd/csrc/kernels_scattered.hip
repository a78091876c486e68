// gfx950 kernels of the scattered-measurement operator (Sec. 6): each
// measurement's row is the Khatri-Rao product of one cubic B-spline basis row
// per mode (the repeated-index product of Sec. 2.2), and the normal operator
// is the CANDECOMP sum over the measurements plus the Kronecker-sum
// regulariser.  Nothing of the system is stored: basis values are evaluated
// from the site coordinates inside the kernels.
//
// Layout.  Sites are sorted on the host into bricks of cells (a cell is one
// knot span per mode; a cubic window covers the span's 4 coefficients).  A
// brick of bc_k cells per mode touches a tile of te_k = bc_k + 3 coefficients
// per mode.  One workgroup takes one chunk of a brick's sites: it stages the
// coefficient tile in LDS, lets every thread gather and scatter its sites'
// 4^N windows on LDS (LDS atomics for the scatter), and writes the tile to its
// own slot of a scratch buffer.  A second kernel sums, for every coefficient,
// the slots of the (at most 2^N) bricks whose tiles cover it, in a fixed
// order, adds the regulariser's 4N+1-point stencil and reduces <P, Q> in FP64.
// No global atomics: the cross-brick sum is deterministic; the order of the
// LDS additions within one tile is not.
#include "launch.hpp"
#include "prof.hpp"
#include "reduce.hpp"

namespace cta {

namespace {

// Non-zero cubic basis values w[0..3] of the functions s..s+3 on knot span s
// at local coordinate u = t * C - s in [0, 1] (C = n - 3 spans).  In the
// scaled coordinate x = t * C the clamped uniform knots are the integers
// kn(i) = clamp(i - 3, 0, C), so the Cox-de Boor recursion (de Boor, 1972),
//   B_{j,p}(x) = (x - kn_j) / (kn_{j+p} - kn_j) B_{j,p-1}
//              + (kn_{j+p+1} - x) / (kn_{j+p+1} - kn_{j+1}) B_{j+1,p-1},
// has the small integers 1, 2, 3 as denominators on any non-empty span, and
// x - kn_j = u + (s - kn_j) with an exact integer offset (no loss of the
// low bits of u when s is large).
template <typename T>
__device__ __forceinline__ void cubic_window(T u, int s, int C, T (&w)[4]) {
    const T inv[4] = {(T)0, (T)1, (T)0.5, (T)1 / (T)3};
    auto kn = [C](int i) -> int { return min(max(i - 3, 0), C); };
    const int sp = s + 3;  // knot index of the span's left end
    T b[4] = {(T)1, (T)0, (T)0, (T)0};
#pragma unroll
    for (int p = 1; p <= 3; ++p) {
        T nb[4];
#pragma unroll
        for (int r = 0; r <= p; ++r) {
            const int j = sp - p + r;  // function B_{j,p}
            T v = (T)0;
            if (r > 0) v += (u + (T)(s - kn(j))) * inv[kn(j + p) - kn(j)] * b[r - 1];
            if (r < p) v += ((T)(kn(j + p + 1) - s) - u) * inv[kn(j + p + 1) - kn(j + 1)] * b[r];
            nb[r] = v;
        }
#pragma unroll
        for (int r = 0; r <= p; ++r) b[r] = nb[r];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) w[r] = b[r];
}

// <window, tile>: sum over the 4^N window at LDS offset `off` (modes K..N-1),
// nested in mode order.
template <typename T, int N, int K>
__device__ __forceinline__ T win_dot(const T* __restrict__ Xs, const T (&w)[4][4], const SopGeom& g,
                                     int off) {
    if constexpr (K == N - 1) {
        return w[K][0] * Xs[off] + w[K][1] * Xs[off + 1] + w[K][2] * Xs[off + 2] + w[K][3] * Xs[off + 3];
    } else {
        T acc = (T)0;
#pragma unroll
        for (int a = 0; a < 4; ++a) acc += w[K][a] * win_dot<T, N, K + 1>(Xs, w, g, off + a * g.ts[K]);
        return acc;
    }
}

template <typename T>
__device__ __forceinline__ void lds_add(T* p, T v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Acc[window] += v * (outer product of the weights)
template <typename T, int N, int K>
__device__ __forceinline__ void win_add(double* Acc, const T (&w)[4][4], const SopGeom& g, int off, T v) {
    if constexpr (K == N - 1) {
#pragma unroll
        for (int a = 0; a < 4; ++a) lds_add(Acc + off + a, (double)(v * w[K][a]));
    } else {
#pragma unroll
        for (int a = 0; a < 4; ++a) win_add<T, N, K + 1>(Acc, w, g, off + a * g.ts[K], v * w[K][a]);
    }
}

}  // namespace

// Threads of a brick workgroup.  A brick holds ~275 sites at the application
// size; 1024 threads take them in one round and give 16 waves per workgroup
// (measured: 3.55 ms with 256 threads, 2.92 ms with 512, 2.84 ms with 1024).
constexpr int kSopWG = 1024;

// One workgroup per chunk of a brick's sites.  MODE: SOP_FWD (y = A X),
// SOP_ADJ (tile of A^T y), SOP_NRM (tile of A^T A X).
template <typename T, int N, int MODE>
__global__ __launch_bounds__(kSopWG) void k_sop_brick(SopGeom g, const float* __restrict__ coords,
                                                      int64_t S, const int* __restrict__ perm,
                                                      const int* __restrict__ cstart,
                                                      const int* __restrict__ cbrick,
                                                      const T* __restrict__ X, const T* __restrict__ yin,
                                                      T* __restrict__ yout, T* __restrict__ tiles,
                                                      const CgScalars* scal) {
    if (scal && scal->done) return;
    // LDS: the accumulator tile in FP64 (FP64 LDS atomics; also for FP32
    // data, whose FP32 LDS atomics measured several times slower), then the
    // coefficient tile in T
    extern __shared__ __align__(16) unsigned char sop_smem[];
    double* Acc = reinterpret_cast<double*>(sop_smem);
    T* Xs = MODE == SOP_FWD ? reinterpret_cast<T*>(sop_smem)
                            : reinterpret_cast<T*>(sop_smem + (size_t)g.tile * sizeof(double));
    const int chunk = blockIdx.x;
    // brick coordinates and the first cell / coefficient of the brick
    int b0[4] = {0, 0, 0, 0};
    {
        int rem = cbrick[chunk];
#pragma unroll
        for (int k = N - 1; k >= 0; --k) {
            b0[k] = (rem % g.nb[k]) * g.bc[k];
            rem /= g.nb[k];
        }
    }
    // stage the coefficient tile (zero outside the tensor) and clear the accumulator
    for (int e = threadIdx.x; e < g.tile; e += kSopWG) {
        if constexpr (MODE != SOP_ADJ) {
            int rem = e;
            int64_t gi = 0;
            bool ok = true;
#pragma unroll
            for (int k = N - 1; k >= 0; --k) {
                const int c = b0[k] + rem % g.te[k];
                rem /= g.te[k];
                ok = ok && c < g.n[k];
                gi += (int64_t)c * g.gs[k];
            }
            Xs[e] = ok ? X[gi] : (T)0;
        }
        if constexpr (MODE != SOP_FWD) Acc[e] = 0.0;
    }
    __syncthreads();
    const int lo = cstart[chunk], hi = cstart[chunk + 1];
    for (int i = lo + (int)threadIdx.x; i < hi; i += kSopWG) {
        T w[4][4];
        int off = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const T t = (T)coords[(int64_t)k * S + i];
            int s = (int)(t * (T)g.C[k]);
            // the host sorted the site by its span in FP64; keep the window in the brick
            s = min(max(s, b0[k]), min(b0[k] + g.bc[k], g.C[k]) - 1);
            // u = t * C - s with one rounding (exact in FP64: t has 24 bits, C < 2^21)
            T u;
            if constexpr (sizeof(T) == 4)
                u = __builtin_fmaf(t, (T)g.C[k], -(T)s);
            else
                u = __builtin_fma(t, (T)g.C[k], -(T)s);
            cubic_window<T>(u, s, g.C[k], w[k]);
            off += (s - b0[k]) * g.ts[k];
        }
#pragma unroll
        for (int k = N; k < 4; ++k)
#pragma unroll
            for (int a = 0; a < 4; ++a) w[k][a] = (T)0;
        if constexpr (MODE == SOP_FWD) {
            yout[perm[i]] = win_dot<T, N, 0>(Xs, w, g, off);
        } else {
            const T v = MODE == SOP_NRM ? win_dot<T, N, 0>(Xs, w, g, off) : yin[perm[i]];
            win_add<T, N, 0>(Acc, w, g, off, v);
        }
    }
    if constexpr (MODE != SOP_FWD) {
        __syncthreads();
        T* dst = tiles + (int64_t)chunk * g.tile;
        for (int e = threadIdx.x; e < g.tile; e += kSopWG) dst[e] = (T)Acc[e];
    }
}

// Q[c] = sum of the tile slots covering c + lam * sum_k (R_k along mode k)(P)[c];
// FP64 partials of <P, Q>.  Workgroups walk the bricks; brick b owns the
// coefficients [b_k bc_k, (b_k + 1) bc_k) per mode (the last brick of a mode
// up to n_k).  An owned coefficient at local offset l_k is also covered by the
// tiles of bricks b_k - j with l_k + j bc_k <= bc_k + 2.  When every bc_k >= 3
// only j in {0, 1} occurs: the chunk ranges of those 2^N bricks are read into
// LDS once per brick, and the 2^N combinations are unrolled so that their
// tile loads issue together; the sum runs over the combinations in a fixed
// order and over each brick's chunks in order.
template <typename T, int N>
__global__ __launch_bounds__(CTA_WG) void k_sop_gather(SopGeom g, const T* __restrict__ tiles,
                                                       const int* __restrict__ bchunk0,
                                                       const T* __restrict__ P, const T* __restrict__ rb,
                                                       T lam, T* __restrict__ Q, double* partials,
                                                       int nbricks, const CgScalars* scal) {
    if (scal && scal->done) return;
    __shared__ double red[4];
    __shared__ int nbr_lo[16], nbr_hi[16];
    bool wide = true;
#pragma unroll
    for (int k = 0; k < N; ++k) wide = wide && g.bc[k] >= 3;
    double dot = 0.0;
    for (int brick = blockIdx.x; brick < nbricks; brick += gridDim.x) {
        int bk[4] = {0, 0, 0, 0}, ob[4] = {1, 1, 1, 1}, bs[4] = {0, 0, 0, 0};
        int owned = 1;
        {
            int rem = brick, st = 1;
#pragma unroll
            for (int k = N - 1; k >= 0; --k) {
                bk[k] = rem % g.nb[k];
                rem /= g.nb[k];
                bs[k] = st;
                st *= g.nb[k];
                ob[k] = bk[k] == g.nb[k] - 1 ? g.n[k] - bk[k] * g.bc[k] : g.bc[k];
                owned *= ob[k];
            }
        }
        if (wide) {
            __syncthreads();  // the previous brick's ranges are no longer read
            if ((int)threadIdx.x < (1 << N)) {
                int br = brick;
                bool ok = true;
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const int jk = ((int)threadIdx.x >> k) & 1;
                    ok = ok && bk[k] - jk >= 0;
                    br -= jk * bs[k];
                }
                nbr_lo[threadIdx.x] = ok ? bchunk0[br] : 0;
                nbr_hi[threadIdx.x] = ok ? bchunk0[br + 1] : 0;
            }
            __syncthreads();
        }
        for (int e = threadIdx.x; e < owned; e += CTA_WG) {
            int l[4] = {0, 0, 0, 0}, jm[4] = {0, 0, 0, 0}, j[4];
            int64_t c = 0;
            {
                int rem = e;
#pragma unroll
                for (int k = N - 1; k >= 0; --k) {
                    l[k] = rem % ob[k];
                    rem /= ob[k];
                    c += (int64_t)(bk[k] * g.bc[k] + l[k]) * g.gs[k];
                    while (bk[k] - jm[k] - 1 >= 0 && l[k] + (jm[k] + 1) * g.bc[k] <= g.bc[k] + 2) ++jm[k];
                    j[k] = jm[k];
                }
            }
            T sum = (T)0;
            if (wide) {
                int base = 0;
#pragma unroll
                for (int k = 0; k < N; ++k) base += l[k] * g.ts[k];
#pragma unroll
                for (int q = 0; q < (1 << N); ++q) {
                    bool cov = true;
                    int local = base;
#pragma unroll
                    for (int k = 0; k < N; ++k) {
                        const int jk = (q >> k) & 1;
                        cov = cov && jk <= jm[k];
                        local += jk * g.bc[k] * g.ts[k];
                    }
                    if (cov) {
                        const int c1 = nbr_hi[q];
                        for (int ch = nbr_lo[q]; ch < c1; ++ch) sum += tiles[(int64_t)ch * g.tile + local];
                    }
                }
            } else {
                for (;;) {
                    int br = brick, local = 0;
#pragma unroll
                    for (int k = 0; k < N; ++k) {
                        br -= j[k] * bs[k];
                        local += (l[k] + j[k] * g.bc[k]) * g.ts[k];
                    }
                    const int c1 = bchunk0[br + 1];
                    for (int ch = bchunk0[br]; ch < c1; ++ch) sum += tiles[(int64_t)ch * g.tile + local];
                    int k = N - 1;
                    for (; k >= 0; --k) {
                        if (--j[k] >= 0) break;
                        j[k] = jm[k];
                    }
                    if (k < 0) break;
                }
            }
            if (P) {
                T reg = (T)0;
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const int ck = bk[k] * g.bc[k] + l[k];
                    const T* row = rb + 5 * ((int64_t)g.roff[k] + ck);
#pragma unroll
                    for (int d = -2; d <= 2; ++d) {
                        const int jj = ck + d;
                        if (jj >= 0 && jj < g.n[k]) reg += row[d + 2] * P[c + (int64_t)d * g.gs[k]];
                    }
                }
                const T q = sum + lam * reg;
                Q[c] = q;
                dot += (double)P[c] * (double)q;
            } else {
                Q[c] = sum;
            }
        }
    }
    if (partials) block_partial(dot, partials, red);
}

// x += alpha p (the previous step's); p = r + beta p
template <typename T>
__global__ __launch_bounds__(CTA_WG) void k_sop_pstep(T* __restrict__ x, T* __restrict__ p,
                                                      const T* __restrict__ r, int64_t n,
                                                      const CgScalars* scal) {
    if (scal->done) return;
    const T alpha = (T)scal->alpha, beta = (T)scal->beta;
    for (int64_t i = (int64_t)blockIdx.x * CTA_WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * CTA_WG) {
        const T pv = p[i];
        x[i] = x[i] + alpha * pv;
        p[i] = r[i] + beta * pv;
    }
}

namespace {

template <typename T, int N>
hipError_t brick_T(int mode, const SopGeom& g, const float* coords, int64_t S, const int* perm,
                   const int* cstart, const int* cbrick, int nchunks, const void* X, const void* yin,
                   void* yout, void* tiles, const CgScalars* scal, hipStream_t s) {
    const size_t lds = mode == SOP_FWD ? (size_t)g.tile * sizeof(T)
                     : mode == SOP_ADJ ? (size_t)g.tile * sizeof(double)
                                       : (size_t)g.tile * (sizeof(double) + sizeof(T));
    if (lds > 65536) {
        // the accumulator and coefficient tiles exceed the default 64 KB of dynamic LDS
        hipError_t e = mode == SOP_NRM
            ? hipFuncSetAttribute(reinterpret_cast<const void*>(k_sop_brick<T, N, SOP_NRM>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
            : hipFuncSetAttribute(reinterpret_cast<const void*>(k_sop_brick<T, N, SOP_ADJ>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (mode == SOP_FWD)
        k_sop_brick<T, N, SOP_FWD><<<nchunks, kSopWG, lds, s>>>(g, coords, S, perm, cstart, cbrick,
                                                                (const T*)X, nullptr, (T*)yout, nullptr, scal);
    else if (mode == SOP_ADJ)
        k_sop_brick<T, N, SOP_ADJ><<<nchunks, kSopWG, lds, s>>>(g, coords, S, perm, cstart, cbrick, nullptr,
                                                                (const T*)yin, nullptr, (T*)tiles, scal);
    else
        k_sop_brick<T, N, SOP_NRM><<<nchunks, kSopWG, lds, s>>>(g, coords, S, perm, cstart, cbrick,
                                                                (const T*)X, nullptr, nullptr, (T*)tiles, scal);
    return hipGetLastError();
}

template <typename T>
hipError_t brick_N(int mode, const SopGeom& g, const float* coords, int64_t S, const int* perm,
                   const int* cstart, const int* cbrick, int nchunks, const void* X, const void* yin,
                   void* yout, void* tiles, const CgScalars* scal, hipStream_t s) {
    switch (g.N) {
        case 2: return brick_T<T, 2>(mode, g, coords, S, perm, cstart, cbrick, nchunks, X, yin, yout, tiles, scal, s);
        case 3: return brick_T<T, 3>(mode, g, coords, S, perm, cstart, cbrick, nchunks, X, yin, yout, tiles, scal, s);
        case 4: return brick_T<T, 4>(mode, g, coords, S, perm, cstart, cbrick, nchunks, X, yin, yout, tiles, scal, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t gather_N(const SopGeom& g, const void* tiles, const int* bchunk0, const void* P, const void* rb,
                    double lam, void* Q, double* partials, const CgScalars* scal, int grid, hipStream_t s) {
    const int nbricks = g.nb[0] * (g.N > 1 ? g.nb[1] : 1) * (g.N > 2 ? g.nb[2] : 1) * (g.N > 3 ? g.nb[3] : 1);
    switch (g.N) {
        case 2:
            k_sop_gather<T, 2><<<grid, CTA_WG, 0, s>>>(g, (const T*)tiles, bchunk0, (const T*)P, (const T*)rb,
                                                      (T)lam, (T*)Q, partials, nbricks, scal);
            break;
        case 3:
            k_sop_gather<T, 3><<<grid, CTA_WG, 0, s>>>(g, (const T*)tiles, bchunk0, (const T*)P, (const T*)rb,
                                                      (T)lam, (T*)Q, partials, nbricks, scal);
            break;
        case 4:
            k_sop_gather<T, 4><<<grid, CTA_WG, 0, s>>>(g, (const T*)tiles, bchunk0, (const T*)P, (const T*)rb,
                                                      (T)lam, (T*)Q, partials, nbricks, scal);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sop_brick(int dt, int mode, const SopGeom& g, const float* coords, int64_t S,
                            const int* perm, const int* cstart, const int* cbrick, int nchunks,
                            const void* X, const void* yin, void* yout, void* tiles,
                            const CgScalars* scal, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    static const char* names[2][3] = {{"sop_fwd.f64", "sop_adj.f64", "sop_brick.f64"},
                                      {"sop_fwd.f32", "sop_adj.f32", "sop_brick.f32"}};
    if ((dt != DT_F64 && dt != DT_F32) || mode < 0 || mode > 2) return hipErrorInvalidValue;
    ProfScope ps(names[dt][mode], s);
    return dt == DT_F64 ? brick_N<double>(mode, g, coords, S, perm, cstart, cbrick, nchunks, X, yin, yout, tiles, scal, s)
                        : brick_N<float>(mode, g, coords, S, perm, cstart, cbrick, nchunks, X, yin, yout, tiles, scal, s);
}

hipError_t launch_sop_gather(int dt, const SopGeom& g, const void* tiles, const int* bchunk0, const void* P,
                             const void* rb, double lam, void* Q, double* partials, CgScalars* scal, int post,
                             double* out, hipStream_t s) {
    int64_t nbr = 1;
    for (int k = 0; k < g.N; ++k) nbr *= g.nb[k];
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(nbr, kMaxGrid));
    {
        ProfScope ps(dt == DT_F64 ? "sop_gather.f64" : "sop_gather.f32", s);
        hipError_t e = dt == DT_F64 ? gather_N<double>(g, tiles, bchunk0, P, rb, lam, Q, partials, scal, grid, s)
                     : dt == DT_F32 ? gather_N<float>(g, tiles, bchunk0, P, rb, lam, Q, partials, scal, grid, s)
                                    : hipErrorInvalidValue;
        if (e != hipSuccess) return e;
    }
    if (!partials || post == POST_NONE) return hipSuccess;
    return launch_finalize(partials, grid, scal, post, out, s);
}

hipError_t launch_sop_pstep(int dt, void* x, void* p, const void* r, int64_t n, const CgScalars* scal,
                            hipStream_t s) {
    ProfScope ps(dt == DT_F64 ? "sop_pstep.f64" : "sop_pstep.f32", s);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + CTA_WG * 4 - 1) / (CTA_WG * 4), 65536));
    if (dt == DT_F64)
        k_sop_pstep<double><<<grid, CTA_WG, 0, s>>>((double*)x, (double*)p, (const double*)r, n, scal);
    else if (dt == DT_F32)
        k_sop_pstep<float><<<grid, CTA_WG, 0, s>>>((float*)x, (float*)p, (const float*)r, n, scal);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace cta
