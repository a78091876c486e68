// gfx950 kernels and launchers of the mode-product passes and of the
// normal-operator pass (see ttm.hpp for the tiling).
#include <algorithm>
#include <atomic>
#include <type_traits>

#include "launch.hpp"
#include "prof.hpp"
#include "reduce.hpp"
#include "ttm.hpp"

namespace cta {

template <int DTV> struct DType;
template <> struct DType<DT_F64> { typedef double T; };
template <> struct DType<DT_F32> { typedef float T; };
template <> struct DType<DT_BF16> { typedef bf16 T; };

static int grid_for(int64_t units, int cap) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(units, cap));
}

static int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
    }
    return cus;
}

// Raise the dynamic-LDS limit of a kernel once when it needs more than 64 KiB.
template <typename K>
static hipError_t ensure_lds(K kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// ------------------------------------------------------------------ strided
template <typename Tin, typename Tout, typename Tc, int JT, int WJ, int CT>
__global__ __launch_bounds__(CTA_WG) void k_strided(StridedArgs a, const int* done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    Tc* Xs = reinterpret_cast<Tc*>(smem);
    double unused = 0.0;
    for (int64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x)
        strided_tile<Tin, Tout, Tc, JT, WJ, CT, false>(a, tile, Xs, nullptr, unused);
}

template <typename Tin, typename Tout, typename Tc, int JT, int WJ, int CT>
static hipError_t go_strided(StridedArgs a, const int* done, hipStream_t s) {
    constexpr int TN = 16 * CT * (CTA_WAVES / WJ);
    a.ntt = (a.trail + TN - 1) / TN;
    a.ntiles = a.lead * a.ntt;
    const size_t lds = (size_t)TN * (a.kpad + 16 / sizeof(Tc)) * sizeof(Tc);
    auto kern = k_strided<Tin, Tout, Tc, JT, WJ, CT>;
    hipError_t e = ensure_lds(kern, lds);
    if (e != hipSuccess) return e;
    kern<<<grid_for(a.ntiles, 65536), CTA_WG, lds, s>>>(a, done);
    return hipGetLastError();
}

// Persistent, pipelined strided pass (BF16, K, J <= 128, trail % 64 == 0):
// each wave's factor fragments (its 32 output rows) are loaded into registers
// once per workgroup, and the next 64-column X tile is loaded into registers
// while the current one multiplies from LDS, so the only vector-memory loads
// of a tile are its successor's.  Same sums, in the
// same order, as strided_tile with JT = 2, WJ = 4, CT = 4.
constexpr int SPIPE_TN = 64;
constexpr int SPIPE_LD = 128 + 8;   // LDS pitch (bf16) of the factor rows
constexpr int SPIPE_XLD = 128;      // LDS pitch (bf16) of the X columns
constexpr int SPIPE_YLD = 64 + 8;   // LDS pitch (bf16) of the output rows (over the X tile)
constexpr int SPIPE_XYS = 128 * SPIPE_YLD > SPIPE_TN * SPIPE_XLD ? 128 * SPIPE_YLD : SPIPE_TN * SPIPE_XLD;

// An X tile sits in LDS as [64 columns t][128 K values] (zero past K), with the
// sixteen 16-byte chunks of column t permuted by XOR with xs_swz(t).  A wave's
// transposing stores (one K pair of the 8 columns t = 8 cg + c, fixed c) and
// the fragment reads (16 lanes, 16 consecutive columns, one chunk each) then
// both touch 64 distinct banks.
__device__ __forceinline__ int xs_swz(int t) { return 2 * ((t & 7) ^ (t >> 3)) + ((t >> 3) & 1); }

// Registers of spipe_load -> the swizzled X tile.
__device__ __forceinline__ void xs_store(bf16* Xs, const bf16x8 (&r)[4]) {
    typedef bf16 __attribute__((ext_vector_type(2))) bf16x2;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int u = threadIdx.x + CTA_WG * i;
        const int cg = u & 7, kp = u >> 3;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int t = cg * 8 + c;
            bf16x2 pr;
            pr[0] = r[2 * i][c];
            pr[1] = r[2 * i + 1][c];
            *reinterpret_cast<bf16x2*>(Xs + t * SPIPE_XLD + (((kp >> 2) ^ xs_swz(t)) << 3) + 2 * (kp & 3)) = pr;
        }
    }
}

// The 8 K values [8 chunk, 8 chunk + 8) of column t.
template <typename F>
__device__ __forceinline__ F xs_frag(const bf16* Xs, int t, int chunk) {
    return *reinterpret_cast<const F*>(Xs + t * SPIPE_XLD + ((chunk ^ xs_swz(t)) << 3));
}

__device__ __forceinline__ void spipe_load(const StridedArgs& a, int64_t tile, bf16x8 (&r)[4]) {
    const bf16* __restrict__ X = reinterpret_cast<const bf16*>(a.X);
    const int b = fast_div((int)tile, a.tmul, a.tshift);  // tile / ntt
    const int64_t t0 = (tile - (int64_t)b * a.ntt) * SPIPE_TN;
    const bf16* xb = X + (int64_t)b * a.K * a.trail + t0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int u = threadIdx.x + CTA_WG * i;
        const int cg = u & 7, kp = u >> 3;   // column group of 8, row pair
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = 2 * kp + h;
            bf16x8 v;
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = (bf16)0.f;
            // the input is dead after this pass: non-temporal, so that it leaves
            // the caches before the vectors the next passes read
            if (k < a.K) v = __builtin_nontemporal_load(reinterpret_cast<const bf16x8*>(xb + (int64_t)k * a.trail + cg * 8));
            r[2 * i + h] = v;
        }
    }
}

__global__ __launch_bounds__(CTA_WG) void k_strided_pipe(StridedArgs a, const int* done) {
    if (done && *done) return;
    typedef MT<bf16> T;
    constexpr int JT = 2, CT = 4, VEC = T::VEC;
    extern __shared__ __align__(16) unsigned char smem[];
    bf16* Xs = reinterpret_cast<bf16*>(smem);                  // [64][SPIPE_XLD], swizzled; SPIPE_XYS
    const bf16* __restrict__ M = reinterpret_cast<const bf16*>(a.M);
    const int64_t first = xcd_logical_block(blockIdx.x, gridDim.x), step = gridDim.x;
    bf16x8 r[4];
    if (first < a.ntiles) spipe_load(a, first, r);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, l16 = lane & 15;
    const int jb = wave * JT * 16;
    // this wave's factor fragments (its 32 output rows, zero past J) stay in
    // registers for the workgroup's whole life
    constexpr int NKS = 128 / T::KSTEP;
    const int nks = a.kpad / T::KSTEP;
    typename T::frag mreg[JT][NKS];
#pragma unroll
    for (int x = 0; x < JT; ++x) {
        const int j = jb + x * 16 + l16;
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
            mreg[x][ks] = T::zfrag();
            if (ks < nks && j < a.J)
                mreg[x][ks] = *reinterpret_cast<const typename T::frag*>(M + (int64_t)j * a.ldm + ks * T::KSTEP +
                                                                          VEC * g);
        }
    }
    bf16* __restrict__ Y = reinterpret_cast<bf16*>(a.Y);
    for (int64_t tile = first; tile < a.ntiles; tile += step) {
        xs_store(Xs, r);
        __syncthreads();
        if (tile + step < a.ntiles) spipe_load(a, tile + step, r);
        typename T::acc acc[JT][CT];
#pragma unroll
        for (int x = 0; x < JT; ++x)
#pragma unroll
            for (int y = 0; y < CT; ++y) acc[x][y] = T::zero();
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
            if (ks >= nks) break;
            const int k0 = ks * T::KSTEP + VEC * g;
            typename T::frag xa[CT];
#pragma unroll
            for (int y = 0; y < CT; ++y) xa[y] = xs_frag<typename T::frag>(Xs, y * 16 + l16, k0 >> 3);
#pragma unroll
            for (int x = 0; x < JT; ++x)
#pragma unroll
                for (int y = 0; y < CT; ++y) acc[x][y] = T::mma(xa[y], mreg[x][ks], acc[x][y]);
        }
        const int b = fast_div((int)tile, a.tmul, a.tshift);
        const int64_t t0 = (tile - (int64_t)b * a.ntt) * SPIPE_TN;
        bf16* yb = Y + (int64_t)b * a.J * a.trail + t0;
        // the output tile goes through LDS (over the X tile) so that every row's
        // 128 bytes leave as whole 16-byte pieces, 8 lanes to a row
        __syncthreads();  // every wave has read its X fragments
        bf16* Ys = Xs;    // [128][SPIPE_YLD]
#pragma unroll
        for (int x = 0; x < JT; ++x) {
            const int j = jb + x * 16 + l16;
#pragma unroll
            for (int y = 0; y < CT; ++y) {
                typedef bf16 __attribute__((ext_vector_type(4))) bf16x4;
                bf16x4 o;
#pragma unroll
                for (int q = 0; q < 4; ++q) o[q] = (bf16)acc[x][y][q];
                *reinterpret_cast<bf16x4*>(Ys + j * SPIPE_YLD + y * 16 + 4 * g) = o;
            }
        }
        __syncthreads();
        for (int u = threadIdx.x; u < a.J * 8; u += CTA_WG) {
            const int j = u >> 3, c8 = (u & 7) * 8;
            // the output is read once, by the next pass: non-temporal
            __builtin_nontemporal_store(*reinterpret_cast<const bf16x8*>(Ys + j * SPIPE_YLD + c8),
                                        reinterpret_cast<bf16x8*>(yb + (int64_t)j * a.trail + c8));
        }
        __syncthreads();  // Xs is rewritten by the next tile
    }
}

static hipError_t go_strided_pipe(StridedArgs a, const int* done, hipStream_t s) {
    if (a.kpad > 128 || a.J > 128 || a.trail % SPIPE_TN != 0) return hipErrorNotSupported;
    a.ntt = a.trail / SPIPE_TN;
    a.ntiles = a.lead * a.ntt;
    if (a.ntiles >= ((int64_t)1 << 30)) return hipErrorNotSupported;
    fastdiv_init((uint32_t)a.ntt, &a.tmul, &a.tshift);
    const size_t lds = (size_t)SPIPE_XYS * sizeof(bf16);
    hipError_t e = ensure_lds(k_strided_pipe, lds);
    if (e != hipSuccess) return e;
    // persistent grid: the workgroups per CU that are resident at once
    static std::atomic<int> cached{0};
    int per_cu = cached.load(std::memory_order_relaxed);
    if (per_cu <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_strided_pipe, CTA_WG, lds) != hipSuccess)
            per_cu = 0;
        per_cu = std::max(1, std::min(per_cu, 8));
        cached.store(per_cu, std::memory_order_relaxed);
    }
    int grid = (int)std::min<int64_t>(a.ntiles, (int64_t)device_cus() * per_cu);
    grid = (grid + CTA_XCDS - 1) / CTA_XCDS * CTA_XCDS;
    k_strided_pipe<<<grid, CTA_WG, lds, s>>>(a, done);
    return hipGetLastError();
}

template <typename Tin, typename Tout, typename Tc, int JT, int WJ, int CT>
__global__ __launch_bounds__(CTA_WG) void k_strided_flat(StridedArgs a, const int* done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    Tc* Xs = reinterpret_cast<Tc*>(smem);
    for (int64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x)
        strided_flat_tile<Tin, Tout, Tc, JT, WJ, CT>(a, tile, Xs);
}

template <typename Tin, typename Tout, typename Tc, int JT, int WJ, int CT>
static hipError_t go_strided_flat(StridedArgs a, const int* done, hipStream_t s) {
    constexpr int TN = 16 * CT * (CTA_WAVES / WJ);
    a.ntiles = (a.lead * a.trail + TN - 1) / TN;
    fastdiv_init((uint32_t)a.trail, &a.tmul, &a.tshift);
    const size_t lds = (size_t)TN * (a.kpad + 16 / sizeof(Tc)) * sizeof(Tc);
    auto kern = k_strided_flat<Tin, Tout, Tc, JT, WJ, CT>;
    hipError_t e = ensure_lds(kern, lds);
    if (e != hipSuccess) return e;
    kern<<<grid_for(a.ntiles, 65536), CTA_WG, lds, s>>>(a, done);
    return hipGetLastError();
}

// Flattened columns pay off when the per-b tiles of 64 columns would leave
// more than an eighth of the MFMA columns empty (short or ragged trail).
template <typename Tin, typename Tc>
static bool use_flat(const StridedArgs& a) {
    constexpr int LV = 16 / sizeof(Tin);
    if (a.lead < 2 || a.trail % LV != 0 || (MT<Tc>::CONSEC && a.trail % 4 != 0)) return false;
    if (a.lead * a.trail >= ((int64_t)1 << 31)) return false;
    const int64_t padded = (a.trail + 63) / 64 * 64;
    return (padded - a.trail) * 8 > padded;
}

// variant 0: 64-column tiles; variant 1: 128-column tiles (twice the columns
// per wave); either takes flattened 64-column tiles when use_flat says so
template <typename Tin, typename Tout, typename Tc>
static hipError_t strided_T(StridedArgs a, int variant, const int* done, hipStream_t s) {
    const int jt = (a.J + 15) / 16;
    if constexpr (std::is_same<Tin, bf16>::value && std::is_same<Tout, bf16>::value &&
                  std::is_same<Tc, bf16>::value) {
        // variant 2: persistent pipelined pass where its shape allows, else as 1
        if (variant == 2) {
            const hipError_t e = go_strided_pipe(a, done, s);
            if (e != hipErrorNotSupported) return e;
        }
    }
    if (variant == 2) variant = 1;
    if (use_flat<Tin, Tc>(a)) {
        if (jt <= 1) return go_strided_flat<Tin, Tout, Tc, 1, 1, 1>(a, done, s);
        if (jt <= 2) return go_strided_flat<Tin, Tout, Tc, 1, 2, 2>(a, done, s);
        if (jt <= 4) return go_strided_flat<Tin, Tout, Tc, 1, 4, 4>(a, done, s);
        if (jt <= 6) return go_strided_flat<Tin, Tout, Tc, 3, 2, 2>(a, done, s);
        if (jt <= 8) return go_strided_flat<Tin, Tout, Tc, 2, 4, 4>(a, done, s);
        if (jt <= 12) return go_strided_flat<Tin, Tout, Tc, 3, 4, 4>(a, done, s);
        if (jt <= 16) return go_strided_flat<Tin, Tout, Tc, 4, 4, 4>(a, done, s);
        return hipErrorInvalidValue;
    }
    if (variant == 1) {
        if (jt <= 1) return go_strided<Tin, Tout, Tc, 1, 1, 2>(a, done, s);
        if (jt <= 2) return go_strided<Tin, Tout, Tc, 1, 2, 4>(a, done, s);
        if (jt <= 4) return go_strided<Tin, Tout, Tc, 1, 4, 8>(a, done, s);
        if (jt <= 6) return go_strided<Tin, Tout, Tc, 3, 2, 4>(a, done, s);
        if (jt <= 8) return go_strided<Tin, Tout, Tc, 2, 4, 8>(a, done, s);
    }
    if (jt <= 1) return go_strided<Tin, Tout, Tc, 1, 1, 1>(a, done, s);
    if (jt <= 2) return go_strided<Tin, Tout, Tc, 1, 2, 2>(a, done, s);
    if (jt <= 4) return go_strided<Tin, Tout, Tc, 1, 4, 4>(a, done, s);
    if (jt <= 6) return go_strided<Tin, Tout, Tc, 3, 2, 2>(a, done, s);
    if (jt <= 8) return go_strided<Tin, Tout, Tc, 2, 4, 4>(a, done, s);
    if (jt <= 12) return go_strided<Tin, Tout, Tc, 3, 4, 4>(a, done, s);
    if (jt <= 16) return go_strided<Tin, Tout, Tc, 4, 4, 4>(a, done, s);
    return hipErrorInvalidValue;
}

hipError_t launch_strided(int tc, const void* X, void* Y, const Mat& M, int64_t lead, int K, int J,
                          int64_t trail, const int* done, hipStream_t s, int variant) {
    StridedArgs a{};
    a.X = X; a.Y = Y; a.M = M.p; a.ldm = M.ld;
    a.K = K; a.J = J; a.kpad = (K + dt_kstep(tc) - 1) / dt_kstep(tc) * dt_kstep(tc);
    a.lead = lead; a.trail = trail;
    if (a.kpad > M.ld) return hipErrorInvalidValue;
    ProfScope ps(tc == DT_F64 ? "strided.f64" : tc == DT_F32 ? "strided.f32" : "strided.bf16", s);
    switch (tc) {
        case DT_F64: return strided_T<double, double, double>(a, variant, done, s);
        case DT_F32: return strided_T<float, float, float>(a, variant, done, s);
        case DT_BF16: return strided_T<bf16, bf16, bf16>(a, variant, done, s);
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ normal-operator last pass
// Windowed epilogue (normal_last_tile) when its LDS fits, otherwise the
// epilogue that reads every stencil point from memory (strided_tile<EPI>).
template <typename Tmid, typename Tvec, typename Tc, int JT, int WJ, int CT, bool WINDOW>
__global__ __launch_bounds__(CTA_WG) void k_normal_last(StridedArgs a, StencilArgs<Tvec> st,
                                                        const int* done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[4];
    double dot = 0.0;
    const int64_t lb = xcd_logical_block(blockIdx.x, gridDim.x);
    for (int64_t tile = lb; tile < a.ntiles; tile += gridDim.x) {
        if constexpr (WINDOW)
            normal_last_tile<Tmid, Tvec, Tc, JT, WJ, CT>(a, tile, smem, st, dot);
        else
            strided_tile<Tmid, Tvec, Tc, JT, WJ, CT, true>(a, tile, reinterpret_cast<Tc*>(smem), &st, dot);
    }
    block_partial(dot, st.partials, red);
}

template <typename Tmid, typename Tvec, typename Tc, int JT, int WJ, int CT>
static hipError_t go_last(StridedArgs a, const StencilArgs<Tvec>& st, int* grid_out,
                          const int* done, hipStream_t s) {
    constexpr int TN = 16 * CT * (CTA_WAVES / WJ);
    a.ntt = (a.trail + TN - 1) / TN;
    a.ntiles = a.lead * a.ntt;
    if (a.pgroup > 0 && a.plane % TN != 0) a.pgroup = 0;
    const size_t xs = (size_t)TN * (a.kpad + 16 / sizeof(Tc)) * sizeof(Tc);
    const int nN = (int)st.ext[st.order - 1];
    const size_t win = normal_last_lds<Tvec, Tc, TN>(a.kpad, a.K, a.J, nN);
    const bool window = win <= 160 * 1024 && a.trail < (int64_t(1) << 30);
    // a multiple of the XCD count, for the XCD-aware tile order
    const int grid = (grid_for(a.ntiles, kMaxGrid) + CTA_XCDS - 1) / CTA_XCDS * CTA_XCDS;
    *grid_out = grid;
    hipError_t e;
    if (window) {
        auto kern = k_normal_last<Tmid, Tvec, Tc, JT, WJ, CT, true>;
        e = ensure_lds(kern, win);
        if (e != hipSuccess) return e;
        kern<<<grid, CTA_WG, win, s>>>(a, st, done);
    } else {
        auto kern = k_normal_last<Tmid, Tvec, Tc, JT, WJ, CT, false>;
        e = ensure_lds(kern, xs);
        if (e != hipSuccess) return e;
        kern<<<grid, CTA_WG, xs, s>>>(a, st, done);
    }
    return hipGetLastError();
}

// Pipelined persistent last pass (normal_last_pipe): BF16 chain, FP32 vectors,
// 96 < K <= 128.
// three workgroups per CU (the LDS budget) need at most 168 registers per lane
__global__ __launch_bounds__(CTA_WG) __attribute__((amdgpu_waves_per_eu(3))) void k_normal_last_pipe(StridedArgs a, StencilArgs<float> st,
                                                             const int* done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[4];
    double dot = 0.0;
    normal_last_pipe(a, smem, st, dot, xcd_logical_block(blockIdx.x, gridDim.x), gridDim.x);
    block_partial(dot, st.partials, red);
}


// Variant 6: the pipelined pass with fewer LDS and vector instructions per
// item (normal_last_pipe6); LDS: 4 more window rows and 3 more floats per
// mode-1 band row.
// Tile range of a persistent last-pass workgroup (see StridedArgs::xsweep).
__device__ __forceinline__ void last_tile_range(const StridedArgs& a, int64_t& first, int64_t& step,
                                                int64_t& end) {
    first = xcd_logical_block(blockIdx.x, gridDim.x);
    step = gridDim.x;
    end = a.ntiles;
    if (a.xsweep) {
        const int64_t per = (a.ntiles + CTA_XCDS - 1) / CTA_XCDS, x = blockIdx.x % CTA_XCDS;
        step = gridDim.x / CTA_XCDS;
        first = x * per + blockIdx.x / CTA_XCDS;
        end = min((x + 1) * per, a.ntiles);
    }
}

__global__ __launch_bounds__(CTA_WG) __attribute__((amdgpu_waves_per_eu(3))) void k_normal_last_pipe6(
    StridedArgs a, StencilArgs<float> st, const int* done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[4];
    double dot = 0.0;
    int64_t first, step, end;
    last_tile_range(a, first, step, end);
    normal_last_pipe6<CTA_WG>(a, smem, st, dot, first, step, end);
    block_partial(dot, st.partials, red);
}

// Variant 7: variant 6 with 512 threads (8 waves) per workgroup, two
// workgroups per CU.
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_normal_last_pipe7(
    StridedArgs a, StencilArgs<float> st, const int* done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[8];
    double dot = 0.0;
    int64_t first, step, end;
    last_tile_range(a, first, step, end);
    normal_last_pipe6<512>(a, smem, st, dot, first, step, end);
    const double s = block_sum_w<8>(dot, red);
    if (threadIdx.x == 0) st.partials[blockIdx.x] = s;
}

// Variant 8 (normal_last_ring): one workgroup of NT threads per CU, gathers GD
// tiles ahead, WPE waves per SIMD.
template <int NT, int GD, int WPE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE))) void k_normal_last_ring(
    StridedArgs a, StencilArgs<float> st, RingGeom rg, const int* done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[NT / 64];
    double dot = 0.0;
    normal_last_ring<NT, GD>(a, smem, st, rg, dot);
    dot = wave_sum(dot);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dot;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += red[w];
        st.partials[blockIdx.x] = s;
    }
}

// Variant 8 when the shape allows it (order 4, K = J <= 128, n_N % 4 == 0 and
// n_N <= 24, planes of the second mode a multiple of 32 columns, P below 4 GiB);
// hipErrorNotSupported otherwise.
static hipError_t go_last_ring(StridedArgs a, const StencilArgs<float>& st, int* grid_out, const int* done,
                               hipStream_t s) {
    if (st.order != 4 || a.kpad != 128 || a.K != a.J || a.K < 1) return hipErrorNotSupported;
    const int nN = (int)st.ext[3], n3 = (int)st.ext[2], n2 = (int)st.ext[1];
    const int64_t plane = st.stride[1];
    if (nN % 4 != 0 || nN > 24 || plane % RING_TN != 0 || plane < RING_TN || n2 * plane != a.trail ||
        a.trail >= (int64_t(1) << 30) || (uint64_t)a.K * (uint64_t)a.trail * sizeof(float) >= (uint64_t(1) << 32))
        return hipErrorNotSupported;
    const size_t lds = ring_lds_bytes(a.K, n3, nN);
    if (lds > 160 * 1024) return hipErrorNotSupported;
    RingGeom rg;
    rg.nplane = n2;
    rg.plane = (int)plane;
    rg.cpp = (int)(plane / RING_TN);
    const int cus = device_cus();
    rg.nseg = std::max(1, std::min(rg.cpp, (cus + n2 - 1) / n2));
    rg.seg_len = (rg.cpp + rg.nseg - 1) / rg.nseg;
    int grid = n2 * rg.nseg;
    grid = (grid + CTA_XCDS - 1) / CTA_XCDS * CTA_XCDS;
    if (grid > kMaxGrid) return hipErrorNotSupported;   // one partial per workgroup
    hipError_t e = ensure_lds(k_normal_last_ring<RING_NT, 1, 4>, lds);
    if (e != hipSuccess) return e;
    *grid_out = grid;
    k_normal_last_ring<RING_NT, 1, 4><<<grid, RING_NT, lds, s>>>(a, st, rg, done);
    return hipGetLastError();
}

// variant: 5 (k_normal_last_pipe), 6 (k_normal_last_pipe6) or 7 (k_normal_last_pipe7)
static hipError_t go_last_pipe(StridedArgs a, const StencilArgs<float>& st, int* grid_out, const int* done,
                               hipStream_t s, int variant) {
    const int N = st.order;
    const int nN = (int)st.ext[N - 1];
    if (a.kpad != 128 || a.K != a.J || a.trail % PIPE_TN != 0 || nN % 4 != 0 ||
        a.trail / PIPE_TN >= (int64_t(1) << 22) ||   // tile columns from float reciprocals
        (uint64_t)a.K * (uint64_t)a.trail * sizeof(float) >= (uint64_t(1) << 32))   // 32-bit offsets into P
        return hipErrorNotSupported;
    const bool colaff = variant >= 6;
    a.ntt = a.trail / PIPE_TN;
    a.ntiles = a.ntt;
    a.pgroup = 0;
    const int64_t plane = N >= 3 ? st.stride[1] : 0;
    const int nplane = N >= 3 ? (int)st.ext[1] : 0;
    if (plane > 0 && plane % PIPE_TN == 0 && nplane % 8 == 0 && plane * nplane == a.trail) {
        a.plane = plane;
        a.nplane = nplane;
        // variants 6 and 7 walk groups of 16 planes inside per-XCD tile ranges
        a.pgroup = colaff && nplane % 16 == 0 ? 16 : 8;
    }
    a.xsweep = colaff ? 1 : 0;
    const size_t xq = std::max<size_t>((size_t)PIPE_TN * (128 + 8) * 2, (size_t)128 * (PIPE_TN + 4) * 4);
    const size_t lds = colaff ? (xq + 15) / 16 * 16 + (size_t)(128 + 4) * PIPE_LDP * 4 + (size_t)128 * 8 * 4 +
                                    (size_t)nN * 5 * 4
                              : (xq + 15) / 16 * 16 + (size_t)128 * PIPE_LDP * 4 + (size_t)(128 + nN) * 5 * 4;
    if (lds > 64 * 1024) return hipErrorNotSupported;
    // persistent grid: three workgroups of 256 threads (two of 512) per CU, a
    // multiple of the XCD count
    const int per_cu = variant == 7 ? 2 : 3;
    int grid = (int)std::min<int64_t>(a.ntiles, (int64_t)device_cus() * per_cu);
    grid = (grid + CTA_XCDS - 1) / CTA_XCDS * CTA_XCDS;
    *grid_out = grid;
    if (variant == 7) {
        hipError_t e = ensure_lds(k_normal_last_pipe7, lds);
        if (e != hipSuccess) return e;
        k_normal_last_pipe7<<<grid, 512, lds, s>>>(a, st, done);
        return hipGetLastError();
    }
    if (variant == 6) {
        hipError_t e = ensure_lds(k_normal_last_pipe6, lds);
        if (e != hipSuccess) return e;
        k_normal_last_pipe6<<<grid, CTA_WG, lds, s>>>(a, st, done);
        return hipGetLastError();
    }
    hipError_t e = ensure_lds(k_normal_last_pipe, lds);
    if (e != hipSuccess) return e;
    k_normal_last_pipe<<<grid, CTA_WG, lds, s>>>(a, st, done);
    return hipGetLastError();
}

// Row-block last pass (normal_last_jtile): FP32 vectors, tensor order 3 or 4.
template <typename Tmid, typename Tc, int NF>
__global__ __launch_bounds__(CTA_WG) void k_normal_last_js(StridedArgs a, StencilArgs<float> st, JsGeom gm,
                                                           const int* done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[4];
    double dot = 0.0;
    const int64_t lb = xcd_logical_block(blockIdx.x, gridDim.x);
    for (int64_t tile = lb; tile < a.ntiles; tile += gridDim.x)
        normal_last_jtile<Tmid, Tc, NF>(a, tile, smem, st, gm, dot);
    block_partial(dot, st.partials, red);
}

// Variant 4 applies when the shape allows it (see normal_last_jtile); returns
// hipErrorNotSupported otherwise, and the caller falls back to variant 2.
template <typename Tmid, typename Tc>
static hipError_t go_last_js(StridedArgs a, const StencilArgs<float>& st, int* grid_out, const int* done,
                             hipStream_t s) {
    const int N = st.order;
    if (N != 3 && N != 4) return hipErrorNotSupported;
    const int nN = (int)st.ext[N - 1], nM = (int)st.ext[N - 2];
    const int64_t sM = st.stride[N - 2];
    constexpr int LV = 16 / sizeof(Tmid);
    if (nN % 4 != 0 || sM != nN || a.trail % JS_TN != 0 || a.trail % LV != 0 || a.trail >= (int64_t(1) << 30) ||
        (int64_t)a.K * a.trail >= (int64_t(1) << 31) || a.K > 256)
        return hipErrorNotSupported;
    JsGeom gm{};
    gm.nN = nN;
    gm.nM = nM;
    gm.sM = (int)sM;
    gm.H = 2 * nN;
    gm.LDW = JS_TN + 2 * gm.H;
    if (N == 4) {
        gm.nF = (int)st.ext[1];
        gm.sF = st.stride[1];
        if (gm.sF % JS_TN != 0) return hipErrorNotSupported;
    }
    const int NF = N == 4 ? 1 : 0;
    const size_t lds = js_lds_bytes<Tc>(a.kpad, gm.H, NF, nN, nM);
    if (lds > 64 * 1024) return hipErrorNotSupported;
    // tile order: the row blocks of a column tile first, column tiles plane-grouped
    const int njb = (a.K + JS_JB - 1) / JS_JB;
    a.ntt = a.trail / JS_TN;
    a.ntiles = a.ntt * njb;
    a.pgroup = 0;
    if (N == 4 && gm.nF % 8 == 0) {
        a.plane = gm.sF;
        a.nplane = gm.nF;
        a.pgroup = 8;
    }
    a.xsweep = 0;
    const int grid = (grid_for(a.ntiles, kMaxGrid) + CTA_XCDS - 1) / CTA_XCDS * CTA_XCDS;
    *grid_out = grid;
    hipError_t e;
    if (NF) {
        auto kern = k_normal_last_js<Tmid, Tc, 1>;
        e = ensure_lds(kern, lds);
        if (e != hipSuccess) return e;
        kern<<<grid, CTA_WG, lds, s>>>(a, st, gm, done);
    } else {
        auto kern = k_normal_last_js<Tmid, Tc, 0>;
        e = ensure_lds(kern, lds);
        if (e != hipSuccess) return e;
        kern<<<grid, CTA_WG, lds, s>>>(a, st, gm, done);
    }
    return hipGetLastError();
}

template <typename Tmid, typename Tvec, typename Tc>
static hipError_t last_T(StridedArgs a, const StencilDesc& d, double* partials, int* grid,
                         const int* done, hipStream_t s, int variant) {
    StencilArgs<Tvec> st{};
    st.P = reinterpret_cast<const Tvec*>(d.P);
    for (int k = 0; k < 8; ++k) {
        st.rband[k] = reinterpret_cast<const Tvec*>(d.rband[k]);
        st.ext[k] = d.ext[k];
        st.stride[k] = d.stride[k];
    }
    st.order = d.order;
    st.lam = d.lam;
    st.partials = partials;
    for (int k = 0; k < 8; ++k) {
        fastdiv_init((uint32_t)std::max<int64_t>(1, std::min<int64_t>(d.stride[k], INT32_MAX)), &st.smul[k],
                     &st.sshift[k]);
        fastdiv_init((uint32_t)std::max<int64_t>(1, std::min<int64_t>(d.ext[k], INT32_MAX)), &st.emul[k],
                     &st.eshift[k]);
    }
    const int jt = (a.J + 15) / 16;
    // variant 4: row blocks with the whole stencil staged in LDS (FP32
    // vectors, order 3 or 4); falls back to variant 2 when the shape does not
    // allow it
    if (variant == 4) {
        if constexpr (sizeof(Tvec) == 4) {
            const hipError_t e = go_last_js<Tmid, Tc>(a, st, grid, done, s);
            if (e != hipErrorNotSupported) return e;
        }
        variant = 2;
    }
    // variants 5, 6 and 7: persistent and pipelined (BF16 chains, 96 < K <= 128);
    // 6 and 7 with vector band reads and per-XCD tile ranges, 7 with 512 threads;
    // 8: one workgroup per CU sweeping a plane with P in an LDS ring
    if (variant == 8) {
        if constexpr (sizeof(Tvec) == 4 && sizeof(Tc) == 2) {
            const hipError_t e = go_last_ring(a, st, grid, done, s);
            if (e != hipErrorNotSupported) return e;
        }
        variant = 6;
    }
    if (variant >= 5 && variant <= 7) {
        if constexpr (sizeof(Tvec) == 4 && sizeof(Tc) == 2) {
            const hipError_t e = go_last_pipe(a, st, grid, done, s, variant);
            if (e != hipErrorNotSupported) return e;
        }
        variant = 2;
    }
    // variants 2 and 3: 32-column tiles walked plane-fastest (groups of 8
    // planes, or all planes) along the second mode; fall back to variant 1
    // when the shape does not allow it
    a.pgroup = 0;
    if (variant >= 2) {
        const int64_t plane = d.order >= 3 ? d.stride[1] : 0;
        const int nplane = d.order >= 3 ? (int)d.ext[1] : 0;
        const int g = variant == 2 ? 8 : nplane;
        if (plane > 0 && plane % 32 == 0 && g > 0 && nplane % g == 0 && plane * nplane == a.trail) {
            a.plane = plane;
            a.nplane = nplane;
            a.pgroup = g;
        }
        variant = 1;
    }
    if (variant == 1) {  // 32-column tiles: less LDS per workgroup, more workgroups per CU
        if (jt <= 2) return go_last<Tmid, Tvec, Tc, 1, 2, 1>(a, st, grid, done, s);
        if (jt <= 4) return go_last<Tmid, Tvec, Tc, 1, 4, 2>(a, st, grid, done, s);
        if (jt <= 6) return go_last<Tmid, Tvec, Tc, 3, 2, 1>(a, st, grid, done, s);
        if (jt <= 8) return go_last<Tmid, Tvec, Tc, 2, 4, 2>(a, st, grid, done, s);
    }
    if (jt <= 1) return go_last<Tmid, Tvec, Tc, 1, 1, 1>(a, st, grid, done, s);
    if (jt <= 2) return go_last<Tmid, Tvec, Tc, 1, 2, 2>(a, st, grid, done, s);
    if (jt <= 4) return go_last<Tmid, Tvec, Tc, 1, 4, 4>(a, st, grid, done, s);
    if (jt <= 6) return go_last<Tmid, Tvec, Tc, 3, 2, 2>(a, st, grid, done, s);
    if (jt <= 8) return go_last<Tmid, Tvec, Tc, 2, 4, 4>(a, st, grid, done, s);
    if (jt <= 12) return go_last<Tmid, Tvec, Tc, 3, 4, 4>(a, st, grid, done, s);
    if (jt <= 16) return go_last<Tmid, Tvec, Tc, 4, 4, 4>(a, st, grid, done, s);
    return hipErrorInvalidValue;
}

// Last pass without a regulariser (the preconditioner's mode-1 pass, BF16
// chain): Z = T x_1 M in FP32 and the FP64 partials of <R, Z>.  Persistent
// like k_strided_pipe (M in LDS, the next 64-column tile prefetched into
// registers); the R values a tile needs are loaded before that prefetch, so
// their wait does not include it.
__global__ __launch_bounds__(CTA_WG) void k_last_nr_pipe(StridedArgs a, const float* __restrict__ R,
                                                         double* partials, const int* done) {
    if (done && *done) return;
    typedef MT<bf16> T;
    constexpr int JT = 2, CT = 4, VEC = T::VEC;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[CTA_WAVES];
    bf16* Ms = reinterpret_cast<bf16*>(smem);
    bf16* Xs = Ms + 128 * SPIPE_LD;
    const bf16* __restrict__ M = reinterpret_cast<const bf16*>(a.M);
    const int64_t first = xcd_logical_block(blockIdx.x, gridDim.x), step = gridDim.x;
    bf16x8 r[4];
    if (first < a.ntiles) spipe_load(a, first, r);   // in flight while the factor is staged
    for (int u = threadIdx.x; u < 128 * 16; u += CTA_WG) {
        const int j = u >> 4, c8 = (u & 15) * 8;
        bf16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (bf16)0.f;
        if (j < a.J && c8 < a.kpad) v = *reinterpret_cast<const bf16x8*>(M + (int64_t)j * a.ldm + c8);
        *reinterpret_cast<bf16x8*>(Ms + j * SPIPE_LD + c8) = v;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, l16 = lane & 15;
    const int jb = wave * JT * 16;
    float* __restrict__ Z = reinterpret_cast<float*>(a.Y);
    double dot = 0.0;
    for (int64_t tile = first; tile < a.ntiles; tile += step) {
        xs_store(Xs, r);
        __syncthreads();
        // R of this tile's outputs (rows past J read row J-1 and are not used)
        const int64_t t0 = tile * SPIPE_TN;
        floatx4 rv[JT][CT];
#pragma unroll
        for (int x = 0; x < JT; ++x)
#pragma unroll
            for (int y = 0; y < CT; ++y) {
                const int j = min(jb + x * 16 + l16, a.J - 1);
                // r is next read one iteration later: non-temporal
                rv[x][y] = __builtin_nontemporal_load(
                    reinterpret_cast<const floatx4*>(R + (int64_t)j * a.trail + t0 + y * 16 + 4 * g));
            }
        if (tile + step < a.ntiles) spipe_load(a, tile + step, r);
        typename T::acc acc[JT][CT];
#pragma unroll
        for (int x = 0; x < JT; ++x)
#pragma unroll
            for (int y = 0; y < CT; ++y) acc[x][y] = T::zero();
        const int nks = a.kpad / T::KSTEP;
        for (int ks = 0; ks < nks; ++ks) {
            const int k0 = ks * T::KSTEP + VEC * g;
            typename T::frag xa[CT], mb[JT];
#pragma unroll
            for (int y = 0; y < CT; ++y) xa[y] = xs_frag<typename T::frag>(Xs, y * 16 + l16, k0 >> 3);
#pragma unroll
            for (int x = 0; x < JT; ++x)
                mb[x] = *reinterpret_cast<const typename T::frag*>(Ms + (jb + x * 16 + l16) * SPIPE_LD + k0);
#pragma unroll
            for (int x = 0; x < JT; ++x)
#pragma unroll
                for (int y = 0; y < CT; ++y) acc[x][y] = T::mma(xa[y], mb[x], acc[x][y]);
        }
#pragma unroll
        for (int x = 0; x < JT; ++x) {
            const int j = jb + x * 16 + l16;
            if (j >= a.J) continue;
#pragma unroll
            for (int y = 0; y < CT; ++y) {
                *reinterpret_cast<floatx4*>(Z + (int64_t)j * a.trail + t0 + y * 16 + 4 * g) = acc[x][y];
#pragma unroll
                for (int q = 0; q < 4; ++q) dot += (double)rv[x][y][q] * (double)acc[x][y][q];
            }
        }
        __syncthreads();  // Xs is rewritten by the next tile
    }
    block_partial(dot, partials, red);
}

// The preconditioner's last pass in the pipelined form when the shape allows
// (BF16 chain, n_1 <= 128, trail % 64 == 0); hipErrorNotSupported otherwise.
hipError_t launch_last_nr(const void* X, void* Z, const void* R, const Mat& M, int K, int64_t trail,
                          double* partials, CgScalars* scal, int post, double* dot_out, const int* done,
                          hipStream_t s) {
    StridedArgs a{};
    a.X = X; a.Y = Z; a.M = M.p; a.ldm = M.ld;
    a.K = K; a.J = K; a.kpad = (K + dt_kstep(DT_BF16) - 1) / dt_kstep(DT_BF16) * dt_kstep(DT_BF16);
    a.lead = 1; a.trail = trail;
    if (a.kpad > 128 || a.kpad > M.ld || trail % SPIPE_TN != 0) return hipErrorNotSupported;
    a.ntt = trail / SPIPE_TN;
    a.ntiles = a.ntt;
    if (a.ntiles >= ((int64_t)1 << 30)) return hipErrorNotSupported;
    fastdiv_init((uint32_t)a.ntt, &a.tmul, &a.tshift);   // spipe_load: tile / ntt (= 0 here)
    const size_t lds = ((size_t)128 * SPIPE_LD + (size_t)SPIPE_TN * SPIPE_XLD) * sizeof(bf16);
    hipError_t e = ensure_lds(k_last_nr_pipe, lds);
    if (e != hipSuccess) return e;
    int grid = (int)std::min<int64_t>(a.ntiles, (int64_t)device_cus() * 3);
    grid = (grid + CTA_XCDS - 1) / CTA_XCDS * CTA_XCDS;
    {
        ProfScope ps("normal_last_nr.bf16", s);
        k_last_nr_pipe<<<grid, CTA_WG, lds, s>>>(a, reinterpret_cast<const float*>(R), partials, done);
        e = hipGetLastError();
    }
    if (e != hipSuccess || post == POST_NONE) return e;
    return launch_finalize(partials, grid, scal, post, dot_out, s);
}

hipError_t launch_normal_last(int tmid, int tvec, int tc, const void* X, void* Q, const Mat& M,
                              int K, int J, int64_t trail, const StencilDesc& st,
                              double* partials, CgScalars* scal, int post, double* dot_out,
                              const int* done, hipStream_t s, int variant) {
    StridedArgs a{};
    a.X = X; a.Y = Q; a.M = M.p; a.ldm = M.ld;
    a.K = K; a.J = J; a.kpad = (K + dt_kstep(tc) - 1) / dt_kstep(tc) * dt_kstep(tc);
    a.lead = 1; a.trail = trail;
    if (a.kpad > M.ld || K != J) return hipErrorInvalidValue;
    int grid = 0;
    hipError_t e = hipErrorInvalidValue;
    {
        ProfScope ps(tc == DT_F64 ? "normal_last.f64" : tc == DT_F32 ? "normal_last.f32" : "normal_last.bf16", s);
        if (tmid == DT_BF16 && tvec == DT_F32 && tc == DT_BF16)
            e = last_T<bf16, float, bf16>(a, st, partials, &grid, done, s, variant);
        else if (tmid == DT_F32 && tvec == DT_F32 && tc == DT_F32)
            e = last_T<float, float, float>(a, st, partials, &grid, done, s, variant);
        else if (tmid == DT_F64 && tvec == DT_F64 && tc == DT_F64)
            e = last_T<double, double, double>(a, st, partials, &grid, done, s, variant);
    }
    if (e != hipSuccess || post == POST_NONE) return e;
    return launch_finalize(partials, grid, scal, post, dot_out, s);
}

// ------------------------------------------------------------------ tail
template <typename Tin, typename Tout, typename Tc, int J2T, bool FUSE_P>
__global__ __launch_bounds__(CTA_WG) void k_tail(TailArgs a) {
    if (a.done && *a.done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t ngroups = (a.nblk + a.nbg - 1) / a.nbg;
    for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
        const int64_t blk0 = grp * a.nbg;
        const int nb = (int)std::min<int64_t>(a.nbg, a.nblk - blk0);
        tail_group<Tin, Tout, Tc, J2T, FUSE_P>(a, blk0, nb, a.nbg, smem);
    }
}

// K1 is padded to the MFMA K step and to the 16-row tiles of the first step.
static int tail_k1pad(int tc, int K1) {
    const int g = std::max(dt_kstep(tc), 16);
    return (K1 + g - 1) / g * g;
}

static size_t tail_lds_nb(int tc, int tout, int K1, int J1, int J2, int nb) {
    const size_t z = (size_t)nb * tail_zt_elems(tail_k1pad(tc, K1), J2, dt_size(tc)) * dt_size(tc);
    return (z + 15) / 16 * 16 + (size_t)nb * J1 * J2 * dt_size(tout);
}

// Blocks per group: enough 16-row tiles to keep the four waves equally busy,
// within a 64 KiB LDS budget.
static int tail_nb(int tc, int tout, int K1, int J1, int J2) {
    const int ni1t = tail_k1pad(tc, K1) / 16;
    int nb = (ni1t % 4 == 0) ? 1 : (ni1t % 2 == 0 ? 2 : 4);
    while (nb > 1 && tail_lds_nb(tc, tout, K1, J1, J2, nb) > 64 * 1024) nb /= 2;
    return nb;
}

bool tail_fits(int tc, int K1, int J2) {
    // the output staging uses the widest output type of any caller (8 bytes)
    return J2 <= 256 && K1 <= 256 && tail_lds_nb(tc, DT_F64, K1, K1, J2, 1) <= 160 * 1024;
}

template <typename Tin, typename Tout, typename Tc, bool FUSE_P>
static hipError_t tail_T(const TailArgs& a, size_t lds, hipStream_t s) {
    const int j2t = (a.J2 + 15) / 16;
    const int64_t ngroups = (a.nblk + a.nbg - 1) / a.nbg;
    const int grid = grid_for(ngroups, 65536);
#define CTA_TAIL_GO(N)                                                          \
    {                                                                           \
        auto kern = k_tail<Tin, Tout, Tc, N, FUSE_P>;                           \
        hipError_t e = ensure_lds(kern, lds);                                   \
        if (e != hipSuccess) return e;                                          \
        kern<<<grid, CTA_WG, lds, s>>>(a);                                      \
        return hipGetLastError();                                               \
    }
    if (j2t <= 2) CTA_TAIL_GO(2)
    if (j2t <= 4) CTA_TAIL_GO(4)
    if (j2t <= 8) CTA_TAIL_GO(8)
    if (j2t <= 16) CTA_TAIL_GO(16)
#undef CTA_TAIL_GO
    return hipErrorInvalidValue;
}

// Persistent, pipelined fused tail pass (BF16 chain, x and p updates fused):
// M1 and M2 are staged in LDS once per workgroup, and the r, p (and x)
// fragments of the workgroup's next group of blocks are loaded into registers
// right after the current group's new values are stored, so they arrive while
// the second MFMA step and the write-back run (which touch only LDS and
// store).  Every lane loads every slot, at a clamped address where the slot is
// unused, so that no register keeps an old value across the load and nothing
// waits for the loads before the next group.  Same sums, in the same order,
// as tail_group.  Shapes: k1pad and
// J1 <= 128, K2 <= 32 with K2 % 8 == 0, J2 <= 32, at most TPIPE_TPW 16-row
// tiles per wave per group.
constexpr int TPIPE_TPW = 3;

struct TailPipeGeom {
    int ld1, ld2, ldz, zsz, nj1t, nj2t, ni1t, bout;
};

__host__ __device__ inline TailPipeGeom tail_pipe_geom(int k1pad, int J1, int J2) {
    TailPipeGeom g;
    g.ld1 = k1pad + 8;
    g.ld2 = 32 + 8;
    g.ldz = k1pad + 8;
    g.nj1t = (J1 + 15) / 16;
    g.nj2t = (J2 + 15) / 16;
    g.ni1t = k1pad / 16;
    g.zsz = g.nj2t * 16 * g.ldz;
    g.bout = J1 * J2;
    return g;
}

static size_t tail_pipe_lds(const TailPipeGeom& g, int nbg) {
    return ((size_t)g.nj1t * 16 * g.ld1 + (size_t)g.nj2t * 16 * g.ld2 + (size_t)nbg * g.zsz +
            (size_t)nbg * g.bout) * sizeof(bf16);
}

// FR: the preconditioner's form, r = r - alpha q (R = Pvec, q = Qvec) with the
// FP64 partials of <r, r>, instead of the x and p updates.
template <bool FR>
__global__ __launch_bounds__(CTA_WG) void k_tail_pipe(TailArgs a) {
    if (a.done && *a.done) return;
    typedef MT<bf16> T;
    constexpr int VEC = T::VEC;
    constexpr int J2T = 2;
    typedef float __attribute__((ext_vector_type(4))) f4;
    extern __shared__ __align__(16) unsigned char smem[];
    const TailPipeGeom gm = tail_pipe_geom(a.k1pad, a.J1, a.J2);
    bf16* M1s = reinterpret_cast<bf16*>(smem);
    bf16* M2s = M1s + gm.nj1t * 16 * gm.ld1;
    bf16* Zt = M2s + gm.nj2t * 16 * gm.ld2;
    bf16* Ys = Zt + a.nbg * gm.zsz;
    const bf16* __restrict__ M1 = reinterpret_cast<const bf16*>(a.M1);
    const bf16* __restrict__ M2 = reinterpret_cast<const bf16*>(a.M2);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, l16 = lane & 15;
    const int64_t bin = (int64_t)a.K1 * a.K2;
    const float beta = FR ? 0.f : (float)*a.beta;
    const float alpha = (FR || a.Xsol) ? (float)*a.alpha : 0.f;
    // FR: rr = r (read from and written to Pvec), pp = q
    const float* __restrict__ R = reinterpret_cast<const float*>(FR ? a.Pvec : a.X);
    float* __restrict__ Pg = reinterpret_cast<float*>(FR ? const_cast<void*>(a.Qvec) : a.Pvec);
    float* __restrict__ Xg = FR ? nullptr : reinterpret_cast<float*>(a.Xsol);
    float* __restrict__ Rw = reinterpret_cast<float*>(a.Pvec);
    __shared__ double red[CTA_WAVES];
    double dot = 0.0;
    const int k2 = VEC * g;
    const int64_t ngroups = (a.nblk + a.nbg - 1) / a.nbg;
    const int64_t first = xcd_logical_block(blockIdx.x, gridDim.x), step = gridDim.x;
    f4 rr[TPIPE_TPW][2], pp[TPIPE_TPW][2], xx[TPIPE_TPW][2];
    // Every lane loads every slot: slots past the group's tiles, rows past K1 and
    // columns past K2 read a clamped (valid, unused) address instead of
    // skipping the load, so no register has to keep its old value and the
    // loads stay in flight until step 1 of the next group uses them.
    const float* __restrict__ Xsrc = Xg ? Xg : R;
    auto fetch = [&](int64_t grp) {
        const int64_t blk0 = grp * a.nbg;
        const int nb = (int)std::min<int64_t>(a.nbg, a.nblk - blk0);
#pragma unroll
        for (int i = 0; i < TPIPE_TPW; ++i) {
            int it = wave + CTA_WAVES * i;
            if (it >= nb * gm.ni1t) it = 0;
            const int bl = it / gm.ni1t, ti = it - bl * gm.ni1t;
            const int i1 = min(ti * 16 + l16, a.K1 - 1);
            const int kc = min(k2, a.K2 - VEC);
            const int64_t off = (blk0 + bl) * bin + (int64_t)i1 * a.K2 + kc;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                // the fused tail's r is next read by the update one iteration later:
                // non-temporal, so that p, T and X stay cached for the passes in between
                // (the preconditioner's form reads its r again at once and keeps it)
                rr[i][h] = FR ? *reinterpret_cast<const f4*>(R + off + 4 * h)
                              : __builtin_nontemporal_load(reinterpret_cast<const f4*>(R + off + 4 * h));
                pp[i][h] = *reinterpret_cast<const f4*>(Pg + off + 4 * h);
                // x is next touched one iteration later: non-temporal, so that it
                // does not push the vectors read soon (T, p, r) out of the caches
                if constexpr (!FR) xx[i][h] = __builtin_nontemporal_load(reinterpret_cast<const f4*>(Xsrc + off + 4 * h));
            }
        }
    };
    if (first < ngroups) fetch(first);   // in flight while the factors are staged
    // factors into LDS (rows past the padded extents are never read)
    for (int u = threadIdx.x; u < gm.nj1t * 16 * (a.k1pad / 8); u += CTA_WG) {
        const int j = u / (a.k1pad / 8), c8 = (u - j * (a.k1pad / 8)) * 8;
        *reinterpret_cast<bf16x8*>(M1s + j * gm.ld1 + c8) =
            *reinterpret_cast<const bf16x8*>(M1 + (int64_t)j * a.ldm1 + c8);
    }
    for (int u = threadIdx.x; u < gm.nj2t * 16 * 4; u += CTA_WG) {
        const int j = u >> 2, c8 = (u & 3) * 8;
        *reinterpret_cast<bf16x8*>(M2s + j * gm.ld2 + c8) =
            *reinterpret_cast<const bf16x8*>(M2 + (int64_t)j * a.ldm2 + c8);
    }
    __syncthreads();  // factors staged
    for (int64_t grp = first; grp < ngroups; grp += step) {
        const int64_t blk0 = grp * a.nbg;
        const int nb = (int)std::min<int64_t>(a.nbg, a.nblk - blk0);
        // ---- step 1 from the fetched fragments: x += alpha p, p = r + beta p, Zt ----
        // All new values are formed before the first store: a wait for fetched
        // data issued after a store also waits for that store.
        f4 nv[TPIPE_TPW][2], nx[TPIPE_TPW][2];   // new p (FR: new r) and new x
#pragma unroll
        for (int i = 0; i < TPIPE_TPW; ++i) {
            const int it = wave + CTA_WAVES * i;
            if (it >= nb * gm.ni1t) continue;
            const int bl = it / gm.ni1t, ti = it - bl * gm.ni1t;
            const int i1 = ti * 16 + l16;
            typename T::frag xf = T::zfrag();
            if (i1 < a.K1 && k2 < a.K2) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if constexpr (FR) {
                        nv[i][h] = rr[i][h] - alpha * pp[i][h];
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            xf[4 * h + v] = (bf16)nv[i][h][v];
                            dot += (double)nv[i][h][v] * (double)nv[i][h][v];
                        }
                    } else {
                        if (Xg) nx[i][h] = xx[i][h] + alpha * pp[i][h];
                        nv[i][h] = rr[i][h] + beta * pp[i][h];
#pragma unroll
                        for (int v = 0; v < 4; ++v) xf[4 * h + v] = (bf16)nv[i][h][v];
                    }
                }
            }
            bf16* Zb = Zt + bl * gm.zsz;
#pragma unroll
            for (int x = 0; x < J2T; ++x) {
                if (x < gm.nj2t) {
                    const typename T::frag mf =
                        *reinterpret_cast<const typename T::frag*>(M2s + (x * 16 + l16) * gm.ld2 + k2);
                    const typename T::acc acc = T::mma(xf, mf, T::zero());
                    const int j2 = x * 16 + l16;
#pragma unroll
                    for (int r = 0; r < 4; ++r) Zb[j2 * gm.ldz + ti * 16 + T::arow(lane, r)] = (bf16)acc[r];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < TPIPE_TPW; ++i) {
            const int it = wave + CTA_WAVES * i;
            if (it >= nb * gm.ni1t) continue;
            const int bl = it / gm.ni1t, ti = it - bl * gm.ni1t;
            const int i1 = ti * 16 + l16;
            if (i1 < a.K1 && k2 < a.K2) {
                const int64_t off = (blk0 + bl) * bin + (int64_t)i1 * a.K2 + k2;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if constexpr (FR) {
                        *reinterpret_cast<f4*>(Rw + off + 4 * h) = nv[i][h];
                    } else {
                        if (Xg) __builtin_nontemporal_store(nx[i][h], reinterpret_cast<f4*>(Xg + off + 4 * h));
                        *reinterpret_cast<f4*>(Pg + off + 4 * h) = nv[i][h];
                    }
                }
            }
        }
        // the next group's fragments load while steps 2 and 3 run
        if (grp + step < ngroups) fetch(grp + step);
        __syncthreads();
        // ---- step 2: Ys[b][j1][j2] = sum_i1 M1[j1][i1] Zt[b][j2][i1] ----
        const int nsub = gm.nj2t * gm.nj1t;
        const int nks1 = a.k1pad / T::KSTEP;
        for (int sidx = wave; sidx < nb * nsub; sidx += CTA_WAVES) {
            const int bl = sidx / nsub, sb = sidx - bl * nsub;
            const int x1 = sb / gm.nj2t, x2 = sb - x1 * gm.nj2t;
            const bf16* zrow = Zt + bl * gm.zsz + (x2 * 16 + l16) * gm.ldz + VEC * g;
            const bf16* mrow = M1s + (x1 * 16 + l16) * gm.ld1 + VEC * g;
            typename T::acc acc = T::zero();
            for (int ks = 0; ks < nks1; ++ks) {
                const typename T::frag zf = *reinterpret_cast<const typename T::frag*>(zrow + ks * T::KSTEP);
                const typename T::frag mf = *reinterpret_cast<const typename T::frag*>(mrow + ks * T::KSTEP);
                acc = T::mma(zf, mf, acc);
            }
            const int j1 = x1 * 16 + l16;
            if (j1 < a.J1) {
                bf16* yb = Ys + bl * gm.bout + j1 * a.J2;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j2 = x2 * 16 + T::arow(lane, r);
                    if (j2 < a.J2) yb[j2] = (bf16)acc[r];
                }
            }
        }
        __syncthreads();
        // ---- step 3: contiguous write-back of the nb output blocks ----
        bf16* __restrict__ Y = reinterpret_cast<bf16*>(a.Y) + blk0 * gm.bout;
        const int total = nb * gm.bout;
        if ((reinterpret_cast<uintptr_t>(Y) & 15) == 0 && (total % 8) == 0) {
            for (int i = threadIdx.x * 8; i < total; i += CTA_WG * 8)
                *reinterpret_cast<bf16x8*>(Y + i) = *reinterpret_cast<const bf16x8*>(Ys + i);
        } else {
            for (int i = threadIdx.x; i < total; i += CTA_WG) Y[i] = Ys[i];
        }
        __syncthreads();  // Zt and Ys are reused by the next group
    }
    if constexpr (FR) block_partial(dot, a.partials, red);
}

template <bool FR>
static hipError_t go_tail_pipe(TailArgs a, hipStream_t s, int* grid_out = nullptr) {
    const TailPipeGeom gm = tail_pipe_geom(a.k1pad, a.J1, a.J2);
    if (a.k1pad > 128 || a.J1 > 128 || a.k2pad > 32 || a.J2 > 32 || a.K2 % 8 != 0 ||
        a.nbg * gm.ni1t > CTA_WAVES * TPIPE_TPW || a.k1pad > a.ldm1 || a.k2pad > a.ldm2)
        return hipErrorNotSupported;
    const size_t lds = tail_pipe_lds(gm, a.nbg);
    if (lds > 64 * 1024) return hipErrorNotSupported;
    const int64_t ngroups = (a.nblk + a.nbg - 1) / a.nbg;
    hipError_t e = ensure_lds(k_tail_pipe<FR>, lds);
    if (e != hipSuccess) return e;
    // persistent grid: as many workgroups per CU as are resident at once (at
    // most 3; the x and p form holds enough registers for 2), a multiple of
    // the XCD count
    static std::atomic<int64_t> cached{-1};   // lds << 8 | workgroups per CU
    int64_t c = cached.load(std::memory_order_relaxed);
    int per_cu;
    if (c >= 0 && (size_t)(c >> 8) == lds) {
        per_cu = (int)(c & 255);
    } else {
        per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tail_pipe<FR>, CTA_WG, lds) != hipSuccess)
            per_cu = 0;
        per_cu = std::max(1, std::min(per_cu, 3));
        cached.store((int64_t)lds << 8 | per_cu, std::memory_order_relaxed);
    }
    int grid = (int)std::min<int64_t>(ngroups, (int64_t)device_cus() * per_cu);
    grid = (grid + CTA_XCDS - 1) / CTA_XCDS * CTA_XCDS;
    if (grid_out) *grid_out = grid;
    k_tail_pipe<FR><<<grid, CTA_WG, lds, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_tail(int tin, int tout, int tc, const void* X, void* Y, const Mat& M1,
                       const Mat& M2, int64_t nblk, int K1, int K2, int J1, int J2, void* Pvec,
                       const double* beta, const int* done, hipStream_t s, int variant, void* Xsol,
                       const double* alpha) {
    if (!tail_fits(tc, K1, J2) || J1 > 256) return hipErrorInvalidValue;
    const int ks = dt_kstep(tc);
    TailArgs a{};
    a.X = X; a.Y = Y; a.M1 = M1.p; a.M2 = M2.p; a.ldm1 = M1.ld; a.ldm2 = M2.ld;
    a.K1 = K1; a.K2 = K2; a.J1 = J1; a.J2 = J2;
    a.k1pad = tail_k1pad(tc, K1);
    a.k2pad = (K2 + ks - 1) / ks * ks;
    a.nblk = nblk; a.Pvec = Pvec; a.beta = beta; a.done = done;
    a.Xsol = Pvec ? Xsol : nullptr; a.alpha = alpha;
    a.nbg = tail_nb(tc, tout, K1, J1, J2);
    if (variant == 1 && tail_lds_nb(tc, tout, K1, J1, J2, 2 * a.nbg) <= 64 * 1024) a.nbg *= 2;
    if (a.k1pad > M1.ld || a.k2pad > M2.ld) return hipErrorInvalidValue;
    const size_t lds = tail_lds_nb(tc, tout, K1, J1, J2, a.nbg);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const bool fuse = Pvec != nullptr;
    ProfScope ps(fuse ? (tc == DT_F64 ? "tail_p.f64" : tc == DT_F32 ? "tail_p.f32" : "tail_p.bf16")
                      : (tc == DT_F64 ? "tail.f64" : tc == DT_F32 ? "tail.f32" : "tail.bf16"), s);
    if (variant == 2 && fuse && tin == DT_F32 && tout == DT_BF16 && tc == DT_BF16) {
        // persistent pipelined form where the shape allows, else as variant 0
        const hipError_t e = go_tail_pipe<false>(a, s);
        if (e != hipErrorNotSupported) return e;
    }
    if (tin == DT_F32 && tout == DT_BF16 && tc == DT_BF16)
        return fuse ? tail_T<float, bf16, bf16, true>(a, lds, s)
                    : tail_T<float, bf16, bf16, false>(a, lds, s);
    if (tin == DT_F32 && tout == DT_F32 && tc == DT_F32)
        return fuse ? tail_T<float, float, float, true>(a, lds, s)
                    : tail_T<float, float, float, false>(a, lds, s);
    if (tin == DT_F64 && tout == DT_F64 && tc == DT_F64)
        return fuse ? tail_T<double, double, double, true>(a, lds, s)
                    : tail_T<double, double, double, false>(a, lds, s);
    if (!fuse && tin == DT_BF16 && tout == DT_BF16 && tc == DT_BF16)
        return tail_T<bf16, bf16, bf16, false>(a, lds, s);
    return hipErrorInvalidValue;
}

// Tail pass of the preconditioner with the residual update fused (BF16 chain):
// r = r - alpha q is formed on the fly, written back, fed to the chain, and
// <r, r> is reduced (partials, then the finalize kernel with POST_RHO).
template <int J2T>
__global__ __launch_bounds__(CTA_WG) void k_tail_r(TailArgs a) {
    if (a.done && *a.done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[CTA_WAVES];
    double dot = 0.0;
    const int64_t ngroups = (a.nblk + a.nbg - 1) / a.nbg;
    for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
        const int64_t blk0 = grp * a.nbg;
        const int nb = (int)std::min<int64_t>(a.nbg, a.nblk - blk0);
        tail_group<float, bf16, bf16, J2T, false, true>(a, blk0, nb, a.nbg, smem, &dot);
    }
    block_partial(dot, a.partials, red);
}

hipError_t launch_tail_r(void* R, const void* Q, void* Y, const Mat& M1, const Mat& M2, int64_t nblk, int K1,
                         int K2, int J1, int J2, const double* alpha, const int* done, double* partials,
                         CgScalars* scal, hipStream_t s, int variant) {
    if (!tail_fits(DT_BF16, K1, J2) || J1 > 256) return hipErrorInvalidValue;
    const int ks = dt_kstep(DT_BF16);
    TailArgs a{};
    a.X = R; a.Y = Y; a.M1 = M1.p; a.M2 = M2.p; a.ldm1 = M1.ld; a.ldm2 = M2.ld;
    a.K1 = K1; a.K2 = K2; a.J1 = J1; a.J2 = J2;
    a.k1pad = tail_k1pad(DT_BF16, K1);
    a.k2pad = (K2 + ks - 1) / ks * ks;
    a.nblk = nblk; a.Pvec = R; a.Qvec = Q; a.alpha = alpha; a.done = done; a.partials = partials;
    a.nbg = tail_nb(DT_BF16, DT_BF16, K1, J1, J2);
    if (variant == 1 && tail_lds_nb(DT_BF16, DT_BF16, K1, J1, J2, 2 * a.nbg) <= 64 * 1024) a.nbg *= 2;
    if (a.k1pad > M1.ld || a.k2pad > M2.ld) return hipErrorInvalidValue;
    const size_t lds = tail_lds_nb(DT_BF16, DT_BF16, K1, J1, J2, a.nbg);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const int64_t ngroups = (a.nblk + a.nbg - 1) / a.nbg;
    int grid = grid_for(ngroups, kMaxGrid);  // one partial per workgroup
    const int j2t = (J2 + 15) / 16;
    hipError_t e = hipErrorInvalidValue;
    {
        ProfScope ps("tail_r.bf16", s);
        if (variant == 2) e = go_tail_pipe<true>(a, s, &grid);   // pipelined form where it fits
        if (variant != 2 || e == hipErrorNotSupported) {
            e = hipErrorInvalidValue;
#define CTA_TAIL_R_GO(N)                                                        \
            {                                                                   \
                auto kern = k_tail_r<N>;                                        \
                e = ensure_lds(kern, lds);                                      \
                if (e == hipSuccess) {                                          \
                    kern<<<grid, CTA_WG, lds, s>>>(a);                          \
                    e = hipGetLastError();                                      \
                }                                                               \
            }
            if (j2t <= 2) CTA_TAIL_R_GO(2)
            else if (j2t <= 4) CTA_TAIL_R_GO(4)
            else if (j2t <= 8) CTA_TAIL_R_GO(8)
            else if (j2t <= 16) CTA_TAIL_R_GO(16)
#undef CTA_TAIL_R_GO
        }
    }
    if (e != hipSuccess) return e;
    return launch_finalize(partials, grid, scal, POST_RHO, nullptr, s);
}

// ------------------------------------------------------------------ contiguous
template <typename Tin, typename Tout, typename Tc, int JT>
__global__ __launch_bounds__(CTA_WG) void k_contig(ContigArgs a, const int* done) {
    if (done && *done) return;
    const int64_t nrt = (a.rows + 15) / 16;
    const int wave = threadIdx.x >> 6;
    for (int64_t rt = (int64_t)blockIdx.x * CTA_WAVES + wave; rt < nrt;
         rt += (int64_t)gridDim.x * CTA_WAVES)
        contig_rows<Tin, Tout, Tc, JT>(a, rt);
}

template <typename Tc>
static hipError_t contig_T(ContigArgs a, const int* done, hipStream_t s) {
    const int64_t nrt = (a.rows + 15) / 16;
    const int grid = grid_for((nrt + CTA_WAVES - 1) / CTA_WAVES, 65536);
    const int jt = (a.J + 15) / 16;
    if (jt <= 1) {
        a.j0 = 0;
        k_contig<Tc, Tc, Tc, 1><<<grid, CTA_WG, 0, s>>>(a, done);
        return hipGetLastError();
    }
    if (jt <= 2) {
        a.j0 = 0;
        k_contig<Tc, Tc, Tc, 2><<<grid, CTA_WG, 0, s>>>(a, done);
        return hipGetLastError();
    }
    for (int j0 = 0; j0 < a.J; j0 += 64) {
        a.j0 = j0;
        k_contig<Tc, Tc, Tc, 4><<<grid, CTA_WG, 0, s>>>(a, done);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_contig(int tc, const void* X, void* Y, const Mat& M, int64_t rows, int K, int J,
                         const int* done, hipStream_t s) {
    ContigArgs a{};
    a.X = X; a.Y = Y; a.M = M.p; a.ldm = M.ld;
    a.K = K; a.J = J; a.kpad = (K + dt_kstep(tc) - 1) / dt_kstep(tc) * dt_kstep(tc);
    a.rows = rows;
    if (a.kpad > M.ld) return hipErrorInvalidValue;
    ProfScope ps(tc == DT_F64 ? "contig.f64" : tc == DT_F32 ? "contig.f32" : "contig.bf16", s);
    switch (tc) {
        case DT_F64: return contig_T<double>(a, done, s);
        case DT_F32: return contig_T<float>(a, done, s);
        case DT_BF16: return contig_T<bf16>(a, done, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace cta
