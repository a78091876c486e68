// Shared device-side definitions for the gfx950 kernels: element types, MFMA
// operand traits, conversions and wave/workgroup reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef __bf16 bf16;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
typedef __attribute__((ext_vector_type(4))) float floatx4;
typedef __attribute__((ext_vector_type(2))) float floatx2;
typedef __attribute__((ext_vector_type(2))) double doublex2;
typedef __attribute__((ext_vector_type(4))) double doublex4;

#define CTA_WG 256          // threads per workgroup (4 waves of 64)
#define CTA_WAVES 4
#define CTA_XCDS 8          // MI355X: workgroups are dealt round-robin to 8 XCDs

// XCD-aware workgroup order.  Hardware deals workgroup b to XCD b % 8; this
// renumbering gives XCD x the contiguous range [x*G/8, (x+1)*G/8) of logical
// ids (in dispatch order), so tiles that are neighbours in memory run on the
// same XCD and share its L2.  G must be a multiple of 8.
__device__ __forceinline__ int64_t xcd_logical_block(int64_t b, int64_t G) {
    return (b % CTA_XCDS) * (G / CTA_XCDS) + b / CTA_XCDS;
}

// ---------------------------------------------------------------------------
// Conversions (float -> bf16 rounds to nearest even on gfx950).
template <typename To, typename From>
__device__ __forceinline__ To cvt(From x) { return (To)x; }
template <> __device__ __forceinline__ bf16 cvt<bf16, double>(double x) { return (bf16)(float)x; }
template <> __device__ __forceinline__ double cvt<double, bf16>(bf16 x) { return (double)(float)x; }

// ---------------------------------------------------------------------------
// MFMA operand traits.  Both operands are given as 16 x KSTEP tiles whose K
// index is contiguous per lane: lane l holds row (l % 16), K entries
// [VEC*(l/16), VEC*(l/16)+VEC).  mma() accumulates D[i][j] += sum_k A[i][k]*B[j][k]
// over one KSTEP; output register r of lane l is D[arow(l, r)][l % 16].
//   bf16: v_mfma_f32_16x16x32_bf16 (native layout)
//   f32 : four v_mfma_f32_16x16x4f32, step s pairs k = VEC*(l/16) + s
//   f64 : two  v_mfma_f64_16x16x4f64, step s pairs k = VEC*(l/16) + s
template <typename Tc> struct MT;

template <> struct MT<bf16> {
    static constexpr int VEC = 8;
    static constexpr int KSTEP = 32;
    typedef bf16x8 frag;
    typedef floatx4 acc;
    typedef float acc_t;
    __device__ __forceinline__ static acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
    __device__ __forceinline__ static frag zfrag() {
        frag f;
#pragma unroll
        for (int v = 0; v < 8; ++v) f[v] = (bf16)0.f;
        return f;
    }
    __device__ __forceinline__ static acc mma(const frag& a, const frag& b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static int arow(int lane, int r) { return 4 * (lane >> 4) + r; }
    static constexpr bool CONSEC = true;  // a lane's 4 outputs are consecutive rows
};

template <> struct MT<float> {
    static constexpr int VEC = 4;
    static constexpr int KSTEP = 16;
    typedef floatx4 frag;
    typedef floatx4 acc;
    typedef float acc_t;
    __device__ __forceinline__ static acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
    __device__ __forceinline__ static frag zfrag() { return frag{0.f, 0.f, 0.f, 0.f}; }
    __device__ __forceinline__ static acc mma(const frag& a, const frag& b, acc c) {
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], c, 0, 0, 0);
        return c;
    }
    __device__ __forceinline__ static int arow(int lane, int r) { return 4 * (lane >> 4) + r; }
    static constexpr bool CONSEC = true;
};

template <> struct MT<double> {
    static constexpr int VEC = 2;
    static constexpr int KSTEP = 8;
    typedef doublex2 frag;
    typedef doublex4 acc;
    typedef double acc_t;
    __device__ __forceinline__ static acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
    __device__ __forceinline__ static frag zfrag() { return frag{0.0, 0.0}; }
    __device__ __forceinline__ static acc mma(const frag& a, const frag& b, acc c) {
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], c, 0, 0, 0);
        return c;
    }
    // f64 16x16x4 output: register r of lane l is row (l/16) + 4r
    __device__ __forceinline__ static int arow(int lane, int r) { return (lane >> 4) + 4 * r; }
    static constexpr bool CONSEC = false;
};

// ---------------------------------------------------------------------------
// Load VEC consecutive elements of Tin starting at p (elements [0, nvalid) are
// read, the rest are zero) and convert them to an MFMA fragment of Tc.  The
// vector path needs p aligned to VEC elements (``aligned``).
template <typename Tc, typename Tin>
__device__ __forceinline__ typename MT<Tc>::frag load_frag(const Tin* __restrict__ p, int nvalid,
                                                           bool aligned) {
    typedef typename MT<Tc>::frag F;
    constexpr int V = MT<Tc>::VEC;
    F f;
    if (nvalid >= V && aligned) {
        if constexpr (sizeof(Tin) * V == 16) {
            // one 16-byte load, no conversion when Tin == Tc
            typedef Tin __attribute__((ext_vector_type(V))) vin;
            vin x = *reinterpret_cast<const vin*>(p);
#pragma unroll
            for (int v = 0; v < V; ++v) f[v] = cvt<Tc>(x[v]);
        } else if constexpr (sizeof(Tin) * V == 32) {
            typedef Tin __attribute__((ext_vector_type(V / 2))) vin;
            vin x0 = *reinterpret_cast<const vin*>(p);
            vin x1 = *reinterpret_cast<const vin*>(p + V / 2);
#pragma unroll
            for (int v = 0; v < V / 2; ++v) {
                f[v] = cvt<Tc>(x0[v]);
                f[v + V / 2] = cvt<Tc>(x1[v]);
            }
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) f[v] = cvt<Tc>(p[v]);
        }
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v) f[v] = v < nvalid ? cvt<Tc>(p[v]) : cvt<Tc>(0.f);
    }
    return f;
}

// ---------------------------------------------------------------------------
// FP64 reductions.  Wave reduction by xor-shuffles (fixed pattern, so the
// result is reproducible), then across the 4 waves through LDS.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// All threads of the workgroup must call; returns the sum on every thread.
__device__ __forceinline__ double block_sum(double v, double* red /* >= 4 doubles in LDS */) {
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    double s = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return s;
}

// The same for workgroups of NW = 4 or 8 waves (red >= NW doubles in LDS).
template <int NW>
__device__ __forceinline__ double block_sum_w(double v, double* red) {
    static_assert(NW == 4 || NW == 8, "4 or 8 waves");
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    double s = (red[0] + red[1]) + (red[2] + red[3]);
    if constexpr (NW == 8) s += (red[4] + red[5]) + (red[6] + red[7]);
    __syncthreads();
    return s;
}

template <typename T> __device__ __forceinline__ bool is_finite_val(T x) {
    return __builtin_isfinite((double)x);
}
