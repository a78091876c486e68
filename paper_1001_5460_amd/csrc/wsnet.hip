// Learned warm start: a separable network f whose layers are 1-D convolutions
// along one mode each (the convolution row of Table 1: an N-D convolution as
// separable per-mode transforms), trained with hand-written backward kernels
// (derivative rule of App. A.8: backpropagation applies the transposed maps).
//
//   h0 = lw * b + lb                         pointwise lift 1 -> C
//   block: z1 = relu(conv_1(h) + c1), z2 = relu(conv_2(z1) + c2),
//          z3 = relu(conv_3(z2) + c3), h = h + conv_4(z3) + c4
//   out = pw . h + pb                        pointwise projection C -> 1
//   X0  = s * out(B / s),  s = RMS of B
//
// Storage: activations and activation gradients channel-last [voxel][C] in
// BF16 (64 bytes per voxel for C = 32); FP32 master parameters, gradients and
// Adam moments; BF16 copies of the convolution weights in two layouts (forward
// [tap][co][ci], backward-data [flipped tap][ci][co]).
//
// Convolution (forward and backward-data) on MFMA: for 16 voxels and all 32
// output channels, D[co][voxel] = sum over 5 taps x 32 input channels, with
// v_mfma_f32_16x16x32_bf16 (K = 32 = the channels of one tap); the weights
// stay in registers for the whole launch, the input rows of the 5 taps are
// 16-byte loads of 8 channels (zero outside the mode's extent = zero padding).
// Weight gradient: dW[co][(tap, ci)] = sum over voxels g[v][co] x[v + d][ci]
// is a contraction over voxels; 64-voxel chunks of g and of the 5 shifted
// inputs are transposed into LDS (voxel index contiguous) and multiplied on
// MFMA; each workgroup writes a partial, a second kernel sums the partials in
// workgroup order (deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/cta.h"
#include "abi_internal.hpp"
#include "common.hpp"
#include "launch.hpp"
#include "prof.hpp"
#include "reduce.hpp"

namespace cta {
namespace ws {

constexpr int C = 32;
constexpr int WID = 5;
constexpr int NWPAR = C * C * WID;       // weights of one convolution
constexpr int NCONV = NWPAR + C;         // weights + bias of one convolution
constexpr int WG_PART = NCONV;           // floats per workgroup partial of a weight gradient

enum { EPI_RELU = 0, EPI_RES = 1, EPI_MASK = 2, EPI_ADD = 3 };

__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = (bf16)0.f;
    return z;
}

// ------------------------------------------------------------------ convolution
// out[v][ch] for all 32 channels: EPI_RELU relu(acc + bias); EPI_RES acc + bias + aux;
// EPI_MASK acc * (aux > 0); EPI_ADD acc + aux.  `out` may alias `aux` (same element).
template <int EPI>
__global__ __launch_bounds__(CTA_WG) void k_conv(const bf16* __restrict__ in,
                                                 const bf16* __restrict__ Wr,
                                                 const float* __restrict__ bias, const bf16* aux,
                                                 bf16* out, int V, int nk, int sk) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, l16 = lane & 15;
    bf16x8 wf[WID][2];
#pragma unroll
    for (int w = 0; w < WID; ++w)
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
            wf[w][rt] = *reinterpret_cast<const bf16x8*>(Wr + ((w * C) + rt * 16 + l16) * C + 8 * g);
    float bv[2][4];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            bv[rt][r] = (EPI == EPI_RELU || EPI == EPI_RES) ? bias[rt * 16 + 4 * g + r] : 0.f;
    const int ntiles = (V + 15) / 16;
    for (int tile = blockIdx.x * CTA_WAVES + wave; tile < ntiles; tile += gridDim.x * CTA_WAVES) {
        const int vox = tile * 16 + l16;
        const bool inb = vox < V;
        const int ik = inb ? (vox / sk) % nk : 0;
        floatx4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int w = 0; w < WID; ++w) {
            const int d = w - WID / 2;
            bf16x8 bfr = zero8();
            if (inb && ik + d >= 0 && ik + d < nk)
                bfr = *reinterpret_cast<const bf16x8*>(in + (int64_t)(vox + d * sk) * C + 8 * g);
            acc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[w][0], bfr, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[w][1], bfr, acc[1], 0, 0, 0);
        }
        if (!inb) continue;
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            const int ch = rt * 16 + 4 * g;
            float y[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) y[r] = acc[rt][r] + bv[rt][r];
            if constexpr (EPI != EPI_RELU) {
                const bf16x4 a4 = *reinterpret_cast<const bf16x4*>(aux + (int64_t)vox * C + ch);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float av = (float)a4[r];
                    if constexpr (EPI == EPI_MASK) y[r] = av > 0.f ? y[r] : 0.f;
                    else y[r] += av;
                }
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) y[r] = fmaxf(y[r], 0.f);
            }
            bf16x4 o;
#pragma unroll
            for (int r = 0; r < 4; ++r) o[r] = (bf16)y[r];
            *reinterpret_cast<bf16x4*>(out + (int64_t)vox * C + ch) = o;
        }
    }
}

// Column form of the same convolution, for modes whose stride sk is at least
// 16: a wave owns 16 consecutive trailing indices t of one leading index and
// walks i = 0..nk-1 along the mode, keeping the five input rows of the stencil
// (positions i-2..i+2) in registers and the next two prefetched, so every
// input row is read from memory once.  Same arithmetic as k_conv (same taps,
// same order of the MFMA sums), so the two forms give identical results.
template <int EPI>
__global__ __launch_bounds__(CTA_WG) void k_conv_col(const bf16* __restrict__ in,
                                                     const bf16* __restrict__ Wr,
                                                     const float* __restrict__ bias, const bf16* aux,
                                                     bf16* out, int nk, int sk, int tb, int64_t ncols) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, l16 = lane & 15;
    bf16x8 wf[WID][2];
#pragma unroll
    for (int w = 0; w < WID; ++w)
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
            wf[w][rt] = *reinterpret_cast<const bf16x8*>(Wr + ((w * C) + rt * 16 + l16) * C + 8 * g);
    float bv[2][4];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            bv[rt][r] = (EPI == EPI_RELU || EPI == EPI_RES) ? bias[rt * 16 + 4 * g + r] : 0.f;
    for (int64_t col = (int64_t)blockIdx.x * CTA_WAVES + wave; col < ncols;
         col += (int64_t)gridDim.x * CTA_WAVES) {
        const int64_t li = col / tb;
        const int t = (int)(col - li * tb) * 16 + l16;
        const bool ok = t < sk;
        const int64_t base = li * nk * (int64_t)sk + t;  // voxel (li, 0, t)
        auto ld = [&](int i) -> bf16x8 {
            return (ok && i < nk) ? *reinterpret_cast<const bf16x8*>(in + (base + (int64_t)i * sk) * C + 8 * g)
                                  : zero8();
        };
        bf16x8 r0 = zero8(), r1 = zero8(), r2 = ld(0), r3 = ld(1), r4 = ld(2), p0 = ld(3), p1 = ld(4);
        for (int i = 0; i < nk; ++i) {
            const int64_t vox = base + (int64_t)i * sk;
            bf16x4 a4[2];
            if constexpr (EPI != EPI_RELU) {
                if (ok) {
                    a4[0] = *reinterpret_cast<const bf16x4*>(aux + vox * C + 4 * g);
                    a4[1] = *reinterpret_cast<const bf16x4*>(aux + vox * C + 16 + 4 * g);
                }
            }
            floatx4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
            const bf16x8 rw[WID] = {r0, r1, r2, r3, r4};
#pragma unroll
            for (int w = 0; w < WID; ++w) {
                acc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[w][0], rw[w], acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[w][1], rw[w], acc[1], 0, 0, 0);
            }
            r0 = r1;
            r1 = r2;
            r2 = r3;
            r3 = r4;
            r4 = p0;
            p0 = p1;
            p1 = ld(i + 5);
            if (!ok) continue;
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                float y[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) y[r] = acc[rt][r] + bv[rt][r];
                if constexpr (EPI != EPI_RELU) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float av = (float)a4[rt][r];
                        if constexpr (EPI == EPI_MASK) y[r] = av > 0.f ? y[r] : 0.f;
                        else y[r] += av;
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) y[r] = fmaxf(y[r], 0.f);
                }
                bf16x4 o;
#pragma unroll
                for (int r = 0; r < 4; ++r) o[r] = (bf16)y[r];
                *reinterpret_cast<bf16x4*>(out + vox * C + rt * 16 + 4 * g) = o;
            }
        }
    }
}

// Contiguous-mode form (stride 1, the last mode): each wave stages the rows
// of its 16 voxels plus two on each side in LDS once (16-byte loads) and
// reads the five tap fragments from there.  The tile loop is uniform over the
// workgroup so that every wave reaches each barrier.  Same sums as k_conv.
constexpr int LROWS = 16 + 4;
constexpr int LPITCH = C + 8;  // bf16 per staged row (padding against bank conflicts)

template <int EPI>
__global__ __launch_bounds__(CTA_WG) void k_conv_line(const bf16* __restrict__ in,
                                                      const bf16* __restrict__ Wr,
                                                      const float* __restrict__ bias, const bf16* aux,
                                                      bf16* out, int V, int nk) {
    __shared__ __align__(16) bf16 rows[CTA_WAVES][LROWS * LPITCH];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, l16 = lane & 15;
    bf16* rw = rows[wave];
    bf16x8 wf[WID][2];
#pragma unroll
    for (int w = 0; w < WID; ++w)
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
            wf[w][rt] = *reinterpret_cast<const bf16x8*>(Wr + ((w * C) + rt * 16 + l16) * C + 8 * g);
    float bv[2][4];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            bv[rt][r] = (EPI == EPI_RELU || EPI == EPI_RES) ? bias[rt * 16 + 4 * g + r] : 0.f;
    const int ntiles = (V + 15) / 16;
    for (int base = blockIdx.x * CTA_WAVES; base < ntiles; base += gridDim.x * CTA_WAVES) {
        const int tile = base + wave;
        const int v0 = tile * 16;
        // stage voxels v0-2 .. v0+17 (row q holds voxel v0 - 2 + q; zero outside [0, V))
        for (int u = lane; u < LROWS * 4; u += 64) {
            const int q = u >> 2, part = u & 3;
            const int v = v0 - 2 + q;
            const bf16x8 val = (tile < ntiles && v >= 0 && v < V)
                                   ? *reinterpret_cast<const bf16x8*>(in + (int64_t)v * C + 8 * part)
                                   : zero8();
            *reinterpret_cast<bf16x8*>(rw + q * LPITCH + 8 * part) = val;
        }
        __syncthreads();
        const int vox = v0 + l16;
        const bool inb = tile < ntiles && vox < V;
        const int ik = inb ? vox % nk : 0;
        floatx4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int w = 0; w < WID; ++w) {
            const int d = w - WID / 2;
            bf16x8 bfr = zero8();
            if (inb && ik + d >= 0 && ik + d < nk)
                bfr = *reinterpret_cast<const bf16x8*>(rw + (l16 + 2 + d) * LPITCH + 8 * g);
            acc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[w][0], bfr, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[w][1], bfr, acc[1], 0, 0, 0);
        }
        __syncthreads();  // the rows are restaged by the next tile
        if (!inb) continue;
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            const int ch = rt * 16 + 4 * g;
            float y[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) y[r] = acc[rt][r] + bv[rt][r];
            if constexpr (EPI != EPI_RELU) {
                const bf16x4 a4 = *reinterpret_cast<const bf16x4*>(aux + (int64_t)vox * C + ch);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float av = (float)a4[r];
                    if constexpr (EPI == EPI_MASK) y[r] = av > 0.f ? y[r] : 0.f;
                    else y[r] += av;
                }
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) y[r] = fmaxf(y[r], 0.f);
            }
            bf16x4 o;
#pragma unroll
            for (int r = 0; r < 4; ++r) o[r] = (bf16)y[r];
            *reinterpret_cast<bf16x4*>(out + (int64_t)vox * C + ch) = o;
        }
    }
}

// ------------------------------------------------------------------ weight gradient
constexpr int WCH = 64;        // voxels per chunk
constexpr int WLD = WCH + 8;   // LDS row pitch (bf16)

__global__ __launch_bounds__(CTA_WG) void k_wgrad(const bf16* __restrict__ gr,
                                                  const bf16* __restrict__ x, int V, int nk, int sk,
                                                  float* __restrict__ part) {
    __shared__ __align__(16) bf16 gT[C][WLD];
    __shared__ __align__(16) bf16 xT[WID * C][WLD];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, l16 = lane & 15;
    floatx4 acc[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
    float db = 0.f;
    const int vl = threadIdx.x >> 2, pt = threadIdx.x & 3;
    const int nch = (V + WCH - 1) / WCH;
    for (int chunk = blockIdx.x; chunk < nch; chunk += gridDim.x) {
        const int vox = chunk * WCH + vl;
        const bool inb = vox < V;
        const int ik = inb ? (vox / sk) % nk : 0;
        {
            const bf16x8 gv = inb ? *reinterpret_cast<const bf16x8*>(gr + (int64_t)vox * C + 8 * pt) : zero8();
#pragma unroll
            for (int e = 0; e < 8; ++e) gT[8 * pt + e][vl] = gv[e];
        }
#pragma unroll
        for (int w = 0; w < WID; ++w) {
            const int d = w - WID / 2;
            const bool ok = inb && ik + d >= 0 && ik + d < nk;
            const bf16x8 xv = ok ? *reinterpret_cast<const bf16x8*>(x + (int64_t)(vox + d * sk) * C + 8 * pt) : zero8();
#pragma unroll
            for (int e = 0; e < 8; ++e) xT[w * C + 8 * pt + e][vl] = xv[e];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < WCH / 32; ++ks) {
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const int idx = wave + 4 * q;
                const int ct = idx / 10, kt = idx % 10;
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(&gT[ct * 16 + l16][ks * 32 + 8 * g]);
                const bf16x8 b = *reinterpret_cast<const bf16x8*>(&xT[kt * 16 + l16][ks * 32 + 8 * g]);
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[q], 0, 0, 0);
            }
        }
        if (threadIdx.x < C)
            for (int v = 0; v < WCH; ++v) db += (float)gT[threadIdx.x][v];
        __syncthreads();
    }
    float* pp = part + (size_t)blockIdx.x * WG_PART;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const int idx = wave + 4 * q;
        const int ct = idx / 10, kt = idx % 10;
        const int kk = kt * 16 + l16;
        const int w = kk / C, ci = kk % C;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int co = ct * 16 + 4 * g + r;
            pp[(co * C + ci) * WID + w] = acc[q][r];
        }
    }
    if (threadIdx.x < C) pp[NWPAR + threadIdx.x] = db;
}

// grad[i] += sum over workgroups of part[b][i] (in workgroup order)
__global__ __launch_bounds__(CTA_WG) void k_reduce_add(const float* __restrict__ part, int nblk,
                                                       int count, int stride, float* __restrict__ grad) {
    const int i = blockIdx.x * CTA_WG + threadIdx.x;
    if (i >= count) return;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * stride + i];
    grad[i] += s;
}

// ------------------------------------------------------------------ pointwise layers
__device__ __forceinline__ float rms_of(const double* ss, int V) {
    return (float)sqrt(*ss / (double)V);
}

__global__ __launch_bounds__(CTA_WG) void k_lift(const float* __restrict__ B, const double* ss, int V,
                                                 const float* __restrict__ lw,
                                                 const float* __restrict__ lb,
                                                 float* __restrict__ bhat, bf16* __restrict__ h0) {
    const float s = rms_of(ss, V);
    const float inv = s > 0.f ? 1.f / s : 0.f;
    for (int v = blockIdx.x * CTA_WG + threadIdx.x; v < V; v += gridDim.x * CTA_WG) {
        const float bh = B[v] * inv;
        bhat[v] = bh;
#pragma unroll
        for (int c0 = 0; c0 < C; c0 += 8) {
            bf16x8 o;
#pragma unroll
            for (int e = 0; e < 8; ++e) o[e] = (bf16)(lw[c0 + e] * bh + lb[c0 + e]);
            *reinterpret_cast<bf16x8*>(h0 + (int64_t)v * C + c0) = o;
        }
    }
}

__global__ __launch_bounds__(CTA_WG) void k_proj(const bf16* __restrict__ h, const float* __restrict__ pw,
                                                 const float* __restrict__ pb, const double* ss, int V,
                                                 float* __restrict__ X0) {
    const float s = rms_of(ss, V);
    for (int v = blockIdx.x * CTA_WG + threadIdx.x; v < V; v += gridDim.x * CTA_WG) {
        float acc = pb[0];
#pragma unroll
        for (int c0 = 0; c0 < C; c0 += 8) {
            const bf16x8 hv = *reinterpret_cast<const bf16x8*>(h + (int64_t)v * C + c0);
#pragma unroll
            for (int e = 0; e < 8; ++e) acc += pw[c0 + e] * (float)hv[e];
        }
        X0[v] = s * acc;
    }
}

// L = mean(((X0 - T) / s)^2) (partials), dX0 = 2 (X0 - T) / (V s^2)
__global__ __launch_bounds__(CTA_WG) void k_mse(const float* __restrict__ X0, const float* __restrict__ T,
                                                const double* ss, int V, float* __restrict__ dX0,
                                                double* partials) {
    __shared__ double red[4];
    const double s2 = *ss / (double)V;
    const float k2 = s2 > 0.0 ? (float)(2.0 / ((double)V * s2)) : 0.f;
    double acc = 0.0;
    for (int v = blockIdx.x * CTA_WG + threadIdx.x; v < V; v += gridDim.x * CTA_WG) {
        const float d = X0[v] - T[v];
        dX0[v] = k2 * d;
        acc += (double)d * (double)d;
    }
    block_partial(s2 > 0.0 ? acc / s2 : 0.0, partials, red);
}

// block sum of NV per-thread float vectors into part[blockIdx][0..NV)
template <int NV>
__device__ __forceinline__ void block_vec_partial(const float (&a)[NV], float* part) {
    __shared__ float red[CTA_WAVES][NV];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        float v = a[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wave][i] = v;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NV; i += CTA_WG)
        part[(size_t)blockIdx.x * NV + i] = (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]);
    __syncthreads();
}

// dout = dX0 * s; dh[v][c] = dout * pw[c]; partials of dpw[c] = sum dout h[v][c], dpb = sum dout
__global__ __launch_bounds__(CTA_WG) void k_proj_bwd(const float* __restrict__ dX0, const double* ss,
                                                     const bf16* __restrict__ h,
                                                     const float* __restrict__ pw, int V,
                                                     bf16* __restrict__ dh, float* __restrict__ part) {
    const float s = rms_of(ss, V);
    float a[C + 1];
#pragma unroll
    for (int i = 0; i <= C; ++i) a[i] = 0.f;
    for (int v = blockIdx.x * CTA_WG + threadIdx.x; v < V; v += gridDim.x * CTA_WG) {
        const float dout = dX0[v] * s;
        a[C] += dout;
#pragma unroll
        for (int c0 = 0; c0 < C; c0 += 8) {
            const bf16x8 hv = *reinterpret_cast<const bf16x8*>(h + (int64_t)v * C + c0);
            bf16x8 o;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                a[c0 + e] += dout * (float)hv[e];
                o[e] = (bf16)(dout * pw[c0 + e]);
            }
            *reinterpret_cast<bf16x8*>(dh + (int64_t)v * C + c0) = o;
        }
    }
    block_vec_partial<C + 1>(a, part);
}

// partials of dlw[c] = sum dh0[v][c] bhat[v], dlb[c] = sum dh0[v][c]
__global__ __launch_bounds__(CTA_WG) void k_lift_bwd(const bf16* __restrict__ dh0,
                                                     const float* __restrict__ bhat, int V,
                                                     float* __restrict__ part) {
    float a[2 * C];
#pragma unroll
    for (int i = 0; i < 2 * C; ++i) a[i] = 0.f;
    for (int v = blockIdx.x * CTA_WG + threadIdx.x; v < V; v += gridDim.x * CTA_WG) {
        const float bh = bhat[v];
#pragma unroll
        for (int c0 = 0; c0 < C; c0 += 8) {
            const bf16x8 gv = *reinterpret_cast<const bf16x8*>(dh0 + (int64_t)v * C + c0);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float gg = (float)gv[e];
                a[c0 + e] += gg * bh;
                a[C + c0 + e] += gg;
            }
        }
    }
    block_vec_partial<2 * C>(a, part);
}

__global__ __launch_bounds__(CTA_WG) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                                 float* __restrict__ m, float* __restrict__ v, int n,
                                                 float lr, float b1, float b2, float eps, float bc1,
                                                 float bc2) {
    const int i = blockIdx.x * CTA_WG + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// BF16 weight copies: Wf[conv][w][co][ci], Wb[conv][w'][ci][co] = W[co][ci][4 - w']
__global__ __launch_bounds__(CTA_WG) void k_refresh(const float* __restrict__ params, int nconv,
                                                    int off0, bf16* __restrict__ Wf,
                                                    bf16* __restrict__ Wb) {
    const int total = nconv * NWPAR;
    for (int e = blockIdx.x * CTA_WG + threadIdx.x; e < total; e += gridDim.x * CTA_WG) {
        const int cv = e / NWPAR, r = e % NWPAR;
        const int co = r / (C * WID), ci = (r / WID) % C, w = r % WID;
        const bf16 val = (bf16)params[off0 + cv * NCONV + r];
        Wf[(size_t)cv * NWPAR + ((w * C) + co) * C + ci] = val;
        Wb[(size_t)cv * NWPAR + (((WID - 1 - w) * C) + ci) * C + co] = val;
    }
}

}  // namespace ws
}  // namespace cta

using namespace cta;
using namespace cta::ws;

struct cta_ws_s {
    int order = 4;
    int64_t n[4] = {0, 0, 0, 0};
    int V = 0;
    int blocks = 0;
    int64_t P = 0;        // parameter count
    int step = 0;         // Adam steps taken
    float* params = nullptr;
    float* grad = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    bf16* Wf = nullptr;
    bf16* Wb = nullptr;
    float* bhat = nullptr;
    std::vector<bf16*> h;   // blocks + 1 block inputs/outputs
    std::vector<bf16*> z;   // 3 per block
    bf16* G[3] = {nullptr, nullptr, nullptr};
    float* part = nullptr;  // workgroup partials
    double* dpart = nullptr;
    double* ss = nullptr;   // sum of squares of B (device)
    CgScalars* scal = nullptr;
    std::vector<void*> allocs;
    int conv_grid = 0, wg_grid = 0, pw_grid = 0;
};

namespace {

int64_t off_conv(int b, int k) { return 2 * C + (int64_t)(b * 4 + k) * NCONV; }
int64_t off_pw(int blocks) { return 2 * C + (int64_t)blocks * 4 * NCONV; }

// SplitMix64 and Box-Muller for the initial parameters (host).
uint64_t splitmix(uint64_t& s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
double unif(uint64_t& s) { return ((splitmix(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
double gauss(uint64_t& s) {
    const double u1 = unif(s), u2 = unif(s);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

#define WS_HIP(x)                                                                         \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) return fail(CTA_ERR_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

cta_status ws_refresh(cta_ws_s* w, hipStream_t s) {
    const int nconv = w->blocks * 4;
    k_refresh<<<256, CTA_WG, 0, s>>>(w->params, nconv, (int)off_conv(0, 0), w->Wf, w->Wb);
    WS_HIP(hipGetLastError());
    return CTA_OK;
}

}  // namespace

extern "C" cta_status cta_ws_create(cta_ws* out, int order, const int64_t* n, int channels, int width,
                                    int blocks, uint64_t seed, void* stream) {
    if (!out || !n) return fail(CTA_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (order != 4) return fail(CTA_ERR_UNSUPPORTED, "the warm-start network takes order-4 tensors");
    if (channels != C || width != WID) return fail(CTA_ERR_UNSUPPORTED, "this build uses 32 channels and width 5");
    if (blocks < 1 || blocks > 16) return fail(CTA_ERR_ARG, "blocks must be in [1, 16]");
    int64_t V = 1;
    for (int k = 0; k < 4; ++k) {
        if (n[k] < 1) return fail(CTA_ERR_SHAPE, "extent %d is %lld", k, (long long)n[k]);
        V *= n[k];
    }
    if (V > (int64_t(1) << 26)) return fail(CTA_ERR_SHAPE, "tensor too large for the warm-start network");
    hipStream_t s = (hipStream_t)stream;
    cta_ws_s* w = new cta_ws_s();
    for (int k = 0; k < 4; ++k) w->n[k] = n[k];
    w->V = (int)V;
    w->blocks = blocks;
    w->P = off_pw(blocks) + C + 1;
    auto al = [&](size_t bytes) -> void* {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) return nullptr;
        w->allocs.push_back(p);
        return p;
    };
    const size_t act = (size_t)V * C * sizeof(bf16);
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete w;
        return fail(CTA_ERR_HIP, "device query failed");
    }
    w->conv_grid = prop.multiProcessorCount * 8;
    w->wg_grid = prop.multiProcessorCount;  // one weight-gradient partial per CU: the fixed-order sum stays short
    w->pw_grid = prop.multiProcessorCount * 4;
    bool ok = true;
    ok &= (w->params = (float*)al(w->P * 4)) != nullptr;
    ok &= (w->grad = (float*)al(w->P * 4)) != nullptr;
    ok &= (w->m = (float*)al(w->P * 4)) != nullptr;
    ok &= (w->v = (float*)al(w->P * 4)) != nullptr;
    ok &= (w->Wf = (bf16*)al((size_t)blocks * 4 * NWPAR * 2)) != nullptr;
    ok &= (w->Wb = (bf16*)al((size_t)blocks * 4 * NWPAR * 2)) != nullptr;
    ok &= (w->bhat = (float*)al((size_t)V * 4)) != nullptr;
    for (int i = 0; i <= blocks && ok; ++i) {
        w->h.push_back((bf16*)al(act));
        ok &= w->h.back() != nullptr;
    }
    for (int i = 0; i < 3 * blocks && ok; ++i) {
        w->z.push_back((bf16*)al(act));
        ok &= w->z.back() != nullptr;
    }
    for (int i = 0; i < 3 && ok; ++i) ok &= (w->G[i] = (bf16*)al(act)) != nullptr;
    ok &= (w->part = (float*)al((size_t)std::max(w->wg_grid * WG_PART, w->pw_grid * 2 * C) * 4)) != nullptr;
    ok &= (w->dpart = (double*)al(kMaxGrid * 8)) != nullptr;
    ok &= (w->ss = (double*)al(64)) != nullptr;
    ok &= (w->scal = (CgScalars*)al(sizeof(CgScalars))) != nullptr;
    if (!ok) {
        cta_ws_destroy(w);
        return fail(CTA_ERR_NOMEM, "allocation of the warm-start network failed");
    }
    // initial parameters: He-scaled convolutions (the residual branch's last
    // convolution scaled by 0.1), unit lift, 1/sqrt(C) projection, zero biases
    std::vector<float> p0(w->P, 0.f);
    uint64_t st = seed ^ 0x5eedull;
    for (int c = 0; c < C; ++c) p0[c] = (float)gauss(st);
    for (int b = 0; b < blocks; ++b)
        for (int k = 0; k < 4; ++k) {
            const double sd = std::sqrt(2.0 / (C * WID)) * (k == 3 ? 0.1 : 1.0);
            for (int i = 0; i < NWPAR; ++i) p0[off_conv(b, k) + i] = (float)(sd * gauss(st));
        }
    for (int c = 0; c < C; ++c) p0[off_pw(blocks) + c] = (float)(gauss(st) / std::sqrt((double)C));
    cta_status rs = CTA_OK;
    if (hipMemcpy(w->params, p0.data(), w->P * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(w->grad, 0, w->P * 4) != hipSuccess || hipMemset(w->m, 0, w->P * 4) != hipSuccess ||
        hipMemset(w->v, 0, w->P * 4) != hipSuccess || hipMemset(w->scal, 0, sizeof(CgScalars)) != hipSuccess)
        rs = fail(CTA_ERR_HIP, "initialisation copies failed");
    if (rs == CTA_OK) rs = ws_refresh(w, s);
    if (rs == CTA_OK && hipStreamSynchronize(s) != hipSuccess) rs = fail(CTA_ERR_HIP, "synchronize failed");
    if (rs != CTA_OK) {
        cta_ws_destroy(w);
        return rs;
    }
    *out = w;
    return CTA_OK;
}

extern "C" cta_status cta_ws_destroy(cta_ws w) {
    if (!w) return CTA_OK;
    (void)hipDeviceSynchronize();
    for (void* p : w->allocs) (void)hipFree(p);
    delete w;
    return CTA_OK;
}

extern "C" int64_t cta_ws_num_params(cta_ws w) { return w ? w->P : 0; }

// tracer names per epilogue: [EPI][flat, column, line]
static const char* const kConvName[4][3] = {
    {"ws_conv.flat.relu", "ws_conv.col.relu", "ws_conv.line.relu"},
    {"ws_conv.flat.res", "ws_conv.col.res", "ws_conv.line.res"},
    {"ws_conv.flat.mask", "ws_conv.col.mask", "ws_conv.line.mask"},
    {"ws_conv.flat.add", "ws_conv.col.add", "ws_conv.line.add"}};

template <int EPI>
static void conv_go(cta_ws_s* w, const bf16* in, const bf16* Wr, const float* bias, const bf16* aux,
                    bf16* out, int nk, int sk, hipStream_t s) {
    if (sk >= 16) {
        const int tb = (sk + 15) / 16;
        const int64_t ncols = (int64_t)(w->V / ((int64_t)nk * sk)) * tb;
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((ncols + CTA_WAVES - 1) / CTA_WAVES, 65536));
        ProfScope ps(kConvName[EPI][1], s);
        k_conv_col<EPI><<<grid, CTA_WG, 0, s>>>(in, Wr, bias, aux, out, nk, sk, tb, ncols);
    } else if (sk == 1) {
        ProfScope ps(kConvName[EPI][2], s);
        k_conv_line<EPI><<<w->conv_grid, CTA_WG, 0, s>>>(in, Wr, bias, aux, out, w->V, nk);
    } else {
        ProfScope ps(kConvName[EPI][0], s);
        k_conv<EPI><<<w->conv_grid, CTA_WG, 0, s>>>(in, Wr, bias, aux, out, w->V, nk, sk);
    }
}

static cta_status conv_launch(cta_ws_s* w, int epi, const bf16* in, const bf16* Wr, const float* bias,
                              const bf16* aux, bf16* out, int k, hipStream_t s) {
    int sk = 1;
    for (int l = k + 1; l < 4; ++l) sk *= (int)w->n[l];
    const int nk = (int)w->n[k];
    switch (epi) {
        case EPI_RELU: conv_go<EPI_RELU>(w, in, Wr, bias, aux, out, nk, sk, s); break;
        case EPI_RES: conv_go<EPI_RES>(w, in, Wr, bias, aux, out, nk, sk, s); break;
        case EPI_MASK: conv_go<EPI_MASK>(w, in, Wr, bias, aux, out, nk, sk, s); break;
        default: conv_go<EPI_ADD>(w, in, Wr, bias, aux, out, nk, sk, s); break;
    }
    WS_HIP(hipGetLastError());
    return CTA_OK;
}

extern "C" cta_status cta_ws_forward(cta_ws w, const void* B, void* X0, int training, void* stream) {
    (void)training;  // activations are always kept: the memory is allocated at creation
    if (!w || !B || !X0) return fail(CTA_ERR_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    WS_HIP(launch_dot(DT_F32, B, B, w->V, w->dpart, w->scal, w->ss, s));
    const float* P = w->params;
    {
        ProfScope ps("ws_lift", s);
        k_lift<<<w->pw_grid, CTA_WG, 0, s>>>((const float*)B, w->ss, w->V, P, P + C, w->bhat, w->h[0]);
    }
    WS_HIP(hipGetLastError());
    for (int b = 0; b < w->blocks; ++b) {
        const bf16* hin = w->h[b];
        bf16* z1 = w->z[3 * b];
        bf16* z2 = w->z[3 * b + 1];
        bf16* z3 = w->z[3 * b + 2];
        const bf16* Wf = w->Wf + (size_t)(b * 4) * NWPAR;
        cta_status st;
        st = conv_launch(w, EPI_RELU, hin, Wf, P + off_conv(b, 0) + NWPAR, nullptr, z1, 0, s);
        if (st == CTA_OK) st = conv_launch(w, EPI_RELU, z1, Wf + NWPAR, P + off_conv(b, 1) + NWPAR, nullptr, z2, 1, s);
        if (st == CTA_OK) st = conv_launch(w, EPI_RELU, z2, Wf + 2 * NWPAR, P + off_conv(b, 2) + NWPAR, nullptr, z3, 2, s);
        if (st == CTA_OK) st = conv_launch(w, EPI_RES, z3, Wf + 3 * NWPAR, P + off_conv(b, 3) + NWPAR, hin, w->h[b + 1], 3, s);
        if (st != CTA_OK) return st;
    }
    const int64_t op = off_pw(w->blocks);
    {
        ProfScope ps("ws_proj", s);
        k_proj<<<w->pw_grid, CTA_WG, 0, s>>>(w->h[w->blocks], P + op, P + op + C, w->ss, w->V, (float*)X0);
    }
    WS_HIP(hipGetLastError());
    return CTA_OK;
}

extern "C" cta_status cta_ws_mse(cta_ws w, const void* X0, const void* T, void* dX0, double* loss,
                                 void* stream) {
    if (!w || !X0 || !T || !dX0) return fail(CTA_ERR_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    const int g = std::min(w->pw_grid, kMaxGrid);
    {
        ProfScope ps("ws_mse", s);
        k_mse<<<g, CTA_WG, 0, s>>>((const float*)X0, (const float*)T, w->ss, w->V, (float*)dX0, w->dpart);
    }
    WS_HIP(hipGetLastError());
    if (loss) {
        // mean = total / V: the finalize writes the total; scale on the device
        WS_HIP(launch_finalize(w->dpart, g, w->scal, POST_DOT, loss, s));
        WS_HIP(launch_axpby(DT_F64, 0.0, loss, 1.0 / (double)w->V, loss, 1, s));
    }
    return CTA_OK;
}

static cta_status wgrad_launch(cta_ws_s* w, const bf16* g, const bf16* x, int k, float* grad_conv,
                               hipStream_t s) {
    int sk = 1;
    for (int l = k + 1; l < 4; ++l) sk *= (int)w->n[l];
    {
        ProfScope ps("ws_wgrad", s);
        k_wgrad<<<w->wg_grid, CTA_WG, 0, s>>>(g, x, w->V, (int)w->n[k], sk, w->part);
    }
    WS_HIP(hipGetLastError());
    ProfScope ps("ws_reduce", s);
    k_reduce_add<<<(NCONV + CTA_WG - 1) / CTA_WG, CTA_WG, 0, s>>>(w->part, w->wg_grid, NCONV, WG_PART, grad_conv);
    WS_HIP(hipGetLastError());
    return CTA_OK;
}

extern "C" cta_status cta_ws_backward(cta_ws w, const void* dX0, void* stream) {
    if (!w || !dX0) return fail(CTA_ERR_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    const float* P = w->params;
    const int64_t op = off_pw(w->blocks);
    bf16* dh = w->G[0];
    {
        ProfScope ps("ws_proj_bwd", s);
        k_proj_bwd<<<w->pw_grid, CTA_WG, 0, s>>>((const float*)dX0, w->ss, w->h[w->blocks], P + op, w->V, dh, w->part);
    }
    WS_HIP(hipGetLastError());
    k_reduce_add<<<1, CTA_WG, 0, s>>>(w->part, w->pw_grid, C + 1, C + 1, w->grad + op);
    WS_HIP(hipGetLastError());
    for (int b = w->blocks - 1; b >= 0; --b) {
        const bf16* hin = w->h[b];
        const bf16* z1 = w->z[3 * b];
        const bf16* z2 = w->z[3 * b + 1];
        const bf16* z3 = w->z[3 * b + 2];
        const bf16* Wb = w->Wb + (size_t)(b * 4) * NWPAR;
        cta_status st;
        // conv 4 (mode 4): gradient at its output is dh
        st = wgrad_launch(w, dh, z3, 3, w->grad + off_conv(b, 3), s);
        if (st == CTA_OK) st = conv_launch(w, EPI_MASK, dh, Wb + 3 * NWPAR, nullptr, z3, w->G[1], 3, s);
        if (st == CTA_OK) st = wgrad_launch(w, w->G[1], z2, 2, w->grad + off_conv(b, 2), s);
        if (st == CTA_OK) st = conv_launch(w, EPI_MASK, w->G[1], Wb + 2 * NWPAR, nullptr, z2, w->G[2], 2, s);
        if (st == CTA_OK) st = wgrad_launch(w, w->G[2], z1, 1, w->grad + off_conv(b, 1), s);
        if (st == CTA_OK) st = conv_launch(w, EPI_MASK, w->G[2], Wb + NWPAR, nullptr, z1, w->G[1], 1, s);
        if (st == CTA_OK) st = wgrad_launch(w, w->G[1], hin, 0, w->grad + off_conv(b, 0), s);
        // gradient of the block input: through conv 1 plus the residual skip (in place)
        if (st == CTA_OK) st = conv_launch(w, EPI_ADD, w->G[1], Wb, nullptr, dh, dh, 0, s);
        if (st != CTA_OK) return st;
    }
    {
        ProfScope ps("ws_lift_bwd", s);
        k_lift_bwd<<<w->pw_grid, CTA_WG, 0, s>>>(dh, w->bhat, w->V, w->part);
    }
    WS_HIP(hipGetLastError());
    k_reduce_add<<<1, CTA_WG, 0, s>>>(w->part, w->pw_grid, C, 2 * C, w->grad);
    WS_HIP(hipGetLastError());
    k_reduce_add<<<1, CTA_WG, 0, s>>>(w->part + C, w->pw_grid, C, 2 * C, w->grad + C);
    WS_HIP(hipGetLastError());
    return CTA_OK;
}

extern "C" cta_status cta_ws_zero_grad(cta_ws w, void* stream) {
    if (!w) return fail(CTA_ERR_ARG, "NULL argument");
    WS_HIP(launch_fill_zero(w->grad, w->P * 4, (hipStream_t)stream));
    return CTA_OK;
}

extern "C" cta_status cta_ws_adam_step(cta_ws w, float lr, float beta1, float beta2, float eps,
                                       void* stream) {
    if (!w) return fail(CTA_ERR_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    w->step += 1;
    const float bc1 = (float)(1.0 - std::pow((double)beta1, w->step));
    const float bc2 = (float)(1.0 - std::pow((double)beta2, w->step));
    {
        ProfScope ps("ws_adam", s);
        k_adam<<<(int)((w->P + CTA_WG - 1) / CTA_WG), CTA_WG, 0, s>>>(w->params, w->grad, w->m, w->v, (int)w->P,
                                                                 lr, beta1, beta2, eps, bc1, bc2);
    }
    WS_HIP(hipGetLastError());
    return ws_refresh(w, s);
}

extern "C" cta_status cta_ws_params(cta_ws w, void* host_buf, size_t bytes, int set, void* stream) {
    if (!w || !host_buf) return fail(CTA_ERR_ARG, "NULL argument");
    if (bytes != (size_t)w->P * 4) return fail(CTA_ERR_ARG, "expected %lld bytes", (long long)(w->P * 4));
    hipStream_t s = (hipStream_t)stream;
    WS_HIP(hipStreamSynchronize(s));
    if (set == 1) {
        WS_HIP(hipMemcpy(w->params, host_buf, bytes, hipMemcpyHostToDevice));
        cta_status st = ws_refresh(w, s);
        if (st != CTA_OK) return st;
        WS_HIP(hipStreamSynchronize(s));
    } else if (set == 0 || set == 2) {
        WS_HIP(hipMemcpy(host_buf, set == 0 ? w->params : w->grad, bytes, hipMemcpyDeviceToHost));
    } else {
        return fail(CTA_ERR_ARG, "set must be 0, 1 or 2");
    }
    return CTA_OK;
}
