// Mode-product (TTM) building blocks for gfx950.
//
// A mode-k product (Sec. 2.1, eq. separable_transf) on a row-major tensor is
// viewed as (lead, K, trail): Y[b, j, t] = sum_i M[j, i] X[b, i, t].  Every
// pass is a batched dense contraction on MFMA; no transpose ever goes through
// HBM:
//  * strided pass  -- mode with trail > 1: a tile of TN consecutive t columns
//    of one b is staged in LDS transposed (K contiguous per column) and
//    multiplied by M; each lane ends up owning 4 consecutive t of one output
//    row j, so stores are short contiguous runs.
//  * tail pass     -- the last two modes together on one contiguous block
//    X_b (K1 x K2): Z = X_b M2^T (read straight from HBM, K2 contiguous),
//    Z^T kept in LDS, then Y_b = M1 Z.  One HBM round trip for two modes.
//  * contiguous pass -- the last mode alone: rows of K contiguous elements
//    are MFMA operands as loaded.
// M is read from a zero-padded copy (rows and columns padded to the MFMA
// tile), so padding never needs a branch in the inner loop.
#pragma once

#include "common.hpp"

namespace cta {

// ---------------------------------------------------------------------------
// Regularised normal-operator epilogue: Q = acc + lam * sum_k P x_k R_k on the
// output element, plus the FP64 partial of <P, Q>.  R_k is banded with
// half-bandwidth <= 2 and stored as rband[k][i*5 + d + 2] = R_k[i][i + d].
template <typename Tv>
struct StencilArgs {
    const Tv* P;            // same shape as the output (lead == 1)
    const Tv* rband[8];     // per mode, nullptr = no regulariser on that mode
    int64_t ext[8];         // extents of the full tensor
    int64_t stride[8];      // element strides of the full tensor
    int order;
    double lam;
    double* partials;       // one double per workgroup
};

struct StridedArgs {
    const void* X;
    void* Y;
    const void* M;   // Tc, row-major [>= JPAD][ldm], zero padded
    int ldm;
    int K, J, kpad;  // kpad: K rounded up to the MFMA KSTEP
    int64_t lead, trail;
    int64_t ntt;     // t tiles per b
    int64_t ntiles;  // lead * ntt
};

struct TailArgs {
    const void* X;   // (nblk, K1, K2)  (or r when fused with the p update)
    void* Y;         // (nblk, J1, J2)
    const void* M1;  // Tc [>= J1 pad][ldm1]
    const void* M2;  // Tc [>= J2 pad][ldm2]
    int ldm1, ldm2;
    int K1, K2, J1, J2;
    int k1pad, k2pad;  // K1 rounded up to max(KSTEP, 16), K2 to KSTEP
    int64_t nblk;
    // fused CG direction update p = r + beta p (the chain input is the new p)
    void* Pvec;
    const double* beta;
    const int* done;
};

struct ContigArgs {
    const void* X;   // (rows, K)
    void* Y;         // (rows, J)
    const void* M;
    int ldm;
    int K, J, kpad;
    int64_t rows;
    int j0;          // first output row handled by this launch (j chunking)
};

// ---------------------------------------------------------------------------
// Strided pass.  Waves are arranged WJ x WC; a wave owns JT j-tiles and CT
// column tiles of 16.  TN = 16*CT*WC columns, JPAD = 16*JT*WJ output rows.
template <typename Tin, typename Tout, typename Tc, int JT, int WJ, int CT, bool EPI>
__device__ __forceinline__ void strided_tile(const StridedArgs& a, int64_t tile, Tc* Xs,
                                             const StencilArgs<Tout>* st, double& dot_acc) {
    typedef MT<Tc> T;
    constexpr int WC = CTA_WAVES / WJ;
    constexpr int TN = 16 * CT * WC;
    constexpr int VEC = T::VEC;
    constexpr int LV = 16 / sizeof(Tin);  // elements of one 16-byte global load
    const int ldx = a.kpad + 16 / (int)sizeof(Tc);
    const int64_t b = tile / a.ntt;
    const int64_t t0 = (tile - b * a.ntt) * TN;
    const Tin* __restrict__ X = reinterpret_cast<const Tin*>(a.X) + b * (int64_t)a.K * a.trail;
    Tout* __restrict__ Y = reinterpret_cast<Tout*>(a.Y) + b * (int64_t)a.J * a.trail;
    const Tc* __restrict__ M = reinterpret_cast<const Tc*>(a.M);

    // ---- stage X[b, 0:kpad, t0:t0+TN] into LDS as Xs[t][k] ----
    const bool vec_ok = (a.trail % LV) == 0;
    constexpr int TCH = TN / LV;              // 16-byte chunks per row
    const int nunits = (a.kpad / VEC) * TCH;  // (VEC rows) x (LV columns) units
    for (int u = threadIdx.x; u < nunits; u += CTA_WG) {
        const int tc = u % TCH;
        const int kg = u / TCH;
        const int64_t t = t0 + (int64_t)tc * LV;
        Tin v[VEC][LV];
#pragma unroll
        for (int r = 0; r < VEC; ++r) {
            const int k = kg * VEC + r;
            if (k < a.K && vec_ok && t + LV <= a.trail) {
                typedef Tin __attribute__((ext_vector_type(LV))) vin;
                vin x = *reinterpret_cast<const vin*>(X + (int64_t)k * a.trail + t);
#pragma unroll
                for (int c = 0; c < LV; ++c) v[r][c] = x[c];
            } else {
#pragma unroll
                for (int c = 0; c < LV; ++c)
                    v[r][c] = (k < a.K && t + c < a.trail) ? X[(int64_t)k * a.trail + t + c]
                                                          : cvt<Tin>(0.f);
            }
        }
#pragma unroll
        for (int c = 0; c < LV; ++c) {
            typename T::frag f;
#pragma unroll
            for (int r = 0; r < VEC; ++r) f[r] = cvt<Tc>(v[r][c]);
            *reinterpret_cast<typename T::frag*>(Xs + (tc * LV + c) * ldx + kg * VEC) = f;
        }
    }
    __syncthreads();

    // ---- MFMA: D[c][j] = sum_k Xs[c][k] * M[j][k] ----
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wj = wave % WJ, wc = wave / WJ;
    const int cb = wc * CT * 16, jb = wj * JT * 16;
    const int g = lane >> 4, l16 = lane & 15;
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
        for (int y = 0; y < CT; ++y)
            xa[y] = *reinterpret_cast<const typename T::frag*>(Xs + (cb + y * 16 + l16) * ldx + k0);
#pragma unroll
        for (int x = 0; x < JT; ++x)
            mb[x] = *reinterpret_cast<const typename T::frag*>(M + (int64_t)(jb + x * 16 + l16) * a.ldm + k0);
#pragma unroll
        for (int x = 0; x < JT; ++x)
#pragma unroll
            for (int y = 0; y < CT; ++y) acc[x][y] = T::mma(xa[y], mb[x], acc[x][y]);
    }

    // ---- epilogue / store: lane owns rows j, columns c = arow(lane, r) ----
#pragma unroll
    for (int x = 0; x < JT; ++x) {
        const int j = jb + x * 16 + l16;
        if (j >= a.J) continue;
#pragma unroll
        for (int y = 0; y < CT; ++y) {
            const int cbase = cb + y * 16;
            if constexpr (!EPI) {
                if constexpr (T::CONSEC) {
                    const int64_t t = t0 + cbase + 4 * g;
                    Tout* dst = Y + (int64_t)j * a.trail + t;
                    if (vec_ok && (a.trail % 4) == 0 && t + 4 <= a.trail) {
                        typedef Tout __attribute__((ext_vector_type(4))) vout;
                        vout o;
#pragma unroll
                        for (int r = 0; r < 4; ++r) o[r] = cvt<Tout>(acc[x][y][r]);
                        *reinterpret_cast<vout*>(dst) = o;
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (t + r < a.trail) dst[r] = cvt<Tout>(acc[x][y][r]);
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t t = t0 + cbase + T::arow(lane, r);
                        if (t < a.trail) Y[(int64_t)j * a.trail + t] = cvt<Tout>(acc[x][y][r]);
                    }
                }
            } else {
                // normal-operator epilogue (lead == 1): add the banded regulariser
                const Tout* __restrict__ P = st->P;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t t = t0 + cbase + T::arow(lane, r);
                    if (t >= a.trail) continue;
                    const int64_t base = (int64_t)j * a.trail + t;
                    Tout s = cvt<Tout>(0.f);
                    for (int k = 0; k < st->order; ++k) {
                        const Tout* __restrict__ rb = st->rband[k];
                        if (!rb) continue;
                        const int64_t n = st->ext[k], sk = st->stride[k];
                        const int64_t ik = (k == 0) ? (int64_t)j : (t / sk) % n;
                        const Tout* row = rb + ik * 5;
#pragma unroll
                        for (int d = -2; d <= 2; ++d) {
                            const int64_t q = ik + d;
                            if (q >= 0 && q < n) s += row[d + 2] * P[base + d * sk];
                        }
                    }
                    const Tout pv = P[base];
                    const Tout qv = cvt<Tout>(acc[x][y][r]) + cvt<Tout>(st->lam) * s;
                    Y[base] = qv;
                    dot_acc += (double)pv * (double)qv;
                }
            }
        }
    }
    __syncthreads();  // Xs is reused by the next tile
}

// ---------------------------------------------------------------------------
// Tail pass on blocks of the last two modes.  J2T: maximum number of 16-wide
// j2 tiles (compile time), the runtime count is (J2 + 15) / 16.
template <typename Tin, typename Tout, typename Tc, int J2T, bool FUSE_P>
__device__ __forceinline__ void tail_block(const TailArgs& a, int64_t blk, Tc* Zt) {
    typedef MT<Tc> T;
    constexpr int VEC = T::VEC;
    const int ldz = a.k1pad + 16 / (int)sizeof(Tc);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, l16 = lane & 15;
    const int64_t in_off = blk * (int64_t)a.K1 * a.K2;
    const Tin* __restrict__ X = reinterpret_cast<const Tin*>(a.X) + in_off;
    Tin* __restrict__ Pv = FUSE_P ? reinterpret_cast<Tin*>(a.Pvec) + in_off : nullptr;
    const Tc* __restrict__ M1 = reinterpret_cast<const Tc*>(a.M1);
    const Tc* __restrict__ M2 = reinterpret_cast<const Tc*>(a.M2);
    Tin beta = cvt<Tin>(0.f);
    if constexpr (FUSE_P) beta = cvt<Tin>(*a.beta);
    const int nj2t = (a.J2 + 15) / 16;
    const int ni1t = a.k1pad / 16;
    const int nks2 = a.k2pad / T::KSTEP;

    // ---- step 1: Zt[j2][i1] = sum_k2 X[i1][k2] M2[j2][k2] ----
    for (int it = wave; it < ni1t; it += CTA_WAVES) {
        const int i1 = it * 16 + l16;
        typename T::acc acc[J2T];
#pragma unroll
        for (int x = 0; x < J2T; ++x) acc[x] = T::zero();
        for (int ks = 0; ks < nks2; ++ks) {
            const int k2 = ks * T::KSTEP + VEC * g;
            typename T::frag xf;
            const int nv = (i1 < a.K1) ? max(0, min(VEC, a.K2 - k2)) : 0;
            if constexpr (FUSE_P) {
                // p = r + beta * p on the fly; the new p is written back once
                xf = T::zfrag();
                const int64_t off = (int64_t)i1 * a.K2 + k2;
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    if (v < nv) {
                        const Tin pn = X[off + v] + beta * Pv[off + v];
                        Pv[off + v] = pn;
                        xf[v] = cvt<Tc>(pn);
                    }
                }
            } else {
                xf = (nv > 0) ? load_frag<Tc>(X + (int64_t)i1 * a.K2 + k2, nv, (a.K2 % VEC) == 0)
                               : T::zfrag();
            }
#pragma unroll
            for (int x = 0; x < J2T; ++x) {
                if (x < nj2t) {
                    const typename T::frag mf = *reinterpret_cast<const typename T::frag*>(
                        M2 + (int64_t)(x * 16 + l16) * a.ldm2 + k2);
                    acc[x] = T::mma(xf, mf, acc[x]);
                }
            }
        }
        // D[i1][j2]: lane owns i1 = it*16 + arow(lane, r), j2 = x*16 + l16
#pragma unroll
        for (int x = 0; x < J2T; ++x) {
            if (x < nj2t) {
                const int j2 = x * 16 + l16;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    Zt[j2 * ldz + it * 16 + T::arow(lane, r)] = cvt<Tc>(acc[x][r]);
            }
        }
    }
    __syncthreads();

    // ---- step 2: Y[j1][j2] = sum_i1 M1[j1][i1] Zt[j2][i1]; D[j2][j1] ----
    const int nj1t = (a.J1 + 15) / 16;
    const int nsub = nj2t * nj1t;
    const int nks1 = a.k1pad / T::KSTEP;
    Tout* __restrict__ Y = reinterpret_cast<Tout*>(a.Y) + blk * (int64_t)a.J1 * a.J2;
    for (int s = wave; s < nsub; s += CTA_WAVES) {
        const int x2 = s % nj2t, x1 = s / nj2t;
        typename T::acc acc = T::zero();
        for (int ks = 0; ks < nks1; ++ks) {
            const int k1 = ks * T::KSTEP + VEC * g;
            const typename T::frag zf =
                *reinterpret_cast<const typename T::frag*>(Zt + (x2 * 16 + l16) * ldz + k1);
            const typename T::frag mf = *reinterpret_cast<const typename T::frag*>(
                M1 + (int64_t)(x1 * 16 + l16) * a.ldm1 + k1);
            acc = T::mma(zf, mf, acc);
        }
        const int j1 = x1 * 16 + l16;
        if (j1 < a.J1) {
            if constexpr (T::CONSEC) {
                const int j2 = x2 * 16 + 4 * g;
                Tout* dst = Y + (int64_t)j1 * a.J2 + j2;
                if ((a.J2 % 4) == 0 && j2 + 4 <= a.J2) {
                    typedef Tout __attribute__((ext_vector_type(4))) vout;
                    vout o;
#pragma unroll
                    for (int r = 0; r < 4; ++r) o[r] = cvt<Tout>(acc[r]);
                    *reinterpret_cast<vout*>(dst) = o;
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (j2 + r < a.J2) dst[r] = cvt<Tout>(acc[r]);
                }
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j2 = x2 * 16 + T::arow(lane, r);
                    if (j2 < a.J2) Y[(int64_t)j1 * a.J2 + j2] = cvt<Tout>(acc[r]);
                }
            }
        }
    }
    __syncthreads();  // Zt is reused by the next block
}

// ---------------------------------------------------------------------------
// Contiguous (last-mode) pass: Y[row][j] = sum_k X[row][k] M[j][k] with
// D[j][row] = M x X^T so a lane owns 4 consecutive j of one row.  Each wave
// handles 16 rows and JT j tiles starting at a.j0.
template <typename Tin, typename Tout, typename Tc, int JT>
__device__ __forceinline__ void contig_rows(const ContigArgs& a, int64_t rtile) {
    typedef MT<Tc> T;
    constexpr int VEC = T::VEC;
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, l16 = lane & 15;
    const int64_t row = rtile * 16 + l16;
    const Tin* __restrict__ X = reinterpret_cast<const Tin*>(a.X);
    Tout* __restrict__ Y = reinterpret_cast<Tout*>(a.Y);
    const Tc* __restrict__ M = reinterpret_cast<const Tc*>(a.M);
    typename T::acc acc[JT];
#pragma unroll
    for (int x = 0; x < JT; ++x) acc[x] = T::zero();
    const int nks = a.kpad / T::KSTEP;
    for (int ks = 0; ks < nks; ++ks) {
        const int k = ks * T::KSTEP + VEC * g;
        const int nv = (row < a.rows) ? max(0, min(VEC, a.K - k)) : 0;
        const typename T::frag xf =
            (nv > 0) ? load_frag<Tc>(X + row * a.K + k, nv, (a.K % VEC) == 0) : T::zfrag();
#pragma unroll
        for (int x = 0; x < JT; ++x) {
            const typename T::frag mf = *reinterpret_cast<const typename T::frag*>(
                M + (int64_t)(a.j0 + x * 16 + l16) * a.ldm + k);
            acc[x] = T::mma(mf, xf, acc[x]);
        }
    }
    if (row >= a.rows) return;
#pragma unroll
    for (int x = 0; x < JT; ++x) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = a.j0 + x * 16 + T::arow(lane, r);
            if (j < a.J) Y[row * a.J + j] = cvt<Tout>(acc[x][r]);
        }
    }
}

}  // namespace cta
