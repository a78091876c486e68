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
    // division by stride[k] and ext[k] as multiply-high and shift (see
    // fastdiv_init); valid for dividends below 2^31
    uint32_t smul[8], emul[8];
    int sshift[8], eshift[8];
};

// floor(n / d) for n < 2^31 from (mul, shift) = fastdiv_init(d)
__device__ __forceinline__ int fast_div(int n, uint32_t mul, int shift) {
    return (int)((__umulhi(mul, (uint32_t)n) + (uint32_t)n) >> shift);
}

// floor(n / d) for 0 <= n < 2^22 and d >= 1, with inv = 1.0f / d: the float
// quotient is within one of the exact one, and one correction step fixes it
// (a few instructions instead of an integer division)
__device__ __forceinline__ int small_div(int n, int d, float inv) {
    int q = (int)((float)n * inv);
    const int r = n - q * d;
    q += (r >= d) - (r < 0);
    return q;
}

struct StridedArgs {
    const void* X;
    void* Y;
    const void* M;   // Tc, row-major [>= JPAD][ldm], zero padded
    int ldm;
    int K, J, kpad;  // kpad: K rounded up to the MFMA KSTEP
    int64_t lead, trail;
    int64_t ntt;     // t tiles per b
    int64_t ntiles;  // lead * ntt
    // Tile order of the normal-operator last pass (lead == 1).  pgroup == 0:
    // tile i covers columns [i*TN, (i+1)*TN).  pgroup > 0: the trail is
    // nplane planes of `plane` columns (plane % TN == 0, nplane % pgroup == 0);
    // consecutive tiles walk the plane index fastest within groups of pgroup
    // planes, so the neighbours that the regulariser reads along the plane
    // mode are loaded by tiles that run at nearly the same time.
    int64_t plane;
    int nplane, pgroup;
    // Persistent last pass: xsweep != 0 gives the workgroups of XCD x (block
    // index mod 8) the contiguous tile range [x per, (x + 1) per), per =
    // ceil(ntiles / 8), walked by its blocks in steps of their count, so that
    // the tiles of one XCD sweep one block of planes and the regulariser's
    // neighbour loads find the neighbouring tiles in that XCD's L2.
    int xsweep;
    // flattened-column pass (strided_flat_tile): division by trail
    uint32_t tmul;
    int tshift;
};

// First column of tile `tile` of the last pass (see StridedArgs::pgroup).
template <int TN>
__device__ __forceinline__ int64_t last_tile_col(const StridedArgs& a, int64_t tile) {
    if (a.pgroup <= 0) return tile * TN;
    const int64_t cpp = a.plane / TN;            // tiles per plane
    const int64_t per = cpp * a.pgroup;          // tiles per group of planes
    const int64_t grp = tile / per, r = tile - grp * per;
    const int64_t c = r / a.pgroup, ig = r - c * a.pgroup;
    return (grp * a.pgroup + ig) * a.plane + c * TN;
}

struct TailArgs {
    int nbg;         // blocks per workgroup group
    const void* X;   // (nblk, K1, K2)  (or r when fused with the p update)
    void* Y;         // (nblk, J1, J2)
    const void* M1;  // Tc [>= J1 pad][ldm1]
    const void* M2;  // Tc [>= J2 pad][ldm2]
    int ldm1, ldm2;
    int K1, K2, J1, J2;
    int k1pad, k2pad;  // K1 rounded up to max(KSTEP, 16), K2 to KSTEP
    int64_t nblk;
    // fused CG direction update p = r + beta p (the chain input is the new p);
    // with Xsol, the previous step's x += alpha p (p before its update) is
    // applied on the same pass, since p is read there anyway
    void* Pvec;
    const double* beta;
    const int* done;
    void* Xsol;
    const double* alpha;
    // fused residual update (preconditioned CG): the chain input is
    // r = r - alpha q, written back to Pvec (r) with q = Qvec, and the FP64
    // partial sums of <r, r> go to partials[blockIdx.x]
    const void* Qvec;
    double* partials;
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
// Stage TN columns of K rows into LDS transposed, Xs[c * ldx + k] in Tc, rows
// K..kpad-1 zero.  A unit is VEC rows x LV columns (one 16-byte load per row);
// col(tc) gives the address of row 0 of the LV columns tc*LV.. and whether
// they exist (when not, the address must still be readable and the unit is
// stored as zero).  Rows are `pitch` elements apart.  Row indices are clamped
// so every load is valid, and the loads of UB units are issued before the
// first LDS write, so a thread keeps UB * VEC loads in flight instead of one
// (units past the last whole batch of UB * CTA_WG go one at a time).
template <typename Tin>
struct ColPtr {
    const Tin* p;
    bool ok;
};

template <typename Tin, typename Tc, int TN, typename ColFn>
__device__ __forceinline__ void stage_units(ColFn col, int64_t pitch, int K, int kpad, Tc* Xs,
                                            int ldx) {
    typedef MT<Tc> T;
    constexpr int VEC = T::VEC;
    constexpr int LV = 16 / sizeof(Tin);
    constexpr int TCH = TN / LV;  // 16-byte chunks per slab row
    constexpr int UB = 4;
    typedef Tin __attribute__((ext_vector_type(LV))) vin;
    const int nunits = (kpad / VEC) * TCH;
    auto store = [&](int u, const vin (&v)[VEC], bool ok) {
        const int tc = u % TCH, kg = u / TCH;
#pragma unroll
        for (int c = 0; c < LV; ++c) {
            typename T::frag f;
#pragma unroll
            for (int r = 0; r < VEC; ++r)
                f[r] = ok && kg * VEC + r < K ? cvt<Tc>(v[r][c]) : cvt<Tc>(0.f);
            *reinterpret_cast<typename T::frag*>(Xs + (tc * LV + c) * ldx + kg * VEC) = f;
        }
    };
    const int nfull = nunits / (CTA_WG * UB) * (CTA_WG * UB);
    for (int u0 = threadIdx.x; u0 < nfull; u0 += CTA_WG * UB) {
        vin v[UB][VEC];
        bool ok[UB];
#pragma unroll
        for (int i = 0; i < UB; ++i) {
            const int u = u0 + i * CTA_WG;
            const int tc = u % TCH, kg = u / TCH;
            const auto cp = col(tc);
            ok[i] = cp.ok;
#pragma unroll
            for (int r = 0; r < VEC; ++r) {
                const int k = min(kg * VEC + r, K - 1);
                v[i][r] = *reinterpret_cast<const vin*>(cp.p + (int64_t)k * pitch);
            }
        }
#pragma unroll
        for (int i = 0; i < UB; ++i) store(u0 + i * CTA_WG, v[i], ok[i]);
    }
    for (int u = nfull + threadIdx.x; u < nunits; u += CTA_WG) {
        const int tc = u % TCH, kg = u / TCH;
        const auto cp = col(tc);
        vin v[VEC];
#pragma unroll
        for (int r = 0; r < VEC; ++r) {
            const int k = min(kg * VEC + r, K - 1);
            v[r] = *reinterpret_cast<const vin*>(cp.p + (int64_t)k * pitch);
        }
        store(u, v, cp.ok);
    }
}

// Stage columns [t0, t0 + TN) of a row-major K x ncol slab X (row pitch
// `pitch` elements) into LDS transposed (see stage_units); columns at or past
// ncol are zero.  Interior tiles take the batched path of stage_units.
template <typename Tin, typename Tc, int TN>
__device__ __forceinline__ void stage_cols(const Tin* __restrict__ X, int64_t pitch, int K,
                                           int kpad, int64_t t0, int64_t ncol, Tc* Xs, int ldx) {
    typedef MT<Tc> T;
    constexpr int VEC = T::VEC;
    constexpr int LV = 16 / sizeof(Tin);
    constexpr int TCH = TN / LV;
    typedef Tin __attribute__((ext_vector_type(LV))) vin;
    const int nunits = (kpad / VEC) * TCH;
    if ((pitch % LV) == 0 && t0 + TN <= ncol) {
        const Tin* __restrict__ Xt = X + t0;
        stage_units<Tin, Tc, TN>([&](int tc) { return ColPtr<Tin>{Xt + tc * LV, true}; }, pitch, K,
                                 kpad, Xs, ldx);
        return;
    }
    const bool vec_ok = (pitch % LV) == 0;
    for (int u = threadIdx.x; u < nunits; u += CTA_WG) {
        const int tc = u % TCH;
        const int kg = u / TCH;
        const int64_t t = t0 + (int64_t)tc * LV;
        Tin v[VEC][LV];
#pragma unroll
        for (int r = 0; r < VEC; ++r) {
            const int k = kg * VEC + r;
            if (k < K && vec_ok && t + LV <= ncol) {
                vin x = *reinterpret_cast<const vin*>(X + (int64_t)k * pitch + t);
#pragma unroll
                for (int c = 0; c < LV; ++c) v[r][c] = x[c];
            } else {
#pragma unroll
                for (int c = 0; c < LV; ++c)
                    v[r][c] = (k < K && t + c < ncol) ? X[(int64_t)k * pitch + t + c] : cvt<Tin>(0.f);
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
}

// ---------------------------------------------------------------------------
// acc[x][y] += Xs columns (cb + 16y ...) times M rows (jb + 16x ...) over kpad.
// The M fragments of the next k step are loaded while the current one
// multiplies (M is read from the cache hierarchy, not LDS, so its latency is
// hidden by the MFMAs of the step before).
template <typename Tc, int JT, int CT>
__device__ __forceinline__ void mfma_cols(const Tc* Xs, int ldx, const Tc* __restrict__ M, int ldm,
                                          int cb, int jb, int kpad,
                                          typename MT<Tc>::acc (&acc)[JT][CT]) {
    typedef MT<Tc> T;
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, l16 = lane & 15;
    const int nks = kpad / T::KSTEP;
    const Tc* mrow[JT];
#pragma unroll
    for (int x = 0; x < JT; ++x) mrow[x] = M + (int64_t)(jb + x * 16 + l16) * ldm + T::VEC * g;
    typename T::frag mb[JT];
#pragma unroll
    for (int x = 0; x < JT; ++x) mb[x] = *reinterpret_cast<const typename T::frag*>(mrow[x]);
    for (int ks = 0; ks < nks; ++ks) {
        const int k0 = ks * T::KSTEP + T::VEC * g;
        const int kn = (ks + 1 < nks ? ks + 1 : ks) * T::KSTEP;
        typename T::frag xa[CT], mn[JT];
#pragma unroll
        for (int x = 0; x < JT; ++x) mn[x] = *reinterpret_cast<const typename T::frag*>(mrow[x] + kn);
#pragma unroll
        for (int y = 0; y < CT; ++y)
            xa[y] = *reinterpret_cast<const typename T::frag*>(Xs + (cb + y * 16 + l16) * ldx + k0);
#pragma unroll
        for (int x = 0; x < JT; ++x)
#pragma unroll
            for (int y = 0; y < CT; ++y) acc[x][y] = T::mma(xa[y], mb[x], acc[x][y]);
#pragma unroll
        for (int x = 0; x < JT; ++x) mb[x] = mn[x];
    }
}

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
    stage_cols<Tin, Tc, TN>(X, a.trail, a.K, a.kpad, t0, a.trail, Xs, ldx);
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
    mfma_cols<Tc, JT, CT>(Xs, ldx, M, a.ldm, cb, jb, a.kpad, acc);

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
// Strided pass over flattened columns: the lead * trail columns (b, t) are
// numbered c = b * trail + t and tiled TN at a time across b, so a trail that
// is short or not a multiple of TN wastes no MFMA columns.  Needs
// trail % LV == 0 (a 16-byte unit never straddles two b), trail % 4 == 0 when
// T::CONSEC (nor does a 4-column output run) and lead * trail < 2^31.
template <typename Tin, typename Tout, typename Tc, int JT, int WJ, int CT>
__device__ __forceinline__ void strided_flat_tile(const StridedArgs& a, int64_t tile, Tc* Xs) {
    typedef MT<Tc> T;
    constexpr int WC = CTA_WAVES / WJ;
    constexpr int TN = 16 * CT * WC;
    constexpr int LV = 16 / sizeof(Tin);
    const int ldx = a.kpad + 16 / (int)sizeof(Tc);
    const int trail = (int)a.trail;
    const int ncol = (int)(a.lead * a.trail);
    const int c0 = (int)tile * TN;
    const int64_t bin = (int64_t)a.K * trail, bout = (int64_t)a.J * trail;
    const Tin* __restrict__ X = reinterpret_cast<const Tin*>(a.X);
    Tout* __restrict__ Y = reinterpret_cast<Tout*>(a.Y);
    const Tc* __restrict__ M = reinterpret_cast<const Tc*>(a.M);

    stage_units<Tin, Tc, TN>(
        [&](int tc) {
            const int c = c0 + tc * LV;
            const bool ok = c < ncol;
            const int cc = ok ? c : 0;
            const int b = fast_div(cc, a.tmul, a.tshift);
            return ColPtr<Tin>{X + b * bin + (cc - b * trail), ok};
        },
        trail, a.K, a.kpad, Xs, ldx);
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wj = wave % WJ, wc = wave / WJ;
    const int cb = wc * CT * 16, jb = wj * JT * 16;
    const int g = lane >> 4, l16 = lane & 15;
    typename T::acc acc[JT][CT];
#pragma unroll
    for (int x = 0; x < JT; ++x)
#pragma unroll
        for (int y = 0; y < CT; ++y) acc[x][y] = T::zero();
    mfma_cols<Tc, JT, CT>(Xs, ldx, M, a.ldm, cb, jb, a.kpad, acc);

#pragma unroll
    for (int x = 0; x < JT; ++x) {
        const int j = jb + x * 16 + l16;
        if (j >= a.J) continue;
#pragma unroll
        for (int y = 0; y < CT; ++y) {
            const int cbase = c0 + cb + y * 16;
            if constexpr (T::CONSEC) {
                const int c = cbase + 4 * g;
                if (c >= ncol) continue;
                const int b = fast_div(c, a.tmul, a.tshift);
                typedef Tout __attribute__((ext_vector_type(4))) vout;
                vout o;
#pragma unroll
                for (int r = 0; r < 4; ++r) o[r] = cvt<Tout>(acc[x][y][r]);
                *reinterpret_cast<vout*>(Y + b * bout + (int64_t)j * trail + (c - b * trail)) = o;
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = cbase + T::arow(lane, r);
                    if (c >= ncol) continue;
                    const int b = fast_div(c, a.tmul, a.tshift);
                    Y[b * bout + (int64_t)j * trail + (c - b * trail)] = cvt<Tout>(acc[x][y][r]);
                }
            }
        }
    }
    __syncthreads();  // Xs is reused by the next tile
}

// ---------------------------------------------------------------------------
// Normal-operator last pass (mode 1 of a (K, trail) tensor, lead == 1):
//   Q[j, t] = sum_i M[j, i] X[i, t] + lam * sum_k (P x_k R_k)[j, t],  dot += P Q.
// LDS holds the transposed X tile (MFMA operand), then -- reusing that space --
// the MFMA result Qs[j][c]; beside it a window of P (all K rows, TN + 8
// columns with 4 columns of halo per side) and the band rows of R_1 and R_N.
// The epilogue runs one item per thread per iteration: E = 16 / sizeof(Tv)
// consecutive columns of one row, so global loads and stores are 16-byte
// vectors and consecutive threads touch consecutive memory.  Modes 1 and N
// of the regulariser read the window; the modes in between (strides of whole
// mode-N rows) read P from memory.  Index arithmetic is 32-bit (the launcher
// checks trail < 2^30).
template <typename Tv>
struct LastLds {
    static constexpr int H = 4;  // halo columns per side
};

// NORD > 0 fixes the tensor order at compile time (the batched solver uses 3),
// so the per-mode loops unroll with constant indices.
template <typename Tin, typename Tv, typename Tc, int JT, int WJ, int CT, int NORD = 0>
__device__ __forceinline__ void normal_last_tile(const StridedArgs& a, int64_t tile,
                                                 unsigned char* smem, const StencilArgs<Tv>& st,
                                                 double& dot_acc) {
    typedef MT<Tc> T;
    constexpr int WC = CTA_WAVES / WJ;
    constexpr int TN = 16 * CT * WC;
    constexpr int VEC = T::VEC;
    constexpr int LV = 16 / sizeof(Tin);
    constexpr int E = 16 / sizeof(Tv);      // epilogue item width (one 16-byte vector)
    constexpr int H = LastLds<Tv>::H;
    constexpr int LDP = TN + 2 * H;         // P window pitch
    constexpr int LDQ = TN + E;             // Qs pitch
    typedef Tv __attribute__((ext_vector_type(E))) vt;
    const int ldx = a.kpad + 16 / (int)sizeof(Tc);
    const int K = a.K;
    const int trail = (int)a.trail;
    const int t0 = (int)last_tile_col<TN>(a, tile);
    const int N = NORD > 0 ? NORD : st.order;
    const int nN = (int)st.ext[N - 1];
    const size_t xs_bytes = (size_t)TN * ldx * sizeof(Tc);
    const size_t qs_bytes = (size_t)a.J * LDQ * sizeof(Tv);
    const size_t a_bytes = (xs_bytes > qs_bytes ? xs_bytes : qs_bytes + 0);
    Tc* Xs = reinterpret_cast<Tc*>(smem);
    Tv* Qs = reinterpret_cast<Tv*>(smem);
    Tv* Pw = reinterpret_cast<Tv*>(smem + ((a_bytes + 15) / 16) * 16);
    Tv* band1 = Pw + (size_t)K * LDP;
    Tv* bandN = band1 + (size_t)K * 5;
    const bool has1 = st.rband[0] != nullptr;
    const bool hasN = st.rband[N - 1] != nullptr;
    const Tin* __restrict__ X = reinterpret_cast<const Tin*>(a.X);
    Tv* __restrict__ Q = reinterpret_cast<Tv*>(a.Y);
    const Tv* __restrict__ P = st.P;
    const Tc* __restrict__ M = reinterpret_cast<const Tc*>(a.M);

    // ---- stage the X tile (transposed, Tc) ----
    stage_cols<Tin, Tc, TN>(X, trail, K, a.kpad, t0, trail, Xs, ldx);
    // ---- stage the P window and the band rows ----
    const bool pvec = (trail % E) == 0;
    {
        constexpr int PCH = LDP / E;
        for (int u = threadIdx.x; u < K * PCH; u += CTA_WG) {
            const int row = u / PCH, ch = u % PCH;
            const int t = t0 - H + ch * E;
            const Tv* src = P + (int64_t)row * trail + t;
            Tv* dst = Pw + row * LDP + ch * E;
            if (pvec && t >= 0 && t + E <= trail) {
                *reinterpret_cast<vt*>(dst) = *reinterpret_cast<const vt*>(src);
            } else {
#pragma unroll
                for (int c = 0; c < E; ++c) dst[c] = (t + c >= 0 && t + c < trail) ? src[c] : Tv(0);
            }
        }
        if (has1)
            for (int u = threadIdx.x; u < K * 5; u += CTA_WG) band1[u] = st.rband[0][u];
        if (hasN)
            for (int u = threadIdx.x; u < nN * 5; u += CTA_WG) bandN[u] = st.rband[N - 1][u];
    }
    __syncthreads();

    // ---- MFMA ----
    {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int wj = wave % WJ, wc = wave / WJ;
        const int cb = wc * CT * 16, jb = wj * JT * 16;
        const int g = lane >> 4, l16 = lane & 15;
        typename T::acc acc[JT][CT];
#pragma unroll
        for (int x = 0; x < JT; ++x)
#pragma unroll
            for (int y = 0; y < CT; ++y) acc[x][y] = T::zero();
        mfma_cols<Tc, JT, CT>(Xs, ldx, M, a.ldm, cb, jb, a.kpad, acc);
        __syncthreads();  // Xs is dead; its space becomes Qs
#pragma unroll
        for (int x = 0; x < JT; ++x) {
            const int j = jb + x * 16 + l16;
            if (j >= a.J) continue;
#pragma unroll
            for (int y = 0; y < CT; ++y) {
                if constexpr (T::CONSEC && E == 4) {
                    vt o;
#pragma unroll
                    for (int r = 0; r < 4; ++r) o[r] = cvt<Tv>(acc[x][y][r]);
                    *reinterpret_cast<vt*>(Qs + j * LDQ + cb + y * 16 + 4 * g) = o;
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        Qs[j * LDQ + cb + y * 16 + T::arow(lane, r)] = cvt<Tv>(acc[x][y][r]);
                }
            }
        }
    }
    __syncthreads();

    // ---- epilogue: one item = E consecutive columns of one row ----
    const Tv lam = (Tv)st.lam;
    const bool fast = pvec && (nN % E) == 0;
    constexpr int GPR = TN / E;  // items per row
#pragma unroll 2
    for (int it = threadIdx.x; it < a.J * GPR; it += CTA_WG) {
        const int j = it / GPR;
        const int c = (it - j * GPR) * E;
        const int t = t0 + c;
        if (t >= trail) continue;
        const Tv* prow = Pw + j * LDP + H + c;  // prow[0] is P[j][t]
        const int64_t base = (int64_t)j * trail + t;
        if (fast) {
            // Branch-free taps: a tap outside the tensor has a zero band
            // coefficient (R_k[i][i+d] with i+d out of range is stored as 0), so
            // its address is clamped to a valid one instead of tested.
            const vt pc = *reinterpret_cast<const vt*>(prow);
            vt s = *reinterpret_cast<const vt*>(Qs + j * LDQ + c);  // chain part, lam applied below
            vt reg;
#pragma unroll
            for (int e = 0; e < E; ++e) reg[e] = Tv(0);
            // summation order (kept by every last-pass variant): the middle modes,
            // then mode 1, then mode N
            const Tv* __restrict__ pb = P + base;
            for (int k = 1; k < N - 1; ++k) {
                const Tv* __restrict__ rb = st.rband[k];
                if (!rb) continue;
                const int sk = (int)st.stride[k], nk = (int)st.ext[k];
                const int u = fast_div(t, st.smul[k], st.sshift[k]);
                const int ik = u - fast_div(u, st.emul[k], st.eshift[k]) * nk;
                const Tv* br = rb + ik * 5;
                vt nbv[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int d = q < 2 ? q - 2 : q - 1;  // -2, -1, 1, 2
                    const int dd = (ik + d >= 0 && ik + d < nk) ? d : 0;
                    nbv[q] = *reinterpret_cast<const vt*>(pb + dd * sk);
                }
                reg += br[2] * pc;
#pragma unroll
                for (int q = 0; q < 4; ++q) reg += br[q < 2 ? q : q + 1] * nbv[q];
            }
            if (has1) {
#pragma unroll
                for (int d = -2; d <= 2; ++d) {
                    const int jj = min(max(j + d, 0), K - 1);
                    reg += band1[j * 5 + d + 2] * *reinterpret_cast<const vt*>(Pw + jj * LDP + H + c);
                }
            }
            if (hasN) {
                Tv w[3 * E];
                const vt pl = *reinterpret_cast<const vt*>(prow - E);
                const vt pr = *reinterpret_cast<const vt*>(prow + E);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    w[e] = pl[e];
                    w[E + e] = pc[e];
                    w[2 * E + e] = pr[e];
                }
                const int i0 = t - fast_div(t, st.emul[N - 1], st.eshift[N - 1]) * nN;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const Tv* bN = bandN + (i0 + e) * 5;
#pragma unroll
                    for (int d = -2; d <= 2; ++d) reg[e] += bN[d + 2] * w[E + e + d];
                }
            }
            const vt qv = s + lam * reg;
            *reinterpret_cast<vt*>(Q + base) = qv;
#pragma unroll
            for (int e = 0; e < E; ++e) dot_acc += (double)pc[e] * (double)qv[e];
        } else {
            for (int e = 0; e < E && t + e < trail; ++e) {
                const int te = t + e;
                const int64_t be = base + e;
                Tv sv = Tv(0);
                for (int k = 0; k < N; ++k) {
                    const Tv* __restrict__ rb = st.rband[k];
                    if (!rb) continue;
                    const int sk = (int)st.stride[k], nk = (int)st.ext[k];
                    const int ik = (k == 0) ? j : (te / sk) % nk;
                    const Tv* br = rb + ik * 5;
                    for (int d = -2; d <= 2; ++d)
                        if (ik + d >= 0 && ik + d < nk) sv += br[d + 2] * P[be + (int64_t)d * sk];
                }
                const Tv pv = P[be];
                const Tv qv = Qs[j * LDQ + c + e] + lam * sv;
                Q[be] = qv;
                dot_acc += (double)pv * (double)qv;
            }
        }
    }
    __syncthreads();  // LDS is reused by the next tile
}

// LDS bytes of normal_last_tile.
template <typename Tv, typename Tc, int TN>
inline size_t normal_last_lds(int kpad, int K, int J, int nN) {
    const size_t xs = (size_t)TN * (kpad + 16 / sizeof(Tc)) * sizeof(Tc);
    const size_t qs = (size_t)J * (TN + 16 / sizeof(Tv)) * sizeof(Tv);
    const size_t a = ((xs > qs ? xs : qs) + 15) / 16 * 16;
    return a + (size_t)K * (TN + 2 * LastLds<Tv>::H) * sizeof(Tv) + (size_t)(K + nN) * 5 * sizeof(Tv);
}

// ---------------------------------------------------------------------------
// Pipelined form of normal_last_tile for BF16 chains with FP32 vectors, 32
// columns per tile, persistent workgroups: the global loads of the next tile
// (its X tile, two 16-byte rows per thread, and its P window) are issued into
// registers before the current tile's MFMA and epilogue and written to LDS
// after them, so they are in flight while the current tile computes.  The
// band coefficients are staged once per workgroup.  Same sums in the same
// order as normal_last_tile (identical Q).
template <int NT>
struct PipeRegsT {
    bf16x8 x[2];                     // rows 2 kp, 2 kp + 1 of the X tile, 8 columns (threads < 256)
    floatx4 p[(1280 + NT - 1) / NT]; // P window chunks owned by this thread (K <= 128 rows x 10 chunks)
};
typedef PipeRegsT<CTA_WG> PipeRegs;

constexpr int PIPE_TN = 32;
constexpr int PIPE_H = 4;
constexpr int PIPE_LDP = PIPE_TN + 2 * PIPE_H;   // 40 floats: 10 chunks of 4 per row

template <int KPAD, int NT = CTA_WG>
__device__ __forceinline__ void pipe_load(const StridedArgs& a, const float* __restrict__ P, int t0, int K,
                                          PipeRegsT<NT>& r) {
    const bf16* __restrict__ X = reinterpret_cast<const bf16*>(a.X);
    const int trail = (int)a.trail;
    // X: unit = (row pair kp, column group cg of 8), cg fastest so that 4 lanes read a row's 64 bytes;
    // the first 256 threads own the 256 units
    if (NT == 256 || threadIdx.x < 256) {
        const int cg = threadIdx.x & 3, kp = threadIdx.x >> 2;  // kp < 64 covers K <= 128
        const int t = t0 + cg * 8;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = 2 * kp + h;
            bf16x8 v;
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = (bf16)0.f;
            if (k < K) v = *reinterpret_cast<const bf16x8*>(X + (int64_t)k * trail + t);
            r.x[h] = v;
        }
    }
    // P window: K rows x 10 chunks of 4 floats, chunk u = threadIdx.x + NT i
#pragma unroll
    for (int i = 0; i < (1280 + NT - 1) / NT; ++i) {
        const int u = threadIdx.x + NT * i;
        const int row = u / 10, ch = u - row * 10;
        const int t = t0 - PIPE_H + ch * 4;
        floatx4 v = {0.f, 0.f, 0.f, 0.f};
        if (row < K && t >= 0 && t < trail) v = *reinterpret_cast<const floatx4*>(P + (int64_t)row * trail + t);
        r.p[i] = v;
    }
}

template <int KPAD, int NT = CTA_WG>
__device__ __forceinline__ void pipe_store(const PipeRegsT<NT>& r, bf16* Xs, float* Pw, int K) {
    constexpr int ldx = KPAD + 8;
    if (NT == 256 || threadIdx.x < 256) {
        const int cg = threadIdx.x & 3, kp = threadIdx.x >> 2;
        if (2 * kp < KPAD) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                typedef bf16 __attribute__((ext_vector_type(2))) bf16x2;
                bf16x2 pr;
                pr[0] = r.x[0][c];
                pr[1] = r.x[1][c];
                *reinterpret_cast<bf16x2*>(Xs + (cg * 8 + c) * ldx + 2 * kp) = pr;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < (1280 + NT - 1) / NT; ++i) {
        const int u = threadIdx.x + NT * i;
        const int row = u / 10, ch = u - row * 10;
        if (row < K) *reinterpret_cast<floatx4*>(Pw + row * PIPE_LDP + ch * 4) = r.p[i];
    }
}

// Middle-mode regulariser taps of a thread's IPT items (the band rows of R_k,
// k = 2 .. N-1): rmid[i] += R_k taps of P around the item's E columns, modes in
// ascending order and, per mode, the centre first and then the offsets -2, -1,
// +1, +2 (out-of-range offsets read the centre against a zero coefficient).
// Item i of a thread is row j = threadIdx.x / GPR + i * (NT / GPR) at the
// column c = (threadIdx.x % GPR) * E of every item, so the mode index, its band
// row and the neighbour offsets are formed once per mode.  Rows past J - 1 read
// row J - 1 and are not used.  P is addressed with 32-bit byte offsets from its
// base (the launcher checks that P spans less than 4 GiB).
template <int IPT, int GPR, int E, int LDP, int H, int NT = CTA_WG>
__device__ __forceinline__ void mid_taps(const StencilArgs<float>& st, const float* Pw, int J, int trail,
                                         int t0, floatx4 (&rmid)[IPT]) {
    typedef floatx4 vt;
    const char* __restrict__ Pb = reinterpret_cast<const char*>(st.P);
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));   // rows and offsets are re-formed per tile, not held in registers
    const int c = (tid % GPR) * E;
    const int t = t0 + c;
    const int N = st.order;
    for (int k = 1; k < N - 1; ++k) {
        const float* __restrict__ rb = st.rband[k];
        if (!rb) continue;
        const int sk = (int)st.stride[k], nk = (int)st.ext[k];
        const int u = fast_div(t, st.smul[k], st.sshift[k]);
        const int ik = u - fast_div(u, st.emul[k], st.eshift[k]) * nk;
        const float* br = rb + ik * 5;
        const float b0 = br[0], b1 = br[1], b2 = br[2], b3 = br[3], b4 = br[4];
        uint32_t off[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int d = q < 2 ? q - 2 : q - 1;  // -2, -1, 1, 2
            const int dd = (ik + d >= 0 && ik + d < nk) ? d : 0;
            off[q] = (uint32_t)(dd * sk) * 4u;
        }
#pragma unroll 2
        for (int i = 0; i < IPT; ++i) {   // at most two items' gathers in flight
            const int j = min(tid / GPR + i * (NT / GPR), J - 1);
            const vt pc = *reinterpret_cast<const vt*>(Pw + j * LDP + H + c);
            const uint32_t base = (uint32_t)(j * trail + t) * 4u;
            vt nbv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) nbv[q] = *reinterpret_cast<const vt*>(Pb + (base + off[q]));
            rmid[i] += b2 * pc;
            rmid[i] += b0 * nbv[0];
            rmid[i] += b1 * nbv[1];
            rmid[i] += b3 * nbv[2];
            rmid[i] += b4 * nbv[3];
        }
    }
}

// Persistent, pipelined last pass (see PipeRegs); K <= 128, kpad == 128.
__device__ __forceinline__ void normal_last_pipe(const StridedArgs& a, unsigned char* smem,
                                                 const StencilArgs<float>& st, double& dot_acc,
                                                 int64_t first, int64_t step) {
    typedef MT<bf16> T;
    typedef float Tv;
    typedef floatx4 vt;
    constexpr int KPAD = 128;
    constexpr int TN = PIPE_TN, H = PIPE_H, LDP = PIPE_LDP;
    constexpr int E = 4, LDQ = TN + E, VEC = T::VEC;
    constexpr int JT = 2, CT = 2;
    const int K = a.K;
    const int trail = (int)a.trail;
    const int N = st.order;
    const int nN = (int)st.ext[N - 1];
    constexpr int ldx = KPAD + 8;
    constexpr size_t a_bytes = ((size_t)(TN * ldx * 2) > (size_t)(KPAD * LDQ * 4) ? (size_t)(TN * ldx * 2)
                                                                                    : (size_t)(KPAD * LDQ * 4));
    bf16* Xs = reinterpret_cast<bf16*>(smem);
    float* Qs = reinterpret_cast<float*>(smem);
    float* Pw = reinterpret_cast<float*>(smem + (a_bytes + 15) / 16 * 16);
    float* band1 = Pw + (size_t)KPAD * LDP;
    float* bandN = band1 + (size_t)KPAD * 5;
    const bool has1 = st.rband[0] != nullptr;
    const bool hasN = st.rband[N - 1] != nullptr;
    float* __restrict__ Q = reinterpret_cast<float*>(a.Y);
    const float* __restrict__ P = st.P;
    const bf16* __restrict__ M = reinterpret_cast<const bf16*>(a.M);
    // first column of a tile (last_tile_col) with 32-bit quotients from float
    // reciprocals: the tile count is below 2^22 (checked by the launcher)
    const int cpp = (int)(a.plane / TN), per = cpp * a.pgroup;
    const float inv_per = a.pgroup > 0 ? 1.0f / (float)per : 0.f;
    const float inv_pg = a.pgroup > 0 ? 1.0f / (float)a.pgroup : 0.f;
    auto tcol = [&](int64_t tl) -> int {
        const int t = (int)tl;
        if (a.pgroup <= 0) return t * TN;
        const int grp = small_div(t, per, inv_per), rr = t - grp * per;
        const int c = small_div(rr, a.pgroup, inv_pg), ig = rr - c * a.pgroup;
        return (grp * a.pgroup + ig) * (int)a.plane + c * TN;
    };
    PipeRegs r;
    if (first < a.ntiles) pipe_load<KPAD>(a, P, tcol(first), K, r);
    if (has1)
        for (int u = threadIdx.x; u < K * 5; u += CTA_WG) band1[u] = st.rband[0][u];
    if (hasN)
        for (int u = threadIdx.x; u < nN * 5; u += CTA_WG) bandN[u] = st.rband[N - 1][u];
    const Tv lam = (Tv)st.lam;
    // Order of the memory traffic inside one tile.  The vector-memory counter
    // retires loads in issue order, so a load waits for every load issued
    // before it.  The middle-mode taps (gathered from memory) therefore come
    // first, then the MFMA with its G_1 fragments, and only then the prefetch
    // of the next tile, which lands while the epilogue runs on LDS alone.
    constexpr int GPR = TN / E;                 // items per row
    constexpr int IPT = KPAD * GPR / CTA_WG;    // items per thread (rows <= KPAD)
    const int nitem = a.J * GPR;
    for (int64_t tile = first; tile < a.ntiles; tile += step) {
        const int t0 = tcol(tile);
        pipe_store<KPAD>(r, Xs, Pw, K);
        __syncthreads();
        // ---- middle-mode regulariser taps of this tile's items ----
        // (summed first: the order of every last-pass variant is the middle
        // modes, then mode 1, then mode N)
        vt rmid[IPT];
#pragma unroll
        for (int i = 0; i < IPT; ++i)
#pragma unroll
            for (int e = 0; e < E; ++e) rmid[i][e] = Tv(0);
        mid_taps<IPT, GPR, E, LDP, H>(st, Pw, a.J, trail, t0, rmid);
        // ---- MFMA (as normal_last_tile with JT = 2, WJ = 4, CT = 2) ----
        {
            const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
            const int jb = wave * JT * 16;
            const int g = lane >> 4, l16 = lane & 15;
            typename T::acc acc[JT][CT];
#pragma unroll
            for (int x = 0; x < JT; ++x)
#pragma unroll
                for (int y = 0; y < CT; ++y) acc[x][y] = T::zero();
            mfma_cols<bf16, JT, CT>(Xs, ldx, M, a.ldm, 0, jb, KPAD, acc);
            if (tile + step < a.ntiles) pipe_load<KPAD>(a, P, tcol(tile + step), K, r);
            __syncthreads();  // Xs is dead; its space becomes Qs
#pragma unroll
            for (int x = 0; x < JT; ++x) {
                const int j = jb + x * 16 + l16;
                if (j >= a.J) continue;
#pragma unroll
                for (int y = 0; y < CT; ++y) {
                    vt o;
#pragma unroll
                    for (int q = 0; q < 4; ++q) o[q] = acc[x][y][q];
                    *reinterpret_cast<vt*>(Qs + j * LDQ + y * 16 + 4 * g) = o;
                }
            }
        }
        __syncthreads();
        // ---- epilogue: modes 1 and N from the LDS window ----
#pragma unroll 1
        for (int i = 0; i < IPT; ++i) {
            const int it = threadIdx.x + i * CTA_WG;
            if (it >= nitem) break;
            const int j = it / GPR;
            const int c = (it - j * GPR) * E;
            const int t = t0 + c;
            const Tv* prow = Pw + j * LDP + H + c;  // prow[0] is P[j][t]
            const int64_t base = (int64_t)j * trail + t;
            // Branch-free taps: a tap outside the tensor has a zero band
            // coefficient (R_k[i][i+d] with i+d out of range is stored as 0), so
            // its address is clamped to a valid one instead of tested.
            const vt pc = *reinterpret_cast<const vt*>(prow);
            vt s = *reinterpret_cast<const vt*>(Qs + j * LDQ + c);  // chain part, lam applied below
            vt reg = rmid[i];
            if (has1) {
#pragma unroll
                for (int d = -2; d <= 2; ++d) {
                    const int jj = min(max(j + d, 0), K - 1);
                    reg += band1[j * 5 + d + 2] * *reinterpret_cast<const vt*>(Pw + jj * LDP + H + c);
                }
            }
            if (hasN) {
                Tv w[3 * E];
                const vt pl = *reinterpret_cast<const vt*>(prow - E);
                const vt pr = *reinterpret_cast<const vt*>(prow + E);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    w[e] = pl[e];
                    w[E + e] = pc[e];
                    w[2 * E + e] = pr[e];
                }
                const int i0 = t - fast_div(t, st.emul[N - 1], st.eshift[N - 1]) * nN;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const Tv* bN = bandN + (i0 + e) * 5;
#pragma unroll
                    for (int d = -2; d <= 2; ++d) reg[e] += bN[d + 2] * w[E + e + d];
                }
            }
            const vt qv = s + lam * reg;
            *reinterpret_cast<vt*>(Q + base) = qv;
#pragma unroll
            for (int e = 0; e < E; ++e) dot_acc += (double)pc[e] * (double)qv[e];
        }
        __syncthreads();  // LDS is reused by the next tile
    }
}

// ---------------------------------------------------------------------------
// Variant 6 of the pipelined last pass: normal_last_pipe's tiles, item layout,
// prefetch and MFMA, with fewer LDS and vector instructions per item:
//  * the P window has two zero rows above and below (rows -2, -1, K, K + 1),
//    so the mode-1 taps need no clamping (their band coefficients are zero
//    there anyway);
//  * the band rows of mode 1 are staged 8 floats apart and those of mode N
//    contiguously, so an item reads its 5 mode-1 and 4 x 5 mode-N
//    coefficients as 16-byte vectors (2 + 5 reads instead of 25).
// The G_1 fragments a wave multiplies with (its 16 JT rows, all K) are
// loaded into registers once per workgroup instead of from the cache for
// every tile.  Every element's sums are the same as normal_last_pipe's, in
// the same order (identical Q).  NT = 256 (4 waves, 4 items per thread) is variant 6;
// NT = 512 (8 waves of 16 output rows, 2 items per thread, so that a thread's
// gathers of one mode are all in flight together) is variant 7.
template <int NT>
__device__ __forceinline__ void normal_last_pipe6(const StridedArgs& a, unsigned char* smem,
                                                  const StencilArgs<float>& st, double& dot_acc,
                                                  int64_t first, int64_t step, int64_t end) {
    typedef MT<bf16> T;
    typedef float Tv;
    typedef floatx4 vt;
    constexpr int KPAD = 128;
    constexpr int TN = PIPE_TN, H = PIPE_H, LDP = PIPE_LDP;
    constexpr int E = 4, LDQ = TN + E;
    constexpr int JT = 8 * 64 / NT, CT = 2;   // a wave owns 16 JT output rows
    const int K = a.K;
    const int trail = (int)a.trail;
    const int N = st.order;
    const int nN = (int)st.ext[N - 1];
    constexpr int ldx = KPAD + 8;
    constexpr size_t a_bytes = ((size_t)(TN * ldx * 2) > (size_t)(KPAD * LDQ * 4) ? (size_t)(TN * ldx * 2)
                                                                                    : (size_t)(KPAD * LDQ * 4));
    bf16* Xs = reinterpret_cast<bf16*>(smem);
    float* Qs = reinterpret_cast<float*>(smem);
    float* Pw0 = reinterpret_cast<float*>(smem + (a_bytes + 15) / 16 * 16);  // KPAD + 4 rows
    float* Pw = Pw0 + 2 * LDP;                                                // row j at Pw + j * LDP
    float* band1 = Pw0 + (size_t)(KPAD + 4) * LDP;                            // [j][8]
    float* bandN = band1 + (size_t)KPAD * 8;                                  // [i][5]
    const bool has1 = st.rband[0] != nullptr;
    const bool hasN = st.rband[N - 1] != nullptr;
    float* __restrict__ Q = reinterpret_cast<float*>(a.Y);
    const float* __restrict__ P = st.P;
    const bf16* __restrict__ M = reinterpret_cast<const bf16*>(a.M);
    const int cpp = (int)(a.plane / TN), per = cpp * a.pgroup;
    const float inv_per = a.pgroup > 0 ? 1.0f / (float)per : 0.f;
    const float inv_pg = a.pgroup > 0 ? 1.0f / (float)a.pgroup : 0.f;
    auto tcol = [&](int64_t tl) -> int {
        const int t = (int)tl;
        if (a.pgroup <= 0) return t * TN;
        const int grp = small_div(t, per, inv_per), rr = t - grp * per;
        const int c = small_div(rr, a.pgroup, inv_pg), ig = rr - c * a.pgroup;
        return (grp * a.pgroup + ig) * (int)a.plane + c * TN;
    };
    PipeRegsT<NT> r;
    if (first < end) pipe_load<KPAD, NT>(a, P, tcol(first), K, r);   // in flight while the bands are staged
    if (has1)
        for (int u = threadIdx.x; u < K * 8; u += NT) {
            const int jj = u >> 3, d = u & 7;
            band1[u] = d < 5 ? st.rband[0][jj * 5 + d] : 0.f;
        }
    if (hasN)
        for (int u = threadIdx.x; u < nN * 5; u += NT) bandN[u] = st.rband[N - 1][u];
    // zero rows around the window: -2, -1 and K, K + 1 (never written by the tiles)
    for (int u = threadIdx.x; u < 4 * LDP; u += NT) {
        const int rr = u / LDP, cc = u - rr * LDP;
        const int row = rr < 2 ? rr - 2 : K + rr - 2;
        Pw[row * LDP + cc] = 0.f;
    }
    const Tv lam = (Tv)st.lam;
    constexpr int GPR = TN / E;
    constexpr int IPT = KPAD * GPR / NT;
    const int nitem = a.J * GPR;
    // this wave's G_1 fragments (16 JT output rows, all KPAD columns) stay in
    // registers for the workgroup's whole life
    constexpr int NKS = KPAD / T::KSTEP;
    typename T::frag mreg[JT][NKS];
    {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int jb = wave * JT * 16;
#pragma unroll
        for (int x = 0; x < JT; ++x)
#pragma unroll
            for (int ks = 0; ks < NKS; ++ks)
                mreg[x][ks] = *reinterpret_cast<const typename T::frag*>(
                    M + (int64_t)(jb + x * 16 + (lane & 15)) * a.ldm + ks * T::KSTEP + T::VEC * (lane >> 4));
    }
    for (int64_t tile = first; tile < end; tile += step) {
        const int t0 = tcol(tile);
        pipe_store<KPAD, NT>(r, Xs, Pw, K);
        __syncthreads();
        // ---- middle-mode regulariser taps (summed first, as every variant) ----
        vt rmid[IPT];
#pragma unroll
        for (int i = 0; i < IPT; ++i)
#pragma unroll
            for (int e = 0; e < E; ++e) rmid[i][e] = Tv(0);
        mid_taps<IPT, GPR, E, LDP, H, NT>(st, Pw, a.J, trail, t0, rmid);
        // ---- MFMA (as normal_last_pipe) ----
        {
            const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
            const int jb = wave * JT * 16;
            const int g = lane >> 4, l16 = lane & 15;
            typename T::acc acc[JT][CT];
#pragma unroll
            for (int x = 0; x < JT; ++x)
#pragma unroll
                for (int y = 0; y < CT; ++y) acc[x][y] = T::zero();
#pragma unroll
            for (int ks = 0; ks < NKS; ++ks) {
                typename T::frag xa[CT];
#pragma unroll
                for (int y = 0; y < CT; ++y)
                    xa[y] = *reinterpret_cast<const typename T::frag*>(Xs + (y * 16 + l16) * ldx + ks * T::KSTEP +
                                                                        T::VEC * g);
#pragma unroll
                for (int x = 0; x < JT; ++x)
#pragma unroll
                    for (int y = 0; y < CT; ++y) acc[x][y] = T::mma(xa[y], mreg[x][ks], acc[x][y]);
            }
            if (tile + step < end) pipe_load<KPAD, NT>(a, P, tcol(tile + step), K, r);
            __syncthreads();  // Xs is dead; its space becomes Qs
#pragma unroll
            for (int x = 0; x < JT; ++x) {
                const int j = jb + x * 16 + l16;
                if (j >= a.J) continue;
#pragma unroll
                for (int y = 0; y < CT; ++y) {
                    vt o;
#pragma unroll
                    for (int q = 0; q < 4; ++q) o[q] = acc[x][y][q];
                    *reinterpret_cast<vt*>(Qs + j * LDQ + y * 16 + 4 * g) = o;
                }
            }
        }
        __syncthreads();
        // ---- epilogue: modes 1 and N from the LDS window ----
#pragma unroll 1
        for (int i = 0; i < IPT; ++i) {
            const int it = threadIdx.x + i * NT;
            if (it >= nitem) break;
            const int j = it / GPR;
            const int c = (it - j * GPR) * E;
            const int t = t0 + c;
            const Tv* prow = Pw + j * LDP + H + c;  // prow[0] is P[j][t]
            const int64_t base = (int64_t)j * trail + t;
            const vt pc = *reinterpret_cast<const vt*>(prow);
            vt s = *reinterpret_cast<const vt*>(Qs + j * LDQ + c);  // chain part, lam applied below
            vt reg = rmid[i];
            if (has1) {
                const vt bl = *reinterpret_cast<const vt*>(band1 + j * 8);
                const Tv b4 = band1[j * 8 + 4];
                reg += bl[0] * *reinterpret_cast<const vt*>(prow - 2 * LDP);
                reg += bl[1] * *reinterpret_cast<const vt*>(prow - LDP);
                reg += bl[2] * pc;
                reg += bl[3] * *reinterpret_cast<const vt*>(prow + LDP);
                reg += b4 * *reinterpret_cast<const vt*>(prow + 2 * LDP);
            }
            if (hasN) {
                Tv w[3 * E];
                const vt pl = *reinterpret_cast<const vt*>(prow - E);
                const vt pr = *reinterpret_cast<const vt*>(prow + E);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    w[e] = pl[e];
                    w[E + e] = pc[e];
                    w[2 * E + e] = pr[e];
                }
                const int i0 = t - fast_div(t, st.emul[N - 1], st.eshift[N - 1]) * nN;
                // the 4 x 5 coefficients are 20 consecutive floats (i0 % 4 == 0):
                // coefficient x = 5 e + d + 2 multiplies tap d of column e, and
                // each column's taps are taken in increasing d
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    const vt v = *reinterpret_cast<const vt*>(bandN + i0 * 5 + 4 * q);
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int x = 4 * q + m, e = x / 5, d = x - 5 * e - 2;
                        reg[e] += v[m] * w[E + e + d];
                    }
                }
            }
            const vt qv = s + lam * reg;
            *reinterpret_cast<vt*>(Q + base) = qv;
#pragma unroll
            for (int e = 0; e < E; ++e) dot_acc += (double)pc[e] * (double)qv[e];
        }
        __syncthreads();  // LDS is reused by the next tile
    }
}

// ---------------------------------------------------------------------------
// Variant 8 of the pipelined last pass (tensor order 4, BF16 chain, K = J <=
// 128, n_N <= 24, n_N % 4 == 0, the plane of the second mode a multiple of 32
// columns).  One workgroup per CU sweeps a run of consecutive 32-column
// tiles of one plane of the second mode; the workgroups of one XCD hold
// neighbouring planes, so the second mode's neighbour planes are read by
// neighbouring workgroups at nearly the same time and come from that XCD's
// L2.  P stays in LDS as a ring of 128 columns (the tile and 48 columns
// either side) that slides by 32 columns per tile: the third mode's taps
// (columns +- n_N, +- 2 n_N), the last mode's and the first mode's come from
// LDS; only the second mode's four planes are gathered.  A tile's 32 new ring
// columns and its X rows are loaded into registers two tiles ahead, its
// gathers GD tiles ahead, and issued in the order they are waited for.  An
// item is 4 columns of one row; a workgroup of NT threads gives each thread
// 1024 / NT of them (the launcher uses 1024 threads, one item each).  Every
// element's sums are those of the other variants, in the same order
// (identical Q).
constexpr int RING_TN = 32;
constexpr int RING_W = 128;          // ring columns (power of two)
constexpr int RING_LD = RING_W + 8;  // pitch: rows 4 apart fall in disjoint halves of the banks
constexpr int RING_NT = 1024;
constexpr int RING_XLD = 128 + 8;    // X tile pitch (bf16)
constexpr int RING_LDQ = RING_TN + 4;

struct RingGeom {
    int nplane, plane, nseg, cpp, seg_len;  // planes, plane width, segments per plane, chunks per plane
};

// band blocks start on 16-byte boundaries (the mode-N rows are read as float4)
__host__ __device__ inline int ring_pad4(int n) { return (n + 3) & ~3; }

// LDS bytes of variant 8 (ring, X tile, Q tile, band rows of modes 1, 3, N)
__host__ __device__ inline size_t ring_lds_bytes(int K, int n3, int nN) {
    return (size_t)(K + 4) * RING_LD * 4 + (size_t)RING_TN * RING_XLD * 2 + (size_t)128 * RING_LDQ * 4 +
           (size_t)128 * 8 * 4 + (size_t)ring_pad4(n3 * 5) * 4 + (size_t)nN * 5 * 4;
}

// Registers of a tile's prefetched data: IPT rows' 4 of the 32 new ring
// columns (rows tid / 8 + h NT / 8) and, for threads < 256, rows 2 kp and
// 2 kp + 1 of the X tile, 8 columns.
template <int IPT>
struct RingRegs {
    floatx4 p[IPT];
    bf16x8 x[2];
};

// Row of a thread's item: within each wave's block of 8 rows, lanes 8q .. 8q+7
// take row 4 (q mod 2) + q / 2, so one 16-lane LDS access reads rows 4 apart.
__device__ __forceinline__ int ring_row(int tid) {
    const int q = (tid >> 3) & 7;
    return (tid >> 6) * 8 + (q & 1) * 4 + (q >> 1);
}

// A tile starting at column T reads the ring window [T - 48, T + 80); going
// from the tile at T - 32 to it, the new columns are [T + 48, T + 80), which
// take the ring slots of [T - 80, T - 48).  ring_get_cols loads a thread's 4
// of those 32 columns of its rows (tid / 8 + h NT / 8); rows past K and
// columns outside the tensor read a clamped address and are stored as zero by
// ring_put_cols.
template <int NT, int IPT>
__device__ __forceinline__ void ring_get_cols(const float* __restrict__ P, int trail, int T, int K,
                                              floatx4 (&v)[IPT]) {
    const int ch = threadIdx.x & 7;
    const int t = T + 48 + 4 * ch;
#pragma unroll
    for (int h = 0; h < IPT; ++h) {
        const int row = (threadIdx.x >> 3) + h * (NT / 8);
        const bool ok = row < K && t >= 0 && t < trail;
        v[h] = *reinterpret_cast<const floatx4*>(P + (int64_t)(ok ? row : 0) * trail + (ok ? t : 0));
    }
}

template <int NT, int IPT>
__device__ __forceinline__ void ring_put_cols(const floatx4 (&v)[IPT], float* ring, int trail, int T, int K) {
    const int ch = threadIdx.x & 7;
    const int t = T + 48 + 4 * ch;
#pragma unroll
    for (int h = 0; h < IPT; ++h) {
        const int row = (threadIdx.x >> 3) + h * (NT / 8);
        if (row < K) {
            floatx4 w = v[h];
            if (t < 0 || t >= trail) w = floatx4{0.f, 0.f, 0.f, 0.f};
            *reinterpret_cast<floatx4*>(ring + (row + 2) * RING_LD + (t & (RING_W - 1))) = w;
        }
    }
}

__device__ __forceinline__ void ring_get_x(const StridedArgs& a, int T, int K, bf16x8 (&x)[2]) {
    if (threadIdx.x < 256) {
        const bf16* __restrict__ X = reinterpret_cast<const bf16*>(a.X);
        const int cg = threadIdx.x & 3, kp = threadIdx.x >> 2;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = min(2 * kp + h, K - 1);
            // X is dead after this pass (non-temporal, as the middle pass's input)
            x[h] = __builtin_nontemporal_load(reinterpret_cast<const bf16x8*>(X + (int64_t)k * a.trail + T + cg * 8));
        }
    }
}

__device__ __forceinline__ void ring_put_x(const bf16x8 (&x)[2], bf16* Xs, int K) {
    if (threadIdx.x < 256) {
        const int cg = threadIdx.x & 3, kp = threadIdx.x >> 2;
        typedef bf16 __attribute__((ext_vector_type(2))) bf16x2;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            bf16x2 pr;
            pr[0] = 2 * kp < K ? x[0][c] : (bf16)0.f;
            pr[1] = 2 * kp + 1 < K ? x[1][c] : (bf16)0.f;
            *reinterpret_cast<bf16x2*>(Xs + (cg * 8 + c) * RING_XLD + 2 * kp) = pr;
        }
    }
}

// NT threads per workgroup, IPT = 1024 / NT items per thread (rows j and
// j + NT / 8 of the same 4 columns, so the column's mode indices and band
// rows are formed once), and the second mode's gathers issued GD tiles ahead.
template <int NT, int GD>
__device__ __forceinline__ void normal_last_ring(const StridedArgs& a, unsigned char* smem,
                                                 const StencilArgs<float>& st, const RingGeom& rg,
                                                 double& dot_acc) {
    typedef MT<bf16> T;
    typedef floatx4 vt;
    constexpr int E = 4, NKS = 4;
    constexpr int IPT = 1024 / NT;
    constexpr int RS = NT / 8;
    const int K = a.K;
    const int trail = (int)a.trail;
    const int nN = (int)st.ext[3], n3 = (int)st.ext[2], n2 = (int)st.ext[1];
    float* ring = reinterpret_cast<float*>(smem);                              // [K + 4][RING_LD]
    bf16* Xs = reinterpret_cast<bf16*>(ring + (size_t)(K + 4) * RING_LD);      // [32][RING_XLD]
    float* Qs = reinterpret_cast<float*>(Xs + (size_t)RING_TN * RING_XLD);     // [128][RING_LDQ]
    float* band1 = Qs + (size_t)128 * RING_LDQ;                                // [j][8]
    float* band3 = band1 + (size_t)128 * 8;                                    // [i3][5]
    float* bandN = band3 + ring_pad4(n3 * 5);                                  // [i4][5]
    const float* __restrict__ P = st.P;
    float* __restrict__ Q = reinterpret_cast<float*>(a.Y);
    const bf16* __restrict__ M = reinterpret_cast<const bf16*>(a.M);
    const bool has1 = st.rband[0] != nullptr, has2 = st.rband[1] != nullptr;
    const bool has3 = st.rband[2] != nullptr, hasN = st.rband[3] != nullptr;
    // this workgroup's plane and run of chunks: segment-major, so that an XCD
    // holds a run of consecutive planes of one segment and most second-mode
    // neighbours are read from its own L2
    const int L = (int)xcd_logical_block(blockIdx.x, gridDim.x);
    const int seg = L / rg.nplane, p = L - seg * rg.nplane;
    const int cbeg = seg * rg.seg_len, cend = min(rg.cpp, cbeg + rg.seg_len);
    if (p >= rg.nplane || cbeg >= cend) return;   // uniform: the whole workgroup leaves
    const int tbase = p * rg.plane;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, g = lane >> 4, l16 = lane & 15;
    // band rows and the ring's zero rows (-2, -1, K, K + 1)
    if (has1)
        for (int u = tid; u < K * 8; u += NT) {
            const int jj = u >> 3, d = u & 7;
            band1[u] = d < 5 ? st.rband[0][jj * 5 + d] : 0.f;
        }
    if (has3)
        for (int u = tid; u < n3 * 5; u += NT) band3[u] = st.rband[2][u];
    if (hasN)
        for (int u = tid; u < nN * 5; u += NT) bandN[u] = st.rband[3][u];
    for (int u = tid; u < 4 * RING_LD; u += NT) {
        const int rr = u / RING_LD, cc = u - rr * RING_LD;
        const int row = rr < 2 ? rr : K + rr;   // ring rows 0, 1 and K + 2, K + 3
        ring[row * RING_LD + cc] = 0.f;
    }
    // the second mode's band row and in-range neighbour offsets: one plane per workgroup
    float b2c[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    uint32_t off2[4] = {0u, 0u, 0u, 0u};
    if (has2) {
#pragma unroll
        for (int q = 0; q < 5; ++q) b2c[q] = st.rband[1][p * 5 + q];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int d = q < 2 ? q - 2 : q - 1;
            const int dd = (p + d >= 0 && p + d < n2) ? d : 0;
            off2[q] = (uint32_t)(dd * rg.plane) * 4u;
        }
    }
    // this wave's 16 x 16 blocks (IPT of them, blocks wave IPT .. : rows 16 (b / 2),
    // columns 16 (b % 2)) share their G_1 rows; the fragments stay in registers
    const int blk0 = wave * IPT;
    const int rt = blk0 >> 1;
    typename T::frag mreg[NKS];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks)
        mreg[ks] = *reinterpret_cast<const typename T::frag*>(M + (int64_t)(rt * 16 + l16) * a.ldm +
                                                              ks * T::KSTEP + T::VEC * g);
    // the items: rows j[h], columns c .. c + 3 of every tile
    const int c = (tid & 7) * E;
    int jr[IPT], jc[IPT];
    bool jok[IPT];
#pragma unroll
    for (int h = 0; h < IPT; ++h) {
        jr[h] = ring_row(tid) + h * RS;
        jok[h] = jr[h] < K;
        jc[h] = jok[h] ? jr[h] : K - 1;
    }
    const char* __restrict__ Pb = reinterpret_cast<const char*>(P);
    auto gather = [&](int t0, vt (&gv)[IPT][4]) {
#pragma unroll
        for (int h = 0; h < IPT; ++h) {
            const uint32_t base = (uint32_t)(jc[h] * trail + t0 + c) * 4u;
#pragma unroll
            for (int q = 0; q < 4; ++q) gv[h][q] = *reinterpret_cast<const vt*>(Pb + (base + off2[q]));
        }
    };
    // prologue: the first tile's ring window [t0 - 48, t0 + 80) (the new
    // columns of the tiles at t0 - 96, t0 - 64, t0 - 32 and t0) and X tile,
    // the second tile's data, the first GD tiles' gathers
    const int t_first = tbase + cbeg * RING_TN;
    {
        floatx4 w[4][IPT];
#pragma unroll
        for (int b = 0; b < 4; ++b) ring_get_cols<NT, IPT>(P, trail, t_first - 96 + 32 * b, K, w[b]);
        bf16x8 x0[2];
        ring_get_x(a, t_first, K, x0);
#pragma unroll
        for (int b = 0; b < 4; ++b) ring_put_cols<NT, IPT>(w[b], ring, trail, t_first - 96 + 32 * b, K);
        ring_put_x(x0, Xs, K);
    }
    RingRegs<IPT> rA, rB;   // the data of tile i + 1 is in rB before tile i for i - cbeg even, in rA for odd
    vt gA[IPT][4], gB[IPT][4];   // GD = 2: gathers of tile i in gA for i - cbeg even, in gB for odd
    gather(t_first, gA);
    if constexpr (GD == 2) gather(tbase + min(cbeg + 1, cend - 1) * RING_TN, gB);
    {
        const int t1 = tbase + min(cbeg + 1, cend - 1) * RING_TN;
        ring_get_cols<NT, IPT>(P, trail, t1, K, rB.p);
        ring_get_x(a, t1, K, rB.x);
    }
    const float lam = (float)st.lam;
    auto run_tile = [&](int ci, RingRegs<IPT>& rnext, RingRegs<IPT>& rfree, vt (&gv)[IPT][4]) {
        const int t0 = tbase + ci * RING_TN;
        __syncthreads();   // ring window, X tile and bands of this tile are in LDS
        const int t = t0 + c;
        const int col = t & (RING_W - 1);
        const float* rrow[IPT];
        vt pc[IPT], rmid[IPT];
#pragma unroll
        for (int h = 0; h < IPT; ++h) {
            rrow[h] = ring + (jc[h] + 2) * RING_LD;
            pc[h] = *reinterpret_cast<const vt*>(rrow[h] + col);
        }
        // ---- middle modes, second then third (as every variant) ----
#pragma unroll
        for (int h = 0; h < IPT; ++h) {
            rmid[h] = vt{0.f, 0.f, 0.f, 0.f};
            if (has2) {
                rmid[h] += b2c[2] * pc[h];
                rmid[h] += b2c[0] * gv[h][0];
                rmid[h] += b2c[1] * gv[h][1];
                rmid[h] += b2c[3] * gv[h][2];
                rmid[h] += b2c[4] * gv[h][3];
            }
        }
        // the gathers of the tile GD ahead, then the data of the tile after next
        gather(tbase + min(ci + GD, cend - 1) * RING_TN, gv);
        {
            const int t2 = tbase + min(ci + 2, cend - 1) * RING_TN;
            ring_get_cols<NT, IPT>(P, trail, t2, K, rfree.p);
            ring_get_x(a, t2, K, rfree.x);
        }
        if (has3) {
            const int u = fast_div(t, st.smul[2], st.sshift[2]);
            const int i3 = u - fast_div(u, st.emul[2], st.eshift[2]) * n3;
            const float* br = band3 + i3 * 5;
            int cq[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int d = q < 2 ? q - 2 : q - 1;
                const int dd = (i3 + d >= 0 && i3 + d < n3) ? d : 0;
                cq[q] = (t + dd * nN) & (RING_W - 1);
            }
#pragma unroll
            for (int h = 0; h < IPT; ++h) {
                vt nb[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) nb[q] = *reinterpret_cast<const vt*>(rrow[h] + cq[q]);
                rmid[h] += br[2] * pc[h];
                rmid[h] += br[0] * nb[0];
                rmid[h] += br[1] * nb[1];
                rmid[h] += br[3] * nb[2];
                rmid[h] += br[4] * nb[3];
            }
        }
        // ---- MFMA: this wave's 16 x 16 blocks of the chain part ----
#pragma unroll
        for (int b = 0; b < IPT; ++b) {
            const int ct = (blk0 + b) & 1;
            typename T::acc acc = T::zero();
#pragma unroll
            for (int ks = 0; ks < NKS; ++ks) {
                const typename T::frag xa = *reinterpret_cast<const typename T::frag*>(
                    Xs + (ct * 16 + l16) * RING_XLD + ks * T::KSTEP + T::VEC * g);
                acc = T::mma(xa, mreg[ks], acc);
            }
            const int jo = rt * 16 + l16;
            vt o;
#pragma unroll
            for (int q = 0; q < 4; ++q) o[q] = acc[q];
            *reinterpret_cast<vt*>(Qs + jo * RING_LDQ + ct * 16 + 4 * g) = o;
        }
        __syncthreads();   // Q tile complete
        // ---- epilogue: modes 1 and N from the ring ----
        vt reg[IPT];
#pragma unroll
        for (int h = 0; h < IPT; ++h) {
            reg[h] = rmid[h];
            if (has1) {
                const vt bl = *reinterpret_cast<const vt*>(band1 + jc[h] * 8);
                const float b4 = band1[jc[h] * 8 + 4];
                reg[h] += bl[0] * *reinterpret_cast<const vt*>(rrow[h] - 2 * RING_LD + col);
                reg[h] += bl[1] * *reinterpret_cast<const vt*>(rrow[h] - RING_LD + col);
                reg[h] += bl[2] * pc[h];
                reg[h] += bl[3] * *reinterpret_cast<const vt*>(rrow[h] + RING_LD + col);
                reg[h] += b4 * *reinterpret_cast<const vt*>(rrow[h] + 2 * RING_LD + col);
            }
        }
        if (hasN) {
            float w[IPT][3 * E];
#pragma unroll
            for (int h = 0; h < IPT; ++h) {
                const vt pl = *reinterpret_cast<const vt*>(rrow[h] + ((t - E) & (RING_W - 1)));
                const vt pr = *reinterpret_cast<const vt*>(rrow[h] + ((t + E) & (RING_W - 1)));
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    w[h][e] = pl[e];
                    w[h][E + e] = pc[h][e];
                    w[h][2 * E + e] = pr[e];
                }
            }
            const int i0 = t - fast_div(t, st.emul[3], st.eshift[3]) * nN;
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const vt v = *reinterpret_cast<const vt*>(bandN + i0 * 5 + 4 * q);
#pragma unroll
                for (int h = 0; h < IPT; ++h)
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int x = 4 * q + m, e = x / 5, d = x - 5 * e - 2;
                        reg[h][e] += v[m] * w[h][E + e + d];
                    }
            }
        }
#pragma unroll
        for (int h = 0; h < IPT; ++h) {
            if (jok[h]) {
                const vt s = *reinterpret_cast<const vt*>(Qs + jr[h] * RING_LDQ + c);
                const vt qv = s + lam * reg[h];
                *reinterpret_cast<vt*>(Q + (int64_t)jr[h] * trail + t) = qv;
#pragma unroll
                for (int e = 0; e < E; ++e) dot_acc += (double)pc[h][e] * (double)qv[e];
            }
        }
        __syncthreads();   // the ring's oldest 32 columns, the X and Q tiles are free
        if (ci + 1 < cend) {
            ring_put_cols<NT, IPT>(rnext.p, ring, trail, tbase + (ci + 1) * RING_TN, K);
            ring_put_x(rnext.x, Xs, K);
        }
    };
    for (int ci = cbeg; ci < cend; ci += 2) {
        run_tile(ci, rB, rA, gA);
        if (ci + 1 >= cend) break;
        if constexpr (GD == 2)
            run_tile(ci + 1, rA, rB, gB);
        else
            run_tile(ci + 1, rA, rB, gA);
    }
}

// ---------------------------------------------------------------------------
// Last pass in row blocks (FP32 vectors, tensor order 3 or 4): a tile is 32
// output rows x 32 columns, and everything the 17-point stencil reads is staged
// in LDS with coalesced loads: P rows j0-2 .. j0+33 over the columns
// t0-H .. t0+32+H with H = 2 n_N (the contiguous mode and the second-to-last
// mode, whose stride is n_N), and for order 4 the four neighbour planes of the
// second mode (t +- stride, +- 2 stride).  One epilogue item (4 columns of one
// row) per thread, no gathers from memory.  The X tile (all K rows) is staged
// once per row block; the row blocks of a column tile run consecutively, so
// its re-reads come from L2.  The chain part and every stencil sum are formed
// in the same order as normal_last_tile, so both give identical Q.
constexpr int JS_JB = 32;  // output rows per tile
constexpr int JS_TN = 32;  // columns per tile

struct JsGeom {
    int nN, nM, sM, H, LDW;  // contiguous extent, halo-mode extent and stride, halo, window pitch
    int nF;                  // far-mode extent (order 4), 0 for order 3
    int64_t sF;              // far-mode stride
};

template <typename Tc>
__host__ __device__ inline size_t js_lds_bytes(int kpad, int H, int NF, int nN, int nM) {
    const size_t xs = (size_t)JS_TN * (kpad + 16 / sizeof(Tc)) * sizeof(Tc);
    const size_t qs = (size_t)JS_JB * (JS_TN + 4) * 4;
    const size_t a = ((xs > qs ? xs : qs) + 15) / 16 * 16;
    const size_t pw = (size_t)(JS_JB + 4) * (JS_TN + 2 * H) * 4;
    const size_t pf = (size_t)NF * 4 * JS_JB * JS_TN * 4;
    const size_t bands = (size_t)(JS_JB + nN + nM + 8) * 5 * 4;
    return a + pw + pf + bands;
}

template <typename Tin, typename Tc, int NF>
__device__ __forceinline__ void normal_last_jtile(const StridedArgs& a, int64_t tile, unsigned char* smem,
                                                  const StencilArgs<float>& st, const JsGeom& gm,
                                                  double& dot_acc) {
    typedef MT<Tc> T;
    typedef float __attribute__((ext_vector_type(4))) vt;
    constexpr int TN = JS_TN, JB = JS_JB;
    constexpr int VEC = T::VEC;
    constexpr int LV = 16 / sizeof(Tin);
    constexpr int LDQ = TN + 4;
    constexpr int N = NF ? 4 : 3;
    const int K = a.K;
    const int trail = (int)a.trail;
    const int njb = (K + JB - 1) / JB;
    const int jblk = (int)(tile % njb);
    const int j0 = jblk * JB;
    const int t0 = (int)last_tile_col<TN>(a, tile / njb);
    const int ldx = a.kpad + 16 / (int)sizeof(Tc);
    const int H = gm.H, LDW = gm.LDW;
    const size_t xs_bytes = (size_t)TN * ldx * sizeof(Tc);
    const size_t qs_bytes = (size_t)JB * LDQ * 4;
    const size_t a_bytes = ((xs_bytes > qs_bytes ? xs_bytes : qs_bytes) + 15) / 16 * 16;
    Tc* Xs = reinterpret_cast<Tc*>(smem);
    float* Qs = reinterpret_cast<float*>(smem);
    float* Pw = reinterpret_cast<float*>(smem + a_bytes);
    float* Pf = Pw + (size_t)(JB + 4) * LDW;
    float* b1 = Pf + (size_t)NF * 4 * JB * TN;
    float* bN = b1 + JB * 5;
    float* bM = bN + gm.nN * 5;
    float* bF = bM + gm.nM * 5;
    const bool has1 = st.rband[0] != nullptr;
    const bool hasN = st.rband[N - 1] != nullptr;
    const bool hasM = st.rband[N - 2] != nullptr;
    const bool hasF = NF && st.rband[1] != nullptr;
    const Tin* __restrict__ X = reinterpret_cast<const Tin*>(a.X);
    float* __restrict__ Q = reinterpret_cast<float*>(a.Y);
    const float* __restrict__ P = st.P;
    const Tc* __restrict__ M = reinterpret_cast<const Tc*>(a.M);
    // plane index of the tile along the far mode (TN divides its stride)
    const int iF = NF ? (int)((t0 / gm.sF) % gm.nF) : 0;

    // ---- stage the X tile (all K rows, transposed, Tc) ----
    stage_cols<Tin, Tc, TN>(X, trail, K, a.kpad, t0, trail, Xs, ldx);
    // ---- stage the P window (rows j0-2 .. j0+JB+1, zero outside the tensor) ----
    {
        const int cpr = LDW / 4;
        for (int u = threadIdx.x; u < (JB + 4) * cpr; u += CTA_WG) {
            const int r = u / cpr, ch = u - r * cpr;
            const int j = j0 - 2 + r;
            const int t = t0 - H + ch * 4;
            vt v = {0.f, 0.f, 0.f, 0.f};
            if (j >= 0 && j < K && t >= 0 && t < trail) v = *reinterpret_cast<const vt*>(P + (int64_t)j * trail + t);
            *reinterpret_cast<vt*>(Pw + r * LDW + ch * 4) = v;
        }
    }
    // ---- stage the far-mode neighbour planes (order 4) ----
    if constexpr (NF) {
        constexpr int cpr = TN / 4;
        for (int u = threadIdx.x; u < 4 * JB * cpr; u += CTA_WG) {
            const int q = u / (JB * cpr), rem = u - q * (JB * cpr);
            const int r = rem / cpr, ch = rem - r * cpr;
            const int d = q < 2 ? q - 2 : q - 1;
            const int j = j0 + r;
            vt v = {0.f, 0.f, 0.f, 0.f};
            if (j < K && iF + d >= 0 && iF + d < gm.nF)
                v = *reinterpret_cast<const vt*>(P + (int64_t)j * trail + t0 + (int64_t)d * gm.sF + ch * 4);
            *reinterpret_cast<vt*>(Pf + (q * JB + r) * TN + ch * 4) = v;
        }
    }
    // ---- band coefficients ----
    for (int u = threadIdx.x; u < JB * 5; u += CTA_WG) {
        const int j = j0 + u / 5;
        b1[u] = (has1 && j < K) ? st.rband[0][j * 5 + u % 5] : 0.f;
    }
    if (hasN)
        for (int u = threadIdx.x; u < gm.nN * 5; u += CTA_WG) bN[u] = st.rband[N - 1][u];
    if (hasM)
        for (int u = threadIdx.x; u < gm.nM * 5; u += CTA_WG) bM[u] = st.rband[N - 2][u];
    if (hasF && threadIdx.x < 5) bF[threadIdx.x] = st.rband[1][iF * 5 + threadIdx.x];
    __syncthreads();

    // ---- MFMA: wave w computes rows j0 + 16 (w >> 1) .. +16, columns 16 (w & 1) .. +16 ----
    {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int g = lane >> 4, l16 = lane & 15;
        const int jr = (wave >> 1) * 16, cb = (wave & 1) * 16;
        typename T::acc acc = T::zero();
        const int nks = a.kpad / T::KSTEP;
        for (int ks = 0; ks < nks; ++ks) {
            const int k0 = ks * T::KSTEP + VEC * g;
            const typename T::frag xa = *reinterpret_cast<const typename T::frag*>(Xs + (cb + l16) * ldx + k0);
            const typename T::frag mb = *reinterpret_cast<const typename T::frag*>(
                M + (int64_t)(j0 + jr + l16) * a.ldm + k0);
            acc = T::mma(xa, mb, acc);
        }
        __syncthreads();  // Xs is dead; its space becomes Qs
        vt o;
#pragma unroll
        for (int r = 0; r < 4; ++r) o[r] = acc[r];
        *reinterpret_cast<vt*>(Qs + (jr + l16) * LDQ + cb + 4 * g) = o;
    }
    __syncthreads();

    // ---- epilogue: one item (4 columns of one row) per thread ----
    {
        const float lam = (float)st.lam;
        const int it = threadIdx.x;
        const int jr = it >> 3, c = (it & 7) * 4;
        const int j = j0 + jr;
        const int t = t0 + c;
        if (j < K) {
            const float* prow = Pw + (jr + 2) * LDW + H + c;  // prow[0] is P[j][t]
            const vt pc = *reinterpret_cast<const vt*>(prow);
            const vt s = *reinterpret_cast<const vt*>(Qs + jr * LDQ + c);
            vt reg = {0.f, 0.f, 0.f, 0.f};
            // middle modes first, then mode 1, then mode N (the order of every variant)
            if constexpr (NF) {
                if (hasF) {
                    reg += bF[2] * pc;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        reg += bF[q < 2 ? q : q + 1] * *reinterpret_cast<const vt*>(Pf + (q * JB + jr) * TN + c);
                }
            }
            if (hasM) {
                const int u = fast_div(t, st.smul[N - 2], st.sshift[N - 2]);
                const int iM = u - fast_div(u, st.emul[N - 2], st.eshift[N - 2]) * gm.nM;
                const float* br = bM + iM * 5;
                reg += br[2] * pc;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int d = q < 2 ? q - 2 : q - 1;
                    reg += br[q < 2 ? q : q + 1] * *reinterpret_cast<const vt*>(prow + d * gm.sM);
                }
            }
            if (has1) {
#pragma unroll
                for (int d = -2; d <= 2; ++d)
                    reg += b1[jr * 5 + d + 2] * *reinterpret_cast<const vt*>(prow + d * LDW);
            }
            if (hasN) {
                float w[12];
                const vt pl = *reinterpret_cast<const vt*>(prow - 4);
                const vt pr = *reinterpret_cast<const vt*>(prow + 4);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    w[e] = pl[e];
                    w[4 + e] = pc[e];
                    w[8 + e] = pr[e];
                }
                const int i0 = t - fast_div(t, st.emul[N - 1], st.eshift[N - 1]) * gm.nN;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float* bb = bN + (i0 + e) * 5;
#pragma unroll
                    for (int d = -2; d <= 2; ++d) reg[e] += bb[d + 2] * w[4 + e + d];
                }
            }
            const vt qv = s + lam * reg;
            *reinterpret_cast<vt*>(Q + (int64_t)j * trail + t) = qv;
#pragma unroll
            for (int e = 0; e < 4; ++e) dot_acc += (double)pc[e] * (double)qv[e];
        }
    }
    __syncthreads();  // LDS is reused by the next tile
}

// ---------------------------------------------------------------------------
// Tail pass on groups of `nb` consecutive blocks of the last two modes.  J2T:
// maximum number of 16-wide j2 tiles (compile time); the runtime count is
// (J2 + 15) / 16.  LDS: Zt for every block of the group, then the output
// blocks Ys, which are written back as one contiguous run (consecutive blocks
// are adjacent in memory).
__host__ __device__ inline int tail_zt_elems(int k1pad, int J2, int tc_size) {
    return ((J2 + 15) / 16) * 16 * (k1pad + 16 / tc_size);
}

template <typename Tin, typename Tout, typename Tc, int J2T, bool FUSE_P, bool FUSE_R = false>
__device__ __forceinline__ void tail_group(const TailArgs& a, int64_t blk0, int nb, int nbmax,
                                           unsigned char* smem, double* dot_acc = nullptr) {
    typedef MT<Tc> T;
    constexpr int VEC = T::VEC;
    const int ldz = a.k1pad + 16 / (int)sizeof(Tc);
    const int zsz = tail_zt_elems(a.k1pad, a.J2, (int)sizeof(Tc));
    Tc* Zt = reinterpret_cast<Tc*>(smem);
    Tout* Ys = reinterpret_cast<Tout*>(smem + (((size_t)nbmax * zsz * sizeof(Tc) + 15) / 16) * 16);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, l16 = lane & 15;
    const int64_t bin = (int64_t)a.K1 * a.K2;
    const int bout = a.J1 * a.J2;
    const Tc* __restrict__ M1 = reinterpret_cast<const Tc*>(a.M1);
    const Tc* __restrict__ M2 = reinterpret_cast<const Tc*>(a.M2);
    Tin beta = cvt<Tin>(0.f), alpha = cvt<Tin>(0.f);
    if constexpr (FUSE_P) {
        beta = cvt<Tin>(*a.beta);
        if (a.Xsol) alpha = cvt<Tin>(*a.alpha);
    }
    if constexpr (FUSE_R) alpha = cvt<Tin>(*a.alpha);
    const int nj2t = (a.J2 + 15) / 16;
    const int ni1t = a.k1pad / 16;
    const int nks2 = a.k2pad / T::KSTEP;
    // tile indices are split with a float reciprocal (small_div), not integer division
    const float inv_ni1t = 1.0f / (float)ni1t, inv_nj2t = 1.0f / (float)nj2t;
    const bool aligned2 = (a.K2 % VEC) == 0;

    // ---- step 1: Zt[b][j2][i1] = sum_k2 X_b[i1][k2] M2[j2][k2] ----
    if (!FUSE_P && !FUSE_R && nks2 == 1) {
        // one k step: the M2 fragments are the same for every tile, and a wave
        // loads the X fragments of TB tiles before the first MFMA, so TB loads
        // are in flight together (tiles past the end load the last tile again
        // and store nothing)
        constexpr int TB = 4;
        const int ntile = nb * ni1t;
        typename T::frag mf[J2T];
#pragma unroll
        for (int x = 0; x < J2T; ++x)
            mf[x] = *reinterpret_cast<const typename T::frag*>(
                M2 + (int64_t)(min(x, nj2t - 1) * 16 + l16) * a.ldm2 + VEC * g);
        const int k2 = VEC * g;
        for (int it0 = wave; it0 < ntile; it0 += CTA_WAVES * TB) {
            typename T::frag xf[TB];
#pragma unroll
            for (int i = 0; i < TB; ++i) {
                const int it = min(it0 + i * CTA_WAVES, ntile - 1);
                const int bl = small_div(it, ni1t, inv_ni1t), ti = it - bl * ni1t;
                const int i1 = ti * 16 + l16;
                const Tin* __restrict__ X = reinterpret_cast<const Tin*>(a.X) + (blk0 + bl) * bin;
                const int nv = (i1 < a.K1) ? max(0, min(VEC, a.K2 - k2)) : 0;
                xf[i] = nv > 0 ? load_frag<Tc>(X + (int64_t)i1 * a.K2 + k2, nv, aligned2) : T::zfrag();
            }
#pragma unroll
            for (int i = 0; i < TB; ++i) {
                const int it = it0 + i * CTA_WAVES;
                typename T::acc acc[J2T];
#pragma unroll
                for (int x = 0; x < J2T; ++x)
                    acc[x] = x < nj2t ? T::mma(xf[i], mf[x], T::zero()) : T::zero();
                if (it >= ntile) continue;
                const int bl = small_div(it, ni1t, inv_ni1t), ti = it - bl * ni1t;
                Tc* Zb = Zt + bl * zsz;
#pragma unroll
                for (int x = 0; x < J2T; ++x) {
                    if (x < nj2t) {
                        const int j2 = x * 16 + l16;
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            Zb[j2 * ldz + ti * 16 + T::arow(lane, r)] = cvt<Tc>(acc[x][r]);
                    }
                }
            }
        }
    } else
    for (int it = wave; it < nb * ni1t; it += CTA_WAVES) {
        const int bl = small_div(it, ni1t, inv_ni1t), ti = it - bl * ni1t;
        const int64_t off0 = (blk0 + bl) * bin;
        const Tin* __restrict__ X = reinterpret_cast<const Tin*>(a.X) + off0;
        const int i1 = ti * 16 + l16;
        typename T::acc acc[J2T];
#pragma unroll
        for (int x = 0; x < J2T; ++x) acc[x] = T::zero();
        if constexpr (!FUSE_P && !FUSE_R) {
            // X and M2 fragments of the next k step are loaded while the
            // current one multiplies (j2 tiles past nj2t read the last valid
            // one and are not used)
            const Tin* __restrict__ xrow = X + (int64_t)i1 * a.K2;
            auto xload = [&](int ks) {
                const int k2 = ks * T::KSTEP + VEC * g;
                const int nv = (i1 < a.K1) ? max(0, min(VEC, a.K2 - k2)) : 0;
                return nv > 0 ? load_frag<Tc>(xrow + k2, nv, aligned2) : T::zfrag();
            };
            typename T::frag xf = xload(0), mf[J2T];
#pragma unroll
            for (int x = 0; x < J2T; ++x)
                mf[x] = *reinterpret_cast<const typename T::frag*>(
                    M2 + (int64_t)(min(x, nj2t - 1) * 16 + l16) * a.ldm2 + VEC * g);
            for (int ks = 0; ks < nks2; ++ks) {
                const int kn = ks + 1 < nks2 ? ks + 1 : ks;
                const typename T::frag xn = xload(kn);
                typename T::frag mn[J2T];
#pragma unroll
                for (int x = 0; x < J2T; ++x)
                    mn[x] = *reinterpret_cast<const typename T::frag*>(
                        M2 + (int64_t)(min(x, nj2t - 1) * 16 + l16) * a.ldm2 + kn * T::KSTEP + VEC * g);
#pragma unroll
                for (int x = 0; x < J2T; ++x)
                    if (x < nj2t) acc[x] = T::mma(xf, mf[x], acc[x]);
                xf = xn;
#pragma unroll
                for (int x = 0; x < J2T; ++x) mf[x] = mn[x];
            }
        } else
        for (int ks = 0; ks < nks2; ++ks) {
            const int k2 = ks * T::KSTEP + VEC * g;
            const int nv = (i1 < a.K1) ? max(0, min(VEC, a.K2 - k2)) : 0;
            typename T::frag xf = T::zfrag();
            if constexpr (FUSE_R) {
                // r = r - alpha q on the fly, written back once, and its square
                // summed in FP64
                Tin* __restrict__ Rv = reinterpret_cast<Tin*>(a.Pvec) + off0;
                const Tin* __restrict__ Qv = reinterpret_cast<const Tin*>(a.Qvec) + off0;
                const int64_t off = (int64_t)i1 * a.K2 + k2;
                constexpr int LV = 16 / sizeof(Tin);
                if (nv == VEC && aligned2 && (VEC % LV) == 0) {
                    typedef Tin __attribute__((ext_vector_type(LV))) vin;
#pragma unroll
                    for (int h = 0; h < VEC / LV; ++h) {
                        const vin rv = *reinterpret_cast<const vin*>(Rv + off + h * LV);
                        const vin qv = *reinterpret_cast<const vin*>(Qv + off + h * LV);
                        const vin rn = rv - alpha * qv;
                        *reinterpret_cast<vin*>(Rv + off + h * LV) = rn;
#pragma unroll
                        for (int v = 0; v < LV; ++v) {
                            xf[h * LV + v] = cvt<Tc>(rn[v]);
                            *dot_acc += (double)rn[v] * (double)rn[v];
                        }
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) {
                        if (v < nv) {
                            const Tin rn = Rv[off + v] - alpha * Qv[off + v];
                            Rv[off + v] = rn;
                            xf[v] = cvt<Tc>(rn);
                            *dot_acc += (double)rn * (double)rn;
                        }
                    }
                }
            } else {
                // x += alpha p (previous step, optional), then p = r + beta * p on
                // the fly; the new p is written back once
                Tin* __restrict__ Pv = reinterpret_cast<Tin*>(a.Pvec) + off0;
                Tin* __restrict__ Xs = a.Xsol ? reinterpret_cast<Tin*>(a.Xsol) + off0 : nullptr;
                const int64_t off = (int64_t)i1 * a.K2 + k2;
                constexpr int LV = 16 / sizeof(Tin);
                if (nv == VEC && aligned2 && (VEC % LV) == 0) {
                    typedef Tin __attribute__((ext_vector_type(LV))) vin;
#pragma unroll
                    for (int h = 0; h < VEC / LV; ++h) {
                        const vin rv = *reinterpret_cast<const vin*>(X + off + h * LV);
                        const vin pv = *reinterpret_cast<const vin*>(Pv + off + h * LV);
                        if (Xs) {
                            const vin xv = *reinterpret_cast<const vin*>(Xs + off + h * LV);
                            *reinterpret_cast<vin*>(Xs + off + h * LV) = xv + alpha * pv;
                        }
                        const vin pn = rv + beta * pv;
                        *reinterpret_cast<vin*>(Pv + off + h * LV) = pn;
#pragma unroll
                        for (int v = 0; v < LV; ++v) xf[h * LV + v] = cvt<Tc>(pn[v]);
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) {
                        if (v < nv) {
                            const Tin po = Pv[off + v];
                            if (Xs) Xs[off + v] = Xs[off + v] + alpha * po;
                            const Tin pn = X[off + v] + beta * po;
                            Pv[off + v] = pn;
                            xf[v] = cvt<Tc>(pn);
                        }
                    }
                }
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
        Tc* Zb = Zt + bl * zsz;
#pragma unroll
        for (int x = 0; x < J2T; ++x) {
            if (x < nj2t) {
                const int j2 = x * 16 + l16;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    Zb[j2 * ldz + ti * 16 + T::arow(lane, r)] = cvt<Tc>(acc[x][r]);
            }
        }
    }
    __syncthreads();

    // ---- step 2: Ys[b][j1][j2] = sum_i1 M1[j1][i1] Zt[b][j2][i1] ----
    const int nj1t = (a.J1 + 15) / 16;
    const int nsub = nj2t * nj1t;
    const float inv_nsub = 1.0f / (float)nsub;
    const int nks1 = a.k1pad / T::KSTEP;
    for (int sidx = wave; sidx < nb * nsub; sidx += CTA_WAVES) {
        const int bl = small_div(sidx, nsub, inv_nsub), sb = sidx - bl * nsub;
        const int x1 = small_div(sb, nj2t, inv_nj2t), x2 = sb - x1 * nj2t;
        const Tc* Zb = Zt + bl * zsz;
        typename T::acc acc = T::zero();
        // the M1 fragment of the next k step is loaded during the current MFMA
        const Tc* __restrict__ m1row = M1 + (int64_t)(x1 * 16 + l16) * a.ldm1 + VEC * g;
        const Tc* zrow = Zb + (x2 * 16 + l16) * ldz + VEC * g;
        typename T::frag mf = *reinterpret_cast<const typename T::frag*>(m1row);
        for (int ks = 0; ks < nks1; ++ks) {
            const int kn = (ks + 1 < nks1 ? ks + 1 : ks) * T::KSTEP;
            const typename T::frag mn = *reinterpret_cast<const typename T::frag*>(m1row + kn);
            const typename T::frag zf = *reinterpret_cast<const typename T::frag*>(zrow + ks * T::KSTEP);
            acc = T::mma(zf, mf, acc);
            mf = mn;
        }
        const int j1 = x1 * 16 + l16;
        if (j1 < a.J1) {
            Tout* yb = Ys + bl * bout + j1 * a.J2;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j2 = x2 * 16 + T::arow(lane, r);
                if (j2 < a.J2) yb[j2] = cvt<Tout>(acc[r]);
            }
        }
    }
    __syncthreads();

    // ---- contiguous write-back of the nb output blocks ----
    Tout* __restrict__ Y = reinterpret_cast<Tout*>(a.Y) + blk0 * bout;
    const int total = nb * bout;
    constexpr int OV = 16 / sizeof(Tout);
    if ((reinterpret_cast<uintptr_t>(Y) & 15) == 0 && (total % OV) == 0) {
        typedef Tout __attribute__((ext_vector_type(OV))) vo;
        for (int i = threadIdx.x * OV; i < total; i += CTA_WG * OV)
            *reinterpret_cast<vo*>(Y + i) = *reinterpret_cast<const vo*>(Ys + i);
    } else {
        for (int i = threadIdx.x; i < total; i += CTA_WG) Y[i] = Ys[i];
    }
    __syncthreads();  // LDS is reused by the next group
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
    // the X and M fragments of the next k step are loaded while the current
    // one multiplies
    auto xload = [&](int ks) {
        const int k = ks * T::KSTEP + VEC * g;
        const int nv = (row < a.rows) ? max(0, min(VEC, a.K - k)) : 0;
        return (nv > 0) ? load_frag<Tc>(X + row * a.K + k, nv, (a.K % VEC) == 0) : T::zfrag();
    };
    const Tc* mrow[JT];
#pragma unroll
    for (int x = 0; x < JT; ++x) mrow[x] = M + (int64_t)(a.j0 + x * 16 + l16) * a.ldm + VEC * g;
    typename T::frag xf = xload(0), mf[JT];
#pragma unroll
    for (int x = 0; x < JT; ++x) mf[x] = *reinterpret_cast<const typename T::frag*>(mrow[x]);
    for (int ks = 0; ks < nks; ++ks) {
        const int kn = ks + 1 < nks ? ks + 1 : ks;
        const typename T::frag xn = xload(kn);
        typename T::frag mn[JT];
#pragma unroll
        for (int x = 0; x < JT; ++x)
            mn[x] = *reinterpret_cast<const typename T::frag*>(mrow[x] + kn * T::KSTEP);
#pragma unroll
        for (int x = 0; x < JT; ++x) acc[x] = T::mma(mf[x], xf, acc[x]);
        xf = xn;
#pragma unroll
        for (int x = 0; x < JT; ++x) mf[x] = mn[x];
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
