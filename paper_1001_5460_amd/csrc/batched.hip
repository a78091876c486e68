// Batched persistent solver: many independent order-3 tensor equations (each
// with its own extents, factors and lambda) solved by the tensor CG of
// Fig. Tensor_CG in ONE kernel launch.
//
// Work distribution.  The grid is split into teams of S workgroups; every
// team owns a list of problems, assigned on the host largest-first to the
// least-loaded team (so big problems start first and the tail of the
// schedule is made of small ones).  Inside a team each CG phase -- fused tail
// pass (p = r + beta p, modes 2 and 3), mode-1 pass with the banded
// regulariser and <p, q>, vector update with <r, r> -- is split across the
// team's workgroups, and the team synchronises between phases:
//   S == 1: __syncthreads only (no fences, no atomics);
//   S  > 1: a device-memory barrier (agent-scope release/acquire around an
//           arrival counter and a generation word) with a bounded spin: a
//           wait that exceeds the limit sets an error flag and the kernel
//           exits, so every workgroup always finishes.
// Members of a team are placed on the same XCD (workgroup b runs on XCD b % 8).
// Scalars (rho, alpha, beta) are formed by every member from the team's
// partials in member order, so all members agree bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/cta.h"
#include "abi_internal.hpp"
#include "launch.hpp"
#include "prof.hpp"
#include "reduce.hpp"
#include "ttm.hpp"

namespace cta {

struct BatchProblem {
    int n0, n1, n2;
    int64_t N;
    const float* G[3];
    int ldG[3];
    const float* rb[3];
    double lam;
    const float* b;
    float* x;
    float* r;
    float* p;
    float* q;
    float* t1;
    double rtol2;
    int max_iter;
    int jcls;   // mode-1 tile class (see last_tile_dispatch)
    int j2cls;  // tail j2 class
    int nbg;    // tail blocks per group
};

struct BatchResult {
    int status;  // DONE_* flag
    int iters;
    double rho;
    double bnorm2;
};

struct TeamSync {
    unsigned count;
    unsigned gen;
    unsigned pad[62];  // one 256-byte line per team
};

constexpr int kBatchSpin = 1 << 24;

// Team barrier.  S == 1 needs only the workgroup barrier.
__device__ __forceinline__ bool team_barrier(TeamSync* ts, int S, unsigned& gen, int* err) {
    __syncthreads();
    if (S == 1) return true;
    __shared__ int s_ok;
    if (threadIdx.x == 0) {
        __threadfence();  // release this workgroup's writes
        const unsigned g = gen;
        int ok = 1;
        if (atomicAdd(&ts->count, 1u) == (unsigned)S - 1u) {
            __hip_atomic_store(&ts->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            atomicAdd(&ts->gen, 1u);
        } else {
            int spins = 0;
            while (__hip_atomic_load(&ts->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > kBatchSpin || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 0;
                    atomicExch(err, 1);
                    break;
                }
            }
        }
        __threadfence();  // acquire the other members' writes
        gen = g + 1;
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Sum of the team's partial values in member order (identical on every member).
__device__ __forceinline__ double team_total(const double* part, int S) {
    double t = 0.0;
    for (int m = 0; m < S; ++m) t += __hip_atomic_load(&part[m], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return t;
}

template <int JT, int WJ, int CT>
__device__ void last_tiles(const BatchProblem& pb, unsigned char* smem, int member, int S,
                           double& dot, int variant_tn32) {
    StridedArgs a{};
    a.X = pb.t1;
    a.Y = pb.q;
    a.M = pb.G[0];
    a.ldm = pb.ldG[0];
    a.K = pb.n0;
    a.J = pb.n0;
    a.kpad = (pb.n0 + 15) / 16 * 16;
    a.lead = 1;
    a.trail = (int64_t)pb.n1 * pb.n2;
    constexpr int TN = 16 * CT * (CTA_WAVES / WJ);
    a.ntt = (a.trail + TN - 1) / TN;
    a.ntiles = a.ntt;
    StencilArgs<float> st{};
    st.P = pb.p;
    st.rband[0] = pb.rb[0];
    st.rband[1] = pb.rb[1];
    st.rband[2] = pb.rb[2];
    st.ext[0] = pb.n0;
    st.ext[1] = pb.n1;
    st.ext[2] = pb.n2;
    st.stride[0] = (int64_t)pb.n1 * pb.n2;
    st.stride[1] = pb.n2;
    st.stride[2] = 1;
    st.order = 3;
    st.lam = pb.lam;
    st.partials = nullptr;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        fastdiv_init((uint32_t)st.stride[k], &st.smul[k], &st.sshift[k]);
        fastdiv_init((uint32_t)st.ext[k], &st.emul[k], &st.eshift[k]);
    }
    for (int64_t tile = member; tile < a.ntiles; tile += S)
        normal_last_tile<float, float, float, JT, WJ, CT, 3>(a, tile, smem, st, dot);
}

// Mode-1 pass for the problem's n0: the same tile classes as the single-problem path.
__device__ void last_tile_dispatch(const BatchProblem& pb, unsigned char* smem, int member, int S,
                                   double& dot) {
    switch (pb.jcls) {
        case 1: last_tiles<1, 2, 2>(pb, smem, member, S, dot, 0); break;
        case 2: last_tiles<1, 4, 4>(pb, smem, member, S, dot, 0); break;
        case 3: last_tiles<3, 2, 2>(pb, smem, member, S, dot, 0); break;
        case 5: last_tiles<1, 2, 1>(pb, smem, member, S, dot, 1); break;
        case 6: last_tiles<1, 4, 2>(pb, smem, member, S, dot, 1); break;
        case 7: last_tiles<3, 2, 1>(pb, smem, member, S, dot, 1); break;
        default: break;
    }
}

template <int J2T>
__device__ void tail_blocks(const BatchProblem& pb, unsigned char* smem, int member, int S,
                            const double* beta) {
    TailArgs a{};
    a.X = pb.r;
    a.Y = pb.t1;
    a.M1 = pb.G[1];
    a.M2 = pb.G[2];
    a.ldm1 = pb.ldG[1];
    a.ldm2 = pb.ldG[2];
    a.K1 = pb.n1;
    a.K2 = pb.n2;
    a.J1 = pb.n1;
    a.J2 = pb.n2;
    a.k1pad = (pb.n1 + 15) / 16 * 16;
    a.k2pad = (pb.n2 + 15) / 16 * 16;
    a.nblk = pb.n0;
    a.Pvec = pb.p;
    a.beta = beta;
    a.done = nullptr;
    a.nbg = pb.nbg;
    const int64_t ngroups = (a.nblk + a.nbg - 1) / a.nbg;
    for (int64_t g = member; g < ngroups; g += S) {
        const int64_t blk0 = g * a.nbg;
        const int nb = (int)std::min<int64_t>(a.nbg, a.nblk - blk0);
        tail_group<float, float, float, J2T, true>(a, blk0, nb, a.nbg, smem);
    }
}

__global__ __launch_bounds__(CTA_WG) void k_batched(const BatchProblem* __restrict__ probs,
                                                    const int* __restrict__ plist,
                                                    const int2* __restrict__ team_range,
                                                    BatchResult* res, TeamSync* sync,
                                                    double* team_part, int S, int* err) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[4];
    __shared__ double s_beta;
    const int G = gridDim.x;
    const int b = blockIdx.x;
    // XCD-aware team membership: members of a team share b % 8
    const int x = b % CTA_XCDS, li = b / CTA_XCDS;
    const int teams_per_xcd = G / CTA_XCDS / S;
    const int team = x * teams_per_xcd + li / S;
    const int member = li % S;
    TeamSync* ts = sync + team;
    double* part = team_part + (size_t)team * S * 4;
    unsigned gen = 0;
    const int2 rg = team_range[team];
    for (int pi = rg.x; pi < rg.y; ++pi) {
        const BatchProblem pb = probs[plist[pi]];
        const int64_t N = pb.N;
        const int64_t chunk = (int64_t)CTA_WG * 4;
        const int64_t nch = (N + chunk - 1) / chunk;
        // ---- setup: x = 0, p = 0, r = b, rho = <b, b> ----
        double acc = 0.0;
        for (int64_t c = member; c < nch; c += S) {
            for (int64_t i = c * chunk + threadIdx.x; i < std::min<int64_t>((c + 1) * chunk, N); i += CTA_WG) {
                const float bv = pb.b[i];
                pb.r[i] = bv;
                pb.x[i] = 0.f;
                pb.p[i] = 0.f;
                acc += (double)bv * (double)bv;
            }
        }
        double sacc = block_sum(acc, red);
        if (threadIdx.x == 0) __hip_atomic_store(&part[member], sacc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!team_barrier(ts, S, gen, err)) return;
        const double bnorm2 = team_total(part, S);
        double rho = bnorm2;
        const double thr = pb.rtol2 * bnorm2;
        int status = DONE_RUNNING, it = 0;
        if (!__builtin_isfinite(rho)) status = DONE_BREAKDOWN;
        else if (rho <= thr) status = DONE_CONVERGED;
        else if (pb.max_iter <= 0) status = DONE_MAXITER;
        double beta = 0.0;
        while (status == DONE_RUNNING) {
            // ---- tail pass on (r + beta p), writes p and t1 ----
            if (threadIdx.x == 0) s_beta = beta;
            __syncthreads();
            switch (pb.j2cls) {
                case 0: tail_blocks<2>(pb, smem, member, S, &s_beta); break;
                case 1: tail_blocks<4>(pb, smem, member, S, &s_beta); break;
                default: tail_blocks<8>(pb, smem, member, S, &s_beta); break;
            }
            if (!team_barrier(ts, S, gen, err)) return;
            // ---- mode-1 pass + regulariser, <p, q> ----
            double dot = 0.0;
            last_tile_dispatch(pb, smem, member, S, dot);
            sacc = block_sum(dot, red);
            if (threadIdx.x == 0) __hip_atomic_store(&part[S + member], sacc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!team_barrier(ts, S, gen, err)) return;
            const double pq = team_total(part + S, S);
            if (!(pq > 0.0) || !__builtin_isfinite(pq)) {
                status = DONE_BREAKDOWN;
                break;
            }
            const double alpha = rho / pq;
            const float af = (float)alpha;
            // ---- x += alpha p, r -= alpha q, <r, r> ----
            acc = 0.0;
            for (int64_t c = member; c < nch; c += S) {
                for (int64_t i = c * chunk + threadIdx.x; i < std::min<int64_t>((c + 1) * chunk, N); i += CTA_WG) {
                    pb.x[i] += af * pb.p[i];
                    const float rv = pb.r[i] - af * pb.q[i];
                    pb.r[i] = rv;
                    acc += (double)rv * (double)rv;
                }
            }
            sacc = block_sum(acc, red);
            if (threadIdx.x == 0) __hip_atomic_store(&part[2 * S + member], sacc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!team_barrier(ts, S, gen, err)) return;
            const double rho1 = team_total(part + 2 * S, S);
            beta = rho1 / rho;
            rho = rho1;
            ++it;
            if (!__builtin_isfinite(rho1)) status = DONE_BREAKDOWN;
            else if (rho1 <= thr) status = DONE_CONVERGED;
            else if (it >= pb.max_iter) status = DONE_MAXITER;
        }
        if (member == 0 && threadIdx.x == 0) {
            BatchResult rr;
            rr.status = status;
            rr.iters = it;
            rr.rho = rho;
            rr.bnorm2 = bnorm2;
            res[plist[pi]] = rr;
        }
        // the next problem's setup overwrites vectors of another problem only
        if (!team_barrier(ts, S, gen, err)) return;
    }
}

// ---------------------------------------------------------------------------
// host side
namespace {

// Mode-1 tile class of the batched kernel (extents 17..96; the classes are
// the single-problem shapes for those extents).
int jclass(int n0, int variant) {
    const int jt = (n0 + 15) / 16;
    if (jt < 2 || jt > 6) return -1;
    if (variant == 1) return jt <= 2 ? 5 : (jt <= 4 ? 6 : 7);
    return jt <= 2 ? 1 : (jt <= 4 ? 2 : 3);
}

int tn_of_class(int c) {
    switch (c) {
        case 0: return 64;  // (1,1,1): 16*1*4
        case 1: return 64;
        case 2: return 64;
        case 3: return 64;
        case 4: return 64;
        default: return 32;
    }
}

size_t last_lds(int n0, int n1, int n2, int cls) {
    const int TN = tn_of_class(cls);
    const int kpad = (n0 + 15) / 16 * 16;
    const size_t xs = (size_t)TN * (kpad + 4) * 4;
    const size_t qs = (size_t)n0 * (TN + 4) * 4;
    const size_t a = ((std::max(xs, qs)) + 15) / 16 * 16;
    (void)n1;
    return a + (size_t)n0 * (TN + 8) * 4 + (size_t)(n0 + n2) * 5 * 4;
}

size_t tail_lds_f32(int n1, int n2, int nb) {
    const int k1pad = (n1 + 15) / 16 * 16;
    const size_t z = (size_t)nb * ((n2 + 15) / 16) * 16 * (k1pad + 4) * 4;
    return (z + 15) / 16 * 16 + (size_t)nb * n1 * n2 * 4;
}

struct BatchCfg {
    int S = 1;
    int last_variant = 0;
};

std::map<std::string, BatchCfg> g_cache;

std::string batch_key(int count, cta_op const* ops) {
    std::vector<std::string> shapes;
    for (int i = 0; i < count; ++i)
        shapes.push_back(std::to_string(ops[i]->n[0]) + "x" + std::to_string(ops[i]->n[1]) + "x" +
                         std::to_string(ops[i]->n[2]));
    std::sort(shapes.begin(), shapes.end());
    // key: count and a hash of the sorted shape list
    uint64_t h = 1469598103934665603ull;
    for (auto& s : shapes)
        for (char c : s) h = (h ^ (unsigned char)c) * 1099511628211ull;
    char buf[64];
    snprintf(buf, sizeof buf, "gfx950/batched/%d/%016llx", count, (unsigned long long)h);
    return buf;
}

}  // namespace

cta_status true_residual(cta_op_s* op, const void* B, const void* X, int tx, hipStream_t s,
                         double* res);

// Run the persistent kernel for `count` problems with configuration cfg.
static cta_status run_batched(int count, const cta_op* ops, const void* const* B, void* const* X,
                              const cta_cg_opts* opts, const BatchCfg& cfg, hipStream_t s,
                              std::vector<BatchResult>& out, double* kernel_ms) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(CTA_ERR_HIP, "hipGetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(CTA_ERR_HIP, "hipGetDeviceProperties failed");
    // problem descriptors
    std::vector<BatchProblem> pbs(count);
    size_t lds = 0;
    for (int i = 0; i < count; ++i) {
        const cta_op_s* op = ops[i];
        BatchProblem& pb = pbs[i];
        pb.n0 = (int)op->n[0];
        pb.n1 = (int)op->n[1];
        pb.n2 = (int)op->n[2];
        pb.N = op->N;
        for (int k = 0; k < 3; ++k) {
            pb.G[k] = reinterpret_cast<const float*>(op->G[DT_F32][k].p);
            pb.ldG[k] = op->G[DT_F32][k].ld;
            pb.rb[k] = reinterpret_cast<const float*>(op->rband[1][k]);
        }
        pb.lam = op->lam;
        pb.b = reinterpret_cast<const float*>(B[i]);
        pb.x = reinterpret_cast<float*>(X[i]);
        pb.r = reinterpret_cast<float*>(op->vr);
        pb.p = reinterpret_cast<float*>(op->vp);
        pb.q = reinterpret_cast<float*>(op->vq);
        pb.t1 = reinterpret_cast<float*>(op->T1);
        pb.rtol2 = opts->rtol * opts->rtol;
        pb.max_iter = opts->max_iter;
        pb.jcls = jclass(pb.n0, cfg.last_variant);
        if (pb.jcls < 0) return fail(CTA_ERR_SHAPE, "problem %d: n1 = %d outside [17, 96]", i, pb.n0);
        const int j2t = (pb.n2 + 15) / 16;
        pb.j2cls = j2t <= 2 ? 0 : (j2t <= 4 ? 1 : 2);
        if (j2t > 8) return fail(CTA_ERR_SHAPE, "problem %d: n3 = %d above 128", i, pb.n2);
        const int ni1t = (pb.n1 + 15) / 16;
        pb.nbg = (ni1t % 4 == 0) ? 1 : (ni1t % 2 == 0 ? 2 : 4);
        while (pb.nbg > 1 && tail_lds_f32(pb.n1, pb.n2, pb.nbg) > 64 * 1024) pb.nbg /= 2;
        lds = std::max(lds, last_lds(pb.n0, pb.n1, pb.n2, pb.jcls));
        lds = std::max(lds, tail_lds_f32(pb.n1, pb.n2, pb.nbg));
    }
    if (lds > 160 * 1024) return fail(CTA_ERR_SHAPE, "batched problems need %zu bytes of LDS", lds);
    // co-resident grid, a multiple of 8 * S
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batched, CTA_WG, lds) != hipSuccess || per_cu < 1)
        return fail(CTA_ERR_HIP, "occupancy query failed");
    const int S = cfg.S;
    int G = std::min(per_cu, 2) * prop.multiProcessorCount;
    G = G / (CTA_XCDS * S) * (CTA_XCDS * S);
    if (G < CTA_XCDS * S) return fail(CTA_ERR_UNSUPPORTED, "grid too small for team size %d", S);
    const int T = G / S;
    // largest-first assignment to the least-loaded team (static LPT schedule)
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return pbs[a].N > pbs[b].N; });
    std::vector<std::vector<int>> lists(T);
    std::vector<double> load(T, 0.0);
    for (int i : order) {
        const int t = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        lists[t].push_back(i);
        load[t] += (double)pbs[i].N;
    }
    std::vector<int> plist;
    std::vector<int2> ranges(T);
    for (int t = 0; t < T; ++t) {
        ranges[t].x = (int)plist.size();
        plist.insert(plist.end(), lists[t].begin(), lists[t].end());
        ranges[t].y = (int)plist.size();
    }
    // device copies of the schedule in one buffer owned by the first problem's
    // handle: allocated on first use, grown when a larger set needs more, freed
    // with that handle (a call synchronises its stream before returning, so
    // the buffer is idle between calls)
    auto al = [](size_t b) { return (std::max<size_t>(b, 1) + 255) / 256 * 256; };
    const size_t o_pb = 0;
    const size_t o_pl = o_pb + al(sizeof(BatchProblem) * count);
    const size_t o_rg = o_pl + al(sizeof(int) * count);
    const size_t o_res = o_rg + al(sizeof(int2) * T);
    const size_t o_sync = o_res + al(sizeof(BatchResult) * count);
    const size_t o_part = o_sync + al(sizeof(TeamSync) * T);
    const size_t o_err = o_part + al(sizeof(double) * T * S * 4);
    const size_t total = o_err + al(sizeof(int) * 64);
    cta_op_s* owner = ops[0];
    if (owner->batch_bytes < total) {
        if (owner->batch_buf) (void)hipFree(owner->batch_buf);
        owner->batch_buf = nullptr;
        owner->batch_bytes = 0;
        if (hipMalloc(&owner->batch_buf, total) != hipSuccess) {
            owner->batch_buf = nullptr;
            return fail(CTA_ERR_NOMEM, "allocation of the batched schedule failed");
        }
        owner->batch_bytes = total;
    }
    char* base = (char*)owner->batch_buf;
    BatchProblem* d_pb = (BatchProblem*)(base + o_pb);
    int* d_plist = (int*)(base + o_pl);
    int2* d_rg = (int2*)(base + o_rg);
    BatchResult* d_res = (BatchResult*)(base + o_res);
    TeamSync* d_sync = (TeamSync*)(base + o_sync);
    double* d_part = (double*)(base + o_part);
    int* d_err = (int*)(base + o_err);
    hipError_t e = hipMemcpyAsync(d_pb, pbs.data(), sizeof(BatchProblem) * count, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_plist, plist.data(), sizeof(int) * count, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_rg, ranges.data(), sizeof(int2) * T, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(d_sync, 0, sizeof(TeamSync) * T, s);
    if (e == hipSuccess) e = hipMemsetAsync(d_err, 0, sizeof(int) * 64, s);
    if (e == hipSuccess) e = hipMemsetAsync(d_res, 0, sizeof(BatchResult) * count, s);
    if (e == hipSuccess && lds > 65536)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_batched),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess) {
        ProfScope ps("batched", s);
        int Sv = S;
        if (S == 1) {
            k_batched<<<G, CTA_WG, lds, s>>>(d_pb, d_plist, d_rg, d_res, d_sync, d_part, Sv, d_err);
            e = hipGetLastError();
        } else {
            void* args[] = {&d_pb, &d_plist, &d_rg, &d_res, &d_sync, &d_part, &Sv, &d_err};
            e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_batched), dim3(G), dim3(CTA_WG),
                                           args, lds, s);
        }
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    int herr = 0;
    out.assign(count, BatchResult{});
    if (e == hipSuccess) e = hipMemcpyAsync(out.data(), d_res, sizeof(BatchResult) * count, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&herr, d_err, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(CTA_ERR_HIP, "batched launch: %s", hipGetErrorString(e));
    if (herr) return fail(CTA_ERR_HIP, "a team barrier exceeded its spin limit");
    if (kernel_ms) *kernel_ms = ms;
    return CTA_OK;
}

}  // namespace cta

using namespace cta;

static cta_status check_batch(int count, const cta_op* ops, const void* const* B, void* const* X,
                              cta_dtype dtype, const cta_cg_opts* opts) {
    if (count < 1 || !ops || !B || !X || !opts) return fail(CTA_ERR_ARG, "NULL argument or count < 1");
    if (dtype != CTA_F32 || opts->precision != CTA_PREC_F32)
        return fail(CTA_ERR_DTYPE, "the batched solver runs in CTA_PREC_F32 on CTA_F32 tensors");
    if (opts->x0_given) return fail(CTA_ERR_UNSUPPORTED, "the batched solver starts from zero");
    if (opts->precond) return fail(CTA_ERR_UNSUPPORTED, "the batched solver has no preconditioner");
    for (int i = 0; i < count; ++i) {
        if (!ops[i] || !B[i] || !X[i]) return fail(CTA_ERR_ARG, "problem %d: NULL handle or tensor", i);
        if (ops[i]->user_order != 3) return fail(CTA_ERR_SHAPE, "problem %d: the batched solver takes order-3 problems", i);
        if (ops[i]->n[0] < 17 || ops[i]->n[0] > 96 || ops[i]->n[1] > 128 || ops[i]->n[2] > 128)
            return fail(CTA_ERR_SHAPE, "problem %d: batched extents are n1 in [17, 96], n2 and n3 <= 128", i);
    }
    return CTA_OK;
}

extern "C" cta_status cta_solve_batched(int count, const cta_op* ops, const void* const* B,
                                        void* const* X, cta_dtype dtype, const cta_cg_opts* opts,
                                        cta_cg_info* host_infos, void* stream) {
    cta_status st = check_batch(count, ops, B, X, dtype, opts);
    if (st != CTA_OK) return st;
    if (!host_infos) return fail(CTA_ERR_ARG, "host_infos is NULL");
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    BatchCfg cfg;
    auto it = g_cache.find(batch_key(count, ops));
    if (it != g_cache.end()) cfg = it->second;
    std::vector<BatchResult> res;
    double ms = 0;
    st = run_batched(count, ops, B, X, opts, cfg, s, res, &ms);
    if (st != CTA_OK) return st;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    cta_status worst = CTA_OK;
    for (int i = 0; i < count; ++i) {
        cta_cg_info& inf = host_infos[i];
        std::memset(&inf, 0, sizeof inf);
        inf.iters = res[i].iters;
        inf.rel_res_recursive = std::sqrt(std::max(0.0, res[i].rho) / std::max(res[i].bnorm2, 1e-300));
        double tr = 0;
        st = true_residual(ops[i], B[i], X[i], DT_F32, s, &tr);
        if (st != CTA_OK) return st;
        inf.rel_res_true = res[i].bnorm2 > 0 ? tr / std::sqrt(res[i].bnorm2) : tr;
        inf.seconds = secs;
        int done = res[i].status;
        if (done == DONE_CONVERGED && std::isfinite(inf.rel_res_true) && inf.rel_res_true > opts->rtol &&
            res[i].iters < opts->max_iter) {
            // the recursive residual met the tolerance but the recomputed one did
            // not: restart once from the current iterate (the CG of the
            // single-problem path, which recomputes the residual first)
            cta_cg_opts o2 = *opts;
            o2.x0_given = 1;
            o2.fallback_zero = 0;
            o2.max_iter = opts->max_iter - res[i].iters;
            cta_cg_info i2;
            const cta_status s2 = cta_cg_solve(ops[i], B[i], X[i], CTA_F32, &o2, &i2, stream);
            if (s2 != CTA_OK && s2 != CTA_NOT_CONVERGED && s2 != CTA_ERR_BREAKDOWN) return s2;
            inf.iters += i2.iters;
            inf.rel_res_recursive = i2.rel_res_recursive;
            inf.rel_res_true = i2.rel_res_true;
            done = s2 == CTA_OK ? DONE_CONVERGED : (s2 == CTA_ERR_BREAKDOWN ? DONE_BREAKDOWN : DONE_MAXITER);
        }
        if (done == DONE_CONVERGED && std::isfinite(inf.rel_res_true) && inf.rel_res_true > opts->rtol)
            done = DONE_MAXITER;
        inf.status = done == DONE_CONVERGED ? CTA_OK : (done == DONE_BREAKDOWN ? CTA_ERR_BREAKDOWN : CTA_NOT_CONVERGED);
        if (inf.status == CTA_ERR_BREAKDOWN) worst = CTA_ERR_BREAKDOWN;
        else if (inf.status == CTA_NOT_CONVERGED && worst == CTA_OK) worst = CTA_NOT_CONVERGED;
    }
    const double secs_all = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < count; ++i) host_infos[i].seconds = secs_all;
    if (worst == CTA_ERR_BREAKDOWN) return fail(CTA_ERR_BREAKDOWN, "CG breakdown in at least one problem");
    if (worst == CTA_NOT_CONVERGED) return fail(CTA_NOT_CONVERGED, "at least one problem did not converge");
    return CTA_OK;
}

// Autotuner of the batched solver: candidate team sizes and mode-1 tile
// shapes are each run for a fixed number of CG iterations on the given
// problems (timed by events around the persistent launch, median of `reps`);
// candidates whose iterates differ from the reference configuration by more
// than 1e-4 (relative, after the same iterations) are rejected.  The fastest
// goes into the process-wide cache under a key made of the problem shapes.
extern "C" cta_status cta_tune_batched(int count, const cta_op* ops, int reps, const char* cache_path,
                                       void* stream) {
    if (count < 1 || !ops) return fail(CTA_ERR_ARG, "NULL argument or count < 1");
    hipStream_t s = (hipStream_t)stream;
    if (reps < 1) reps = 3;
    cta_cg_opts o;
    cta_cg_opts_default(&o);
    o.precision = CTA_PREC_F32;
    o.rtol = 0.0;
    o.max_iter = 20;
    // inputs: a fixed pattern as B, outputs in the handles' spare vector
    std::vector<const void*> Bs(count);
    std::vector<void*> Xs(count);
    for (int i = 0; i < count; ++i) {
        if (!ops[i] || ops[i]->user_order != 3) return fail(CTA_ERR_SHAPE, "problem %d: order-3 handles only", i);
        cta_status st = launch_fill_pattern(DT_F32, ops[i]->vaux, ops[i]->N, s) == hipSuccess ? CTA_OK
                       : fail(CTA_ERR_HIP, "pattern fill failed");
        if (st != CTA_OK) return st;
        Bs[i] = ops[i]->vaux;
        Xs[i] = reinterpret_cast<char*>(ops[i]->vaux) + ((ops[i]->N * 4 + 255) / 256) * 256;
    }
    const BatchCfg cands[] = {{1, 0}, {1, 1}, {2, 0}, {2, 1}, {4, 0}, {4, 1}};
    BatchCfg best;
    double best_ms = 1e30;
    std::vector<std::vector<float>> ref(count);
    for (size_t ci = 0; ci < sizeof cands / sizeof cands[0]; ++ci) {
        std::vector<double> times;
        std::vector<BatchResult> res;
        bool ok = true;
        for (int r = 0; r < reps && ok; ++r) {
            double ms = 0;
            cta_status st = run_batched(count, ops, Bs.data(), Xs.data(), &o, cands[ci], s, res, &ms);
            if (st != CTA_OK) {
                ok = false;
                break;
            }
            times.push_back(ms);
        }
        if (!ok) continue;
        // compare the iterates with the reference configuration
        for (int i = 0; i < count && ok; ++i) {
            std::vector<float> h(ops[i]->N);
            if (hipMemcpy(h.data(), Xs[i], h.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
                return fail(CTA_ERR_HIP, "copy of a tuning iterate failed");
            if (ci == 0) {
                ref[i] = h;
            } else {
                double num = 0, den = 0;
                for (size_t k = 0; k < h.size(); ++k) {
                    const double d = (double)h[k] - (double)ref[i][k];
                    num += d * d;
                    den += (double)ref[i][k] * ref[i][k];
                }
                if (!(num <= 1e-8 * den)) ok = false;
            }
        }
        if (!ok) continue;
        std::sort(times.begin(), times.end());
        const double med = times[times.size() / 2];
        if (med < best_ms) {
            best_ms = med;
            best = cands[ci];
        }
    }
    const std::string key = batch_key(count, ops);
    g_cache[key] = best;
    if (cache_path) {
        FILE* f = fopen(cache_path, "w");
        if (!f) return fail(CTA_ERR_ARG, "cannot write %s", cache_path);
        fprintf(f, "{\n");
        size_t k = 0;
        for (auto& kv : g_cache)
            fprintf(f, "  \"%s\": {\"team\": %d, \"last_variant\": %d}%s\n", kv.first.c_str(), kv.second.S,
                    kv.second.last_variant, ++k < g_cache.size() ? "," : "");
        fprintf(f, "}\n");
        fclose(f);
    }
    return CTA_OK;
}

extern "C" cta_status cta_tune_load(const char* cache_path) {
    if (!cache_path) return fail(CTA_ERR_ARG, "cache_path is NULL");
    FILE* f = fopen(cache_path, "r");
    if (!f) return fail(CTA_ERR_ARG, "cannot read %s", cache_path);
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    fclose(f);
    // entries of the form "key": {"team": S, "last_variant": v}
    size_t pos = 0;
    int loaded = 0;
    while ((pos = text.find('"', pos)) != std::string::npos) {
        const size_t end = text.find('"', pos + 1);
        if (end == std::string::npos) break;
        const std::string key = text.substr(pos + 1, end - pos - 1);
        pos = end + 1;
        if (key.rfind("gfx950/", 0) != 0) continue;
        BatchCfg c;
        const size_t tpos = text.find("\"team\":", pos);
        const size_t vpos = text.find("\"last_variant\":", pos);
        if (tpos == std::string::npos || vpos == std::string::npos) break;
        c.S = atoi(text.c_str() + tpos + 7);
        c.last_variant = atoi(text.c_str() + vpos + 15);
        if (c.S != 1 && c.S != 2 && c.S != 4) return fail(CTA_ERR_ARG, "bad team size in %s", cache_path);
        if (c.last_variant != 0 && c.last_variant != 1) return fail(CTA_ERR_ARG, "bad variant in %s", cache_path);
        g_cache[key] = c;
        ++loaded;
        pos = vpos + 15;
    }
    if (!loaded) return fail(CTA_ERR_ARG, "no entries in %s", cache_path);
    return CTA_OK;
}

extern "C" cta_status cta_tune_dump(char* host_buf, size_t bytes, size_t* needed) {
    std::string out = "{";
    size_t k = 0;
    for (auto& kv : g_cache) {
        char buf[256];
        snprintf(buf, sizeof buf, "%s\"%s\": {\"team\": %d, \"last_variant\": %d}", k++ ? ", " : "",
                 kv.first.c_str(), kv.second.S, kv.second.last_variant);
        out += buf;
    }
    out += "}";
    if (needed) *needed = out.size();
    if (host_buf && bytes > 0) {
        const size_t n = std::min(bytes - 1, out.size());
        std::memcpy(host_buf, out.data(), n);
        host_buf[n] = 0;
    }
    return CTA_OK;
}
