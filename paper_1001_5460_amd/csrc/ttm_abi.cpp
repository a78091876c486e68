// C ABI of the general multi-mode product (Sec. 2.1, eq. separable_transf).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/cta.h"
#include "abi_internal.hpp"
#include "launch.hpp"

using namespace cta;

namespace {

struct TtmPlan {
    int N = 0;
    int64_t in_ext[CTA_MAX_ORDER], out_ext[CTA_MAX_ORDER];
    int rows_st[CTA_MAX_ORDER], ld[CTA_MAX_ORDER];
    size_t mat_off[CTA_MAX_ORDER];
    std::vector<int> modes, order;
    size_t buf_off0 = 0, buf_off1 = 0, total = 0;
};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

cta_status make_plan(int order, const int64_t* x_dims, uint32_t mode_mask, uint32_t trans_mask,
                     const int64_t* m_rows, const int64_t* m_cols, cta_dtype compute, TtmPlan* p) {
    if (order < 1 || order > CTA_MAX_ORDER) return fail(CTA_ERR_ARG, "order %d outside [1, %d]", order, CTA_MAX_ORDER);
    if (!x_dims) return fail(CTA_ERR_ARG, "x_dims is NULL");
    if (compute != CTA_F64 && compute != CTA_F32 && compute != CTA_BF16)
        return fail(CTA_ERR_DTYPE, "unknown compute dtype %d", (int)compute);
    if (mode_mask >> order) return fail(CTA_ERR_ARG, "mode_mask has bits beyond the order");
    if (mode_mask && (!m_rows || !m_cols)) return fail(CTA_ERR_ARG, "m_rows / m_cols are NULL");
    p->N = order;
    const int es = dt_size(compute);
    size_t off = 0;
    int64_t total_in = 1;
    for (int k = 0; k < order; ++k) {
        if (x_dims[k] < 1) return fail(CTA_ERR_SHAPE, "x_dims[%d] = %lld", k, (long long)x_dims[k]);
        p->in_ext[k] = p->out_ext[k] = x_dims[k];
        total_in *= x_dims[k];
        if (!((mode_mask >> k) & 1u)) continue;
        const bool tr = (trans_mask >> k) & 1u;
        const int64_t R = tr ? m_cols[k] : m_rows[k];
        const int64_t C = tr ? m_rows[k] : m_cols[k];
        if (C != x_dims[k])
            return fail(CTA_ERR_SHAPE, "mode %d: factor has %lld columns, tensor extent is %lld", k,
                        (long long)C, (long long)x_dims[k]);
        if (R < 1 || R > CTA_MAX_EXTENT || C > CTA_MAX_EXTENT)
            return fail(CTA_ERR_SHAPE, "mode %d: factor %lld x %lld outside the %d limit", k,
                        (long long)R, (long long)C, CTA_MAX_EXTENT);
        p->out_ext[k] = R;
        p->modes.push_back(k);
        p->rows_st[k] = (int)((R + 63) / 64 * 64);
        p->ld[k] = (int)((C + 31) / 32 * 32);
        p->mat_off[k] = off;
        off = align256(off + (size_t)p->rows_st[k] * p->ld[k] * es);
    }
    int64_t mx = total_in;
    p->order = plan_order(order, p->in_ext, p->out_ext, p->modes, &mx);
    mx = std::max<int64_t>(mx, total_in);
    p->buf_off0 = off;
    p->buf_off1 = align256(off + (size_t)mx * es);
    p->total = align256(p->buf_off1 + (size_t)mx * es);
    return CTA_OK;
}

}  // namespace

extern "C" size_t cta_ttm_workspace_bytes(int order, const int64_t* x_dims, uint32_t mode_mask,
                                          uint32_t trans_mask, const int64_t* m_rows,
                                          const int64_t* m_cols, cta_dtype compute) {
    TtmPlan p;
    if (make_plan(order, x_dims, mode_mask, trans_mask, m_rows, m_cols, compute, &p) != CTA_OK) return 0;
    return p.total;
}

// ---------------------------------------------------------------------------
// Fixed scratch of cta_ttm_noalloc: one array per GPU in the code object's
// device memory, reached only through the address hipGetSymbolAddress returns
// for the current device (the array's name in host code is not a device
// address).  Calls on one GPU share it.
static __device__ __align__(256) unsigned char scratch[CTA_TTM_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

cta_status scratch_for_current_device(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(CTA_ERR_HIP, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices) return fail(CTA_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(CTA_ERR_HIP, "hipGetSymbolAddress of the scratch array: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return CTA_OK;
}
}  // namespace

extern "C" cta_status cta_ttm(int order, const int64_t* x_dims, const void* X, cta_dtype x_dtype,
                              uint32_t mode_mask, uint32_t trans_mask, const void* const* M,
                              const int64_t* m_rows, const int64_t* m_cols, cta_dtype m_dtype,
                              cta_dtype compute, void* Y, cta_dtype y_dtype, void* workspace,
                              size_t workspace_bytes, void* stream) {
    TtmPlan p;
    cta_status st = make_plan(order, x_dims, mode_mask, trans_mask, m_rows, m_cols, compute, &p);
    if (st != CTA_OK) return st;
    for (cta_dtype d : {x_dtype, m_dtype, y_dtype})
        if (d != CTA_F64 && d != CTA_F32 && d != CTA_BF16) return fail(CTA_ERR_DTYPE, "unknown dtype %d", (int)d);
    if (!X || !Y) return fail(CTA_ERR_ARG, "X or Y is NULL");
    if (mode_mask && !M) return fail(CTA_ERR_ARG, "M is NULL");
    if (!workspace || workspace_bytes < p.total)
        return fail(CTA_ERR_ARG, "workspace of %zu bytes needed, %zu given", p.total, workspace_bytes);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(CTA_ERR_ARG, "workspace must be 256-byte aligned");
    if ((reinterpret_cast<uintptr_t>(X) & 15) || (reinterpret_cast<uintptr_t>(Y) & 15))
        return fail(CTA_ERR_ARG, "X and Y must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
    Mat mats[CTA_MAX_ORDER];
    for (int k : p.modes) {
        if (!M[k]) return fail(CTA_ERR_ARG, "M[%d] is NULL", k);
        const bool tr = (trans_mask >> k) & 1u;
        hipError_t e = launch_pad_matrix((int)m_dtype, (int)compute, M[k], (int)m_rows[k], (int)m_cols[k],
                                         tr ? 1 : 0, ws + p.mat_off[k], p.rows_st[k], p.ld[k], s);
        if (e != hipSuccess) return fail(CTA_ERR_HIP, "factor padding launch: %s", hipGetErrorString(e));
        mats[k].p = ws + p.mat_off[k];
        mats[k].ld = p.ld[k];
        mats[k].rows = (int)p.out_ext[k];
        mats[k].cols = (int)p.in_ext[k];
    }
    return run_chain(order, p.in_ext, p.out_ext, mats, p.order, X, (int)x_dtype, Y, (int)y_dtype,
                     (int)compute, ws + p.buf_off0, ws + p.buf_off1, s);
}

extern "C" cta_status cta_ttm_noalloc(int order, const int64_t* x_dims, const void* X, cta_dtype x_dtype,
                                      uint32_t mode_mask, uint32_t trans_mask, const void* const* M,
                                      const int64_t* m_rows, const int64_t* m_cols, cta_dtype m_dtype,
                                      cta_dtype compute, void* Y, cta_dtype y_dtype, void* stream) {
    TtmPlan p;
    cta_status st = make_plan(order, x_dims, mode_mask, trans_mask, m_rows, m_cols, compute, &p);
    if (st != CTA_OK) return st;
    if (p.total > (size_t)CTA_TTM_SCRATCH_BYTES)
        return fail(CTA_ERR_SHAPE, "this product needs %zu bytes of scratch; cta_ttm_noalloc has %zu",
                    p.total, (size_t)CTA_TTM_SCRATCH_BYTES);
    void* ws = nullptr;
    st = scratch_for_current_device(&ws);
    if (st != CTA_OK) return st;
    return cta_ttm(order, x_dims, X, x_dtype, mode_mask, trans_mask, M, m_rows, m_cols, m_dtype, compute, Y,
                   y_dtype, ws, (size_t)CTA_TTM_SCRATCH_BYTES, stream);
}
