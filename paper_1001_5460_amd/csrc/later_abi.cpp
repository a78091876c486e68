// Entry points of the learned warm start that this build does not provide
// yet: they report CTA_ERR_UNSUPPORTED.
#include "../../include/cta.h"
#include "abi_internal.hpp"

using namespace cta;

extern "C" cta_status cta_ws_create(cta_ws* out, int, const int64_t*, int, int, int, uint64_t, void*) {
    if (out) *out = nullptr;
    return fail(CTA_ERR_UNSUPPORTED, "the warm-start network is not available in this build");
}
extern "C" cta_status cta_ws_destroy(cta_ws) { return CTA_OK; }
extern "C" int64_t cta_ws_num_params(cta_ws) { return 0; }
extern "C" cta_status cta_ws_forward(cta_ws, const void*, void*, int, void*) {
    return fail(CTA_ERR_UNSUPPORTED, "the warm-start network is not available in this build");
}
extern "C" cta_status cta_ws_backward(cta_ws, const void*, void*) {
    return fail(CTA_ERR_UNSUPPORTED, "the warm-start network is not available in this build");
}
extern "C" cta_status cta_ws_mse(cta_ws, const void*, const void*, void*, double*, void*) {
    return fail(CTA_ERR_UNSUPPORTED, "the warm-start network is not available in this build");
}
extern "C" cta_status cta_ws_zero_grad(cta_ws, void*) {
    return fail(CTA_ERR_UNSUPPORTED, "the warm-start network is not available in this build");
}
extern "C" cta_status cta_ws_adam_step(cta_ws, float, float, float, float, void*) {
    return fail(CTA_ERR_UNSUPPORTED, "the warm-start network is not available in this build");
}
extern "C" cta_status cta_ws_params(cta_ws, void*, size_t, int, void*) {
    return fail(CTA_ERR_UNSUPPORTED, "the warm-start network is not available in this build");
}
