"""MI355X (gfx950) solver for regularised separable tensor equations.

The product is the C ABI library ``libcta.so`` (declared in ``include/cta.h``);
this package only loads it and marshals PyTorch device tensors into its calls.
Nothing here computes: if the library is missing, every call raises.
"""
from ._lib import (  # noqa: F401
    CtaError,
    CTA_OK,
    CTA_NOT_CONVERGED,
    PREC_F64,
    PREC_F32,
    PREC_BF16,
    PREC_BF16_REFINE,
    load_library,
    library_path,
    cta_version,
    cta_last_error,
    cta_ttm,
    cta_ttm_workspace_bytes,
    cta_op_create,
    cta_op_destroy,
    cta_op_device_bytes,
    cta_forward,
    cta_rhs,
    cta_apply_normal_op,
    cta_cg_opts_default,
    cta_cg_solve,
    cta_solve_batched,
    cta_tune_batched,
    cta_tune_load,
    cta_tune_dump,
    cta_ws_create,
    cta_ws_destroy,
    cta_ws_num_params,
    cta_ws_forward,
    cta_ws_backward,
    cta_ws_mse,
    cta_ws_zero_grad,
    cta_ws_adam_step,
    cta_ws_params,
    Operator,
    exported_symbols,
)
