"""ctypes binding of libcta.so: argument marshalling only.

Tensors are PyTorch tensors on the current HIP device (``torch.cuda``);
their ``data_ptr()`` and torch's current stream are handed to the C calls.
Every call checks device, dtype, shape and contiguity before calling, and
raises :class:`CtaError` with the library's message on a non-OK status
(``CTA_NOT_CONVERGED`` is returned in the info dict instead).
"""
import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
_LIB = None

CTA_OK = 0
CTA_NOT_CONVERGED = 1
F64, F32, BF16 = 0, 1, 2
PREC_F64, PREC_F32, PREC_BF16, PREC_BF16_REFINE, PREC_BF16_RELIABLE = 0, 1, 2, 3, 4
_STATUS = {0: "CTA_OK", 1: "CTA_NOT_CONVERGED", -1: "CTA_ERR_ARG", -2: "CTA_ERR_SHAPE",
           -3: "CTA_ERR_DTYPE", -4: "CTA_ERR_HIP", -5: "CTA_ERR_NOMEM",
           -6: "CTA_ERR_BREAKDOWN", -7: "CTA_ERR_UNSUPPORTED"}
_PREC = {"f64": PREC_F64, "f32": PREC_F32, "bf16": PREC_BF16, "bf16_refine": PREC_BF16_REFINE,
         "bf16_reliable": PREC_BF16_RELIABLE}


class CtaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


def library_path():
    return os.path.join(HERE, "libcta.so")


class _CgOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("rtol", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("x0_given", ctypes.c_int),
                ("fallback_zero", ctypes.c_int), ("inner_rtol", ctypes.c_double),
                ("max_refine", ctypes.c_int), ("check_every", ctypes.c_int),
                ("precond", ctypes.c_int)]


class _CgInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int),
                ("refine_steps", ctypes.c_int), ("rel_res_recursive", ctypes.c_double),
                ("rel_res_true", ctypes.c_double), ("seconds", ctypes.c_double)]


_P = ctypes.c_void_p
_I64P = ctypes.POINTER(ctypes.c_int64)
_SIGS = {
    "cta_last_error": (ctypes.c_char_p, []),
    "cta_version": (ctypes.c_char_p, []),
    "cta_ttm_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, _I64P, ctypes.c_uint32,
                                                  ctypes.c_uint32, _I64P, _I64P, ctypes.c_int]),
    "cta_ttm": (ctypes.c_int, [ctypes.c_int, _I64P, _P, ctypes.c_int, ctypes.c_uint32,
                               ctypes.c_uint32, ctypes.POINTER(_P), _I64P, _I64P, ctypes.c_int,
                               ctypes.c_int, _P, ctypes.c_int, _P, ctypes.c_size_t, _P]),
    "cta_ttm_noalloc": (ctypes.c_int, [ctypes.c_int, _I64P, _P, ctypes.c_int, ctypes.c_uint32,
                                       ctypes.c_uint32, ctypes.POINTER(_P), _I64P, _I64P, ctypes.c_int,
                                       ctypes.c_int, _P, ctypes.c_int, _P]),
    "cta_op_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _I64P, _I64P,
                                     ctypes.POINTER(_P), ctypes.POINTER(_P), _I64P,
                                     ctypes.c_double, _P]),
    "cta_op_destroy": (ctypes.c_int, [_P]),
    "cta_op_device_bytes": (ctypes.c_size_t, [_P]),
    "cta_forward": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, ctypes.c_int, ctypes.c_int, _P]),
    "cta_rhs": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, ctypes.c_int, ctypes.c_int, _P]),
    "cta_apply_normal_op": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.c_int, _P, _P]),
    "cta_op_set_preconditioner": (ctypes.c_int, [_P, ctypes.c_double]),
    "cta_apply_precond": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.c_int, _P, _P]),
    "cta_tune_preconditioner": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.POINTER(_CgOpts),
                                               ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                               ctypes.POINTER(ctypes.c_double), _P]),
    "cta_cg_opts_default": (None, [ctypes.POINTER(_CgOpts)]),
    "cta_cg_solve": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.POINTER(_CgOpts),
                                    ctypes.POINTER(_CgInfo), _P]),
    "cta_solve_batched": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                         ctypes.POINTER(_P), ctypes.c_int,
                                         ctypes.POINTER(_CgOpts), ctypes.POINTER(_CgInfo), _P]),
    "cta_tune_batched": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_P), ctypes.c_int,
                                        ctypes.c_char_p, _P]),
    "cta_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "cta_tune_dump": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t,
                                     ctypes.POINTER(ctypes.c_size_t)]),
    "cta_ws_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _I64P, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_uint64, _P]),
    "cta_ws_destroy": (ctypes.c_int, [_P]),
    "cta_ws_num_params": (ctypes.c_int64, [_P]),
    "cta_ws_forward": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P]),
    "cta_ws_backward": (ctypes.c_int, [_P, _P, _P]),
    "cta_ws_mse": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "cta_ws_zero_grad": (ctypes.c_int, [_P, _P]),
    "cta_ws_adam_step": (ctypes.c_int, [_P, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_float, _P]),
    "cta_ws_params": (ctypes.c_int, [_P, _P, ctypes.c_size_t, ctypes.c_int, _P]),
    "cta_tune_op": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P]),
    "cta_op_get_tuning": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "cta_op_set_tuning": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "cta_op_set_banded": (ctypes.c_int, [_P, ctypes.c_int]),
    "cta_op_band_width": (ctypes.c_int, [_P]),
    "cta_sop_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _I64P, ctypes.c_int64, _P,
                                      ctypes.POINTER(_P), _I64P, ctypes.c_double]),
    "cta_sop_destroy": (ctypes.c_int, [_P]),
    "cta_sop_layout": (ctypes.c_int, [_P, _I64P]),
    "cta_sop_forward": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P]),
    "cta_sop_adjoint": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P]),
    "cta_sop_apply_normal": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P, _P]),
    "cta_sop_cg_solve": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.POINTER(_CgOpts),
                                        ctypes.POINTER(_CgInfo), _P]),
    "cta_apply_jacobi": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.c_double, _P, _P]),
    "cta_jacobi_solve": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.POINTER(_CgOpts), ctypes.c_double,
                                        ctypes.POINTER(_CgInfo), _P]),
    "cta_op_set_multigrid": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_double]),
    "cta_op_multigrid_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), _I64P,
                                             ctypes.POINTER(ctypes.c_double), ctypes.c_int]),
    "cta_apply_multigrid": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.c_int, _P, _P]),
    "cta_prof_enable": (ctypes.c_int, [ctypes.c_int]),
    "cta_prof_reset": (ctypes.c_int, []),
    "cta_prof_read": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t,
                                     ctypes.POINTER(ctypes.c_size_t)]),
}


def load_library(path=None):
    """Load libcta.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    path = path or library_path()
    if not os.path.exists(path):
        raise CtaError(-7, f"{path} not found: build it with paper_1001_5460_amd.build")
    # torch first: libcta then binds to the HIP runtime torch already loaded,
    # so the process has one runtime and torch's streams and memory are
    # valid in the library (loaded first, libcta would pull in a second
    # runtime that holds the device)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def exported_symbols():
    """Function names declared in include/cta.h."""
    with open(os.path.join(ROOT, "include", "cta.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cta_[a-z0-9_]+)\s*\(", text)))


def _check(status, allow_not_converged=False):
    if status == CTA_OK or (allow_not_converged and status == CTA_NOT_CONVERGED):
        return status
    raise CtaError(status, _LIB.cta_last_error().decode())


def _torch():
    import torch
    return torch


def _dt(t):
    torch = _torch()
    m = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}
    if t.dtype not in m:
        raise CtaError(-3, f"unsupported tensor dtype {t.dtype}")
    return m[t.dtype]


def _dev(t, name="tensor"):
    if not t.is_cuda:
        raise CtaError(-1, f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise CtaError(-1, f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _i64(vals):
    return (ctypes.c_int64 * len(vals))(*[int(v) for v in vals])


def cta_version():
    return load_library().cta_version().decode()


def cta_last_error():
    return load_library().cta_last_error().decode()


_DT_NAME = {"f64": F64, "f32": F32, "bf16": BF16}


def cta_ttm_workspace_bytes(x_dims, mats_shapes, trans=(), compute="f32"):
    lib = load_library()
    order = len(x_dims)
    mask = 0
    rows = [0] * order
    cols = [0] * order
    for k, sh in enumerate(mats_shapes):
        if sh is not None:
            mask |= 1 << k
            rows[k], cols[k] = sh
    tmask = sum(1 << k for k in trans)
    return lib.cta_ttm_workspace_bytes(order, _i64(x_dims), mask, tmask, _i64(rows), _i64(cols),
                                       _DT_NAME[compute])


def cta_ttm(X, mats, trans=(), compute="f32", out=None, out_dtype=None, stream=None):
    """Y = X x_k op(M_k) for every k with mats[k] not None (op = transpose for k in trans)."""
    torch = _torch()
    lib = load_library()
    order = X.dim()
    if len(mats) != order:
        raise CtaError(-1, "one entry per mode is required in mats")
    mask, tmask = 0, 0
    rows, cols = [0] * order, [0] * order
    ptrs = (ctypes.c_void_p * order)()
    out_shape = list(X.shape)
    m_dtype = None
    for k, M in enumerate(mats):
        if M is None:
            continue
        mask |= 1 << k
        if M.dim() != 2:
            raise CtaError(-2, f"mats[{k}] must be a matrix")
        if m_dtype is None:
            m_dtype = M.dtype
        elif M.dtype != m_dtype:
            raise CtaError(-3, "all factors must share one dtype")
        rows[k], cols[k] = M.shape
        ptrs[k] = _dev(M, f"mats[{k}]").value
        if k in trans:
            tmask |= 1 << k
            out_shape[k] = M.shape[1]
        else:
            out_shape[k] = M.shape[0]
    if out is None:
        out = torch.empty(out_shape, dtype=out_dtype or X.dtype, device=X.device)
    if list(out.shape) != out_shape:
        raise CtaError(-2, f"out has shape {tuple(out.shape)}, expected {tuple(out_shape)}")
    cdt = _DT_NAME[compute]
    mdt = _dt(torch.empty(0, dtype=m_dtype)) if m_dtype is not None else F32
    ws_bytes = lib.cta_ttm_workspace_bytes(order, _i64(X.shape), mask, tmask, _i64(rows),
                                           _i64(cols), cdt)
    if ws_bytes == 0:
        _check(-2)
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=X.device)
    base = ws.data_ptr()
    aligned = (base + 255) // 256 * 256
    _check(lib.cta_ttm(order, _i64(X.shape), _dev(X, "X"), _dt(X), mask, tmask, ptrs,
                       _i64(rows), _i64(cols), mdt, cdt, _dev(out, "out"), _dt(out),
                       ctypes.c_void_p(aligned), ws_bytes, _stream(stream)))
    return out


def cta_ttm_noalloc(X, mats, trans=(), compute="f32", out=None, out_dtype=None, stream=None):
    """As cta_ttm, with the library's fixed scratch instead of a workspace (no allocation
    inside the library; ``out`` is allocated here only when not given)."""
    torch = _torch()
    lib = load_library()
    order = X.dim()
    if len(mats) != order:
        raise CtaError(-1, "one entry per mode is required in mats")
    mask, tmask = 0, 0
    rows, cols = [0] * order, [0] * order
    ptrs = (ctypes.c_void_p * order)()
    out_shape = list(X.shape)
    m_dtype = None
    for k, M in enumerate(mats):
        if M is None:
            continue
        mask |= 1 << k
        if m_dtype is None:
            m_dtype = M.dtype
        elif M.dtype != m_dtype:
            raise CtaError(-3, "all factors must share one dtype")
        rows[k], cols[k] = M.shape
        ptrs[k] = _dev(M, f"mats[{k}]").value
        out_shape[k] = M.shape[1] if k in trans else M.shape[0]
        if k in trans:
            tmask |= 1 << k
    if out is None:
        out = torch.empty(out_shape, dtype=out_dtype or X.dtype, device=X.device)
    if list(out.shape) != out_shape:
        raise CtaError(-2, f"out has shape {tuple(out.shape)}, expected {tuple(out_shape)}")
    mdt = _dt(torch.empty(0, dtype=m_dtype)) if m_dtype is not None else F32
    _check(lib.cta_ttm_noalloc(order, _i64(X.shape), _dev(X, "X"), _dt(X), mask, tmask, ptrs, _i64(rows),
                               _i64(cols), mdt, _DT_NAME[compute], _dev(out, "out"), _dt(out), _stream(stream)))
    return out


def cta_op_create(A, D, lam, stream=None):
    """Handle for factors A_k (m_k x n_k) and D_k (p_k x n_k, or None) given as host arrays."""
    lib = load_library()
    order = len(A)
    A64 = [np.ascontiguousarray(a, dtype=np.float64) for a in A]
    n = [a.shape[1] for a in A64]
    m = [a.shape[0] for a in A64]
    a_ptrs = (ctypes.c_void_p * order)(*[a.ctypes.data for a in A64])
    keep = [A64]
    if D is not None:
        D64 = [np.ascontiguousarray(d, dtype=np.float64) if d is not None
               else np.zeros((0, n[k])) for k, d in enumerate(D)]
        keep.append(D64)
        d_ptrs = (ctypes.c_void_p * order)(*[d.ctypes.data if d.size else None for d in D64])
        p = _i64([d.shape[0] for d in D64])
    else:
        d_ptrs = None
        p = None
    h = ctypes.c_void_p()
    _check(lib.cta_op_create(ctypes.byref(h), order, _i64(n), _i64(m), a_ptrs, d_ptrs, p,
                             float(lam), _stream(stream) if stream is not None else None))
    return h


def cta_op_destroy(h):
    if h:
        load_library().cta_op_destroy(h)


def cta_op_device_bytes(h):
    return load_library().cta_op_device_bytes(h)


def cta_forward(h, X, Y, chain="f64", stream=None):
    _check(load_library().cta_forward(h, _dev(X, "X"), _dt(X), _dev(Y, "Y"), _dt(Y),
                                      _PREC[chain], _stream(stream)))
    return Y


def cta_rhs(h, Y, B, chain="f64", stream=None):
    _check(load_library().cta_rhs(h, _dev(Y, "Y"), _dt(Y), _dev(B, "B"), _dt(B), _PREC[chain],
                                  _stream(stream)))
    return B


def cta_apply_normal_op(h, P, Q, chain="f32", dot=None, stream=None):
    """Q = N(P); when ``dot`` (a device float64 tensor of one element) is given, <P, Q> goes there."""
    dptr = _dev(dot, "dot") if dot is not None else None
    _check(load_library().cta_apply_normal_op(h, _dev(P, "P"), _dev(Q, "Q"), _dt(P), _PREC[chain],
                                              dptr, _stream(stream)))
    return Q


def cta_op_set_preconditioner(h, c):
    """Tensor-inverse preconditioner (G_k + c R_k)^-1 per mode; c < 0 removes it."""
    _check(load_library().cta_op_set_preconditioner(h, float(c)))


def cta_apply_precond(h, R, Z, chain="f32", dot=None, stream=None):
    dp = _dev(dot, "dot") if dot is not None else None
    _check(load_library().cta_apply_precond(h, _dev(R, "R"), _dev(Z, "Z"), _dt(R), _PREC[chain], dp,
                                            _stream(stream)))
    return Z


def cta_tune_preconditioner(h, B, X, candidates, stream=None, **opts):
    """Time one solve per strength c in ``candidates`` and keep the fastest; returns its c."""
    o = _opts(**opts)
    cs = (ctypes.c_double * len(candidates))(*[float(c) for c in candidates])
    best = ctypes.c_double(-1.0)
    _check(load_library().cta_tune_preconditioner(h, _dev(B, "B"), _dev(X, "X"), _dt(B), ctypes.byref(o),
                                                  cs, len(candidates), ctypes.byref(best),
                                                  _stream(stream)))
    return best.value


def cta_apply_jacobi(h, R, Z, omega=1.0, dot=None, stream=None):
    """Z = omega R / diag(N) elementwise; <R, Z> to ``dot`` when given."""
    dp = _dev(dot, "dot") if dot is not None else None
    _check(load_library().cta_apply_jacobi(h, _dev(R, "R"), _dev(Z, "Z"), _dt(R), float(omega), dp,
                                           _stream(stream)))
    return Z


def cta_jacobi_solve(h, B, X, omega, stream=None, **opts):
    """Stationary damped Jacobi for N(X) = B (precision 'f64' or 'f32')."""
    o = _opts(**opts)
    info = _CgInfo()
    st = load_library().cta_jacobi_solve(h, _dev(B, "B"), _dev(X, "X"), _dt(B), ctypes.byref(o), float(omega),
                                         ctypes.byref(info), _stream(stream))
    _check(st, allow_not_converged=True)
    return _info_dict(info)


def cta_op_set_multigrid(h, max_levels=8, coarse_max=2048, nu=1, omega_scale=1.5):
    _check(load_library().cta_op_set_multigrid(h, int(max_levels), int(coarse_max), int(nu),
                                               float(omega_scale)))


def cta_op_multigrid_info(h, order):
    """{"levels": L, "extents": [[n_k] per scale], "omega": [per scale]}."""
    lib = load_library()
    lv = ctypes.c_int(0)
    _check(lib.cta_op_multigrid_info(h, ctypes.byref(lv), None, None, 0))
    L = lv.value
    ext = (ctypes.c_int64 * max(1, L * order))()
    om = (ctypes.c_double * max(1, L))()
    _check(lib.cta_op_multigrid_info(h, ctypes.byref(lv), ext, om, L))
    return {"levels": L, "extents": [tuple(ext[l * order:(l + 1) * order]) for l in range(L)],
            "omega": [om[l] for l in range(L)]}


def cta_apply_multigrid(h, R, Z, chain="f32", dot=None, stream=None):
    dp = _dev(dot, "dot") if dot is not None else None
    _check(load_library().cta_apply_multigrid(h, _dev(R, "R"), _dev(Z, "Z"), _dt(R), _PREC[chain], dp,
                                              _stream(stream)))
    return Z


def cta_tune_op(h, chain="bf16", reps=5, stream=None):
    """Pick the fastest bit-identical tile shapes of the operator's passes; returns them."""
    lib = load_library()
    _check(lib.cta_tune_op(h, _PREC[chain], reps, _stream(stream)))
    v = (ctypes.c_int * 3)()
    _check(lib.cta_op_get_tuning(h, _PREC[chain], v))
    return {"tail": v[0], "middle": v[1], "last": v[2]}


def cta_op_set_banded(h, enable):
    _check(load_library().cta_op_set_banded(h, int(enable)))


def cta_op_band_width(h):
    return load_library().cta_op_band_width(h)


def cta_op_set_tuning(h, chain, tail, middle, last):
    v = (ctypes.c_int * 3)(tail, middle, last)
    _check(load_library().cta_op_set_tuning(h, _PREC[chain], v))


def cta_cg_opts_default():
    o = _CgOpts()
    load_library().cta_cg_opts_default(ctypes.byref(o))
    return {f: getattr(o, f) for f, _ in _CgOpts._fields_}


def _opts(**kw):
    o = _CgOpts()
    load_library().cta_cg_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = _PREC[v]
        setattr(o, k, v)
    return o


def _info_dict(info):
    return {f: getattr(info, f) for f, _ in _CgInfo._fields_}


def cta_cg_solve(h, B, X, stream=None, **opts):
    """Solve N(X) = B; options as in cta_cg_opts (precision may be 'f64', 'f32', 'bf16', 'bf16_refine', 'bf16_reliable')."""
    o = _opts(**opts)
    info = _CgInfo()
    st = load_library().cta_cg_solve(h, _dev(B, "B"), _dev(X, "X"), _dt(B), ctypes.byref(o),
                                     ctypes.byref(info), _stream(stream))
    _check(st, allow_not_converged=True)
    return _info_dict(info)


def cta_solve_batched(handles, Bs, Xs, stream=None, **opts):
    lib = load_library()
    n = len(handles)
    o = _opts(**opts)
    infos = (_CgInfo * n)()
    hs = (ctypes.c_void_p * n)(*[h.value for h in handles])
    bp = (ctypes.c_void_p * n)(*[_dev(b, "B").value for b in Bs])
    xp = (ctypes.c_void_p * n)(*[_dev(x, "X").value for x in Xs])
    st = lib.cta_solve_batched(n, hs, bp, xp, _dt(Bs[0]), ctypes.byref(o), infos, _stream(stream))
    _check(st, allow_not_converged=True)
    return [_info_dict(i) for i in infos]


def cta_tune_batched(handles, reps=5, cache_path=None, stream=None):
    n = len(handles)
    hs = (ctypes.c_void_p * n)(*[h.value for h in handles])
    _check(load_library().cta_tune_batched(n, hs, reps, cache_path.encode() if cache_path else None,
                                           _stream(stream)))


def cta_tune_load(path):
    _check(load_library().cta_tune_load(path.encode()))


def cta_tune_dump():
    lib = load_library()
    need = ctypes.c_size_t(0)
    _check(lib.cta_tune_dump(None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(need.value + 1)
    _check(lib.cta_tune_dump(buf, need.value + 1, ctypes.byref(need)))
    return buf.value.decode()


def cta_ws_create(n, channels=32, width=5, blocks=5, seed=0, stream=None):
    h = ctypes.c_void_p()
    _check(load_library().cta_ws_create(ctypes.byref(h), len(n), _i64(n), channels, width, blocks,
                                        seed, _stream(stream)))
    return h


def cta_ws_destroy(h):
    if h:
        load_library().cta_ws_destroy(h)


def cta_ws_num_params(h):
    return load_library().cta_ws_num_params(h)


def cta_ws_forward(h, B, X0, training=False, stream=None):
    _check(load_library().cta_ws_forward(h, _dev(B, "B"), _dev(X0, "X0"), int(training),
                                         _stream(stream)))
    return X0


def cta_ws_backward(h, dX0, stream=None):
    _check(load_library().cta_ws_backward(h, _dev(dX0, "dX0"), _stream(stream)))


def cta_ws_mse(h, X0, T, dX0, loss=None, stream=None):
    lp = _dev(loss, "loss") if loss is not None else None
    _check(load_library().cta_ws_mse(h, _dev(X0, "X0"), _dev(T, "T"), _dev(dX0, "dX0"), lp,
                                     _stream(stream)))


def cta_ws_zero_grad(h, stream=None):
    _check(load_library().cta_ws_zero_grad(h, _stream(stream)))


def cta_ws_adam_step(h, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(load_library().cta_ws_adam_step(h, lr, beta1, beta2, eps, _stream(stream)))


def cta_ws_params(h, host=None, set=0, stream=None):
    """set=0: return FP32 parameters; set=2: return the gradient; set=1: load ``host``."""
    n = cta_ws_num_params(h)
    if set == 1:
        buf = np.ascontiguousarray(host, dtype=np.float32)
        if buf.size != n:
            raise CtaError(-2, f"expected {n} parameters")
    else:
        buf = np.empty(n, dtype=np.float32)
    _check(load_library().cta_ws_params(h, ctypes.c_void_p(buf.ctypes.data), 4 * n, set,
                                        _stream(stream)))
    return buf


def cta_prof_enable(on=True):
    _check(load_library().cta_prof_enable(int(bool(on))))


def cta_prof_reset():
    _check(load_library().cta_prof_reset())


def cta_prof_read():
    """Per-kernel totals recorded by the tracer: {name: {count, total_ms, min_ms, max_ms}}."""
    import json
    lib = load_library()
    need = ctypes.c_size_t(0)
    _check(lib.cta_prof_read(None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(need.value + 1)
    _check(lib.cta_prof_read(buf, need.value + 1, ctypes.byref(need)))
    return json.loads(buf.value.decode())


class Operator:
    """Owning wrapper of a cta_op handle (factors A_k, D_k, weight lam)."""

    def __init__(self, A, D, lam, stream=None):
        self.n = tuple(int(a.shape[1]) for a in A)
        self.m = tuple(int(a.shape[0]) for a in A)
        self.lam = float(lam)
        self.handle = cta_op_create(A, D, lam, stream)

    def close(self):
        if self.handle:
            cta_op_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, X, Y=None, chain="f64", stream=None):
        torch = _torch()
        if Y is None:
            Y = torch.empty(self.m, dtype=X.dtype, device=X.device)
        return cta_forward(self.handle, X, Y, chain, stream)

    def rhs(self, Y, B=None, chain="f64", stream=None):
        torch = _torch()
        if B is None:
            B = torch.empty(self.n, dtype=Y.dtype, device=Y.device)
        return cta_rhs(self.handle, Y, B, chain, stream)

    def apply(self, P, Q=None, chain="f32", dot=None, stream=None):
        torch = _torch()
        if Q is None:
            Q = torch.empty_like(P)
        return cta_apply_normal_op(self.handle, P, Q, chain, dot, stream)

    def set_banded(self, enable):
        cta_op_set_banded(self.handle, enable)

    @property
    def band_width(self):
        return cta_op_band_width(self.handle)

    def tune(self, chain="bf16", reps=5, stream=None):
        return cta_tune_op(self.handle, chain, reps, stream)

    def set_preconditioner(self, c):
        cta_op_set_preconditioner(self.handle, c)

    def tune_preconditioner(self, B, candidates, X=None, stream=None, **opts):
        torch = _torch()
        if X is None:
            X = torch.empty_like(B)
        return cta_tune_preconditioner(self.handle, B, X, candidates, stream, **opts)

    def precond(self, R, Z=None, chain="f32", dot=None, stream=None):
        torch = _torch()
        if Z is None:
            Z = torch.empty_like(R)
        return cta_apply_precond(self.handle, R, Z, chain, dot, stream)

    def solve(self, B, X=None, stream=None, **opts):
        torch = _torch()
        if X is None:
            X = torch.zeros_like(B)
        info = cta_cg_solve(self.handle, B, X, stream, **opts)
        return X, info

    def jacobi(self, R, Z=None, omega=1.0, dot=None, stream=None):
        torch = _torch()
        if Z is None:
            Z = torch.empty_like(R)
        return cta_apply_jacobi(self.handle, R, Z, omega, dot, stream)

    def jacobi_solve(self, B, omega, X=None, stream=None, **opts):
        torch = _torch()
        if X is None:
            X = torch.zeros_like(B)
        info = cta_jacobi_solve(self.handle, B, X, omega, stream, **opts)
        return X, info

    def set_multigrid(self, max_levels=8, coarse_max=2048, nu=1, omega_scale=1.5):
        cta_op_set_multigrid(self.handle, max_levels, coarse_max, nu, omega_scale)

    def multigrid_info(self):
        return cta_op_multigrid_info(self.handle, len(self.n))

    def multigrid(self, R, Z=None, chain="f32", dot=None, stream=None):
        torch = _torch()
        if Z is None:
            Z = torch.empty_like(R)
        return cta_apply_multigrid(self.handle, R, Z, chain, dot, stream)


# ---------------------------------------------------------------- scattered operator
def cta_sop_create(coords, n, D, lam):
    """Handle of the scattered-measurement operator: ``coords`` (order, count)
    host float32 sites in [0, 1], extents ``n``, host factors D_k (or None)."""
    lib = load_library()
    c = np.ascontiguousarray(coords, dtype=np.float32)
    order = len(n)
    if c.ndim != 2 or c.shape[0] != order:
        raise CtaError(-1, "coords must have shape (order, count)")
    keep = [c]
    if D is not None:
        D64 = [np.ascontiguousarray(d, dtype=np.float64) if d is not None
               else np.zeros((0, int(n[k]))) for k, d in enumerate(D)]
        keep.append(D64)
        d_ptrs = (ctypes.c_void_p * order)(*[d.ctypes.data if d.size else None for d in D64])
        p = _i64([d.shape[0] for d in D64])
    else:
        d_ptrs = None
        p = None
    h = ctypes.c_void_p()
    _check(lib.cta_sop_create(ctypes.byref(h), order, _i64(n), int(c.shape[1]),
                              c.ctypes.data if c.size else None, d_ptrs, p, float(lam)))
    return h


def cta_sop_destroy(h):
    if h:
        load_library().cta_sop_destroy(h)


def cta_sop_layout(h):
    out = (ctypes.c_int64 * 8)()
    _check(load_library().cta_sop_layout(h, out))
    v = list(out)
    return {"brick_cells": v[:4], "tile": v[4], "chunks": v[5], "bricks": v[6], "device_bytes": v[7]}


def cta_sop_forward(h, X, y, stream=None):
    _check(load_library().cta_sop_forward(h, _dev(X, "X"), _dev(y, "y") if y.numel() else None,
                                          _dt(X), _stream(stream)))
    return y


def cta_sop_adjoint(h, y, B, stream=None):
    _check(load_library().cta_sop_adjoint(h, _dev(y, "y") if y.numel() else None, _dev(B, "B"),
                                          _dt(B), _stream(stream)))
    return B


def cta_sop_apply_normal(h, P, Q, dot=None, stream=None):
    dptr = _dev(dot, "dot") if dot is not None else None
    _check(load_library().cta_sop_apply_normal(h, _dev(P, "P"), _dev(Q, "Q"), _dt(P), dptr,
                                               _stream(stream)))
    return Q


def cta_sop_cg_solve(h, B, X, rtol=1e-6, max_iter=10000, check_every=16, stream=None, **opts):
    """CG on the scattered operator; options as in cta_cg_opts (x0_given, fallback_zero)."""
    o = _opts(rtol=float(rtol), max_iter=int(max_iter), check_every=int(check_every), **opts)
    info = _CgInfo()
    st = load_library().cta_sop_cg_solve(h, _dev(B, "B"), _dev(X, "X"), _dt(B), ctypes.byref(o),
                                         ctypes.byref(info), _stream(stream))
    _check(st, allow_not_converged=True)
    return _info_dict(info)


class ScatteredOperator:
    """Owning wrapper of a cta_sop handle (sites, extents, D_k, lam)."""

    def __init__(self, coords, n, D, lam):
        self.n = tuple(int(v) for v in n)
        self.count = int(np.asarray(coords).shape[1])
        self.lam = float(lam)
        self.handle = cta_sop_create(coords, self.n, D, lam)

    def close(self):
        if self.handle:
            cta_sop_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def layout(self):
        return cta_sop_layout(self.handle)

    def forward(self, X, y=None, stream=None):
        torch = _torch()
        if tuple(X.shape) != self.n:
            raise CtaError(-2, f"X has shape {tuple(X.shape)}, expected {self.n}")
        if y is None:
            y = torch.empty(self.count, dtype=X.dtype, device=X.device)
        return cta_sop_forward(self.handle, X, y, stream)

    def rhs(self, y, B=None, stream=None):
        torch = _torch()
        if y.numel() != self.count:
            raise CtaError(-2, f"y has {y.numel()} entries, expected {self.count}")
        if B is None:
            B = torch.empty(self.n, dtype=y.dtype, device=y.device)
        return cta_sop_adjoint(self.handle, y, B, stream)

    def apply(self, P, Q=None, dot=None, stream=None):
        torch = _torch()
        if tuple(P.shape) != self.n:
            raise CtaError(-2, f"P has shape {tuple(P.shape)}, expected {self.n}")
        if Q is None:
            Q = torch.empty_like(P)
        return cta_sop_apply_normal(self.handle, P, Q, dot, stream)

    def solve(self, B, X=None, rtol=1e-6, max_iter=10000, check_every=16, stream=None, **opts):
        torch = _torch()
        if X is None:
            X = torch.empty_like(B)
        info = cta_sop_cg_solve(self.handle, B, X, rtol, max_iter, check_every, stream, **opts)
        return X, info
