"""GPU parity of the mode-product passes against the FP64 oracle.

Integer inputs are exact in every arithmetic (BF16 cases keep |sum| <= 256,
FP32 cases <= 2^24), so those comparisons are bit for bit.  Random inputs are
compared by relative Frobenius error: FP64 <= 1e-12, FP32 <= 1e-5 (per mode
product), BF16 <= 2e-2 (inputs and intermediates rounded to 8 bits).
"""
import numpy as np
import pytest

import oracle
import workload
from gpu_util import dev, host, rel_fro, torch_cuda

import paper_1001_5460_amd as cta

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2}

# (shape, mode, rows of M): several tiles and ragged tails on every pass kind
SINGLE = [
    ((5, 37, 70), 0, 9),      # strided, trail 2590 (ragged 64-column tiles)
    ((5, 37, 70), 1, 40),     # strided, trail 70
    ((5, 37, 70), 2, 33),     # contiguous, K = 70 (not a multiple of 8)
    ((3, 130, 24), 1, 130),   # strided, 9 j-tiles
    ((64, 24), 1, 24),        # contiguous, K = 24
    ((7, 96, 48), 0, 20),
    ((2, 3, 192, 8), 2, 128), # rectangular 192 -> 128
    ((300, 16), 1, 256),      # widest output
    # short trails: 64-column tiles span several leading indices, last tile ragged
    ((11, 29, 12), 1, 31),    # trail 12, 132 columns
    ((13, 45, 40), 1, 50),    # trail 40, 520 columns
]


def _torch_dtype(name):
    torch = torch_cuda()
    return {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[name]


@pytest.mark.parametrize("compute", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("shape,mode,rows", SINGLE)
def test_single_mode_integer_exact(shape, mode, rows, compute):
    K = shape[mode]
    lim = {"f64": 3, "f32": 4, "bf16": 2}[compute]
    if compute == "bf16" and K * lim * lim > 256:
        lim = 1
    if compute == "bf16" and K > 256:
        pytest.skip("exact bf16 needs K <= 256")
    X = workload.integer_tensor(shape, -lim, lim, seed=1 + mode)
    M = workload.integer_tensor((rows, K), -lim, lim, seed=100 + mode)
    mats = [None] * len(shape)
    mats[mode] = M
    ref = oracle.mode_product(X, M, mode)
    dt = _torch_dtype(compute)
    Xd = dev(X, dt)
    Md = [None] * len(shape)
    Md[mode] = dev(M, dt)
    Y = cta.cta_ttm(Xd, Md, compute=compute)
    out = host(Y)
    assert out.shape == ref.shape
    assert np.array_equal(out, ref), f"max abs diff {np.abs(out - ref).max()}"


@pytest.mark.parametrize("compute", ["f64", "f32", "bf16"])
def test_chain_random_vs_oracle(compute):
    torch = torch_cuda()
    rng = np.random.default_rng(5)
    shape = (19, 33, 26, 21)
    rows = (24, 17, 40, 21)
    X = rng.standard_normal(shape)
    mats = [rng.standard_normal((r, s)) for r, s in zip(rows, shape)]
    ref = oracle.multi_mode_product(X, mats)
    Y = cta.cta_ttm(dev(X, torch.float64), [dev(m, torch.float64) for m in mats],
                    compute=compute)
    err = rel_fro(host(Y), ref)
    # a chain of 4 products: FP32 gets 4x the single-product budget
    tol = {"f64": 1e-12, "f32": 4e-5, "bf16": 4e-2}[compute]
    assert err <= tol, err


@pytest.mark.parametrize("compute", ["f64", "f32"])
def test_transposed_factors_and_dtype_conversion(compute):
    torch = torch_cuda()
    rng = np.random.default_rng(6)
    shape = (12, 40, 9)
    X = rng.standard_normal(shape)
    Ms = [rng.standard_normal((12, 7)), None, rng.standard_normal((9, 30))]
    ref = oracle.multi_mode_product(X, [Ms[0].T, None, Ms[2].T], modes=[0, 2])
    Y = cta.cta_ttm(dev(X, torch.float32), [dev(Ms[0], torch.float64), None, dev(Ms[2], torch.float64)],
                    trans=(0, 2), compute=compute, out_dtype=torch.float64)
    assert Y.dtype == torch.float64 and tuple(Y.shape) == (7, 40, 30)
    # input was rounded to FP32 on the way in
    assert rel_fro(host(Y), ref) <= 2e-6


def test_empty_mask_copies():
    torch = torch_cuda()
    X = np.arange(24, dtype=np.float64).reshape(2, 3, 4)
    Y = cta.cta_ttm(dev(X, torch.float32), [None, None, None], compute="f32")
    assert np.array_equal(host(Y), X)


def test_shape_error_raises():
    torch = torch_cuda()
    X = torch.zeros((4, 5), device="cuda")
    with pytest.raises(cta.CtaError):
        cta.cta_ttm(X, [torch.zeros((3, 6), device="cuda"), None])
