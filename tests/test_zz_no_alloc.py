"""cta_ttm_noalloc (the product without a workspace argument, for callers that
cannot allocate) against cta_ttm with a caller workspace: the same kernels and
plan, so the outputs must be identical, on two calls in a row (the second with
a smaller input, which finds the first call's data in the fixed scratch), and
a product needing more than the fixed scratch is refused."""
import numpy as np
import pytest

from gpu_util import dev, torch_cuda

import paper_1001_5460_amd as cta

pytestmark = pytest.mark.gpu


def _case(shape, out_rows, seed, dtype):
    torch = torch_cuda()
    rng = np.random.default_rng(seed)
    X = dev(rng.standard_normal(shape), dtype)
    mats = [None if r is None else dev(rng.standard_normal((r, n)), dtype) for r, n in zip(out_rows, shape)]
    return X, mats


@pytest.mark.parametrize("compute", ["f32", "f64", "bf16"])
def test_noalloc_matches_workspace_form_on_two_calls(compute):
    torch = torch_cuda()
    dt = torch.float64 if compute == "f64" else torch.float32
    cases = [((40, 36, 30, 20), (50, 24, 45, 20), 1),     # every mode, ragged extents
             ((12, 10, 9), (None, 15, 6), 2)]             # smaller, two modes, one shrinking
    for shape, rows, seed in cases:
        X, mats = _case(shape, rows, seed, dt)
        ref = cta.cta_ttm(X, mats, trans=(), compute=compute)
        out = cta.cta_ttm_noalloc(X, mats, trans=(), compute=compute)
        torch.cuda.synchronize()
        assert out.shape == ref.shape
        assert torch.equal(out, ref), (shape, compute)


def test_noalloc_transposed_factor_and_limit():
    torch = torch_cuda()
    rng = np.random.default_rng(3)
    X = dev(rng.standard_normal((20, 18, 16)), torch.float32)
    M = dev(rng.standard_normal((18, 30)), torch.float32)          # applied transposed on mode 2
    ref = cta.cta_ttm(X, [None, M, None], trans=(1,), compute="f32")
    out = cta.cta_ttm_noalloc(X, [None, M, None], trans=(1,), compute="f32")
    assert torch.equal(out, ref)
    # more than the fixed scratch (32 MiB): refused before any launch
    big = torch.zeros((256, 256, 64), dtype=torch.float32, device="cuda")
    G = torch.zeros((256, 256), dtype=torch.float32, device="cuda")
    with pytest.raises(cta.CtaError):
        cta.cta_ttm_noalloc(big, [G, None, None], compute="f32")
