"""Learned warm start end to end on the GPU: a network trained by the
library's own forward/backward/Adam kernels on solves the library generates
proposes CG starting tensors; CG from them must reach the tolerance (judged
by the FP64 oracle) in fewer iterations than CG from zero on held-out seeds.

A reduced shape (24x24x24x8, 2 residual blocks, 600 training solves) keeps
the test within seconds; the 64x64x64x16 network of the warm-start workload
is trained and evaluated by ``python -m paper_1001_5460_amd.warmstart``.
"""
import numpy as np
import pytest

import oracle
import workload
from gpu_util import host, torch_cuda

pytestmark = pytest.mark.gpu

N_SMALL = (24, 24, 24, 8)
M_SMALL = (36, 36, 36, 12)


def test_trained_start_saves_iterations():
    torch_cuda()
    from paper_1001_5460_amd import warmstart as ws

    smp = ws.Sampler(N_SMALL, M_SMALL, 1e-3)
    net = ws.WarmStart(N_SMALL, blocks=2, seed=0)
    val = []
    for seed in range(20000, 20008):  # validation seeds, outside training and test
        B = smp.rhs(seed)
        val.append((B, smp.target(B)[0]))
    before = ws.validation_loss(net, smp, val)
    net, smp, rec = ws.train(N_SMALL, M_SMALL, 1e-3, samples=600, batch=4, lr=2e-3, log_every=25,
                             smp=smp, net=net)
    after = ws.validation_loss(net, smp, val)
    print("loss history", [round(l, 5) for _, l in rec["loss_history"]])
    print(f"validation loss {before:.4e} -> {after:.4e}")
    assert after < 0.5 * before
    rows, kept = ws.evaluate(net, smp, range(10000, 10012), rtol=1e-8, keep=2)
    s = ws.summarize(rows)
    print(s)
    assert s["all_converged"]
    assert s["warm_iters_mean"] < s["zero_iters_mean"]
    assert s["start_res_median"] < 1.0
    A, D = workload.factors(N_SMALL, M_SMALL)
    ref = oracle.NormalOperator(A, D, 1e-3)
    for B, Xz, Xw in kept:
        Bh = host(B)
        for X in (Xz, Xw):
            assert oracle.relative_residual(host(X), Bh, ref) <= 1.05e-8


def test_fallback_to_zero_on_bad_start():
    """A start worse than zero (residual above ||B||) is replaced by zero:
    the solve then takes exactly the zero-start path."""
    torch = torch_cuda()
    from paper_1001_5460_amd import warmstart as ws

    smp = ws.Sampler(N_SMALL, M_SMALL, 1e-3)
    B = smp.rhs(10500).double()
    Xz = torch.zeros_like(B)
    _, iz = smp.op.solve(B, Xz, precision="bf16_refine", rtol=1e-8, max_iter=20000)
    Xw = 1e3 * torch.ones_like(B)
    _, iw = smp.op.solve(B, Xw, precision="bf16_refine", rtol=1e-8, max_iter=20000, x0_given=1,
                         fallback_zero=1)
    assert iz["status"] == 0 and iw["status"] == 0
    assert iw["iters"] == iz["iters"]
    assert torch.equal(Xw, Xz)
