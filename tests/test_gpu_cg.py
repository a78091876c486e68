"""GPU tensor CG (Fig. Tensor_CG) against the FP64 oracle.

Every GPU solution is judged by the oracle's FP64 relative residual
||B - N(X)|| / ||B||.  Small problems are also compared with the oracle's own
CG solution (error within kappa * tolerance) and iteration count (within 10%
plus 2 for FP32/FP64 arithmetic).
"""
import numpy as np
import pytest

import oracle
import workload
from gpu_util import dev, host, rel_fro, torch_cuda

import paper_1001_5460_amd as cta

pytestmark = pytest.mark.gpu


def _setup(p):
    ref = oracle.NormalOperator(p.A, p.D, p.lam)
    Y = ref.forward(p.X_true) + p.noise
    B = ref.rhs(Y)
    return ref, Y, B


def test_config0_f64_matches_oracle():
    torch = torch_cuda()
    p = workload.config_problem(0)
    ref, Y, B = _setup(p)
    ores = oracle.cg(ref, B, rtol=p.rtol)
    op = cta.Operator(p.A, p.D, p.lam)
    X, info = op.solve(dev(B, torch.float64), precision="f64", rtol=p.rtol, max_iter=2000)
    assert info["status"] == 0, info
    x = host(X)
    res = oracle.relative_residual(x, B, ref)
    assert res <= p.rtol * 1.01, res
    assert abs(info["rel_res_true"] - res) <= 1e-3 * res + 1e-15
    lo, hi = oracle.lanczos_extremes(ores.alphas, ores.betas)
    assert rel_fro(x, ores.x) <= (hi / lo) * p.rtol * 2
    assert abs(info["iters"] - ores.iters) <= 0.1 * ores.iters + 2


@pytest.mark.parametrize("scale", [4, 2])
def test_config1_shape_f32_small(scale):
    torch = torch_cuda()
    p = workload.config_problem(1, scale=scale)
    ref, Y, B = _setup(p)
    ores = oracle.cg(ref, B, rtol=p.rtol)
    op = cta.Operator(p.A, p.D, p.lam)
    X, info = op.solve(dev(B, torch.float32), precision="f32", rtol=p.rtol, max_iter=3000)
    assert info["status"] == 0, info
    res = oracle.relative_residual(host(X), B, ref)
    assert res <= p.rtol * 1.05, res
    assert abs(info["iters"] - ores.iters) <= 0.1 * ores.iters + 2


def test_config1_full_f32_judged():
    torch = torch_cuda()
    p = workload.config_problem(1)
    op = cta.Operator(p.A, p.D, p.lam)
    ref = oracle.NormalOperator(p.A, p.D, p.lam)
    # inputs formed by the oracle on the host (forward model + noise, then rhs)
    B = ref.rhs(ref.forward(p.X_true) + p.noise)
    X, info = op.solve(dev(B, torch.float32), precision="f32", rtol=p.rtol, max_iter=3000)
    assert info["status"] == 0, info
    res = oracle.relative_residual(host(X), B, ref)
    assert res <= p.rtol * 1.05, res


@pytest.mark.parametrize("prec,eta", [("bf16_refine", 1e-2), ("bf16_reliable", 1e-1),
                                      ("bf16_reliable", 1e-2)])
def test_bf16_mixed_small_reaches_1e8(prec, eta):
    """Both mixed-precision forms reach 1e-8, judged by the oracle's FP64 residual."""
    torch = torch_cuda()
    p = workload.config_problem(2, scale=8)
    ref, Y, B = _setup(p)
    op = cta.Operator(p.A, p.D, p.lam)
    X, info = op.solve(dev(B, torch.float64), precision=prec, rtol=1e-8, max_iter=2000,
                       inner_rtol=eta, max_refine=60)
    print(prec, eta, info)
    assert info["status"] == 0, info
    res = oracle.relative_residual(host(X), B, ref)
    assert res <= 1e-8 * 1.01, res
    assert abs(info["rel_res_true"] - res) <= 1e-3 * res + 1e-12
    assert info["refine_steps"] >= 1


def test_bf16_reliable_from_given_start_and_fallback():
    torch = torch_cuda()
    p = workload.config_problem(2, scale=8)
    ref, Y, B = _setup(p)
    op = cta.Operator(p.A, p.D, p.lam)
    Bd = dev(B, torch.float64)
    X0, _ = op.solve(Bd, precision="f64", rtol=1e-3, max_iter=2000)
    X, info = op.solve(Bd, X0.clone(), precision="bf16_reliable", rtol=1e-8, max_iter=2000,
                       inner_rtol=1e-1, max_refine=60, x0_given=1, fallback_zero=1)
    Xz, infoz = op.solve(Bd, precision="bf16_reliable", rtol=1e-8, max_iter=2000, inner_rtol=1e-1,
                         max_refine=60)
    assert info["status"] == 0 and infoz["status"] == 0
    assert info["iters"] < infoz["iters"]
    Xb, infob = op.solve(Bd, torch.full_like(Bd, 1e3), precision="bf16_reliable", rtol=1e-8,
                         max_iter=2000, inner_rtol=1e-1, max_refine=60, x0_given=1, fallback_zero=1)
    assert infob["iters"] == infoz["iters"] and torch.equal(Xb, Xz)
    for Xs in (X, Xz):
        assert oracle.relative_residual(host(Xs), B, ref) <= 1e-8 * 1.01


def test_f64_and_f32_agree_with_dense_solution_tiny():
    torch = torch_cuda()
    p = workload.make_problem((6, 5, 7), (9, 8, 11), 1e-3, 0.01, 3, 1e-10)
    ref, Y, B = _setup(p)
    xs = oracle.dense_solve(ref, B)
    op = cta.Operator(p.A, p.D, p.lam)
    X, info = op.solve(dev(B, torch.float64), precision="f64", rtol=1e-12, max_iter=500)
    assert rel_fro(host(X), xs) <= 1e-9
    X32, info32 = op.solve(dev(B, torch.float32), precision="f32", rtol=1e-5, max_iter=500)
    assert oracle.relative_residual(host(X32), B, ref) <= 1.05e-5


def test_breakdown_reported():
    torch = torch_cuda()
    p = workload.make_problem((8, 8, 8), (12, 12, 12), -50.0, 0.01, 1, 1e-8)
    ref = oracle.NormalOperator(p.A, p.D, 1e-3)
    B = ref.rhs(ref.forward(p.X_true) + p.noise)
    op = cta.Operator(p.A, p.D, -50.0)
    with pytest.raises(cta.CtaError) as e:
        op.solve(dev(B, torch.float64), precision="f64", rtol=1e-8, max_iter=100)
    assert e.value.status == -6


def test_iteration_limit_not_converged():
    torch = torch_cuda()
    p = workload.config_problem(0, scale=2)
    ref, Y, B = _setup(p)
    op = cta.Operator(p.A, p.D, p.lam)
    X, info = op.solve(dev(B, torch.float64), precision="f64", rtol=1e-12, max_iter=3, check_every=2)
    assert info["status"] == 1 and info["iters"] == 3
    # the returned X is the CG iterate after 3 steps
    ores = oracle.cg(ref, B, rtol=0.0, max_iter=3, restart=False)
    assert rel_fro(host(X), ores.x) <= 1e-10


def test_warm_start_and_fallback():
    torch = torch_cuda()
    p = workload.config_problem(0, scale=2)
    ref, Y, B = _setup(p)
    xs = oracle.cg(ref, B, rtol=1e-12).x
    op = cta.Operator(p.A, p.D, p.lam)
    # a good start converges at once
    X0 = dev(xs, torch.float64)
    X, info = op.solve(dev(B, torch.float64), X=X0, precision="f64", rtol=1e-8, x0_given=1)
    assert info["iters"] <= 1
    # a start worse than zero is replaced by zero when fallback_zero is set
    bad = dev(xs * 1e3, torch.float64)
    X, info = op.solve(dev(B, torch.float64), X=bad, precision="f64", rtol=1e-8, x0_given=1,
                       fallback_zero=1)
    Xz, infoz = op.solve(dev(B, torch.float64), precision="f64", rtol=1e-8)
    assert info["iters"] == infoz["iters"]
    assert rel_fro(host(X), host(Xz)) <= 1e-12


def test_repeat_solve_bit_identical():
    torch = torch_cuda()
    p = workload.config_problem(0, scale=2)
    ref, Y, B = _setup(p)
    op = cta.Operator(p.A, p.D, p.lam)
    Bd = dev(B, torch.float32)
    X1, _ = op.solve(Bd, precision="f32", rtol=1e-6)
    X2, _ = op.solve(Bd, precision="f32", rtol=1e-6)
    assert torch.equal(X1, X2)
