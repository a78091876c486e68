"""GPU tensor-inverse preconditioner (the separable part of N inverted mode by
mode, Sec. 3) and preconditioned CG, against the FP64 oracle.

The library forms (G_k + c R_k)^-1 by its own Cholesky factorisation on the
host; the oracle by numpy.linalg.inv.  Tolerances of the apply: F64 1e-11
(condition numbers of G_k + c R_k stay below ~1e3), F32 1e-5 (FP32 chain),
BF16 3e-2 (inverse factors and chain inputs rounded to BF16, ~2^-9 each,
through four modes with the inverses' alternating-sign entries).  Solutions
are judged by the oracle's FP64 relative residual."""
import numpy as np
import pytest

import oracle
import workload
from oracle import precond
from gpu_util import dev, host, rel_fro, torch_cuda

import paper_1001_5460_amd as cta

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-11, "f32": 1e-5, "bf16": 3e-2}


def _setup(n, lam, seed=0):
    m = tuple((3 * v) // 2 for v in n)
    p = workload.make_problem(n, m, lam, 0.01, seed, 1e-8)
    ref = oracle.NormalOperator(p.A, p.D, p.lam)
    B = ref.rhs(ref.forward(p.X_true) + p.noise)
    return p, ref, B


@pytest.mark.parametrize("chain", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n", [(16, 12, 10, 8), (20, 18, 24), (33, 17, 24, 16)])
def test_apply_matches_oracle(n, chain):
    torch = torch_cuda()
    p, ref, _ = _setup(n, 1e-3)
    c = 1.6e-2
    op = cta.Operator(p.A, p.D, p.lam)
    op.set_preconditioner(c)
    dt = torch.float64 if chain == "f64" else torch.float32
    R = dev(np.random.default_rng(5).standard_normal(n), dt)
    dot = torch.zeros(1, dtype=torch.float64, device="cuda")
    Z = op.precond(R, chain=chain, dot=dot)
    torch.cuda.synchronize()
    inv = precond.inverse_factors(ref.G, ref.R, c)
    Zr = precond.apply(host(R), inv)
    err = rel_fro(host(Z), Zr)
    print(f"precond apply n={n} {chain}: rel err {err:.2e}")
    assert err <= TOL[chain]
    dref = float(np.sum(host(R) * host(Z)))
    assert abs(float(dot.item()) - dref) <= 1e-9 * abs(dref)


def test_exact_inverse_one_step():
    """lambda = 0, c = 0: M = N, so preconditioned CG converges at once."""
    torch = torch_cuda()
    p, ref, B = _setup((12, 10, 8), 0.0)
    op = cta.Operator(p.A, p.D, 0.0)
    op.set_preconditioner(0.0)
    X, info = op.solve(dev(B, torch.float64), precision="f64", rtol=1e-10, max_iter=20, precond=1)
    assert info["status"] == 0 and info["iters"] <= 2, info
    assert oracle.relative_residual(host(X), B, ref) <= 1.01e-10


@pytest.mark.parametrize("prec,dtype,rtol", [("f64", "f64", 1e-10), ("f32", "f32", 1e-5),
                                             ("bf16_reliable", "f64", 1e-8),
                                             ("bf16_refine", "f64", 1e-8)])
def test_preconditioned_solve_judged_by_oracle(prec, dtype, rtol):
    torch = torch_cuda()
    n = (24, 20, 16, 12)
    p, ref, B = _setup(n, 1e-3, seed=3)
    op = cta.Operator(p.A, p.D, p.lam)
    op.set_preconditioner(1.6e-2)
    dt = torch.float64 if dtype == "f64" else torch.float32
    Bd = dev(B, dt)
    opts = dict(precision=prec, rtol=rtol, max_iter=3000, inner_rtol=0.1, max_refine=80)
    X, info = op.solve(Bd, **opts, precond=1)
    Xp, infop = op.solve(Bd, **opts)
    print(prec, "preconditioned", info["iters"], "plain", infop["iters"])
    assert info["status"] == 0, info
    Bj = host(Bd)
    assert oracle.relative_residual(host(X), Bj, ref) <= rtol * 1.05
    assert info["iters"] < infop["iters"] / 2


def test_preconditioner_errors_and_removal():
    torch = torch_cuda()
    p, ref, B = _setup((12, 10, 8), 1e-3)
    op = cta.Operator(p.A, p.D, p.lam)
    Bd = dev(B, torch.float32)
    with pytest.raises(cta.CtaError):
        op.solve(Bd, precision="f32", rtol=1e-5, precond=1)
    with pytest.raises(cta.CtaError):
        op.precond(Bd)
    op.set_preconditioner(1e-2)
    X, info = op.solve(Bd, precision="f32", rtol=1e-5, precond=1)
    assert info["status"] == 0
    op.set_preconditioner(-1.0)
    with pytest.raises(cta.CtaError):
        op.solve(Bd, precision="f32", rtol=1e-5, precond=1)
    with pytest.raises(cta.CtaError):
        cta.cta_solve_batched([op.handle], [Bd], [torch.zeros_like(Bd)], precision="f32", rtol=1e-5,
                              precond=1)


def test_tune_preconditioner_picks_a_converging_strength():
    torch = torch_cuda()
    p, ref, B = _setup((24, 20, 16, 12), 1e-3, seed=4)
    op = cta.Operator(p.A, p.D, p.lam)
    Bd = dev(B, torch.float64)
    cands = [1e-3, 1.6e-2, 6.4e-2]
    c = op.tune_preconditioner(Bd, cands, precision="bf16_reliable", rtol=1e-8, inner_rtol=0.1,
                               max_iter=3000, max_refine=80)
    assert c in cands
    X, info = op.solve(Bd, precision="bf16_reliable", rtol=1e-8, inner_rtol=0.1, max_iter=3000,
                       max_refine=80, precond=1)
    assert info["status"] == 0
    assert oracle.relative_residual(host(X), B, ref) <= 1.05e-8


@pytest.mark.parametrize("tuning", [(0, 0, 0), (2, 2, 5)])
def test_preconditioned_solve_with_pipelined_passes(tuning):
    """Tail variant 2 (also the preconditioner's first pass with the residual
    update), middle variant 2 and last variant 5 in the preconditioned
    mixed-precision solve, judged by the oracle."""
    torch = torch_cuda()
    n = (16, 12, 40, 24)
    p, ref, B = _setup(n, 1e-3, seed=4)
    op = cta.Operator(p.A, p.D, p.lam)
    op.set_preconditioner(1.6e-2)
    cta.cta_op_set_tuning(op.handle, "bf16", *tuning)
    X, info = op.solve(dev(B, torch.float64), precision="bf16_reliable", rtol=1e-8, inner_rtol=0.03,
                       max_iter=3000, max_refine=80, precond=1)
    assert info["status"] == 0, info
    assert oracle.relative_residual(host(X), B, ref) <= 1.05e-8
