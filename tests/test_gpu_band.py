"""GPU parity of the band-aware normal operator (banded Gram factors).

Cubic B-spline collocation factors give Gram matrices of half-bandwidth 3
(each sample touches 4 basis functions per mode, Sec. 6), and the handle then
applies N in FP64/FP32 as banded streaming passes.  The banded result must
match the FP64 oracle with the dense chain's bounds (FP64 1e-12, FP32 1e-5
relative Frobenius) and the dense GPU chain to rounding.  Dense factors must
keep the dense passes.
"""
import numpy as np
import pytest

import oracle
import workload
from gpu_util import dev, host, rel_fro, torch_cuda

import paper_1001_5460_amd as cta
from workload.bspline import second_difference

pytestmark = pytest.mark.gpu

PROBLEMS = [
    ((8, 8, 8), (12, 12, 12), 1e-2),
    ((13, 9, 21), (20, 14, 31), 1e-3),          # ragged: scalar units (21 % 2 != 0)
    ((16, 12, 10, 8), (24, 18, 15, 12), 1e-3),  # 4-D, vector units
    ((20, 24, 33, 17), (30, 36, 49, 25), 1e-4), # 4-D ragged
    ((40, 50), (60, 75), 1e-2),                 # order 2 (lifted to order 3)
    ((96, 6, 96), (144, 9, 144), 1e-3),         # wide tail, short middle mode
    ((5, 4, 7), (8, 6, 11), 1e-3),              # extents at the band edge
]
TOL = {"f64": 1e-12, "f32": 1e-5}


def _problem(n, m, lam):
    return workload.make_problem(n, m, lam, 0.01, seed=sum(n) + 3, rtol=1e-8)


def test_bspline_gram_half_bandwidth_is_three():
    p = _problem((16, 12, 10), (24, 18, 15), 1e-3)
    op = cta.Operator(p.A, p.D, p.lam)
    assert op.band_width == 3


def test_dense_factors_keep_dense_passes():
    torch = torch_cuda()
    rng = np.random.default_rng(4)
    n = (9, 8, 7)
    A = [rng.standard_normal((k + 3, k)) for k in n]
    D = [second_difference(k) for k in n]
    op = cta.Operator(A, D, 1e-3)
    assert op.band_width > 4
    with pytest.raises(cta.CtaError):
        op.set_banded(True)
    op.set_banded(False)
    P = rng.standard_normal(n)
    ref = oracle.NormalOperator(A, D, 1e-3)(P)
    Q = op.apply(dev(P, torch.float64), chain="f64")
    assert rel_fro(host(Q), ref) <= 1e-12


@pytest.mark.parametrize("chain", ["f64", "f32"])
@pytest.mark.parametrize("n,m,lam", PROBLEMS)
def test_banded_apply_vs_oracle_and_dense(n, m, lam, chain):
    torch = torch_cuda()
    p = _problem(n, m, lam)
    ref = oracle.NormalOperator(p.A, p.D, p.lam)
    rng = np.random.default_rng(11)
    P = rng.standard_normal(n)
    want = ref(P)
    op = cta.Operator(p.A, p.D, p.lam)
    assert op.band_width <= 4
    dt = torch.float64 if chain == "f64" else torch.float32
    Pd = dev(P, dt)
    dot = torch.zeros(1, dtype=torch.float64, device="cuda")
    op.set_banded(True)
    Qb = host(op.apply(Pd, chain=chain, dot=dot))
    dot_b = dot.item()
    op.set_banded(False)
    Qd = host(op.apply(Pd, chain=chain))
    assert rel_fro(Qb, want) <= TOL[chain]
    assert rel_fro(Qb, Qd) <= 2 * TOL[chain]
    ref_dot = oracle.inner(host(Pd), want)
    assert abs(dot_b - ref_dot) <= TOL[chain] * abs(ref_dot)


def test_banded_apply_without_regulariser():
    torch = torch_cuda()
    p = _problem((10, 11, 12), (15, 16, 18), 0.0)
    op = cta.Operator(p.A, None, 0.0)
    P = np.random.default_rng(9).standard_normal(p.n)
    ref = oracle.normal_apply(P, [oracle.gram(a) for a in p.A], [np.zeros((k, k)) for k in p.n], 0.0)
    op.set_banded(True)
    Q = op.apply(dev(P, torch.float64), chain="f64")
    assert rel_fro(host(Q), ref) <= 1e-12


@pytest.mark.parametrize("banded", [True, False])
def test_reliable_solve_with_banded_updates(banded):
    """The mixed-precision solve forms its residual updates with the banded
    passes (FP32 and FP64); the FP64 oracle judges the solution."""
    torch = torch_cuda()
    p = workload.make_problem((24, 20, 16, 12), (36, 30, 24, 18), 1e-4, 0.01, seed=5, rtol=1e-8)
    ref = oracle.NormalOperator(p.A, p.D, p.lam)
    B = ref.rhs(ref.forward(p.X_true) + p.noise)
    op = cta.Operator(p.A, p.D, p.lam)
    op.set_banded(banded)
    X, info = op.solve(dev(B, torch.float64), precision="bf16_reliable", rtol=1e-8, inner_rtol=0.1,
                       max_refine=60)
    assert info["status"] == 0, info
    res = oracle.relative_residual(host(X), B, ref)
    assert res <= 1.01e-8, res


@pytest.mark.parametrize("chain", ["f64", "f32"])
@pytest.mark.parametrize("n,m,lam", PROBLEMS)
def test_banded_forward_and_rhs_vs_oracle_and_dense(n, m, lam, chain):
    """Forward model X x_k A_k and right-hand side Y x_k A_k^T with the banded
    rows of the collocation factors, against the oracle and the dense chain."""
    torch = torch_cuda()
    p = _problem(n, m, lam)
    ref = oracle.NormalOperator(p.A, p.D, p.lam)
    rng = np.random.default_rng(12)
    X = rng.standard_normal(n)
    Y = rng.standard_normal(m)
    op = cta.Operator(p.A, p.D, p.lam)
    dt = torch.float64 if chain == "f64" else torch.float32
    out = {}
    for banded in (True, False):
        op.set_banded(banded)
        out[banded] = (host(op.forward(dev(X, dt), chain=chain)), host(op.rhs(dev(Y, dt), chain=chain)))
    want_f, want_b = ref.forward(X), ref.rhs(Y)
    # four mode products per chain: four times the single-product FP32 budget
    tol = {"f64": 1e-12, "f32": 4e-5}[chain]
    assert rel_fro(out[True][0], want_f) <= tol
    assert rel_fro(out[True][1], want_b) <= tol
    assert rel_fro(out[True][0], out[False][0]) <= 2 * tol
    assert rel_fro(out[True][1], out[False][1]) <= 2 * tol
