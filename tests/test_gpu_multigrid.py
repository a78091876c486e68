"""GPU tensor Jacobi (Fig. Tensor_Jacobi) and tensor multigrid V-cycle
(Fig. TMG) against the FP64 oracle (oracle.jacobi, oracle.multigrid).

Tolerances (relative Frobenius):
* the diagonal step z = omega r / d: F64 1e-14 (one division per element;
  the diagonal's product and sum are formed in another order), F32 1e-6;
* one V-cycle: F64 1e-12 (every step is a linear map of condition ~1e2 on
  rounding-level differences, including the smoother weight, whose eigenvalue
  bound both sides compute with their own eigen-solvers; measured <= 3e-14),
  F32 1e-6 (FP32 chains, transfers and coarsest inverse; measured <= 5e-8),
  BF16 1e-2 (the smoother's operator applies run the BF16 chain, a few 1e-3
  each, through 2 nu + 1 applies per scale, and the smoother damps them;
  measured <= 2e-3);
* solves are judged by the oracle's FP64 relative residual, and the FP64
  iteration counts are held within 10% of the oracle's.
"""
import numpy as np
import pytest

import oracle
import workload
from gpu_util import dev, host, rel_fro, torch_cuda
from oracle import jacobi, multigrid, precond

import paper_1001_5460_amd as cta

pytestmark = pytest.mark.gpu


def _setup(n, lam, seed=0):
    m = tuple((3 * v) // 2 for v in n)
    p = workload.make_problem(n, m, lam, 0.01, seed, 1e-8)
    ref = oracle.NormalOperator(p.A, p.D, p.lam)
    B = ref.rhs(ref.forward(p.X_true) + p.noise)
    return p, ref, B


SHAPES = [(16, 12, 10, 8), (13, 9, 21), (40, 50), (20, 18, 7, 6), (33, 17, 24, 16)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", SHAPES)
def test_jacobi_apply_vs_oracle(n, dtype):
    torch = torch_cuda()
    p, ref, _ = _setup(n, 1e-3)
    op = cta.Operator(p.A, p.D, p.lam)
    dt = torch.float64 if dtype == "f64" else torch.float32
    R = dev(np.random.default_rng(1).standard_normal(n), dt)
    dot = torch.zeros(1, dtype=torch.float64, device="cuda")
    Z = op.jacobi(R, omega=0.7, dot=dot)
    torch.cuda.synchronize()
    d = jacobi.diagonal(ref.G, ref.R, p.lam)
    Zr = 0.7 * host(R) / d
    tol = 1e-14 if dtype == "f64" else 1e-6
    assert rel_fro(host(Z), Zr) <= tol
    dref = float(np.sum(host(R) * Zr))
    assert abs(dot.item() - dref) <= tol * abs(dref)


def test_jacobi_solve_matches_oracle_iteration():
    """The stationary iteration of Fig. Tensor_Jacobi with damping: the same
    number of sweeps as the oracle (the test before every sweep is the
    figure's), the answer judged by the oracle."""
    torch = torch_cuda()
    n = (10, 8, 9)
    p, ref, B = _setup(n, 0.5)
    omega = 1.0 / jacobi.smoother_bound(ref.G, ref.R, p.lam)
    d = jacobi.diagonal(ref.G, ref.R, p.lam)
    Ur, it_ref, ok = jacobi.jacobi(ref, B, d, omega=omega, rtol=1e-8, max_iter=20000)
    assert ok
    op = cta.Operator(p.A, p.D, p.lam)
    X, info = op.jacobi_solve(dev(B, torch.float64), omega, precision="f64", rtol=1e-8, max_iter=20000,
                              check_every=64)
    print("jacobi sweeps gpu", info["iters"], "oracle", it_ref)
    assert info["status"] == 0
    assert abs(info["iters"] - it_ref) <= 1
    assert oracle.relative_residual(host(X), B, ref) <= 1.01e-8
    assert rel_fro(host(X), Ur) <= 1e-6
    # the undamped (printed) iteration diverges on this operator
    X1, info1 = op.jacobi_solve(dev(B, torch.float64), 1.0, precision="f64", rtol=1e-8, max_iter=30,
                                check_every=8)
    assert info1["status"] == 1 and info1["iters"] == 30 and info1["rel_res_true"] > 1.0


def test_jacobi_solve_zero_rhs_and_given_start():
    torch = torch_cuda()
    n = (8, 8, 8)
    p, ref, B = _setup(n, 0.5)
    op = cta.Operator(p.A, p.D, p.lam)
    omega = 1.0 / jacobi.smoother_bound(ref.G, ref.R, p.lam)
    Z = torch.zeros(n, dtype=torch.float64, device="cuda")
    X, info = op.jacobi_solve(Z, omega, precision="f64", rtol=1e-8)
    assert info["status"] == 0 and info["iters"] == 0 and float(X.abs().max()) == 0.0
    # a start that already meets the tolerance takes no sweep
    Xs = dev(oracle.dense_solve(ref, B), torch.float64)
    X2, info2 = op.jacobi_solve(dev(B, torch.float64), omega, X=Xs.clone(), precision="f64", rtol=1e-8,
                                x0_given=1)
    assert info2["iters"] == 0 and torch.equal(X2, Xs)


@pytest.mark.parametrize("prec,dtype,rtol", [("f64", "f64", 1e-10), ("f32", "f32", 1e-5),
                                             ("bf16_reliable", "f64", 1e-8)])
def test_jacobi_preconditioned_cg_judged_by_oracle(prec, dtype, rtol):
    torch = torch_cuda()
    n = (24, 20, 16, 12)
    p, ref, B = _setup(n, 1e-3, seed=3)
    op = cta.Operator(p.A, p.D, p.lam)
    dt = torch.float64 if dtype == "f64" else torch.float32
    X, info = op.solve(dev(B, dt), precision=prec, rtol=rtol, max_iter=3000, inner_rtol=0.1, max_refine=80,
                       precond=2)
    res = oracle.relative_residual(host(X), B, ref)
    print(prec, "jacobi-pcg iters", info["iters"], "residual", res)
    assert info["status"] == 0
    assert res <= 1.01 * rtol
    if prec == "f64":
        d = jacobi.diagonal(ref.G, ref.R, p.lam)
        _, it_ref, ok = precond.pcg(ref, B, jacobi.precondition(d), rtol=rtol)
        assert ok and abs(info["iters"] - it_ref) <= 0.1 * it_ref + 1


MG_CASES = [((16, 12, 10, 8), 200), ((13, 9, 21), 60), ((40, 50), 100), ((33, 17, 24, 16), 2048)]


def _mg_oracle(p, coarse_max, nu):
    return multigrid.build_scales(p.A, p.D, p.lam, coarse_max=coarse_max, omega_scale=1.5)


@pytest.mark.parametrize("n,coarse_max", MG_CASES)
def test_multigrid_hierarchy_matches_oracle(n, coarse_max):
    p, ref, _ = _setup(n, 1e-3)
    op = cta.Operator(p.A, p.D, p.lam)
    op.set_multigrid(coarse_max=coarse_max, nu=1, omega_scale=1.5)
    info = op.multigrid_info()
    scales, _ = _mg_oracle(p, coarse_max, 1)
    assert info["levels"] == len(scales) >= 2
    assert info["extents"] == [s.op.shape for s in scales]
    for om, s in zip(info["omega"], scales):
        assert abs(om - s.omega) <= 1e-12 * s.omega


@pytest.mark.parametrize("nu", [1, 2])
@pytest.mark.parametrize("chain", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n,coarse_max", MG_CASES)
def test_vcycle_apply_vs_oracle(n, coarse_max, chain, nu):
    torch = torch_cuda()
    p, ref, _ = _setup(n, 1e-3)
    op = cta.Operator(p.A, p.D, p.lam)
    op.set_multigrid(coarse_max=coarse_max, nu=nu, omega_scale=1.5)
    scales, chol = multigrid.build_scales(p.A, p.D, p.lam, coarse_max=coarse_max, omega_scale=1.5)
    dt = torch.float64 if chain == "f64" else torch.float32
    R = dev(np.random.default_rng(2).standard_normal(n), dt)
    dot = torch.zeros(1, dtype=torch.float64, device="cuda")
    Z = op.multigrid(R, chain=chain, dot=dot)
    torch.cuda.synchronize()
    Zr = multigrid.vcycle(scales, chol, 0, np.zeros(n), host(R), nu)
    err = rel_fro(host(Z), Zr)
    tol = {"f64": 1e-12, "f32": 1e-6, "bf16": 1e-2}[chain]
    print(f"vcycle {n} {chain} nu={nu}: rel err {err:.2e}")
    assert err <= tol
    dref = float(np.sum(host(R) * host(Z)))
    assert abs(dot.item() - dref) <= 1e-10 * abs(dref)


def test_vcycle_is_symmetric_on_the_gpu():
    torch = torch_cuda()
    n = (16, 12, 10, 8)
    p, ref, _ = _setup(n, 1e-3)
    op = cta.Operator(p.A, p.D, p.lam)
    op.set_multigrid(coarse_max=200, nu=2)
    rng = np.random.default_rng(4)
    u = dev(rng.standard_normal(n), torch.float64)
    v = dev(rng.standard_normal(n), torch.float64)
    a = float((u * op.multigrid(v, chain="f64")).sum())
    b = float((op.multigrid(u, chain="f64") * v).sum())
    assert abs(a - b) <= 1e-12 * abs(a)


@pytest.mark.parametrize("prec,dtype,rtol", [("f64", "f64", 1e-10), ("f32", "f32", 1e-5),
                                             ("bf16_reliable", "f64", 1e-8)])
def test_multigrid_preconditioned_cg_judged_by_oracle(prec, dtype, rtol):
    torch = torch_cuda()
    n = (24, 20, 16, 12)
    p, ref, B = _setup(n, 1e-3, seed=3)
    op = cta.Operator(p.A, p.D, p.lam)
    op.set_multigrid(coarse_max=600, nu=2)
    dt = torch.float64 if dtype == "f64" else torch.float32
    X, info = op.solve(dev(B, dt), precision=prec, rtol=rtol, max_iter=3000, inner_rtol=0.1, max_refine=80,
                       precond=3)
    res = oracle.relative_residual(host(X), B, ref)
    print(prec, "tmg-pcg iters", info["iters"], "residual", res)
    assert info["status"] == 0
    assert res <= 1.01 * rtol
    if prec == "f64":
        scales, chol = multigrid.build_scales(p.A, p.D, p.lam, coarse_max=600, omega_scale=1.5)
        _, it_ref, ok = precond.pcg(ref, B, multigrid.preconditioner(scales, chol, nu=2), rtol=rtol)
        plain = oracle.cg(ref, B, rtol=rtol)
        print("oracle tmg-pcg", it_ref, "plain cg", plain.iters)
        assert ok and abs(info["iters"] - it_ref) <= 0.1 * it_ref + 1
        assert info["iters"] < plain.iters


def test_multigrid_errors_and_removal():
    torch = torch_cuda()
    p, ref, B = _setup((12, 10, 8), 1e-3)
    op = cta.Operator(p.A, p.D, p.lam)
    with pytest.raises(cta.CtaError):
        op.solve(dev(B, torch.float64), precision="f64", precond=3)      # no hierarchy yet
    with pytest.raises(cta.CtaError):
        op.set_multigrid(coarse_max=100000)                             # nothing to coarsen
    with pytest.raises(cta.CtaError):
        op.set_multigrid(omega_scale=2.5)
    op.set_multigrid(coarse_max=100)
    assert op.multigrid_info()["levels"] >= 2
    op.set_multigrid(max_levels=1)
    assert op.multigrid_info()["levels"] == 0
