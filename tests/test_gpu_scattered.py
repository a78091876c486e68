"""GPU parity of the scattered-measurement operator (Sec. 6, Khatri-Rao rows of Sec. 2.2).

Forward model, adjoint, normal operator with its FP64 <P, Q> and the CG solve
through the C ABI, against the FP64 oracle on the same seeded sites.
Tolerances (relative Frobenius): FP64 1e-12 (sums of at most a few thousand
terms); FP32 2e-5 (24-bit storage of X and the basis values, accumulation over
the 4^N window and the sites of a coefficient).  At the application size
(128x128x128x16, 9M sites) the oracle checks sampled sites and sampled
coefficients one by one, and the identity <X, N X> = ||A X||^2 + lam <X, R X>
holds for the whole tensor.
"""
import numpy as np
import pytest

import oracle
import workload
from gpu_util import dev, host, rel_fro, torch_cuda
from oracle import scattered as sc

import paper_1001_5460_amd as cta

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-5}

# (n, sites, clustered fraction, lam)
CASES = [
    ((9, 8, 7), 2000, 0.0, 1e-2),
    ((12, 10, 9, 8), 5000, 0.5, 1e-3),
    ((20, 17), 800, 0.0, 1e-2),
    ((5, 4, 6, 4), 300, 0.0, 1e-1),      # n = 4: a single knot span
    ((40, 36, 24, 12), 60000, 0.3, 1e-3),  # many bricks per mode, ragged last bricks
    ((20, 20, 20), 60000, 0.9, 1e-3),      # dense clusters: bricks cut into several chunks
]


def _problem(n, S, clustered, lam, seed=21):
    p = workload.scattered_problem(n, S, lam, 0.01, seed=seed + S, rtol=1e-8, clustered=clustered)
    p.coords = workload.with_endpoints(p.coords)
    return p


def _dt(chain):
    torch = torch_cuda()
    return torch.float64 if chain == "f64" else torch.float32


@pytest.mark.parametrize("chain", ["f64", "f32"])
@pytest.mark.parametrize("n,S,clustered,lam", CASES)
def test_forward_adjoint_normal_vs_oracle(n, S, clustered, lam, chain):
    torch = torch_cuda()
    p = _problem(n, S, clustered, lam)
    ref = sc.ScatteredOperator(p.coords, n, p.D, p.lam)
    op = cta.ScatteredOperator(p.coords, n, p.D, p.lam)
    rng = np.random.default_rng(7)
    X = rng.standard_normal(n)
    y = rng.standard_normal(S)
    dt = _dt(chain)
    Xd, yd = dev(X, dt), dev(y, dt)
    # the oracle sees what the device sees (FP32 inputs rounded)
    Xh, yh = host(Xd), host(yd)
    f = host(op.forward(Xd))
    assert rel_fro(f, ref.forward(Xh)) <= TOL[chain]
    B = host(op.rhs(yd))
    assert rel_fro(B, ref.rhs(yh)) <= TOL[chain]
    dot = torch.zeros(1, dtype=torch.float64, device="cuda")
    Q = host(op.apply(Xd, dot=dot))
    want = ref(Xh)
    assert rel_fro(Q, want) <= TOL[chain]
    ref_dot = oracle.inner(Xh, want)
    assert abs(dot.item() - ref_dot) <= 4 * TOL[chain] * abs(ref_dot)


def test_layout_chunks_dense_clusters():
    p = _problem((20, 20, 20), 60000, 0.9, 1e-3)
    op = cta.ScatteredOperator(p.coords, p.n, p.D, p.lam)
    lay = op.layout
    assert lay["chunks"] > 0 and lay["tile"] <= 8192
    cells = [v for v in lay["brick_cells"] if v]
    assert len(cells) == 3 and all(1 <= c <= 17 for c in cells)


def test_empty_site_set_is_the_regulariser():
    torch = torch_cuda()
    n = (7, 6, 5)
    D = [workload.second_difference(k) for k in n]
    coords = np.zeros((3, 0), dtype=np.float32)
    op = cta.ScatteredOperator(coords, n, D, 0.5)
    ref = sc.ScatteredOperator(coords, n, D, 0.5)
    X = np.random.default_rng(3).standard_normal(n)
    Q = host(op.apply(dev(X, torch.float64)))
    assert rel_fro(Q, ref(X)) <= 1e-13
    y = op.forward(dev(X, torch.float64))
    assert y.numel() == 0
    B = host(op.rhs(torch.zeros(0, dtype=torch.float64, device="cuda")))
    assert np.all(B == 0)


def test_no_regulariser_and_bad_sites():
    torch = torch_cuda()
    n = (8, 9, 7)
    p = _problem(n, 3000, 0.0, 0.0)
    op = cta.ScatteredOperator(p.coords, n, None, 0.0)
    ref = sc.ScatteredOperator(p.coords, n, None, 0.0)
    X = np.random.default_rng(4).standard_normal(n)
    assert rel_fro(host(op.apply(dev(X, torch.float64))), ref(X)) <= 1e-12
    bad = p.coords.copy()
    bad[1, 5] = 1.5
    with pytest.raises(cta.CtaError):
        cta.ScatteredOperator(bad, n, None, 0.0)
    with pytest.raises(cta.CtaError):
        cta.ScatteredOperator(p.coords, (8, 9, 3), None, 0.0)


@pytest.mark.parametrize("chain,rtol", [("f64", 1e-10), ("f32", 1e-5)])
def test_cg_solve_judged_by_oracle(chain, rtol):
    """The solve is judged by the oracle's FP64 residual (a restart from the
    recomputed residual makes the true residual meet rtol), and its iteration
    count is held within 10% of the oracle's CG under the same storage
    precision: FP64 vectors for the FP64 solve, FP32 vectors with FP64 dots for
    the FP32 solve (the oracle's storage model).  At kappa ~ 1.4e4 FP32
    rounding alone costs this problem about 25% more iterations than FP64
    (218 against ~275), which the storage model reproduces."""
    torch = torch_cuda()
    n = (16, 14, 12, 10)
    p = workload.scattered_problem(n, 20000, 1e-2, 0.01, seed=33, rtol=rtol, clustered=0.3)
    ref = sc.ScatteredOperator(p.coords, n, p.D, p.lam)
    y = ref.forward(p.X_true) + p.noise
    B = ref.rhs(y)
    op = cta.ScatteredOperator(p.coords, n, p.D, p.lam)
    X, info = op.solve(dev(B, _dt(chain)), rtol=rtol, max_iter=5000)
    assert info["status"] == 0, info
    Xh = host(X)
    res = np.linalg.norm((B - ref(Xh)).ravel()) / np.linalg.norm(B.ravel())
    assert res <= 1.01 * rtol, res
    ocg = oracle.cg(ref, B, rtol=rtol, max_iter=5000, store=None if chain == "f64" else np.float32)
    print(chain, "gpu iterations", info["iters"], "oracle", ocg.iters)
    assert abs(info["iters"] - ocg.iters) <= max(3, ocg.iters // 10), (info["iters"], ocg.iters)


def test_cg_solve_from_a_given_start():
    """x0_given: a start near the solution finishes in fewer iterations;
    fallback_zero replaces a start worse than zero."""
    torch = torch_cuda()
    n = (12, 10, 9)
    p = workload.scattered_problem(n, 6000, 1e-2, 0.01, seed=34, rtol=1e-10)
    ref = sc.ScatteredOperator(p.coords, n, p.D, p.lam)
    B = ref.rhs(ref.forward(p.X_true) + p.noise)
    op = cta.ScatteredOperator(p.coords, n, p.D, p.lam)
    Bd = dev(B, torch.float64)
    X0, info0 = op.solve(Bd, rtol=1e-10, max_iter=5000)
    near = X0 + 1e-6 * dev(np.random.default_rng(5).standard_normal(n), torch.float64)
    X1, info1 = op.solve(Bd, near.clone(), rtol=1e-10, max_iter=5000, x0_given=1)
    assert info1["status"] == 0 and info1["iters"] < info0["iters"]
    assert oracle.relative_residual(host(X1), B, ref) <= 1.01e-10
    bad = 1e3 * dev(np.random.default_rng(6).standard_normal(n), torch.float64)
    X2, info2 = op.solve(Bd, bad.clone(), rtol=1e-10, max_iter=5000, x0_given=1, fallback_zero=1)
    # the same solve from zero.  The LDS additions inside a tile run in no fixed
    # order, so repeated zero-start solves differ in rounding: 190..193 iterations
    # over 12 solves of this problem.  Keeping the start of 1e3 instead takes 247.
    assert info2["status"] == 0 and abs(info2["iters"] - info0["iters"]) <= max(3, info0["iters"] // 20)
    assert oracle.relative_residual(host(X2), B, ref) <= 1.01e-10


def test_application_size_sampled():
    """128x128x128x16 coefficients, 9M uniform sites (the bench configuration)."""
    torch = torch_cuda()
    p = workload.scattered_config(with_data=False)
    n = p.n
    op = cta.ScatteredOperator(p.coords, n, p.D, p.lam)
    rng = np.random.default_rng(17)
    X = rng.standard_normal(n)
    Xd = dev(X, torch.float64)
    # sampled sites of the forward model
    f = host(op.forward(Xd))
    idx = rng.choice(p.count, 4000, replace=False)
    want = sc.forward(X, p.coords[:, idx])
    assert rel_fro(f[idx], want) <= 1e-12
    # whole-tensor identity <X, N X> = ||A X||^2 + lam <X, R X>
    dot = torch.zeros(1, dtype=torch.float64, device="cuda")
    Q = host(op.apply(Xd, dot=dot))
    R = [oracle.reg_factor(d) for d in p.D]
    regX = oracle.regulariser_apply(X, R, p.lam)
    ident = float(f @ f) + oracle.inner(X, regX)
    assert abs(dot.item() - ident) <= 1e-10 * abs(ident)
    # sampled coefficients: Q[c] = sum over the sites whose window holds c of
    # a_i[c] <a_i, X>, plus the regulariser
    first = [np.clip(np.floor(p.coords[k].astype(np.float64) * (n[k] - 3)).astype(np.int64), 0, n[k] - 4)
             for k in range(4)]
    for _ in range(12):
        c = tuple(int(rng.integers(0, nk)) for nk in n)
        mask = np.ones(p.count, dtype=bool)
        for k in range(4):
            mask &= (first[k] >= c[k] - 3) & (first[k] <= c[k])
        sel = np.nonzero(mask)[0]
        rows = sc.sample_rows(p.coords[:, sel], n)
        fs = sc.forward(X, p.coords[:, sel], rows)
        coef = np.ones(sel.size)
        for k, (fk, wk) in enumerate(rows):
            off = c[k] - fk
            ok = (off >= 0) & (off < 4)
            coef *= np.where(ok, wk[np.arange(sel.size), np.clip(off, 0, 3)], 0.0)
        want_c = float(coef @ fs) + regX[c]
        assert abs(Q[c] - want_c) <= 1e-12 * max(1.0, abs(want_c)), (c, Q[c], want_c)


def test_cg_iteration_limit_reports_not_converged():
    torch = torch_cuda()
    n = (12, 10, 9, 8)
    p = workload.scattered_problem(n, 4000, 1e-3, 0.01, seed=41, rtol=1e-10)
    ref = sc.ScatteredOperator(p.coords, n, p.D, p.lam)
    B = ref.rhs(ref.forward(p.X_true) + p.noise)
    op = cta.ScatteredOperator(p.coords, n, p.D, p.lam)
    X, info = op.solve(dev(B, torch.float64), rtol=1e-12, max_iter=3, check_every=2)
    assert info["status"] == cta.CTA_NOT_CONVERGED and info["iters"] == 3, info
    # three CG steps from zero: the same iterate as the oracle's three steps
    ocg = oracle.cg(ref, B, rtol=0.0, max_iter=3, restart=False)
    assert rel_fro(host(X), ocg.x) <= 1e-12


def test_repeated_applies_agree_to_rounding():
    """The order of the LDS additions inside a tile is not fixed: two applies
    may differ by rounding only."""
    torch = torch_cuda()
    p = _problem((24, 20, 16, 12), 40000, 0.5, 1e-3)
    op = cta.ScatteredOperator(p.coords, p.n, p.D, p.lam)
    X = dev(np.random.default_rng(8).standard_normal(p.n), torch.float64)
    Q1 = host(op.apply(X))
    Q2 = host(op.apply(X))
    assert rel_fro(Q1, Q2) <= 1e-14
