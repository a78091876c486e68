"""Parity of the BF16 operator passes at the full 4-D size, 128 x 128 x 96 x 24.

At this size the persistent passes run many tiles per workgroup (the grid is
three workgroups per CU): the last pass (mode 1 with the regulariser and
<P, Q>) walks 9,216 tiles of 32 columns, the middle pass 4,608 tiles of 64
columns and the fused tail pass 8,192 groups of two blocks, so the loops over
tiles and the prefetch of the next tile run under test.

* Integer inputs make the BF16 chain exact: the factors A_k are 0/1 matrices
  (two ones per row and per column), so G_k = A_k^T A_k has small integer
  entries scattered over the whole matrix; P takes
  values in {-1, 0, 1}; R_k is the integer second-difference Gram; lambda is a
  power of two.  Every value the chain stores (P, G_k, the intermediates after
  modes 4, 3 and 2) is then an integer of magnitude <= 256, which BF16 holds
  exactly, the FP32 accumulation and the FP32 regulariser are exact, and so is
  the FP64 dot.  The GPU result must equal the FP64 oracle bit for bit
  (Sec. 2.1 eq. separable_transf; the Kronecker-sum regulariser of Sec. 4.1).
* Random inputs are checked element by element against the oracle with a bound
  derived from the BF16 roundings (unit roundoff u = 2^-8): P, the four G_k and
  the three stored intermediates are rounded once each, so
  |Q_gpu - Q| <= 8u (|G_1| ... |G_4| chain applied to |P|) to first order; the
  FP32 regulariser adds a relative 1e-6.
* The fused CG passes (x += alpha p and p = r + beta p inside the tail pass,
  Fig. Tensor_CG) in their persistent form give iterates bit-identical to the
  one-tile-per-workgroup form over several iterations.
"""
import numpy as np
import pytest

import oracle
import workload
from gpu_util import dev, host, torch_cuda

import paper_1001_5460_amd as cta

pytestmark = pytest.mark.gpu

N = (128, 128, 96, 24)
M = (192, 192, 144, 36)
PIPE = (2, 2, 5)      # persistent tail, middle and last passes
PIPE6 = (2, 2, 6)     # the same with vector band reads and per-XCD tile ranges
PIPE7 = (2, 2, 7)     # the same with 512-thread workgroups in the last pass
PIPE8 = (2, 2, 8)     # the last pass sweeping planes with P in an LDS ring
PLAIN = (0, 0, 0)     # one tile per workgroup
U_BF16 = 2.0 ** -8


def _integer_factors(seed):
    """0/1 factors A_k (n_k x n_k): row i has ones in columns i and pi(i) for a
    random derangement pi, so every column holds two ones and G_k = A_k^T A_k
    has 2 on the diagonal and two off-diagonal ones per row at random
    positions (row sums of |G_k| are 4: after three modes |T| <= 64)."""
    rng = np.random.default_rng(seed)
    A = []
    for n in N:
        while True:
            pi = rng.permutation(n)
            if np.all(pi != np.arange(n)):
                break
        a = np.zeros((n, n))
        a[np.arange(n), np.arange(n)] = 1.0
        a[np.arange(n), pi] = 1.0
        A.append(a)
    return A


def _chain_intermediates_fit_bf16(P, G):
    """Every tensor the BF16 chain stores (modes 4, then 3, then 2) is an
    integer of magnitude <= 256 (exact in BF16)."""
    T = P
    for k in (3, 2, 1):
        T = oracle.mode_product(T, G[k], k)
        if np.abs(T).max() > 256 or not np.array_equal(T, np.round(T)):
            return False
    return True


def test_integer_apply_bit_exact_at_full_size():
    torch = torch_cuda()
    A = _integer_factors(41)
    D = [workload.bspline.second_difference(n) for n in N]
    lam = 2.0 ** -4
    ref = oracle.NormalOperator(A, D, lam)
    assert all(np.abs(g).max() <= 256 for g in ref.G)
    rng = np.random.default_rng(42)
    P = rng.choice(np.array([-1.0, 0.0, 1.0]), size=N, p=[0.25, 0.5, 0.25])
    assert _chain_intermediates_fit_bf16(P, ref.G)
    Qref = ref(P)
    dref = oracle.inner(P, Qref)

    op = cta.Operator(A, D, lam)
    assert op.band_width > 4          # random columns: the dense passes run
    Pd = dev(P, torch.float32)
    dot = torch.zeros(1, dtype=torch.float64, device="cuda")
    for variants in (PIPE, PIPE6, PIPE7, PIPE8, PLAIN):
        cta.cta_op_set_tuning(op.handle, "bf16", *variants)
        Q = op.apply(Pd, chain="bf16", dot=dot)
        torch.cuda.synchronize()
        Qh = host(Q)
        bad = np.argwhere(Qh != Qref)
        assert bad.size == 0, (variants, len(bad), bad[:4].tolist())
        assert dot.item() == dref, (variants, dot.item(), dref)
    op.close()


def test_random_apply_elementwise_bound_at_full_size():
    torch = torch_cuda()
    p = workload.make_problem(N, M, 1e-4, 0.01, 2000, 1e-8, with_data=False)
    ref = oracle.NormalOperator(p.A, p.D, p.lam)
    P = np.random.default_rng(43).standard_normal(N)
    Pd = dev(P, torch.float32)
    P32 = host(Pd)
    Qref = ref(P32)
    chain_abs = oracle.normal_apply(np.abs(P32), [np.abs(g) for g in ref.G],
                                    [np.zeros_like(r) for r in ref.R], 0.0)
    reg_abs = oracle.regulariser_apply(np.abs(P32), [np.abs(r) for r in ref.R], p.lam)
    bound = 8.5 * U_BF16 * chain_abs + 1e-6 * reg_abs + 1e-30

    op = cta.Operator(p.A, p.D, p.lam)
    for variants in (PIPE, PIPE6, PIPE7, PIPE8):
        cta.cta_op_set_tuning(op.handle, "bf16", *variants)
        Q = op.apply(Pd, chain="bf16")
        torch.cuda.synchronize()
        err = np.abs(host(Q) - Qref)
        worst = float((err / bound).max())
        print(f"BF16 apply at {N} {variants}: max |dQ| / bound = {worst:.3f}, "
              f"max rel = {float(err.max() / np.abs(Qref).max()):.2e}")
        assert worst <= 1.0
    op.close()


@pytest.mark.parametrize("precond", [0, 1])
def test_persistent_cg_passes_match_plain_at_full_size(precond):
    """Iterates of the BF16-chain CG (plain, and with the tensor-inverse
    preconditioner) with every pass persistent equal those with one tile per
    workgroup, bit for bit."""
    torch = torch_cuda()
    p = workload.make_problem(N, M, 1e-4, 0.01, 2000, 1e-8, with_data=False)
    op = cta.Operator(p.A, p.D, p.lam)
    if precond:
        op.set_preconditioner(181 * p.lam)
    B = dev(np.random.default_rng(44).standard_normal(N), torch.float32)
    out = []
    for variants in (PLAIN, PIPE, PIPE6, PIPE7, PIPE8):
        cta.cta_op_set_tuning(op.handle, "bf16", *variants)
        X, info = op.solve(B, precision="bf16", rtol=1e-30, max_iter=6, check_every=6,
                           precond=precond)
        assert info["iters"] == 6, info
        out.append(X.clone())
    assert all(torch.equal(out[0], o) for o in out[1:])
    if precond:
        R = dev(np.random.default_rng(45).standard_normal(N), torch.float32)
        Z = []
        for variants in (PLAIN, PIPE):
            cta.cta_op_set_tuning(op.handle, "bf16", *variants)
            Z.append(op.precond(R, chain="bf16").clone())
        assert torch.equal(Z[0], Z[1])
    op.close()
