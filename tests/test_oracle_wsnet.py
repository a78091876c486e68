"""Pins of the warm-start network oracle (separable convolutions, Table 1;
gradients by the derivative rule of App. A.8)."""
import numpy as np
import pytest

import oracle
from oracle import wsnet


def _rand_params(C, width, blocks, order, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return wsnet.unpack(scale * rng.standard_normal(wsnet.param_count(C, width, blocks, order)),
                        C, width, blocks, order)


def test_headline_parameter_count():
    assert wsnet.param_count(32, 5, 5, 4) == 103137


@pytest.mark.parametrize("k", [0, 1, 2])
def test_conv_is_toeplitz_mode_product(k):
    # Table 1: a 1-D convolution along a mode is a mode product with a banded
    # Toeplitz matrix; with channels it is a sum of such products per channel pair
    rng = np.random.default_rng(1 + k)
    shape = (7, 6, 5)
    Cin, Cout, width = 3, 2, 5
    z = rng.standard_normal((Cin,) + shape)
    W = rng.standard_normal((Cout, Cin, width))
    out = wsnet.conv(z, W, k)
    n = shape[k]
    for co in range(Cout):
        ref = np.zeros(shape)
        for ci in range(Cin):
            T = np.zeros((n, n))
            for i in range(n):
                for ip in range(n):
                    if abs(ip - i) <= width // 2:
                        T[i, ip] = W[co, ci, ip - i + width // 2]
            ref += oracle.mode_product(z[ci], T, k)
        np.testing.assert_allclose(out[co], ref, rtol=1e-13, atol=1e-13)


def test_gradient_matches_central_differences():
    C, width, blocks, order = 4, 5, 2, 4
    shape = (6, 5, 4, 3)
    rng = np.random.default_rng(3)
    theta = 0.3 * rng.standard_normal(wsnet.param_count(C, width, blocks, order))
    B = rng.standard_normal(shape)
    T = rng.standard_normal(shape)
    L0, g = wsnet.mse_loss(wsnet.unpack(theta, C, width, blocks, order), B, T)
    h = 1e-6
    fd = np.zeros_like(theta)
    for i in range(theta.size):
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        Lp, _ = wsnet.mse_loss(wsnet.unpack(tp, C, width, blocks, order), B, T)
        Lm, _ = wsnet.mse_loss(wsnet.unpack(tm, C, width, blocks, order), B, T)
        fd[i] = (Lp - Lm) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-9)


def test_linear_without_activation():
    P = _rand_params(3, 5, 2, 3, seed=5)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((5, 4, 6))
    y = rng.standard_normal((5, 4, 6))
    f0 = wsnet.forward(P, np.zeros_like(x), relu=False)
    fx = wsnet.forward(P, x, relu=False) - f0
    fy = wsnet.forward(P, y, relu=False) - f0
    fxy = wsnet.forward(P, 2.0 * x - 0.5 * y, relu=False) - f0
    np.testing.assert_allclose(fxy, 2.0 * fx - 0.5 * fy, rtol=1e-11, atol=1e-11)


def test_warm_start_scale_equivariant():
    P = _rand_params(3, 5, 1, 3, seed=7)
    B = np.random.default_rng(8).standard_normal((5, 4, 6))
    np.testing.assert_allclose(wsnet.warm_start(P, 4.0 * B), 4.0 * wsnet.warm_start(P, B),
                               rtol=1e-12, atol=1e-12)


def test_adam_first_step_is_sign_step():
    rng = np.random.default_rng(9)
    theta = rng.standard_normal(20)
    g = rng.standard_normal(20)
    new, m, v = wsnet.adam_step(theta, g, np.zeros(20), np.zeros(20), 1, lr=1e-2, eps=0.0)
    np.testing.assert_allclose(new, theta - 1e-2 * np.sign(g), rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_pack_unpack_roundtrip():
    C, width, blocks, order = 4, 5, 2, 4
    theta = np.arange(wsnet.param_count(C, width, blocks, order), dtype=float)
    assert np.array_equal(wsnet.pack(wsnet.unpack(theta, C, width, blocks, order)), theta)


def test_bf16_round_ties_to_even():
    u = 2.0 ** -8  # half an ulp of BF16 at 1.0
    x = np.array([1.0 + u, 1.0 + 3 * u, 1.0 + u + 2.0 ** -20, -(1.0 + u), 3.0, 0.0, 2.0 ** -130])
    want = np.array([1.0, 1.0 + 4 * u, 1.0 + 2 * u, -1.0, 3.0, 0.0, 2.0 ** -130])
    assert np.array_equal(wsnet.bf16_round(x), want)


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(5).standard_normal(10000) * 10.0 ** np.random.default_rng(6).integers(-6, 6, 10000)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).double().numpy()
    assert np.array_equal(wsnet.bf16_round(x), ref)


def test_store_model_exact_on_representable_values():
    """With integer weights in {-1, 0, 1}, zero biases and small integer
    inputs every activation is a small integer, exact in BF16: the storage
    model must then reproduce the exact network bit for bit."""
    rng = np.random.default_rng(8)
    C, width, blocks, order = 4, 5, 1, 3
    theta = rng.integers(-1, 2, wsnet.param_count(C, width, blocks, order)).astype(np.float64)
    P = wsnet.unpack(theta, C, width, blocks, order)
    for cs in P["c"]:
        for c in cs:
            c[:] = 0.0
    P["lb"][:] = 0.0
    b = rng.integers(-1, 2, (3, 4, 3)).astype(np.float64)
    exact = wsnet.forward(P, b)
    assert np.max(np.abs(exact)) < 256
    assert np.array_equal(wsnet.forward(P, b, store=wsnet.bf16_round), exact)
    _, acts = wsnet.forward(P, b, keep=True)
    _, acts_s = wsnet.forward(P, b, keep=True, store=wsnet.bf16_round)
    dout = rng.integers(-1, 2, b.shape).astype(np.float64)
    G = wsnet.pack(wsnet.backward(P, acts, dout))
    Gs = wsnet.pack(wsnet.backward(P, acts_s, dout, store=wsnet.bf16_round))
    assert np.array_equal(G, Gs)


def test_store_model_rounds_activations():
    """With BF16 storage every kept activation is a BF16 value and the output
    moves away from the exact one by about the BF16 unit roundoff."""
    C, width, blocks, order = 8, 5, 2, 3
    theta = np.random.default_rng(9).standard_normal(wsnet.param_count(C, width, blocks, order)) * 0.2
    P = wsnet.unpack(theta, C, width, blocks, order)
    b = np.random.default_rng(10).standard_normal((5, 6, 4))
    out, acts = wsnet.forward(P, b, keep=True, store=wsnet.bf16_round)
    for t in acts["h"] + [z for zs in acts["z"] for z in zs]:
        assert np.array_equal(wsnet.bf16_round(t), t)
    exact = wsnet.forward(P, b)
    rel = np.linalg.norm(out - exact) / np.linalg.norm(exact)
    assert 1e-5 < rel < 3e-2


def test_adam_bias_correction_with_constant_gradient():
    """With the same gradient g at every step the bias-corrected moments are
    exactly g and g^2 at every t (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so
    each step moves theta by lr * sign(g) when eps = 0: a wrong exponent in the
    correction breaks this from t = 2 on."""
    rng = np.random.default_rng(10)
    theta0 = rng.standard_normal(16)
    g = rng.standard_normal(16)
    theta, m, v = theta0.copy(), np.zeros(16), np.zeros(16)
    for t in (1, 2, 3):
        theta, m, v = wsnet.adam_step(theta, g, m, v, t, lr=1e-2, beta1=0.9, beta2=0.999, eps=0.0)
        np.testing.assert_allclose(m, (1 - 0.9 ** t) * g, rtol=1e-13)
        np.testing.assert_allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-12)
        np.testing.assert_allclose(theta, theta0 - t * 1e-2 * np.sign(g), rtol=1e-12, atol=1e-14)


def test_adam_second_and_third_steps_by_hand():
    """Two scalar gradients 3 and -1, then 2: the moments and the update
    written out by hand from the definitions (Kingma and Ba), b1 = 0.5,
    b2 = 0.75, lr = 0.1, eps = 0."""
    th, m, v = np.array([1.0]), np.zeros(1), np.zeros(1)
    th, m, v = wsnet.adam_step(th, np.array([3.0]), m, v, 1, lr=0.1, beta1=0.5, beta2=0.75, eps=0.0)
    # m1 = 1.5, v1 = 2.25, mhat = 3, vhat = 9: step 0.1 * 3 / 3
    assert np.isclose(th[0], 0.9, rtol=1e-15)
    th, m, v = wsnet.adam_step(th, np.array([-1.0]), m, v, 2, lr=0.1, beta1=0.5, beta2=0.75, eps=0.0)
    # m2 = 0.75 - 0.5 = 0.25, v2 = 1.6875 + 0.25 = 1.9375; mhat = 0.25 / 0.75 = 1/3,
    # vhat = 1.9375 / (1 - 0.5625) = 4.428571..., step 0.1 * (1/3) / sqrt(vhat)
    assert np.isclose(m[0], 0.25) and np.isclose(v[0], 1.9375)
    th2 = 0.9 - 0.1 * (1.0 / 3.0) / np.sqrt(1.9375 / 0.4375)
    assert np.isclose(th[0], th2, rtol=1e-14)
    th, m, v = wsnet.adam_step(th, np.array([2.0]), m, v, 3, lr=0.1, beta1=0.5, beta2=0.75, eps=0.0)
    # m3 = 0.125 + 1 = 1.125, v3 = 1.453125 + 1 = 2.453125; corrections 1 - 0.125, 1 - 0.421875
    assert np.isclose(m[0], 1.125) and np.isclose(v[0], 2.453125)
    th3 = th2 - 0.1 * (1.125 / 0.875) / np.sqrt(2.453125 / 0.578125)
    assert np.isclose(th[0], th3, rtol=1e-14)


def test_what_a_start_can_save_on_the_blob_workload():
    """How much any starting tensor that captures the solution's structure can
    save on the warm-start workload (blob fields plus N(0, 0.1) white noise,
    collocation 1.5n x n, lambda 1e-3), by the oracle's CG to 1e-8: starting
    from the exact noise-free blob field, or from the coarse-grid projection of
    the exact solution, saves at most a few percent of the iterations.  CG's
    count is set by the rough (noise) part of the solution, which a start can
    only supply by applying the inverse operator itself."""
    import workload
    from oracle import multigrid
    n, m = (24, 24, 24, 8), (36, 36, 36, 12)
    A, D = workload.factors(n, m)
    op = oracle.NormalOperator(A, D, 1e-3)
    rng = np.random.default_rng(10000)
    X = workload.blob_field(n, rng, 0.1)
    B = op.rhs(op.forward(X) + 0.01 * rng.standard_normal(m))
    exact = oracle.cg(op, B, rtol=1e-13)
    zero = oracle.cg(op, B, rtol=1e-8).iters
    smooth = workload.blob_field(n, np.random.default_rng(10000), 0.0)
    P = [multigrid.interpolation(k, (k + 1) // 2) for k in n]
    Xc = exact.x
    for k in range(4):
        Xc = oracle.mode_product(Xc, np.linalg.solve(P[k].T @ P[k], P[k].T), k)
    coarse = multigrid.prolong(Xc, P)
    for x0 in (smooth, coarse):
        its = oracle.cg(op, B, x0=x0, rtol=1e-8).iters
        assert its >= 0.93 * zero, (its, zero)
