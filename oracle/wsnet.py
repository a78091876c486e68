"""Learned warm-start network (oracle; test infrastructure only).

A separable network proposes the starting tensor of CG: each layer is a
1-D convolution along one mode, i.e. a mode product with a banded Toeplitz
matrix per channel pair (the convolution row of Table 1 expresses an
N-D convolution as such separable 1-D transforms).  Gradients follow the
derivative rule of App. A.8 (the derivative of a linear tensor map is the map
itself, so backpropagation applies the transposed maps) and the chain rule
through the pointwise nonlinearity.  Everything is float64 NumPy; the
convolution is written as an explicit loop over taps.

Architecture for an order-N input tensor b (extents n):
    h0[c]   = lw[c] * b + lb[c]                               (lift, 1 -> C)
    block:  z1 = relu(conv_1(h) + c1)                          (mode 1)
            z2 = relu(conv_2(z1) + c2)                         (mode 2)
            ...                                                (modes 3 .. N-1)
            h  = h + conv_N(z_{N-1}) + cN                      (mode N, residual)
    out     = sum_c pw[c] * h[c] + pb                         (projection, C -> 1)
conv_k(z)[co, i] = sum_{ci, w} W[co, ci, w] * z[ci, i + (w - width//2) e_k] with
zero padding.  The warm start for a right-hand side B is X0 = s * out(B / s)
with s the RMS of B (||B||_2 / sqrt(#entries)): N^{-1} is linear, so the
network sees inputs of unit RMS whatever the scale of B.

Storage precision model.  The warm-start form fixes BF16 weights and
activations with FP32 accumulation.  Every function below takes an optional
``store`` callable (``bf16_round`` or None): when given, the convolution
weights and every stored activation and activation gradient (h, z, the
gradients between convolutions) are rounded with it, while sums stay in
float64.  With store=None the network is exact float64.

Flat parameter layout (shared with the GPU library):
    lw (C), lb (C), then for each block and each mode k: W_k (C*C*width, index
    (co*C + ci)*width + w) and c_k (C); then pw (C), pb (1).
"""
import numpy as np


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even) via float32: keep the
    upper 16 bits of the float32 pattern after adding half an ulp of BF16
    (0x7fff plus the lowest kept bit)."""
    x32 = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    bits = x32.view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(x))


def _ident(x):
    return x


def param_count(C, width, blocks, order):
    return 2 * C + blocks * order * (C * C * width + C) + C + 1


def unpack(theta, C, width, blocks, order):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == param_count(C, width, blocks, order)
    o = 0

    def take(k):
        nonlocal o
        v = theta[o:o + k]
        o += k
        return v

    P = {"lw": take(C), "lb": take(C), "W": [], "c": []}
    for _ in range(blocks):
        Ws, cs = [], []
        for _ in range(order):
            Ws.append(take(C * C * width).reshape(C, C, width))
            cs.append(take(C))
        P["W"].append(Ws)
        P["c"].append(cs)
    P["pw"] = take(C)
    P["pb"] = take(1)[0]
    return P


def pack(P):
    parts = [P["lw"], P["lb"]]
    for Ws, cs in zip(P["W"], P["c"]):
        for W, c in zip(Ws, cs):
            parts += [np.asarray(W).reshape(-1), c]
    parts += [P["pw"], np.array([P["pb"]])]
    return np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1) for p in parts])


def _shift(z, k, d):
    """z shifted along spatial mode k (axis k+1) by d with zero fill: out[i] = z[i + d]."""
    out = np.zeros_like(z)
    n = z.shape[k + 1]
    src = [slice(None)] * z.ndim
    dst = [slice(None)] * z.ndim
    if d >= 0:
        src[k + 1] = slice(d, n)
        dst[k + 1] = slice(0, n - d)
    else:
        src[k + 1] = slice(0, n + d)
        dst[k + 1] = slice(-d, n)
    out[tuple(dst)] = z[tuple(src)]
    return out


def conv(z, W, k):
    """1-D convolution along spatial mode k of a (C_in, n...) tensor with W (C_out, C_in, width)."""
    width = W.shape[2]
    half = width // 2
    out = np.zeros((W.shape[0],) + z.shape[1:])
    for w in range(width):
        zs = _shift(z, k, w - half)
        out += np.tensordot(W[:, :, w], zs, axes=([1], [0]))
    return out


def conv_backward(g, zin, W, k):
    """Gradients of sum(g * conv(zin, W, k)) w.r.t. zin and W."""
    width = W.shape[2]
    half = width // 2
    dz = np.zeros_like(zin)
    dW = np.zeros_like(W)
    for w in range(width):
        d = w - half
        zs = _shift(zin, k, d)
        dW[:, :, w] = np.tensordot(g, zs, axes=(list(range(1, g.ndim)), list(range(1, zs.ndim))))
        # transpose of "shift by d then mix channels": mix back, then shift by -d
        dz += _shift(np.tensordot(W[:, :, w].T, g, axes=([1], [0])), k, -d)
    return dz, dW


def forward(P, b, relu=True, keep=False, store=None):
    """Network output for a normalised input b (no scaling).  keep=True also
    returns the activations needed by backward()."""
    st = store or _ident
    b = np.asarray(b, dtype=np.float64)
    order = b.ndim
    h = P["lw"][:, None] * b.reshape(1, -1) + P["lb"][:, None]
    h = st(h.reshape((-1,) + b.shape))
    acts = {"b": b, "h": [h], "z": []}
    act = (lambda x: np.maximum(x, 0.0)) if relu else (lambda x: x)
    for Ws, cs in zip(P["W"], P["c"]):
        zs = []
        z = h
        for k in range(order):
            y = conv(z, st(Ws[k]), k) + cs[k].reshape((-1,) + (1,) * order)
            if k < order - 1:
                z = st(act(y))
                zs.append(z)
            else:
                h = st(h + y)
        acts["z"].append(zs)
        acts["h"].append(h)
    out = np.tensordot(P["pw"], h, axes=([0], [0])) + P["pb"]
    return (out, acts) if keep else out


def backward(P, acts, dout, relu=True, store=None):
    """Gradient (same dict structure as P) of sum(dout * forward(P, b)); pass
    the same ``store`` as to the forward that produced ``acts``."""
    st = store or _ident
    b = acts["b"]
    order = b.ndim
    G = {"lw": None, "lb": None, "W": [], "c": [], "pw": None, "pb": None}
    h_last = acts["h"][-1]
    G["pw"] = np.tensordot(h_last, dout, axes=(list(range(1, h_last.ndim)), list(range(dout.ndim))))
    G["pb"] = float(np.sum(dout))
    dh = st(P["pw"].reshape((-1,) + (1,) * order) * dout[None])
    nblocks = len(P["W"])
    Wg = [None] * nblocks
    cg = [None] * nblocks
    for bi in reversed(range(nblocks)):
        Ws, zs = P["W"][bi], acts["z"][bi]
        hin = acts["h"][bi]
        Wg[bi] = [None] * order
        cg[bi] = [None] * order
        g = dh  # gradient at the last convolution's output (before the residual sum)
        for k in reversed(range(order)):
            zin = hin if k == 0 else zs[k - 1]
            cg[bi][k] = np.sum(g, axis=tuple(range(1, g.ndim)))
            dz, dW = conv_backward(g, zin, st(Ws[k]), k)
            Wg[bi][k] = dW
            if k > 0:
                g = st(dz * (zs[k - 1] > 0) if relu else dz)
            else:
                dh = st(dh + dz)  # residual skip plus the path through the block
    G["W"] = Wg
    G["c"] = cg
    h0grad = dh
    G["lw"] = np.tensordot(h0grad, b, axes=(list(range(1, h0grad.ndim)), list(range(b.ndim))))
    G["lb"] = np.sum(h0grad, axis=tuple(range(1, h0grad.ndim)))
    return G


def rms(B):
    B = np.asarray(B, dtype=np.float64)
    return float(np.linalg.norm(B) / np.sqrt(B.size))


def warm_start(P, B, relu=True, store=None):
    """X0 = s * f(B / s), s = RMS of B."""
    s = rms(B)
    if s == 0.0:
        return np.zeros_like(B, dtype=np.float64)
    return s * forward(P, np.asarray(B) / s, relu=relu, store=store)


def mse_loss(P, B, T, relu=True, store=None):
    """L = mean((f(B/s) - T/s)^2) and dL/dtheta (flat), s = RMS of B."""
    s = rms(B)
    out, acts = forward(P, np.asarray(B) / s, relu=relu, keep=True, store=store)
    diff = out - np.asarray(T, dtype=np.float64) / s
    L = float(np.mean(diff ** 2))
    dout = 2.0 * diff / diff.size
    G = backward(P, acts, dout, relu=relu, store=store)
    return L, pack(G)


def adam_step(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba): returns new theta, m, v; t is the 1-based step."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
