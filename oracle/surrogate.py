"""FP64 reference of the warm-start network (test infrastructure only).

The network maps per-node maps of a cross-section to its steady fields; its
layers are listed in the C header of the library (three levels, 3x3
convolutions with ReLU, 2x2 average pooling, nearest x2 upsampling
concatenated with the skip tensor, a 1x1 linear head).  This module writes the
forward pass, the loss, the backward pass (chain rule, layer by layer) and the
Adam update out in numpy, images NHWC, parameters in the same flat order as
the library: per layer W[c_out][c_in][ky][kx], then b[c_out].

Pinned in tests/test_oracle_surrogate.py by central finite differences of the
loss, brute-force loops on tiny images and the closed form of one Adam step.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

# (name, input tensor, c_in multiplier or None for in_ch, c_out multiplier or
# None for out_ch, kernel size)
_LAYERS = [
    ("e1a", "in", None, 1, 3), ("e1b", "e1a", 1, 1, 3),
    ("e2a", "p1", 1, 2, 3), ("e2b", "e2a", 2, 2, 3),
    ("e3a", "p2", 2, 4, 3), ("e3b", "e3a", 4, 4, 3),
    ("d2a", "u2", 6, 2, 3), ("d2b", "d2a", 2, 2, 3),
    ("d1a", "u1", 3, 1, 3), ("d1b", "d1a", 1, 1, 3),
    ("head", "d1b", 1, None, 1),
]


def layer_shapes(in_ch: int, out_ch: int, width: int) -> List[Tuple[str, int, int, int]]:
    out = []
    for name, _, ci, co, k in _LAYERS:
        out.append((name, in_ch if ci is None else ci * width, out_ch if co is None else co * width, k))
    return out


def num_params(in_ch: int = 4, out_ch: int = 2, width: int = 32) -> int:
    return sum(co * ci * k * k + co for _, ci, co, k in layer_shapes(in_ch, out_ch, width))


def unpack(theta: np.ndarray, in_ch: int, out_ch: int, width: int):
    """flat parameters -> {name: (W [co, ci, k, k], b [co])}"""
    params, o = {}, 0
    for name, ci, co, k in layer_shapes(in_ch, out_ch, width):
        nW = co * ci * k * k
        W = theta[o:o + nW].reshape(co, ci, k, k)
        o += nW
        b = theta[o:o + co]
        o += co
        params[name] = (W, b)
    assert o == theta.size
    return params


def pack(grads: dict, in_ch: int, out_ch: int, width: int) -> np.ndarray:
    parts = []
    for name, _, _, _ in layer_shapes(in_ch, out_ch, width):
        dW, db = grads[name]
        parts += [dW.ravel(), db.ravel()]
    return np.concatenate(parts)


# ---------------------------------------------------------------------------
# layers (x: [N, H, W, C])
# ---------------------------------------------------------------------------
def conv(x, W, b):
    """y[n, i, j, o] = b[o] + sum_{c, ky, kx} x[n, i + ky - p, j + kx - p, c] W[o, c, ky, kx]
    with zeros outside the image (p = k // 2)."""
    k = W.shape[2]
    p = k // 2
    N, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (0, 0)))
    y = np.zeros((N, H, Wd, W.shape[0]))
    for ky in range(k):
        for kx in range(k):
            y += xp[:, ky:ky + H, kx:kx + Wd, :] @ W[:, :, ky, kx].T
    return y + b


def conv_backward(x, W, dy):
    """gradients of conv with respect to x, W and b."""
    k = W.shape[2]
    p = k // 2
    N, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (0, 0)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for ky in range(k):
        for kx in range(k):
            dxp[:, ky:ky + H, kx:kx + Wd, :] += dy @ W[:, :, ky, kx]
            dW[:, :, ky, kx] = np.tensordot(dy, xp[:, ky:ky + H, kx:kx + Wd, :], axes=([0, 1, 2], [0, 1, 2]))
    return dxp[:, p:p + H, p:p + Wd, :], dW, dy.sum(axis=(0, 1, 2))


def pool(x):
    """2x2 average."""
    return 0.25 * (x[:, 0::2, 0::2] + x[:, 1::2, 0::2] + x[:, 0::2, 1::2] + x[:, 1::2, 1::2])


def pool_backward(dy):
    N, H, W, C = dy.shape
    dx = np.zeros((N, 2 * H, 2 * W, C))
    for i in (0, 1):
        for j in (0, 1):
            dx[:, i::2, j::2] = 0.25 * dy
    return dx


def upsample(x):
    """nearest x2."""
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample_backward(dy):
    return dy[:, 0::2, 0::2] + dy[:, 1::2, 0::2] + dy[:, 0::2, 1::2] + dy[:, 1::2, 1::2]


def relu(z):
    return np.maximum(z, 0.0)


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def forward(theta, x, in_ch: int, out_ch: int, width: int):
    """output [N, S, S, out_ch] and the tensors the backward pass needs."""
    P = unpack(np.asarray(theta, np.float64), in_ch, out_ch, width)
    t = {"in": np.asarray(x, np.float64)}
    z = {}

    def layer(name, src):
        W, b = P[name]
        z[name] = conv(t[src], W, b)
        t[name] = relu(z[name]) if name != "head" else z[name]

    layer("e1a", "in")
    layer("e1b", "e1a")
    t["p1"] = pool(t["e1b"])
    layer("e2a", "p1")
    layer("e2b", "e2a")
    t["p2"] = pool(t["e2b"])
    layer("e3a", "p2")
    layer("e3b", "e3a")
    t["u2"] = np.concatenate([upsample(t["e3b"]), t["e2b"]], axis=3)
    layer("d2a", "u2")
    layer("d2b", "d2a")
    t["u1"] = np.concatenate([upsample(t["d2b"]), t["e1b"]], axis=3)
    layer("d1a", "u1")
    layer("d1b", "d1a")
    layer("head", "d1b")
    return t["head"], (P, t, z)


def loss(y, target, weight):
    """sum_p weight_p sum_c (y - target)^2 / C and its gradient in y."""
    C = y.shape[3]
    d = y - target
    L = float((weight[..., None] * d * d).sum() / C)
    return L, 2.0 * weight[..., None] * d / C


def backward(cache, dy, in_ch: int, out_ch: int, width: int):
    """flat parameter gradient for the output gradient dy."""
    P, t, z = cache
    g = {}
    dt = {}

    def back(name, src, d_out):
        W, _ = P[name]
        dz = d_out if name == "head" else d_out * (z[name] > 0)
        dx, dW, db = conv_backward(t[src], W, dz)
        g[name] = (dW, db)
        return dx

    w = width
    dt["d1b"] = back("head", "d1b", dy)
    dt["d1a"] = back("d1b", "d1a", dt["d1b"])
    du1 = back("d1a", "u1", dt["d1a"])
    dt["d2b"] = upsample_backward(du1[..., :2 * w])
    dt["e1b"] = du1[..., 2 * w:]
    dt["d2a"] = back("d2b", "d2a", dt["d2b"])
    du2 = back("d2a", "u2", dt["d2a"])
    dt["e3b"] = upsample_backward(du2[..., :4 * w])
    dt["e2b"] = du2[..., 4 * w:]
    dt["e3a"] = back("e3b", "e3a", dt["e3b"])
    dp2 = back("e3a", "p2", dt["e3a"])
    dt["e2b"] = dt["e2b"] + pool_backward(dp2)
    dt["e2a"] = back("e2b", "e2a", dt["e2b"])
    dp1 = back("e2a", "p1", dt["e2a"])
    dt["e1b"] = dt["e1b"] + pool_backward(dp1)
    dt["e1a"] = back("e1b", "e1a", dt["e1b"])
    back("e1a", "in", dt["e1a"])
    return pack(g, in_ch, out_ch, width)


def loss_and_grad(theta, x, target, weight, in_ch: int, out_ch: int, width: int):
    y, cache = forward(theta, x, in_ch, out_ch, width)
    L, dy = loss(y, target, weight)
    return L, backward(cache, dy, in_ch, out_ch, width), y


def adam(theta, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """one Adam update (Kingma and Ba), step number t >= 1; returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
