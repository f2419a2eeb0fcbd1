"""Pins of the FP64 warm-start network reference: its layers against
brute-force loops on tiny images, its backward pass against central finite
differences of its own loss, and one Adam step against the closed form."""
import numpy as np
import pytest

from oracle import surrogate as S
from scenes import SplitMix64


def _rand(shape, seed, scale=1.0):
    rng = SplitMix64(seed)
    return rng.normal_array(int(np.prod(shape))).reshape(shape) * scale


def test_conv_against_loops():
    x = _rand((2, 5, 4, 3), 1)
    for k in (3, 1):
        W = _rand((4, 3, k, k), 2)
        b = _rand((4,), 3)
        y = S.conv(x, W, b)
        p = k // 2
        ref = np.zeros_like(y)
        for n in range(2):
            for i in range(5):
                for j in range(4):
                    for o in range(4):
                        s = b[o]
                        for c in range(3):
                            for ky in range(k):
                                for kx in range(k):
                                    ii, jj = i + ky - p, j + kx - p
                                    if 0 <= ii < 5 and 0 <= jj < 4:
                                        s += x[n, ii, jj, c] * W[o, c, ky, kx]
                        ref[n, i, j, o] = s
        assert np.allclose(y, ref, rtol=0, atol=1e-13)


def test_conv_identity_kernel_and_shift():
    x = _rand((1, 6, 6, 2), 4)
    W = np.zeros((2, 2, 3, 3))
    W[0, 0, 1, 1] = W[1, 1, 1, 1] = 1.0
    assert np.array_equal(S.conv(x, W, np.zeros(2)), x)
    W = np.zeros((1, 2, 3, 3))
    W[0, 1, 0, 0] = 1.0  # picks channel 1 at (i - 1, j - 1)
    y = S.conv(x, W, np.zeros(1))[0, :, :, 0]
    assert np.array_equal(y[1:, 1:], x[0, :-1, :-1, 1])
    assert not y[0].any() and not y[:, 0].any()


def test_pool_and_upsample_against_loops():
    x = _rand((2, 4, 6, 3), 5)
    p = S.pool(x)
    for n in range(2):
        for i in range(2):
            for j in range(3):
                assert np.allclose(p[n, i, j], x[n, 2 * i:2 * i + 2, 2 * j:2 * j + 2].mean(axis=(0, 1)), atol=1e-15)
    u = S.upsample(p)
    for i in range(4):
        for j in range(6):
            assert np.array_equal(u[:, i, j], p[:, i // 2, j // 2])
    # adjoints: <pool x, y> = <x, pool^T y>, <up x, y> = <x, up^T y>
    y = _rand(p.shape, 6)
    assert np.isclose((S.pool(x) * y).sum(), (x * S.pool_backward(y)).sum(), atol=1e-12)
    z = _rand(x.shape, 7)
    assert np.isclose((S.upsample(p) * z).sum(), (p * S.upsample_backward(z)).sum(), atol=1e-12)


def test_parameter_count():
    assert S.num_params(4, 2, 32) == 471874


@pytest.fixture(scope="module")
def small_net():
    in_ch, out_ch, width, size = 4, 2, 32, 8
    npar = S.num_params(in_ch, out_ch, width)
    theta = np.zeros(npar)
    o = 0
    for name, ci, co, k in S.layer_shapes(in_ch, out_ch, width):
        nW = co * ci * k * k
        theta[o:o + nW] = _rand((nW,), 100 + o, np.sqrt(2.0 / (ci * k * k)))
        theta[o + nW:o + nW + co] = _rand((co,), 200 + o, 0.05)
        o += nW + co
    x = _rand((2, size, size, in_ch), 8)
    t = _rand((2, size, size, out_ch), 9)
    w = np.abs(_rand((2, size, size), 10)) / (2 * size * size)
    return theta, x, t, w, (in_ch, out_ch, width)


def test_backward_matches_central_differences(small_net):
    theta, x, t, w, dims = small_net
    L, g, _ = S.loss_and_grad(theta, x, t, w, *dims)
    assert L > 0
    # parameters spread over every layer (weights and biases)
    idx = []
    o = 0
    for name, ci, co, k in S.layer_shapes(*dims):
        nW = co * ci * k * k
        idx += [o, o + nW // 3, o + nW - 1, o + nW, o + nW + co - 1]
        o += nW + co
    h = 1e-6
    errs = []
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (S.loss_and_grad(tp, x, t, w, *dims)[0] - S.loss_and_grad(tm, x, t, w, *dims)[0]) / (2 * h)
        errs.append(abs(fd - g[i]) / max(abs(fd), abs(g[i]), 1e-8))
    errs = np.array(errs)
    assert np.median(errs) < 1e-6, errs
    assert errs.max() < 1e-4, errs


def test_loss_gradient_in_output(small_net):
    _, _, t, w, _ = small_net
    y = _rand(t.shape, 11)
    L, dy = S.loss(y, t, w)
    h = 1e-6
    for k in (0, 17, 100):
        yp, ym = y.copy(), y.copy()
        yp.flat[k] += h
        ym.flat[k] -= h
        fd = (S.loss(yp, t, w)[0] - S.loss(ym, t, w)[0]) / (2 * h)
        assert abs(fd - dy.flat[k]) < 1e-8


def test_adam_first_step_closed_form():
    g = _rand((50,), 12)
    theta = _rand((50,), 13)
    lr, eps = 1e-3, 1e-8
    th, m, v = S.adam(theta, g, np.zeros(50), np.zeros(50), 1, lr, eps=eps)
    assert np.allclose(th, theta - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    # with a constant gradient the bias-corrected step stays lr * sign(g)
    th2, _, _ = S.adam(th, g, m, v, 2, lr, eps=0.0)
    assert np.allclose(th2 - th, -lr * np.sign(g), atol=1e-12)
