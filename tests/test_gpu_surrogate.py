"""Warm-start network kernels (lbm_nn_*) against the FP64 numpy reference:
forward pass, loss, parameter gradients and the Adam update, in the FP32
debug mode and in BF16; and a short training run that lowers the loss."""
import numpy as np
import pytest

from oracle import surrogate as S
from scenes import SplitMix64
from paper_2506_00907_amd import lbm

pytestmark = pytest.mark.gpu

DIMS = (4, 2, 32)


def he_init(seed=1234, dims=DIMS):
    rng = SplitMix64(seed)
    parts = []
    for name, ci, co, k in S.layer_shapes(*dims):
        parts.append(rng.normal_array(co * ci * k * k) * np.sqrt(2.0 / (ci * k * k)))
        parts.append(rng.normal_array(co) * 0.05)
    return np.concatenate(parts)


def batch(n, size, seed):
    rng = SplitMix64(seed)
    x = rng.normal_array(n * size * size * 4).reshape(n, size, size, 4)
    t = rng.normal_array(n * size * size * 2).reshape(n, size, size, 2)
    w = (rng.uniform_array(n * size * size).reshape(n, size, size) > 0.3) / (n * size * size)
    return x, t, w.astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def layer_errors(g, go):
    out, o = {}, 0
    for name, ci, co, k in S.layer_shapes(*DIMS):
        n = co * ci * k * k + co
        out[name] = rel(g[o:o + n], go[o:o + n])
        o += n
    return out


@pytest.mark.parametrize("prec,tol_y,tol_g", [("f32", 1e-6, 1e-5), ("bf16", 1e-2, 3e-2)])
@pytest.mark.parametrize("size,n", [(32, 2), (40, 1)])
def test_forward_backward_against_reference(prec, tol_y, tol_g, size, n):
    theta = he_init()
    x, t, w = batch(n, size, 7)
    net = lbm.Network(n, size, precision=prec)
    net.set_params(theta)
    y = net.forward(x).cpu().numpy()
    L = net.backward(t, w)
    g = net.grads().cpu().numpy()
    # the reference sees the parameters and inputs as the kernels do (FP32)
    th32 = theta.astype(np.float32).astype(np.float64)
    x32 = x.astype(np.float32).astype(np.float64)
    Lo, go, yo = S.loss_and_grad(th32, x32, t.astype(np.float32).astype(np.float64),
                                 w.astype(np.float32).astype(np.float64), *DIMS)
    ey = rel(y, yo)
    eg = layer_errors(g, go)
    print(f"[{prec} S={size}] output {ey:.2e} loss {abs(L - Lo) / Lo:.2e} grads", {k: f"{v:.1e}" for k, v in eg.items()})
    assert ey < tol_y
    assert abs(L - Lo) / Lo < tol_y
    assert max(eg.values()) < tol_g
    assert rel(g, go) < tol_g


def test_adam_step_matches_reference():
    theta = he_init(99)
    x, t, w = batch(2, 32, 8)
    net = lbm.Network(2, 32, precision="f32")
    net.set_params(theta)
    net.forward(x)
    net.backward(t, w)
    g = net.grads().cpu().numpy().astype(np.float64)
    th32 = theta.astype(np.float32).astype(np.float64)
    m = np.zeros_like(th32)
    v = np.zeros_like(th32)
    ref = th32
    for step in (1, 2):
        net.adam_step(1e-3)
        ref, m, v = S.adam(ref, g, m, v, step, 1e-3)
        if step == 1:
            net.forward(x)
            net.backward(t, w)  # same batch, new parameters: a different gradient
            g2 = net.grads().cpu().numpy().astype(np.float64)
    # second step used g2 on the device; redo the reference with it
    ref, m, v = S.adam(th32, g, np.zeros_like(g), np.zeros_like(g), 1, 1e-3)
    ref, m, v = S.adam(ref, g2, m, v, 2, 1e-3)
    got = net.params().cpu().numpy().astype(np.float64)
    assert np.abs(got - ref).max() < 1e-6


def test_training_lowers_the_loss():
    size, n = 64, 4
    rng = SplitMix64(5)
    x = rng.normal_array(n * size * size * 4).reshape(n, size, size, 4)
    # a target the network can represent: smooth functions of the inputs
    t = np.stack([np.tanh(x[..., 0] + 0.5 * x[..., 1]), 0.3 * x[..., 2] - 0.2 * x[..., 3]], axis=-1)
    w = np.full((n, size, size), 1.0 / (n * size * size))
    net = lbm.Network(n, size, precision="bf16")
    net.set_params(he_init(3))
    losses = []
    for it in range(80):
        net.forward(x)
        losses.append(net.backward(t, w))
        net.adam_step(2e-3)
    print("loss", losses[0], losses[-1])
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.3 * losses[0]
