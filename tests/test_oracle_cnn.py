"""Pins of the surrogate network's oracle (CPU, FP64) against library routines and calculus.

* one convolution layer against scipy.signal.correlate (stride taken by subsampling, zero pad);
* every parameter gradient of the backward pass against central differences of the forward
  pass on a small network (4 stride-2 layers from 9^3 nodes);
* the MSE gradient against central differences;
* Adam's first step against its closed form -lr g / (|g| + eps);
* bfloat16 rounding against torch's conversion, and its ties-to-even cases.
"""
import numpy as np
import pytest
import scipy.signal

from oracle import cnn


def _random_params(n_in, ch, n_out, seed):
    rng = np.random.default_rng(seed)
    flat = rng.standard_normal(sum(int(np.prod(s)) for _, s in cnn.shapes(n_in, ch, n_out))) * 0.3
    return cnn.unflatten(flat, n_in, ch, n_out)


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    B, n, ci, co = 2, 7, 3, 4
    x = rng.standard_normal((B, n, n, n, ci))
    W = rng.standard_normal((co, 27, ci))
    b = rng.standard_normal(co)
    got = cnn.conv_forward(x, W, b)
    m = cnn.out_size(n)
    assert got.shape == (B, m, m, m, co)
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    for bb in range(B):
        for o in range(co):
            acc = np.zeros((n, n, n))
            for c in range(ci):
                acc += scipy.signal.correlate(xp[bb, :, :, :, c], W[o, :, c].reshape(3, 3, 3), mode="valid")
            np.testing.assert_allclose(got[bb, :, :, :, o], acc[::2, ::2, ::2] + b[o], rtol=1e-12, atol=1e-12)


def test_backward_matches_central_differences():
    n_in, ch, n_out = 9, 3, 5
    params = _random_params(n_in, ch, n_out, seed=1)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, n_in, n_in, n_in))
    dy = rng.standard_normal((2, n_out))
    y, acts = cnn.forward(params, x)
    grads = cnn.backward(params, acts, dy)
    eps = 1e-6
    worst = 0.0
    for name, g in grads.items():
        flat = params[name].reshape(-1)
        idx = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + eps
            jp = float(np.sum(dy * cnn.forward(params, x)[0]))
            flat[i] = old - eps
            jm = float(np.sum(dy * cnn.forward(params, x)[0]))
            flat[i] = old
            fd = (jp - jm) / (2 * eps)
            err = abs(fd - g.reshape(-1)[i]) / max(1e-8, abs(fd))
            worst = max(worst, err)
            assert abs(fd - g.reshape(-1)[i]) <= 1e-6 * max(1.0, abs(fd)), (name, i, fd, g.reshape(-1)[i])
    print(f"network gradient vs central differences: worst relative difference {worst:.1e}")


def test_mse_gradient():
    rng = np.random.default_rng(3)
    y, t = rng.standard_normal((3, 4)), rng.standard_normal((3, 4))
    loss, g = cnn.mse(y, t)
    eps = 1e-7
    for i in range(y.size):
        yp = y.copy().reshape(-1)
        yp[i] += eps
        ym = y.copy().reshape(-1)
        ym[i] -= eps
        fd = (cnn.mse(yp.reshape(y.shape), t)[0] - cnn.mse(ym.reshape(y.shape), t)[0]) / (2 * eps)
        assert abs(fd - g.reshape(-1)[i]) < 1e-7


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    p = {"w": rng.standard_normal(10)}
    g = {"w": rng.standard_normal(10)}
    w0 = p["w"].copy()
    cnn.adam(p, g, {}, step=1, lr=1e-3, eps=1e-8)
    np.testing.assert_allclose(p["w"], w0 - 1e-3 * g["w"] / (np.abs(g["w"]) + 1e-8), rtol=1e-12)


def test_bf16_rounding():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = rng.standard_normal(10000) * 10.0 ** rng.uniform(-5, 5, 10000)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16(x), ref)
    assert cnn.bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0               # tie -> even (down)
    assert cnn.bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6  # tie -> even (up)


def test_input_gradient_matches_central_differences():
    n_in, ch, n_out = 9, 3, 5
    params = _random_params(n_in, ch, n_out, seed=6)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((2, n_in, n_in, n_in))
    dy = rng.standard_normal((2, n_out))
    _, acts = cnn.forward(params, x)
    g = cnn.input_gradient(params, acts, dy)
    assert g.shape == x.shape
    eps = 1e-6
    for i in rng.choice(x.size, size=12, replace=False):
        xp, xm = x.copy().reshape(-1), x.copy().reshape(-1)
        xp[i] += eps
        xm[i] -= eps
        fd = (np.sum(dy * cnn.forward(params, xp.reshape(x.shape))[0])
              - np.sum(dy * cnn.forward(params, xm.reshape(x.shape))[0])) / (2 * eps)
        assert abs(fd - g.reshape(-1)[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g.reshape(-1)[i])
