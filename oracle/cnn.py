"""The 3D convolutional network of the learned ROM surrogate, in plain FP64: forward pass, the
backward pass written out from the chain rule, the mean-squared-error loss and Adam.

Oracle code (test infrastructure): NumPy loops over the 27 taps of each 3 x 3 x 3 kernel, no
fusion.  The network maps a subdomain's sound speed on its (n+1)^3 nodes to a vector of
normalised S-fraction coefficients:

    x -> [conv 3^3, stride 2, zero pad 1, + bias, ReLU] x 4 -> flatten -> dense (+ bias) -> y

Layouts shared with the device implementation (the parameter vector is exchanged as one flat
array):
  * activations are channels-last, [batch][z][y][x][channel]; the input has one channel;
  * conv weights W[co][t][ci] with tap t = 9 dz + 3 dy + dx (dz, dy, dx in 0..2), then bias[co];
  * the dense layer sees the last activation flattened in its [z][y][x][channel] order,
    weights Wd[j][i] then bias bd[j];
  * the flat parameter vector is W1, b1, W2, b2, W3, b3, W4, b4, Wd, bd.
Output size of a stride-2, pad-1, size-3 convolution: (n_in - 1) // 2 + 1.

``quant`` (default identity) is applied to both operands of every product (activations, weights
and incoming gradients) so that a device implementation with rounded operands can be compared
in the same precision; the sums stay FP64.
"""
from __future__ import annotations

from typing import Callable, Dict, List, Tuple

import numpy as np

Quant = Callable[[np.ndarray], np.ndarray]


def _identity(a: np.ndarray) -> np.ndarray:
    return a


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (round to nearest, ties to even) and return as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def out_size(n: int) -> int:
    return (n - 1) // 2 + 1


def shapes(n_in: int, channels: int, n_out: int, n_conv: int = 4) -> List[Tuple[str, Tuple[int, ...]]]:
    """Names and shapes of the parameters in flat order."""
    out = []
    ci, n = 1, n_in
    for l in range(n_conv):
        out.append((f"W{l + 1}", (channels, 27, ci)))
        out.append((f"b{l + 1}", (channels,)))
        ci, n = channels, out_size(n)
    out.append(("Wd", (n_out, n * n * n * channels)))
    out.append(("bd", (n_out,)))
    return out


def unflatten(flat: np.ndarray, n_in: int, channels: int, n_out: int) -> Dict[str, np.ndarray]:
    params, o = {}, 0
    for name, shp in shapes(n_in, channels, n_out):
        size = int(np.prod(shp))
        params[name] = np.asarray(flat[o:o + size], dtype=np.float64).reshape(shp)
        o += size
    assert o == flat.size
    return params


def flatten(params: Dict[str, np.ndarray], n_in: int, channels: int, n_out: int) -> np.ndarray:
    return np.concatenate([params[name].ravel() for name, _ in shapes(n_in, channels, n_out)])


def _taps():
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                yield 9 * dz + 3 * dy + dx, dz, dy, dx


def conv_forward(x: np.ndarray, W: np.ndarray, b: np.ndarray, q: Quant = _identity) -> np.ndarray:
    """x [B][n][n][n][Ci] -> pre-activation [B][m][m][m][Co], m = out_size(n)."""
    B, n = x.shape[0], x.shape[1]
    m = out_size(n)
    xp = np.pad(q(x), ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    Wq = q(W)
    out = np.zeros((B, m, m, m, W.shape[0]))
    for t, dz, dy, dx in _taps():
        xs = xp[:, dz:dz + 2 * m:2, dy:dy + 2 * m:2, dx:dx + 2 * m:2, :]
        out += np.einsum("bzyxc,oc->bzyxo", xs, Wq[:, t, :])
    return out + b


def conv_backward(x: np.ndarray, W: np.ndarray, dpre: np.ndarray, q: Quant = _identity):
    """Gradients of sum(dpre * conv_forward(x, W, b)) with respect to x, W and b."""
    B, n = x.shape[0], x.shape[1]
    m = dpre.shape[1]
    xp = np.pad(q(x), ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    Wq, dq = q(W), q(dpre)
    dW = np.zeros_like(W, dtype=np.float64)
    dxp = np.zeros(xp.shape)
    for t, dz, dy, dx in _taps():
        sl = (slice(None), slice(dz, dz + 2 * m, 2), slice(dy, dy + 2 * m, 2), slice(dx, dx + 2 * m, 2), slice(None))
        dW[:, t, :] = np.einsum("bzyxo,bzyxc->oc", dq, xp[sl])
        dxp[sl] += np.einsum("bzyxo,oc->bzyxc", dq, Wq[:, t, :])
    db = dpre.sum(axis=(0, 1, 2, 3))
    return dxp[:, 1:n + 1, 1:n + 1, 1:n + 1, :], dW, db


def forward(params: Dict[str, np.ndarray], x: np.ndarray, q: Quant = _identity):
    """x [B][n][n][n] (one channel) -> (y [B][n_out], cache)."""
    a = np.asarray(x, dtype=np.float64)[..., None]
    acts = [a]
    l = 1
    while f"W{l}" in params:
        a = np.maximum(conv_forward(a, params[f"W{l}"], params[f"b{l}"], q), 0.0)
        acts.append(a)
        l += 1
    feat = a.reshape(a.shape[0], -1)
    y = q(feat) @ q(params["Wd"]).T + params["bd"]
    return y, acts


def _backward(params: Dict[str, np.ndarray], acts, dy: np.ndarray, q: Quant):
    grads = {}
    a = acts[-1]
    feat = a.reshape(a.shape[0], -1)
    grads["Wd"] = q(dy).T @ q(feat)
    grads["bd"] = dy.sum(axis=0)
    da = (q(dy) @ q(params["Wd"])).reshape(a.shape)
    L = len(acts) - 1
    for l in range(L, 0, -1):
        dpre = da * (acts[l] > 0)                       # ReLU: the output is positive where the input was
        dx, grads[f"W{l}"], grads[f"b{l}"] = conv_backward(acts[l - 1], params[f"W{l}"], dpre, q)
        da = dx
    return grads, da[..., 0]


def backward(params: Dict[str, np.ndarray], acts, dy: np.ndarray, q: Quant = _identity) -> Dict[str, np.ndarray]:
    """Parameter gradients of sum(dy * y) for the forward pass that produced ``acts``."""
    return _backward(params, acts, dy, q)[0]


def input_gradient(params: Dict[str, np.ndarray], acts, dy: np.ndarray, q: Quant = _identity) -> np.ndarray:
    """Gradient of sum(dy * y) with respect to the input x [B][n][n][n] of that forward pass."""
    return _backward(params, acts, dy, q)[1]


def mse(y: np.ndarray, target: np.ndarray) -> Tuple[float, np.ndarray]:
    """Mean over all entries of (y - target)^2 and its gradient with respect to y."""
    r = np.asarray(y, dtype=np.float64) - target
    return float(np.mean(r * r)), 2.0 * r / r.size


def adam(params: Dict[str, np.ndarray], grads: Dict[str, np.ndarray], state: Dict[str, np.ndarray], step: int,
         lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    """One Adam update (Kingma and Ba, bias-corrected moments), in place; step counts from 1."""
    for name, g in grads.items():
        m = state.setdefault("m_" + name, np.zeros_like(g))
        v = state.setdefault("v_" + name, np.zeros_like(g))
        m *= beta1
        m += (1 - beta1) * g
        v *= beta2
        v += (1 - beta2) * g * g
        mh = m / (1 - beta1 ** step)
        vh = v / (1 - beta2 ** step)
        params[name] -= lr * mh / (np.sqrt(vh) + eps)
