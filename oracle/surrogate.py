"""The sound-speed gradient through the learned ROM surrogate, in plain FP64.

Oracle code (test infrastructure): the chain rule written out step by step, no fusion.

The network (``oracle.cnn``) reads log(c / 3000 m/s) on a subdomain box's (n+1)^3 nodes, [z][y][x],
and predicts the upper triangles (row-major, i <= l) of Gamma_1..Gamma_k, then
Gamma-hat_1..Gamma-hat_k, each as mean + sd * (network output).  Gamma-hat_1 (the face masses)
comes from block Lanczos, never from the network.  Boxes are equal cubes of n cells, numbered with
x fastest; box b along an axis holds nodes b n .. (b + 1) n, so nodes on a cut plane belong to two
boxes per axis.

For a misfit J that depends on the blocks, with gradients dJ/dGamma_j and dJ/dGamma-hat_j (p x p,
every entry taken as independent; the symmetric parts that the adjoint returns serve as well), the
gradient with respect to the sound speed when the blocks are the network's prediction is

    dJ/dc(node) = (1 / c(node)) sum over boxes s holding the node of dJ/dx_s(local node),
    dJ/dx_s     = input gradient of the network for dJ/dy_s,
    dJ/dy_s     = sd * dJ/du_s,   u = a block's upper triangle:
                  dJ/du_(i,i) = dJ/dB[i][i],  dJ/du_(i,l) = dJ/dB[i][l] + dJ/dB[l][i]  (i < l),
                  and zero on the triangle of Gamma-hat_1.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

from . import cnn


def box_grid(c: np.ndarray, n: int) -> Tuple[int, int, int]:
    """Boxes per axis (x, y, z) of a node field c [nz+1][ny+1][nx+1] cut into cubes of n cells."""
    nz, ny, nx = (d - 1 for d in c.shape)
    assert nx % n == 0 and ny % n == 0 and nz % n == 0
    return nx // n, ny // n, nz // n


def box_inputs(c: np.ndarray, n: int) -> np.ndarray:
    """Network inputs log(c / 3000) of every box: [S][n+1][n+1][n+1]."""
    bx, by, bz = box_grid(c, n)
    out = []
    for s in range(bx * by * bz):
        ix, iy, iz = s % bx, (s // bx) % by, s // (bx * by)
        box = c[iz * n:iz * n + n + 1, iy * n:iy * n + n + 1, ix * n:ix * n + n + 1]
        out.append(np.log(np.asarray(box, dtype=np.float64) / 3000.0))
    return np.stack(out)


def blocks_from_output(y: np.ndarray, k: int, p: int) -> Tuple[np.ndarray, np.ndarray]:
    """Symmetric blocks (gamma [k][p][p], gamma_hat [k][p][p]) from one prediction vector y."""
    iu = np.triu_indices(p)
    ntri = len(iu[0])
    assert y.size == 2 * k * ntri
    blocks = np.zeros((2 * k, p, p))
    for b in range(2 * k):
        blocks[b][iu] = y[b * ntri:(b + 1) * ntri]
        blocks[b].T[iu] = y[b * ntri:(b + 1) * ntri]
    return blocks[:k], blocks[k:]


def output_gradient(gg: np.ndarray, gh: np.ndarray) -> np.ndarray:
    """dJ/du over the prediction vector of one box from block gradients gg, gh [k][p][p]."""
    k, p = gg.shape[0], gg.shape[1]
    iu = np.triu_indices(p)
    diag = iu[0] == iu[1]
    parts = []
    for b in range(2 * k):
        G = gg[b] if b < k else gh[b - k]
        d = G[iu] + G.T[iu]
        d[diag] = G[iu][diag]
        if b == k:
            d = np.zeros_like(d)                 # Gamma-hat_1: from Lanczos
        parts.append(d)
    return np.concatenate(parts)


def predict(params: Dict[str, np.ndarray], x: np.ndarray, mean: np.ndarray, sd: np.ndarray,
            q: cnn.Quant = cnn._identity):
    """Scaled predictions mean + sd * net(x) of boxes x [S][n+1]^3 and the forward cache."""
    y, acts = cnn.forward(params, x, q)
    return mean + sd * y, acts


def velocity_gradient(params: Dict[str, np.ndarray], c: np.ndarray, n: int, gg: np.ndarray, gh: np.ndarray,
                      mean: np.ndarray, sd: np.ndarray, q: cnn.Quant = cnn._identity) -> np.ndarray:
    """dJ/dc on the nodes of c for block gradients gg, gh [S][k][p][p]."""
    x = box_inputs(c, n)
    _, acts = predict(params, x, mean, sd, q)
    dy = np.stack([sd * output_gradient(gg[s], gh[s]) for s in range(x.shape[0])])
    dx = cnn.input_gradient(params, acts, dy, q)                  # [S][n+1]^3
    bx, by, _ = box_grid(c, n)
    out = np.zeros(c.shape)
    for s in range(x.shape[0]):
        ix, iy, iz = s % bx, (s // bx) % by, s // (bx * by)
        out[iz * n:iz * n + n + 1, iy * n:iy * n + n + 1, ix * n:ix * n + n + 1] += dx[s]
    return out / c


def block_functional(params: Dict[str, np.ndarray], c: np.ndarray, n: int, gg: np.ndarray, gh: np.ndarray,
                     mean: np.ndarray, sd: np.ndarray, k: int, p: int, q: cnn.Quant = cnn._identity) -> float:
    """J(c) = sum over boxes and levels of <gg, Gamma_j> + <gh, Gamma-hat_j> (j >= 2) with the
    blocks predicted from c: a linear functional whose c-gradient is velocity_gradient's."""
    y, _ = predict(params, box_inputs(c, n), mean, sd, q)
    J = 0.0
    for s in range(y.shape[0]):
        gam, hat = blocks_from_output(y[s], k, p)
        J += float(np.sum(gg[s] * gam)) + float(np.sum(gh[s, 1:] * hat[1:]))
    return J
