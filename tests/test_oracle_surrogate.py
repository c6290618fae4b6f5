"""Pins of the sound-speed gradient through the surrogate (oracle, CPU, FP64).

* the whole chain (box inputs, network, output scale, triangle-to-block map, Gamma-hat_1 held
  out, shared nodes of neighbouring boxes, the 1 / c of the log input) against central
  differences of the block functional J(c) = sum <dJ/dGamma, Gamma(c)> + <dJ/dGamma-hat,
  Gamma-hat(c)> along random directions, on 2 x 2 x 2 boxes of 8^3 cells;
* the output gradient on one off-diagonal entry against its definition (both mirror entries);
* a node inside one box receives only that box's input gradient, a cut-plane corner all eight.
"""
import numpy as np

from oracle import cnn, surrogate

K, P, N = 2, 6, 8          # levels, block size, cells per box edge


def _setup(seed=0):
    rng = np.random.default_rng(seed)
    n_in, ch = N + 1, 3
    n_out = 2 * K * P * (P + 1) // 2
    flat = rng.standard_normal(sum(int(np.prod(s)) for _, s in cnn.shapes(n_in, ch, n_out))) * 0.3
    params = cnn.unflatten(flat, n_in, ch, n_out)
    c = 2000.0 + 1500.0 * rng.random((2 * N + 1, 2 * N + 1, 2 * N + 1))
    gg = rng.standard_normal((8, K, P, P))
    gh = rng.standard_normal((8, K, P, P))
    gg = gg + np.swapaxes(gg, -1, -2)
    mean = rng.standard_normal(n_out)
    sd = 0.5 + rng.random(n_out)
    return rng, params, c, gg, gh, mean, sd


def test_velocity_gradient_matches_central_differences():
    rng, params, c, gg, gh, mean, sd = _setup()
    g = surrogate.velocity_gradient(params, c, N, gg, gh, mean, sd)
    assert g.shape == c.shape
    for trial in range(4):
        v = rng.standard_normal(c.shape)
        eps = 1e-4                            # relative change 1e-4 / 2000 of c
        jp = surrogate.block_functional(params, c + eps * v, N, gg, gh, mean, sd, K, P)
        jm = surrogate.block_functional(params, c - eps * v, N, gg, gh, mean, sd, K, P)
        fd = (jp - jm) / (2 * eps)
        an = float(np.sum(g * v))
        assert abs(fd - an) <= 1e-6 * abs(fd), (trial, fd, an)


def test_output_gradient_definition():
    rng = np.random.default_rng(3)
    gg, gh = rng.standard_normal((K, P, P)), rng.standard_normal((K, P, P))
    d = surrogate.output_gradient(gg, gh)
    ntri = P * (P + 1) // 2
    iu = np.triu_indices(P)
    e = int(np.flatnonzero((iu[0] == 1) & (iu[1] == 4))[0])
    assert d[e] == gg[0][1, 4] + gg[0][4, 1]                  # Gamma_1 entry (1, 4) and (4, 1)
    e0 = int(np.flatnonzero((iu[0] == 2) & (iu[1] == 2))[0])
    assert d[ntri + e0] == gg[1][2, 2]                        # Gamma_2 diagonal
    assert not d[2 * ntri:3 * ntri].any()                    # Gamma-hat_1 held out
    assert d[3 * ntri + e] == gh[1][1, 4] + gh[1][4, 1]


def test_shared_nodes_collect_every_box():
    _, params, c, gg, gh, mean, sd = _setup(1)
    g = surrogate.velocity_gradient(params, c, N, gg, gh, mean, sd)
    x = surrogate.box_inputs(c, N)
    _, acts = surrogate.predict(params, x, mean, sd)
    dy = np.stack([sd * surrogate.output_gradient(gg[s], gh[s]) for s in range(8)])
    dx = cnn.input_gradient(params, acts, dy)
    assert np.isclose(g[3, 2, 5] * c[3, 2, 5], dx[0][3, 2, 5], rtol=1e-13)          # inside box 0
    corner = sum(dx[s][0 if s & 4 else N, 0 if s & 2 else N, 0 if s & 1 else N] for s in range(8))
    assert np.isclose(g[N, N, N] * c[N, N, N], corner, rtol=1e-12)                  # shared by all 8
