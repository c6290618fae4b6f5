"""GPU parity of the surrogate network's bf16 matrix-core kernels against the FP64 oracle network.

The device rounds both operands of every product to bfloat16 and accumulates in FP32.  The
oracle is run twice on the same inputs and parameters: exactly (FP64), and with its product
operands rounded to bfloat16 at the same places (``oracle.cnn.bf16``, sums in FP64).  delta, the
distance between the two oracle runs, is the effect of the operand precision itself; the device
must sit within a tenth of delta of the rounded oracle (what is left is FP32 accumulation order
and the rare operand that rounds to the other bfloat16 neighbour) and within 2 delta of the exact
one.  Sizes are ragged: 17^3 inputs (17 -> 9 -> 5 -> 3 -> 2 nodes), 8 channels, 37 outputs,
batch 3, so no product dimension is a multiple of its 64 x 64 x 16 tile.
"""
import numpy as np
import pytest

from oracle import cnn
from tests.cases import rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N_IN, CH, N_OUT, B = 17, 8, 37, 3


def _setup(seed=0):
    from paper_1406_6923_amd import sfm
    net = sfm.Cnn(N_IN, CH, N_OUT, max_batch=8, seed=seed)
    rng = np.random.default_rng(seed)
    flat = (rng.standard_normal(net.n_params) * 0.2).astype(np.float32)
    net.set_params(flat)
    x = rng.standard_normal((B, N_IN, N_IN, N_IN)).astype(np.float32)
    params = cnn.unflatten(flat.astype(np.float64), N_IN, CH, N_OUT)
    return net, flat, params, x


def _compare(got, ref_q, ref_x, what):
    delta = rel_l2(ref_q, ref_x)
    e_q, e_x = rel_l2(got, ref_q), rel_l2(got, ref_x)
    print(f"{what}: device vs bf16-operand oracle {e_q:.2e}, vs exact oracle {e_x:.2e}, delta {delta:.2e}")
    # the dense bias gradient is a plain FP32 sum of dy (no rounded operand): delta = 0, FP32 bar
    assert e_q < max(0.1 * delta, 1e-5), (what, e_q, delta)
    assert e_x < max(2.0 * delta, 1e-5), (what, e_x, delta)


def test_cnn_forward_matches_oracle():
    print("[case] cnn forward 17^3 x 8 channels -> 37", flush=True)
    net, flat, params, x = _setup()
    assert net.nodes == [17, 9, 5, 3, 2] and net.features == 8 * 8
    x_d = torch.from_numpy(x).cuda()
    y_d = torch.empty((B, N_OUT), dtype=torch.float32, device="cuda")
    net.forward(x_d, y_d)
    torch.cuda.synchronize()
    ref_x, _ = cnn.forward(params, x)
    ref_q, _ = cnn.forward(params, x, q=cnn.bf16)
    _compare(y_d.cpu().numpy(), ref_q, ref_x, "forward")
    net.close()


def test_cnn_backward_matches_oracle():
    print("[case] cnn backward", flush=True)
    net, flat, params, x = _setup(seed=1)
    rng = np.random.default_rng(9)
    dy = rng.standard_normal((B, N_OUT)).astype(np.float32)
    x_d = torch.from_numpy(x).cuda()
    net.forward(x_d)
    g_d = torch.zeros(net.n_params, dtype=torch.float32, device="cuda")
    net.backward(torch.from_numpy(dy).cuda(), g_d)
    torch.cuda.synchronize()
    got = cnn.unflatten(g_d.cpu().numpy().astype(np.float64), N_IN, CH, N_OUT)
    _, acts_x = cnn.forward(params, x)
    _, acts_q = cnn.forward(params, x, q=cnn.bf16)
    gx = cnn.backward(params, acts_x, dy.astype(np.float64))
    gq = cnn.backward(params, acts_q, dy.astype(np.float64), q=cnn.bf16)
    for name in gx:
        _compare(got[name], gq[name], gx[name], f"gradient {name}")
    net.close()


def test_cnn_training_step_and_loss_decrease():
    """One Adam step on a full batch against the oracle's step, then loss decreasing over training."""
    print("[case] cnn training", flush=True)
    from paper_1406_6923_amd import sfm
    net, flat, params, x = _setup(seed=2)
    rng = np.random.default_rng(3)
    target = rng.standard_normal((B, N_OUT)).astype(np.float32)
    x_d, t_d = torch.from_numpy(x).cuda(), torch.from_numpy(target).cuda()
    lr = 1e-3
    net.train(x_d, t_d, batch=B, epochs=1, lr=lr, seed=0)
    step = net.get_params().astype(np.float64) - flat
    y, acts = cnn.forward(params, x, q=cnn.bf16)
    loss, dy = cnn.mse(y, target)
    grads = cnn.backward(params, acts, dy, q=cnn.bf16)
    ref = {k: v.copy() for k, v in params.items()}
    cnn.adam(ref, grads, {}, step=1, lr=lr)
    ref_step = cnn.flatten(ref, N_IN, CH, N_OUT) - flat
    # the first Adam step is lr sign(g) wherever |g| >> eps: compare the signs that are decided
    g_flat = cnn.flatten(grads, N_IN, CH, N_OUT)
    big = np.abs(g_flat) > 1e-3 * np.abs(g_flat).max()
    agree = np.mean(np.sign(step[big]) == np.sign(ref_step[big]))
    print(f"first Adam step: {agree * 100:.2f}% of {big.sum()} decided signs agree, "
          f"rel-L2 {rel_l2(step, ref_step):.2e}")
    assert agree > 0.99
    assert rel_l2(step, ref_step) < 0.1
    # a learnable map: targets = a fixed random linear function of the input means per octant
    n = 64
    xs = rng.standard_normal((n, N_IN, N_IN, N_IN)).astype(np.float32)
    feats = np.stack([xs[:, :9, :9, :9].mean((1, 2, 3)), xs[:, 8:, 8:, 8:].mean((1, 2, 3))], 1)
    ts = (feats @ rng.standard_normal((2, N_OUT)) * 5).astype(np.float32)
    net2 = sfm.Cnn(N_IN, CH, N_OUT, max_batch=8, seed=5)
    losses = net2.train(torch.from_numpy(xs).cuda(), torch.from_numpy(ts).cuda(), batch=8, epochs=30, lr=3e-3, seed=1)
    print(f"training loss {losses[0]:.3e} -> {losses[-1]:.3e} over {len(losses)} epochs")
    assert np.isfinite(losses).all() and losses[-1] < 0.5 * losses[0]
    net.close()
    net2.close()


def test_cnn_errors():
    from paper_1406_6923_amd import sfm
    with pytest.raises(sfm.SfmError) as ei:
        sfm.Cnn(2, 8, 10, 4)
    assert ei.value.status == sfm.SFM_EINVAL
    net = sfm.Cnn(N_IN, CH, N_OUT, max_batch=2)
    with pytest.raises(sfm.SfmError) as ei:
        net.backward(torch.zeros((2, N_OUT), device="cuda"), torch.zeros(net.n_params, device="cuda"))
    assert ei.value.status == sfm.SFM_ESTATE
    with pytest.raises(sfm.SfmError) as ei:
        net.input_grad(torch.zeros((2, N_OUT), device="cuda"), torch.zeros((2, N_IN, N_IN, N_IN), device="cuda"))
    assert ei.value.status == sfm.SFM_ESTATE
    with pytest.raises(sfm.SfmError) as ei:
        net.forward(torch.zeros((3, N_IN, N_IN, N_IN), device="cuda"))
    assert ei.value.status == sfm.SFM_EINVAL
    net.forward(torch.zeros((2, N_IN, N_IN, N_IN), device="cuda"))
    with pytest.raises(sfm.SfmError) as ei:
        net.input_grad(torch.zeros((2, N_OUT), device="cuda"), None)
    assert ei.value.status == sfm.SFM_EINVAL
    net.close()


def test_cnn_input_gradient_matches_oracle():
    print("[case] cnn input gradient, scaled outputs", flush=True)
    net, flat, params, x = _setup(seed=2)
    rng = np.random.default_rng(11)
    tgt = (rng.standard_normal((20, N_OUT)) * rng.uniform(0.1, 3.0, N_OUT) + rng.standard_normal(N_OUT))
    mean, sd = net.fit_scale(torch.from_numpy(tgt.astype(np.float32)).cuda())
    dy = rng.standard_normal((B, N_OUT)).astype(np.float32)
    net.forward(torch.from_numpy(x).cuda())
    dx_d = torch.zeros((B, N_IN, N_IN, N_IN), dtype=torch.float32, device="cuda")
    net.input_grad(torch.from_numpy(dy).cuda(), dx_d)
    torch.cuda.synchronize()
    dye = dy.astype(np.float64) * sd.astype(np.float64)       # gradient carried to the unscaled output
    _, acts_x = cnn.forward(params, x)
    _, acts_q = cnn.forward(params, x, q=cnn.bf16)
    _compare(dx_d.cpu().numpy(), cnn.input_gradient(params, acts_q, dye, q=cnn.bf16),
             cnn.input_gradient(params, acts_x, dye), "input gradient")
    net.close()
