"""GPU parity of the discrete adjoint (misfit gradients with respect to the S-fraction blocks)
against the FP64 oracle adjoint, itself pinned by central differences (tests/test_oracle_adjoint.py).

The GPU forward and adjoint run in FP32 (states, coefficients) with FP64 gradient sums; the
oracle in FP64.  Both gradients are compared as one vector over all Gamma_j and over all
Gamma-hat_j (j >= 2) blocks: relative L2 below 1e-4.  The FP32 forward alone moves the traces
by ~1e-6 relative (tests/test_gpu_step.py), and the gradient is a sum of products of two FP32
state histories (forward and adjoint), so a correct FP32 implementation sits around 1e-5; a
wrong pairing, sign or index shows up at O(1).
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint
from tests.cases import oracle_case, rel_l2, rom_arrays

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _setup(name, nsteps):
    from paper_1406_6923_amd import sfm
    cfg, c, subs, roms, cs = oracle_case(name)
    gam, hat, src, rec = rom_arrays(cs)
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k)
    sfm.sfm_load_roms(h.ctx, gam, hat, cfg.sources(), src, cfg.receivers(), rec)
    dt = 0.9 * cs.cfl_dt()
    wav = W.ricker(cfg.f_peak, dt, nsteps)[:, None]
    traces, _ = adjoint.forward(cs, dt, wav)
    rng = np.random.default_rng(11)
    observed = 0.7 * traces + 0.05 * np.abs(traces).max() * rng.standard_normal(traces.shape)
    return h, cfg, cs, dt, wav, observed


def _gpu_gradient(h, cs, dt, wav, observed, L):
    from paper_1406_6923_amd import sfm
    nsteps = len(wav)
    wav_d = torch.tensor(wav, dtype=torch.float32, device="cuda")
    tr = torch.zeros((len(cs.receivers), nsteps), dtype=torch.float32, device="cuda")
    sfm.sfm_step(h.ctx, nsteps, dt, wav_d, tr)
    resid = tr - torch.tensor(observed, dtype=torch.float32, device="cuda")
    sfm.sfm_reset_state(h.ctx, dt)
    return sfm.sfm_adjoint_gradient(h.ctx, nsteps, dt, wav_d, resid.contiguous(), L)


@pytest.mark.parametrize("name, nsteps, L", [("small", 200, 64), ("ragged", 150, 40)])
def test_adjoint_gradient_matches_oracle(name, nsteps, L):
    print(f"[case] adjoint {name}: {nsteps} steps, checkpoints every {L}", flush=True)
    h, cfg, cs, dt, wav, observed = _setup(name, nsteps)
    g_gam, g_hat = _gpu_gradient(h, cs, dt, wav, observed, L)
    J, r_gam, r_hat = adjoint.gradient(cs, dt, wav, observed)
    e_gam = rel_l2(g_gam, r_gam)
    e_hat = rel_l2(g_hat[:, 1:], r_hat[:, 1:])
    print(f"{name}: gradient rel-L2 Gamma {e_gam:.2e}, Gamma-hat {e_hat:.2e}")
    assert not g_hat[:, 0].any()
    assert e_gam < 1e-4 and e_hat < 1e-4
    h.close()


def test_adjoint_checkpoint_interval_does_not_change_the_gradient():
    h, cfg, cs, dt, wav, observed = _setup("small", 160)
    a_gam, a_hat = _gpu_gradient(h, cs, dt, wav, observed, 160)     # one segment
    b_gam, b_hat = _gpu_gradient(h, cs, dt, wav, observed, 23)      # 7 segments, ragged last
    e = max(rel_l2(b_gam, a_gam), rel_l2(b_hat[:, 1:], a_hat[:, 1:]))
    print(f"checkpoint interval 160 vs 23: gradient rel-L2 {e:.2e}")
    assert e < 1e-5                  # the windows of FP32 partial sums are grouped differently
    h.close()


def test_adjoint_autograd_function():
    from paper_1406_6923_amd import sfm
    from paper_1406_6923_amd.autograd import RomTraces, rom_traces
    cfg, c, subs, roms, cs = oracle_case("small")
    gam, hat, src, rec = rom_arrays(cs)
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k)
    nsteps = 120
    dt = 0.9 * cs.cfl_dt()
    wav = W.ricker(cfg.f_peak, dt, nsteps)[:, None]
    model = RomTraces(h, cfg.sources(), src, cfg.receivers(), rec, dt,
                      torch.tensor(wav, dtype=torch.float32, device="cuda"), nsteps, checkpoint_every=50)
    traces_ref, _ = adjoint.forward(cs, dt, wav)
    observed = torch.tensor(0.8 * traces_ref, dtype=torch.float32, device="cuda")
    J, r_gam, r_hat = adjoint.gradient(cs, dt, wav, 0.8 * traces_ref)
    # blocks on the host, then on the device (gradients come back where the blocks live)
    for dev in ("cpu", "cuda"):
        g = torch.tensor(gam, requires_grad=True, device=dev)
        gh = torch.tensor(hat, requires_grad=True, device=dev)
        tr = rom_traces(g, gh, model)
        loss = 0.5 * ((tr - observed) ** 2).sum()
        loss.backward()
        assert g.grad.device == g.device and gh.grad.dtype == gh.dtype
        e = max(rel_l2(g.grad.cpu().numpy(), r_gam), rel_l2(gh.grad.cpu().numpy()[:, 1:], r_hat[:, 1:]))
        print(f"autograd ({dev} blocks): loss {loss.item():.6e} (oracle {J:.6e}), gradient rel-L2 {e:.2e}")
        assert abs(loss.item() - J) < 1e-4 * J
        assert e < 1e-4
    h.close()


def test_velocity_gradient_through_surrogate_autograd():
    """Sound speed -> network blocks -> traces -> misfit, differentiated by torch.autograd through
    the library's adjoint and the network's input gradient; reference: the oracle adjoint at the
    oracle network's blocks, then the oracle chain to the sound speed (bf16 operands as the device)."""
    from paper_1406_6923_amd import sfm
    from paper_1406_6923_amd.autograd import RomTraces, rom_traces, surrogate_blocks
    from oracle import cnn, surrogate
    print("[case] autograd: sound speed -> surrogate blocks -> traces, small case, 100 steps", flush=True)
    cfg, c, subs, roms, cs = oracle_case("small")
    gam, hat, src, rec = rom_arrays(cs)
    S, k, p, n = len(subs), cfg.k, cfg.p, cfg.sub_cells[0]
    ntri = p * (p + 1) // 2
    iu = np.triu_indices(p)
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k)
    sfm.sfm_load_roms(h.ctx, gam, hat, cfg.sources(), src, cfg.receivers(), rec)
    # a network whose prediction is a valid ROM: the subdomain average of the Lanczos blocks (SPD)
    # plus a small input-dependent part, through the output scale (one mean and sd per output,
    # shared by all subdomains): mean = the average triangles, sd = 1e-3 of each block's largest entry
    rng = np.random.default_rng(31)
    net = sfm.Cnn(n + 1, 8, 2 * k * ntri, max_batch=3, seed=9)
    flat = (rng.standard_normal(net.n_params) * 0.1).astype(np.float32)
    net.set_params(flat)
    gbar, hbar = gam.mean(axis=0), hat.mean(axis=0)
    t = np.concatenate([b[iu] for b in list(gbar) + list(hbar)])
    amp = np.concatenate([np.full(ntri, 1e-3 * np.abs(b).max()) for b in list(gbar) + list(hbar)])
    mean, sd = net.fit_scale(torch.from_numpy(np.stack([t + amp, t - amp]).astype(np.float32)).cuda())
    params = cnn.unflatten(flat.astype(np.float64), n + 1, 8, 2 * k * ntri)
    m64, s64 = mean.astype(np.float64), sd.astype(np.float64)
    y, _ = surrogate.predict(params, surrogate.box_inputs(c, n), m64, s64, q=cnn.bf16)
    pred = [surrogate.blocks_from_output(y[a], k, p) for a in range(S)]
    dg = [pg - gam[a] for a, (pg, _) in enumerate(pred)]
    dh = [ph - hat[a] for a, (_, ph) in enumerate(pred)]
    cs_p = adjoint.perturbed_system(cs, dg, dh, 1.0)      # Gamma-hat_1 stays the Lanczos one
    nsteps = 100
    dt = 0.8 * cs_p.cfl_dt()
    wav = W.ricker(cfg.f_peak, dt, nsteps)[:, None]
    traces_ref, _ = adjoint.forward(cs_p, dt, wav)
    observed = 0.8 * traces_ref
    model = RomTraces(h, cfg.sources(), src, cfg.receivers(), rec, dt,
                      torch.tensor(wav, dtype=torch.float32, device="cuda"), nsteps, checkpoint_every=40)
    vel = torch.tensor(c.astype(np.float32), device="cuda", requires_grad=True)
    g, gh = surrogate_blocks(vel, net, h)
    g.retain_grad()
    gh.retain_grad()
    loss = 0.5 * ((rom_traces(g, gh, model) - torch.tensor(observed, dtype=torch.float32, device="cuda")) ** 2).sum()
    loss.backward()
    got = vel.grad.cpu().numpy()
    # the network's blocks
    ref_g = np.stack([pg for pg, _ in pred])
    ref_h = np.stack([ph for _, ph in pred])
    ref_h[:, 0] = hat[:, 0]
    assert rel_l2(g.detach().numpy(), ref_g) < 1e-6 and rel_l2(gh.detach().numpy(), ref_h) < 1e-6
    # the block gradients: the oracle adjoint at the network's blocks (FP32 adjoint bar)
    J, r_gam, r_hat = adjoint.gradient(cs_p, dt, wav, observed)
    d_gam, d_hat = g.grad.numpy(), gh.grad.numpy()
    e_blk = max(rel_l2(d_gam, r_gam), rel_l2(d_hat[:, 1:], r_hat[:, 1:]))
    # the chain to the sound speed: the oracle chain fed the device's own block gradients (bf16
    # operands as the device: within a tenth of the bf16 effect), and end to end from the oracle's
    # block gradients.  bf16 rounding is discontinuous: block gradients that differ at the FP32
    # adjoint's 1e-6 level round some small dy entries to the other neighbour, which moves the
    # bf16 chain by up to a few 1e-3 (the exact chain moves by 1e-5), so the end-to-end bar is the
    # bf16 effect itself.
    chain_q = surrogate.velocity_gradient(params, c, n, d_gam, d_hat, m64, s64, q=cnn.bf16)
    chain_x = surrogate.velocity_gradient(params, c, n, d_gam, d_hat, m64, s64)
    delta = rel_l2(chain_q, chain_x)
    e_chain = rel_l2(got, chain_q)
    ref_x = surrogate.velocity_gradient(params, c, n, r_gam, r_hat, m64, s64)
    e_end = rel_l2(got, ref_x)
    print(f"autograd through the surrogate: loss {loss.item():.6e} (oracle {J:.6e}); block gradients rel-L2 "
          f"{e_blk:.2e}; sound-speed gradient vs the oracle chain on the device's block gradients {e_chain:.2e} "
          f"(bf16 effect {delta:.2e}), end to end vs the exact oracle {e_end:.2e}")
    assert abs(loss.item() - J) < 1e-4 * J
    assert np.isfinite(got).all()
    assert e_blk < 1e-4
    assert e_chain < max(0.1 * delta, 1e-5), (e_chain, delta)
    assert e_end < 2.0 * delta, (e_end, delta)
    net.close()
    h.close()


def test_adjoint_errors():
    from paper_1406_6923_amd import sfm
    cfg, c, subs, roms, cs = oracle_case("small")
    gam, hat, src, rec = rom_arrays(cs)
    g = torch.zeros((len(cs.receivers), 10), device="cuda")
    w = torch.zeros((10, 1), device="cuda")
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k)
    with pytest.raises(sfm.SfmError) as ei:
        sfm.sfm_adjoint_gradient(h.ctx, 10, 1e-3, w, g)
    assert ei.value.status == sfm.SFM_ESTATE
    sfm.sfm_load_roms(h.ctx, gam, hat, cfg.sources(), src, None, None)
    with pytest.raises(sfm.SfmError) as ei:            # no receivers: no misfit
        sfm.sfm_adjoint_gradient(h.ctx, 10, 1e-3, w, g)
    assert ei.value.status == sfm.SFM_EINVAL
    sfm.sfm_load_roms(h.ctx, gam, hat, cfg.sources(), src, cfg.receivers(), rec)
    with pytest.raises(sfm.SfmError) as ei:
        sfm.sfm_adjoint_gradient(h.ctx, 10, 1e-3, w, g, checkpoint_every=0)
    assert ei.value.status == sfm.SFM_EINVAL
    h.close()
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k, precision=sfm.SFM_PREC_BF16_FP32ACC)
    sfm.sfm_load_roms(h.ctx, gam, hat, cfg.sources(), src, cfg.receivers(), rec)
    with pytest.raises(sfm.SfmError) as ei:
        sfm.sfm_adjoint_gradient(h.ctx, 10, 1e-3, w, g)
    assert ei.value.status == sfm.SFM_EINVAL
    h.close()
