"""Learned ROMs with block Lanczos as judge and fallback, through the C ABI.

* network inputs (log c / 3000 m/s per subdomain box) and training targets (upper triangles of the
  S-fraction blocks) against the same quantities formed from the oracle's ROMs;
* the device NtD judge against the oracle's matrix S-fraction (``ntd_continued_fraction``) on
  perturbed coefficient sets: relative agreement 1e-6;
* the accept / fallback logic: with tol = inf every subdomain without sources or receivers takes
  the prediction (Gamma-hat_1 from Lanczos), with tol = 0 none does;
* a trained network on the 32^3 parity grid's split (16^3-cell boxes, m = 4, k = 8): trained on
  the ROMs of 400 subdomains of seeded layered / lognormal / blob media, applied to unseen media;
  every accepted subdomain's NtD error (re-evaluated by the oracle) is within tol, every rejected
  one keeps the exact Lanczos blocks, and the report states what the network achieved;
* the sound-speed gradient through the network against the oracle chain (``oracle.surrogate``)
  with the same bfloat16 operand rounding, on the 32^3 grid's 2 x 2 x 2 boxes in ragged batches.
"""
import numpy as np
import pytest

import workloads as W
from oracle import sfraction
from tests.cases import oracle_case, rom_arrays

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ctx(cfg, sub=None):
    from paper_1406_6923_amd import sfm
    return sfm.Sfm(cfg.ncell, cfg.sub_cells if sub is None else sub, cfg.h, cfg.m, cfg.k, precision=sfm.SFM_PREC_FP64)


def test_inputs_and_targets_match_oracle():
    from paper_1406_6923_amd import sfm
    print("[case] surrogate inputs and targets", flush=True)
    cfg, c, subs, roms, cs = oracle_case("small")
    gam, hat, src, rec = rom_arrays(cs)
    h = _ctx(cfg)
    sfm.sfm_load_roms(h.ctx, gam, hat, cfg.sources(), src, cfg.receivers(), rec)
    S, k, p = len(subs), cfg.k, cfg.p
    n = cfg.sub_cells[0] + 1
    x = torch.zeros((S, n ** 3), dtype=torch.float32, device="cuda")
    sfm.sfm_rom_inputs(h.ctx, torch.from_numpy(c.astype(np.float32)).cuda(), x)
    for a, sd in enumerate(subs):
        box = c[sd.origin[2]:sd.origin[2] + n, sd.origin[1]:sd.origin[1] + n, sd.origin[0]:sd.origin[0] + n]
        np.testing.assert_allclose(x[a].cpu().numpy(), np.log(box.astype(np.float32) / 3000.0).ravel(), rtol=0,
                                   atol=1e-6)
    ntri = p * (p + 1) // 2
    t = torch.zeros((S, 2 * k * ntri), dtype=torch.float32, device="cuda")
    sfm.sfm_rom_targets(h.ctx, t)
    iu = np.triu_indices(p)
    ref = np.stack([np.concatenate([g[iu] for g in list(gam[a]) + list(hat[a])]) for a in range(S)]).astype(np.float32)
    assert np.array_equal(t.cpu().numpy(), ref)
    h.close()


def test_ntd_judge_matches_oracle():
    from paper_1406_6923_amd import sfm
    print("[case] surrogate NtD judge", flush=True)
    cfg, c, subs, roms, cs = oracle_case("small")
    gam, hat, src, rec = rom_arrays(cs)
    h = _ctx(cfg)
    sfm.sfm_load_roms(h.ctx, gam, hat, cfg.sources(), src, cfg.receivers(), rec)
    rng = np.random.default_rng(4)
    for scale in (1e-6, 1e-3, 1e-1):
        pg = gam * (1 + scale * rng.standard_normal(gam.shape))
        ph = hat * (1 + scale * rng.standard_normal(hat.shape))
        pg = 0.5 * (pg + np.swapaxes(pg, -1, -2))
        ph = 0.5 * (ph + np.swapaxes(ph, -1, -2))
        coef = torch.from_numpy(np.stack([pg, ph], axis=1).copy()).cuda()
        got = sfm.sfm_ntd_error(h.ctx, coef, cfg.f_peak)
        ref = []
        for a in range(len(subs)):
            sa = sfraction.SFraction(gamma=list(pg[a]), gamma_hat=list(ph[a]), G=[])
            sb = sfraction.SFraction(gamma=list(gam[a]), gamma_hat=list(hat[a]), G=[])
            e = 0.0
            for s in sfraction.ntd_frequencies(cfg.f_peak):
                ma, mb = sfraction.ntd_continued_fraction(sa, s), sfraction.ntd_continued_fraction(sb, s)
                e = max(e, np.linalg.norm(ma - mb) / np.linalg.norm(mb))
            ref.append(e)
        ref = np.array(ref)
        print(f"perturbation {scale:.0e}: judge {got.max():.3e} vs oracle {ref.max():.3e}")
        np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-13)
    h.close()


def test_surrogate_accept_and_fallback():
    from paper_1406_6923_amd import sfm
    print("[case] surrogate accept / fallback", flush=True)
    cfg, c, subs, roms, cs = oracle_case("small")
    gam, hat, _, _ = rom_arrays(cs)
    S, k, p = len(subs), cfg.k, cfg.p
    n_out = 2 * k * p * (p + 1) // 2
    net = sfm.Cnn(cfg.sub_cells[0] + 1, 8, n_out, max_batch=4, seed=3)
    vel = torch.from_numpy(c.astype(np.float32)).cuda()
    for tol, expect_all in ((np.inf, True), (0.0, False)):
        h = _ctx(cfg)
        acc, err, secs = sfm.sfm_build_roms_surrogate(h.ctx, net, tol, cfg.f_peak, vel, cfg.sources(),
                                                      cfg.receivers())
        g2, h2 = sfm.sfm_export_roms(h.ctx)
        pinned = {cs.sources[0][0]} | {a for a, _ in cs.receivers}
        for a in range(S):
            assert acc[a] == (expect_all and a not in pinned)
            if acc[a]:
                assert np.abs(g2[a] - gam[a]).max() > 1e-3 * np.abs(gam[a]).max()     # a prediction
                np.testing.assert_allclose(h2[a, 0], hat[a, 0], rtol=1e-12, atol=0)      # exact face masses
            else:
                np.testing.assert_allclose(g2[a], gam[a], rtol=0, atol=1e-9 * np.abs(gam[a]).max())
        print(f"tol {tol}: accepted {acc.sum()} of {S} ({len(pinned)} pinned); seconds {np.round(secs, 4)}")
        h.close()
    net.close()


def test_trained_surrogate_on_unseen_media():
    from paper_1406_6923_amd import sfm
    cfg = W.CFG_SMALL
    k, p, n = cfg.k, cfg.p, cfg.sub_cells[0] + 1
    ntri = p * (p + 1) // 2
    # training set: 400 subdomains (10 x 10 x 4 boxes of 16^3 cells) of seeded media
    print("[case] surrogate training set: 400 subdomains", flush=True)
    train_cells = (160, 160, 64)
    ct = W.surrogate_velocity(tuple(x + 1 for x in train_cells), seed=21).astype(np.float32)
    ht = sfm.Sfm(train_cells, cfg.sub_cells, cfg.h, cfg.m, cfg.k, precision=sfm.SFM_PREC_FP64)
    vt = torch.from_numpy(ct).cuda()
    sfm.sfm_build_roms(ht.ctx, vt)
    St = sfm.sfm_query(ht.ctx)["n_subdomains"]
    xt = torch.zeros((St, n ** 3), dtype=torch.float32, device="cuda")
    tt = torch.zeros((St, 2 * k * ntri), dtype=torch.float32, device="cuda")
    sfm.sfm_rom_inputs(ht.ctx, vt, xt)
    sfm.sfm_rom_targets(ht.ctx, tt)
    ht.close()
    net = sfm.Cnn(n, 32, 2 * k * ntri, max_batch=16, seed=7)
    net.fit_scale(tt)
    print("[case] surrogate training: 40 epochs", flush=True)
    losses = net.train(xt, tt, batch=16, epochs=40, lr=1e-3, seed=2)
    print(f"training loss (normalised targets) {losses[0]:.3f} -> {losses[-1]:.3f}")
    assert np.isfinite(losses).all() and losses[-1] < losses[0]
    # unseen media on the 32^3 grid, judged at three tolerances
    c = W.surrogate_velocity(cfg.nodes, seed=99).astype(np.float32)
    vel = torch.from_numpy(c).cuda()
    for tol in (1e-3, 1e-2, 1e-1):
        print(f"[case] surrogate build, tol {tol}", flush=True)
        h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k, precision=sfm.SFM_PREC_FP64)
        acc, err, secs = sfm.sfm_build_roms_surrogate(h.ctx, net, tol, cfg.f_peak, vel)
        g2, h2 = sfm.sfm_export_roms(h.ctx)
        href = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k, precision=sfm.SFM_PREC_FP64)
        sfm.sfm_build_roms(href.ctx, vel)
        gr, hr = sfm.sfm_export_roms(href.ctx)
        for a in range(len(acc)):
            if acc[a]:
                sa = sfraction.SFraction(gamma=list(g2[a]), gamma_hat=list(h2[a]), G=[])
                sb = sfraction.SFraction(gamma=list(gr[a]), gamma_hat=list(hr[a]), G=[])
                e = max(np.linalg.norm(sfraction.ntd_continued_fraction(sa, s) - sfraction.ntd_continued_fraction(sb, s))
                        / np.linalg.norm(sfraction.ntd_continued_fraction(sb, s))
                        for s in sfraction.ntd_frequencies(cfg.f_peak))
                assert e <= tol * (1 + 1e-6), (a, e)
            else:
                np.testing.assert_allclose(g2[a], gr[a], rtol=0, atol=1e-9 * np.abs(gr[a]).max())
        print(f"tol {tol}: accepted {int(acc.sum())} of {len(acc)}, NtD errors of the predictions "
              f"min {err.min():.2e} median {np.median(err):.2e} max {err.max():.2e}; seconds {np.round(secs, 4)}")
        h.close()
        href.close()
    net.close()


def test_velocity_gradient_matches_oracle():
    from paper_1406_6923_amd import sfm
    from oracle import cnn, surrogate
    from tests.cases import rel_l2
    print("[case] sound-speed gradient through the surrogate, 32^3 grid, batches 3 + 3 + 2", flush=True)
    cfg = W.CFG_SMALL
    rng = np.random.default_rng(21)
    c = (cfg.velocity_model() * (1.0 + 0.05 * rng.standard_normal(tuple(n + 1 for n in cfg.ncell)[::-1])))
    c = c.astype(np.float32)
    S, k, p, n = 8, cfg.k, cfg.p, cfg.sub_cells[0]
    ntri = p * (p + 1) // 2
    h = _ctx(cfg)
    net = sfm.Cnn(n + 1, 8, 2 * k * ntri, max_batch=3, seed=5)
    flat = (rng.standard_normal(net.n_params) * 0.1).astype(np.float32)
    net.set_params(flat)
    tgt = rng.standard_normal((16, 2 * k * ntri)) * rng.uniform(0.1, 2.0, 2 * k * ntri)
    mean, sd = net.fit_scale(torch.from_numpy(tgt.astype(np.float32)).cuda())
    gg = rng.standard_normal((S, k, p, p))
    gh = rng.standard_normal((S, k, p, p))
    gg, gh = gg + np.swapaxes(gg, -1, -2), gh + np.swapaxes(gh, -1, -2)
    out = torch.zeros(c.shape, dtype=torch.float32, device="cuda")
    sfm.sfm_surrogate_velocity_gradient(h.ctx, net, torch.from_numpy(c).cuda(), gg, gh, out)
    got = out.cpu().numpy()
    params = cnn.unflatten(flat.astype(np.float64), n + 1, 8, 2 * k * ntri)
    c64, m64, s64 = c.astype(np.float64), mean.astype(np.float64), sd.astype(np.float64)
    ref_q = surrogate.velocity_gradient(params, c64, n, gg, gh, m64, s64, q=cnn.bf16)
    ref_x = surrogate.velocity_gradient(params, c64, n, gg, gh, m64, s64)
    delta = rel_l2(ref_q, ref_x)
    e_q, e_x = rel_l2(got, ref_q), rel_l2(got, ref_x)
    print(f"velocity gradient: device vs bf16-operand oracle {e_q:.2e}, vs exact oracle {e_x:.2e}, delta {delta:.2e}")
    assert np.isfinite(got).all()
    assert e_q < max(0.1 * delta, 1e-5) and e_x < max(2.0 * delta, 1e-5), (e_q, e_x, delta)
    net.close()
    h.close()


def test_velocity_gradient_and_predict_errors():
    from paper_1406_6923_amd import sfm
    print("[case] surrogate gradient / prediction argument errors", flush=True)
    cfg = W.CFG_SMALL
    S, k, p, n = 8, cfg.k, cfg.p, cfg.sub_cells[0]
    ntri = p * (p + 1) // 2
    h = _ctx(cfg)
    net = sfm.Cnn(n + 1, 4, 2 * k * ntri, max_batch=2, seed=1)
    vel = torch.full(tuple(c + 1 for c in cfg.ncell[::-1]), 2000.0, dtype=torch.float32, device="cuda")
    coef = torch.zeros((S, 2, k, p, p), dtype=torch.float64, device="cuda")
    with pytest.raises(sfm.SfmError) as ei:                 # Gamma-hat_1 needs ROMs
        sfm.sfm_surrogate_predict(h.ctx, net, vel, coef)
    assert ei.value.status == sfm.SFM_ESTATE
    g = np.zeros((S, k, p, p))
    out = torch.zeros_like(vel)
    with pytest.raises(ValueError):                         # block gradients of the wrong size
        sfm.sfm_surrogate_velocity_gradient(h.ctx, net, vel, g[:, :1], g, out)
    bad = sfm.Cnn(n + 3, 4, 2 * k * ntri, max_batch=2, seed=1)
    with pytest.raises(sfm.SfmError) as ei:                 # network input size
        sfm.sfm_surrogate_velocity_gradient(h.ctx, bad, vel, g, g, out)
    assert ei.value.status == sfm.SFM_EINVAL
    bad.close()
    bad = sfm.Cnn(n + 1, 4, 2 * k * ntri + 1, max_batch=2, seed=1)
    with pytest.raises(sfm.SfmError) as ei:                 # network output size
        sfm.sfm_surrogate_velocity_gradient(h.ctx, bad, vel, g, g, out)
    assert ei.value.status == sfm.SFM_EINVAL
    bad.close()
    with pytest.raises(sfm.SfmError) as ei:
        sfm.sfm_surrogate_velocity_gradient(h.ctx, net, vel, g, g, None)
    assert ei.value.status == sfm.SFM_EINVAL
    h.close()
    hu = _ctx(cfg, sub=((16, 16), (8, 24), (16, 16)))        # boxes that are not equal cubes
    gu = np.zeros((sfm.sfm_query(hu.ctx)["n_subdomains"], k, p, p))
    with pytest.raises(sfm.SfmError) as ei:
        sfm.sfm_surrogate_velocity_gradient(hu.ctx, net, vel, gu, gu, out)
    assert ei.value.status == sfm.SFM_EINVAL
    hu.close()
    net.close()
