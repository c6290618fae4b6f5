"""GPU parity with a ROM size of its own on every subdomain (Algorithm 1, Stage 1 run with k_s steps
on subdomain s, Stage 2 coupling ROMs of different sizes through the boundary layer alone).

The library is loaded with the k-level ROMs and told k_s per subdomain (sfm_set_levels); the
oracle builds each subdomain's ROM independently with k_s steps.  Agreement therefore checks the
kernels' level bounds and the reading that the first k_s levels of a k-level ROM are the k_s-level
ROM (pinned on the CPU in tests/test_oracle_pins.py).  Bars as for one size everywhere: one
operator application 1e-5 rel-L2 (FP32), traces 1e-5, gradients 1e-4; levels past k_s stay exactly
zero.
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, coupled
from tests.cases import mixed_level_case, oracle_case, pad_levels, rel_l2, rom_arrays

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NSHOT = 64


def _loaded(name):
    from paper_1406_6923_amd import sfm
    cfg, c, subs, roms, cs = oracle_case(name)
    cfg, subs, roms_ks, cs_ks, ks = mixed_level_case(name)
    gam, hat, src, rec = rom_arrays(cs)
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k)
    sfm.sfm_load_roms(h.ctx, gam, hat, cfg.sources(), src, cfg.receivers(), rec)
    sfm.sfm_set_levels(h.ctx, ks)
    assert np.array_equal(sfm.sfm_get_levels(h.ctx), ks)
    return h, cfg, cs_ks, ks


def _random_state(cs_ks, k, seed):
    rng = np.random.default_rng(seed)
    return pad_levels(cs_ks.scatter(rng.standard_normal(cs_ks._dof_layout()[1])), k)


def _check_levels(got, ref, ks, tol, what):
    for a, kk in enumerate(ks):
        assert not got[a, kk:].any(), (what, a, "levels past k_s must stay zero")
    err = rel_l2(got, ref)
    assert err < tol, (what, err)
    return err


@pytest.mark.parametrize("name", ["small", "ragged"])
def test_levels_operator_matches_oracle(name):
    from paper_1406_6923_amd import sfm
    print(f"[case] levels operator {name}", flush=True)
    h, cfg, cs_ks, ks = _loaded(name)
    U = _random_state(cs_ks, cfg.k, seed=12)
    ref = pad_levels(cs_ks.accel([U[a, :kk] for a, kk in enumerate(ks)]), cfg.k)
    # nonzero input past k_s must be ignored
    U_in = U.copy()
    for a, kk in enumerate(ks):
        U_in[a, kk:] = 1.0
    u_d = torch.tensor(U_in, dtype=torch.float32, device="cuda")
    a_d = torch.full_like(u_d, 7.0)
    sfm.sfm_apply_operator(h.ctx, u_d, a_d)
    torch.cuda.synchronize()
    err = _check_levels(a_d.cpu().numpy(), ref, ks, 1e-5, "operator")
    print(f"{name}: levels {ks.tolist()}, operator rel-L2 {err:.2e}")
    h.close()


@pytest.mark.parametrize("name, nsteps", [("small", 500), ("ragged", 300)])
def test_levels_traces_and_cfl_match_oracle(name, nsteps):
    from paper_1406_6923_amd import sfm
    print(f"[case] levels traces {name}, {nsteps} steps", flush=True)
    h, cfg, cs_ks, ks = _loaded(name)
    dt_ref = cs_ks.cfl_dt()
    dt_gpu = sfm.sfm_cfl_dt(h.ctx, iters=400)
    print(f"{name}: dt_max device {dt_gpu:.8e}, oracle {dt_ref:.8e} (ratio {dt_gpu / dt_ref:.6f})")
    assert dt_ref * (1 - 1e-3) <= dt_gpu <= dt_ref * (1 + 1e-6)     # certified: never above the limit
    dt = 0.9 * dt_ref
    wav = W.ricker(cfg.f_peak, dt, nsteps)[:, None]
    ref = cs_ks.run(dt, wav)
    tr_d = torch.zeros((len(cs_ks.receivers), nsteps), dtype=torch.float32, device="cuda")
    sfm.sfm_step(h.ctx, nsteps, dt, torch.tensor(wav, dtype=torch.float32, device="cuda"), tr_d)
    torch.cuda.synchronize()
    err = rel_l2(tr_d.cpu().numpy(), ref)
    print(f"{name}: dt_max GPU {dt_gpu:.4e} oracle {dt_ref:.4e}; traces rel-L2 {err:.2e}")
    assert err < 1e-5
    u, d, n = sfm.sfm_get_state(h.ctx)
    for a, kk in enumerate(ks):
        assert not u[a, kk:].any() and not d[a, kk:].any()
    # a full-size state restored with set_state loses its levels past k_s
    sfm.sfm_set_state(h.ctx, np.ones_like(u), np.ones_like(d), 0)
    u2, d2, _ = sfm.sfm_get_state(h.ctx)
    for a, kk in enumerate(ks):
        assert not u2[a, kk:].any() and (u2[a, :kk] == 1).all()
    h.close()


@pytest.mark.parametrize("name", ["small", "ragged"])
def test_levels_shots_operator_matches_oracle(name):
    from paper_1406_6923_amd import sfm
    print(f"[case] levels shots operator {name}, {NSHOT} shots", flush=True)
    h, cfg, cs_ks, ks = _loaded(name)
    sfm.sfm_shots_init(h.ctx, NSHOT, np.full(NSHOT, -1))
    U = np.stack([_random_state(cs_ks, cfg.k, seed=200 + n) for n in range(NSHOT)], axis=-1).astype(np.float32)
    U_in = U.copy()
    for a, kk in enumerate(ks):
        U_in[a, kk:] = 1.0
    sfm.sfm_shots_set_state(h.ctx, U_in, np.zeros_like(U))
    sfm.sfm_shots_step(h.ctx, 1, 1.0, torch.zeros((1, NSHOT), dtype=torch.float32, device="cuda"), None)
    u_out, a = sfm.sfm_shots_get_state(h.ctx, NSHOT)
    worst = 0.0
    for n in range(NSHOT):
        ref = pad_levels(cs_ks.accel([U[a_, :kk, :, n].astype(np.float64) for a_, kk in enumerate(ks)]), cfg.k)
        worst = max(worst, _check_levels(a[..., n], ref, ks, 1e-5, f"shot {n}"))
    for a_, kk in enumerate(ks):
        assert not u_out[a_, kk:].any()
    print(f"{name}: levels shots operator worst rel-L2 {worst:.2e}")
    h.close()


@pytest.mark.parametrize("name, nsteps, L", [("small", 200, 64), ("ragged", 150, 40)])
def test_levels_adjoint_gradient_matches_oracle(name, nsteps, L):
    from paper_1406_6923_amd import sfm
    print(f"[case] levels adjoint {name}: {nsteps} steps, checkpoints every {L}", flush=True)
    h, cfg, cs_ks, ks = _loaded(name)
    dt = 0.9 * cs_ks.cfl_dt()
    wav = W.ricker(cfg.f_peak, dt, nsteps)[:, None]
    traces, _ = adjoint.forward(cs_ks, dt, wav)
    rng = np.random.default_rng(11)
    observed = 0.7 * traces + 0.05 * np.abs(traces).max() * rng.standard_normal(traces.shape)
    wav_d = torch.tensor(wav, dtype=torch.float32, device="cuda")
    tr = torch.zeros((len(cs_ks.receivers), nsteps), dtype=torch.float32, device="cuda")
    sfm.sfm_step(h.ctx, nsteps, dt, wav_d, tr)
    resid = (tr - torch.tensor(observed, dtype=torch.float32, device="cuda")).contiguous()
    g_gam, g_hat = sfm.sfm_adjoint_gradient(h.ctx, nsteps, dt, wav_d, resid, L)
    J, r_gam, r_hat = adjoint.gradient(cs_ks, dt, wav, observed)
    for a, kk in enumerate(ks):
        assert not g_gam[a, kk:].any() and not g_hat[a, kk:].any()
    e_gam = rel_l2(g_gam, r_gam)
    e_hat = rel_l2(g_hat[:, 1:], r_hat[:, 1:])
    print(f"{name}: levels gradient rel-L2 Gamma {e_gam:.2e}, Gamma-hat {e_hat:.2e}")
    assert e_gam < 1e-4 and e_hat < 1e-4
    h.close()


def test_levels_errors_and_reset():
    from paper_1406_6923_amd import sfm
    cfg, c, subs, roms, cs = oracle_case("small")
    S = len(subs)
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k)
    with pytest.raises(sfm.SfmError) as ei:                 # no ROMs yet
        sfm.sfm_set_levels(h.ctx, np.full(S, 2))
    assert ei.value.status == sfm.SFM_ESTATE
    gam, hat, src, rec = rom_arrays(cs)
    sfm.sfm_load_roms(h.ctx, gam, hat, cfg.sources(), src, cfg.receivers(), rec)
    assert (sfm.sfm_get_levels(h.ctx) == cfg.k).all()
    good = np.full(S, 3)
    sfm.sfm_set_levels(h.ctx, good)
    for bad in (1, cfg.k + 1):
        ks = good.copy()
        ks[S // 2] = bad
        with pytest.raises(sfm.SfmError) as ei:
            sfm.sfm_set_levels(h.ctx, ks)
        assert ei.value.status == sfm.SFM_EINVAL
        assert (sfm.sfm_get_levels(h.ctx) == 3).all()      # the previous table stays
    sfm.sfm_set_levels(h.ctx, None)
    assert (sfm.sfm_get_levels(h.ctx) == cfg.k).all()
    sfm.sfm_set_levels(h.ctx, good)
    sfm.sfm_load_roms(h.ctx, gam, hat, cfg.sources(), src, cfg.receivers(), rec)   # a new load clears it
    assert (sfm.sfm_get_levels(h.ctx) == cfg.k).all()
    h.close()


@pytest.mark.parametrize("name, nsteps", [("small", 500), ("uneven", 300)])
def test_levels_build_matches_oracle(name, nsteps):
    """The device build run k_s steps per subdomain: blocks within the per-level FP64 tolerance of
    the oracle's k_s-step ROMs, zero past k_s; projections 1e-7; traces 1e-5."""
    from paper_1406_6923_amd import sfm
    from tests.cases import case_level_tolerance
    cfg, c, subs, roms, cs = oracle_case(name)
    cfg, subs, roms_ks, cs_ks, ks = mixed_level_case(name)
    print(f"[case] levels build {name}: {ks.tolist()}", flush=True)
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k)
    sfm.sfm_build_roms_levels(h.ctx, ks, torch.from_numpy(c.astype(np.float32)).cuda(), cfg.sources(),
                              cfg.receivers())
    assert np.array_equal(sfm.sfm_get_levels(h.ctx), ks)
    gam, hat = sfm.sfm_export_roms(h.ctx)
    tol = case_level_tolerance(name)
    for a, r in enumerate(roms_ks):
        for j in range(cfg.k):
            if j >= ks[a]:
                assert not gam[a, j].any() and not hat[a, j].any()
                continue
            for got, ref in ((gam[a, j], r.sf.gamma[j]), (hat[a, j], r.sf.gamma_hat[j])):
                assert np.abs(got - ref).max() / np.abs(ref).max() < tol[j], (a, j)
    src, rec = sfm.sfm_export_projections(h.ctx)
    ref_src = pad_levels([v for (_, v, _) in cs_ks.sources], cfg.k)
    ref_rec = pad_levels([row for (_, row) in cs_ks.receivers], cfg.k)
    for got, ref in ((src, ref_src), (rec, ref_rec)):
        if np.linalg.norm(ref) == 0:           # a point deeper than a k_s-level ROM reaches
            assert not got.any()
        else:
            assert rel_l2(got, ref) < 1e-7
    dt = 0.9 * cs_ks.cfl_dt()
    wav = W.ricker(cfg.f_peak, dt, nsteps)[:, None]
    ref = cs_ks.run(dt, wav)
    tr = torch.zeros((len(cs_ks.receivers), nsteps), dtype=torch.float32, device="cuda")
    sfm.sfm_step(h.ctx, nsteps, dt, torch.tensor(wav, dtype=torch.float32, device="cuda"), tr)
    torch.cuda.synchronize()
    err = rel_l2(tr.cpu().numpy(), ref)
    print(f"{name}: levels build, traces rel-L2 {err:.2e}")
    assert err < 1e-5
    h.close()
