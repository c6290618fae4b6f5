"""GPU parity on a tensor product of boxes of uneven size (x: 12 | 16, y: 8 | 12, z: 10 | 8 cells),
the decomposition of the Introduction without equal subdomains.

The device build groups subdomains of one shape into a batch, so every one of the eight shapes
here runs its own batch.  Bars as on equal boxes: S-fraction blocks per level at 30 times the
oracle's own FP64 reproducibility, projections 1e-7, the projected initial state 1e-6, traces of
the GPU-built ROMs 1e-5 against the oracle's.  The last test combines uneven boxes, a ROM size of
its own per subdomain and 64 shots (8 driven) against 8 oracle runs of ROMs built at those sizes.
"""
import numpy as np
import pytest

import workloads as W
from oracle import coupled, rom
from tests.cases import case_level_tolerance, level_table, oracle_case, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NAME = "uneven"
NSHOT = 64


def _build(**kw):
    from paper_1406_6923_amd import sfm
    cfg, c, subs, roms, cs = oracle_case(NAME)
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k)
    vel = torch.tensor(c, dtype=torch.float32, device="cuda")
    sfm.sfm_build_roms(h.ctx, vel, cfg.sources(), cfg.receivers(), **kw)
    return h, cfg, c, subs, roms, cs


def test_boxes_build_matches_oracle():
    from paper_1406_6923_amd import sfm
    print(f"[case] uneven boxes build", flush=True)
    h, cfg, c, subs, roms, cs = _build()
    assert len({sd.cells for sd in subs}) == 8
    gam, hat = sfm.sfm_export_roms(h.ctx)
    tol = case_level_tolerance(NAME)
    worst = 0.0
    for s, r in enumerate(roms):
        for j in range(cfg.k):
            for got, ref in ((gam[s, j], r.sf.gamma[j]), (hat[s, j], r.sf.gamma_hat[j])):
                err = np.abs(got - ref).max() / np.abs(ref).max()
                worst = max(worst, err / tol[j])
                assert err < tol[j], (s, j, err, tol[j])
    src, rec = sfm.sfm_export_projections(h.ctx)
    assert rel_l2(src, np.stack([v for (_, v, _) in cs.sources])) < 1e-7
    assert rel_l2(rec, np.stack([r for (_, r) in cs.receivers])) < 1e-7
    nsteps = 300
    dt = 0.9 * cs.cfl_dt()
    wav = W.ricker(cfg.f_peak, dt, nsteps)[:, None]
    ref = cs.run(dt, wav)
    tr = torch.zeros((len(cs.receivers), nsteps), dtype=torch.float32, device="cuda")
    sfm.sfm_step(h.ctx, nsteps, dt, torch.tensor(wav, dtype=torch.float32, device="cuda"), tr)
    torch.cuda.synchronize()
    err = rel_l2(tr.cpu().numpy(), ref)
    print(f"uneven: worst block error / tolerance {worst:.2f}; end-to-end traces rel-L2 {err:.2e}")
    assert err < 1e-5
    h.close()


def test_boxes_initial_condition_projection():
    from paper_1406_6923_amd import sfm
    print(f"[case] uneven boxes initial condition", flush=True)
    cfg, c, subs, roms, cs = oracle_case(NAME)
    nz, ny, nx = c.shape
    l, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u0 = np.exp(-((i - 11.0) ** 2 + (j - 9.0) ** 2 + (l - 8.0) ** 2) / 10.0)
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k)
    dev = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    sfm.sfm_build_roms(h.ctx, dev(c), None, cfg.receivers(), dev(u0), None)
    U0 = []
    for sd, r in zip(subs, roms):
        sl = (slice(sd.origin[2], sd.origin[2] + sd.shape[0]), slice(sd.origin[1], sd.origin[1] + sd.shape[1]),
              slice(sd.origin[0], sd.origin[0] + sd.shape[2]))
        U0.append(r.project_state(sd, u0[sl]))
    u, d, n = sfm.sfm_get_state(h.ctx)
    err = rel_l2(u, np.stack(U0))
    print(f"uneven: projected initial state rel-L2 {err:.2e}")
    assert err < 1e-6
    h.close()


def _surface_sources(cfg, n, seed=7):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        ijk = (int(rng.integers(1, cfg.ncell[0])), int(rng.integers(1, cfg.ncell[1])), 2)
        if cfg.on_box_plane(ijk) or ijk in out:
            continue
        out.append(ijk)
    return out


def test_boxes_levels_and_shots_match_oracle():
    from paper_1406_6923_amd import sfm
    cfg, c, subs, roms, cs = oracle_case(NAME)
    nrun, nsteps = 8, 300
    srcs = _surface_sources(cfg, nrun)
    ks = level_table(len(subs), cfg.k, seed=4)
    print(f"[case] uneven boxes, levels {ks.tolist()}, {NSHOT} shots ({nrun} driven), {nsteps} steps", flush=True)
    roms_ks = [rom.build_rom(sd, int(kk)) for sd, kk in zip(subs, ks)]
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k)
    sfm.sfm_build_roms(h.ctx, torch.tensor(c, dtype=torch.float32, device="cuda"), np.asarray(srcs),
                       cfg.receivers())
    sfm.sfm_set_levels(h.ctx, ks)
    shot_src = np.full(NSHOT, -1)
    shot_src[:nrun] = np.arange(nrun)[::-1]
    sfm.sfm_shots_init(h.ctx, NSHOT, shot_src)
    cs0 = coupled.CoupledSystem(subs, roms_ks, [srcs[0]], cfg.receivers())
    dt = 0.9 * cs0.cfl_dt()
    wav = np.zeros((nsteps, NSHOT))
    for n in range(nrun):
        wav[:, n] = W.ricker(cfg.f_peak * (0.8 + 0.05 * n), dt, nsteps)
    tr = torch.zeros((NSHOT, len(cfg.receivers()), nsteps), dtype=torch.float32, device="cuda")
    sfm.sfm_shots_step(h.ctx, nsteps, dt, torch.tensor(wav, dtype=torch.float32, device="cuda"), tr)
    torch.cuda.synchronize()
    got = tr.cpu().numpy()
    worst = 0.0
    for n in range(nrun):
        cs_n = coupled.CoupledSystem(subs, roms_ks, [srcs[shot_src[n]]], cfg.receivers())
        ref = cs_n.run(dt, wav[:, n:n + 1])
        err = rel_l2(got[n], ref)
        worst = max(worst, err)
        assert err < 1e-5, (n, err)
    assert not got[nrun:].any()
    print(f"uneven + levels: {nrun} shots, worst traces rel-L2 {worst:.2e}")
    h.close()
