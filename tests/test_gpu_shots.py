"""GPU parity of the many-shot step (64-column MFMA block products) against the FP64 oracle.

Every shot is an independent run of Algorithm 1, Stage 2 through the same ROMs, so the oracle
for shot n is the oracle's coupled system driven by shot n's source alone.  The operator is
checked on all 64 shots at once: with D = 0 and dt = 1 one step leaves D = a(U) exactly (FP32
fma with a zero addend), compared entry by entry with the oracle's accelerations of each shot's
random state, at the same relative bars as the single-shot FP32 operator (1e-5 at p <= 24, 5e-5
at p = 96, where FP32 rounding of the stored coefficients dominates).  Traces of 8 shots with 8
distinct sources and wavelets are held to 1e-5 against 8 separate oracle runs.  With FP64
coefficient storage (FP64 matrix cores) the operator is held to 1e-6 at every size.
"""
import numpy as np
import pytest

import workloads as W
from oracle import coupled
from tests.cases import oracle_case, random_consistent_state, rel_l2, rom_arrays

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NSHOT = 64


def _load(cfg, cs, src_ijk=None, src_vec=None, precision=0):
    from paper_1406_6923_amd import sfm
    gam, hat, src, rec = rom_arrays(cs)
    if src_ijk is None:
        src_ijk, src_vec = cfg.sources(), src
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k, precision=precision)
    sfm.sfm_load_roms(h.ctx, gam, hat, src_ijk, src_vec, cfg.receivers(), rec)
    return h


# FP64 coefficients (FP64 matrix cores): only the FP32 state and the FP32 result round, so the
# bar is 1e-6 at every size.
@pytest.mark.parametrize("name, tol, precision", [("small", 1e-5, 0), ("ragged", 1e-5, 0), ("mid", 5e-5, 0),
                                                  ("small", 1e-6, 2), ("ragged", 1e-6, 2), ("mid", 1e-6, 2)])
def test_shots_operator_matches_oracle(name, tol, precision):
    from paper_1406_6923_amd import sfm
    cfg, c, subs, roms, cs = oracle_case(name)
    print(f"[case] shots operator {name}, {NSHOT} shots, precision {precision}", flush=True)
    h = _load(cfg, cs, precision=precision)
    sfm.sfm_shots_init(h.ctx, NSHOT, np.full(NSHOT, -1))
    chosen, variants = sfm.sfm_shots_tuning(h.ctx)
    print(f"{name}: autotuner {variants} -> {chosen} waves per SIMD")
    assert chosen in [w for w, _ in variants] and all(ms > 0 for _, ms in variants)
    assert min(variants, key=lambda v: v[1])[0] == chosen
    U = np.stack([random_consistent_state(cs, seed=100 + n) for n in range(NSHOT)], axis=-1).astype(np.float32)
    sfm.sfm_shots_set_state(h.ctx, U, np.zeros_like(U))
    wav = torch.zeros((1, NSHOT), dtype=torch.float32, device="cuda")
    sfm.sfm_shots_step(h.ctx, 1, 1.0, wav, None)
    _, a = sfm.sfm_shots_get_state(h.ctx, NSHOT)
    worst = 0.0
    for n in range(NSHOT):
        ref = np.stack(cs.accel(list(U[..., n].astype(np.float64))))
        err = rel_l2(a[..., n], ref)
        worst = max(worst, err)
        assert rel_l2(a[:, 0, :, n], ref[:, 0]) < tol, (n, "boundary layer")
        assert rel_l2(a[:, 1:, :, n], ref[:, 1:]) < tol, (n, "interior layers")
    print(f"{name} (precision {precision}): shots operator worst rel-L2 over {NSHOT} shots {worst:.2e}")
    assert worst < tol
    h.close()


@pytest.mark.parametrize("name, tol, precision", [("ragged", 1e-5, 0), ("mid", 5e-5, 0), ("ragged", 1e-6, 2),
                                                  ("mid", 1e-6, 2)])
def test_every_shot_variant_matches_oracle(name, tol, precision):
    """Every compiled variant of the shot kernel that fits this 6m (forced with sfm_shots_select),
    not only the autotuner's choice: the operator of 64 shots against the oracle, and bit-equal
    across the variants (each output element takes the same products in the same order)."""
    from paper_1406_6923_amd import sfm
    cfg, c, subs, roms, cs = oracle_case(name)
    print(f"[case] every shot variant {name}, precision {precision}", flush=True)
    h = _load(cfg, cs, precision=precision)
    sfm.sfm_shots_init(h.ctx, NSHOT, np.full(NSHOT, -1))
    chosen, variants = sfm.sfm_shots_tuning(h.ctx, every_variant=True)
    U = np.stack([random_consistent_state(cs, seed=300 + n) for n in range(NSHOT)], axis=-1).astype(np.float32)
    refs = [np.stack(cs.accel(list(U[..., n].astype(np.float64)))) for n in range(NSHOT)]
    wav = torch.zeros((1, NSHOT), dtype=torch.float32, device="cuda")
    first = None
    ran = 0
    for v, (waves, ms) in enumerate(variants):
        if ms < 0:                       # work-group limit or prefetch capacity below this 6m
            with pytest.raises(sfm.SfmError) as ei:
                sfm.sfm_shots_select(h.ctx, v)
            assert ei.value.status == sfm.SFM_EINVAL
            continue
        sfm.sfm_shots_select(h.ctx, v)
        sfm.sfm_shots_set_state(h.ctx, U, np.zeros_like(U))
        sfm.sfm_shots_step(h.ctx, 1, 1.0, wav, None)
        _, a = sfm.sfm_shots_get_state(h.ctx, NSHOT)
        worst = max(rel_l2(a[..., n], refs[n]) for n in range(NSHOT))
        print(f"{name} precision {precision}: variant {v} ({waves} waves per SIMD, {ms:.3f} ms) worst {worst:.2e}")
        assert worst < tol, v
        if first is None:
            first = a
        else:
            assert np.array_equal(a, first), v
        ran += 1
    assert ran >= 1
    sfm.sfm_shots_select(h.ctx, -1)
    with pytest.raises(sfm.SfmError):
        sfm.sfm_shots_select(h.ctx, len(variants))
    h.close()


def _shot_sources(cfg, n):
    """n surface-near source nodes strictly inside subdomains (off every interface plane)."""
    rng = np.random.default_rng(7)
    out = []
    while len(out) < n:
        i, j = (int(x) for x in rng.integers(1, min(cfg.ncell[:2]), size=2))
        l = 2
        if i % cfg.sub_cells[0] == 0 or j % cfg.sub_cells[1] == 0 or (i, j, l) in out:
            continue
        out.append((i, j, l))
    return out


@pytest.mark.parametrize("name, nsteps, precision", [("small", 500, 0), ("ragged", 300, 0), ("ragged", 300, 2)])
def test_shots_traces_match_oracle(name, nsteps, precision):
    from paper_1406_6923_amd import sfm
    cfg, c, subs, roms, cs = oracle_case(name)
    nrun = 8
    srcs = _shot_sources(cfg, nrun)
    cs_all = coupled.CoupledSystem(subs, roms, srcs, cfg.receivers())
    _, _, src_vec, _ = rom_arrays(cs_all)
    h = _load(cfg, cs, np.asarray(srcs), src_vec, precision=precision)
    # shots 0..7 driven by sources 7..0 (a non-identity map), the other 56 shots silent
    shot_src = np.full(NSHOT, -1)
    shot_src[:nrun] = np.arange(nrun)[::-1]
    sfm.sfm_shots_init(h.ctx, NSHOT, shot_src)
    dt = 0.9 * cs.cfl_dt()
    wav = np.zeros((nsteps, NSHOT))
    for n in range(nrun):
        wav[:, n] = W.ricker(cfg.f_peak * (0.8 + 0.05 * n), dt, nsteps)
    tr = torch.zeros((NSHOT, len(cs.receivers), nsteps), dtype=torch.float32, device="cuda")
    print(f"[case] shots traces {name}, {nrun} driven shots, {nsteps} steps", flush=True)
    sfm.sfm_shots_step(h.ctx, nsteps, dt, torch.tensor(wav, dtype=torch.float32, device="cuda"), tr)
    torch.cuda.synchronize()
    got = tr.cpu().numpy()
    worst = 0.0
    for n in range(nrun):
        cs_n = coupled.CoupledSystem(subs, roms, [srcs[shot_src[n]]], cfg.receivers())
        ref = cs_n.run(dt, wav[:, n:n + 1])
        err = rel_l2(got[n], ref)
        worst = max(worst, err)
        assert err < 1e-5, (n, err)
    assert not got[nrun:].any()
    print(f"{name} (precision {precision}): {nrun} shots, worst traces rel-L2 {worst:.2e}")
    h.close()


def test_sampled_shot_timing_leaves_traces_alone():
    """Shot steps timed one in three (events pooled, read back once by sfm_shots_timing): the
    count matches and the traces equal those of an untimed run bit for bit."""
    from paper_1406_6923_amd import sfm
    cfg, c, subs, roms, cs = oracle_case("small")
    h = _load(cfg, cs)
    shot_src = np.full(NSHOT, -1)
    shot_src[0] = 0
    sfm.sfm_shots_init(h.ctx, NSHOT, shot_src)
    u0, d0 = sfm.sfm_shots_get_state(h.ctx, NSHOT)
    dt = 0.9 * cs.cfl_dt()
    nsteps = 40
    wav = torch.tensor(np.repeat(W.ricker(cfg.f_peak, dt, nsteps)[:, None], NSHOT, axis=1),
                       dtype=torch.float32, device="cuda")
    nrec = len(cfg.receivers())
    out = []
    for every in (0, 3):
        sfm.sfm_shots_set_state(h.ctx, u0, d0)
        sfm.sfm_shots_timing(h.ctx)
        sfm.sfm_set_timing(h.ctx, every > 0, every=max(every, 1))
        tr = torch.zeros((NSHOT, nrec, nsteps), dtype=torch.float32, device="cuda")
        sfm.sfm_shots_step(h.ctx, nsteps, dt, wav, tr)
        torch.cuda.synchronize()
        sfm.sfm_set_timing(h.ctx, False)
        nt, ms = sfm.sfm_shots_timing(h.ctx)
        assert nt == (0 if every == 0 else (nsteps + every - 1) // every), (every, nt)
        if every:
            assert ms[0] > 0 and ms[1] > 0
        out.append(tr.cpu().numpy())
    assert np.array_equal(out[0], out[1])
    assert np.abs(out[0]).max() > 0
    h.close()


def test_shots_errors():
    from paper_1406_6923_amd import sfm
    cfg, c, subs, roms, cs = oracle_case("small")
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k)
    with pytest.raises(sfm.SfmError) as ei:
        sfm.sfm_shots_init(h.ctx, 4)
    assert ei.value.status == sfm.SFM_ESTATE
    h.close()
    h = _load(cfg, cs)
    with pytest.raises(sfm.SfmError) as ei:
        sfm.sfm_shots_step(h.ctx, 1, 1e-3, None, None)
    assert ei.value.status == sfm.SFM_ESTATE
    for bad in (0, 65):
        with pytest.raises(sfm.SfmError) as ei:
            sfm.sfm_shots_init(h.ctx, bad, np.full(max(bad, 1), -1)[:bad] if bad else None)
        assert ei.value.status == sfm.SFM_EINVAL
    with pytest.raises(sfm.SfmError) as ei:     # source index out of range
        sfm.sfm_shots_init(h.ctx, 2, np.array([0, 5]))
    assert ei.value.status == sfm.SFM_EINVAL
    with pytest.raises(sfm.SfmError) as ei:     # one source driving two shots
        sfm.sfm_shots_init(h.ctx, 2, np.array([0, 0]))
    assert ei.value.status == sfm.SFM_EINVAL
    sfm.sfm_shots_init(h.ctx, 1)
    dt_max = sfm.sfm_cfl_dt(h.ctx, 100)
    with pytest.raises(sfm.SfmError) as ei:
        sfm.sfm_shots_step(h.ctx, 1, 1.5 * dt_max, torch.zeros((1, 1), device="cuda"), None)
    assert ei.value.status == sfm.SFM_EUNSTABLE
    h.close()
    gam, hat, src, rec = rom_arrays(cs)
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k, precision=sfm.SFM_PREC_BF16_FP32ACC)
    sfm.sfm_load_roms(h.ctx, gam, hat, cfg.sources(), src, cfg.receivers(), rec)
    with pytest.raises(sfm.SfmError) as ei:
        sfm.sfm_shots_init(h.ctx, 1)
    assert ei.value.status == sfm.SFM_EINVAL
    h.close()


def test_shots_graph_replay_is_bit_identical():
    """Graph-replayed windows of 32 steps against every kernel launched directly: four calls of
    100, 64, 96 and 40 steps (a fresh capture, a new trace buffer, a cached graph, a call too
    short to replay), with state reads between them; traces and states bit-identical."""
    from paper_1406_6923_amd import sfm
    cfg, c, subs, roms, cs = oracle_case("small")
    nrun = 8
    srcs = _shot_sources(cfg, nrun)
    cs_all = coupled.CoupledSystem(subs, roms, srcs, cfg.receivers())
    _, _, src_vec, _ = rom_arrays(cs_all)
    shot_src = np.full(NSHOT, -1)
    shot_src[:nrun] = np.arange(nrun)
    hs = []
    for graph in (0, 1):
        h = _load(cfg, cs, np.asarray(srcs), src_vec)
        sfm.sfm_shots_init(h.ctx, NSHOT, shot_src)
        sfm.sfm_shots_graph(h.ctx, graph)
        hs.append(h)
    dt = 0.9 * cs.cfl_dt()
    wav = np.zeros((100, NSHOT))
    for n in range(nrun):
        wav[:, n] = W.ricker(cfg.f_peak * (0.8 + 0.05 * n), dt, 100)
    wav_d = torch.tensor(wav, dtype=torch.float32, device="cuda")
    nrec = len(cfg.receivers())
    bufs = [[torch.full((NSHOT, nrec, 100), -1.0, device="cuda") for _ in range(2)] for _ in hs]
    for call, (nsteps, b) in enumerate([(100, 0), (64, 1), (96, 1), (40, 0)]):
        print(f"[case] shots graph replay: call {call}, {nsteps} steps", flush=True)
        out = []
        for h, bb in zip(hs, bufs):
            sfm.sfm_shots_step(h.ctx, nsteps, dt, wav_d, bb[b], 100)
            torch.cuda.synchronize()
            out.append((bb[b][..., :nsteps].cpu().numpy(), sfm.sfm_shots_get_state(h.ctx, NSHOT)))
        (t0, (u0, d0)), (t1, (u1, d1)) = out
        assert np.array_equal(t0, t1), call
        assert np.array_equal(u0, u1) and np.array_equal(d0, d1), call
        assert np.abs(t0[:nrun]).max() > 0
    assert sfm.sfm_shots_graph(hs[0].ctx) == 0
    assert sfm.sfm_shots_graph(hs[1].ctx) == 3 + 2 + 3
    for h in hs:
        h.close()
