"""The many-shot workload at full size, in the launch configuration bench.py times: 384 x 384 x 256
cells as 936 boxes of 24, 32 or 48 cells per axis, ROMs built on the device with a ROM size per
subdomain from {8, 12, 16, 24, 32} (k_s Lanczos steps each) and FP64 coefficient storage, 64 shots
through the FP64 shot kernel, 36864 receivers.

The oracle builds sampled subdomains (24 x 24 x 32 boxes at their own k_s: one of 8 or 12 levels,
one of 24 and one of 32) and checks:
  * the device's k_s-level coefficients, per level within 30x the oracle's own FP64 response to a
    1e-15 perturbation of the subdomain operator, and zero past k_s;
  * one application of the shot operator to a random state of all 64 shots, on every entry that
    depends only on that subdomain (interior layers j = 2..k_s, outer-face boundary entries),
    elementwise within a forward error bound from the coefficient tolerance, FP64 products and
    the final rounding to FP32; the levels past k_s stay zero.
Whole-run properties: 64 steps of all 64 shots from the graph-replayed loop give finite traces
and bit-identical traces when run again from rest.
"""
import numpy as np
import pytest

import workloads as W
from oracle import rom, subdomains
from tests.cases import level_tolerance, perturbation_profile

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NSHOT = 64
U32 = 2.0 ** -24


def _box_index(cfg, s):
    nb = cfg.nsub
    return s % nb[0], (s // nb[0]) % nb[1], s // (nb[0] * nb[1])


@pytest.fixture(scope="module")
def many():
    from paper_1406_6923_amd import sfm
    cfg = W.CFG_SHOTS
    print(f"[case] many-shot workload {cfg.name}: device build", flush=True)
    c = cfg.velocity_model().astype(np.float32)
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k, precision=sfm.SFM_PREC_FP64)
    S = h.info()["n_subdomains"]
    ks = W.level_choices(S, seed=W.SHOTS_LEVEL_SEED)
    vel = torch.from_numpy(c).cuda()
    sfm.sfm_build_roms_levels(h.ctx, ks, vel, np.asarray(W.surface_shots(cfg, NSHOT)), cfg.receivers())
    del vel
    sfm.sfm_shots_init(h.ctx, NSHOT, np.arange(NSHOT))
    yield cfg, c.astype(np.float64), h, ks
    h.close()


def _oracle_sub(cfg, c, s, k):
    b = _box_index(cfg, s)
    cuts = [np.concatenate([[0], np.cumsum(cfg.box_cells(d))]) for d in range(3)]
    o = [int(cuts[d][b[d]]) for d in range(3)]
    w = [int(cuts[d][b[d] + 1] - cuts[d][b[d]]) for d in range(3)]
    box = c[o[2]:o[2] + w[2] + 1, o[1]:o[1] + w[1] + 1, o[0]:o[0] + w[0] + 1]
    sd = subdomains.decompose(box, cfg.h, tuple(w), cfg.m)[0]
    nsub = cfg.nsub
    nb = []
    for f in range(6):
        d, side = divmod(f, 2)
        bb = list(b)
        bb[d] += 1 if side else -1
        nb.append(-1 if not (0 <= bb[d] < nsub[d]) else (bb[2] * nsub[1] + bb[1]) * nsub[0] + bb[0])
    E, keys = subdomains._basis(sd.shape, tuple(w), tuple(b), tuple(nsub), nb, cfg.h, cfg.m,
                                *subdomains.factor_patches(cfg.m), "patches", tuple(o), cfg.nodes, s)
    sd.E, sd.port_keys, sd.neighbours = E, keys, tuple(nb)
    sd.origin, sd.index = tuple(o), s
    return sd, rom.build_rom(sd, k), nb


def _sample(cfg, ks, levels):
    """The first subdomain of the smallest box shape (a 24 x 24 x 32 box) whose ROM size is in levels."""
    for s in range(len(ks)):
        b = _box_index(cfg, s)
        w = [cfg.box_cells(d)[b[d]] for d in range(3)]
        if sorted(w) == [24, 24, 32] and ks[s] in levels:
            return s
    pytest.skip(f"no 24 x 24 x 32 box with k_s in {levels} in this draw")


# k_s = 24 and 32 are the deep ROMs whose blocks do not survive FP32 storage, the reason the
# workload streams FP64 coefficients through the FP64 shot kernel.
@pytest.mark.parametrize("levels", [(8, 12), (24,), (32,)])
def test_many_shots_sampled_subdomain_matches_oracle(many, levels):
    from paper_1406_6923_amd import sfm
    cfg, c, h, ks = many
    s = _sample(cfg, ks, levels)
    k = int(ks[s])
    print(f"[case] many-shot sampled subdomain {s}, k_s = {k}: oracle build", flush=True)
    sd, r, nb = _oracle_sub(cfg, c, s, k)
    tau = level_tolerance(perturbation_profile(sd, r))
    gam, hat = sfm.sfm_export_roms(h.ctx)
    for j in range(k):
        assert np.abs(gam[s, j] - r.sf.gamma[j]).max() / np.abs(r.sf.gamma[j]).max() < tau[j], j
        assert np.abs(hat[s, j] - r.sf.gamma_hat[j]).max() / np.abs(r.sf.gamma_hat[j]).max() < tau[j], j
    assert not gam[s, k:].any() and not hat[s, k:].any()
    del gam, hat
    S, K, p, m = len(ks), cfg.k, cfg.p, cfg.m
    rng = np.random.default_rng(5)
    U = rng.standard_normal((S, K, p, NSHOT)).astype(np.float32)
    for a in range(S):      # consistent shared boundary entries: the lower-index side's value wins
        for f in range(6):
            d, side = divmod(f, 2)
            bb = list(_box_index(cfg, a))
            bb[d] += 1 if side else -1
            if 0 <= bb[d] < cfg.nsub[d]:
                nbi = (bb[2] * cfg.nsub[1] + bb[1]) * cfg.nsub[0] + bb[0]
                if nbi < a:
                    U[a, 0, f * m:(f + 1) * m] = U[nbi, 0, (f ^ 1) * m:((f ^ 1) + 1) * m]
    print(f"[case] many-shot operator, {NSHOT} shots", flush=True)
    sfm.sfm_shots_set_state(h.ctx, U, np.zeros_like(U))
    sfm.sfm_shots_step(h.ctx, 1, 1.0, torch.zeros((1, NSHOT), dtype=torch.float32, device="cuda"), None)
    _, a = sfm.sfm_shots_get_state(h.ctx, NSHOT)
    got = a[s].astype(np.float64)                     # [K][p][64]
    assert not got[k:].any()
    Us = U[s, :k].astype(np.float64)                  # [k][p][64]
    dU = np.concatenate([Us[1:], np.zeros((1, p, NSHOT))]) - Us
    phi = np.stack([r.sf.gamma[j] @ dU[j] for j in range(k)])
    worst = 0.0
    dphi = [tau[j] * (np.abs(r.sf.gamma[j]) @ np.abs(dU[j])) for j in range(k)]
    for j in range(1, k):
        ref = r.sf.gamma_hat[j] @ (phi[j] - phi[j - 1])
        Gh = np.abs(r.sf.gamma_hat[j])
        bound = (tau[j] * (Gh @ np.abs(phi[j] - phi[j - 1])) + Gh @ (dphi[j] + dphi[j - 1])
                 + U32 * np.abs(ref) + 1e-300)
        ratio = float(np.max(np.abs(got[j] - ref) / bound))
        worst = max(worst, ratio)
        assert ratio < 2.0, (j, ratio)
    H = np.diag(r.sf.gamma_hat[0])
    outer = [q for q in range(p) if nb[q // m] < 0]
    if outer:
        # an outer-face entry is C_f phi_1 with C_f = H stored in FP32, phi_1 exchanged in FP32 and
        # the product rounded: three FP32 roundings on top of the coefficient tolerance
        ref0 = H[outer, None] * phi[0][outer]
        b0 = H[outer, None] * (tau[0] * (np.abs(r.sf.gamma[0]) @ np.abs(dU[0]))[outer]) + 3 * U32 * np.abs(ref0)
        r0 = float(np.max(np.abs(got[0][outer] - ref0) / (2 * b0 + 1e-300)))
        assert r0 <= 1.0, r0
    print(f"subdomain {s} (k_s = {k}, {len(outer)} outer-face entries): worst interior error / bound {worst:.3f}"
          + (f", outer-face entries {r0:.3f}" if outer else ""))


def test_many_shots_run_is_finite_and_reproducible(many):
    from paper_1406_6923_amd import sfm
    cfg, c, h, ks = many
    dt = 0.9 * sfm.sfm_cfl_dt(h.ctx, 100)
    nsteps = 64
    wav = torch.tensor(np.repeat(W.ricker(cfg.f_peak, dt, nsteps)[:, None], NSHOT, axis=1), dtype=torch.float32,
                       device="cuda")
    nrec = len(cfg.receivers())
    outs = []
    for rep in range(2):
        print(f"[case] many-shot run {rep}: {nsteps} steps, {NSHOT} shots, {nrec} receivers", flush=True)
        sfm.sfm_shots_init(h.ctx, NSHOT, np.arange(NSHOT))
        tr = torch.zeros((NSHOT, nrec, nsteps), dtype=torch.float32, device="cuda")
        r0 = sfm.sfm_shots_graph(h.ctx)
        sfm.sfm_shots_step(h.ctx, nsteps, dt, wav, tr)
        torch.cuda.synchronize()
        assert sfm.sfm_shots_graph(h.ctx) - r0 == nsteps // 32
        outs.append(tr.cpu().numpy())
        del tr
    assert np.isfinite(outs[0]).all() and np.abs(outs[0]).max() > 0
    assert np.array_equal(outs[0], outs[1])
    print(f"many-shot run: dt_max {dt / 0.9:.3e}, traces finite and bit-reproducible")
