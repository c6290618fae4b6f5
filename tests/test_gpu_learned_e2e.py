"""The 256^3 learned-ROM workload end to end on the device, judged on receiver traces against the
FP64 oracle: a network trained on the device (one 8 x 8 x 8 domain of 32^3-cell subdomains of
seeded media, m = 8, k = 16, labelled by the device Lanczos build), the learned build of the 512
subdomains of the evaluation medium (network prediction, NtD judge at 1e-3 on 8 frequencies,
Lanczos fallback for every rejected or source/receiver subdomain), then 500 FP32 leapfrog steps;
the receiver traces must lie within 1e-3 rel-L2 of the oracle's (tests/golden/learned_e2e_traces.npz,
written by tests/golden/make_learned_e2e_traces.py from oracle ROMs of the same medium)."""
import os
import sys

import numpy as np
import pytest

from tests.cases import rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "learned_e2e_traces.npz")


def test_learned_build_256_traces_within_1e3_of_the_oracle():
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_learned_e2e_traces as G

    import workloads as W
    from paper_1406_6923_amd import sfm
    gold = np.load(GOLDEN)
    rec = G.receivers()
    assert np.array_equal(rec, gold["receivers"]) and np.array_equal(G.SOURCE, gold["source"])
    dt = float(gold["dt"])
    ref = gold["traces"].astype(np.float64)
    nsteps = ref.shape[1]
    p = 6 * G.M
    n_out = 2 * G.K * p * (p + 1) // 2
    nn = G.SUB[0] + 1

    print("[case] learned e2e: labelling 512 training subdomains on the device", flush=True)
    tcells = tuple(8 * s for s in G.SUB)
    ct = W.surrogate_velocity(tuple(x + 1 for x in tcells), seed=5000).astype(np.float32)
    vt = torch.from_numpy(ct).cuda()
    ht = sfm.Sfm(tcells, G.SUB, G.H, G.M, G.K, precision=sfm.SFM_PREC_FP64)
    sfm.sfm_build_roms(ht.ctx, vt)
    St = sfm.sfm_query(ht.ctx)["n_subdomains"]
    xt = torch.zeros((St, nn ** 3), dtype=torch.float32, device="cuda")
    tt = torch.zeros((St, n_out), dtype=torch.float32, device="cuda")
    sfm.sfm_rom_inputs(ht.ctx, vt, xt)
    sfm.sfm_rom_targets(ht.ctx, tt)
    ht.close()
    del vt
    net = sfm.Cnn(nn, 32, n_out, max_batch=64, seed=11)
    net.fit_scale(tt)
    losses = net.train(xt, tt, batch=64, epochs=2, lr=1e-3, seed=3)
    del xt, tt
    print(f"training loss {losses[0]:.3f} -> {losses[-1]:.3f}", flush=True)

    print("[case] learned e2e: learned build of the 512 evaluation subdomains, tol 1e-3", flush=True)
    c = W.surrogate_velocity(tuple(x + 1 for x in G.NCELL), seed=G.SEED).astype(np.float32)
    vel = torch.from_numpy(c).cuda()
    h = sfm.Sfm(G.NCELL, G.SUB, G.H, G.M, G.K)
    acc, err, secs = sfm.sfm_build_roms_surrogate(h.ctx, net, 1e-3, G.F_PEAK, vel, G.SOURCE, rec)
    dt_max = sfm.sfm_cfl_dt(h.ctx)
    print(f"accepted {int(acc.sum())} of {len(acc)} predictions (NtD error median {np.median(err):.2e}); "
          f"dt {dt:.5e} (oracle 0.9 limit), certified device limit {dt_max:.5e}", flush=True)
    assert dt <= dt_max
    print(f"[case] learned e2e: {nsteps} FP32 steps", flush=True)
    wav = torch.tensor(W.ricker(G.F_PEAK, dt, nsteps)[:, None], dtype=torch.float32, device="cuda")
    tr = torch.zeros((len(rec), nsteps), dtype=torch.float32, device="cuda")
    sfm.sfm_step(h.ctx, nsteps, dt, wav, tr)
    torch.cuda.synchronize()
    got = tr.cpu().numpy()
    e = rel_l2(got, ref)
    print(f"learned build of 256^3: traces rel-L2 {e:.2e} against the FP64 oracle over {nsteps} steps")
    assert np.isfinite(got).all()
    assert e < 1e-3
    h.close()
    net.close()
