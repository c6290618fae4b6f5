"""GPU parity at odd tile counts and the named workloads' ROM shapes, against the FP64 oracle.

6m = 48 (m = 8: three 16-row tiles, the learned-ROM workload's shape) and 6m = 72 padded to 80
(m = 12: five tiles, the gradient and many-shot workloads' shape), both with k = 16 on a 2 x 2 x 2
split of 32^3-cell boxes.  An odd tile count gives every block a job that holds a single tile
strip (the middle one), and 6m = 72 adds four padded rows per block; the even shapes of the other
tests (6m = 18, 24, 96) never reach either in the step, adjoint or operator kernels.  The ROMs come
from the oracle (sfm_load_roms), so the kernels are isolated from the device build, except in
test_device_build_traces, which runs the whole path.  test_wide_blocks adds 6m = 108 and 144
(seven and nine tiles) with k = 3, where the stability certificate leaves LDS for global memory.

Bars.  One application of the step operator is held elementwise to the first-order forward error
bound of FP32 storage and FP32 dot products (tests.cases.operator_error_bound); its rel-L2 is
printed.  Traces (Stage 2 over 500 steps) 1e-5 rel-L2, the FP32 bar; the FP64 coefficient stream
1e-6 on one operator application; gradients 1e-4 as in test_gpu_adjoint (FP32 state histories,
FP64 sums).
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint
from tests.cases import operator_error_bound, oracle_case, random_consistent_state, rel_l2, rom_arrays

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = ["m8", "m12"]


def _loaded(name, precision=0, receivers=True):
    from paper_1406_6923_amd import sfm
    print(f"[case] {name}: oracle ROMs", flush=True)
    cfg, c, subs, roms, cs = oracle_case(name)
    gam, hat, src, rec = rom_arrays(cs)
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k, precision=precision)
    sfm.sfm_load_roms(h.ctx, gam, hat, cfg.sources(), src, cfg.receivers() if receivers else None,
                      rec if receivers else None)
    return h, cfg, cs


def _apply(h, U):
    from paper_1406_6923_amd import sfm
    u_d = torch.tensor(U, dtype=torch.float32, device="cuda")
    a_d = torch.empty_like(u_d)
    sfm.sfm_apply_operator(h.ctx, u_d, a_d)
    torch.cuda.synchronize()
    return a_d.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("state", ["random", "wavefield"])
def test_step_operator_within_forward_error_bound(name, state):
    h, cfg, cs = _loaded(name)
    if state == "random":
        U = random_consistent_state(cs, seed=11).astype(np.float32).astype(np.float64)
    else:
        dt = 0.9 * cs.cfl_dt()
        wav = W.ricker(cfg.f_peak, dt, 150)[:, None]
        _, Ul, _ = cs.run(dt, wav, return_state=True)
        U = np.stack(Ul).astype(np.float32).astype(np.float64)
    print(f"[case] {name} operator on a {state} state", flush=True)
    ref = np.stack(cs.accel(list(U)))
    got = _apply(h, U)
    bound = operator_error_bound(cs, U)
    ratio = np.abs(got - ref) / bound
    print(f"{name} {state}: operator rel-L2 {rel_l2(got, ref):.2e} (boundary {rel_l2(got[:, 0], ref[:, 0]):.2e}, "
          f"interior {rel_l2(got[:, 1:], ref[:, 1:]):.2e}); max error / bound {ratio.max():.3f}")
    assert ratio.max() < 1.0
    h.close()


@pytest.mark.parametrize("name", CASES)
def test_step_operator_fp64_coefficients(name):
    from paper_1406_6923_amd import sfm
    h, cfg, cs = _loaded(name, sfm.SFM_PREC_FP64)
    U = random_consistent_state(cs, seed=12).astype(np.float32).astype(np.float64)
    ref = np.stack(cs.accel(list(U)))
    got = _apply(h, U)
    errs = (rel_l2(got, ref), rel_l2(got[:, 0], ref[:, 0]), rel_l2(got[:, 1:], ref[:, 1:]))
    print(f"{name}: FP64 operator rel-L2 all {errs[0]:.2e}, boundary {errs[1]:.2e}, interior {errs[2]:.2e}")
    assert max(errs) < 1e-6
    h.close()


@pytest.mark.parametrize("name", CASES)
def test_traces_500_steps(name):
    from paper_1406_6923_amd import sfm
    h, cfg, cs = _loaded(name)
    dt = 0.9 * cs.cfl_dt()
    nsteps = 500
    print(f"[case] {name}: {nsteps}-step traces, dt {dt:.4e}", flush=True)
    wav = W.ricker(cfg.f_peak, dt, nsteps)[:, None]
    ref = cs.run(dt, wav)
    tr = torch.zeros((len(cs.receivers), nsteps), dtype=torch.float32, device="cuda")
    sfm.sfm_step(h.ctx, nsteps, dt, torch.tensor(wav, dtype=torch.float32, device="cuda"), tr)
    torch.cuda.synchronize()
    got = tr.cpu().numpy()
    err = rel_l2(got, ref)
    print(f"{name}: {nsteps}-step traces rel-L2 {err:.2e}")
    assert err < 1e-5
    h.close()


@pytest.mark.parametrize("name", CASES)
def test_cfl_limit(name):
    """The device's stable step against the oracle's exact limit 2 / sqrt(rho) of the coupled ROM."""
    from paper_1406_6923_amd import sfm
    h, cfg, cs = _loaded(name, receivers=False)
    dt_ref = cs.cfl_dt()
    dt_gpu = sfm.sfm_cfl_dt(h.ctx)
    print(f"{name}: dt_max device {dt_gpu:.6e}, oracle {dt_ref:.6e} (ratio {dt_gpu / dt_ref:.5f})")
    assert dt_gpu <= dt_ref * (1 + 1e-6)
    assert dt_gpu >= 0.95 * dt_ref
    h.close()


@pytest.mark.parametrize("name, nsteps, L", [("m12", 160, 50), ("m8", 160, 160), ("mid", 120, 40)])
def test_adjoint_gradient(name, nsteps, L):
    """Adjoint gradient at 6m = 72 (five tiles), 48 (three) and 96 (six tiles: several jobs per
    block for every wave) against the oracle adjoint."""
    from paper_1406_6923_amd import sfm
    h, cfg, cs = _loaded(name)
    dt = 0.9 * cs.cfl_dt()
    print(f"[case] adjoint {name}: {nsteps} steps, checkpoints every {L}", flush=True)
    wav = W.ricker(cfg.f_peak, dt, nsteps)[:, None]
    traces, _ = adjoint.forward(cs, dt, wav)
    rng = np.random.default_rng(17)
    observed = 0.7 * traces + 0.05 * np.abs(traces).max() * rng.standard_normal(traces.shape)
    wav_d = torch.tensor(wav, dtype=torch.float32, device="cuda")
    tr = torch.zeros((len(cs.receivers), nsteps), dtype=torch.float32, device="cuda")
    sfm.sfm_step(h.ctx, nsteps, dt, wav_d, tr)
    resid = tr - torch.tensor(observed, dtype=torch.float32, device="cuda")
    sfm.sfm_reset_state(h.ctx, dt)
    g_gam, g_hat = sfm.sfm_adjoint_gradient(h.ctx, nsteps, dt, wav_d, resid.contiguous(), L)
    J, r_gam, r_hat = adjoint.gradient(cs, dt, wav, observed)
    e_gam = rel_l2(g_gam, r_gam)
    e_hat = rel_l2(g_hat[:, 1:], r_hat[:, 1:])
    print(f"adjoint {name}: gradient rel-L2 Gamma {e_gam:.2e}, Gamma-hat {e_hat:.2e}")
    assert not g_hat[:, 0].any()
    assert e_gam < 1e-4 and e_hat < 1e-4
    h.close()


@pytest.mark.parametrize("name", CASES)
def test_device_build_traces(name):
    """The whole path at these shapes: device ROM build from the sound speed, then 300 device steps,
    against the oracle's ROMs stepped by the oracle."""
    from paper_1406_6923_amd import sfm
    cfg, c, subs, roms, cs = oracle_case(name)
    print(f"[case] {name}: device build + 300 steps", flush=True)
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k)
    sfm.sfm_build_roms(h.ctx, torch.tensor(c.astype(np.float32), device="cuda"), cfg.sources(), cfg.receivers())
    dt = 0.9 * cs.cfl_dt()
    nsteps = 300
    wav = W.ricker(cfg.f_peak, dt, nsteps)[:, None]
    ref = cs.run(dt, wav)
    tr = torch.zeros((len(cs.receivers), nsteps), dtype=torch.float32, device="cuda")
    sfm.sfm_step(h.ctx, nsteps, dt, torch.tensor(wav, dtype=torch.float32, device="cuda"), tr)
    torch.cuda.synchronize()
    err = rel_l2(tr.cpu().numpy(), ref)
    print(f"{name}: device build + device step, {nsteps}-step traces rel-L2 {err:.2e}")
    assert err < 1e-5
    h.close()


@pytest.mark.parametrize("name", ["m18", "m24"])
def test_wide_blocks(name):
    """6m = 108 and 144 (seven and nine tiles, k = 3): the step operator within its forward-error
    bound, 200-step traces at 1e-5, and the stability limit, whose certificate runs its
    factor-and-solve (6m > 100) and, at 6m = 144, its Cholesky (6m > 143) on global memory instead of
    LDS; the no-allocation variant returns the same limit."""
    from paper_1406_6923_amd import sfm
    h, cfg, cs = _loaded(name)
    U = random_consistent_state(cs, seed=21).astype(np.float32).astype(np.float64)
    ref = np.stack(cs.accel(list(U)))
    got = _apply(h, U)
    ratio = (np.abs(got - ref) / operator_error_bound(cs, U)).max()
    print(f"{name}: operator rel-L2 {rel_l2(got, ref):.2e}, max error / bound {ratio:.3f}")
    assert ratio < 1.0
    dt_ref = cs.cfl_dt()
    dt_gpu = sfm.sfm_cfl_dt(h.ctx)
    dt_na = sfm.sfm_cfl_dt_noalloc(h.ctx)
    print(f"{name}: dt_max device {dt_gpu:.6e} (no-alloc {dt_na:.6e}), oracle {dt_ref:.6e} "
          f"(ratio {dt_gpu / dt_ref:.5f})")
    assert dt_gpu <= dt_ref * (1 + 1e-6) and dt_gpu >= 0.95 * dt_ref
    assert dt_na == dt_gpu
    dt = 0.9 * dt_ref
    nsteps = 200
    wav = W.ricker(cfg.f_peak, dt, nsteps)[:, None]
    tref = cs.run(dt, wav)
    tr = torch.zeros((len(cs.receivers), nsteps), dtype=torch.float32, device="cuda")
    sfm.sfm_set_state(h.ctx, None, None, 0)
    sfm.sfm_step(h.ctx, nsteps, dt, torch.tensor(wav, dtype=torch.float32, device="cuda"), tr)
    torch.cuda.synchronize()
    err = rel_l2(tr.cpu().numpy(), tref)
    print(f"{name}: {nsteps}-step traces rel-L2 {err:.2e}")
    assert err < 1e-5
    h.close()
