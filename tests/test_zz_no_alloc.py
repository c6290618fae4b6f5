"""sfm_cfl_dt_noalloc (the stability limit with its certificate scratch in a static device array)
against sfm_cfl_dt through the C ABI: the same kernels, with each subdomain's arithmetic the same in
any batch of subdomains, so the limits, estimates and bounds agree exactly; two calls in a row on
different contexts, the second on a smaller system; a system of more subdomains than the static
array holds at once (smaller batches than the allocating call's); no device memory is allocated by
a call once the array is resident; sizes beyond the static limit are rejected."""
import pytest

import workloads as W
from tests.cases import oracle_case, rom_arrays

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _loaded(name):
    from paper_1406_6923_amd import sfm
    cfg, c, subs, roms, cs = oracle_case(name)
    gam, hat, src, rec = rom_arrays(cs)
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k)
    sfm.sfm_load_roms(h.ctx, gam, hat, cfg.sources(), src, cfg.receivers(), rec)
    return h, cs


def test_noalloc_limit_equals_the_allocating_call():
    from paper_1406_6923_amd import sfm
    print("[case] no-alloc CFL: mid (6m = 96, k = 16) then small (6m = 24, k = 8)", flush=True)
    ha, csa = _loaded("mid")
    hb, csb = _loaded("small")
    ref_a = sfm.sfm_cfl_dt(ha.ctx, 100)
    info_a = ha.info()
    ref_b = sfm.sfm_cfl_dt(hb.ctx, 100)
    info_b = hb.info()
    got_a = sfm.sfm_cfl_dt_noalloc(ha.ctx, 100)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    got_b = sfm.sfm_cfl_dt_noalloc(hb.ctx, 100)
    free1 = torch.cuda.mem_get_info()[0]
    print(f"mid: {got_a:.10e} vs {ref_a:.10e}; small: {got_b:.10e} vs {ref_b:.10e}; free memory change "
          f"{free1 - free0} bytes")
    assert got_a == ref_a and got_b == ref_b
    assert ha.info()["rho_bound"] == info_a["rho_bound"] and hb.info()["rho_bound"] == info_b["rho_bound"]
    assert ha.info()["rho_estimate"] == info_a["rho_estimate"]
    assert free1 >= free0
    # both limits are certified against the oracle's exact ones
    assert got_a <= csa.cfl_dt() * (1 + 1e-6) and got_b <= csb.cfl_dt() * (1 + 1e-6)
    # and the limit it sets is the one sfm_step enforces
    with pytest.raises(sfm.SfmError) as ei:
        sfm.sfm_step(hb.ctx, 1, 1.001 * got_b, torch.zeros((1, 1), device="cuda"))
    assert ei.value.status == sfm.SFM_EUNSTABLE
    ha.close()
    hb.close()


def test_noalloc_limit_with_more_subdomains_than_one_batch():
    from paper_1406_6923_amd import sfm
    cfg = W.scaled_large((8, 8, 4))
    print(f"[case] no-alloc CFL: {cfg.name}, 256 subdomains at 6m = 96 (125 per static batch)", flush=True)
    c = torch.from_numpy(cfg.velocity_model().astype("float32")).cuda()
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k)
    sfm.sfm_build_roms(h.ctx, c, cfg.sources(), cfg.receivers())
    ref = sfm.sfm_cfl_dt(h.ctx, 50)
    info = h.info()
    got = sfm.sfm_cfl_dt_noalloc(h.ctx, 50)
    print(f"{got:.12e} vs {ref:.12e}; rho bound {h.info()['rho_bound']:.12e} vs {info['rho_bound']:.12e}")
    assert got == ref and h.info()["rho_bound"] == info["rho_bound"]
    h.close()


def test_noalloc_rejects_sizes_beyond_the_static_scratch():
    from paper_1406_6923_amd import sfm
    print("[case] no-alloc CFL: 70^3 subdomains (above the 262,144 limit)", flush=True)
    h = sfm.Sfm((140, 140, 140), (2, 2, 2), 10.0, 1, 2)
    with pytest.raises(sfm.SfmError) as ei:
        sfm.sfm_cfl_dt_noalloc(h.ctx, 20)
    assert ei.value.status == sfm.SFM_EINVAL and "static scratch" in str(ei.value)
    h.close()
    cfg = W.CFG_SMALL
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k)
    with pytest.raises(sfm.SfmError) as ei:            # no ROMs yet
        sfm.sfm_cfl_dt_noalloc(h.ctx, 20)
    assert ei.value.status == sfm.SFM_ESTATE
    h.close()
