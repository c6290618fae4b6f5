"""Oracle-side fixtures shared by the GPU parity tests (CPU only, FP64)."""
from __future__ import annotations

import functools

import numpy as np

import workloads as W
from oracle import coupled, grid, rom, subdomains


@functools.lru_cache(maxsize=4)
def oracle_case(name: str = "small", sigma: float = np.inf):
    """Build the oracle ROMs and coupled system of a named workload."""
    if name == "small":
        cfg = W.CFG_SMALL
    elif name == "ragged":
        # p = 6 * 3 = 18 (not a multiple of 16) on a 3 x 2 x 2 split with uneven boxes
        cfg = W.Workload(name="ragged_p18", ncell=(30, 20, 24), sub_cells=(10, 10, 12), h=10.0, m=3, k=5,
                         f_peak=15.0, nsteps=300, src=((14, 7, 5),), rec_grid=(10, 8),
                         velocity="layered_inclusions", seed=5)
    elif name == "mid":
        # The large workload's subdomain size and ROM sizes (33^3 nodes, m = 16, k = 16) on 2 x 2 x 1.
        cfg = W.scaled_large((2, 2, 1), nsteps=150)
    else:
        raise KeyError(name)
    if cfg.velocity == "layered_inclusions":
        c = W.layered_inclusions_velocity(cfg.nodes, seed=cfg.seed, n_spheres=6,
                                          radius_range=(2.0, 8.0))
    else:
        c = cfg.velocity_model()
    # The library takes the sound speed as FP32; the oracle starts from the same rounded values.
    c = c.astype(np.float32).astype(np.float64)
    subs = subdomains.decompose(c, cfg.h, cfg.sub_cells, cfg.m)
    roms = rom.build_all(subs, cfg.k, sigma)
    src = cfg.sources()
    rec = cfg.receivers()
    cs = coupled.CoupledSystem(subs, roms, src, rec)
    return cfg, c, subs, roms, cs


def rom_arrays(cs: coupled.CoupledSystem):
    """FP64 arrays in the C-ABI layout: gamma/gamma_hat [S][k][p][p], src [nsrc][k][p], rec [nrec][k][p]."""
    gam = np.stack([r.gamma for r in cs.roms])
    hat = np.stack([r.gamma_hat for r in cs.roms])
    src = np.stack([vec for (_, vec, _) in cs.sources]) if cs.sources else np.zeros((0,) + gam.shape[1:3])
    rec = np.stack([row for (_, row) in cs.receivers]) if cs.receivers else np.zeros((0,) + gam.shape[1:3])
    return gam, hat, src, rec


def random_consistent_state(cs: coupled.CoupledSystem, seed: int) -> np.ndarray:
    """Random [S][k][p] state whose shared boundary entries agree on both sides."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal(cs._dof_layout()[1])
    return np.stack(cs.scatter(X))


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
