"""The seeded input recipes (``workloads``) against the definitions their docstrings state, and
the named workload configurations against the sizes the bench and the parity tests are quoted on.
CPU only."""
import math

import numpy as np

import workloads as W


def test_named_workloads():
    s = W.CFG_SMALL
    assert s.ncell == (32, 32, 32) and s.nsub == (2, 2, 2) and (s.m, s.k, s.p) == (4, 8, 24)
    assert len(s.receivers()) == 16 * 16 and s.nsteps == 500
    L = W.CFG_LARGE
    assert L.ncell == (512, 512, 512) and L.nsub == (16, 16, 16) and (L.m, L.k, L.p) == (16, 16, 96)
    assert len(L.receivers()) == 256 * 256 and L.nsteps == 2000 and L.n_subdomains == 4096
    A = W.CFG_ADJOINT
    assert A.ncell == (256, 256, 256) and A.nsub == (8, 8, 8) and (A.m, A.k) == (12, 16)
    assert len(A.receivers()) == 128 * 128 and A.nsteps == 4000
    S = W.CFG_SHOTS
    assert S.ncell == (384, 384, 256) and (S.m, S.k) == (12, 32) and S.nsteps == 1500
    for d in range(3):
        cells = S.box_cells(d)
        assert sum(cells) == S.ncell[d] and set(cells) <= {24, 32, 48}


def test_uneven_boxes_fill_the_axis_with_the_given_sizes():
    for n in (256, 384):
        for seed in range(20):
            b = W.uneven_boxes(n, seed=seed)
            assert sum(b) == n and set(b) <= {24, 32, 48}
    assert W.uneven_boxes(384, seed=3) == W.uneven_boxes(384, seed=3)
    assert len({W.uneven_boxes(384, seed=q) for q in range(20)}) > 1


def test_level_choices_uniform_over_the_set():
    v = W.level_choices(5000, seed=1)
    assert v.dtype == np.int32 and set(v.tolist()) == {8, 12, 16, 24, 32}
    counts = np.array([(v == x).sum() for x in (8, 12, 16, 24, 32)])
    assert np.all(np.abs(counts - 1000) < 4 * math.sqrt(5000 * 0.2 * 0.8))
    assert np.array_equal(W.level_choices(100, seed=7), W.level_choices(100, seed=7))


def test_surface_shots_distinct_interior_and_off_box_planes():
    cfg = W.CFG_SHOTS
    pts = W.surface_shots(cfg, 64)
    assert len(set(pts)) == 64
    for i, j, l in pts:
        assert l == 2 and 0 < i < cfg.ncell[0] and 0 < j < cfg.ncell[1]
        assert not cfg.on_box_plane((i, j, l))


def test_receiver_grid_odd_surface_nodes():
    r = W.receiver_grid(4, 3)
    assert r.shape == (12, 3) and r.dtype == np.int32
    assert set(r[:, 0].tolist()) == {1, 3, 5, 7} and set(r[:, 1].tolist()) == {1, 3, 5} and not r[:, 2].any()


def test_gaussian_anomaly_closed_form():
    c = np.full((41, 41, 41), 2000.0)
    g = W.gaussian_anomaly(c, center=(20, 20, 20), radius=10.0, amplitude=0.05)
    assert g[20, 20, 20] == 2000.0 * 1.05
    assert math.isclose(g[20, 20, 30], 2000.0 * (1.0 + 0.05 / math.e), rel_tol=1e-14)   # r = radius along x
    assert math.isclose(g[30, 20, 20], g[20, 30, 20], rel_tol=1e-14)                     # isotropic
    assert abs(g[0, 0, 0] / 2000.0 - 1.0) < 0.05 * math.exp(-3 * 400 / 100) * 1.0001


def test_layered_inclusions_structure():
    nodes = (33, 29, 37)
    c0 = W.layered_inclusions_velocity(nodes, seed=5, n_spheres=0)
    assert c0.shape == (37, 29, 33)
    assert np.all(c0 == c0[:, :1, :1])                          # horizontal layers
    assert c0.min() >= 1500.0 and c0.max() <= 4500.0
    assert 2 <= len(np.unique(c0)) <= 20
    c = W.layered_inclusions_velocity(nodes, seed=5)             # same layers, then the spheres
    ratio = c / c0
    ok = np.zeros(ratio.shape, dtype=bool)
    for a in range(51):                                          # overlapping spheres multiply
        for b in range(51 - a):
            ok |= np.isclose(ratio, 1.3 ** a * 0.7 ** b, rtol=1e-12)
    assert ok.all() and (ratio != 1.0).any()                     # each sphere scales by 1 +- 0.3


def test_ricker_closed_form():
    f, dt = 15.0, 1e-4
    w = W.ricker(f, dt, 2000)
    n0 = int(round(1.5 / f / dt))
    assert math.isclose(w[n0], 1.0, rel_tol=1e-12) and w.argmax() == n0
    tz = 1.0 / (math.pi * f * math.sqrt(2.0))                   # zero crossing of 1 - 2 pi^2 f^2 tau^2
    assert abs(W.ricker(f, tz, 2, delay=0.0)[1]) < 1e-12
