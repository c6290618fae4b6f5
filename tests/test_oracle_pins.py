"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them compares the oracle with
itself through a retyped formula: the expected values are closed forms,
textbook special cases, identities with an independent evaluation, brute-force
limits (ROM exact when the Krylov space is the whole space) or conservation
laws.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import coupled, grid, lanczos, rom, sfraction, subdomains

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------- fixtures
@pytest.fixture(scope="module")
def small_case():
    cfg = W.CFG_SMALL
    c = cfg.velocity_model()
    subs = subdomains.decompose(c, cfg.h, cfg.sub_cells, cfg.m)
    roms = rom.build_all(subs, cfg.k)
    return cfg, c, subs, roms


def tiny_box(shape_cells, seed):
    nodes = tuple(s + 1 for s in shape_cells)
    return W.random_velocity(nodes, seed)


# ----------------------------------------------------------------------------- fine grid
def test_fine_operator_is_mirror_neumann_7point():
    """K and M reproduce the textbook 7-point Laplacian with mirror ghost nodes (fine grid, eq. "wave")."""
    rng = np.random.default_rng(3)
    c = rng.uniform(1000, 3000, size=(5, 6, 7))
    h = 7.0
    g = grid.FineGrid(c, h)
    u = rng.standard_normal(c.shape)
    # -M^{-1} K u must equal c^2 * (sum of mirrored neighbours - 6u) / h^2 at every node.
    up = np.pad(u, 1, mode="reflect")
    lap = (up[2:, 1:-1, 1:-1] + up[:-2, 1:-1, 1:-1] + up[1:-1, 2:, 1:-1] + up[1:-1, :-2, 1:-1]
           + up[1:-1, 1:-1, 2:] + up[1:-1, 1:-1, :-2] - 6 * u) / h ** 2
    got = -(g.K @ u.ravel()) / g.M
    np.testing.assert_allclose(got, (c ** 2 * lap).ravel(), rtol=1e-12, atol=1e-12 * np.abs(got).max())


@pytest.mark.parametrize("cells, split", [((6, 4, 6), (3, 2, 2)), ((7, 4, 6), ((3, 4), (2, 2), (4, 2)))])
def test_subdomain_operators_sum_to_global(cells, split):
    """Shared interface nodes get complementary halves: sum_alpha M^alpha = M, sum K^alpha = K
    (equal boxes, and a tensor product of boxes of uneven size)."""
    c = tiny_box(cells, seed=5)
    h = 3.0
    g = grid.FineGrid(c, h)
    subs = subdomains.decompose(c, h, split, m=1)
    Msum = np.zeros(g.M.size)
    Ksum = sp.csr_matrix(g.K.shape)
    nz, ny, nx = c.shape
    for sd in subs:
        i0, j0, l0 = sd.origin
        snz, sny, snx = sd.shape
        l, j, i = np.meshgrid(np.arange(snz), np.arange(sny), np.arange(snx), indexing="ij")
        gidx = ((l + l0) * ny + (j + j0)) * nx + (i + i0)
        gidx = gidx.ravel()
        np.add.at(Msum, gidx, sd.M)
        P = sp.csr_matrix((np.ones(gidx.size), (gidx, np.arange(gidx.size))), shape=(g.M.size, gidx.size))
        Ksum = Ksum + P @ sd.K @ P.T
    np.testing.assert_allclose(Msum, g.M, rtol=1e-14)
    assert abs(Ksum - g.K).max() < 1e-12 * abs(g.K).max()


def test_homogeneous_cfl_is_h_over_sqrt3_c():
    """Checkerboard is an exact eigenvector: lambda_max = 12 c^2/h^2, dt_max = h/(sqrt(3) c)."""
    c = np.full((9, 8, 7), 1800.0)
    h = 10.0
    g = grid.FineGrid(c, h)
    assert g.cfl_dt() == pytest.approx(h / (math.sqrt(3.0) * 1800.0), rel=1e-10)


@pytest.mark.parametrize("factor, grows", [(0.99, False), (1.01, True)])
def test_fine_leapfrog_cfl_transition(factor, grows):
    """Leapfrog is bounded just below dt_max and blows up just above (P9, fine grid)."""
    c = np.full((8, 8, 8), 1500.0)
    h = 10.0
    g = grid.FineGrid(c, h)
    dt = factor * h / (math.sqrt(3.0) * 1500.0)
    rng = np.random.default_rng(1)
    u0 = rng.standard_normal(c.size)
    tr = g.fdtd(dt, np.zeros((300, 1)), [(3, 3, 3)], [(1, 2, 3), (4, 4, 4)], u0=u0)
    peak = np.abs(tr).max()
    assert (peak > 1e6) == grows


def test_green_function_second_order():
    """Homogeneous medium: FDTD -> f(t - r/c)/(4 pi r) before reflections, error / 4 per h / 2 (P10)."""
    c0, f0, L, r = 1000.0, 5.0, 960.0, 120.0
    errs = []
    for h in (20.0, 10.0):
        n = int(round(L / h))
        c = np.full((n + 1, n + 1, n + 1), c0)
        g = grid.FineGrid(c, h)
        dt = 0.5 * h / (math.sqrt(3.0) * c0)
        tend = (L - r) / c0 - 0.02
        nsteps = int(tend / dt)
        wav = W.ricker(f0, dt, nsteps)
        s = n // 2
        off = int(round(r / h))
        tr = g.fdtd(dt, wav[:, None], [(s, s, s)], [(s + off, s, s)])[0]
        # sample n is u at t_{n+1}; the exact field is f(t - r/c) / (4 pi r)
        exact = W.ricker(f0, dt, nsteps + 1, delay=1.5 / f0 + r / c0)[1:] / (4 * math.pi * r)
        errs.append(np.linalg.norm(tr - exact) / np.linalg.norm(exact))
    assert errs[1] < 0.05
    assert 3.0 < errs[0] / errs[1] < 6.0


# ----------------------------------------------------------------------------- basis F
def test_face_basis_diagonal_and_consistent(small_case):
    """Gamma-hat_1 = F^T F is diagonal (non-overlapping boundary functions, eq. "bdrytstep" remark),
    every boundary node has exactly one owner, and both sides of a shared face agree on ports."""
    cfg, c, subs, roms = small_case
    for sd, r in zip(subs, roms):
        F = sd.F().toarray()
        FtF = F.T @ F
        assert np.abs(FtF - np.diag(np.diag(FtF))).max() == 0.0
        np.testing.assert_allclose(r.sf.gamma_hat[0], FtF, rtol=1e-12)
        nnz_per_node = (sd.E != 0).sum(axis=1).A.ravel()
        nz, ny, nx = sd.shape
        l, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        on_boundary = ((i == 0) | (i == nx - 1) | (j == 0) | (j == ny - 1) | (l == 0) | (l == nz - 1)).ravel()
        assert np.all(nnz_per_node[on_boundary] == 1)
        assert np.all(nnz_per_node[~on_boundary] == 0)
    # shared face: same global nodes and weights on both sides for each interface port
    n_ports, ids = subdomains.port_table(subs)
    seen = {}
    for sd in subs:
        E = sd.E.tocsc()
        for col, key in enumerate(sd.port_keys):
            rows = E.indices[E.indptr[col]:E.indptr[col + 1]]
            vals = E.data[E.indptr[col]:E.indptr[col + 1]]
            nz_, ny_, nx_ = sd.shape
            loc = np.stack(np.unravel_index(rows, sd.shape), axis=1)  # (l, j, i)
            glob = [(int(q[2]) + sd.origin[0], int(q[1]) + sd.origin[1], int(q[0]) + sd.origin[2]) for q in loc]
            item = dict(zip(glob, vals))
            if key in seen:
                assert seen[key] == item
            else:
                seen[key] = item
    assert len(seen) == n_ports


def test_patch_factorisation():
    assert subdomains.factor_patches(4) == (2, 2)
    assert subdomains.factor_patches(16) == (4, 4)
    assert subdomains.factor_patches(12) == (4, 3)
    assert subdomains.factor_patches(8) == (4, 2)
    assert subdomains.factor_patches(25) == (5, 5)
    assert subdomains.factor_patches(7) == (7, 1)


# ----------------------------------------------------------------------------- Lanczos / ROM
def test_lanczos_basis_and_tridiagonal(small_case):
    """Z orthonormal, T = Z^T A_+ Z block tridiagonal, R = Z^T F = E_1 B_1 (Stage 2, eq. before "NtDtri")."""
    cfg, c, subs, roms = small_case
    sd, r = subs[3], roms[3]
    Z = r.tri.Z
    A = sd.A_plus()
    assert np.abs(Z.T @ Z - np.eye(Z.shape[1])).max() < 1e-12
    T = r.tri.T()
    assert np.abs(Z.T @ (A @ Z) - T).max() < 1e-12 * np.abs(T).max()
    np.testing.assert_allclose(Z.T @ sd.F().toarray(), r.tri.R(), atol=1e-12 * np.abs(r.tri.R()).max())


def test_markov_moments_match_below_2k():
    """Polynomial block Krylov (sigma = inf) matches F^T A^i F = R^T T^i R exactly for i < 2k and
    not at i = 2k (P3: the moment-matching property of block Lanczos)."""
    c = tiny_box((6, 6, 6), seed=11)
    sd = subdomains.decompose(c, 5.0, (6, 6, 6), m=1)[0]
    A = sd.A_plus().toarray()
    A = A / np.linalg.norm(A, 2)
    F = sd.F().toarray()
    F = F / np.linalg.norm(F, 2)
    k = 4
    tri = lanczos.block_lanczos(lambda X: A @ X, F, k)
    T, R = tri.T(), tri.R()
    rel = []
    for i in range(2 * k + 1):
        exact = F.T @ np.linalg.matrix_power(A, i) @ F
        red = R.T @ np.linalg.matrix_power(T, i) @ R
        rel.append(np.linalg.norm(exact - red) / np.linalg.norm(exact))
    assert max(rel[:2 * k]) < 1e-12
    assert rel[2 * k] > 1e-6


def test_rom_exact_when_krylov_space_is_full():
    """k p = N with a random F: the ROM NtD map equals F^T (A_+ + s^2)^{-1} F (P2)."""
    c = tiny_box((2, 2, 3), seed=2)          # 3 x 3 x 4 = 36 nodes
    sd = subdomains.decompose(c, 10.0, (2, 2, 3), m=1)[0]
    A = sd.A_plus()
    rng = np.random.default_rng(7)
    F = rng.standard_normal((sd.N, 6))
    tri = lanczos.lanczos_infinite(A, F, k=6)
    sf = sfraction.sfraction(tri)
    # The floating subdomain has a null mode, so M(s) ~ 1/s^2 near s = 0 and the
    # continued-fraction evaluation (not the coefficients) loses digits there; the
    # tridiagonal form is checked down to s = 5, the continued fraction from s = 50.
    for s in (5.0, 50.0, 300.0, 2000.0):
        exact = sfraction.ntd_resolvent(A, F, s)
        tri_val = sfraction.ntd_tridiagonal(tri, s)
        assert np.linalg.norm(tri_val - exact) / np.linalg.norm(exact) < 1e-10
        if s >= 50.0:
            cf = sfraction.ntd_continued_fraction(sf, s)
            assert np.linalg.norm(cf - exact) / np.linalg.norm(exact) < 1e-9


def test_continued_fraction_equals_tridiagonal_transfer(small_case):
    """Matrix S-fraction equals R^T (T + s^2)^{-1} R (eq. "NtDtri" vs the continued fraction; P1)."""
    cfg, c, subs, roms = small_case
    r = roms[5]
    for s in sfraction.ntd_frequencies(cfg.f_peak):
        a = sfraction.ntd_tridiagonal(r.tri, s)
        b = sfraction.ntd_continued_fraction(r.sf, s)
        assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-12


def test_sfraction_change_of_coordinates(small_case):
    """G^{-T} T G^{-1} = D^T Gamma D, G^{-T} G^{-1} = Gamma-hat^{-1}, Gamma_j > 0 for j < k (P5)."""
    cfg, c, subs, roms = small_case
    r = roms[0]
    Gd = sfraction.blockdiag(r.sf.G)
    Gi = np.linalg.inv(Gd)
    lhs = Gi.T @ r.tri.T() @ Gi
    rhs = sfraction.difference_stiffness(r.sf)
    assert np.abs(lhs - rhs).max() < 1e-9 * np.abs(rhs).max()
    hat_inv = sfraction.blockdiag([np.linalg.inv(g) for g in r.sf.gamma_hat])
    assert np.abs(Gi.T @ Gi - hat_inv).max() < 1e-9 * np.abs(hat_inv).max()
    for j in range(r.k - 1):
        assert np.linalg.eigvalsh(r.sf.gamma[j])[0] > 0


def test_sfraction_invariant_under_block_rotations(small_case):
    """Q_j -> Q_j O_j changes (A_j, B_j) but leaves Gamma_j, Gamma-hat_j unchanged (P5)."""
    cfg, c, subs, roms = small_case
    r = roms[2]
    rng = np.random.default_rng(0)
    k, p = r.k, r.p
    Os = [np.linalg.qr(rng.standard_normal((p, p)))[0] for _ in range(k)]
    A2 = [Os[j].T @ r.tri.A[j] @ Os[j] for j in range(k)]
    B2 = [Os[0].T @ r.tri.B[0]] + [Os[j].T @ r.tri.B[j] @ Os[j - 1] for j in range(1, k)]
    tri2 = lanczos.BlockTridiagonal(Z=r.tri.Z, A=A2, B=B2)
    sf2 = sfraction.sfraction(tri2)
    for j in range(k):
        scale = np.abs(r.sf.gamma[j]).max()
        assert np.abs(sf2.gamma[j] - r.sf.gamma[j]).max() < 1e-9 * scale
        scale = np.abs(r.sf.gamma_hat[j]).max()
        assert np.abs(sf2.gamma_hat[j] - r.sf.gamma_hat[j]).max() < 1e-9 * scale


@pytest.mark.parametrize("p", [1, 3])
def test_one_dimensional_optimal_grid(p):
    """1-D three-point scheme with primary steps h_j and dual steps h^_j, Neumann input and
    Dirichlet end: the S-fraction recovers Gamma_j = 1/h_j, Gamma-hat_j = 1/h^_j (Stage 2, remark
    after the scalar S-fraction; P4).  p independent chains mixed by a random orthogonal O give
    Gamma_j = O^T diag(1/h_j) O."""
    rng = np.random.default_rng(17 + p)
    k = 7
    hs = rng.uniform(0.5, 2.0, size=(p, k))
    hh = rng.uniform(0.5, 2.0, size=(p, k))
    N = p * k
    Mfine = np.zeros(N)
    Kfine = np.zeros((N, N))
    Fu = np.zeros((N, p))
    for c in range(p):
        base = c * k
        for j in range(k):
            Mfine[base + j] = hh[c, j]
            g = 1.0 / hs[c, j]
            Kfine[base + j, base + j] += g
            if j + 1 < k:
                Kfine[base + j + 1, base + j + 1] += g
                Kfine[base + j, base + j + 1] -= g
                Kfine[base + j + 1, base + j] -= g
        Fu[base, c] = 1.0
    O = np.linalg.qr(rng.standard_normal((p, p)))[0] if p > 1 else np.ones((1, 1))
    S = 1.0 / np.sqrt(Mfine)
    A = S[:, None] * Kfine * S[None, :]
    F = (S[:, None] * Fu) @ O
    tri = lanczos.block_lanczos(lambda X: A @ X, F, k)
    sf = sfraction.sfraction(tri)
    for j in range(k):
        np.testing.assert_allclose(sf.gamma[j], O.T @ np.diag(1.0 / hs[:, j]) @ O, atol=1e-10)
        np.testing.assert_allclose(sf.gamma_hat[j], O.T @ np.diag(1.0 / hh[:, j]) @ O, atol=1e-10)


def test_breakdown_on_rank_deficient_basis():
    c = tiny_box((4, 4, 4), seed=3)
    sd = subdomains.decompose(c, 10.0, (4, 4, 4), m=1)[0]
    F = sd.F().toarray()
    F = np.hstack([F, F[:, :1]])
    with pytest.raises(lanczos.LanczosBreakdown):
        lanczos.lanczos_infinite(sd.A_plus(), F, 3)


def test_homogeneous_cube_exhausts_krylov_space():
    """Cube symmetry confines the block Krylov space of a homogeneous box: with 4^3 cells and one
    patch per face the space stops growing at the third block (breakdown is an error)."""
    c = np.full((5, 5, 5), 2000.0)
    sd = subdomains.decompose(c, 10.0, (4, 4, 4), m=1)[0]
    rom.build_rom(sd, 2)
    with pytest.raises(lanczos.LanczosBreakdown):
        rom.build_rom(sd, 3)


def test_finite_shift_subspace_contains_resolvent_solutions():
    """Rational space: (A_+ + sigma)^{-1} F lies in span(Z) and F does too (Stage 1, K_n(sigma) with F added)."""
    c = tiny_box((4, 4, 4), seed=8)
    sd = subdomains.decompose(c, 10.0, (4, 4, 4), m=1)[0]
    A = sd.A_plus()
    F = sd.F().toarray()
    sigma = 3e4
    tri = lanczos.lanczos_rational(A, F, 3, sigma)
    Z = tri.Z
    X = np.linalg.solve(A.toarray() + sigma * np.eye(sd.N), F)
    for Y in (F, X):
        resid = Y - Z @ (Z.T @ Y)
        assert np.linalg.norm(resid) < 1e-10 * np.linalg.norm(Y)


def test_finite_shift_rom_interpolates_at_shift():
    """The rational ROM matches M(s) exactly at s^2 = sigma (moment matching at the shift)."""
    c = tiny_box((4, 4, 4), seed=9)
    sd = subdomains.decompose(c, 10.0, (4, 4, 4), m=1)[0]
    A, F = sd.A_plus(), sd.F()
    sigma = 2.5e4
    r = rom.build_rom(sd, 3, sigma=sigma)
    s = math.sqrt(sigma)
    exact = sfraction.ntd_resolvent(A, F, s)
    got = sfraction.ntd_continued_fraction(r.sf, s)
    assert np.linalg.norm(got - exact) / np.linalg.norm(exact) < 1e-9


# ----------------------------------------------------------------------------- projections
def test_boundary_layer_is_patch_trace(small_case):
    """U_1 = F^T v = E^T u: the boundary layer is the patch-weighted trace and is continuous
    across a shared face for any field in the ROM subspace of both sides (eq. "Uj", "mass")."""
    cfg, c, subs, roms = small_case
    rng = np.random.default_rng(4)
    for sd, r in zip(subs[:2], roms[:2]):
        y = rng.standard_normal(r.tri.Z.shape[1])
        u = sd.S * (r.tri.Z @ y)
        U = r.project_state(sd, u)
        np.testing.assert_allclose(U[0], sd.E.T @ u, rtol=1e-10, atol=1e-12 * np.abs(U[0]).max())
        np.testing.assert_allclose(r.reconstruct(sd, U), u, rtol=1e-9, atol=1e-12 * np.abs(u).max())


# ----------------------------------------------------------------------------- stepping
def _single_box_case():
    c = tiny_box((2, 2, 3), seed=21)          # 36 nodes, m = 1 -> p = 6, k = 6: k p = N
    h = 10.0
    subs = subdomains.decompose(c, h, (2, 2, 3), m=1)
    roms = rom.build_all(subs, 6)
    return c, h, subs, roms


def test_single_subdomain_full_rom_equals_fdtd():
    """One subdomain with k p = N: ROM leapfrog is a similarity transform of the FDTD (P6)."""
    c, h, subs, roms = _single_box_case()
    src = [(1, 1, 1)]
    rec = [(0, 0, 0), (2, 1, 3), (1, 1, 2), (2, 2, 0)]
    g = grid.FineGrid(c, h)
    dt = 0.9 * g.cfl_dt()
    wav = W.ricker(1.0 / (40 * dt), dt, 400)[:, None]
    cs = coupled.CoupledSystem(subs, roms, src, rec)
    tr = cs.run(dt, wav)
    ref = g.fdtd(dt, wav, src, rec)
    # Exact up to rounding: the deepest S-fraction levels are ill-conditioned (Gamma_k carries the
    # null mode of the floating box, cond ~ 1e17), so the FP64 phase error grows to ~1e-7 over
    # 400 steps; an inexact scheme would be off by O(1).
    assert np.linalg.norm(tr - ref) / np.linalg.norm(ref) < 1e-6
    assert cs.max_eig() == pytest.approx(g.max_eig(), rel=1e-9)


def test_two_subdomains_nodal_interface_equals_fdtd():
    """Two subdomains, one boundary function per interface node, k p = N per side: the coupled
    scheme of eq. "bdrytstep" reproduces the global FDTD (P7)."""
    c = tiny_box((2, 2, 4), seed=31)          # 3 x 3 x 5 nodes
    h = 10.0
    subs = subdomains.decompose(c, h, (2, 2, 2), m=0, mode="interface_nodes")
    assert [sd.p for sd in subs] == [9, 9]
    roms = rom.build_all(subs, 3)
    src = [(1, 1, 1)]
    rec = [(0, 0, 4), (1, 1, 3), (2, 0, 2), (1, 2, 0)]
    g = grid.FineGrid(c, h)
    dt = 0.9 * g.cfl_dt()
    wav = W.ricker(1.0 / (40 * dt), dt, 400)[:, None]
    cs = coupled.CoupledSystem(subs, roms, src, rec)
    tr = cs.run(dt, wav)
    ref = g.fdtd(dt, wav, src, rec)
    assert np.linalg.norm(tr - ref) / np.linalg.norm(ref) < 1e-8


def test_uneven_boxes_own_sizes_nodal_interface_equals_fdtd():
    """Boxes of 3 x 3 x 3 and 3 x 3 x 4 nodes, one boundary function per interface node and each
    ROM at its own k with k p = N (k = 3 and 4): the coupled scheme reproduces the global FDTD
    (P7 with uneven subdomains and ROM sizes)."""
    c = tiny_box((2, 2, 5), seed=33)          # 3 x 3 x 6 nodes
    h = 10.0
    subs = subdomains.decompose(c, h, (2, 2, (2, 3)), m=0, mode="interface_nodes")
    assert [sd.p for sd in subs] == [9, 9] and [sd.N for sd in subs] == [27, 36]
    roms = [rom.build_rom(subs[0], 3), rom.build_rom(subs[1], 4)]
    src = [(1, 1, 1)]
    rec = [(0, 0, 5), (1, 1, 4), (2, 0, 2), (1, 2, 0)]
    g = grid.FineGrid(c, h)
    dt = 0.9 * g.cfl_dt()
    wav = W.ricker(1.0 / (40 * dt), dt, 400)[:, None]
    cs = coupled.CoupledSystem(subs, roms, src, rec)
    tr = cs.run(dt, wav)
    ref = g.fdtd(dt, wav, src, rec)
    assert np.linalg.norm(tr - ref) / np.linalg.norm(ref) < 1e-8


def test_exchange_form_equals_assembled_operator(small_case):
    """Steps 2.1-2.3 applied to a state equal -M^{-1} K X of the assembled scheme."""
    cfg, c, subs, roms = small_case
    cs = coupled.CoupledSystem(subs, roms)
    rng = np.random.default_rng(9)
    X = rng.standard_normal(cs._dof_layout()[1])
    M, K, _ = cs.assemble()
    import scipy.sparse.linalg as spla
    ref = -spla.spsolve(M.tocsc(), K @ X)
    got = cs.gather(cs.accel(cs.scatter(X)))
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-9


def test_energy_conserved(small_case):
    """Leapfrog energy 1/2|X^{n+1}-X^n|_M^2/dt^2 + 1/2 X^{n+1}K X^n is constant without forcing (P8)."""
    cfg, c, subs, roms = small_case
    cs = coupled.CoupledSystem(subs, roms)
    M, K, _ = cs.assemble()
    dt = 0.9 * cs.cfl_dt()
    rng = np.random.default_rng(2)
    U = cs.scatter(rng.standard_normal(cs._dof_layout()[1]))
    Up = [u.copy() for u in U]
    energies = []
    for n in range(300):
        a = cs.accel(U)
        Un = [2 * u - up + dt * dt * aa for u, up, aa in zip(U, Up, a)]
        Up, U = U, Un
        energies.append(cs.energy(M, K, cs.gather(U), cs.gather(Up), dt))
    e = np.array(energies)
    assert np.abs(e - e[0]).max() / abs(e[0]) < 1e-10


@pytest.mark.parametrize("factor, grows", [(0.99, False), (1.01, True)])
def test_rom_cfl_transition(small_case, factor, grows):
    """dt_max = 2/sqrt(rho) of the coupled ROM: bounded below it, exponential growth above (P9)."""
    cfg, c, subs, roms = small_case
    cs = coupled.CoupledSystem(subs, roms, rec_ijk=[(5, 5, 0)])
    dt = factor * cs.cfl_dt()
    rng = np.random.default_rng(6)
    U = cs.scatter(rng.standard_normal(cs._dof_layout()[1]))
    tr = cs.run(dt, np.zeros((400, 0)), U0=U, U_prev=U)
    assert (np.abs(tr).max() > 1e3 * np.abs(cs.record(U)).max() + 1e6) == grows


def test_cfl_bounded_by_subdomain_spectra(small_case):
    """rho(coupled) <= max_alpha lambda_max(T^alpha) (mediant of Rayleigh quotients)."""
    cfg, c, subs, roms = small_case
    cs = coupled.CoupledSystem(subs, roms)
    assert cs.max_eig() <= coupled.subdomain_bound(roms) * (1 + 1e-12)


def test_partitioned_exchange_is_bit_identical(small_case):
    """Two 'ranks' that exchange only boundary-layer face rows give bit-identical traces (section on
    communication: only m numbers per shared face cross a partition)."""
    cfg, c, subs, roms = small_case
    cs = coupled.CoupledSystem(subs, roms, cfg.sources(), cfg.receivers())
    dt = 0.9 * cs.cfl_dt()
    wav = W.ricker(cfg.f_peak, dt, 60)[:, None]
    ref = cs.run(dt, wav)
    rank_of = [sd.box[2] for sd in subs]      # split along z
    U = cs.zero_state()
    Up = cs.zero_state()
    out = np.empty_like(ref)
    for n in range(60):
        phis = cs.fluxes(U)
        partial = []
        for rank in (0, 1):
            mine = [a for a in range(len(subs)) if rank_of[a] == rank]
            partial.append(cs.exchange(phis, subset=mine))
        # each rank receives the other's face rows only for ports it shares
        total = partial[0] + partial[1]
        acc = cs._finish(U, phis, total, wav[n])
        Un = [2 * u - up + dt * dt * a for u, up, a in zip(U, Up, acc)]
        Up, U = U, Un
        out[:, n] = cs.record(U)
    assert np.array_equal(out, ref)


def test_checkpoint_resume_bit_identical(small_case):
    cfg, c, subs, roms = small_case
    cs = coupled.CoupledSystem(subs, roms, cfg.sources(), cfg.receivers())
    dt = 0.9 * cs.cfl_dt()
    wav = W.ricker(cfg.f_peak, dt, 80)[:, None]
    full = cs.run(dt, wav)
    a, U, Up = cs.run(dt, wav[:40], return_state=True)
    b = cs.run(dt, wav[40:], U0=U, U_prev=Up)
    assert np.array_equal(np.hstack([a, b]), full)


def test_sigma_infinity_ntd_errors_match_moment_count(small_case):
    """sigma = inf ROM of a corner subdomain: NtD error decreases with s (polynomial moments are
    matched at s = infinity); recorded values guard against regressions of the basis F."""
    cfg, c, subs, roms = small_case
    sd, r = subs[0], roms[0]
    errs = [sfraction.ntd_rel_error(sd.A_plus(), sd.F(), r.sf, [s])
            for s in sfraction.ntd_frequencies(cfg.f_peak)]
    assert all(a > b for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-3


# ----------------------------------------------------------------------------- paper numbers
def test_e1_rom_size_arithmetic():
    """Numerical experiments section: 6 m n ROM unknowns per unit cube with m = 25, n = 3 give about
    six unknowns per minimal wavelength per dimension, against 16 fine-grid points (P11)."""
    with open(os.path.join(GOLDEN, "e1_sizes.json")) as fh:
        g = json.load(fh)
    dof = 6 * g["m"] * g["n_blocks"]
    assert dof == 450
    per_dim = dof ** (1.0 / 3.0) * g["lambda_min"]
    assert round(per_dim) == g["rom_dof_per_wavelength_per_dimension"]
    assert round(g["subdomain_nodes_per_unit_length"] * g["lambda_min"]) == g["fine_points_per_wavelength"]


# ----------------------------------------------------------------------------- per-subdomain ROM size
@pytest.mark.parametrize("k2", [2, 5])
def test_rom_of_fewer_levels_is_the_leading_part(small_case, k2):
    """Stage 1 with k2 < k steps on a subdomain gives the first k2 blocks of the k-step result:
    block Lanczos and the S-fraction recursion (G_1 = B_1^T, Gamma_j from A_j, G_j and Gamma_{j-1})
    run forward in j, so Gamma_j, Gamma-hat_j, G_j and the source / receiver maps of levels j <= k2
    do not depend on the later steps.  Checked against an independent k2-step build."""
    cfg, c, subs, roms = small_case
    for a in (0, 5):
        sd, big = subs[a], roms[a]
        small = rom.build_rom(sd, k2)
        assert small.k == k2
        for name in ("gamma", "gamma_hat", "G"):
            x = np.stack(getattr(small.sf, name))
            y = np.stack(getattr(big.sf, name))[:k2]
            assert np.abs(x - y).max() <= 1e-12 * np.abs(y).max(), name
        for node in (0, sd.N // 3, sd.N - 1):
            np.testing.assert_allclose(small.source_vector(sd, node), big.source_vector(sd, node)[:k2],
                                       rtol=0, atol=1e-12 * np.abs(big.source_vector(sd, node)).max())
            np.testing.assert_allclose(small.receiver_row(sd, node), big.receiver_row(sd, node)[:k2],
                                       rtol=0, atol=1e-10 * np.abs(big.receiver_row(sd, node)).max())


def _mixed_system(small_case, seed=21):
    cfg, c, subs, roms = small_case
    rng = np.random.default_rng(seed)
    ks = rng.integers(2, cfg.k + 1, size=len(subs))
    ks[0], ks[-1] = cfg.k, 2
    return coupled.CoupledSystem(subs, [rom.build_rom(sd, int(kk)) for sd, kk in zip(subs, ks)])


def test_mixed_sizes_exchange_form_and_energy(small_case):
    """Subdomain ROMs of different sizes couple through the boundary layer alone (steps 2.1-2.3):
    the exchange form equals -M^{-1} K X of the assembled scheme, and leapfrog energy is constant."""
    cs = _mixed_system(small_case)
    assert len({r.k for r in cs.roms}) > 2
    M, K, _ = cs.assemble()
    import scipy.sparse.linalg as spla
    rng = np.random.default_rng(4)
    X = rng.standard_normal(cs._dof_layout()[1])
    ref = -spla.spsolve(M.tocsc(), K @ X)
    assert np.linalg.norm(cs.gather(cs.accel(cs.scatter(X))) - ref) / np.linalg.norm(ref) < 1e-9
    dt = 0.9 * cs.cfl_dt()
    U = cs.scatter(rng.standard_normal(cs._dof_layout()[1]))
    Up = [u.copy() for u in U]
    e = []
    for n in range(200):
        acc = cs.accel(U)
        Un = [2 * u - up + dt * dt * aa for u, up, aa in zip(U, Up, acc)]
        Up, U = U, Un
        e.append(cs.energy(M, K, cs.gather(U), cs.gather(Up), dt))
    e = np.array(e)
    assert np.abs(e - e[0]).max() / abs(e[0]) < 1e-10
    assert cs.max_eig() <= coupled.subdomain_bound(cs.roms) * (1 + 1e-12)
