"""Oracle-side fixtures shared by the GPU parity tests (CPU only, FP64)."""
from __future__ import annotations

import functools

import numpy as np
import scipy.sparse as sp

import workloads as W
from oracle import coupled, grid, lanczos, rom, sfraction, subdomains


def case_config(name: str) -> W.Workload:
    """Workload of a named parity case."""
    if name == "small":
        cfg = W.CFG_SMALL
    elif name == "ragged":
        # p = 6 * 3 = 18 (not a multiple of 16) on a 3 x 2 x 2 split with uneven boxes
        cfg = W.Workload(name="ragged_p18", ncell=(30, 20, 24), sub_cells=(10, 10, 12), h=10.0, m=3, k=5,
                         f_peak=15.0, nsteps=300, src=((14, 7, 5),), rec_grid=(10, 8),
                         velocity="layered_inclusions", seed=5)
    elif name == "uneven":
        # a tensor product of boxes of uneven size: 2 x 2 x 2 boxes from (12, 16) x (8, 12) x (10, 8)
        cfg = W.Workload(name="uneven_28x20x18", ncell=(28, 20, 18), sub_cells=((12, 16), (8, 12), (10, 8)),
                         h=10.0, m=4, k=5, f_peak=15.0, nsteps=300, src=((3, 3, 4),), rec_grid=(10, 8),
                         velocity="layered_inclusions", seed=9)
    elif name == "mid":
        # The large workload's subdomain size and ROM sizes (33^3 nodes, m = 16, k = 16) on 2 x 2 x 1.
        cfg = W.scaled_large((2, 2, 1), nsteps=150)
    elif name in ("m8", "m12"):
        # 32^3-cell boxes on a 2 x 2 x 2 split with k = 16: m = 8 gives 6m = 48 (three 16-row tiles,
        # the learned-ROM workload's shape), m = 12 gives 6m = 72 padded to 80 (five tiles, the
        # gradient and many-shot workloads' shape).  Odd tile counts take the single-strip middle
        # job of the step, adjoint and operator kernels.
        m = 8 if name == "m8" else 12
        cfg = W.Workload(name=f"layered_64c_2x2x2_m{m}_k16", ncell=(64, 64, 64), sub_cells=(32, 32, 32),
                         h=10.0, m=m, k=16, f_peak=12.0, nsteps=500, src=((31, 31, 2),), rec_grid=(32, 32),
                         velocity="layered_inclusions", seed=1406 + m)
    elif name in ("m18", "m24"):
        # Wide blocks with few levels: 16^3-cell boxes on a 2 x 2 x 2 split, k = 3; m = 18 gives
        # 6m = 108 (seven 16-row tiles), m = 24 gives 6m = 144 (nine).  Past 6m = 100 the stability
        # certificate's factor-and-solve no longer fits LDS, past 6m = 143 neither does its
        # Cholesky: both run on global memory there.
        m = 18 if name == "m18" else 24
        cfg = W.Workload(name=f"layered_32c_2x2x2_m{m}_k3", ncell=(32, 32, 32), sub_cells=(16, 16, 16),
                         h=10.0, m=m, k=3, f_peak=15.0, nsteps=200, src=((15, 15, 2),), rec_grid=(16, 16),
                         velocity="layered_inclusions", seed=1406 + m)
    else:
        raise KeyError(name)
    return cfg


@functools.lru_cache(maxsize=6)
def oracle_case(name: str = "small", sigma: float = np.inf):
    """Build the oracle ROMs and coupled system of a named workload."""
    cfg = case_config(name)
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


def level_table(S: int, k: int, seed: int) -> np.ndarray:
    """Seeded ROM size per subdomain in [2, k]; the first subdomain keeps k, the last takes 2."""
    rng = np.random.default_rng(seed)
    ks = rng.integers(2, k + 1, size=S)
    ks[0], ks[-1] = k, 2
    return ks.astype(np.int32)


@functools.lru_cache(maxsize=4)
def mixed_level_case(name: str = "small", seed: int = 21):
    """The named case with every subdomain's ROM built by the oracle at its own size k_s
    (Algorithm 1, Stage 1 per subdomain): (cfg, subs, roms_ks, cs_ks, ks)."""
    cfg, c, subs, roms, cs = oracle_case(name)
    ks = level_table(len(subs), cfg.k, seed)
    roms_ks = [rom.build_rom(sd, int(kk)) for sd, kk in zip(subs, ks)]
    cs_ks = coupled.CoupledSystem(subs, roms_ks, cfg.sources(), cfg.receivers())
    return cfg, subs, roms_ks, cs_ks, ks


def pad_levels(U, k: int) -> np.ndarray:
    """Per-subdomain [k_s][...] arrays stacked into [S][k][...] with zero levels past k_s."""
    out = np.zeros((len(U), k) + np.asarray(U[0]).shape[1:])
    for a, Ua in enumerate(U):
        out[a, :len(Ua)] = Ua
    return out


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


def _level_changes(sf, r) -> np.ndarray:
    out = np.empty(r.k)
    for j in range(r.k):
        out[j] = max(np.abs(sf.gamma[j] - r.sf.gamma[j]).max() / np.abs(r.sf.gamma[j]).max(),
                     np.abs(sf.gamma_hat[j] - r.sf.gamma_hat[j]).max() / np.abs(r.sf.gamma_hat[j]).max())
    return out


def solve_perturbation_profile(sd, r, sigma: float, rtol: float, seed: int = 2) -> np.ndarray:
    """Per-level change of the finite-shift coefficients when every shifted solve is inexact.

    An iterative solve stopped at |b - (A_+ + sigma) x| <= rtol |b| returns the exact solution
    for a right-hand side moved by a residual of relative size rtol; the oracle is rebuilt with
    each column of every right-hand side moved by a random vector of exactly that size.  The
    result is the coefficient change a correct solver at that tolerance can produce."""
    rng = np.random.default_rng(seed)

    def noisy(solve, X):
        X = np.asarray(X)
        R = rng.standard_normal(X.shape)
        R *= rtol * np.linalg.norm(X, axis=0) / np.linalg.norm(R, axis=0)
        return solve(X + R)

    sf = sfraction.sfraction(lanczos.lanczos_rational(sd.A_plus(), sd.F(), r.k, sigma, solve_hook=noisy))
    return _level_changes(sf, r)


def perturbation_profile(sd, r, delta: float = 1e-15, seed: int = 1, sigma: float = np.inf) -> np.ndarray:
    """Per-level reproducibility of the S-fraction coefficients in FP64.

    The subdomain operator's entries are perturbed by a symmetric relative noise of size delta
    and the oracle ROM is rebuilt; the returned array holds, for each level j, the largest
    relative change (max-norm) of Gamma_j and Gamma-hat_j.  Deep levels of a polynomial-Krylov
    S-fraction respond to rounding-size perturbations of the operator by orders of magnitude
    more than shallow ones, so two correct FP64 builds can only agree to about this level."""
    A = sd.A_plus().tocoo()
    rng = np.random.default_rng(seed)
    upper = A.row <= A.col
    noise = np.zeros(A.nnz)
    noise[upper] = delta * rng.standard_normal(int(upper.sum()))
    Ap = sp.coo_matrix((A.data * (1 + noise), (A.row, A.col)), shape=A.shape).tocsr()
    Ap = (sp.triu(Ap) + sp.triu(Ap, 1).T).tocsr()
    if np.isinf(sigma):
        tri = lanczos.lanczos_infinite(Ap, sd.F(), r.k)
    else:
        tri = lanczos.lanczos_rational(Ap, sd.F(), r.k, sigma)
    return _level_changes(sfraction.sfraction(tri), r)


def level_tolerance(profile: np.ndarray) -> np.ndarray:
    """Coefficient tolerance per level: 30 times the FP64 reproducibility, at least 1e-14."""
    return np.maximum(30.0 * profile, 1e-14)


@functools.lru_cache(maxsize=4)
def case_level_tolerance(name: str) -> np.ndarray:
    """Per-level tolerance of a named case: the worst perturbation response over two subdomains."""
    cfg, c, subs, roms, cs = oracle_case(name)
    picks = sorted({0, len(subs) - 1})
    prof = np.max([perturbation_profile(subs[i], roms[i]) for i in picks], axis=0)
    return level_tolerance(prof)


# Shift of the finite-sigma cases in units of (2 pi f_peak)^2, the squared peak angular frequency.
# At k = 16, p = 96 the S-fraction of the rational space for (2 pi f_peak)^2 is not positive
# definite even in FP64 (Gamma_15 has an eigenvalue ratio of 5e-17 and Gamma-hat_16 a negative
# eigenvalue on the 33^3 case): the coefficients spread geometrically over the levels, faster
# the closer the shift is to the bottom of the spectrum; 16 (2 pi f_peak)^2 keeps every level
# positive definite with ratios above 1e-12 there.
SIGMA_FACTOR = {"small": 1.0, "ragged": 1.0, "mid": 16.0}


def case_sigma(name: str, factor: float = None) -> float:
    """Shift of a finite-sigma case: SIGMA_FACTOR[name] (or factor) times (2 pi f_peak)^2."""
    f = SIGMA_FACTOR[name] if factor is None else factor
    return float(f * (2.0 * np.pi * case_config(name).f_peak) ** 2)


@functools.lru_cache(maxsize=4)
def shifted_level_tolerance(name: str, rtol: float) -> np.ndarray:
    """Per-level tolerance of a finite-sigma build with inner solves at rtol: 30 times the larger of
    the FP64 operator-perturbation response and the inexact-solve response, over two subdomains."""
    sigma = case_sigma(name)
    cfg, c, subs, roms, cs = oracle_case(name, sigma)
    picks = sorted({0, len(subs) - 1})
    prof = np.max([np.maximum(perturbation_profile(subs[i], roms[i], sigma=sigma),
                              solve_perturbation_profile(subs[i], roms[i], sigma, rtol)) for i in picks], axis=0)
    return level_tolerance(prof)


def interpolation_error(sd, sf, sigma: float) -> float:
    """Relative Frobenius error of a ROM's NtD map against the exact one at s^2 = sigma."""
    s = float(np.sqrt(sigma))
    exact = sfraction.ntd_resolvent(sd.A_plus(), sd.F(), s)
    return float(np.linalg.norm(sfraction.ntd_continued_fraction(sf, s) - exact) / np.linalg.norm(exact))


def shifted_interp_tolerance(sd, r, sigma: float, rtol: float, seed: int = 3) -> float:
    """Bound on the interpolation error at s^2 = sigma of a finite-shift ROM built with inner solves
    at rtol: 30 times the larger of the oracle ROM's error and that of an oracle ROM whose every
    shifted solve carries a residual of relative size rtol (as in solve_perturbation_profile)."""
    rng = np.random.default_rng(seed)

    def noisy(solve, X):
        X = np.asarray(X)
        R = rng.standard_normal(X.shape)
        R *= rtol * np.linalg.norm(X, axis=0) / np.linalg.norm(R, axis=0)
        return solve(X + R)

    sf_noisy = sfraction.sfraction(lanczos.lanczos_rational(sd.A_plus(), sd.F(), r.k, sigma, solve_hook=noisy))
    e = max(interpolation_error(sd, r.sf, sigma), interpolation_error(sd, sf_noisy, sigma), 1e-15)
    return 30.0 * e



U32 = 2.0 ** -24


def operator_error_bound(cs: coupled.CoupledSystem, U: np.ndarray, tau=None) -> np.ndarray:
    """Elementwise first-order bound, times 2, on |a_gpu - a_oracle| for one application of the
    coupled step operator with FP32 coefficients and state, [S][k][p].

    The kernels round every stored coefficient to FP32 (relative u = 2^-24), form
    x_j = U_{j+1} - U_j (one rounding), phi_j = Gamma_j x_j as FP32 dot products of length p
    (error below p u sum |Gamma_j||x_j|), y_j = phi_j - phi_{j-1} (one rounding) and
    a_j = Gamma-hat_j y_j; on the boundary layer a_f = C_f (phi_f^alpha + phi_f^beta) with C_f, the
    sum and the product rounded once each.  tau[j] (optional) adds a relative coefficient
    difference per level (device-built ROMs against the oracle's)."""
    out = []
    phis, dphis = [], []
    for a, rom in enumerate(cs.roms):
        k, p = rom.k, rom.p
        tj = np.zeros(k) if tau is None else np.asarray(tau)
        Ua = np.asarray(U[a], dtype=np.float64)
        dU = np.vstack([Ua[1:], np.zeros((1, p))]) - Ua
        phi = np.stack([rom.sf.gamma[j] @ dU[j] for j in range(k)])
        dphi = np.stack([((p + 2) * U32 + tj[j]) * (np.abs(rom.sf.gamma[j]) @ np.abs(dU[j])) + U32 * np.abs(phi[j])
                         for j in range(k)])
        phis.append(phi)
        dphis.append(dphi)
        b = np.zeros((k, p))
        for j in range(1, k):
            y = phi[j] - phi[j - 1]
            dy = dphi[j] + dphi[j - 1] + U32 * np.abs(y)
            Gh = np.abs(rom.sf.gamma_hat[j])
            b[j] = Gh @ dy + ((p + 1) * U32 + tj[j]) * (Gh @ np.abs(y)) + U32 * np.abs(rom.sf.gamma_hat[j] @ y)
        out.append(b)
    flux = np.zeros(cs.n_ports)
    dflux = np.zeros(cs.n_ports)
    for a in range(len(cs.roms)):
        np.add.at(flux, cs.port_ids[a], np.abs(phis[a][0]))
        np.add.at(dflux, cs.port_ids[a], dphis[a][0])
    for a in range(len(cs.roms)):
        ids = cs.port_ids[a]
        out[a][0] = cs.C[ids] * (dflux[ids] + 3 * U32 * flux[ids])
    return 2.0 * np.stack(out) + 1e-300
