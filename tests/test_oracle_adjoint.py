"""Pins of the oracle's discrete adjoint (CPU, FP64).

* A^T from the assembled stiffness (-K M^{-1}) against the per-subdomain steps 2.1-2.3 of
  ``CoupledSystem.accel`` through a dot-product test <psi, A x> = <A^T psi, x>;
* the gradient against central finite differences of the oracle's own forward misfit on 20
  random symmetric directions over every Gamma_j and Gamma-hat_j (j >= 2) block, with one ROM
  size for all subdomains and with a seeded size per subdomain;
* zero residual gives a zero gradient.
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, coupled
from tests.cases import mixed_level_case, oracle_case


@pytest.fixture(scope="module")
def small():
    return oracle_case("small")


def test_adjoint_transpose_dot_product(small):
    cfg, c, subs, roms, cs = small
    adj = adjoint.Adjoint(cs)
    rng = np.random.default_rng(3)
    cs0 = coupled.CoupledSystem(subs, roms, (), ())
    for _ in range(3):
        x = rng.standard_normal(adj.n)
        psi = rng.standard_normal(adj.n)
        ax = cs0.gather(cs0.accel(cs0.scatter(x)))
        lhs = psi @ ax
        rhs = adj.apply_transpose(psi) @ x
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.linalg.norm(ax) * np.linalg.norm(psi))


def _case(cs, cfg, nsteps=120):
    dt = 0.9 * cs.cfl_dt()
    wav = W.ricker(cfg.f_peak, dt, nsteps)[:, None]
    traces, _ = adjoint.forward(cs, dt, wav)
    rng = np.random.default_rng(11)
    observed = 0.7 * traces + 0.05 * np.abs(traces).max() * rng.standard_normal(traces.shape)
    return dt, wav, observed


@pytest.mark.parametrize("levels", ["uniform", "mixed"])
def test_adjoint_gradient_matches_central_differences(small, levels):
    cfg, c, subs, roms, cs = small
    if levels == "mixed":                    # every subdomain's ROM at its own size
        cfg, subs, roms, cs, _ = mixed_level_case("small")
    dt, wav, observed = _case(cs, cfg)
    J, g_gam, g_hat = adjoint.gradient(cs, dt, wav, observed)
    assert J > 0 and np.abs(g_gam).max() > 0 and np.abs(g_hat[:, 1:]).max() > 0
    assert not g_hat[:, 0].any()
    rng = np.random.default_rng(5)
    worst = 0.0
    for _ in range(20):
        dgam, dhat = [], []
        for rom in roms:
            dg = [rng.standard_normal((rom.p, rom.p)) for _ in range(rom.k)]
            dh = [rng.standard_normal((rom.p, rom.p)) for _ in range(rom.k)]
            dgam.append([np.abs(g).max() * (x + x.T) / 2 for g, x in zip(rom.sf.gamma, dg)])
            dhat.append([np.abs(g).max() * (x + x.T) / 2 for g, x in zip(rom.sf.gamma_hat, dh)])
        pred = sum(np.sum(g_gam[a, j] * dgam[a][j]) + (np.sum(g_hat[a, j] * dhat[a][j]) if j else 0.0)
                   for a in range(len(roms)) for j in range(roms[a].k))
        eps = 1e-6
        Jp = adjoint.misfit(adjoint.forward(adjoint.perturbed_system(cs, dgam, dhat, eps), dt, wav)[0], observed)
        Jm = adjoint.misfit(adjoint.forward(adjoint.perturbed_system(cs, dgam, dhat, -eps), dt, wav)[0], observed)
        fd = (Jp - Jm) / (2 * eps)
        err = abs(fd - pred) / max(abs(fd), abs(pred))
        worst = max(worst, err)
        assert err < 1e-5, (fd, pred, err)
    print(f"adjoint vs central differences, 20 directions: worst relative difference {worst:.2e}")


def test_adjoint_zero_residual_zero_gradient(small):
    cfg, c, subs, roms, cs = small
    dt = 0.9 * cs.cfl_dt()
    wav = W.ricker(cfg.f_peak, dt, 60)[:, None]
    traces, _ = adjoint.forward(cs, dt, wav)
    J, g_gam, g_hat = adjoint.gradient(cs, dt, wav, traces)
    assert J == 0.0 and not g_gam.any() and not g_hat.any()
