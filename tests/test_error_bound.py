"""The elementwise forward error bound the GPU operator tests use (tests.cases.operator_error_bound),
checked on the oracle alone (CPU): it covers what it is meant to cover and is not vacuous."""
import numpy as np

from tests.cases import U32, operator_error_bound, oracle_case, random_consistent_state


def _rounded_operator(cs, U):
    """The coupled operator with every coefficient rounded to FP32, evaluated in FP64."""
    f32 = lambda a: a.astype(np.float32).astype(np.float64)     # noqa: E731
    phis, out = [], []
    for a, rom in enumerate(cs.roms):
        Ua = U[a]
        dU = np.vstack([Ua[1:], np.zeros((1, rom.p))]) - Ua
        phi = [f32(rom.sf.gamma[j]) @ dU[j] for j in range(rom.k)]
        o = np.zeros_like(Ua)
        for j in range(1, rom.k):
            o[j] = f32(rom.sf.gamma_hat[j]) @ (phi[j] - phi[j - 1])
        phis.append(phi)
        out.append(o)
    flux = np.zeros(cs.n_ports)
    for a in range(len(cs.roms)):
        np.add.at(flux, cs.port_ids[a], phis[a][0])
    for a in range(len(cs.roms)):
        ids = cs.port_ids[a]
        out[a][0] = f32(cs.C[ids]) * flux[ids]
    return np.stack(out)


def test_bound_covers_fp32_coefficients():
    cfg, c, subs, roms, cs = oracle_case("small")
    U = random_consistent_state(cs, seed=3).astype(np.float32).astype(np.float64)
    ref = np.stack(cs.accel(list(U)))
    bound = operator_error_bound(cs, U)
    ratio = np.abs(_rounded_operator(cs, U) - ref) / bound
    assert ratio.max() < 0.5
    assert U32 == 2.0 ** -24


def test_bound_rejects_a_dropped_term():
    """phi_{j-1} left out of one interior layer, or one face side's flux left out, is far outside."""
    cfg, c, subs, roms, cs = oracle_case("small")
    U = random_consistent_state(cs, seed=4).astype(np.float32).astype(np.float64)
    ref = np.stack(cs.accel(list(U)))
    bound = operator_error_bound(cs, U)
    rom = cs.roms[0]
    dU = np.vstack([U[0][1:], np.zeros((1, rom.p))]) - U[0]
    wrong = ref.copy()
    wrong[0, 3] = rom.sf.gamma_hat[3] @ (rom.sf.gamma[3] @ dU[3])
    assert np.max(np.abs(wrong - ref) / bound) > 100.0
    wrong = ref.copy()
    phi1 = rom.sf.gamma[0] @ dU[0]
    wrong[0, 0] = cs.C[cs.port_ids[0]] * phi1          # the neighbours' share of the flux dropped
    shared = np.bincount(np.concatenate(cs.port_ids), minlength=cs.n_ports)[cs.port_ids[0]] > 1
    assert np.max((np.abs(wrong - ref) / bound)[0, 0][shared]) > 100.0
