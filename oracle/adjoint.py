"""Discrete adjoint of the coupled leapfrog scheme: misfit gradients with respect to the
S-fraction blocks (the FWI use the Introduction names as motivation).

Oracle code (test infrastructure): plain FP64 NumPy/SciPy, no blocking or fusion.

Forward scheme (Stage 2 section, end): on the global unknowns X (shared boundary entries once,
then every subdomain's layers 2..k)

    X^{n+1} = 2 X^n - X^{n-1} + dt^2 (A X^n + b f^n),   A = -M^{-1} K,   X^0 = X^{-1} = 0,

with the assembled pair (M, K) of ``CoupledSystem.assemble`` (M^{-1} = Gamma-hat_j on interior
layers and C_f on the boundary entries; K = sum over subdomains of D^T Gamma D, D the layer
differences (D U)_j = U_{j+1} - U_j with U_{k+1} = 0).  Trace sample n is t^n = R X^{n+1}.

Misfit J = 1/2 sum_n ||t^n - d^n||^2.  Its discrete adjoint (reverse of the recursion above):

    psi^m = R^T (t^{m-1} - d^{m-1}) + 2 psi^{m+1} - psi^{m+2} + dt^2 A^T psi^{m+1},  m = N..1,
    psi^{N+1} = psi^{N+2} = 0,   A^T = -K M^{-1},

and for a parameter theta of A,  dJ/dtheta = sum_{n=0}^{N-1} dt^2 <psi^{n+1}, (dA/dtheta) X^n>.
With z = M^{-1} psi scattered to the subdomains:

    dJ/dGamma_j^a     = -dt^2 sum_n sym( (D z^{n+1,a})_j (D X^{n,a})_j^T ),          j = 1..k
    dJ/dGamma-hat_j^a =  dt^2 sum_n sym( psi_j^{n+1,a} (-K X^{n,a})_j^T ),            j = 2..k

where (-K X^a)_j = phi_j - phi_{j-1} is the interior-layer flux difference of the forward step.
Gamma-hat_1 (the face masses) and the source / receiver projections are held fixed.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

from .coupled import CoupledSystem


def _sym(a: np.ndarray) -> np.ndarray:
    return 0.5 * (a + a.T)


def forward(cs: CoupledSystem, dt: float, wavelets: np.ndarray):
    """Leapfrog from rest; returns traces [nrec][N] and the states X^0..X^N (per subdomain)."""
    wavelets = np.asarray(wavelets, dtype=np.float64).reshape(len(wavelets), -1)
    N = wavelets.shape[0]
    U = cs.zero_state()
    Up = cs.zero_state()
    states = [U]
    traces = np.empty((len(cs.receivers), N))
    for n in range(N):
        acc = cs.accel(U, wavelets[n] if cs.sources else ())
        Un = [2.0 * u - up + dt * dt * a for u, up, a in zip(U, Up, acc)]
        Up, U = U, Un
        states.append(U)
        traces[:, n] = cs.record(U)
    return traces, states


def misfit(traces: np.ndarray, observed: np.ndarray) -> float:
    r = np.asarray(traces) - np.asarray(observed)
    return 0.5 * float(np.sum(r * r))


class Adjoint:
    """A^T and R^T on the global unknowns, from the assembled (M, K)."""

    def __init__(self, cs: CoupledSystem):
        self.cs = cs
        _, K, _ = cs.assemble()
        self.K = K.tocsr()
        self.offs, self.n = cs._dof_layout()

    def minv(self, psi: np.ndarray) -> np.ndarray:
        """M^{-1} psi block by block: C_f on the boundary entries, Gamma-hat_j on interior layers."""
        out = np.zeros(self.n)
        out[:self.cs.n_ports] = self.cs.C * psi[:self.cs.n_ports]
        for a, rom in enumerate(self.cs.roms):
            p = rom.p
            for j in range(1, rom.k):
                sl = slice(self.offs[a] + (j - 1) * p, self.offs[a] + j * p)
                out[sl] = rom.sf.gamma_hat[j] @ psi[sl]
        return out

    def apply_transpose(self, psi: np.ndarray) -> np.ndarray:
        """A^T psi = -K M^{-1} psi."""
        return -(self.K @ self.minv(psi))

    def receiver_transpose(self, resid: np.ndarray) -> np.ndarray:
        """R^T resid: each receiver row added to the unknowns of the subdomain that records it."""
        out = np.zeros(self.n)
        for e, (a, row) in zip(resid, self.cs.receivers):
            ids = self.cs.port_ids[a]
            np.add.at(out, ids, e * row[0])
            out[self.offs[a]:self.offs[a] + row[1:].size] += e * row[1:].ravel()
        return out


def interior_flux_difference(cs: CoupledSystem, U: List[np.ndarray]) -> List[np.ndarray]:
    """(-K U^a)_j = phi_j - phi_{j-1} per subdomain, j = 2..k (row 0 unused, zero)."""
    out = []
    for phi in cs.fluxes(U):
        d = np.zeros_like(phi)
        d[1:] = phi[1:] - phi[:-1]
        out.append(d)
    return out


def layer_differences(U: List[np.ndarray]) -> List[np.ndarray]:
    """(D U^a)_j = U_{j+1} - U_j, U_{k+1} = 0."""
    return [np.vstack([Ua[1:], np.zeros((1, Ua.shape[1]))]) - Ua for Ua in U]


def gradient(cs: CoupledSystem, dt: float, wavelets: np.ndarray, observed: np.ndarray):
    """Misfit J and its gradient: (J, grad_gamma [S][k][p][p], grad_gamma_hat [S][k][p][p]);
    grad_gamma_hat[:, 0] is zero (face masses held fixed).  With subdomain ROMs of different
    sizes k is the largest; the blocks past a subdomain's own k are zero."""
    traces, X = forward(cs, dt, wavelets)
    J = misfit(traces, observed)
    resid = traces - np.asarray(observed)
    N = resid.shape[1]
    adj = Adjoint(cs)
    S = len(cs.roms)
    k, p = max(r.k for r in cs.roms), cs.roms[0].p
    g_gam = np.zeros((S, k, p, p))
    g_hat = np.zeros((S, k, p, p))
    psi1 = np.zeros(adj.n)          # psi^{m+1}
    psi2 = np.zeros(adj.n)          # psi^{m+2}
    for m in range(N, 0, -1):
        psi = adj.receiver_transpose(resid[:, m - 1]) + 2.0 * psi1 - psi2 + dt * dt * adj.apply_transpose(psi1)
        # psi^m is known; the parameter term of step n = m - 1 pairs psi^m with X^{m-1}
        n = m - 1
        if n >= 1:                  # X^0 = 0 contributes nothing
            z = cs.scatter(adj.minv(psi))
            pz = cs.scatter(psi)
            Dz = layer_differences(z)
            DX = layer_differences(X[n])
            KX = interior_flux_difference(cs, X[n])
            for a in range(S):
                for j in range(cs.roms[a].k):
                    g_gam[a, j] -= dt * dt * np.outer(Dz[a][j], DX[a][j])
                    if j >= 1:
                        g_hat[a, j] += dt * dt * np.outer(pz[a][j], KX[a][j])
        psi2, psi1 = psi1, psi
    for a in range(S):
        for j in range(k):
            g_gam[a, j] = _sym(g_gam[a, j])
            g_hat[a, j] = _sym(g_hat[a, j])
    return J, g_gam, g_hat


def perturbed_system(cs: CoupledSystem, dgam: Sequence[np.ndarray], dhat: Sequence[np.ndarray],
                     eps: float) -> CoupledSystem:
    """The coupled system with Gamma_j += eps dgam[a][j] and Gamma-hat_j += eps dhat[a][j] (j >= 2),
    sources and receivers projected with the unperturbed ROMs (held fixed as in ``gradient``)."""
    import copy
    roms = []
    for a, rom in enumerate(cs.roms):
        r = copy.copy(rom)
        sf = copy.copy(rom.sf)
        sf.gamma = [g + eps * d for g, d in zip(rom.sf.gamma, dgam[a])]
        sf.gamma_hat = [rom.sf.gamma_hat[0]] + [g + eps * d for g, d in zip(rom.sf.gamma_hat[1:], dhat[a][1:])]
        r.sf = sf
        roms.append(r)
    out = copy.copy(cs)
    out.roms = roms
    return out
