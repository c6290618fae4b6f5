"""Algorithm 1, Stage 1, for one subdomain (steps 1.1-1.4) and the coordinate map of eq. "Uj".

A subdomain ROM is the S-fraction (Gamma_j, Gamma-hat_j) of the block
tridiagonal form of its projected NtD system, plus the maps between fine-grid
fields and ROM layer vectors U_j:

* eq. "Uj" with v = M^{1/2} u:   U = G Z^T M^{1/2} u            (state, step 1.4)
* a point load e_s f(t) in M u_tt = -K u + e_s f:   s = G Z^T M^{-1/2} e_s
* a receiver at node r reconstructs u_r = e_r^T M^{-1/2} Z G^{-1} U.

Here Z = V Q is the N x kp basis and G = blockdiag(G_1 .. G_k).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import lanczos, sfraction
from .subdomains import Subdomain


@dataclasses.dataclass
class SubdomainROM:
    index: int
    tri: lanczos.BlockTridiagonal
    sf: sfraction.SFraction

    @property
    def k(self) -> int:
        return self.sf.k

    @property
    def p(self) -> int:
        return self.sf.p

    @property
    def gamma(self) -> np.ndarray:
        return np.stack(self.sf.gamma)

    @property
    def gamma_hat(self) -> np.ndarray:
        return np.stack(self.sf.gamma_hat)

    @property
    def face_mass(self) -> np.ndarray:
        """Diagonal of Gamma-hat_1 (= F^T F, diagonal for non-overlapping boundary functions)."""
        return np.diag(self.sf.gamma_hat[0]).copy()

    def _Zrow(self, node: int) -> np.ndarray:
        return self.tri.Z[node]

    def source_vector(self, sd: Subdomain, node: int) -> np.ndarray:
        """s = G Z^T M^{-1/2} e_node, shape [k][p]."""
        z = self._Zrow(node) * sd.S[node]
        p = self.p
        return np.stack([self.sf.G[j] @ z[j * p:(j + 1) * p] for j in range(self.k)])

    def receiver_row(self, sd: Subdomain, node: int) -> np.ndarray:
        """r = e_node^T M^{-1/2} Z G^{-1}, shape [k][p] (u_node = sum_j r_j . U_j)."""
        z = self._Zrow(node) * sd.S[node]
        p = self.p
        return np.stack([np.linalg.solve(self.sf.G[j].T, z[j * p:(j + 1) * p])
                         for j in range(self.k)])

    def project_state(self, sd: Subdomain, u_local: np.ndarray) -> np.ndarray:
        """U = G Z^T M^{1/2} u (eq. "Uj" with v = M^{1/2} u), shape [k][p]."""
        y = self.tri.Z.T @ (np.sqrt(sd.M) * np.asarray(u_local, dtype=np.float64).ravel())
        p = self.p
        return np.stack([self.sf.G[j] @ y[j * p:(j + 1) * p] for j in range(self.k)])

    def reconstruct(self, sd: Subdomain, U: np.ndarray) -> np.ndarray:
        """u = M^{-1/2} Z G^{-1} U (inverse of ``project_state`` on the ROM subspace)."""
        p = self.p
        y = np.concatenate([np.linalg.solve(self.sf.G[j], U[j]) for j in range(self.k)])
        return sd.S * (self.tri.Z @ y)


def build_rom(sd: Subdomain, k: int, sigma: float = np.inf) -> SubdomainROM:
    """Steps 1.1-1.3: Krylov basis and block tridiagonal form, then the S-fraction."""
    A = sd.A_plus()
    F = sd.F()
    if np.isinf(sigma):
        tri = lanczos.lanczos_infinite(A, F, k)
    else:
        tri = lanczos.lanczos_rational(A, F, k, sigma)
    return SubdomainROM(index=sd.index, tri=tri, sf=sfraction.sfraction(tri))


def build_all(subs: List[Subdomain], k: int, sigma: float = np.inf) -> List[SubdomainROM]:
    """Stage 1 for every subdomain (independent, no communication)."""
    return [build_rom(sd, k, sigma) for sd in subs]
