"""S-fraction transform and transfer functions (Stage 2 section).

From the block tridiagonal (T, R) of block Lanczos, the recursion of eq.
"GammaTrans" gives the matrix S-fraction coefficients.  In this package's sign
and transpose convention (A_+ = -A, T_{j+1,j} = B_{j+1}, R = E_1 B_1):

    G_1 = B_1^T,  Gamma_0 = 0,  and for j = 1..k
        Gamma-hat_j = G_j G_j^T
        Gamma_j     = G_j^{-T} A_j G_j^{-1} - Gamma_{j-1}
        G_{j+1}     = -Gamma_j^{-1} G_j^{-T} B_{j+1}^T        (j < k)

so that, with D the block forward difference (U_{k+1} = 0) and G = blockdiag(G_j),

    G^{-T} T G^{-1} = D^T Gamma D,   G^{-T} G^{-1} = Gamma-hat^{-1},

which is the second change of coordinates U_j = G_j W_j that turns eq.
"tridiagW" into eq. "GammaU".  The paper's printed recursion (G_1 = B_1,
G_{j+1} = [G_j^* Gamma_j]^{-1} B_{j+1}, Gamma_{j+1} = -G^{-*} A_{j+1} G^{-1} - Gamma_j
with A <= 0) differs only by these transposes and the sign of A; the
coefficients Gamma_j and Gamma-hat_j do not depend on that choice.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .lanczos import BlockTridiagonal


def sym(X: np.ndarray) -> np.ndarray:
    return 0.5 * (X + X.T)


@dataclasses.dataclass
class SFraction:
    gamma: List[np.ndarray]      # Gamma_1 .. Gamma_k
    gamma_hat: List[np.ndarray]  # Gamma-hat_1 .. Gamma-hat_k
    G: List[np.ndarray]          # G_1 .. G_k (coordinate change of eq. "Uj")

    @property
    def k(self) -> int:
        return len(self.gamma)

    @property
    def p(self) -> int:
        return self.gamma[0].shape[0]


def sfraction(tri: BlockTridiagonal) -> SFraction:
    """Recursion of eq. "GammaTrans" (convention in the module docstring), in FP64."""
    k = tri.k
    G = tri.B[0].T.copy()
    gam_prev = np.zeros_like(G)
    gammas, hats, Gs = [], [], []
    for j in range(k):
        Gs.append(G)
        hats.append(sym(G @ G.T))
        Ginv = np.linalg.inv(G)
        gam = sym(Ginv.T @ tri.A[j] @ Ginv - gam_prev)
        gammas.append(gam)
        if j + 1 < k:
            G = -np.linalg.solve(gam, Ginv.T @ tri.B[j + 1].T)
        gam_prev = gam
    return SFraction(gamma=gammas, gamma_hat=hats, G=Gs)


def difference_stiffness(sf: SFraction) -> np.ndarray:
    """D^T Gamma D (kp x kp): diagonal blocks Gamma_j + Gamma_{j-1}, off-diagonal -Gamma_j."""
    k, p = sf.k, sf.p
    K = np.zeros((k * p, k * p))
    for j in range(k):
        K[j * p:(j + 1) * p, j * p:(j + 1) * p] += sf.gamma[j]
        if j + 1 < k:
            K[(j + 1) * p:(j + 2) * p, (j + 1) * p:(j + 2) * p] += sf.gamma[j]
            K[j * p:(j + 1) * p, (j + 1) * p:(j + 2) * p] -= sf.gamma[j]
            K[(j + 1) * p:(j + 2) * p, j * p:(j + 1) * p] -= sf.gamma[j]
    return K


def blockdiag(blocks: List[np.ndarray]) -> np.ndarray:
    n = sum(b.shape[0] for b in blocks)
    out = np.zeros((n, n))
    o = 0
    for b in blocks:
        out[o:o + b.shape[0], o:o + b.shape[1]] = b
        o += b.shape[0]
    return out


# ---------------------------------------------------------------------------------------
# Transfer functions evaluated three ways (eqs. "NtD", "NtDtri" and the continued fraction)
# ---------------------------------------------------------------------------------------

def ntd_resolvent(A_plus, F, s: float) -> np.ndarray:
    """Exact projected NtD map M(s) = F^T (A_+ + s^2 I)^{-1} F (eq. "NtD")."""
    Fd = np.asarray(F.toarray() if sp.issparse(F) else F)
    N = A_plus.shape[0]
    if sp.issparse(A_plus):
        # symmetric positive definite for s > 0: diagonal pivots, symmetric fill-reducing ordering
        X = spla.splu((A_plus + s * s * sp.identity(N)).tocsc(), permc_spec="MMD_AT_PLUS_A",
                      diag_pivot_thresh=0.0, options=dict(SymmetricMode=True)).solve(Fd)
    else:
        X = np.linalg.solve(A_plus + s * s * np.eye(N), Fd)
    return Fd.T @ X


def ntd_tridiagonal(tri: BlockTridiagonal, s: float) -> np.ndarray:
    """ROM NtD map R^T (T + s^2 I)^{-1} R (eq. "NtDtri")."""
    T = tri.T()
    R = tri.R()
    return R.T @ np.linalg.solve(T + s * s * np.eye(T.shape[0]), R)


def ntd_continued_fraction(sf: SFraction, s: float) -> np.ndarray:
    """Matrix S-fraction (the block form of the scalar continued fraction in Stage 2).

    X_k = Gamma-hat_k^{-1} s^2 + Gamma_k,
    X_j = Gamma-hat_j^{-1} s^2 + (Gamma_j^{-1} + X_{j+1}^{-1})^{-1},   M~(s) = X_1^{-1}.
    Obtained by eliminating U_k, U_{k-1}, ... from eq. "GammaU".
    """
    k = sf.k
    X = np.linalg.inv(sf.gamma_hat[k - 1]) * s * s + sf.gamma[k - 1]
    for j in range(k - 2, -1, -1):
        inner = np.linalg.inv(np.linalg.inv(sf.gamma[j]) + np.linalg.inv(X))
        X = np.linalg.inv(sf.gamma_hat[j]) * s * s + inner
    return np.linalg.inv(X)


def ntd_rel_error(A_plus, F, sf: SFraction, s_values) -> float:
    """max_i ||M~(s_i) - M(s_i)||_F / ||M(s_i)||_F over the given Laplace frequencies."""
    err = 0.0
    for s in s_values:
        exact = ntd_resolvent(A_plus, F, s)
        rom = ntd_continued_fraction(sf, s)
        err = max(err, np.linalg.norm(rom - exact) / np.linalg.norm(exact))
    return err


def ntd_frequencies(f_peak: float) -> np.ndarray:
    """Eight Laplace frequencies 2 pi f_p {1/4, 1/2, 3/4, 1, 3/2, 2, 5/2, 3}."""
    return 2.0 * np.pi * f_peak * np.array([0.25, 0.5, 0.75, 1.0, 1.5, 2.0, 2.5, 3.0])
