"""Projection subspaces and block Lanczos tridiagonalisation (Stage 1 and Stage 2 sections).

Conventions (the paper mixes signs and transposes; these readings make every
identity it states hold):

* A_+ = -A is symmetric positive semidefinite and s > 0 is a real Laplace
  frequency, so the transfer function is M(s) = F^T (A_+ + s^2 I)^{-1} F
  (eq. "NtD" with omega^2 read as s^2).
* Block tridiagonal T has diagonal blocks A_j, sub-diagonal blocks
  T_{j+1,j} = B_{j+1} and super-diagonal blocks B_{j+1}^T; the start block is
  F = Q_1 B_1, so R = Q^T F = E_1 B_1 (eq. before "NtDtri").
* QR factors are taken with a positive diagonal in B.  Rotations Q_j -> Q_j O_j
  change A_j, B_j but not the S-fraction coefficients or the ROM state.

Two subspaces:

* sigma = infinity: the polynomial block Krylov space span{F, A_+F, ...,
  A_+^{k-1}F}.  Block Lanczos on (A_+, F) builds the basis and T together
  (the combination of steps 1.1 and 1.2 mentioned in the footnote of
  Algorithm 1).
* finite sigma: the rational space span{F, (A_+ + sigma)^{-1}F, ...,
  (A_+ + sigma)^{-(k-1)}F} obtained by block Lanczos on ((A_+ + sigma I)^{-1}, F),
  the paper's K_n(sigma) with repeated shifts (eq. "krylov0" uses sigma = 0,
  which is singular for a floating subdomain) with F added to the subspace as
  the coupling section requires.  The ROM (A~, F~) = (V^T A_+ V, V^T F) is then
  tridiagonalised by a second, dense block Lanczos (Algorithm 1, step 1.2).
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class LanczosBreakdown(RuntimeError):
    """The next Lanczos block is (numerically) rank deficient."""


def qr_positive(W: np.ndarray):
    """Thin QR, W = Q B with B upper triangular and diag(B) > 0."""
    Q, B = np.linalg.qr(W)
    sgn = np.sign(np.diag(B))
    sgn[sgn == 0] = 1.0
    return Q * sgn[None, :], B * sgn[:, None]


@dataclasses.dataclass
class BlockTridiagonal:
    """Output of block Lanczos: Z = [Q_1 .. Q_k], diagonal blocks A_j, blocks B_1 .. B_k."""

    Z: np.ndarray            # N x kp, orthonormal columns
    A: List[np.ndarray]      # A_1 .. A_k   (p x p, symmetric)
    B: List[np.ndarray]      # B_1 .. B_k   (p x p, upper triangular); B_1 from F = Q_1 B_1

    @property
    def k(self) -> int:
        return len(self.A)

    @property
    def p(self) -> int:
        return self.A[0].shape[0]

    def T(self) -> np.ndarray:
        """Dense block tridiagonal T (kp x kp)."""
        k, p = self.k, self.p
        T = np.zeros((k * p, k * p))
        for j in range(k):
            T[j * p:(j + 1) * p, j * p:(j + 1) * p] = self.A[j]
            if j + 1 < k:
                Bn = self.B[j + 1]
                T[(j + 1) * p:(j + 2) * p, j * p:(j + 1) * p] = Bn
                T[j * p:(j + 1) * p, (j + 1) * p:(j + 2) * p] = Bn.T
        return T

    def R(self) -> np.ndarray:
        """R = Q^T F = [B_1; 0; ...; 0] (kp x p)."""
        k, p = self.k, self.p
        R = np.zeros((k * p, p))
        R[:p] = self.B[0]
        return R


def block_lanczos(apply_op: Callable[[np.ndarray], np.ndarray], F: np.ndarray, k: int,
                  breakdown_tol: float = 1e-12) -> BlockTridiagonal:
    """Block Lanczos on (op, F) for k blocks with full re-orthogonalisation (two passes).

    Q_1 B_1 = F.  For j = 1..k:  W = op Q_j - Q_{j-1} B_j^T,  A_j = Q_j^T op Q_j,
    W -= Q_j A_j, then W -= Z (Z^T W) twice against every block so far, and
    Q_{j+1} B_{j+1} = W (not formed after the last block).  The start block is rank
    deficient when its smallest |diag B_1| falls below ``breakdown_tol * ||B_1||``; a later
    block breaks down when its smallest |diag B_{j+1}| falls below ``breakdown_tol * ||op Q_j||``
    (the new directions are negligible against what the operator produced; relative to the
    operator's own scale, so the test means the same for A_+ and for a resolvent of norm 1/sigma).
    """
    F = np.asarray(F.toarray() if sp.issparse(F) else F, dtype=np.float64)
    N, p = F.shape
    if k * p > N:
        raise ValueError(f"k*p = {k * p} exceeds the operator size {N}")
    Q1, B1 = qr_positive(F)
    scale = np.linalg.norm(B1, 2)
    if np.min(np.abs(np.diag(B1))) < breakdown_tol * scale:
        raise LanczosBreakdown("block 1: the starting block F is rank deficient")
    Qs = [Q1]
    As: List[np.ndarray] = []
    Bs = [B1]
    for j in range(k):
        Qj = Qs[j]
        AQ = apply_op(Qj)
        Aj = Qj.T @ AQ
        Aj = 0.5 * (Aj + Aj.T)
        As.append(Aj)
        if j + 1 == k:
            break
        W = AQ - Qj @ Aj
        if j > 0:
            W = W - Qs[j - 1] @ Bs[j].T
        Z = np.hstack(Qs)
        for _ in range(2):
            W = W - Z @ (Z.T @ W)
        Qn, Bn = qr_positive(W)
        if np.min(np.abs(np.diag(Bn))) < breakdown_tol * np.linalg.norm(AQ, 2):
            raise LanczosBreakdown(f"block {j + 2}: min |diag B| = {np.min(np.abs(np.diag(Bn))):.3e}")
        Qs.append(Qn)
        Bs.append(Bn)
    return BlockTridiagonal(Z=np.hstack(Qs), A=As, B=Bs)


def lanczos_infinite(A_plus: sp.spmatrix, F, k: int) -> BlockTridiagonal:
    """sigma = infinity: block Lanczos on (A_+, F); the basis spans {F, A_+F, ..., A_+^{k-1}F}."""
    return block_lanczos(lambda X: A_plus @ X, F, k)


def lanczos_rational(A_plus: sp.spmatrix, F, k: int, sigma: float,
                     solve_hook: Callable[[Callable, np.ndarray], np.ndarray] = None) -> BlockTridiagonal:
    """Finite sigma: V spans {F, (A_+ + sigma)^{-1}F, ...}; then T from block Lanczos on (V^T A_+ V, V^T F).

    The shifted solves use one sparse LU factorisation reused for all blocks
    (Stage 1 section: a precomputed factorisation can be reused).  Returns Z = V Q.
    solve_hook(solve, X), if given, replaces solve(X) (the tests use it to model inexact solves).
    """
    N = A_plus.shape[0]
    # A_+ + sigma I is symmetric positive definite: diagonal pivots and a symmetric
    # fill-reducing ordering give an exact factorisation with far less fill than COLAMD.
    lu = spla.splu((A_plus + sigma * sp.identity(N)).tocsc(), permc_spec="MMD_AT_PLUS_A",
                   diag_pivot_thresh=0.0, options=dict(SymmetricMode=True))
    if solve_hook is None:
        rational = block_lanczos(lambda X: lu.solve(X), F, k)
    else:
        rational = block_lanczos(lambda X: solve_hook(lu.solve, X), F, k)
    V = rational.Z
    A_rom = V.T @ (A_plus @ V)
    A_rom = 0.5 * (A_rom + A_rom.T)
    F_dense = np.asarray(F.toarray() if sp.issparse(F) else F)
    F_rom = V.T @ F_dense
    inner = block_lanczos(lambda X: A_rom @ X, F_rom, k)
    return BlockTridiagonal(Z=V @ inner.Z, A=inner.A, B=inner.B)
