"""Fine reference grid: node-based 7-point operator with mirror (Neumann) outer boundary.

The paper leaves the fine discretisation open (Introduction, eq. "wave": the
semi-discrete system u_tt = A u with boundary conditions built into A).  The
reading used throughout: constant-density acoustics u_tt = c^2 Lap(u)
(Numerical experiments section), nodes at x = h*(i, j, l), and the
finite-volume form

    M u_tt = -K u + (forcing),   A = -M^{-1} K,

with a lumped dual-cell mass M = diag(w h^3 / c^2), where w halves once for each
boundary plane a node lies on, and a stiffness K = sum over grid edges of
(area/h)(e_a - e_b)(e_a - e_b)^T whose dual face area h^2 halves once for each
boundary plane the edge lies in.  In the interior this is the standard 7-point
Laplacian; on the outer boundary it is the mirror (homogeneous Neumann) closure.

The same construction, applied to a box that is a subdomain, gives that
subdomain's operator, and the subdomain operators sum exactly to the global one
because shared interface nodes and edges receive complementary halves.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def plane_weights(n_nodes: int) -> np.ndarray:
    """1-D factor of the dual volume: 1/2 at the two end nodes of a line of n_nodes nodes."""
    w = np.ones(n_nodes)
    w[0] = 0.5
    w[-1] = 0.5
    return w


def node_mass(c: np.ndarray, h: float) -> np.ndarray:
    """Lumped mass M = w h^3 / c^2 at every node of a box; c is ``[nz][ny][nx]``."""
    nz, ny, nx = c.shape
    w = (plane_weights(nz)[:, None, None] * plane_weights(ny)[None, :, None]
         * plane_weights(nx)[None, None, :])
    return w * h ** 3 / c ** 2


def stiffness(shape, h: float) -> sp.csr_matrix:
    """Geometric stiffness K of a box with ``shape = (nz, ny, nx)`` nodes, as a sparse matrix.

    K = sum_edges (area/h) (e_a - e_b)(e_a - e_b)^T with area = h^2 times 1/2 for
    every box boundary plane that contains the edge.
    """
    nz, ny, nx = shape
    idx = np.arange(nz * ny * nx).reshape(nz, ny, nx)
    wz, wy, wx = plane_weights(nz), plane_weights(ny), plane_weights(nx)
    rows, cols, vals = [], [], []

    def add_edges(a, b, coef):
        a = a.ravel(); b = b.ravel(); coef = coef.ravel()
        rows.extend([a, b, a, b])
        cols.extend([a, b, b, a])
        vals.extend([coef, coef, -coef, -coef])

    # x-edges: lie in the boundary planes normal to y and z that contain them.
    if nx > 1:
        coef = h * (wz[:, None, None] * wy[None, :, None]) * np.ones((1, 1, nx - 1))
        add_edges(idx[:, :, :-1], idx[:, :, 1:], coef)
    if ny > 1:
        coef = h * (wz[:, None, None] * wx[None, None, :]) * np.ones((1, ny - 1, 1))
        add_edges(idx[:, :-1, :], idx[:, 1:, :], coef)
    if nz > 1:
        coef = h * (wy[None, :, None] * wx[None, None, :]) * np.ones((nz - 1, 1, 1))
        add_edges(idx[:-1, :, :], idx[1:, :, :], coef)
    n = nz * ny * nx
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return K.tocsr()


def node_index(shape, ijk) -> int:
    """Flat index of node (i, j, l) = (x, y, z) in a C-ordered ``[nz][ny][nx]`` box."""
    nz, ny, nx = shape
    i, j, l = (int(v) for v in ijk)
    if not (0 <= i < nx and 0 <= j < ny and 0 <= l < nz):
        raise ValueError(f"node {ijk} outside box of shape {shape}")
    return (l * ny + j) * nx + i


class FineGrid:
    """Global fine-grid operator (M, K) for a sound-speed model c ``[nz][ny][nx]``."""

    def __init__(self, c: np.ndarray, h: float):
        self.c = np.asarray(c, dtype=np.float64)
        self.h = float(h)
        self.shape = self.c.shape
        self.M = node_mass(self.c, self.h).ravel()
        self.K = stiffness(self.shape, self.h)

    def max_eig(self, tol: float = 1e-10) -> float:
        """Largest eigenvalue of M^{-1} K (symmetric form M^{-1/2} K M^{-1/2})."""
        from scipy.sparse.linalg import eigsh
        s = 1.0 / np.sqrt(self.M)
        A = sp.diags(s) @ self.K @ sp.diags(s)
        vals = eigsh(A, k=1, which="LA", tol=tol, return_eigenvectors=False)
        return float(vals[0])

    def cfl_dt(self) -> float:
        """Leapfrog stability limit 2 / sqrt(lambda_max(M^{-1} K))."""
        return 2.0 / np.sqrt(self.max_eig())

    def fdtd(self, dt: float, wavelets: np.ndarray, src_ijk, rec_ijk,
             u0: np.ndarray | None = None, v0: np.ndarray | None = None) -> np.ndarray:
        """Leapfrog FDTD  M (u^{n+1} - 2u^n + u^{n-1}) / dt^2 = -K u^n + sum_s e_s f_s(t_n).

        ``wavelets`` is ``[nsteps][nsrc]`` (f at t_n = n dt).  Zero initial state
        unless ``u0`` (and the velocity ``v0`` at t = 0, used through
        u^{-1} = u^0 - dt v0) are given.  Receivers sample u^{n+1} after every
        update, so the trace array is ``[nrec][nsteps]`` with sample n at t_{n+1}.
        """
        wavelets = np.asarray(wavelets, dtype=np.float64).reshape(len(wavelets), -1)
        nsteps = wavelets.shape[0]
        src = [node_index(self.shape, s) for s in np.asarray(src_ijk).reshape(-1, 3)]
        rec = np.array([node_index(self.shape, r) for r in np.asarray(rec_ijk).reshape(-1, 3)],
                       dtype=np.int64)
        n = self.M.size
        u = np.zeros(n) if u0 is None else np.asarray(u0, dtype=np.float64).ravel().copy()
        u_prev = u.copy() if v0 is None else u - dt * np.asarray(v0, dtype=np.float64).ravel()
        minv = 1.0 / self.M
        traces = np.empty((rec.size, nsteps))
        for step in range(nsteps):
            rhs = -(self.K @ u)
            for si, node in enumerate(src):
                rhs[node] += wavelets[step, si]
            u_next = 2.0 * u - u_prev + dt * dt * minv * rhs
            u_prev, u = u, u_next
            traces[:, step] = u[rec]
        return traces
