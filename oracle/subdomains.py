"""Domain decomposition, subdomain operators and the boundary basis F.

Follows the paper's Introduction (split of Omega into box subdomains, one fine
operator A^alpha per subdomain with its boundary conditions built in) and the
Stage 1 section (m boundary functions per shared boundary, all six faces of a
box stacked into F^alpha with 6m columns; functions localised on their face and
non-overlapping, which the coupling section needs for a block-diagonal
Gamma-hat_1).

Readings where the paper is silent:

* Nodes on an interface plane are shared by the subdomains on both sides; each
  subdomain builds its mass and stiffness with the box construction of
  ``oracle.grid`` on its own box, so the subdomain operators sum to the global
  operator exactly.
* Faces are ordered x-, x+, y-, y+, z-, z+.  A face is an interface when a
  neighbour box exists, otherwise it is outer (zero flux).  Each boundary node
  belongs to exactly one face: among the faces whose plane holds it, interface
  faces come before outer ones, then the order above.  Both sides of a shared
  face apply the same rule, so they own the same node set.
* Boundary functions are piecewise-constant patches: m = m1 * m2 with
  m1 >= m2 and m1 - m2 minimal; the first tangential axis (in x, y, z order) is
  cut into m1 strips and the second into m2, a node at tangential offsets (a, b)
  on a face n1 x n2 cells wide going to strip min(floor(a m1 / n1), m1 - 1)
  (likewise for b).  Column index = face * m + strip1 * m2 + strip2.
* The patch function of a node is its dual face area inside the face,
  E = h^2 times 1/2 for each tangential box plane the node lies on, and
  F = M^{-1/2} E in the symmetric variables v = M^{1/2} u.

Each column carries a global "port" key; columns of two subdomains with the
same key are the same shared unknown U_1 of the coupling condition (eq. "mass").
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Tuple

import numpy as np
import scipy.sparse as sp

from . import grid


def factor_patches(m: int) -> Tuple[int, int]:
    """m = m1 * m2 with m1 >= m2 and m1 - m2 as small as possible."""
    best = (m, 1)
    for m2 in range(1, math.isqrt(m) + 1):
        if m % m2 == 0:
            best = (m // m2, m2)
    return best


FACE_NAMES = ("x-", "x+", "y-", "y+", "z-", "z+")


@dataclasses.dataclass
class Subdomain:
    index: int                      # flat box index, x fastest
    box: Tuple[int, int, int]       # (bx, by, bz)
    origin: Tuple[int, int, int]    # global node of local (0, 0, 0), (i, j, l)
    cells: Tuple[int, int, int]     # cells along (x, y, z)
    c: np.ndarray                   # local sound speed [nz][ny][nx]
    M: np.ndarray                   # local lumped mass (flat)
    K: sp.csr_matrix                # local stiffness
    neighbours: Tuple[int, ...]     # per face: neighbour flat index or -1
    E: sp.csr_matrix                # N x p patch functions in u variables
    port_keys: List[tuple]          # per column of E
    h: float

    @property
    def shape(self):
        return self.c.shape

    @property
    def N(self) -> int:
        return self.M.size

    @property
    def p(self) -> int:
        return self.E.shape[1]

    @property
    def S(self) -> np.ndarray:
        """Diagonal of M^{-1/2}, the change to symmetric variables v = M^{1/2} u."""
        return 1.0 / np.sqrt(self.M)

    def A_plus(self) -> sp.csr_matrix:
        """A_+ = M^{-1/2} K M^{-1/2} = -A in symmetric variables (positive semidefinite)."""
        s = sp.diags(self.S)
        return (s @ self.K @ s).tocsr()

    def F(self) -> sp.csr_matrix:
        """F = M^{-1/2} E (N x p)."""
        return (sp.diags(self.S) @ self.E).tocsr()

    def local_index(self, ijk_global) -> int:
        i, j, l = (int(a) - int(b) for a, b in zip(ijk_global, self.origin))
        return grid.node_index(self.shape, (i, j, l))

    def contains(self, ijk_global, strict: bool = False) -> bool:
        rel = [int(a) - int(b) for a, b in zip(ijk_global, self.origin)]
        if strict:
            return all(0 < r < n for r, n in zip(rel, self.cells))
        return all(0 <= r <= n for r, n in zip(rel, self.cells))


def _boundary_faces(loc, cells):
    """For local node coordinates loc = (i, j, l) arrays, a [n, 6] mask of faces holding each node."""
    i, j, l = loc
    sx, sy, sz = cells
    return np.stack([i == 0, i == sx, j == 0, j == sy, l == 0, l == sz], axis=1)


def box_cuts(ncells: int, sub) -> List[int]:
    """Plane positions 0 = x_0 < x_1 < ... = ncells along one axis: ``sub`` is the cell count of
    every box (an int dividing ncells) or the list of the boxes' cell counts in order."""
    if np.ndim(sub) == 0:
        if ncells % int(sub):
            raise ValueError("cells per axis must be a multiple of sub_cells")
        sub = [int(sub)] * (ncells // int(sub))
    cuts = np.concatenate([[0], np.cumsum(np.asarray(sub, dtype=np.int64))]).tolist()
    if cuts[-1] != ncells or min(np.diff(cuts)) < 1:
        raise ValueError("box sizes along an axis must be positive and add up to its cells")
    return [int(x) for x in cuts]


def decompose(c: np.ndarray, h: float, sub_cells, m: int, mode: str = "patches") -> List[Subdomain]:
    """Split the node grid ``c`` ([nz][ny][nx]) into a tensor product of boxes: per axis,
    ``sub_cells`` gives one cell count for all boxes or the list of box cell counts.

    ``mode = "patches"``: the m-patch basis on all six faces (p = 6m).
    ``mode = "interface_nodes"``: one function per node owned by an interface
    face, none on outer faces (used for the exactness pin with two subdomains).
    """
    c = np.asarray(c, dtype=np.float64)
    nz, ny, nx = c.shape
    cx, cy, cz = (box_cuts(n - 1, s) for n, s in zip((nx, ny, nz), sub_cells))
    Bx, By, Bz = len(cx) - 1, len(cy) - 1, len(cz) - 1
    m1, m2 = factor_patches(m) if mode == "patches" else (0, 0)
    subs = []
    for bz in range(Bz):
        for by in range(By):
            for bx in range(Bx):
                idx = (bz * By + by) * Bx + bx
                i0, j0, l0 = cx[bx], cy[by], cz[bz]
                sx, sy, sz = cx[bx + 1] - i0, cy[by + 1] - j0, cz[bz + 1] - l0
                cl = c[l0:l0 + sz + 1, j0:j0 + sy + 1, i0:i0 + sx + 1].copy()
                box = (bx, by, bz)
                nb = []
                for f in range(6):
                    d, s = divmod(f, 2)
                    bb = list(box)
                    bb[d] += -1 if s == 0 else 1
                    lim = (Bx, By, Bz)[d]
                    if 0 <= bb[d] < lim:
                        nb.append((bb[2] * By + bb[1]) * Bx + bb[0])
                    else:
                        nb.append(-1)
                M = grid.node_mass(cl, h).ravel()
                K = grid.stiffness(cl.shape, h)
                E, keys = _basis(cl.shape, (sx, sy, sz), box, (Bx, By, Bz), nb, h, m, m1, m2,
                                 mode, (i0, j0, l0), (nx, ny, nz), idx)
                subs.append(Subdomain(index=idx, box=box, origin=(i0, j0, l0), cells=(sx, sy, sz),
                                      c=cl, M=M, K=K, neighbours=tuple(nb), E=E, port_keys=keys,
                                      h=h))
    return subs


def _basis(shape, cells, box, nbox, nb, h, m, m1, m2, mode, origin, gnodes, idx):
    nz, ny, nx = shape
    sx, sy, sz = cells
    l, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    l, j, i = l.ravel(), j.ravel(), i.ravel()
    on = _boundary_faces((i, j, l), cells)
    is_iface = np.array([nb[f] >= 0 for f in range(6)])
    # Ownership priority: interface faces (in face order) then outer faces (in face order).
    order = [f for f in range(6) if is_iface[f]] + [f for f in range(6) if not is_iface[f]]
    owner = np.full(i.size, -1)
    for f in reversed(order):
        owner[on[:, f]] = f
    coords = (i, j, l)
    half = [(coords[d] == 0) | (coords[d] == cells[d]) for d in range(3)]
    cols_node, cols_col, cols_val = [], [], []
    keys: List[tuple] = []
    col = 0
    for f in range(6):
        d = f // 2
        t1, t2 = [a for a in range(3) if a != d]
        sel = np.nonzero(owner == f)[0]
        w = h * h * np.where(half[t1][sel], 0.5, 1.0) * np.where(half[t2][sel], 0.5, 1.0)
        if mode == "patches":
            a = coords[t1][sel]
            b = coords[t2][sel]
            q1 = np.minimum(a * m1 // cells[t1], m1 - 1)
            q2 = np.minimum(b * m2 // cells[t2], m2 - 1)
            q = q1 * m2 + q2
            for qq in range(m):
                keys.append(_port_key(f, qq, box, nbox, nb, idx))
            cols_node.append(sel)
            cols_col.append(col + q)
            cols_val.append(w)
            col += m
        elif mode == "interface_nodes":
            if nb[f] < 0:
                continue
            gi = i[sel] + origin[0]
            gj = j[sel] + origin[1]
            gl = l[sel] + origin[2]
            gflat = (gl * gnodes[1] + gj) * gnodes[0] + gi
            for g in gflat:
                keys.append(("N", int(g)))
            cols_node.append(sel)
            cols_col.append(col + np.arange(sel.size))
            cols_val.append(w)
            col += sel.size
        else:
            raise ValueError(mode)
    E = sp.coo_matrix((np.concatenate(cols_val), (np.concatenate(cols_node), np.concatenate(cols_col))),
                      shape=(i.size, col)).tocsr()
    return E, keys


def _port_key(f, q, box, nbox, nb, idx):
    d, s = divmod(f, 2)
    if nb[f] < 0:
        return ("O", idx, f, q)
    lower = idx if s == 1 else nb[f]
    return ("I", d, lower, q)


def port_table(subs: List[Subdomain]):
    """Global port numbering: returns (n_ports, [per-subdomain array of port ids])."""
    ids: Dict[tuple, int] = {}
    per = []
    for sd in subs:
        arr = np.empty(sd.p, dtype=np.int64)
        for c, key in enumerate(sd.port_keys):
            if key not in ids:
                ids[key] = len(ids)
            arr[c] = ids[key]
        per.append(arr)
    return len(ids), per


def owner_subdomain(subs: List[Subdomain], ijk, strict: bool = False) -> int:
    """First subdomain (lowest flat index) whose box holds node ijk (strictly inside if ``strict``)."""
    for sd in subs:
        if sd.contains(ijk, strict=strict):
            return sd.index
    return -1
