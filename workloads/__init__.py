"""Seeded synthetic inputs shared by the oracle, the GPU path, the tests and the bench.

This module generates inputs only: grid/decomposition parameters, sound-speed
models, source wavelets and source/receiver positions.  It holds none of the
method's arithmetic (no operators, no Krylov, no S-fraction, no stepping), so
both the CPU oracle and the HIP path can take their inputs from here without
sharing any computation.

Array conventions: nodal arrays are C-ordered ``[z][y][x]`` (x fastest), node
indices are ``(i, j, l)`` = (x, y, z), and ``z = 0`` is the surface.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic experiment: grid, split, ROM sizes, source, receivers."""

    name: str
    ncell: Tuple[int, int, int]          # cells along x, y, z
    sub_cells: tuple                     # per axis (x, y, z): cells of every box, or the box sizes in order
    h: float                             # grid step in metres
    m: int                               # boundary basis functions per face
    k: int                               # S-fraction levels (number of blocks)
    f_peak: float                        # Ricker peak frequency, Hz
    nsteps: int                          # leapfrog steps
    src: Tuple[Tuple[int, int, int], ...]   # source nodes (i, j, l)
    rec_grid: Tuple[int, int]            # receivers (1+2a, 1+2b, 0), a < rx, b < ry
    velocity: str                        # "two_layer" | "layered_inclusions"
    seed: int = 0

    @property
    def nodes(self) -> Tuple[int, int, int]:
        return tuple(c + 1 for c in self.ncell)

    @property
    def nsub(self) -> Tuple[int, int, int]:
        return tuple(len(s) if np.ndim(s) else c // s for c, s in zip(self.ncell, self.sub_cells))

    def box_cells(self, axis: int) -> List[int]:
        """Cell counts of the boxes along one axis."""
        s = self.sub_cells[axis]
        return [int(x) for x in s] if np.ndim(s) else [int(s)] * (self.ncell[axis] // int(s))

    def on_box_plane(self, ijk) -> bool:
        """True when a node lies on a subdomain plane along any axis."""
        for d in range(3):
            cuts = np.concatenate([[0], np.cumsum(self.box_cells(d))])
            if int(ijk[d]) in cuts:
                return True
        return False

    @property
    def n_subdomains(self) -> int:
        a, b, c = self.nsub
        return a * b * c

    @property
    def p(self) -> int:
        return 6 * self.m

    @property
    def n_cells(self) -> int:
        return self.ncell[0] * self.ncell[1] * self.ncell[2]

    def receivers(self) -> np.ndarray:
        return receiver_grid(self.rec_grid[0], self.rec_grid[1])

    def sources(self) -> np.ndarray:
        return np.asarray(self.src, dtype=np.int32).reshape(-1, 3)

    def velocity_model(self) -> np.ndarray:
        if self.velocity == "two_layer":
            return two_layer_velocity(self.nodes, z_interface=13, c_top=1500.0, c_bottom=3000.0)
        if self.velocity == "layered_inclusions":
            return layered_inclusions_velocity(self.nodes, seed=self.seed)
        raise ValueError(f"unknown velocity model {self.velocity!r}")


def receiver_grid(nx: int, ny: int, z: int = 0) -> np.ndarray:
    """Surface receivers at nodes (1+2a, 1+2b, z), a < nx, b < ny; shape [nx*ny, 3] (i, j, l)."""
    a, b = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    out = np.stack([1 + 2 * a.ravel(), 1 + 2 * b.ravel(), np.full(a.size, z)], axis=1)
    return out.astype(np.int32)


def two_layer_velocity(nodes, z_interface: int, c_top: float, c_bottom: float) -> np.ndarray:
    """Two half-spaces with a planar interface: c = c_top for node l < z_interface, else c_bottom."""
    nx, ny, nz = nodes
    c = np.full((nz, ny, nx), c_top, dtype=np.float64)
    c[z_interface:, :, :] = c_bottom
    return c


def layered_inclusions_velocity(nodes, seed: int, n_layers: int = 20, n_spheres: int = 50,
                                c_range=(1500.0, 4500.0), radius_range=(5.0, 20.0),
                                contrast: float = 0.3) -> np.ndarray:
    """Seeded layered model plus spherical inclusions (sizes in cells = node spacings).

    ``n_layers - 1`` interface depths are drawn uniformly over the z extent and
    sorted; each layer's speed is uniform in ``c_range``.  Each sphere has a
    uniformly drawn centre and radius and multiplies the speed inside it by
    ``1 + contrast`` or ``1 - contrast`` (random sign).  Returns float64
    ``[nz][ny][nx]``.
    """
    nx, ny, nz = nodes
    rng = np.random.default_rng(seed)
    depths = np.sort(rng.uniform(0.0, nz - 1, size=n_layers - 1))
    speeds = rng.uniform(c_range[0], c_range[1], size=n_layers)
    layer_of_z = np.searchsorted(depths, np.arange(nz, dtype=np.float64), side="right")
    c = np.empty((nz, ny, nx), dtype=np.float64)
    c[:] = speeds[layer_of_z][:, None, None]
    centres = rng.uniform([0, 0, 0], [nx - 1, ny - 1, nz - 1], size=(n_spheres, 3))
    radii = rng.uniform(radius_range[0], radius_range[1], size=n_spheres)
    signs = rng.choice([-1.0, 1.0], size=n_spheres)
    for (cx, cy, cz), r, s in zip(centres, radii, signs):
        lo = [max(0, int(math.floor(v - r))) for v in (cx, cy, cz)]
        hi = [min(n - 1, int(math.ceil(v + r))) for v, n in zip((cx, cy, cz), (nx, ny, nz))]
        xs = np.arange(lo[0], hi[0] + 1)
        ys = np.arange(lo[1], hi[1] + 1)
        zs = np.arange(lo[2], hi[2] + 1)
        d2 = ((zs[:, None, None] - cz) ** 2 + (ys[None, :, None] - cy) ** 2
              + (xs[None, None, :] - cx) ** 2)
        inside = d2 <= r * r
        view = c[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1]
        view[inside] *= (1.0 + s * contrast)
    return c


def random_velocity(nodes, seed: int, lo: float = 1500.0, hi: float = 4500.0) -> np.ndarray:
    """I.i.d. uniform speeds per node (rough media for exactness tests)."""
    nx, ny, nz = nodes
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(nz, ny, nx))


def ricker(f_peak: float, dt: float, nsteps: int, delay: Optional[float] = None) -> np.ndarray:
    """Ricker wavelet samples f(t_n), t_n = n*dt, n = 0..nsteps-1 (unit amplitude).

    f(t) = (1 - 2 pi^2 f^2 tau^2) exp(-pi^2 f^2 tau^2), tau = t - delay, delay = 1.5/f.
    """
    if delay is None:
        delay = 1.5 / f_peak
    t = np.arange(nsteps, dtype=np.float64) * dt - delay
    a = (math.pi * f_peak * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def gaussian_pulse(f_peak: float, dt: float, nsteps: int) -> np.ndarray:
    """Gaussian pulse exp(-pi^2 f^2 tau^2), tau = t - 1.5/f (smooth, for convergence studies)."""
    t = np.arange(nsteps, dtype=np.float64) * dt - 1.5 / f_peak
    return np.exp(-(math.pi * f_peak * t) ** 2)


# --------------------------------------------------------------------------------------
# Named workloads.  The 32^3 two-layer case is the parity case; the 512^3 layered case
# is the throughput case; the mid-size cases are scaled-down versions of the latter
# with the same statistics, used where a sampled oracle check must span many
# subdomains and ragged tiles.
# --------------------------------------------------------------------------------------

CFG_SMALL = Workload(
    name="twolayer_32c_2x2x2_m4_k8",
    ncell=(32, 32, 32), sub_cells=(16, 16, 16), h=10.0, m=4, k=8,
    f_peak=15.0, nsteps=500, src=((15, 15, 15),), rec_grid=(16, 16),
    velocity="two_layer", seed=0)

CFG_LARGE = Workload(
    name="layered_512c_16x16x16_m16_k16",
    ncell=(512, 512, 512), sub_cells=(32, 32, 32), h=10.0, m=16, k=16,
    f_peak=12.0, nsteps=2000, src=((255, 255, 2),), rec_grid=(256, 256),
    velocity="layered_inclusions", seed=1406)


def scaled_large(nsub: Tuple[int, int, int], seed: int = 1406, nsteps: int = 200,
                 n_spheres: Optional[int] = None) -> Workload:
    """The large workload's subdomain shape, ROM sizes and medium statistics on fewer subdomains."""
    ncell = tuple(32 * s for s in nsub)
    rx = ncell[0] // 2
    ry = ncell[1] // 2
    src = (min(255, ncell[0] // 2 - 1), min(255, ncell[1] // 2 - 1), 2)
    return Workload(
        name=f"layered_{ncell[0]}x{ncell[1]}x{ncell[2]}c_m16_k16",
        ncell=ncell, sub_cells=(32, 32, 32), h=10.0, m=16, k=16, f_peak=12.0,
        nsteps=nsteps, src=(src,), rec_grid=(rx, ry), velocity="layered_inclusions",
        seed=seed)



def gaussian_anomaly(c: np.ndarray, center, radius: float, amplitude: float) -> np.ndarray:
    """c (1 + amplitude exp(-r^2 / radius^2)), r the distance in nodes from center = (i, j, l)."""
    nz, ny, nx = c.shape
    l, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r2 = (i - center[0]) ** 2 + (j - center[1]) ** 2 + (l - center[2]) ** 2
    return c * (1.0 + amplitude * np.exp(-r2 / (radius * radius)))


# Gradient workload: 256^3 cells in 32^3-cell subdomains, m = 12 (p = 72), k = 16, 4000 steps,
# 128 x 128 surface receivers; observed data from the same medium with a +5% Gaussian anomaly
# of radius 30 cells at the centre.
CFG_ADJOINT = Workload(
    name="layered_256c_8x8x8_m12_k16_adjoint", ncell=(256, 256, 256), sub_cells=(32, 32, 32), h=10.0,
    m=12, k=16, f_peak=12.0, nsteps=4000, src=((127, 127, 2),), rec_grid=(128, 128),
    velocity="layered_inclusions", seed=1406)
ADJOINT_ANOMALY = dict(center=(128, 128, 128), radius=30.0, amplitude=0.05)


def uneven_boxes(ncells: int, sizes=(24, 32, 48), seed: int = 0) -> Tuple[int, ...]:
    """Seeded box sizes from ``sizes`` adding up to ``ncells`` along one axis: each box is drawn
    uniformly among the sizes that still leave a remainder the sizes can fill."""
    fill = [True] + [False] * ncells
    for n in range(1, ncells + 1):
        fill[n] = any(n >= s and fill[n - s] for s in sizes)
    if not fill[ncells]:
        raise ValueError(f"{ncells} cells cannot be split into boxes of {sizes}")
    rng = np.random.default_rng(seed)
    out, rem = [], ncells
    while rem:
        opts = [s for s in sizes if s <= rem and fill[rem - s]]
        out.append(int(opts[int(rng.integers(len(opts)))]))
        rem -= out[-1]
    return tuple(out)


def level_choices(n_subdomains: int, levels=(8, 12, 16, 24, 32), seed: int = 0) -> np.ndarray:
    """Seeded ROM size per subdomain, uniform over ``levels``."""
    rng = np.random.default_rng(seed)
    return np.asarray(levels, dtype=np.int32)[rng.integers(len(levels), size=n_subdomains)]


def surface_shots(cfg: Workload, n: int, seed: int = 2024, depth: int = 2) -> List[Tuple[int, int, int]]:
    """n shot nodes uniformly random on the surface (at ``depth`` nodes), off every box plane."""
    rng = np.random.default_rng(seed)
    out: List[Tuple[int, int, int]] = []
    while len(out) < n:
        ijk = (int(rng.integers(1, cfg.ncell[0])), int(rng.integers(1, cfg.ncell[1])), depth)
        if cfg.on_box_plane(ijk) or ijk in out:
            continue
        out.append(ijk)
    return out


# Many-shot workload: 384 x 384 x 256 cells as a tensor product of boxes of 24, 32 or 48 cells per
# axis (seeded), m = 12 (p = 72), ROM size per subdomain from {8, 12, 16, 24, 32} (seeded; built
# with k = 32), 64 shots at random surface nodes, 1500 steps, 192 x 192 surface receivers.
CFG_SHOTS = Workload(
    name="layered_384x384x256_uneven_m12_k8-32_64shots", ncell=(384, 384, 256),
    sub_cells=(uneven_boxes(384, seed=11), uneven_boxes(384, seed=12), uneven_boxes(256, seed=13)),
    h=10.0, m=12, k=32, f_peak=12.0, nsteps=1500, src=(), rec_grid=(192, 192),
    velocity="layered_inclusions", seed=1406)
SHOTS_LEVEL_SEED = 14


def surrogate_velocity(nodes, seed: int, layer_cells: float = 6.0, sigma: float = 0.1, blob_density: float = 2e-5,
                       blob_radius=(3.0, 10.0), blob_speed: float = 4500.0) -> np.ndarray:
    """Training media of the learned ROMs: horizontal layers (thicknesses ~ Exp(layer_cells) cells,
    speeds ~U(1500, 4000) m/s), times a pointwise lognormal factor exp(sigma N(0, 1)), plus
    spherical bodies of ``blob_speed`` (about blob_density per node, radii ~U(blob_radius))."""
    nx, ny, nz = nodes
    rng = np.random.default_rng(seed)
    tops = np.cumsum(rng.exponential(layer_cells, size=int(4 * nz / layer_cells) + 8))
    layer = np.searchsorted(tops, np.arange(nz, dtype=np.float64), side="right")
    speeds = rng.uniform(1500.0, 4000.0, size=layer.max() + 1)
    c = np.empty((nz, ny, nx), dtype=np.float64)
    c[:] = speeds[layer][:, None, None]
    c *= np.exp(sigma * rng.standard_normal(c.shape))
    nblob = rng.poisson(blob_density * nx * ny * nz)
    centres = rng.uniform([0, 0, 0], [nx - 1, ny - 1, nz - 1], size=(nblob, 3))
    radii = rng.uniform(blob_radius[0], blob_radius[1], size=nblob)
    for (cx, cy, cz), r in zip(centres, radii):
        lo = [max(0, int(math.floor(v - r))) for v in (cx, cy, cz)]
        hi = [min(n - 1, int(math.ceil(v + r))) for v, n in zip((cx, cy, cz), (nx, ny, nz))]
        zs, ys, xs = np.arange(lo[2], hi[2] + 1), np.arange(lo[1], hi[1] + 1), np.arange(lo[0], hi[0] + 1)
        d2 = (zs[:, None, None] - cz) ** 2 + (ys[None, :, None] - cy) ** 2 + (xs[None, None, :] - cx) ** 2
        view = c[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1]
        view[d2 <= r * r] = blob_speed
    return c
