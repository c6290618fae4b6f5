"""Write slice_traces.npz: FP64 oracle receiver traces of a 4 x 4 x 4-subdomain slice with the 512^3
workload's subdomain and ROM shape (32^3-cell boxes, m = 16, k = 16; 128^3 cells, interior
subdomains with six interface faces), 2000 leapfrog steps at 0.9 of the oracle's stability limit.

It also records the oracle's own reproducibility: the 8 interior subdomains are rebuilt from their
operators perturbed by a symmetric relative noise of 1e-15, and the rel-L2 of the resulting traces
against the unperturbed ones is stored for the first 500, 1000 and 2000 steps.  The deep S-fraction
levels of an interior subdomain respond to such a perturbation by up to 20% (level 15), so this is
the accuracy to which any FP64 build of these ROMs can reproduce the traces.

Calls only the oracle and the input generators.  The run takes about 30 minutes on 8 cores: the
GPU test (tests/test_gpu_slice.py) reads the stored traces instead of rebuilding 64 ROMs.
Usage: python tests/golden/make_slice_traces.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import adjoint, coupled, lanczos, rom, sfraction, subdomains  # noqa: E402

NSTEPS = 2000
HORIZONS = (500, 1000, 2000)


def interior(cfg: W.Workload):
    """Subdomains with six interface faces."""
    nx, ny, nz = cfg.nsub
    return [(bz * ny + by) * nx + bx for bz in range(1, nz - 1) for by in range(1, ny - 1) for bx in range(1, nx - 1)]


def perturbed_sfraction(sd, k: int, seed: int):
    """S-fraction of the subdomain operator with a symmetric relative perturbation of size 1e-15."""
    A = sd.A_plus().tocoo()
    rng = np.random.default_rng(seed)
    upper = A.row <= A.col
    noise = np.zeros(A.nnz)
    noise[upper] = 1e-15 * rng.standard_normal(int(upper.sum()))
    Ap = sp.coo_matrix((A.data * (1 + noise), (A.row, A.col)), shape=A.shape).tocsr()
    Ap = (sp.triu(Ap) + sp.triu(Ap, 1).T).tocsr()
    return sfraction.sfraction(lanczos.lanczos_infinite(Ap, sd.F(), k))


def slice_config() -> W.Workload:
    return W.scaled_large((4, 4, 4), nsteps=NSTEPS)


def receiver_sample(cfg: W.Workload) -> np.ndarray:
    """An 8 x 8 sub-grid of the surface receivers (every 8th along each axis, offset 3)."""
    rx, ry = cfg.rec_grid
    full = cfg.receivers().reshape(rx, ry, 3)
    return full[3::8, 3::8].reshape(-1, 3).astype(np.int32)


class _Rows:
    """The rows of a basis Z kept for the nodes whose projections are needed."""

    def __init__(self, Z, nodes):
        self.rows = {int(n): Z[int(n)].copy() for n in nodes}

    def __getitem__(self, node):
        return self.rows[int(node)]


def main():
    cfg = slice_config()
    c = cfg.velocity_model().astype(np.float32).astype(np.float64)
    subs = subdomains.decompose(c, cfg.h, cfg.sub_cells, cfg.m)
    rec = receiver_sample(cfg)
    src = cfg.sources()
    points = np.concatenate([rec, src])
    roms = []
    t0 = time.time()
    for sd in subs:
        r = rom.build_rom(sd, cfg.k)
        need = [sd.local_index(x) for x in points if sd.contains(x)]
        r.tri.Z = _Rows(r.tri.Z, need)
        roms.append(r)
        print(f"subdomain {sd.index}: built ({time.time() - t0:.0f} s)", flush=True)
    cs = coupled.CoupledSystem(subs, roms, src, rec)
    dt = 0.9 * cs.cfl_dt()
    wav = W.ricker(cfg.f_peak, dt, NSTEPS)[:, None]
    traces = cs.run(dt, wav)
    # the oracle's own reproducibility: interior subdomains rebuilt from 1e-15-perturbed operators
    # (they hold no source or receiver, so only their blocks change)
    inner = interior(cfg)
    dg = [[np.zeros_like(g) for g in r.sf.gamma] for r in roms]
    dh = [[np.zeros_like(g) for g in r.sf.gamma_hat] for r in roms]
    for s in inner:
        sf = perturbed_sfraction(subs[s], cfg.k, seed=1000 + s)
        dg[s] = [a - b for a, b in zip(sf.gamma, roms[s].sf.gamma)]
        dh[s] = [a - b for a, b in zip(sf.gamma_hat, roms[s].sf.gamma_hat)]
        print(f"subdomain {s}: rebuilt from the perturbed operator ({time.time() - t0:.0f} s)", flush=True)
    traces_p = adjoint.perturbed_system(cs, dg, dh, 1.0).run(dt, wav)
    repro = {str(m): float(np.linalg.norm(traces_p[:, :m] - traces[:, :m]) / np.linalg.norm(traces[:, :m]))
             for m in HORIZONS}
    np.savez_compressed(os.path.join(HERE, "slice_traces.npz"), traces=traces.astype(np.float32),
                        receivers=rec, dt=np.float64(dt))
    with open(os.path.join(HERE, "slice_traces.json"), "w") as fh:
        json.dump({"workload": cfg.name, "steps": NSTEPS, "dt": dt, "receivers": len(rec),
                   "sources": src.tolist(), "peak_abs_trace": float(np.abs(traces).max()),
                   "interior_subdomains": inner, "oracle_reproducibility_rel_l2": repro,
                   "written_by": "tests/golden/make_slice_traces.py (oracle only)"}, fh, indent=1)
    print(f"dt {dt:.6e}; traces {traces.shape}; reproducibility {repro}; {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
