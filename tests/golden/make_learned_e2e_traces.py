"""Write learned_e2e_traces.npz: FP64 oracle receiver traces of the 256^3 learned-ROM workload's
evaluation medium (the seeded layered / lognormal / blob medium of seed 777 on 257^3 nodes, split
into 512 subdomains of 32^3 cells, m = 8, k = 16), 500 leapfrog steps at 0.9 of the oracle's
stability limit, a 12 Hz Ricker source at node (127, 127, 2) and 64 surface receivers, one per
surface subdomain.  The device's learned build (network prediction, NtD judge, Lanczos fallback)
of the same medium is stepped and compared against these traces by tests/test_gpu_learned_e2e.py.

Calls only the oracle and the input generators.  The 512 oracle ROM builds run in a pool of
worker processes (each builds its subdomains and keeps only the basis rows of the source and
receiver nodes); about 20 minutes on 8 cores.
Usage: python tests/golden/make_learned_e2e_traces.py
"""
from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import coupled, rom, subdomains  # noqa: E402

NCELL = (256, 256, 256)
SUB = (32, 32, 32)
H = 10.0
M = 8
K = 16
F_PEAK = 12.0
SEED = 777
NSTEPS = 500
SOURCE = np.array([[127, 127, 2]], dtype=np.int32)


def receivers() -> np.ndarray:
    return np.array([[16 + 32 * a, 16 + 32 * b, 0] for b in range(8) for a in range(8)], dtype=np.int32)


def velocity() -> np.ndarray:
    """The medium as the device receives it (FP32), in FP64."""
    return W.surrogate_velocity(tuple(x + 1 for x in NCELL), seed=SEED).astype(np.float32).astype(np.float64)


class _Rows:
    """The rows of a basis Z kept for the nodes whose projections are needed."""

    def __init__(self, Z, nodes):
        self.rows = {int(n): Z[int(n)].copy() for n in nodes}

    def __getitem__(self, node):
        return self.rows[int(node)]


_SUBS = None


def _init():
    global _SUBS
    _SUBS = subdomains.decompose(velocity(), H, SUB, M)


def _build(idx):
    sd = _SUBS[idx]
    points = np.concatenate([receivers(), SOURCE])
    r = rom.build_rom(sd, K)
    need = [sd.local_index(x) for x in points if sd.contains(x)]
    r.tri.Z = _Rows(r.tri.Z, need)
    return idx, r


def main():
    t0 = time.time()
    subs = subdomains.decompose(velocity(), H, SUB, M)
    nproc = int(os.environ.get("GOLDEN_PROCS", "4"))
    roms = [None] * len(subs)
    with ProcessPoolExecutor(max_workers=nproc, initializer=_init) as ex:
        for n, (idx, r) in enumerate(ex.map(_build, range(len(subs)), chunksize=4)):
            roms[idx] = r
            if n % 32 == 31:
                print(f"{n + 1} of {len(subs)} subdomains built ({time.time() - t0:.0f} s)", flush=True)
    rec = receivers()
    cs = coupled.CoupledSystem(subs, roms, SOURCE, rec)
    dt = 0.9 * cs.cfl_dt()
    wav = W.ricker(F_PEAK, dt, NSTEPS)[:, None]
    traces = cs.run(dt, wav)
    np.savez_compressed(os.path.join(HERE, "learned_e2e_traces.npz"), traces=traces.astype(np.float32),
                        receivers=rec, source=SOURCE, dt=np.float64(dt))
    with open(os.path.join(HERE, "learned_e2e_traces.json"), "w") as fh:
        json.dump({"ncell": NCELL, "sub_cells": SUB, "h": H, "m": M, "k": K, "f_peak": F_PEAK, "seed": SEED,
                   "steps": NSTEPS, "dt": dt, "receivers": len(rec), "source": SOURCE.tolist(),
                   "peak_abs_trace": float(np.abs(traces).max()),
                   "written_by": "tests/golden/make_learned_e2e_traces.py (oracle only)"}, fh, indent=1)
    print(f"dt {dt:.6e}; traces {traces.shape}; {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
