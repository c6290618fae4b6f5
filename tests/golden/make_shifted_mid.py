"""Writes shifted_mid.json: oracle-derived tolerances of the finite-shift parity test on the
33^3-subdomain case (2 x 2 x 1 subdomains, m = 16, k = 16), whose exact-solve oracle ROMs take
minutes per subdomain.  Calls only the oracle (through tests.cases).  Run from the repository root:

    python tests/golden/make_shifted_mid.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import rom, subdomains  # noqa: E402
from tests import cases  # noqa: E402

RTOL = 1e-12
SUBS = (0, 3)


def main():
    name = "mid"
    cfg = cases.case_config(name)
    sigma = cases.case_sigma(name)
    c = cfg.velocity_model().astype(np.float32).astype(np.float64)
    subs = subdomains.decompose(c, cfg.h, cfg.sub_cells, cfg.m)
    out = {"case": name, "sigma": sigma, "rtol": RTOL, "subdomains": {}}
    # the unscaled shift (2 pi f_peak)^2: the oracle's S-fraction of subdomain 0 is indefinite
    sigma1 = cases.case_sigma(name, factor=1.0)
    r1 = rom.build_rom(subs[0], cfg.k, sigma1)
    out["unscaled"] = {
        "sigma": sigma1,
        "min_eig_ratio_gamma": [float(np.linalg.eigvalsh(g)[0] / np.linalg.eigvalsh(g)[-1]) for g in r1.sf.gamma],
        "min_eig_ratio_gamma_hat": [float(np.linalg.eigvalsh(g)[0] / np.linalg.eigvalsh(g)[-1])
                                    for g in r1.sf.gamma_hat],
    }
    print("unscaled", out["unscaled"], flush=True)
    for s in SUBS:
        r = rom.build_rom(subs[s], cfg.k, sigma)
        prof = np.maximum(cases.perturbation_profile(subs[s], r, sigma=sigma),
                          cases.solve_perturbation_profile(subs[s], r, sigma, RTOL))
        out["subdomains"][str(s)] = {
            "level_tolerance": [float(x) for x in cases.level_tolerance(prof)],
            "interp_tolerance": cases.shifted_interp_tolerance(subs[s], r, sigma, RTOL),
        }
        print(s, out["subdomains"][str(s)], flush=True)
    with open(os.path.join(ROOT, "tests", "golden", "shifted_mid.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
