"""Writes the oracle regression fixtures in this folder.

Calls only the FP64 oracle and the seeded input generators; run from the
repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1609_04104_amd import inputs as I  # noqa: E402


def config1_first_frames(T=3):
    c = I.config1(T=T)
    o = oracle.TslOracle(c["n1"], c["n2"], c["r"], 0.1, c["A0"], c["B0"])
    gam, abar = [], []
    for fr in c["frames"]:
        s = o.push_points(fr.mask, fr.y)
        gam.append([s.gamma.real.tolist(), s.gamma.imag.tolist()])
        abar.append(s.alpha_bar)
    return {"what": "oracle gamma_t and alpha_bar_t, 64x64 low-rank points workload, R=8, lambda=0.1",
            "gamma": gam, "alpha_bar": abar}


if __name__ == "__main__":
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "oracle_config1_first_frames.json"), "w") as fh:
        json.dump(config1_first_frames(), fh, indent=1)
