"""Writes the stored expected values under tests/golden/ that come from the oracle.

Run from the repository root:  python tests/golden/make_golden.py
It calls only the oracle package (Maxwell construction of the Peng-Robinson EOS with the
paper's a = 3/49, b = 2/21, R = 1, acentric factor 0.344).
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1912_02018_amd.config import LBMConfig  # noqa: E402


def main():
    cfg = LBMConfig()
    tc = oracle.Tc(cfg)
    out = {"_source": "python tests/golden/make_golden.py (oracle Maxwell construction)",
           "Tc": tc, "coexistence": {}}
    for tr in (0.80, 0.86, 0.90, 0.95):
        rv, rl, ps = oracle.maxwell(cfg, tr * tc)
        out["coexistence"][f"{tr:.2f}"] = {"rho_v": rv, "rho_l": rl, "p_sat": ps,
                                           "h_fg": oracle.hfg(cfg, tr * tc)}
    path = os.path.join(ROOT, "tests", "golden", "maxwell_coexistence.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=2)
    print(path)


if __name__ == "__main__":
    main()
