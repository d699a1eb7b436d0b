"""Writes the frozen oracle values used as regression fixtures by the GPU parity tests.

Calls only ``oracle/`` (and the seeded input generator).  Run from the repo root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import named_config  # noqa: E402

CASES = [("uni_8x8_nt8", 0), ("uni_8x8_nt8", 1), ("coreg3_4x4_nt4", 0), ("uni_6x5_nt5", 2)]


def main():
    out = {}
    for name, seed in CASES:
        m = named_config(name, seed=seed)
        g = oracle.gradient(m, m.theta)
        ev = oracle.objective(m, m.theta)
        out[f"{name}:{seed}"] = {
            "theta": m.theta.tolist(),
            "f": float(g["f"]),
            "grad": [float(v) for v in g["grad"]],
            "logdet_p": float(ev["logdet_p"]),
            "logdet_c": float(ev["logdet_c"]),
            "N": m.N,
        }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_values.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
