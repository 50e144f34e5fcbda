"""Writes the oracle regression fixture oracle_force_plummer16.json.

Calls only the oracle and the seeded input generator: a 16-body Plummer sphere
(seed 99), eps = 1e-2, acceleration and jerk of every body, and the total energy.
The paper prints no worked example, so this fixture guards the oracle against
unintended changes rather than pinning it to the paper.
Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1411_5234_amd import inputs  # noqa: E402


def main():
    s = inputs.plummer(16, 99)
    acc, jerk = oracle.force(s.x, s.v, s.m, 1e-2)
    T, W, E = oracle.energy(s.x, s.v, s.m, 1e-2)
    out = {"source": "oracle (nbody_oracle.c) on inputs.plummer(16, seed=99), eps=1e-2",
           "acc": acc.tolist(), "jerk": jerk.tolist(), "energy": [T, W, E]}
    with open(os.path.join(HERE, "oracle_force_plummer16.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
