"""The oracle still reproduces its stored regression fixture (tests/golden)."""
import json
import os

import numpy as np

from paper_1411_5234_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden", "oracle_force_plummer16.json")


def test_oracle_matches_stored_fixture(orc):
    g = json.load(open(GOLD))
    s = inputs.plummer(16, 99)
    acc, jerk = orc.force(s.x, s.v, s.m, 1e-2)
    np.testing.assert_allclose(acc, np.array(g["acc"]), rtol=1e-15, atol=0)
    np.testing.assert_allclose(jerk, np.array(g["jerk"]), rtol=1e-15, atol=0)
    np.testing.assert_allclose(orc.energy(s.x, s.v, s.m, 1e-2), g["energy"], rtol=1e-15)
