"""Write the oracle's total energy of the N = 2^20 Plummer sphere (seed 3) at t = 0
with eps = 1e-4 (the benchmarked workload): kinetic and potential energy, 5.5e11
pairs (about half an hour on 8 host cores).  The GPU energy diagnostic is compared
with these values on the GPU; the CPU test recomputes the kinetic energy and checks
the stored potential against the Plummer closed form.

    OMP_NUM_THREADS=8 python tests/golden/make_energy_plummer_2pow20.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1411_5234_amd import inputs  # noqa: E402

N, SEED = 1 << 20, 3
OUT = os.path.join(HERE, "energy_plummer_2pow20_seed3.json")


def main():
    s = inputs.plummer(N, SEED)
    rec = {"workload": "equal-mass Plummer, N = 2^20, seed 3, t = 0",
           "made_by": "tests/golden/make_energy_plummer_2pow20.py (oracle.energy)", "energy": {}}
    for eps in (1e-4,):
        t0 = time.time()
        T, W, E = oracle.energy(s.x, s.v, s.m, eps)
        rec["energy"]["%g" % eps] = {"kinetic": T, "potential": W, "total": E}
        print("eps %g: T %.17g W %.17g E %.17g (%.0f s)" % (eps, T, W, E, time.time() - t0),
              flush=True)
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
