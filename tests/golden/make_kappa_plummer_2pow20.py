"""Write the bodies of the N = 2^20 Plummer sphere (seed 3, eps = 1e-4, t = 0) whose
acceleration or jerk has the largest cancellation factor

    kappa_a = sum_j |a_ij| / |a_i|,   kappa_j = sum_j |jerk_ij| / |jerk_i|,

found by a full scan of every body with the oracle (about an hour and a half on 8
host cores).  The N = 2^20 GPU parity test checks these bodies on purpose, beside a
random sample: they are where an FP32 pair sum is furthest from the plain relative
error of the result.

    OMP_NUM_THREADS=8 python tests/golden/make_kappa_plummer_2pow20.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1411_5234_amd import inputs  # noqa: E402

N, SEED, EPS, TOP, CHUNK = 1 << 20, 3, 1e-4, 64, 8192
OUT = os.path.join(HERE, "kappa_plummer_2pow20_seed3.json")


def main():
    s = inputs.plummer(N, SEED)
    ka = np.empty(N)
    kj = np.empty(N)
    t0 = time.time()
    for i0 in range(0, N, CHUNK):
        il = np.arange(i0, min(N, i0 + CHUNK))
        a, j = oracle.force(s.x, s.v, s.m, EPS, il)
        sa, sj = oracle.force_scale(s.x, s.v, s.m, EPS, il)
        ka[il] = sa / np.linalg.norm(a, axis=1)
        kj[il] = sj / np.linalg.norm(j, axis=1)
        print("%d / %d bodies, %.0f s" % (il[-1] + 1, N, time.time() - t0), flush=True)
    top_a = np.argsort(-ka)[:TOP]
    top_j = np.argsort(-kj)[:TOP]
    q = [0.5, 0.9, 0.99, 0.999, 1.0]
    rec = {
        "workload": "equal-mass Plummer, N = 2^20, seed 3, eps = 1e-4, t = 0, all bodies",
        "made_by": "tests/golden/make_kappa_plummer_2pow20.py (oracle.force, oracle.force_scale)",
        "top_kappa_acc": {"index": top_a.tolist(), "kappa": ka[top_a].tolist()},
        "top_kappa_jerk": {"index": top_j.tolist(), "kappa": kj[top_j].tolist()},
        "quantiles": q,
        "kappa_acc_quantiles": np.quantile(ka, q).tolist(),
        "kappa_jerk_quantiles": np.quantile(kj, q).tolist(),
        "share_kappa_acc_le_10": float((ka <= 10).mean()),
        "share_kappa_jerk_le_8": float((kj <= 8).mean()),
    }
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    np.savez_compressed(os.path.join("/tmp", "kappa_plummer_2pow20_seed3_all.npz"), ka=ka, kj=kj)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
