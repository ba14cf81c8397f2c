"""Writes long_runs.json: the FP64 oracle's state after 1000 steps of the
8^3 x 6 Gaussian case (workloads config '1b', N = 3, and the precision case
'3', N = 5; HABC P = 3 on all faces), stored as the l2 norm and 128 evenly
spaced values of every state array, with the initial q3 norm.  It calls
only the oracle and the seeded input module.  Run from the repository root:

    python tests/golden/make_long_runs.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as w  # noqa: E402
from oracle.solver import Oracle  # noqa: E402

ARRAYS = ["q3", "res3", "q2", "res2", "qb3", "q0_3", "q1", "res1", "qb2", "q0_2", "qb1"]
NSAMPLE = 128


def sample_index(size):
    return np.linspace(0, size - 1, min(size, NSAMPLE)).round().astype(np.int64)


def run(name):
    cfg = w.config(name)
    VX, E = w.kuhn_mesh(cfg.n)
    K = E.shape[0]
    o = Oracle(VX, E, cfg.N, cfg.P, np.ones(K), np.ones(K))
    o.s = {k: np.zeros(v) for k, v in o.shapes().items()}
    o.s["q3"][:, 0] = w.gaussian_pulse(o.node_coords(), cfg.extra["center"], cfg.extra["width"])
    q0 = float(np.linalg.norm(o.s["q3"]))
    o.step(cfg.steps, cfg.dt)
    out = {"n": cfg.n, "N": cfg.N, "P": cfg.P, "steps": cfg.steps, "dt": cfg.dt,
           "q3_initial_norm": q0, "arrays": {}}
    for k in ARRAYS:
        a = o.s[k].reshape(-1)
        idx = sample_index(a.size)
        out["arrays"][k] = {"size": int(a.size), "norm": float(np.linalg.norm(a)),
                            "index": idx.tolist(), "values": [float(v) for v in a[idx]]}
    return out


if __name__ == "__main__":
    res = {name: run(name) for name in ("1b", "3")}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "long_runs.json")
    with open(path, "w") as f:
        json.dump(res, f, indent=0)
    print("wrote", path)
