"""Writes long_runs.npz: the FP64 oracle's full state (every array of every
level) after 1000 steps of the 8^3 x 6 Gaussian case with HABC
P = 3 on all faces, at N = 3 (workloads config '1b') and N = 5 (the
precision case, config '3'), with the initial q3 norm.  It calls only the
oracle and the seeded input module.  Keys: '<config>/<steps>/<array>',
'<config>/q3_initial_norm', '<config>/meta' = (n, N, P, dt).  Run from the
repository root:

    python tests/golden/make_long_runs.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as w  # noqa: E402
from oracle.solver import Oracle  # noqa: E402

ARRAYS = ["q3", "res3", "q2", "res2", "qb3", "q0_3", "q1", "res1", "qb2", "q0_2", "qb1"]
SNAPSHOTS = (1000,)


def run(name, out):
    cfg = w.config(name)
    VX, E = w.kuhn_mesh(cfg.n)
    K = E.shape[0]
    o = Oracle(VX, E, cfg.N, cfg.P, np.ones(K), np.ones(K))
    o.s = {k: np.zeros(v) for k, v in o.shapes().items()}
    o.s["q3"][:, 0] = w.gaussian_pulse(o.node_coords(), cfg.extra["center"], cfg.extra["width"])
    out[f"{name}/q3_initial_norm"] = np.array(np.linalg.norm(o.s["q3"]))
    out[f"{name}/meta"] = np.array([cfg.n, cfg.N, cfg.P, cfg.dt])
    done = 0
    for snap in SNAPSHOTS:
        o.step(snap - done, cfg.dt, done * cfg.dt)
        done = snap
        for k in ARRAYS:
            out[f"{name}/{snap}/{k}"] = o.s[k].copy()
        print(f"{name}: {snap} steps", flush=True)


if __name__ == "__main__":
    res = {}
    for name in ("1b", "3"):
        run(name, res)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "long_runs.npz")
    np.savez_compressed(path, **res)
    print("wrote", path, os.path.getsize(path), "bytes")
