"""Helpers shared by the parity tests: build the oracle and the library on
the same seeded inputs, run both, compare array by array."""
import numpy as np

import workloads as w
from oracle.solver import Oracle

ARRAYS = ["q3", "res3", "q2", "res2", "qb3", "q0_3", "q1", "res1", "qb2", "q0_2", "qb1"]


def make_case(n=4, N=3, P=3, face_bc=None, periodic=None, medium="homogeneous", init="gaussian",
              seed=0, width=0.15, center=(0.5, 0.5, 0.5), source=None, lo=(0.0,) * 3,
              hi=(1.0,) * 3):
    VX, E = w.kuhn_mesh(n, lo=lo, hi=hi)
    K = E.shape[0]
    if medium == "layered":
        rho, c, *_ = w.layered_medium(n, seed=2)
    else:
        rho, c = np.ones(K), np.ones(K)
    fb = face_bc if face_bc is not None else ("habc",) * 6
    per = periodic if periodic is not None else (False, False, False)
    o = Oracle(VX, E, N, P, rho, c, face_bc=fb, periodic=per)
    state = {k: np.zeros(v) for k, v in o.shapes().items()}
    if init == "gaussian":
        state["q3"][:, 0] = w.gaussian_pulse(o.node_coords(), center, width)
    elif init == "random":
        rng_seed = seed
        for k in ARRAYS:
            if np.prod(state[k].shape):
                state[k] = w.random_array(state[k].shape, rng_seed)
            rng_seed += 1
    return dict(VX=VX, E=E, N=N, P=P, rho=rho, c=c, face_bc=fb, periodic=per, oracle=o,
                state=state, source=source, box=np.array(list(lo) + list(hi)))


def run_oracle(case, steps, dt, t0=0.0):
    o = case["oracle"]
    o.s = {k: v.copy() for k, v in case["state"].items()}
    if case["source"] is not None:
        xs, f0, ts = case["source"]
        o.sources = []
        o.set_source(xs, f0, ts)
    o.step(steps, dt, t0)
    return o.s


def make_solver(case, precision=0):
    from paper_1610_05023_amd import Solver
    s = Solver(case["VX"], case["E"], case["N"], case["P"], case["rho"], case["c"],
               face_bc=case["face_bc"], periodic=case["periodic"], box=case["box"],
               precision=precision)
    s.bind()
    s.set_state(case["state"])
    if case["source"] is not None:
        xs, f0, ts = case["source"]
        s.set_source(xs, f0, ts)
    return s


def rel_errors(got, ref):
    """Relative l2 error per array; arrays with a negligible reference norm
    are normalised by the norm of q3."""
    scale = np.linalg.norm(ref["q3"])
    out = {}
    for k in ARRAYS:
        if ref[k].size == 0:
            continue
        nr = np.linalg.norm(ref[k])
        den = nr if nr > 1e-30 * scale else scale
        out[k] = float(np.linalg.norm(got[k] - ref[k]) / den) if den > 0 else 0.0
    return out
