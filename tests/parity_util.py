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


# field names of each array's field axis (canonical layouts)
FIELDS = {"q3": (1, ("p", "u", "v", "w")), "res3": (1, ("p", "u", "v", "w")),
          "q2": (2, ("p", "va", "vb")), "res2": (2, ("p", "va", "vb")),
          "q1": (2, ("p", "w")), "res1": (2, ("p", "w"))}


def field_errors(got, ref):
    """Relative l2 error per level and per field: 'q3.p', 'q3.u', ...,
    'q2.p', 'q2.va', 'q2.vb', 'q1.p', 'q1.w' (the residuals likewise) and
    the coupling arrays qb3, q0_3, qb2, q0_2, qb1 whole.  A field whose
    reference norm is below 1e-30 of the q3 norm is normalised by the q3
    norm instead."""
    scale = np.linalg.norm(ref["q3"])
    out = {}
    for k in ARRAYS:
        if ref[k].size == 0:
            continue
        if k in FIELDS:
            ax, names = FIELDS[k]
            parts = [(f"{k}.{nm}", np.take(got[k], i, axis=ax), np.take(ref[k], i, axis=ax))
                     for i, nm in enumerate(names)]
        else:
            parts = [(k, got[k], ref[k])]
        for name, a, b in parts:
            nr = np.linalg.norm(b)
            den = nr if nr > 1e-30 * scale else scale
            out[name] = float(np.linalg.norm(a - b) / den) if den > 0 else 0.0
    return out


def fmt_errors(err):
    return "{" + ", ".join(f"{k}: {v:.1e}" for k, v in err.items()) + "}"


def corner_block(VX, E, n, m):
    """The m^3-cell block at the far corner (x, y, z up to the box's upper
    faces) of the n^3-cell Kuhn mesh ``workloads.kuhn_mesh(n)``: its tets in
    the full mesh's order with the full mesh's coordinates.  Returns
    (VXb, Eb, efull, cmin): the block mesh, the full index of each block
    element and each block element's smallest cell index over the three axes."""
    i0 = n - m
    r = np.arange(i0, n)
    kc, jc, ic = [a.ravel() for a in np.meshgrid(r, r, r, indexing="ij")]
    cell = (kc * n + jc) * n + ic
    efull = (cell[:, None] * 6 + np.arange(6)[None, :]).ravel()
    vids, inv = np.unique(E[efull], return_inverse=True)    # order-preserving renumbering
    cmin = np.repeat(np.minimum(np.minimum(kc, jc), ic), 6)
    return VX[vids], inv.reshape(-1, 4).astype(np.int32), efull, cmin


def kuhn_triangle_order(VX, E, n):
    """Canonical triangle index (domain face, tet, local face) -> row of the
    n^3-cell Kuhn mesh with HABC on all six faces, from the boundary cells."""
    from oracle.reference import FACE_VERTS
    fv = np.array(FACE_VERTS)
    out, base = {}, 0
    c = np.arange(n ** 3)
    cidx = [c % n, (c // n) % n, c // (n * n)]
    for d in range(6):
        ax, hi = d // 2, d % 2
        cells = c[cidx[ax] == (n - 1 if hi else 0)]
        e = (cells[:, None] * 6 + np.arange(6)[None, :]).ravel()
        x = VX[E[e][:, fv], ax]                                    # (tets, 4 faces, 3)
        on = np.all(x == (1.0 if hi else 0.0), axis=2)
        te, tf = np.nonzero(on)
        recs = sorted(zip(e[te].tolist(), tf.tolist()))
        for k, (ee, ff) in enumerate(recs):
            out[(d, ee, ff)] = base + k
        base += len(recs)
    return out


def block_maps(om, VX, E, n, m, efull):
    """Full-mesh rows of every block array (the block's oracle mesh om; full
    mesh with HABC on all faces): tets, triangles, lines (the last m of their
    domain edge) and the corner x+ y+ z+ (index 7).  Also returns each block
    line's position along its edge."""
    tri = kuhn_triangle_order(VX, E, n)
    tmap = np.array([tri[(int(om.tri_dface[t]), int(efull[om.tri_elem[t]]), int(om.tri_face[t]))]
                     for t in range(om.Ktri)], dtype=np.int64)
    first = {int(d): int(np.argmax(om.lin_dedge == d)) for d in np.unique(om.lin_dedge)}
    lpos = np.array([l - first[int(om.lin_dedge[l])] for l in range(om.Klin)], dtype=np.int64)
    lmap = om.lin_dedge * n + (n - m) + lpos
    maps = {"q3": efull, "res3": efull, "q2": tmap, "res2": tmap, "qb3": tmap, "q0_3": tmap,
            "q1": lmap, "res1": lmap, "qb2": lmap, "q0_2": lmap, "qb1": np.array([7])}
    return maps, lpos


def block_sample(om, cmin, lpos, n, m, cut):
    """Rows of the block's arrays at least `cut` cells from its cut faces."""
    far = cmin >= n - m + cut
    keep = {"q3": far, "res3": far, "qb1": np.ones(1, dtype=bool)}
    for k in ("q2", "res2", "qb3", "q0_3"):
        keep[k] = far[om.tri_elem]
    for k in ("q1", "res1", "qb2", "q0_2"):
        keep[k] = lpos >= cut
    return keep

