"""Pins of the oracle's time step against closed forms and invariants:
the LSRK scheme (Carpenter & Kennedy), h-convergence to a plane wave on a
periodic cube, energy decay with the basic ABC / Dirichlet / periodic
conditions (Section 4.1's argument), P = 0 HABC equal to the basic ABC,
the symmetry of the Kuhn mesh, the point-source projection, and the HABC
reflection decreasing with the order against a large-domain run."""
import numpy as np
import pytest

import workloads as w
from oracle.solver import Oracle, LSRK_A, LSRK_B, LSRK_C


def _lsrk_scalar(lam, dt, n=1):
    y, res = 1.0 + 0j, 0j
    for _ in range(n):
        for s in range(5):
            res = LSRK_A[s] * res + dt * lam * y
            y = y + LSRK_B[s] * res
    return y


def test_lsrk_stability_polynomial():
    # R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 + c5 z^5 with c5 = 1/200
    zs = np.array([0.1, -0.3, 0.2j, -1.0 + 0.5j, 0.7j, -0.5 - 0.4j, 0.9, -1.2j])
    R = np.array([_lsrk_scalar(z, 1.0) for z in zs])
    coef = np.linalg.lstsq(np.vander(zs, 6, increasing=True), R, rcond=None)[0]
    assert np.allclose(coef[:5], [1, 1, 0.5, 1 / 6, 1 / 24], atol=1e-12)
    assert abs(coef[5] - 1 / 200) < 1e-9


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_lsrk_exact_for_polynomials_in_time(p):
    # y' = t^p integrated exactly by a 4th order method for p <= 3
    dt, y, res, t = 0.37, 0.0, 0.0, 0.2
    for s in range(5):
        res = LSRK_A[s] * res + dt * (t + LSRK_C[s] * dt) ** p
        y = y + LSRK_B[s] * res
    exact = ((t + dt) ** (p + 1) - t ** (p + 1)) / (p + 1)
    assert abs(y - exact) < 1e-14


def _plane_wave_error(n, N, T=0.05):
    VX, E = w.kuhn_mesh(n)
    K = E.shape[0]
    o = Oracle(VX, E, N, 0, np.ones(K), np.ones(K), face_bc=("abc",) * 6,
               periodic=(True, True, True))
    x = o.node_coords()
    k = 2 * np.pi * np.array([1.0, 1.0, 1.0])
    om = np.linalg.norm(k)
    kh = k / om

    def exact(t):
        p = np.cos(x @ k - om * t)
        return np.stack([p, kh[0] * p, kh[1] * p, kh[2] * p], axis=1)

    o.s["q3"] = exact(0.0)
    dt0 = w.kuhn_dt(n, N, 1.0)
    ns = int(np.ceil(T / dt0))
    o.step(ns, T / ns)
    d = o.s["q3"] - exact(T)
    return np.sqrt(np.sum(o.m.J[:, None] * np.sum(d * (d @ o.m.tet.M.T), axis=2)))


@pytest.mark.parametrize("N,ns", [(1, (8, 16)), (2, (6, 12)), (3, (4, 8))])
def test_plane_wave_h_convergence(N, ns):
    """p = cos(k.x - w t), u = k p / |k| on the periodic unit cube: the L2
    error decreases at rate about N+1 (upwind DG, smooth solution)."""
    e = [_plane_wave_error(n, N) for n in ns]
    rate = np.log2(e[0] / e[1])
    assert rate > N + 0.5, (e, rate)


def _energy_run(face_bc, periodic=(False, False, False), P=0, steps=120):
    n, N = 4, 2
    VX, E = w.kuhn_mesh(n)
    K = E.shape[0]
    o = Oracle(VX, E, N, P, np.ones(K), np.ones(K), face_bc=face_bc, periodic=periodic)
    o.s["q3"][:, 0] = w.gaussian_pulse(o.node_coords(), (0.4, 0.5, 0.6), 0.15)
    dt = w.kuhn_dt(n, N, 1.0)
    es = [o.energy()]
    for _ in range(steps):
        o.step(1, dt)
        es.append(o.energy())
    return np.array(es)


@pytest.mark.parametrize("bc,periodic", [("abc", False), ("dirichlet", False), ("abc", True)])
def test_energy_non_increasing(bc, periodic):
    es = _energy_run((bc,) * 6, periodic=(periodic,) * 3)
    assert np.all(es[1:] <= es[:-1] * (1 + 1e-14))
    if bc == "abc" and not periodic:
        assert es[-1] < 0.5 * es[0]            # energy leaves through the ABC


def test_habc_order_zero_is_basic_abc():
    n, N = 3, 2
    VX, E = w.kuhn_mesh(n)
    K = E.shape[0]
    runs = []
    for bc in ("habc", "abc"):
        o = Oracle(VX, E, N, 0, np.ones(K), np.ones(K), face_bc=(bc,) * 6)
        o.s["q3"] = w.random_array(o.s["q3"].shape, 5)
        o.step(20, 1e-3)
        runs.append(o.s["q3"])
    assert np.array_equal(runs[0], runs[1])


def test_kuhn_symmetry_all_levels_visible_in_volume():
    """Centred pulse, HABC P = 3 on all faces with edges and corners: the 3D
    solution is invariant under the central inversion x -> 1 - x and under
    swapping the x and y axes, which map the Kuhn mesh onto itself.  The run
    is long enough for the wave to reach faces, edges and corners, so the 2D,
    1D and 0D levels all feed back into the volume."""
    n, N, P = 4, 3, 3
    VX, E = w.kuhn_mesh(n)
    K = E.shape[0]
    o = Oracle(VX, E, N, P, np.ones(K), np.ones(K))
    x = o.node_coords()
    o.s["q3"][:, 0] = w.gaussian_pulse(x, (0.5, 0.5, 0.5), 0.15)
    o.step(330, w.kuhn_dt(n, N, 1.0))
    assert np.abs(o.s["qb1"]).max() > 1e-6       # corners active
    q = o.s["q3"].transpose(0, 2, 1).reshape(-1, 4)
    X = x.reshape(-1, 3)
    from scipy.spatial import cKDTree
    # element-wise node sets: map each node to the node of the image element
    cen = x.mean(axis=1)
    tree_c = cKDTree(cen)
    for T, S in ((lambda y: 1.0 - y, np.diag([-1.0, -1.0, -1.0])),
                 (lambda y: y[..., [1, 0, 2]], np.array([[0, 1, 0], [1, 0, 0], [0, 0, 1.0]]))):
        _, eimg = tree_c.query(T(cen))
        worst = 0.0
        for e in range(K):
            xe = T(x[e])
            d = np.linalg.norm(xe[:, None, :] - x[eimg[e]][None, :, :], axis=2)
            nimg = np.argmin(d, axis=1)
            assert d[np.arange(len(nimg)), nimg].max() < 1e-12
            pe, pimg = o.s["q3"][e, 0], o.s["q3"][eimg[e], 0, nimg]
            ue, uimg = o.s["q3"][e, 1:], o.s["q3"][eimg[e], 1:][:, nimg]
            worst = max(worst, np.abs(pe - pimg).max(), np.abs(S @ ue - uimg).max())
        assert worst < 1e-12 * np.abs(q).max(), worst


def test_point_source_projection():
    """The nodal source weights w satisfy M_k w = l(x_s) (the L2 projection of
    delta(x - x_s)): integral 1, first moments x_s."""
    VX, E = w.kuhn_mesh(3)
    K = E.shape[0]
    o = Oracle(VX, E, 3, 0, np.ones(K), np.ones(K), face_bc=("abc",) * 6)
    xs = np.array([0.41, 0.52, 0.33])
    k, wgt = o.set_source(xs, 5.0, 0.2)
    Mk = o.m.J[k] * o.m.tet.M
    assert abs(np.sum(Mk @ wgt) - 1.0) < 1e-12
    assert np.allclose(o.node_coords()[k].T @ (Mk @ wgt), xs, atol=1e-12)


def test_energy_weights():
    VX, E = w.kuhn_mesh(2)
    K = E.shape[0]
    rho, c = np.full(K, 2.0), np.full(K, 3.0)
    o = Oracle(VX, E, 2, 0, rho, c, face_bc=("abc",) * 6)
    o.s["q3"][:, 0] = 1.0
    assert abs(o.energy() - 1.0 / (2 * 2.0 * 9.0)) < 1e-14
    o.s["q3"][:] = 0.0
    o.s["q3"][:, 2] = 1.0
    assert abs(o.energy() - 2.0 / 2) < 1e-14


def test_habc_reflection_decreases_with_order():
    """Against a run on the 2x larger cube (no reflection reaches the unit
    cube before t = 1), the error on the unit cube at t = 0.9 decreases from
    the basic ABC to HABC orders 1 and 3 (Section 4.1: the error minimum
    decreases with the order until the discretisation error dominates)."""
    n, N, width = 4, 3, 0.15

    def run(P, big):
        if big:
            VX, E = w.kuhn_mesh(2 * n, lo=(-0.5,) * 3, hi=(1.5,) * 3)
        else:
            VX, E = w.kuhn_mesh(n)
        K = E.shape[0]
        o = Oracle(VX, E, N, P, np.ones(K), np.ones(K),
                   face_bc=("habc",) * 6 if P > 0 else ("abc",) * 6)
        o.s["q3"][:, 0] = w.gaussian_pulse(o.node_coords(), (0.5, 0.5, 0.5), width)
        dt = w.kuhn_dt(n, N, 1.0)
        o.step(int(0.9 / dt), dt)
        return o.s["q3"]

    i, j, k = w.cell_index_of_element(n)
    t = np.arange(6 * n ** 3) % 6
    big = (((k + n // 2) * 2 * n + (j + n // 2)) * 2 * n + (i + n // 2)) * 6 + t
    ref = run(0, True)[big]
    err = [np.linalg.norm(run(P, False) - ref) / np.linalg.norm(ref) for P in (0, 1, 3)]
    assert err[0] > 5 * err[1] and err[1] > 2 * err[2], err


def test_far_corner_block_reproduces_full_mesh():
    """The sampling used on meshes too large for the oracle: one step on the
    m^3-cell block at the far corner (its other faces cut, basic ABC) equals
    one step on the whole n^3-cell mesh at least six cells from the cuts, in
    every array of every level (one step moves information at most five
    element layers).  Also checks the full mesh's canonical triangle order
    rebuilt from its boundary cells."""
    from parity_util import ARRAYS, block_maps, block_sample, corner_block, kuhn_triangle_order
    n, m, cut, N, P = 14, 12, 6, 3, 2
    h = 1.0 / n
    VX, E = w.kuhn_mesh(n)
    K = E.shape[0]
    full = Oracle(VX, E, N, P, np.ones(K), np.ones(K))
    fm = full.m
    tri = kuhn_triangle_order(VX, E, n)
    assert len(tri) == fm.Ktri
    for t in range(fm.Ktri):
        assert tri[(int(fm.tri_dface[t]), int(fm.tri_elem[t]), int(fm.tri_face[t]))] == t
    VXb, Eb, efull, cmin = corner_block(VX, E, n, m)
    blk = Oracle(VXb, Eb, N, P, np.ones(len(Eb)), np.ones(len(Eb)),
                 face_bc=("abc", "habc", "abc", "habc", "abc", "habc"))
    maps, lpos = block_maps(blk.m, VX, E, n, m, efull)
    # the maps point at the same places: nodes, triangle and line positions
    assert np.array_equal(blk.node_coords(), full.node_coords()[efull])
    assert np.array_equal(blk.m.tri_xn, fm.tri_xn[maps["q2"]])
    assert np.array_equal(blk.m.lin_xn, fm.lin_xn[maps["q1"]])
    shapes = full.shapes()
    full.s = {k: w.random_array(shapes[k], 50 + j) for j, k in enumerate(ARRAYS)}
    blk.s = {k: full.s[k][maps[k]].copy() for k in ARRAYS}
    xs = (1 - 3.3 * h, 1 - 4.2 * h, 1 - 2.1 * h)
    full.set_source(xs, 6.0, 0.0)
    blk.set_source(xs, 6.0, 0.0)
    dt = w.kuhn_dt(n, N, 1.0)
    full.step(1, dt)
    blk.step(1, dt)
    keep = block_sample(blk.m, cmin, lpos, n, m, cut)
    for k in ARRAYS:
        a, b = blk.s[k][keep[k]], full.s[k][maps[k]][keep[k]]
        assert a.size > 0, k
        assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b), k
    # and the cut does matter nearer than that
    near = ~keep["q3"]
    a, b = blk.s["q3"][near], full.s["q3"][maps["q3"]][near]
    assert np.linalg.norm(a - b) > 1e-6 * np.linalg.norm(b)
