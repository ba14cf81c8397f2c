"""Pins of the oracle's material-dependent and mixed-condition arithmetic:
the exact upwind flux between cells of different impedance (Section 3.2),
the rho c^2 and 1/rho factors of the pressure-velocity system (Section 2),
the boundary-cell materials of the face and edge levels, the Dirichlet
condition p = 0 next to HABC faces (Section 2.4), and the source wavelet
(Section 4.1).  Each is checked against closed forms of the continuous
problem or an exact discrete symmetry, never against the oracle's own
formulas."""
import math

import numpy as np
import pytest

import workloads as w
from oracle.solver import Oracle, ricker_integral


def _l2(o, d):
    """Mass-matrix L2 norm of per-element nodal fields d (K, F, Np)."""
    return math.sqrt(float(np.sum(o.m.J[:, None] * np.sum(d * (d @ o.m.tet.M.T), axis=2))))


# ---------------------------------------------------------------- energy ----
def _media(kind, n):
    K = 6 * n ** 3
    if kind == "layered":
        rho, c, *_ = w.layered_medium(n, seed=2, n_layers=3)
        return rho, c
    rng = np.random.default_rng(6)
    return rng.uniform(1.0, 2.5, K), rng.uniform(1.0, 3.0, K)


@pytest.mark.parametrize("medium", ["layered", "random"])
@pytest.mark.parametrize("bc,periodic", [("abc", False), ("dirichlet", False), ("abc", True)])
def test_energy_non_increasing_in_heterogeneous_media(medium, bc, periodic):
    """No source: the upwind flux between cells of different impedance only
    dissipates, so the energy with the weights 1/(rho c^2) and rho never
    grows (Section 4.1's argument, with cellwise materials).  The pulse
    starts where the medium jumps, so every interface carries flux."""
    n, N = 4, 2
    VX, E = w.kuhn_mesh(n)
    rho, c = _media(medium, n)
    o = Oracle(VX, E, N, 0, rho, c, face_bc=(bc,) * 6, periodic=(periodic,) * 3)
    x = o.node_coords()
    o.s["q3"][:, 0] = w.gaussian_pulse(x, (0.45, 0.5, 0.55), 0.2)
    o.s["q3"][:, 3] = 0.7 * w.gaussian_pulse(x, (0.55, 0.45, 0.5), 0.2)
    dt = w.kuhn_dt(n, N, float(c.max()))
    es = [o.energy()]
    for _ in range(80):
        o.step(1, dt)
        es.append(o.energy())
    es = np.array(es)
    assert np.all(es[1:] <= es[:-1] * (1 + 1e-14)), np.max(es[1:] / es[:-1])
    assert es[-1] < 0.995 * es[0]              # the jumps do dissipate


# ------------------------------------------------- plane wave, rho, c != 1 ----
def _plane_wave_error(n, N, rho, c, T):
    VX, E = w.kuhn_mesh(n)
    K = E.shape[0]
    o = Oracle(VX, E, N, 0, np.full(K, rho), np.full(K, c), face_bc=("abc",) * 6,
               periodic=(True, True, True))
    x = o.node_coords()
    k = 2 * np.pi * np.array([1.0, 0.0, 1.0])
    om = c * np.linalg.norm(k)                 # dispersion relation w = c |k|
    kh = k / np.linalg.norm(k)

    def exact(t):
        p = np.cos(x @ k - om * t)
        return np.stack([p, kh[0] * p / (rho * c), kh[1] * p / (rho * c), kh[2] * p / (rho * c)],
                        axis=1)

    o.s["q3"] = exact(0.0)
    dt0 = w.kuhn_dt(n, N, c)
    ns = int(np.ceil(T / dt0))
    o.step(ns, T / ns)
    return _l2(o, o.s["q3"] - exact(T)) / _l2(o, exact(T))


@pytest.mark.parametrize("rho,c", [(0.5, 2.5)])
def test_plane_wave_converges_with_rho_and_c(rho, c):
    """p = cos(k.x - w t), u = k p / (|k| rho c), w = c |k|: the DG solution
    converges to it at about rate N+1 (N = 2), so the wave speed c and the
    impedance rho c of the discrete system are those of the continuum."""
    N, T = 2, 0.06 / c
    e = [_plane_wave_error(n, N, rho, c, T) for n in (6, 12)]
    rate = np.log2(e[0] / e[1])
    assert rate > N + 0.5, (e, rate)
    assert e[1] < 5e-3, e


# -------------------------------------------- normal incidence, interface ----
def test_normal_incidence_reflection_and_transmission():
    """A right-going pressure pulse p = f(z - z0), w = p / Z1 meets a planar
    interface z = zi between impedances Z1 = rho1 c1 and Z2 = rho2 c2.
    Continuity of p and n.u gives, for z < zi, the incident pulse plus the
    reflected one R f(2 zi - z - z0 - c1 t), R = (Z2 - Z1)/(Z2 + Z1),
    travelling back with w = -p/Z1, and for z > zi the transmitted pulse
    T f(zi + (z - zi) c1/c2 - z0 - c1 t), T = 2 Z2/(Z1 + Z2), with w = p/Z2.
    The slab is periodic in x and y (3 x 3 x 16 cubic cells), with the basic
    ABC on the z faces (exact for normal incidence).  Checked when the
    pulses have separated: the whole field against the closed form, and the
    reflected and transmitted pressure integrals against R and T (the
    transmitted pulse is compressed by c2/c1)."""
    nz, N = 16, 3
    (r1, c1), (r2, c2) = (1.0, 1.0), (4.0, 0.75)
    Z1, Z2 = r1 * c1, r2 * c2
    R, T = (Z2 - Z1) / (Z2 + Z1), 2 * Z2 / (Z1 + Z2)
    h = 1.0 / nz
    VX, E = w.kuhn_mesh(0, hi=(3 * h, 3 * h, 1.0), dims=(3, 3, nz))
    _, _, kz = w.cell_index_of_element(0, dims=(3, 3, nz))
    zi, z0, width, t_end = 0.5, 0.25, 0.08, 0.5
    upper = (kz + 0.5) * h > zi
    rho, c = np.where(upper, r2, r1), np.where(upper, c2, c1)
    o = Oracle(VX, E, N, 0, rho, c, face_bc=("abc",) * 6, periodic=(True, True, False))
    z = o.node_coords()[..., 2]
    f = lambda s: np.exp(-(s / width) ** 2)
    o.s["q3"][:, 0] = f(z - z0)
    o.s["q3"][:, 3] = f(z - z0) / Z1
    dt0 = w.kuhn_dt(1, N, max(c1, c2), L=h)
    ns = int(np.ceil(t_end / dt0))
    o.step(ns, t_end / ns)
    below = z < zi
    inc, refl = f(z - z0 - c1 * t_end), R * f(2 * zi - z - z0 - c1 * t_end)
    trans = T * f(zi + (z - zi) * c1 / c2 - z0 - c1 * t_end)
    pin = np.where(below, inc + refl, trans)
    win = np.where(below, (inc - refl) / Z1, trans / Z2)
    ref = np.stack([pin, 0 * pin, 0 * pin, win], axis=1)
    err = _l2(o, o.s["q3"] - ref) / _l2(o, ref)
    assert err < 5e-3, err
    # the pulse integrals (int f = sqrt(pi) width) by the nodal quadrature
    wq = o.m.J[:, None] * o.m.tet.M.sum(axis=0)[None, :] / (3 * h) ** 2
    If = math.sqrt(math.pi) * width
    p, wz = o.s["q3"][:, 0], o.s["q3"][:, 3]
    assert abs(np.sum(wq * p * below) / If - R) < 1e-2 * R
    assert abs(np.sum(wq * p * ~below) / (If * c2 / c1) - T) < 1e-2 * T
    assert abs(np.sum(wq * wz * below) / If + R / Z1) < 1e-2 * R / Z1
    assert abs(np.sum(wq * wz * ~below) / (If * c2 / c1) - T / Z2) < 1e-2 * T / Z2


# ------------------------------------------ HABC with rho, c != 1 (levels) ----
@pytest.mark.parametrize("rho,c", [(0.6, 2.0)])
def test_habc_absorbs_in_a_medium_with_rho_and_c(rho, c):
    """The face and edge levels take the impedance and bulk modulus of their
    boundary cell.  In a homogeneous medium with rho, c != 1 the HABC error
    against a doubled domain decreases with the order as in unit media
    (Section 4.1), which it cannot do if the auxiliary fields use another
    impedance or wave speed than the interior."""
    n, N, width = 4, 3, 0.15

    def run(P, big):
        if big:
            VX, E = w.kuhn_mesh(2 * n, lo=(-0.5,) * 3, hi=(1.5,) * 3)
        else:
            VX, E = w.kuhn_mesh(n)
        K = E.shape[0]
        o = Oracle(VX, E, N, P, np.full(K, rho), np.full(K, c),
                   face_bc=("habc",) * 6 if P > 0 else ("abc",) * 6)
        o.s["q3"][:, 0] = w.gaussian_pulse(o.node_coords(), (0.5, 0.5, 0.5), width)
        dt = w.kuhn_dt(n, N, c)
        o.step(int(0.9 / c / dt), dt)
        return o.s["q3"]

    i, j, k = w.cell_index_of_element(n)
    t = np.arange(6 * n ** 3) % 6
    big = (((k + n // 2) * 2 * n + (j + n // 2)) * 2 * n + (i + n // 2)) * 6 + t
    ref = run(0, True)[big]
    err = [np.linalg.norm(run(P, False) - ref) / np.linalg.norm(ref) for P in (0, 1, 3)]
    assert err[0] > 5 * err[1] and err[1] > 2 * err[2], err


# ------------------------------------------------------ Ricker wavelet ----
def test_source_is_the_integral_of_the_ricker_wavelet():
    """S'(t) = s(t) with s the printed Ricker wavelet of Section 4.1,
    s(t) = (1 - 2 pi^2 f^2 (t - t0)^2) exp(-pi^2 f^2 (t - t0)^2), and S
    vanishes long before the delay."""
    f0, t0 = 2.5, 0.5
    s = lambda t: (1 - 2 * (math.pi * f0 * (t - t0)) ** 2) * math.exp(-(math.pi * f0 * (t - t0)) ** 2)
    hstep = 1e-5
    for t in np.linspace(-0.2, 1.4, 33):
        d = (ricker_integral(t + hstep, f0, t0) - ricker_integral(t - hstep, f0, t0)) / (2 * hstep)
        assert abs(d - s(t)) < 1e-8, (t, d, s(t))
    assert abs(ricker_integral(-1.0, f0, t0)) < 1e-20
    # and the amplitude scales it
    assert ricker_integral(0.3, f0, t0, amp=3.0) == 3.0 * ricker_integral(0.3, f0, t0)


# ----------------------------------------- Dirichlet face, method of images ----
@pytest.mark.parametrize("medium", ["random"])
def test_dirichlet_face_next_to_habc_is_the_odd_image(medium):
    """Free surface (Section 2.4): p = 0 on z = 1, HABC P = 3 on the other
    five faces (edges between two HABC faces keep their 1D levels, the four
    lower corners their 0D systems).  The same problem on the domain doubled
    by its mirror image in z = 1, with HABC on all six faces, the mirrored
    medium and odd initial data p(x, y, 2 - z) = -p(x, y, z), has an odd
    solution whose restriction to the unit cube solves the first problem (the
    method of images).  On the mirrored mesh this holds for the discrete
    solutions too, in every level: the mirror maps elements, faces, lines and
    nodes onto themselves, and at z = 1 the upwind fluxes of the odd
    solution reduce to the p = 0 fluxes of the 3D, 2D and 1D levels."""
    n, N, P = 4, 3, 3
    VX, E = w.kuhn_mesh(n)
    K = E.shape[0]
    if medium == "random":
        rng = np.random.default_rng(12)
        rho, c = rng.uniform(1.0, 2.0, K), rng.uniform(1.0, 1.5, K)
    else:
        rho, c = np.ones(K), np.ones(K)
    top = ("habc", "habc", "habc", "habc", "habc", "dirichlet")
    a = Oracle(VX, E, N, P, rho, c, face_bc=top)
    x = a.node_coords()
    odd = lambda y: (w.gaussian_pulse(y, (0.45, 0.55, 0.7), 0.15)
                     - w.gaussian_pulse(y, (0.45, 0.55, 1.3), 0.15))
    p0 = odd(x)
    a.s["q3"][:, 0] = p0
    VX2, E2, _ = w.mirror_doubled_mesh(VX, E, axis=2, plane=1.0)
    b = Oracle(VX2, E2, N, P, np.concatenate([rho, rho]), np.concatenate([c, c]),
               box=((0.0, 0.0, 0.0), (1.0, 1.0, 2.0)))
    xb = b.node_coords()
    assert np.allclose(xb[:K], x, atol=1e-14)
    b.s["q3"][:, 0] = odd(xb)
    dt = w.kuhn_dt(n, N, float(c.max()))
    steps = int(0.75 / dt)                     # the pulse reaches the faces, edges and corners
    a.step(steps, dt)
    b.step(steps, dt)
    assert np.abs(a.s["qb1"]).max() > 1e-7      # lower corners active
    assert np.abs(a.s["q1"]).max() > 1e-5       # vertical lines touching z = 1 active
    d = np.linalg.norm(a.s["q3"] - b.s["q3"][:K]) / np.linalg.norm(a.s["q3"])
    assert d < 1e-12, d
    # the face level on x- (triangles of the unit cube lie on both meshes)
    ta = a.m.tri_xn.reshape(a.m.Ktri, -1)
    tb = b.m.tri_xn.reshape(b.m.Ktri, -1)
    from scipy.spatial import cKDTree
    dist, idx = cKDTree(tb).query(ta)
    assert dist.max() < 1e-12
    d2 = np.linalg.norm(a.s["q2"] - b.s["q2"][idx]) / np.linalg.norm(a.s["q2"])
    assert d2 < 1e-12, d2
    # the mirror makes the top face matter: the same run with HABC there differs
    h = Oracle(VX, E, N, P, rho, c)
    h.s["q3"][:, 0] = p0
    h.step(steps, dt)
    assert np.linalg.norm(h.s["q3"] - a.s["q3"]) > 0.1 * np.linalg.norm(a.s["q3"])


# --------------------------------- Riemann problems at every face (all levels) ----
def _middle_state(pL, unL, ZL, pR, unR, ZR):
    """Middle state of the Riemann problem of the acoustic system across a
    face with normal n from side L to side R: the characteristic leaving L,
    p + Z_L n.u, and the one leaving R, p - Z_R n.u, keep their values
    (waves move at c_L into L and c_R into R).  Solved as the 2 x 2 system."""
    A = np.array([[1.0, ZL], [1.0, -ZR]])
    return np.linalg.solve(A, np.array([pL + ZL * unL, pR - ZR * unR]))


def _bc_state(kind, pL, unL, Z, rminus=0.0):
    """Boundary middle state: the outgoing characteristic p + Z n.u keeps
    its value; the incoming one (p - Z n.u)/2 is the given r- (HABC, r- = 0
    for the basic ABC), or the pressure vanishes (Dirichlet)."""
    row = [1.0, 0.0] if kind == "dirichlet" else [1.0, -Z]
    rhs = 0.0 if kind == "dirichlet" else 2.0 * rminus
    return np.linalg.solve(np.array([[1.0, Z], row]), np.array([pL + Z * unL, rhs]))


def _mean(Mref, f):
    """Cell mean of nodal fields f (..., Np) under the reference mass matrix."""
    w1 = Mref.sum(axis=0)
    return (f @ w1) / w1.sum()


@pytest.mark.parametrize("face_bc", [
    ("periodic", "periodic", "habc", "abc", "dirichlet", "habc"),
    ("habc", "habc", "habc", "abc", "habc", "dirichlet"),
])
def test_cell_means_follow_riemann_fluxes_in_every_level(face_bc):
    """Piecewise-constant data: every field constant per element (per set on
    the faces and lines), random cellwise rho and c, random incoming
    characteristics qb.  The volume terms vanish and the cell mean of each
    right-hand side is the finite-volume balance of the element,
      d<p>/dt = -(K/|e|) sum_f |f| (n.u)*_f,  d<u>/dt = -(1/(rho |e|)) sum_f |f| p*_f n_f,
    with (p*, (n.u)*) the Riemann middle state of each face between the
    element's own impedance and its neighbour's (or the boundary condition).
    K is rho c^2 in 3D (Section 2), rho c^2/(1 + gamma_i) on the faces and
    rho c^2/(1 + gamma_i + gamma_j) on the lines (Section 3.1's auxiliary
    systems), with the rho and c of the boundary cell.  Geometry (areas,
    lengths, normals, volumes) is taken from the vertex coordinates here."""
    n, N, P = 3, 2, 2
    VX, E = w.kuhn_mesh(n)
    K = E.shape[0]
    rng = np.random.default_rng(21)
    rho, c = rng.uniform(1.0, 2.5, K), rng.uniform(1.0, 3.0, K)
    per = tuple(face_bc[2 * a] == "periodic" for a in range(3))
    o = Oracle(VX, E, N, P, rho, c, face_bc=face_bc, periodic=per)
    m = o.m
    g = o.gamma
    Z = rho * c
    # ---- 3D
    q3 = np.repeat(rng.standard_normal((K, 4))[:, :, None], m.tet.Np, axis=2)
    qb3 = np.repeat(rng.standard_normal((m.Ktri, 1)), m.tri.Np, axis=1)
    got = _mean(m.tet.M, o.rhs3d(q3, qb3, 0.0))            # (K, 4)
    xn = o.node_coords()
    want = np.zeros((K, 4))
    for k in range(K):
        verts = VX[E[k]]
        vol = abs(np.linalg.det((verts[1:] - verts[0]).T)) / 6.0
        for f in range(4):
            fx = xn[k, m.tet.Fmask[f]]
            on = [np.min(np.linalg.norm(fx - v, axis=1)) < 1e-12 for v in verts]
            fv, opp = verts[np.array(on)], verts[~np.array(on)][0]
            cr = np.cross(fv[1] - fv[0], fv[2] - fv[0])
            area = 0.5 * np.linalg.norm(cr)
            nv = cr / np.linalg.norm(cr)
            if np.dot(nv, fv[0] - opp) < 0:
                nv = -nv
            pL, unL = q3[k, 0, 0], nv @ q3[k, 1:, 0]
            k2 = m.EToE[k, f]
            if k2 >= 0:
                ps, uns = _middle_state(pL, unL, Z[k], q3[k2, 0, 0], nv @ q3[k2, 1:, 0], Z[k2])
            else:
                bc = face_bc[m.bface[k, f]]
                rm = qb3[m.face_tri[k, f], 0] if bc == "habc" else 0.0
                ps, uns = _bc_state(bc, pL, unL, Z[k], rm)
            want[k, 0] -= rho[k] * c[k] ** 2 * area * uns / vol
            want[k, 1:] -= area * ps * nv / (rho[k] * vol)
    assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max(), np.abs(got - want).max()
    # ---- 2D (sets i = 0..P-1)
    Kt = m.Ktri
    q2 = np.repeat(rng.standard_normal((Kt, P, 3))[..., None], m.tri.Np, axis=3)
    qb2 = np.repeat(rng.standard_normal((m.Klin, 2, P, 1)), m.line.Np, axis=3)
    got2 = _mean(m.tri.M, o.rhs2d(q2, qb2))                 # (Kt, P, 3)
    want2 = np.zeros((Kt, P, 3))
    Nn = m.tri.Np
    corners = [0, N, Nn - 1]                                # lattice corners (-1,-1), (1,-1), (-1,1)
    for t in range(Kt):
        e = m.tri_elem[t]
        ax = m.tri_axes[t]
        cv = m.tri_xn[t, corners][:, ax]                    # corners in the face plane
        d1, d2 = cv[1] - cv[0], cv[2] - cv[0]
        area = 0.5 * abs(d1[0] * d2[1] - d1[1] * d2[0])
        cen = cv.mean(axis=0)
        for f in range(3):
            ex = m.tri_xn[t, m.tri.Fmask[f]][:, ax]
            a, b = ex[0], ex[-1]
            length = np.linalg.norm(b - a)
            nv = np.array([b[1] - a[1], a[0] - b[0]]) / length
            if np.dot(nv, a - cen) < 0:
                nv = -nv
            for i in range(P):
                Ki = rho[e] * c[e] ** 2 / (1.0 + g[i])
                pL, unL = q2[t, i, 0, 0], nv @ q2[t, i, 1:, 0]
                t2 = m.tri_EToE[t, f]
                if t2 >= 0:
                    e2 = m.tri_elem[t2]
                    ps, uns = _middle_state(pL, unL, Z[e], q2[t2, i, 0, 0], nv @ q2[t2, i, 1:, 0],
                                            Z[e2])
                else:
                    l = m.tri_edge_line[t, f]
                    if l >= 0:
                        ps, uns = _bc_state("habc", pL, unL, Z[e],
                                            qb2[l, m.tri_edge_side[t, f], i, 0])
                    else:
                        bc = face_bc[m.tri_bdface[t, f]]
                        ps, uns = _bc_state("dirichlet" if bc == "dirichlet" else "abc", pL, unL,
                                            Z[e])
                want2[t, i, 0] -= Ki * length * uns / area
                want2[t, i, 1:] -= length * ps * nv / (rho[e] * area)
    assert np.abs(got2 - want2).max() <= 1e-11 * np.abs(want2).max(), np.abs(got2 - want2).max()
    # ---- 1D (sets (i, j))
    Kl = m.Klin
    if Kl == 0:
        return
    q1 = np.repeat(rng.standard_normal((Kl, P * P, 2, 1)), m.line.Np, axis=3)
    qb1 = rng.standard_normal((m.Kpnt, 3, P * P))
    got1 = _mean(m.line.M, o.rhs1d(q1, qb1))                # (Kl, P*P, 2)
    want1 = np.zeros((Kl, P * P, 2))
    kinds = set()
    for l in range(Kl):
        e = m.tri_elem[m.lin_tri[l, 0]]
        a_, b_ = m.lin_xn[l, 0], m.lin_xn[l, -1]
        length = np.linalg.norm(b_ - a_)
        d = (b_ - a_) / length
        axis = int(np.argmax(np.abs(d)))
        for end, nsgn in ((0, -np.sign(d[axis])), (1, np.sign(d[axis]))):
            for i in range(P):
                for j in range(P):
                    s = i * P + j
                    Kij = rho[e] * c[e] ** 2 / (1.0 + g[i] + g[j])
                    pL, unL = q1[l, s, 0, 0], nsgn * q1[l, s, 1, 0]
                    l2 = m.lin_EToE[l, end]
                    if l2 >= 0:
                        e2 = m.tri_elem[m.lin_tri[l2, 0]]
                        ps, uns = _middle_state(pL, unL, Z[e], q1[l2, s, 0, 0],
                                                nsgn * q1[l2, s, 1, 0], Z[e2])
                        kinds.add("interior")
                    elif m.lin_corner[l, end] >= 0:
                        ps, uns = _bc_state("habc", pL, unL, Z[e],
                                            qb1[m.lin_corner[l, end], m.lin_corner_slot[l, end], s])
                        kinds.add("corner")
                    else:
                        bc = m.lin_bc[l, end]
                        ps, uns = _bc_state("dirichlet" if bc == "dirichlet" else "abc", pL, unL,
                                            Z[e])
                        kinds.add(bc)
                    want1[l, s, 0] -= Kij * uns / length
                    want1[l, s, 1] -= nsgn * ps / (rho[e] * length)
    assert np.abs(got1 - want1).max() <= 1e-11 * np.abs(want1).max(), np.abs(got1 - want1).max()
    if face_bc[5] == "dirichlet":
        assert {"interior", "corner", "dirichlet", "abc"} <= kinds, kinds
