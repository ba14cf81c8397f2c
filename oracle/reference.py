"""Nodal reference elements of the oracle (FP64; test infrastructure, never
imported by the library).

Section 3.2 of the paper: nodal DG on tetrahedra, triangles and lines; the
tetrahedron nodes come from the Warp & Blend construction (Warburton 2006)
and the triangle and line nodes are the tetrahedron's face and edge nodes.
Modal basis: orthonormal Jacobi / collapsed-coordinate (Dubiner) bases;
Vandermonde-based differentiation and lifting matrices (Hesthaven & Warburton
2007, cited in Section 3.2).

Node order (part of the canonical state layout): lattice points
(i, j, k), i + j + k <= N, with k slowest and i fastest; the barycentric
coordinates are (N-i-j-k, i, j, k)/N for the reference vertices
(-1,-1,-1), (1,-1,-1), (-1,1,-1), (-1,-1,1).  Triangle nodes are the tet
nodes with k = 0 in the same order; line nodes are GLL points ascending.
"""
from __future__ import annotations

import math

import numpy as np

# Optimised blend parameters of the Warp & Blend construction for the
# tetrahedron, N = 1..15 (Warburton 2006); alpha = 1 beyond.
WB_ALPHA_TET = [0.0, 0.0, 0.0, 0.1002, 1.1332, 1.5608, 1.3413, 1.2577, 1.1603,
                1.10153, 0.6080, 0.4523, 0.8856, 0.8717, 0.9655]

REF_VERTS = np.array([[-1.0, -1.0, -1.0], [1.0, -1.0, -1.0],
                      [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]])
# Local faces by their vertices; face f is the one opposite vertex OPP[f].
FACE_VERTS = [(0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3)]
FACE_OPP = [3, 2, 0, 1]
# Triangle edges: edge 0 is s=-1 (v0,v1), edge 1 r+s=0 (v1,v2), edge 2 r=-1 (v0,v2)
TRI_EDGE_VERTS = [(0, 1), (1, 2), (0, 2)]


# ---------------------------------------------------------------- Jacobi ---
def jacobi_p(x, alpha, beta, n):
    """Orthonormal Jacobi polynomial P_n^{(alpha,beta)} on [-1, 1]
    (three-term recurrence of the normalised polynomials)."""
    x = np.asarray(x, dtype=np.float64)
    # g0 = integral of the weight (1-x)^alpha (1+x)^beta over [-1, 1]
    g0 = (2.0 ** (alpha + beta + 1) * math.gamma(alpha + 1) * math.gamma(beta + 1)
          / math.gamma(alpha + beta + 2))
    p_prev = np.full_like(x, 1.0 / math.sqrt(g0))
    if n == 0:
        return p_prev
    g1 = (alpha + 1) * (beta + 1) / (alpha + beta + 3) * g0
    p = ((alpha + beta + 2) * x / 2 + (alpha - beta) / 2) / math.sqrt(g1)
    if n == 1:
        return p
    a_old = 2.0 / (2 + alpha + beta) * math.sqrt((alpha + 1) * (beta + 1) / (alpha + beta + 3))
    for i in range(1, n):
        h1 = 2 * i + alpha + beta
        a_new = 2.0 / (h1 + 2) * math.sqrt((i + 1) * (i + 1 + alpha + beta) * (i + 1 + alpha)
                                           * (i + 1 + beta) / (h1 + 1) / (h1 + 3))
        b_new = -(alpha * alpha - beta * beta) / h1 / (h1 + 2)
        p_next = (-a_old * p_prev + (x - b_new) * p) / a_new
        p_prev, p = p, p_next
        a_old = a_new
    return p


def grad_jacobi_p(x, alpha, beta, n):
    """d/dx P_n^{(alpha,beta)} = sqrt(n(n+alpha+beta+1)) P_{n-1}^{(alpha+1,beta+1)}."""
    x = np.asarray(x, dtype=np.float64)
    if n == 0:
        return np.zeros_like(x)
    return math.sqrt(n * (n + alpha + beta + 1)) * jacobi_p(x, alpha + 1, beta + 1, n - 1)


def jacobi_gauss(alpha, beta, n):
    """Gauss points of P_{n+1}^{(alpha,beta)}: eigenvalues of the symmetric
    tridiagonal Jacobi matrix (Golub-Welsch)."""
    if n == 0:
        return np.array([-(alpha - beta) / (alpha + beta + 2)])
    k = np.arange(n + 1, dtype=np.float64)
    h1 = 2 * k + alpha + beta
    with np.errstate(divide="ignore", invalid="ignore"):
        diag = -(alpha ** 2 - beta ** 2) / (h1 + 2) / h1
    if alpha + beta < 10 * np.finfo(float).eps:
        diag[0] = 0.0
    kk = k[1:]
    h1b = 2 * kk + alpha + beta
    off = 2.0 / (h1b) * np.sqrt(kk * (kk + alpha + beta) * (kk + alpha) * (kk + beta)
                                / (h1b - 1) / (h1b + 1))
    J = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    return np.sort(np.linalg.eigvalsh(J))


def gll_nodes(N):
    """Gauss-Lobatto-Legendre points on [-1, 1], ascending: the end points
    and the Gauss points of P_{N-1}^{(1,1)}."""
    if N == 1:
        return np.array([-1.0, 1.0])
    inner = jacobi_gauss(1.0, 1.0, N - 2)
    return np.concatenate([[-1.0], inner, [1.0]])


# ------------------------------------------------------------ Warp&Blend ---
def _warp_factor(N, x):
    """1D warp of equispaced points toward GLL points, divided by (1 - x^2):
    w(x) = sum_i (x_i^GLL - x_i^eq) l_i^eq(x) / (1 - x^2), l_i^eq the Lagrange
    polynomials of the equispaced points.  (1 - x^2) divides w exactly since
    w(+-1) = 0; the quotient is evaluated as sum_i d_i l_i(x)/((1-x)(1+x))
    with the two end factors cancelled analytically."""
    xeq = np.linspace(-1.0, 1.0, N + 1)
    xg = gll_nodes(N)
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for i in range(1, N):  # end displacements are zero
        # l_i(x) / ((x - xeq_0)(x - xeq_N)) = prod_{j != i, j != 0, N} (x - xj)/(xi - xj)
        #                                     / ((xi - xeq_0)(xi - xeq_N))
        term = np.full_like(x, (xg[i] - xeq[i]) / ((xeq[i] - xeq[0]) * (xeq[i] - xeq[N])))
        for j in range(1, N):
            if j != i:
                term = term * (x - xeq[j]) / (xeq[i] - xeq[j])
        out += term
    # (x - (-1))(x - 1) = -(1 - x^2)
    return -out


def tet_lattice(N):
    """Lattice indices (i, j, k) in node order (k slowest, i fastest)."""
    idx = []
    for k in range(N + 1):
        for j in range(N + 1 - k):
            for i in range(N + 1 - k - j):
                idx.append((i, j, k))
    return np.array(idx, dtype=np.int64)


def tet_nodes(N):
    """Warp & Blend nodes on the reference tetrahedron, (Np, 3) in (r, s, t).

    Construction (Warburton 2006): start from the equispaced lattice; for each
    face, add a tangential 2D warp (sum over the face's three edges of the 1D
    warp along that edge, blended by the product of the edge's two barycentric
    coordinates and (1 + (alpha*lambda_opp)^2)) times a volume blend that is 1
    on the face and 0 on the other faces; on the tetrahedron's edges the shift
    is the 1D warp itself.  Each edge term displaces along the edge direction,
    so the construction is carried out in reference coordinates directly."""
    lat = tet_lattice(N)
    Np = lat.shape[0]
    lam = np.empty((Np, 4))
    lam[:, 1] = lat[:, 0] / N
    lam[:, 2] = lat[:, 1] / N
    lam[:, 3] = lat[:, 2] / N
    lam[:, 0] = (N - lat.sum(axis=1)) / N
    zero = np.empty((Np, 4), dtype=bool)
    zero[:, 1:] = lat == 0
    zero[:, 0] = lat.sum(axis=1) == N
    X = lam @ REF_VERTS
    alpha = WB_ALPHA_TET[N - 1] if N <= 15 else 1.0
    shift = np.zeros((Np, 3))
    on_edge = zero.sum(axis=1) >= 2
    for f in range(4):
        d = FACE_OPP[f]
        a, b, c = FACE_VERTS[f]
        face_shift = np.zeros((Np, 3))
        for (p, q, r) in ((a, b, c), (b, c, a), (c, a, b)):
            w = (4.0 * lam[:, p] * lam[:, q] * _warp_factor(N, lam[:, q] - lam[:, p])
                 * (1.0 + (alpha * lam[:, r]) ** 2))
            face_shift += w[:, None] * (REF_VERTS[q] - REF_VERTS[p])[None, :] / 2.0
        lb, lc, ld = lam[:, a], lam[:, b], lam[:, c]
        la = lam[:, d]
        denom = (lb + 0.5 * la) * (lc + 0.5 * la) * (ld + 0.5 * la)
        blend = lb * lc * ld
        ok = denom > 1e-14
        blend[ok] = (1.0 + (alpha * la[ok]) ** 2) * blend[ok] / denom[ok]
        shift += blend[:, None] * face_shift
    # nodes on edges: the pure 1D warp along that edge (vertices: no shift)
    for e in np.nonzero(on_edge)[0]:
        nz = np.nonzero(~zero[e])[0]
        if len(nz) == 1:
            shift[e] = 0.0
            continue
        p, q = nz
        x = lam[e, q] - lam[e, p]
        w = 4.0 * lam[e, p] * lam[e, q] * _warp_factor(N, np.array([x]))[0]
        shift[e] = w * (REF_VERTS[q] - REF_VERTS[p]) / 2.0
    return X + shift


def tri_nodes(N):
    """Triangle nodes = tetrahedron nodes of the face t = -1 (k = 0), in
    (r, s) coordinates and tet node order (Section 3.2: triangle nodes match
    the tetrahedron's face nodes)."""
    lat = tet_lattice(N)
    x = tet_nodes(N)
    return x[lat[:, 2] == 0][:, :2].copy()


def line_nodes(N):
    """Line nodes = the tetrahedron's edge nodes = GLL points, ascending."""
    return gll_nodes(N)


# ---------------------------------------------------------------- bases ----
def _collapse3(r, s, t):
    with np.errstate(divide="ignore", invalid="ignore"):
        a = np.where(np.abs(s + t) > 1e-14, 2.0 * (1.0 + r) / (-s - t) - 1.0, -1.0)
        b = np.where(np.abs(t - 1.0) > 1e-14, 2.0 * (1.0 + s) / (1.0 - t) - 1.0, -1.0)
    return a, b, t


def tet_modes(N):
    return [(i, j, k) for i in range(N + 1) for j in range(N + 1 - i) for k in range(N + 1 - i - j)]


def tet_basis(x, N):
    """Orthonormal modal basis on the tetrahedron and its gradient.
    psi_ijk = 2 sqrt(2) P_i(a) P_j^{(2i+1,0)}(b) (1-b)^i P_k^{(2i+2j+2,0)}(c) (1-c)^{i+j}.
    Returns V (n, Np), Vr, Vs, Vt."""
    r, s, t = x[:, 0], x[:, 1], x[:, 2]
    a, b, c = _collapse3(r, s, t)
    modes = tet_modes(N)
    n = len(r)
    V = np.empty((n, len(modes)))
    Vr = np.empty_like(V)
    Vs = np.empty_like(V)
    Vt = np.empty_like(V)
    for m, (i, j, k) in enumerate(modes):
        fa = jacobi_p(a, 0, 0, i)
        dfa = grad_jacobi_p(a, 0, 0, i)
        gb = jacobi_p(b, 2 * i + 1, 0, j)
        dgb = grad_jacobi_p(b, 2 * i + 1, 0, j)
        hc = jacobi_p(c, 2 * i + 2 * j + 2, 0, k)
        dhc = grad_jacobi_p(c, 2 * i + 2 * j + 2, 0, k)
        C = 2.0 * math.sqrt(2.0)
        V[:, m] = C * fa * gb * (1 - b) ** i * hc * (1 - c) ** (i + j)
        # d/dr: fa' * 4/((1-b)(1-c)) * gb (1-b)^i * hc (1-c)^(i+j)
        dr = dfa * gb * hc
        if i > 0:
            dr = dr * (1 - b) ** (i - 1)
        if i + j > 0:
            dr = dr * (1 - c) ** (i + j - 1)
        dr = 4.0 * dr if (i > 0) else np.zeros_like(r)
        # d/ds = fa'*2(1+a)/((1-b)(1-c)) fb fc + fa fb' 2/(1-c) fc
        ds = dr * (1 + a) / 2.0
        fb_prime = dgb * (1 - b) ** i
        if i > 0:
            fb_prime = fb_prime - i * gb * (1 - b) ** (i - 1)
        tmp = fa * fb_prime * hc
        if i + j > 0:
            tmp = tmp * (1 - c) ** (i + j - 1)
        ds = ds + 2.0 * tmp
        # d/dt = fa'*2(1+a)/((1-b)(1-c)) fb fc + fa fb' (1+b)/(1-c) fc + fa fb fc'
        dt = dr * (1 + a) / 2.0 + tmp * (1 + b)
        fc_prime = dhc * (1 - c) ** (i + j)
        if i + j > 0:
            fc_prime = fc_prime - (i + j) * hc * (1 - c) ** (i + j - 1)
        dt = dt + fa * gb * (1 - b) ** i * fc_prime
        Vr[:, m] = C * dr
        Vs[:, m] = C * ds
        Vt[:, m] = C * dt
    return V, Vr, Vs, Vt


def tri_modes(N):
    return [(i, j) for i in range(N + 1) for j in range(N + 1 - i)]


def tri_basis(x, N):
    """Orthonormal modal basis on the triangle and its gradient.
    psi_ij = sqrt(2) P_i(a) P_j^{(2i+1,0)}(b) (1-b)^i, a = 2(1+r)/(1-s) - 1, b = s."""
    r, s = x[:, 0], x[:, 1]
    with np.errstate(divide="ignore", invalid="ignore"):
        a = np.where(np.abs(s - 1.0) > 1e-14, 2.0 * (1.0 + r) / (1.0 - s) - 1.0, -1.0)
    b = s
    modes = tri_modes(N)
    V = np.empty((len(r), len(modes)))
    Vr = np.empty_like(V)
    Vs = np.empty_like(V)
    C = math.sqrt(2.0)
    for m, (i, j) in enumerate(modes):
        fa = jacobi_p(a, 0, 0, i)
        dfa = grad_jacobi_p(a, 0, 0, i)
        gb = jacobi_p(b, 2 * i + 1, 0, j)
        dgb = grad_jacobi_p(b, 2 * i + 1, 0, j)
        V[:, m] = C * fa * gb * (1 - b) ** i
        # d/dr = fa' 2/(1-b) gb (1-b)^i
        dr = dfa * gb
        if i > 0:
            dr = 2.0 * dr * (1 - b) ** (i - 1)
        else:
            dr = np.zeros_like(r)
        # d/ds = fa' (1+a)/(1-b) gb (1-b)^i + fa d/db[gb (1-b)^i]
        ds = dr * (1 + a) / 2.0
        fb_prime = dgb * (1 - b) ** i
        if i > 0:
            fb_prime = fb_prime - i * gb * (1 - b) ** (i - 1)
        ds = ds + fa * fb_prime
        Vr[:, m] = C * dr
        Vs[:, m] = C * ds
    return V, Vr, Vs


def line_basis(x, N):
    V = np.stack([jacobi_p(x, 0, 0, i) for i in range(N + 1)], axis=1)
    Vr = np.stack([grad_jacobi_p(x, 0, 0, i) for i in range(N + 1)], axis=1)
    return V, Vr


# ------------------------------------------------------------ operators ----
class Tet:
    """Reference tetrahedron of degree N: nodes, Vandermonde, Dr/Ds/Dt, mass,
    face masks and LIFT (Section 3.2; the lifting matrix maps face values to
    the volume, M^-1 E)."""

    def __init__(self, N):
        self.N = N
        self.Np = (N + 1) * (N + 2) * (N + 3) // 6
        self.Nfp = (N + 1) * (N + 2) // 2
        self.lat = tet_lattice(N)
        self.x = tet_nodes(N)
        V, Vr, Vs, Vt = tet_basis(self.x, N)
        self.V = V
        Vi = np.linalg.inv(V)
        self.Dr = Vr @ Vi
        self.Ds = Vs @ Vi
        self.Dt = Vt @ Vi
        self.M = np.linalg.inv(V @ V.T)
        i, j, k = self.lat[:, 0], self.lat[:, 1], self.lat[:, 2]
        masks = [k == 0, j == 0, i + j + k == N, i == 0]
        self.Fmask = np.stack([np.nonzero(m)[0] for m in masks])          # (4, Nfp)
        # face-local 2D coordinates of each face's nodes (reference triangle
        # (-1,-1),(1,-1),(-1,1) in the face's two free coordinates)
        facecoords = [(0, 1), (0, 2), (1, 2), (1, 2)]
        E = np.zeros((self.Np, 4 * self.Nfp))
        for f in range(4):
            xf = self.x[self.Fmask[f]][:, facecoords[f]]
            V2, _, _ = tri_basis(xf, N)
            Mf = np.linalg.inv(V2 @ V2.T)
            E[self.Fmask[f], f * self.Nfp:(f + 1) * self.Nfp] = Mf
        self.LIFT = V @ (V.T @ E)


class Tri:
    """Reference triangle of degree N with nodes taken from the tet face t=-1."""

    def __init__(self, N):
        self.N = N
        self.Np = (N + 1) * (N + 2) // 2
        self.Nfp = N + 1
        self.x = tri_nodes(N)
        lat = tet_lattice(N)
        lat = lat[lat[:, 2] == 0]
        self.lat = lat[:, :2]
        V, Vr, Vs = tri_basis(self.x, N)
        self.V = V
        Vi = np.linalg.inv(V)
        self.Dr = Vr @ Vi
        self.Ds = Vs @ Vi
        self.M = np.linalg.inv(V @ V.T)
        i, j = self.lat[:, 0], self.lat[:, 1]
        masks = [j == 0, i + j == N, i == 0]
        self.Fmask = np.stack([np.nonzero(m)[0] for m in masks])          # (3, Nfp)
        edgecoord = [0, 1, 1]   # r along edge 0, s along edges 1 and 2
        E = np.zeros((self.Np, 3 * self.Nfp))
        for f in range(3):
            xf = self.x[self.Fmask[f], edgecoord[f]]
            V1, _ = line_basis(xf, N)
            Mf = np.linalg.inv(V1 @ V1.T)
            E[self.Fmask[f], f * self.Nfp:(f + 1) * self.Nfp] = Mf
        self.LIFT = V @ (V.T @ E)


class Line:
    """Reference line of degree N (GLL nodes)."""

    def __init__(self, N):
        self.N = N
        self.Np = N + 1
        self.x = line_nodes(N)
        V, Vr = line_basis(self.x, N)
        self.V = V
        self.Dr = Vr @ np.linalg.inv(V)
        self.M = np.linalg.inv(V @ V.T)
        E = np.zeros((self.Np, 2))
        E[0, 0] = 1.0
        E[-1, 1] = 1.0
        self.LIFT = V @ (V.T @ E)
