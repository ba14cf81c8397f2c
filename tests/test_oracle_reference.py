"""Pins of the oracle's reference elements (nodal DG, Section 3.2) against
library routines, closed forms and exact identities."""
import itertools

import numpy as np
import pytest
from scipy.special import roots_jacobi, eval_legendre

from oracle.reference import (Tet, Tri, Line, jacobi_p, gll_nodes, tet_nodes, tet_lattice,
                              tri_nodes)


@pytest.mark.parametrize("alpha,beta", [(0, 0), (1, 0), (3, 0), (1, 1), (6, 0)])
def test_jacobi_orthonormal(alpha, beta):
    # Gauss-Jacobi quadrature from scipy (independent of the oracle)
    x, wq = roots_jacobi(20, alpha, beta)
    P = np.stack([jacobi_p(x, alpha, beta, n) for n in range(8)])
    G = (P * wq) @ P.T
    assert np.allclose(G, np.eye(8), atol=1e-13)


@pytest.mark.parametrize("N", range(1, 9))
def test_gll_nodes(N):
    # GLL points: +-1 and the roots of P_N'(x) (Legendre derivative via numpy)
    c = np.zeros(N + 1)
    c[N] = 1.0
    inner = np.sort(np.polynomial.legendre.Legendre(c).deriv().roots().real)
    ref = np.concatenate([[-1.0], inner, [1.0]])
    assert np.allclose(gll_nodes(N), ref, atol=1e-14)


def test_equispaced_for_low_degree():
    # for N <= 2 the GLL points are equispaced, so the warp vanishes
    for N in (1, 2):
        lat = tet_lattice(N)
        eq = -1.0 + 2.0 * lat / N
        assert np.allclose(tet_nodes(N), eq, atol=1e-15)


def _bary(x):
    r, s, t = x[:, 0], x[:, 1], x[:, 2]
    return np.stack([-(1 + r + s + t) / 2, (1 + r) / 2, (1 + s) / 2, (1 + t) / 2], axis=1)


@pytest.mark.parametrize("N", range(1, 8))
def test_tet_nodes_symmetric_and_gll_edges(N):
    x = tet_nodes(N)
    lam = _bary(x)
    assert np.all(lam > -1e-14)
    key = lambda L: np.round(L, 10)
    base = set(map(tuple, key(lam)))
    for perm in itertools.permutations(range(4)):
        assert set(map(tuple, key(lam[:, perm]))) == base
    # nodes on the edge v0-v1 (s = t = -1) are the GLL points
    on = (np.abs(lam[:, 2]) < 1e-14) & (np.abs(lam[:, 3]) < 1e-14)
    assert np.allclose(np.sort(x[on, 0]), gll_nodes(N), atol=1e-14)


@pytest.mark.parametrize("N", range(1, 7))
def test_tet_operators_exact(N):
    T = Tet(N)
    r, s, t = T.x[:, 0], T.x[:, 1], T.x[:, 2]
    for a in range(N + 1):
        for b in range(N + 1 - a):
            for c in range(N + 1 - a - b):
                f = r ** a * s ** b * t ** c
                fr = a * r ** max(a - 1, 0) * s ** b * t ** c
                fs = b * r ** a * s ** max(b - 1, 0) * t ** c
                ft = c * r ** a * s ** b * t ** max(c - 1, 0)
                assert np.allclose(T.Dr @ f, fr, atol=1e-11)
                assert np.allclose(T.Ds @ f, fs, atol=1e-11)
                assert np.allclose(T.Dt @ f, ft, atol=1e-11)
    # mass matrix integrates 1 to the reference volume 4/3
    assert abs(T.M.sum() - 4.0 / 3.0) < 1e-13


@pytest.mark.parametrize("N", range(1, 7))
def test_divergence_theorem_tet(N):
    """int_T d f/dr = sum over faces of f n_r dA, with the lifting matrix
    supplying the face integrals (1^T M LIFT_f g = int_face g)."""
    T = Tet(N)
    rng = np.random.default_rng(N)
    f = rng.standard_normal(T.Np)
    ML = T.M @ T.LIFT
    face_int = lambda k: np.ones(T.Np) @ ML[:, k * T.Nfp:(k + 1) * T.Nfp] @ f[T.Fmask[k]]
    # area vectors n dA in face parameters: face0 (0,0,-1), face1 (0,-1,0),
    # face2 (1,1,1), face3 (-1,0,0)
    lhs = [np.ones(T.Np) @ T.M @ D @ f for D in (T.Dr, T.Ds, T.Dt)]
    rhs = [face_int(2) - face_int(3), face_int(2) - face_int(1), face_int(2) - face_int(0)]
    assert np.allclose(lhs, rhs, atol=1e-12)


@pytest.mark.parametrize("N", range(1, 7))
def test_tri_and_line_from_tet(N):
    T, Tr, L = Tet(N), Tri(N), Line(N)
    # triangle nodes are the tet face-0 nodes; line nodes its edge nodes
    assert np.allclose(Tr.x, T.x[T.Fmask[0]][:, :2], atol=0)
    assert np.allclose(L.x, gll_nodes(N))
    assert abs(Tr.M.sum() - 2.0) < 1e-13 and abs(L.M.sum() - 2.0) < 1e-13
    r, s = Tr.x[:, 0], Tr.x[:, 1]
    for a in range(N + 1):
        for b in range(N + 1 - a):
            f = r ** a * s ** b
            assert np.allclose(Tr.Dr @ f, a * r ** max(a - 1, 0) * s ** b, atol=1e-11)
            assert np.allclose(Tr.Ds @ f, b * r ** a * s ** max(b - 1, 0), atol=1e-11)
    # 2D divergence theorem with the lifting matrix (edge measures in r, s, s)
    g = np.random.default_rng(1).standard_normal(Tr.Np)
    ML = Tr.M @ Tr.LIFT
    e_int = lambda k: np.ones(Tr.Np) @ ML[:, k * Tr.Nfp:(k + 1) * Tr.Nfp] @ g[Tr.Fmask[k]]
    assert np.isclose(np.ones(Tr.Np) @ Tr.M @ Tr.Dr @ g, e_int(1) - e_int(2), atol=1e-12)
    assert np.isclose(np.ones(Tr.Np) @ Tr.M @ Tr.Ds @ g, e_int(1) - e_int(0), atol=1e-12)
    x = L.x
    assert np.allclose(L.Dr @ x ** N, N * x ** (N - 1), atol=1e-11)
    # the tri reference nodes are invariant under the triangle's symmetries
    lam = np.stack([-(r + s) / 2, (1 + r) / 2, (1 + s) / 2], axis=1)
    base = set(map(tuple, np.round(lam, 10)))
    for perm in itertools.permutations(range(3)):
        assert set(map(tuple, np.round(lam[:, perm], 10))) == base


def test_legendre_basis_line():
    # line basis = normalised Legendre polynomials
    x = np.linspace(-1, 1, 7)
    for n in range(6):
        assert np.allclose(jacobi_p(x, 0, 0, n), eval_legendre(n, x) * np.sqrt((2 * n + 1) / 2))
