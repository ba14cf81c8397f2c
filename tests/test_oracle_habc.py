"""Pins of the HABC algebra (Sections 2.1-2.3 and 3.1)."""
import math

import numpy as np
import pytest

from oracle.habc import (pade_gamma, pade_f1, pade_f2, reflection_coefficient, solve_edge,
                         solve_corner, edge_matrix, C2)


def test_gamma_values():
    # tan^2(n pi / M): P = 1 gives tan^2(pi/3) = 3 exactly
    assert abs(pade_gamma(1)[0] - 3.0) < 1e-14
    # trigonometric identities for M = 2P+1: sum_n tan^2(n pi/M) = P M and
    # prod_n tan(n pi/M) = sqrt(M)
    for P in (2, 3, 6, 12):
        g = pade_gamma(P)
        assert abs(g.sum() - P * (2 * P + 1)) < 1e-11 * P * P
        assert abs(np.prod(g) - (2 * P + 1)) < 1e-10 * (2 * P + 1)


@pytest.mark.parametrize("P", [1, 2, 3, 6, 12])
def test_pade_forms_agree(P):
    X = np.linspace(-0.9, 5.0, 41)
    assert np.allclose(pade_f1(X, P), pade_f2(X, P), atol=1e-14, rtol=1e-14)


@pytest.mark.parametrize("P", [1, 2, 3])
def test_pade_order(P):
    """f_P - sqrt(1+X) = O(X^(2P+1)): the ratio error(X)/X^(2P+1) is bounded
    and nonzero as X -> 0 (the order of the (2P+1)-th order Pade approximant)."""
    Xs = np.array([0.2, 0.1, 0.05])
    err = np.abs(pade_f2(Xs, P) - np.sqrt(1.0 + Xs))
    slopes = np.log(err[:-1] / err[1:]) / np.log(2.0)
    # the observed order tends to 2P+1 from below as X -> 0
    assert abs(slopes[-1] - (2 * P + 1)) < 0.3 and slopes[-1] > slopes[0]


def test_reflection_normal_incidence_and_monotone():
    # exact at normal incidence; error decreases with the order at 45 degrees
    for P in (1, 3, 6):
        assert abs(reflection_coefficient(0.0, P)) < 1e-15
    r = [abs(reflection_coefficient(np.pi / 4, P)) for P in (0, 1, 3, 6)]
    assert all(a > b for a, b in zip(r, r[1:]))


def _char(p, zu):
    return 0.5 * (p + zu), 0.5 * (p - zu)


def _gammas(P, kind):
    """Pade coefficients, or coefficients other than Pade's (positive,
    spread: the edge and corner algebra holds for any)."""
    if kind == "pade":
        return pade_gamma(P)
    return np.sort(np.random.default_rng(40 + P).uniform(0.05, 30.0, P))


@pytest.mark.parametrize("kind", ["pade", "other"])
@pytest.mark.parametrize("P", [1, 3, 6])
def test_edge_system_satisfies_first_order_conditions(P, kind):
    """The solution of the characteristic edge equations satisfies the
    first-order edge conditions of Section 2.3,
      p_i - Z v_i = (2/M) sum_j g_j (p_ij - p_i) (face A fields at the edge),
      p_j - Z u_j = (2/M) sum_i g_i (p_ij - p_j) (face B fields),
    with p_i = r+ + r-, Z v_i = r+ - r-, and p_ij rebuilt from p*_ij."""
    g = _gammas(P, kind)
    M = 2 * P + 1
    rng = np.random.default_rng(P)
    n = 5
    pstar = rng.standard_normal((P, P, n))
    rpA, rpB = rng.standard_normal((P, n)), rng.standard_normal((P, n))
    rmA, rmB = solve_edge(g, pstar, rpA, rpB)
    SA, SB = rpA + rmA, rpB + rmB
    pij = pstar + np.array([[C2(g, j, i) for j in range(P)] for i in range(P)])[:, :, None] * SA[:, None, :] \
        + np.array([[C2(g, i, j) for j in range(P)] for i in range(P)])[:, :, None] * SB[None, :, :]
    # the 1D relation of the edge: (1+gi+gj) p_ij = (1+gj) p_i + (1+gi) p_j on the
    # boundary values is what the rebuilt p_ij encodes when p* = 0
    lhsA = SA - (rpA - rmA)
    rhsA = (2.0 / M) * np.einsum("j,ijn->in", g, pij - SA[:, None, :])
    lhsB = SB - (rpB - rmB)
    rhsB = (2.0 / M) * np.einsum("i,ijn->jn", g, pij - SB[None, :, :])
    assert np.allclose(lhsA, rhsA, atol=1e-13)
    assert np.allclose(lhsB, rhsB, atol=1e-13)


@pytest.mark.parametrize("P", [1, 2, 3, 6])
def test_edge_inverse_block_structure(P):
    """The edge matrix and its inverse consist of two distinct P x P blocks
    [[X, Y], [Y, X]] (Section 3.1)."""
    L = edge_matrix(pade_gamma(P))
    Li = np.linalg.inv(L)
    for A in (L, Li):
        assert np.allclose(A[:P, :P], A[P:, P:], atol=1e-14)
        assert np.allclose(A[:P, P:], A[P:, :P], atol=1e-14)


@pytest.mark.parametrize("kind", ["pade", "other"])
@pytest.mark.parametrize("P", [1, 2, 3])
def test_corner_system_satisfies_first_order_conditions(P, kind):
    """Corner: p_0jk - Z u_0jk = (2/M) sum_i g_i (p_ijk - p_0jk) with the 0D
    relation (1+gi+gj+gk) p_ijk = (1+gi) p_0jk + (1+gj) p_i0k + (1+gk) p_ij0
    (Section 2.2), and likewise for the two other edges."""
    g = _gammas(P, kind)
    M = 2 * P + 1
    rng = np.random.default_rng(10 + P)
    n = 3
    rX, rY, rZ = (rng.standard_normal((P * P, n)) for _ in range(3))
    mX, mY, mZ = solve_corner(g, rX, rY, rZ)
    SX, SY, SZ = ((a + b).reshape(P, P, n) for a, b in ((rX, mX), (rY, mY), (rZ, mZ)))
    ZX, ZY, ZZ = ((a - b).reshape(P, P, n) for a, b in ((rX, mX), (rY, mY), (rZ, mZ)))
    pijk = np.empty((P, P, P, n))
    for i in range(P):
        for j in range(P):
            for k in range(P):
                D = 1 + g[i] + g[j] + g[k]
                pijk[i, j, k] = ((1 + g[i]) * SX[j, k] + (1 + g[j]) * SY[i, k]
                                 + (1 + g[k]) * SZ[i, j]) / D
    resX = SX - ZX - (2.0 / M) * np.einsum("i,ijkn->jkn", g, pijk - SX[None])
    resY = SY - ZY - (2.0 / M) * np.einsum("j,ijkn->ikn", g, pijk - SY[:, None])
    resZ = SZ - ZZ - (2.0 / M) * np.einsum("k,ijkn->ijn", g, pijk - SZ[:, :, None])
    for r in (resX, resY, resZ):
        assert np.abs(r).max() < 1e-12


def test_face_rule_equals_first_order_condition():
    """r- = (1/M) sum g_i p*_i with p*_i = p_i - (r+ + r-) is the face
    condition p - Z u = (2/M) sum g_i (p_i - p) of Section 2.3."""
    P = 4
    g = pade_gamma(P)
    M = 2 * P + 1
    rng = np.random.default_rng(3)
    pstar, rp = rng.standard_normal(P), rng.standard_normal()
    rm = np.dot(g, pstar) / M
    p, zu = rp + rm, rp - rm
    pi = pstar + p
    assert abs((p - zu) - (2.0 / M) * np.dot(g, pi - p)) < 1e-14


def test_seam_unknown_counts():
    """The unknown count sum_levels K N_sets N_fields Np reproduces the
    integers of the SEAM performance table (Section 4.2)."""
    from workloads import n_unknowns
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "seam_unknowns.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    for P, K_tet, K_tri, K_lin, expected in ((int(a), int(b), int(c), int(d), int(e))
                                             for a, b, c, d, e in rows):
        assert n_unknowns(K_tet, K_tri, K_lin, 3, P) == expected


def test_angle_matched_coefficients_zero_the_reflection():
    """Coefficients other than Pade's (Section 2.1's remark on other
    parameters): those making the condition exact at 20, 38 and 52 degrees
    zero the plane-wave reflection coefficient there, and over 0-55 degrees
    (the incidences of a centred source on a cube's faces) their largest
    reflection is below the Pade condition's of the same order."""
    from paper_1610_05023_amd.habc_params import angle_matched_gamma
    ang = np.radians([20.0, 38.0, 52.0])
    g = angle_matched_gamma(ang)
    assert np.all(g > 0) and len(g) == 3
    assert np.abs(reflection_coefficient(ang, 3, g)).max() < 1e-12
    th = np.radians(np.linspace(0.0, 55.0, 111))
    ours = np.abs(reflection_coefficient(th, 3, g)).max()
    pade = np.abs(reflection_coefficient(th, 3)).max()
    assert ours < 0.5 * pade, (ours, pade)
