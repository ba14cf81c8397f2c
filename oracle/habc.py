"""Pade-type HABC coefficients and the edge/corner compatibility equations
(oracle, FP64; test infrastructure, never imported by the library).

Section 2.1: f_P(X) approximates sqrt(1+X) with M = 2P+1 and coefficients
gamma_n = tan^2(n pi / M) (the paper's c_n), in the two equivalent forms of
the Pade approximation.  Section 3.1: the incoming characteristics at edges
(a 2P-equation system) and corners (a 3P^2-equation system).  The oracle
assembles these systems from the scalar equations of the procedure and solves
them by LU for every node; it never forms an inverse.

Reading (garbled in the paper's first-order corner conditions): the corner
terms carry (C_ijk - 1), as in the procedure's corner conditions, which is
what the 0D relation gives when substituted into the corner boundary
conditions.
"""
from __future__ import annotations

import math

import numpy as np


def pade_gamma(P):
    """gamma_n = tan^2(n pi / M), n = 1..P, M = 2P+1 (Section 2.1)."""
    M = 2 * P + 1
    return np.array([math.tan(n * math.pi / M) ** 2 for n in range(1, P + 1)])


def pade_ab(P):
    """a_n = sin^2(n pi/M), b_n = cos^2(n pi/M) of the first Pade form."""
    M = 2 * P + 1
    a = np.array([math.sin(n * math.pi / M) ** 2 for n in range(1, P + 1)])
    b = np.array([math.cos(n * math.pi / M) ** 2 for n in range(1, P + 1)])
    return a, b


def pade_f1(X, P):
    """f_P(X) = 1 + (2/M) sum_n a_n X / (1 + b_n X)."""
    M = 2 * P + 1
    a, b = pade_ab(P)
    X = np.asarray(X, dtype=np.float64)
    return 1.0 + (2.0 / M) * sum(a[n] * X / (1.0 + b[n] * X) for n in range(P))


def pade_f2(X, P, gamma=None):
    """f_P(X) = 1 + (2/M) sum_n gamma_n (1 - (1+gamma_n)/(1+gamma_n+X))."""
    M = 2 * P + 1
    g = pade_gamma(P) if gamma is None else gamma
    X = np.asarray(X, dtype=np.float64)
    return 1.0 + (2.0 / M) * sum(g[n] * (1.0 - (1.0 + g[n]) / (1.0 + g[n] + X))
                                 for n in range(P))


def reflection_coefficient(theta, P, gamma=None):
    """Plane-wave reflection of the planar condition (Section 2.1): for a wave
    hitting x = L at angle theta the symbol of the boundary operator gives
    R = (cos(theta) - f_P(-sin^2 theta)) / (cos(theta) + f_P(-sin^2 theta)),
    with the Pade coefficients or the given ones in the second form."""
    f = pade_f2(-np.sin(theta) ** 2, P, gamma)
    return (np.cos(theta) - f) / (np.cos(theta) + f)


def C2(gamma, a, b):
    """C_ab = (1 + gamma_a) / (1 + gamma_a + gamma_b) (edge temporaries)."""
    return (1.0 + gamma[a]) / (1.0 + gamma[a] + gamma[b])


def solve_edge(gamma, pstar, rpA, rpB):
    """Incoming characteristics at edge nodes, Section 3.1 (edge conditions of
    the procedure), for an edge A n B with face-A sets i and face-B sets j:

      rA_i = (1/M) sum_j g_j [p*_ij + (C_ji - 1) SA_i + C_ij SB_j]
      rB_j = (1/M) sum_i g_i [p*_ij + C_ji SA_i + (C_ij - 1) SB_j]

    with S = r- + r+ on both sides.  pstar (P, P, n), rpA (P, n), rpB (P, n);
    returns (rmA (P, n), rmB (P, n)).  The 2P x 2P matrix is assembled
    equation by equation and solved by LU for all n nodes."""
    P = len(gamma)
    M = 2 * P + 1
    n = pstar.shape[2]
    L = np.zeros((2 * P, 2 * P))
    R = np.zeros((2 * P, n))
    for i in range(P):                     # equation for rA_i (row i)
        L[i, i] += 1.0
        for j in range(P):
            g = gamma[j] / M
            R[i] += g * pstar[i, j]
            # (C_ji - 1) (rA_i + rpA_i)
            cA = C2(gamma, j, i) - 1.0
            L[i, i] -= g * cA
            R[i] += g * cA * rpA[i]
            # C_ij (rB_j + rpB_j)
            cB = C2(gamma, i, j)
            L[i, P + j] -= g * cB
            R[i] += g * cB * rpB[j]
    for j in range(P):                     # equation for rB_j (row P + j)
        L[P + j, P + j] += 1.0
        for i in range(P):
            g = gamma[i] / M
            R[P + j] += g * pstar[i, j]
            cA = C2(gamma, j, i)
            L[P + j, i] -= g * cA
            R[P + j] += g * cA * rpA[i]
            cB = C2(gamma, i, j) - 1.0
            L[P + j, P + j] -= g * cB
            R[P + j] += g * cB * rpB[j]
    x = np.linalg.solve(L, R)
    return x[:P], x[P:]


def edge_matrix(gamma):
    """The 2P x 2P matrix of ``solve_edge`` (rows A_i then B_j)."""
    P = len(gamma)
    M = 2 * P + 1
    L = np.eye(2 * P)
    for i in range(P):
        for j in range(P):
            L[i, i] -= gamma[j] / M * (C2(gamma, j, i) - 1.0)
            L[i, P + j] -= gamma[j] / M * C2(gamma, i, j)
            L[P + j, i] -= gamma[i] / M * C2(gamma, j, i)
            L[P + j, P + j] -= gamma[i] / M * (C2(gamma, i, j) - 1.0)
    return L


def solve_corner(gamma, rpX, rpY, rpZ):
    """Incoming characteristics of the three edge fields at a corner
    f n g n h, Section 3.1 (corner conditions of the procedure):

      rX_jk = (1/M) sum_i g_i [(C_ijk - 1) SX_jk + C_jki SY_ik + C_kij SZ_ij]
      rY_ik = (1/M) sum_j g_j [C_ijk SX_jk + (C_jki - 1) SY_ik + C_kij SZ_ij]
      rZ_ij = (1/M) sum_k g_k [C_ijk SX_jk + C_jki SY_ik + (C_kij - 1) SZ_ij]

    X = edge g n h (sets (j,k)), Y = edge f n h ((i,k)), Z = edge f n g ((i,j));
    D = 1 + g_i + g_j + g_k, C_ijk = (1+g_i)/D, C_jki = (1+g_j)/D,
    C_kij = (1+g_k)/D; S = r- + r+.  Inputs (P*P, n) with set index a*P + b;
    returns (rmX, rmY, rmZ)."""
    P = len(gamma)
    M = 2 * P + 1
    n = rpX.shape[1]
    PP = P * P
    L = np.eye(3 * PP)
    R = np.zeros((3 * PP, n))
    X = lambda j, k: 0 * PP + j * P + k
    Y = lambda i, k: 1 * PP + i * P + k
    Z = lambda i, j: 2 * PP + i * P + j
    rp = np.concatenate([rpX, rpY, rpZ], axis=0)

    def add(row, col, coef):
        L[row, col] -= coef
        R[row] += coef * rp[col]

    for i in range(P):
        for j in range(P):
            for k in range(P):
                D = 1.0 + gamma[i] + gamma[j] + gamma[k]
                Ci, Cj, Ck = (1 + gamma[i]) / D, (1 + gamma[j]) / D, (1 + gamma[k]) / D
                gi, gj, gk = gamma[i] / M, gamma[j] / M, gamma[k] / M
                # row X_jk, summed over i
                add(X(j, k), X(j, k), gi * (Ci - 1.0))
                add(X(j, k), Y(i, k), gi * Cj)
                add(X(j, k), Z(i, j), gi * Ck)
                # row Y_ik, summed over j
                add(Y(i, k), X(j, k), gj * Ci)
                add(Y(i, k), Y(i, k), gj * (Cj - 1.0))
                add(Y(i, k), Z(i, j), gj * Ck)
                # row Z_ij, summed over k
                add(Z(i, j), X(j, k), gk * Ci)
                add(Z(i, j), Y(i, k), gk * Cj)
                add(Z(i, j), Z(i, j), gk * (Ck - 1.0))
    x = np.linalg.solve(L, R)
    return x[:PP], x[PP:2 * PP], x[2 * PP:]
