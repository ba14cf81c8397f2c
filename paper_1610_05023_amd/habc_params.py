"""HABC coefficients other than the Pade ones (Section 2.1).

The library takes any positive coefficients gamma_1..gamma_P in the
rational form the paper uses,
    f(X) = 1 + (2/M) sum_n gamma_n (1 - (1 + gamma_n)/(1 + gamma_n + X)),
    M = 2P + 1,
which replaces sqrt(1 + X) in the exact boundary operator; a plane wave
meeting the boundary at angle theta (X = -sin^2 theta) is reflected with
R(theta) = (cos theta - f)/(cos theta + f).  The Pade choice gamma_n =
tan^2(n pi/M) puts every zero of R at normal incidence
(R = -tan^(2M)(theta/2)).  The paper notes that other parameters and other
rational approximations trade accuracy between incidence angles.  This
module gives one such choice: coefficients for which R vanishes at P given
angles, spread over the range of incidences.
"""
from __future__ import annotations

import math

import numpy as np


def rational_f(X, gamma):
    """f(X) of the coefficients gamma (any P)."""
    g = np.asarray(gamma, dtype=np.float64)
    M = 2 * len(g) + 1
    X = np.asarray(X, dtype=np.float64)[..., None]
    return 1.0 + (2.0 / M) * np.sum(g * X / (1.0 + g + X), axis=-1)


def reflection(theta, gamma):
    """Plane-wave reflection coefficient R(theta) of the condition."""
    f = rational_f(-np.sin(theta) ** 2, gamma)
    c = np.cos(theta)
    return (c - f) / (c + f)


def angle_matched_gamma(angles):
    """Coefficients gamma (one per angle, so P = len(angles)) whose
    condition is exact (R = 0) for plane waves at the given incidence angles
    (radians, distinct, in (0, pi/2)): the P equations f(-sin^2 t_k) =
    cos t_k solved by least squares in log(gamma) (so gamma > 0), from the
    Pade coefficients.  With the weights 2/M of the paper's form, R(pi/2)
    = -1 whatever the coefficients, so the zeros can move only over part of
    the range (for P = 3, up to about 60 degrees)."""
    from scipy.optimize import least_squares
    t = np.sort(np.asarray(angles, dtype=np.float64))
    P = len(t)
    M = 2 * P + 1
    X = -np.sin(t) ** 2
    target = np.cos(t)
    y0 = np.log(np.array([math.tan(n * math.pi / M) ** 2 for n in range(1, P + 1)]))
    sol = least_squares(lambda y: rational_f(X, np.exp(y)) - target, y0, xtol=1e-15, ftol=1e-15,
                        gtol=1e-15, max_nfev=2000)
    g = np.sort(np.exp(sol.x))
    if np.abs(rational_f(X, g) - target).max() > 1e-9:
        raise ValueError("no positive coefficients match these angles")
    return g
