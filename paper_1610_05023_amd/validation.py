"""Evaluation of the validation benchmark of Section 4.1 (host side, FP64).

A Ricker point source in free space: the pressure equation carries
delta(x - x_s) S(t) with S the integral of the Ricker wavelet s, so the
pressure obeys p_tt - c^2 lap p = delta(x - x_s) s(t) and the free-space
solution is the retarded potential (Section 4.1's reference solution)
  p(t, x) = s(t - r/c) / (4 pi c^2 r),
  u(t, x) = (x - x_s) / (4 pi rho c^2 r^2) (S(t - r/c)/r + s(t - r/c)/c),
r = |x - x_s| (the paper prints c = 1).  With p = 0 on a plane z = z_top
(the free-surface variant) the method of images adds the same field of a
source mirrored in that plane with the opposite sign.

The error of a numerical state is Section 4.1's relative energy norm,
  Error(t)^2 = int_Omega (p_ref - p)^2/(2 rho c^2) + rho |u_ref - u|^2/2 dx / E_src,
with E_src the energy the source puts into the domain (from a run with
p = 0 on the whole boundary, once the wavelet has been emitted), both
integrals by a quadrature exact for polynomials of degree 7 on every
tetrahedron.  The numerical fields come from the library (read_fields):
this module only measures them.
"""
from __future__ import annotations

import math

import numpy as np


# ---------------------------------------------------------------- source ----
def ricker(t, f0, t0):
    """Ricker wavelet s(t) = (1 - 2 a^2) exp(-a^2), a = pi f0 (t - t0)."""
    a2 = (math.pi * f0 * (np.asarray(t) - t0)) ** 2
    return (1.0 - 2.0 * a2) * np.exp(-a2)


def ricker_integral(t, f0, t0):
    """S(t) = (t - t0) exp(-(pi f0 (t - t0))^2), with S' = s."""
    d = np.asarray(t) - t0
    return d * np.exp(-(math.pi * f0 * d) ** 2)


def free_space(x, t, xs, f0, t0, rho=1.0, c=1.0):
    """Pressure and velocity of the point source at x (..., 3), time t."""
    d = np.asarray(x, dtype=np.float64) - np.asarray(xs, dtype=np.float64)
    r = np.sqrt(np.sum(d * d, axis=-1))
    tau = t - r / c
    s, S = ricker(tau, f0, t0), ricker_integral(tau, f0, t0)
    p = s / (4.0 * math.pi * c * c * r)
    coef = (S / r + s / c) / (4.0 * math.pi * rho * c * c * r * r)
    return p, d * coef[..., None]


def reference(x, t, xs, f0, t0, rho=1.0, c=1.0, z_top=None):
    """Free-space solution, or with p = 0 on z = z_top by the method of
    images (a source of opposite sign at the mirror image of xs)."""
    p, u = free_space(x, t, xs, f0, t0, rho, c)
    if z_top is not None:
        xi = np.array(xs, dtype=np.float64)
        xi[2] = 2.0 * z_top - xi[2]
        pi_, ui = free_space(x, t, xi, f0, t0, rho, c)
        p, u = p - pi_, u - ui
    return p, u


# ------------------------------------------------------------ quadrature ----
def simplex_rule(n=4):
    """Conical-product (Stroud) rule on the unit simplex {l >= 0, l1+l2+l3
    <= 1} with n Gauss-Jacobi points per direction, exact for total degree
    2n - 1 (7 for n = 4).  Returns (lam (nq, 3), w (nq,)), sum w = 1/6."""
    from scipy.special import roots_jacobi
    # l1 = a, l2 = (1 - a) b, l3 = (1 - a)(1 - b) g; Jacobian (1 - a)^2 (1 - b)
    xa, wa = roots_jacobi(n, 2.0, 0.0)
    xb, wb = roots_jacobi(n, 1.0, 0.0)
    xg, wg = roots_jacobi(n, 0.0, 0.0)
    a, b, g = (xa + 1) / 2, (xb + 1) / 2, (xg + 1) / 2
    wa, wb, wg = wa / 8.0, wb / 4.0, wg / 2.0
    A, B, G = np.meshgrid(a, b, g, indexing="ij")
    W = wa[:, None, None] * wb[None, :, None] * wg[None, None, :]
    lam = np.stack([A, (1 - A) * B, (1 - A) * (1 - B) * G], axis=-1).reshape(-1, 3)
    return lam, W.ravel()


def _monomials(lam, N):
    """Monomials l1^i l2^j l3^k, i + j + k <= N, at barycentric points."""
    cols = []
    for tot in range(N + 1):
        for i in range(tot + 1):
            for j in range(tot - i + 1):
                k = tot - i - j
                cols.append(lam[:, 0] ** i * lam[:, 1] ** j * lam[:, 2] ** k)
    return np.stack(cols, axis=1)


class Evaluator:
    """Quadrature points of every tetrahedron of a mesh and the map from a
    tetrahedron's nodal values (the library's nodes) to them."""

    def __init__(self, VX, EToV, node_xyz, N, rho=1.0, c=1.0, n_gauss=4):
        VX = np.asarray(VX, dtype=np.float64)
        E = np.asarray(EToV)
        v = VX[E]                                              # (K, 4, 3)
        Jm = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], axis=2)
        self.vol6 = np.abs(np.linalg.det(Jm))                  # 6 |T|
        # barycentric coordinates of the nodes, the same in every element
        # (the nodes are images of one reference set in vertex order)
        lamn = np.linalg.solve(Jm, (node_xyz - v[:, 0][:, None, :]).transpose(0, 2, 1))
        lamn = lamn.transpose(0, 2, 1)                         # (K, Np, 3)
        if not np.allclose(lamn, lamn[0][None], atol=1e-9):
            raise ValueError("element nodes are not one reference set in vertex order")
        lq, self.wq = simplex_rule(n_gauss)
        V = _monomials(lamn[0], N)
        self.I = _monomials(lq, N) @ np.linalg.inv(V)          # (nq, Np)
        self.xq = v[:, 0][:, None, :] + np.einsum("kij,qj->kqi", Jm, lq)   # (K, nq, 3)
        self.rho, self.c = rho, c

    def integrate(self, f):
        """Integral over the mesh of values f (K, nq) at the quadrature points."""
        return float(np.sum(self.vol6 * (f @ self.wq)))

    def energy(self, q3):
        """int p^2/(2 rho c^2) + rho |u|^2 / 2 dx of nodal fields q3 (K, 4, Np)."""
        fq = np.einsum("qn,kfn->kfq", self.I, q3)
        rho, c = self.rho, self.c
        return self.integrate(fq[:, 0] ** 2 / (2 * rho * c * c)
                              + 0.5 * rho * np.sum(fq[:, 1:] ** 2, axis=1))

    def reference_at(self, t, xs, f0, t0, z_top=None):
        """The reference fields at the quadrature points: (p (K, nq),
        u (K, 3, nq))."""
        p, u = reference(self.xq, t, xs, f0, t0, self.rho, self.c, z_top)
        return p, u.transpose(0, 2, 1)

    def error_energy(self, q3, ref):
        """int (p_ref - p)^2/(2 rho c^2) + rho |u_ref - u|^2/2 dx for nodal
        fields q3 (K, 4, Np) and reference fields from reference_at."""
        fq = np.einsum("qn,kfn->kfq", self.I, q3)
        p, u = ref
        rho, c = self.rho, self.c
        return self.integrate((p - fq[:, 0]) ** 2 / (2 * rho * c * c)
                              + 0.5 * rho * np.sum((u - fq[:, 1:]) ** 2, axis=1))


def run_benchmark(VX, E, dt, N=3, orders=(0, 2, 4, 6, 8, 10, 12),
                  sources=((0.0, 0.0, 0.0), (0.2, 0.1, 0.0)), free_surface=False, t_final=5.0,
                  sample=0.25, f0=2.5, t0=0.5, t_energy=1.5, graph=True, log=None,
                  extra=None):
    """Section 4.1's validation benchmark on the GPU library: a tetrahedral
    mesh (VX, E) of [-0.5, 0.5]^3, degree N, rho = c = 1, time step dt, the
    Ricker source at each of `sources`, HABC of every order in `orders` on
    all faces (order 0: the basic ABC), or on all but the top face z = 0.5,
    which has p = 0 (free_surface).  E_src comes from a run with p = 0 on
    every face at t_energy.  `extra` maps labels to (P, gamma) for runs with
    coefficients other than Pade's.  Returns {source: {"E_src", "times",
    order or label: [Error(t)]}} with Error as defined in the module
    docstring."""
    import torch
    from .binding import Solver
    K = E.shape[0]
    rho, c = np.ones(K), np.ones(K)
    box = np.array([-0.5, -0.5, -0.5, 0.5, 0.5, 0.5])
    ev = None
    z_top = 0.5 if free_surface else None
    out = {}
    times = np.round(np.arange(0.0, t_final + 1e-9, sample), 10)

    def advance(solvers, t_now, t_next):
        k = int(round((t_next - t_now) / dt))
        for s in solvers:
            s.step(k, dt, t_now)
        return t_now + k * dt

    for xs in sources:
        # E_src: p = 0 on every face, energy once the wavelet is emitted
        sd = Solver(VX, E, N, 0, rho, c, face_bc=("dirichlet",) * 6, box=box).bind()
        if ev is None:
            ev = Evaluator(VX, E, sd.node_coords(), N)
        sd.set_source(xs, f0, t0)
        if graph:
            sd.set_graph(True)
        tE = advance([sd], 0.0, t_energy)
        q3 = sd.read_fields(["q3"])["q3"]
        e_src = ev.energy(q3)
        e_lib = sd.energy()
        sd.close()
        rec = {"E_src": e_src, "E_src_library": e_lib, "t_energy": tE, "times": [], "dt": dt}
        solvers = {}
        runs = [(P, P, None) for P in orders] + [(k, P, g) for k, (P, g) in (extra or {}).items()]
        for key, P, gamma in runs:
            fb = ["habc"] * 6
            if free_surface:
                fb[5] = "dirichlet"
            s = Solver(VX, E, N, P, rho, c, face_bc=fb, box=box, gamma=gamma).bind()
            s.set_source(xs, f0, t0)
            if graph:
                s.set_graph(True)
            solvers[key] = s
            rec[key] = []
        t_now = 0.0
        for tt in times:
            t_now = advance(list(solvers.values()), t_now, tt)
            ref = ev.reference_at(t_now, xs, f0, t0, z_top) if t_now > 0 else None
            rec["times"].append(t_now)
            for P, s in solvers.items():
                if ref is None:
                    rec[P].append(0.0)
                    continue
                q3 = s.read_fields(["q3"])["q3"]
                rec[P].append(math.sqrt(max(ev.error_energy(q3, ref), 0.0) / e_src))
            if log:
                log(f"source {xs}: t = {t_now:.3f}: " +
                    ", ".join(f"P={P} {rec[P][-1]:.2e}" for P in solvers))
        for s in solvers.values():
            s.close()
        torch.cuda.synchronize()
        out[tuple(xs)] = rec
    return out
