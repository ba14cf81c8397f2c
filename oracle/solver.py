"""The multidimensional explicit step of the oracle (FP64; test
infrastructure, never imported by the library).

Algorithm 1 of the paper, discretised as in Section 3.2: nodal DG with
upwind fluxes on the volume (3D), the HABC faces (2D, P sets of fields per
face) and the HABC edges (1D, P^2 sets per edge), the corner systems (0D),
and the five-stage fourth-order low-storage Runge-Kutta scheme of Carpenter
and Kennedy.

Each stage s of a step from t_m (stage time tau = t_m + C_s dt):
  1. right-hand sides of all three levels from the stage-start states and the
     incoming characteristics qb of the previous stage;
  2. 3D update: res = A_s res + dt rhs; q = q + B_s res;
  3. 2D update, then the face rule: outgoing r+ from the new 3D trace,
     r- = (1/M) sum_i gamma_i p*_i, the sum S = r+ + r- kept in q0_3, and
     p_i = p*_i + S;
  4. 1D update, then the edge systems from the new 2D traces, giving qb2,
     q0_2 and the rebuilt p_ij;
  5. 0D: the corner systems from the new 1D traces give qb1.

Characteristics (reading of the garbled definitions): r+- = (p +- Z n.u)/2
with Z = rho c and n the outward normal of the boundary at hand; with this
scaling the characteristic form of the flux equals the exact upwind flux and
the face rule equals the first-order face condition.

The 2D and 1D fluxes (not written in the paper) use the same upwind flux with
the impedance of the boundary cell; the stored 2D/1D pressure is the full
auxiliary pressure (p_i, p_ij), the integrated one is p* (Section 3.3's
temporary storage q0 rebuilds p* each stage).
"""
from __future__ import annotations

import math

import numpy as np

from .habc import pade_gamma, solve_edge, solve_corner, C2
from .mesh import Mesh, BC_HABC, BC_ABC, BC_DIRICHLET, DOMAIN_EDGES
from .reference import tet_basis

# Carpenter & Kennedy (1994), five stages, fourth order, 2N storage.
LSRK_A = np.array([0.0,
                   -567301805773.0 / 1357537059087.0,
                   -2404267990393.0 / 2016746695238.0,
                   -3550918686646.0 / 2091501179385.0,
                   -1275806237668.0 / 842570457699.0])
LSRK_B = np.array([1432997174477.0 / 9575080441755.0,
                   5161836677717.0 / 13612068292357.0,
                   1720146321549.0 / 2090206949498.0,
                   3134564353537.0 / 4481467310338.0,
                   2277821191437.0 / 14882151754819.0])
LSRK_C = np.array([0.0,
                   1432997174477.0 / 9575080441755.0,
                   2526269341429.0 / 6820363962896.0,
                   2006345519317.0 / 3224310063776.0,
                   2802321613138.0 / 2924317926251.0])


def upwind_flux(pM, unM, ZM, pP, unP, ZP):
    """Exact-Riemann upwind flux between two cells (Section 3.2):
    p* = ({p/Z} - n.[[u]]) / {1/Z},  (n.u)* = (n.{Z u} - [[p]]) / {Z},
    averages {X} = (X+ + X-)/2, semi-jumps [[X]] = (X+ - X-)/2, n the outward
    normal of the interior (-) cell."""
    avg_pZ = 0.5 * (pP / ZP + pM / ZM)
    jump_un = 0.5 * (unP - unM)
    avg_iZ = 0.5 * (1.0 / ZP + 1.0 / ZM)
    pF = (avg_pZ - jump_un) / avg_iZ
    avg_Zun = 0.5 * (ZP * unP + ZM * unM)
    jump_p = 0.5 * (pP - pM)
    avg_Z = 0.5 * (ZP + ZM)
    unF = (avg_Zun - jump_p) / avg_Z
    return pF, unF


def char_flux(pM, unM, Z, rminus):
    """Characteristic form at a boundary with a given incoming characteristic:
    p* = r+_int + r-_ext, (n.u)* = (r+_int - r-_ext)/Z."""
    rplus = 0.5 * (pM + Z * unM)
    return rplus + rminus, (rplus - rminus) / Z


def dirichlet_flux(pM, unM, Z):
    """p = 0 condition: p* = 0, (n.u)* = n.u_int + p_int / Z."""
    return np.zeros_like(pM), unM + pM / Z


def ricker_integral(t, f0, t0, amp=1.0):
    """S(t) = integral of the Ricker wavelet = (t - t0) exp(-pi^2 f0^2 (t-t0)^2)
    (Section 4.1)."""
    d = t - t0
    return amp * d * math.exp(-(math.pi * f0 * d) ** 2)


class Oracle:
    """FP64 oracle of the full step.  State arrays use the canonical layouts:
    q3 (K, 4, Np) fields (p, u, v, w); q2 (Ktri, P, 3, Np2) fields (p_i, two
    tangential velocities in axis order); q1 (Klin, P*P, 2, Np1) fields
    (p_ij, velocity along +axis), set index = i*P + j with i on the earlier
    face; qb3, q0_3 (Ktri, Np2); qb2, q0_2 (Klin, 2, P, Np1); qb1 (Kpnt, 3, P*P);
    res* have the shape of the matching q*."""

    def __init__(self, VX, EToV, N, P, rho, c, face_bc=(BC_HABC,) * 6,
                 periodic=(False, False, False), gamma=None, box=None):
        self.m = m = Mesh(VX, EToV, N, P, face_bc, periodic, box)
        self.N, self.P = N, P
        self.gamma = pade_gamma(P) if gamma is None else np.asarray(gamma, dtype=np.float64)
        self.M = 2 * P + 1
        self.rho = np.asarray(rho, dtype=np.float64)
        self.c = np.asarray(c, dtype=np.float64)
        self.Z = self.rho * self.c
        self.Kb = self.rho * self.c ** 2                          # bulk modulus rho c^2
        # boundary-level materials: the owning tet of a triangle; the side-A
        # triangle's tet for a line
        self.tri_rho = self.rho[m.tri_elem]
        self.tri_c = self.c[m.tri_elem]
        if m.Klin:
            self.lin_rho = self.tri_rho[m.lin_tri[:, 0]]
            self.lin_c = self.tri_c[m.lin_tri[:, 0]]
        else:
            self.lin_rho = np.zeros(0)
            self.lin_c = np.zeros(0)
        # flat gather indices of interior (iM) and neighbour (iP) face traces
        Np = m.tet.Np
        self.i3M = np.arange(m.K)[:, None, None] * Np + m.tet.Fmask[None, :, :]
        e2 = np.where(m.EToE >= 0, m.EToE, np.arange(m.K)[:, None])
        nn = np.where(m.nbr_node >= 0, m.nbr_node, m.tet.Fmask[None, :, :])
        self.i3P = e2[:, :, None] * Np + nn
        self.Z3M = self.Z[:, None, None]
        self.Z3P = self.Z[e2][:, :, None]
        self.sources = []
        self._boundary_groups()
        self.reset()

    def _boundary_groups(self):
        """Index lists of boundary faces / edges / line ends by condition."""
        m = self.m
        eb, fb = np.nonzero(m.EToE < 0)
        bc = np.array([m.face_bc[d] for d in m.bface[eb, fb]], dtype=object)
        h = bc == BC_HABC
        self.b3_habc = (eb[h], fb[h], m.face_tri[eb[h], fb[h]])
        self.b3_abc = (eb[bc == BC_ABC], fb[bc == BC_ABC])
        self.b3_dir = (eb[bc == BC_DIRICHLET], fb[bc == BC_DIRICHLET])
        tb, fb = np.nonzero(m.tri_EToE < 0)
        ln = m.tri_edge_line[tb, fb]
        has = ln >= 0
        self.b2_line = (tb[has], fb[has], ln[has], m.tri_edge_side[tb[has], fb[has]])
        obc = np.array([m.face_bc[d] for d in m.tri_bdface[tb, fb]], dtype=object)
        d = (~has) & (obc == BC_DIRICHLET)
        a = (~has) & (obc != BC_DIRICHLET)
        self.b2_dir = (tb[d], fb[d])
        self.b2_abc = (tb[a], fb[a])
        ends = np.array([0, m.line.Np - 1])
        li, ei = np.nonzero(m.lin_EToE >= 0)
        self.b1_int = (li, ei, m.lin_EToE[li, ei], ends[m.lin_EToF[li, ei]])
        li, ei = np.nonzero(m.lin_corner >= 0)
        self.b1_corner = (li, ei, m.lin_corner[li, ei], m.lin_corner_slot[li, ei])
        li, ei = np.nonzero((m.lin_EToE < 0) & (m.lin_corner < 0))
        bcs = m.lin_bc[li, ei] if len(li) else np.zeros(0, dtype=object)
        dd = bcs == BC_DIRICHLET
        self.b1_dir = (li[dd], ei[dd])
        self.b1_abc = (li[~dd], ei[~dd])

    # ----------------------------------------------------------- state ----
    def shapes(self):
        m, P = self.m, self.P
        return {
            "q3": (m.K, 4, m.tet.Np), "res3": (m.K, 4, m.tet.Np),
            "q2": (m.Ktri, P, 3, m.tri.Np), "res2": (m.Ktri, P, 3, m.tri.Np),
            "qb3": (m.Ktri, m.tri.Np), "q0_3": (m.Ktri, m.tri.Np),
            "q1": (m.Klin, P * P, 2, m.line.Np), "res1": (m.Klin, P * P, 2, m.line.Np),
            "qb2": (m.Klin, 2, P, m.line.Np), "q0_2": (m.Klin, 2, P, m.line.Np),
            "qb1": (m.Kpnt, 3, P * P),
        }

    def reset(self):
        self.s = {k: np.zeros(v) for k, v in self.shapes().items()}

    def node_coords(self):
        return self.m.xn

    # ---------------------------------------------------------- source ----
    def set_source(self, xs, f0, t0, amp=1.0):
        """Point source delta(x - xs) S(t) in the pressure equation (Section
        4.1).  The nodal weights are M^-1 l(r_s) / J = V psi(r_s) / J for the
        cell containing xs (the most interior one if xs lies on a face)."""
        m = self.m
        v = m.VX[m.EToV]
        Jm = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], axis=2)
        lam = np.linalg.solve(Jm, (np.asarray(xs) - v[:, 0])[:, :, None])[:, :, 0]
        bary = np.concatenate([1.0 - lam.sum(axis=1, keepdims=True), lam], axis=1)
        k = int(np.argmax(bary.min(axis=1)))
        rs = 2.0 * lam[k] - 1.0
        V, _, _, _ = tet_basis(rs[None, :], self.N)
        w = (m.tet.V @ V[0]) / m.J[k]
        self.sources.append((k, w, f0, t0, amp))
        return k, w

    # ------------------------------------------------------------- rhs ----
    def rhs3d(self, q3, qb3, tau):
        """Local right-hand side of the 3D pressure-velocity system (Section
        3.2, strong DG form):
          rhs_p = -rho c^2 div u + LIFT [Fscale rho c^2 (n.u^- - (n.u)*)]
          rhs_u = -(1/rho) grad p + LIFT [Fscale (1/rho) (p^- - p*) n]."""
        m, T = self.m, self.m.tet
        p, u, v, w = q3[:, 0], q3[:, 1], q3[:, 2], q3[:, 3]

        def d_rst(f):
            return f @ T.Dr.T, f @ T.Ds.T, f @ T.Dt.T

        pr, ps, pt = d_rst(p)
        ur, us, ut = d_rst(u)
        vr, vs, vt = d_rst(v)
        wr, ws, wt = d_rst(w)
        col = lambda a: a[:, None]
        px = col(m.rx) * pr + col(m.sx) * ps + col(m.tx) * pt
        py = col(m.ry) * pr + col(m.sy) * ps + col(m.ty) * pt
        pz = col(m.rz) * pr + col(m.sz) * ps + col(m.tz) * pt
        div = (col(m.rx) * ur + col(m.sx) * us + col(m.tx) * ut
               + col(m.ry) * vr + col(m.sy) * vs + col(m.ty) * vt
               + col(m.rz) * wr + col(m.sz) * ws + col(m.tz) * wt)

        nx, ny, nz = m.nrm[:, :, 0, None], m.nrm[:, :, 1, None], m.nrm[:, :, 2, None]
        iM, iP = self.i3M, self.i3P
        pM = p.ravel()[iM]
        unM = nx * u.ravel()[iM] + ny * v.ravel()[iM] + nz * w.ravel()[iM]
        # neighbour traces (boundary faces are overwritten below)
        pP = p.ravel()[iP]
        unP = nx * u.ravel()[iP] + ny * v.ravel()[iP] + nz * w.ravel()[iP]
        pF, unF = upwind_flux(pM, unM, self.Z3M, pP, unP, self.Z3P)
        # boundary faces, grouped by condition
        e, f, t = self.b3_habc
        if len(e):
            rm = qb3[t[:, None], m.facenode_trinode[t]]
            pF[e, f], unF[e, f] = char_flux(pM[e, f], unM[e, f], self.Z[e][:, None], rm)
        e, f = self.b3_abc
        if len(e):
            pF[e, f], unF[e, f] = char_flux(pM[e, f], unM[e, f], self.Z[e][:, None], 0.0)
        e, f = self.b3_dir
        if len(e):
            pF[e, f], unF[e, f] = dirichlet_flux(pM[e, f], unM[e, f], self.Z[e][:, None])
        K = m.K
        Fs = m.Fscale[:, :, None]
        gp = (Fs * col(self.Kb)[:, :, None] * (unM - unF)).reshape(K, -1)
        gu = Fs * (1.0 / col(self.rho))[:, :, None] * (pM - pF)
        out = np.empty_like(q3)
        out[:, 0] = -col(self.Kb) * div + gp @ T.LIFT.T
        out[:, 1] = -px / col(self.rho) + (gu * nx).reshape(K, -1) @ T.LIFT.T
        out[:, 2] = -py / col(self.rho) + (gu * ny).reshape(K, -1) @ T.LIFT.T
        out[:, 3] = -pz / col(self.rho) + (gu * nz).reshape(K, -1) @ T.LIFT.T
        for (k, wgt, f0, t0, amp) in self.sources:
            out[k, 0] += wgt * ricker_integral(tau, f0, t0, amp)
        return out

    def rhs2d(self, q2, qb2):
        """Right-hand side of the 2D systems on the faces, set i (Section 3.1,
        2D relations of the procedure; Section 3.2 DG):
          (1+gamma_i) dp*_i/dt + rho c^2 div_t v_i = 0,  rho dv_i/dt + grad_t p_i = 0,
        flux on the full p_i with Z = rho c; at domain edges the incoming
        characteristic is qb2 (edge system of the previous stage)."""
        m, Tr, P = self.m, self.m.tri, self.P
        out = np.zeros_like(q2)
        if m.Ktri == 0 or P == 0:
            return out
        col = lambda a: a[:, None]
        rho, Z = self.tri_rho, self.tri_rho * self.tri_c
        Fm = Tr.Fmask
        na, nb = m.tri_nrm[:, :, 0, None], m.tri_nrm[:, :, 1, None]
        Fs = m.tri_Fscale[:, :, None]
        ti, fi = np.nonzero(m.tri_EToE >= 0)
        t2, nn = m.tri_EToE[ti, fi], m.tri_nbr_node[ti, fi]
        for i in range(P):
            Ki = self.tri_rho * self.tri_c ** 2 / (1.0 + self.gamma[i])
            p, va, vb = q2[:, i, 0], q2[:, i, 1], q2[:, i, 2]
            pr, ps = p @ Tr.Dr.T, p @ Tr.Ds.T
            pa = col(m.tri_rx) * pr + col(m.tri_sx) * ps
            pb = col(m.tri_ry) * pr + col(m.tri_sy) * ps
            div = (col(m.tri_rx) * (va @ Tr.Dr.T) + col(m.tri_sx) * (va @ Tr.Ds.T)
                   + col(m.tri_ry) * (vb @ Tr.Dr.T) + col(m.tri_sy) * (vb @ Tr.Ds.T))
            pM = p[:, Fm]
            vnM = na * va[:, Fm] + nb * vb[:, Fm]
            pF = np.zeros_like(pM)
            vnF = np.zeros_like(pM)
            pP = p[t2[:, None], nn]
            vnP = na[ti, fi] * va[t2[:, None], nn] + nb[ti, fi] * vb[t2[:, None], nn]
            pF[ti, fi], vnF[ti, fi] = upwind_flux(pM[ti, fi], vnM[ti, fi], Z[ti][:, None],
                                                  pP, vnP, Z[t2][:, None])
            t, f, l, side = self.b2_line
            if len(t):
                rm = qb2[l[:, None], side[:, None], i, m.tri_edge_linenode[t, f]]
                pF[t, f], vnF[t, f] = char_flux(pM[t, f], vnM[t, f], Z[t][:, None], rm)
            t, f = self.b2_dir
            if len(t):
                pF[t, f], vnF[t, f] = dirichlet_flux(pM[t, f], vnM[t, f], Z[t][:, None])
            t, f = self.b2_abc
            if len(t):
                pF[t, f], vnF[t, f] = char_flux(pM[t, f], vnM[t, f], Z[t][:, None], 0.0)
            Kt = m.Ktri
            gp = (Fs * col(Ki)[:, :, None] * (vnM - vnF)).reshape(Kt, -1)
            gv = Fs * (1.0 / col(rho))[:, :, None] * (pM - pF)
            out[:, i, 0] = -col(Ki) * div + gp @ Tr.LIFT.T
            out[:, i, 1] = -pa / col(rho) + (gv * na).reshape(Kt, -1) @ Tr.LIFT.T
            out[:, i, 2] = -pb / col(rho) + (gv * nb).reshape(Kt, -1) @ Tr.LIFT.T
        return out

    def rhs1d(self, q1, qb1):
        """Right-hand side of the 1D systems on the edges, set (i, j):
          (1+gamma_i+gamma_j) dp*_ij/dt + rho c^2 dw_ij/dx = 0,
          rho dw_ij/dt + dp_ij/dx = 0,
        with x along the edge; at corners the incoming characteristic is qb1."""
        m, L, P = self.m, self.m.line, self.P
        out = np.zeros_like(q1)
        if m.Klin == 0 or P == 0:
            return out
        rho, Z = self.lin_rho, self.lin_rho * self.lin_c
        col = lambda a: a[:, None]
        ends = np.array([0, L.Np - 1])
        for i in range(P):
            for j in range(P):
                s = i * P + j
                Kij = self.lin_rho * self.lin_c ** 2 / (1.0 + self.gamma[i] + self.gamma[j])
                p, w = q1[:, s, 0], q1[:, s, 1]
                px = col(m.lin_rx) * (p @ L.Dr.T)
                wx = col(m.lin_rx) * (w @ L.Dr.T)
                pM = p[:, ends]
                wnM = m.lin_nrm * w[:, ends]
                pF = np.zeros_like(pM)
                wnF = np.zeros_like(pM)
                l, e, l2, node2 = self.b1_int
                if len(l):
                    pP = q1[l2, s, 0, node2]
                    wnP = m.lin_nrm[l, e] * q1[l2, s, 1, node2]
                    pF[l, e], wnF[l, e] = upwind_flux(pM[l, e], wnM[l, e], Z[l], pP, wnP, Z[l2])
                l, e, cp, slot = self.b1_corner
                if len(l):
                    pF[l, e], wnF[l, e] = char_flux(pM[l, e], wnM[l, e], Z[l], qb1[cp, slot, s])
                l, e = self.b1_dir
                if len(l):
                    pF[l, e], wnF[l, e] = dirichlet_flux(pM[l, e], wnM[l, e], Z[l])
                l, e = self.b1_abc
                if len(l):
                    pF[l, e], wnF[l, e] = char_flux(pM[l, e], wnM[l, e], Z[l], 0.0)
                Fs = col(m.lin_Fscale)
                gp = Fs * col(Kij) * (wnM - wnF)
                gw = Fs * (1.0 / col(rho)) * (pM - pF) * m.lin_nrm
                out[:, s, 0] = -col(Kij) * wx + gp @ L.LIFT.T
                out[:, s, 1] = -px / col(rho) + gw @ L.LIFT.T
        return out

    # ---------------------------------------------------------- levels ----
    def face_rule(self, q3, pstar):
        """Section 3.1 face procedure at every triangle node: r+ from the new
        3D trace (n = outward domain normal), r- = (1/M) sum_i gamma_i p*_i.
        Returns (r-, S = r+ + r-)."""
        m = self.m
        e, f = m.tri_elem, m.tri_face
        n = m.nrm[e, f]                                           # (Kt, 3)
        nodes = m.tri_tetnode                                     # (Kt, Np2)
        p3 = q3[e[:, None], 0, nodes]
        un = (n[:, 0, None] * q3[e[:, None], 1, nodes] + n[:, 1, None] * q3[e[:, None], 2, nodes]
              + n[:, 2, None] * q3[e[:, None], 3, nodes])
        Z = self.Z[e][:, None]
        rplus = 0.5 * (p3 + Z * un)
        rminus = np.zeros_like(rplus)
        for i in range(self.P):
            rminus += self.gamma[i] * pstar[:, i]
        rminus /= self.M
        return rminus, rplus + rminus

    def edge_rplus(self, q2):
        """Outgoing 2D characteristics at line nodes: face A's fields with the
        normal of face B and vice versa.  Returns (rpA (Kl, P, Np1), rpB)."""
        m, P = self.m, self.P
        out = []
        for side in range(2):
            t = m.lin_tri[:, side]
            nodes = m.lin_trinode[:, side]                          # (Kl, Np1)
            other = [DOMAIN_EDGES[d][1 - side] for d in m.lin_dedge]
            ax = np.array([o // 2 for o in other])
            sgn = np.array([1.0 if o % 2 else -1.0 for o in other])
            comp = np.array([1 + list(m.tri_axes[tt]).index(a) for tt, a in zip(t, ax)])
            Z = (self.tri_rho * self.tri_c)[t]
            p = q2[t[:, None], :, 0, nodes]                         # (Kl, Np1, P)
            vn = sgn[:, None, None] * q2[t[:, None], :, comp[:, None], nodes]
            r = 0.5 * (p + Z[:, None, None] * vn)
            out.append(np.transpose(r, (0, 2, 1)))
        return out[0], out[1]

    def stage(self, s, dt, t):
        A, B, C = LSRK_A[s], LSRK_B[s], LSRK_C[s]
        st, P, m = self.s, self.P, self.m
        tau = t + C * dt
        rhs3 = self.rhs3d(st["q3"], st["qb3"], tau)
        rhs2 = self.rhs2d(st["q2"], st["qb2"])
        rhs1 = self.rhs1d(st["q1"], st["qb1"])
        # 3D
        st["res3"] = A * st["res3"] + dt * rhs3
        st["q3"] = st["q3"] + B * st["res3"]
        if m.Ktri == 0:
            return
        # 2D + face rule
        st["res2"] = A * st["res2"] + dt * rhs2
        pstar = st["q2"][:, :, 0] - st["q0_3"][:, None, :] + B * st["res2"][:, :, 0]
        q2 = st["q2"].copy()
        q2[:, :, 1:] = st["q2"][:, :, 1:] + B * st["res2"][:, :, 1:]
        rm, S = self.face_rule(st["q3"], pstar)
        st["qb3"], st["q0_3"] = rm, S
        q2[:, :, 0] = pstar + S[:, None, :]
        st["q2"] = q2
        if m.Klin == 0 or P == 0:
            return
        # 1D + edge systems
        st["res1"] = A * st["res1"] + dt * rhs1
        g = self.gamma
        CA = np.array([[C2(g, j, i) for j in range(P)] for i in range(P)])   # C_ji at [i, j]
        CB = np.array([[C2(g, i, j) for j in range(P)] for i in range(P)])   # C_ij at [i, j]
        q1 = st["q1"].reshape(m.Klin, P, P, 2, -1).copy()
        SA, SB = st["q0_2"][:, 0], st["q0_2"][:, 1]                        # (Kl, P, Np1)
        pstar1 = (q1[:, :, :, 0] - CA[None, :, :, None] * SA[:, :, None, :]
                  - CB[None, :, :, None] * SB[:, None, :, :]
                  + B * st["res1"].reshape(m.Klin, P, P, 2, -1)[:, :, :, 0])
        q1[:, :, :, 1] += B * st["res1"].reshape(m.Klin, P, P, 2, -1)[:, :, :, 1]
        rpA, rpB = self.edge_rplus(st["q2"])
        Np1 = m.line.Np
        ps = np.transpose(pstar1, (1, 2, 0, 3)).reshape(P, P, -1)            # (P, P, Kl*Np1)
        rmA, rmB = solve_edge(g, ps, np.transpose(rpA, (1, 0, 2)).reshape(P, -1),
                              np.transpose(rpB, (1, 0, 2)).reshape(P, -1))
        rmA = np.transpose(rmA.reshape(P, m.Klin, Np1), (1, 0, 2))
        rmB = np.transpose(rmB.reshape(P, m.Klin, Np1), (1, 0, 2))
        SAn, SBn = rpA + rmA, rpB + rmB
        st["qb2"] = np.stack([rmA, rmB], axis=1)
        st["q0_2"] = np.stack([SAn, SBn], axis=1)
        q1[:, :, :, 0] = (pstar1 + CA[None, :, :, None] * SAn[:, :, None, :]
                          + CB[None, :, :, None] * SBn[:, None, :, :])
        st["q1"] = q1.reshape(m.Klin, P * P, 2, -1)
        if m.Kpnt == 0:
            return
        # 0D corner systems
        rp = np.empty((m.Kpnt, 3, P * P))
        for c in range(m.Kpnt):
            for a in range(3):
                l, end = m.pnt_line[c, a], m.pnt_end[c, a]
                node = Np1 - 1 if end else 0
                Z = self.lin_rho[l] * self.lin_c[l]
                rp[c, a] = 0.5 * (st["q1"][l, :, 0, node]
                                  + Z * m.pnt_nrm[c, a] * st["q1"][l, :, 1, node])
        rX, rY, rZ = solve_corner(g, rp[:, 0].T, rp[:, 1].T, rp[:, 2].T)
        st["qb1"] = np.stack([rX.T, rY.T, rZ.T], axis=1)

    def step(self, n_steps, dt, t_start=0.0):
        t = t_start
        for _ in range(n_steps):
            for s in range(5):
                self.stage(s, dt, t)
            t = t + dt
        return t

    # ---------------------------------------------------------- energy ----
    def energy(self):
        """E = sum_k J_k/2 [p^T M p / (rho c^2) + rho u^T M u] (the energy
        weights of the validation error norm, Section 4.1)."""
        m, T = self.m, self.m.tet
        q = self.s["q3"]
        Mq = q @ T.M.T
        e = (np.sum(q[:, 0] * Mq[:, 0], axis=1) / self.Kb
             + self.rho * np.sum(q[:, 1:] * Mq[:, 1:], axis=(1, 2)))
        return float(np.sum(0.5 * m.J * e))
