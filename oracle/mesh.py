"""Affine geometry and four-level connectivity of the oracle (FP64; test
infrastructure, never imported by the library).

Section 3.2: the volume mesh of K_tet tetrahedra; the surface mesh of the
tetrahedron faces lying on HABC faces of the cuboid (K_tri triangles); the
line mesh of the tetrahedron edges lying on domain edges where two HABC faces
meet (K_lin lines); the corners where three HABC faces meet (K_pnt).
Geometric factors follow the affine map of each cell (Hesthaven & Warburton,
cited in Section 3.2): metric terms, outward unit normals, and the ratio of
surface to volume Jacobians (Fscale).

Canonical orderings (shared interface with the library, which computes its
own):
  domain faces   0..5 = x-, x+, y-, y+, z-, z+; axis = d // 2
  triangles      sorted by (domain face, owning tet, local face of the tet);
                 vertices sorted by global vertex id -> reference vertices
                 (-1,-1), (1,-1), (-1,1); in-plane coordinates are the two
                 tangential Cartesian axes in increasing order
  domain edges   the 12 pairs (A, B) of faces on different axes, A < B,
                 in lexicographic order; A is the "earlier" face
  lines          sorted by (domain edge, smaller vertex id, larger vertex id);
                 node 0 at the smaller vertex id; velocity = +axis component
  corners        c = xb + 2*yb + 4*zb (b = 0 for the low side); edge slots
                 0, 1, 2 = the edges along x, y, z through the corner
"""
from __future__ import annotations

import numpy as np

from .reference import Tet, Tri, Line, FACE_VERTS, TRI_EDGE_VERTS

BC_HABC, BC_ABC, BC_DIRICHLET, BC_PERIODIC = "habc", "abc", "dirichlet", "periodic"

DOMAIN_EDGES = [(a, b) for a in range(6) for b in range(6) if a < b and a // 2 != b // 2]


def _match_nodes(xa, xb, box_len, periodic, tol):
    """For each row of points xa (F, n, 3) find the index of the coincident
    point in xb (F, n, 3) (coordinates compared modulo the box on periodic
    axes).  Returns (F, n) int."""
    F, n, _ = xa.shape
    out = np.empty((F, n), dtype=np.int64)
    chunk = 20000
    for s in range(0, F, chunk):
        a = xa[s:s + chunk, :, None, :]
        b = xb[s:s + chunk, None, :, :]
        d = a - b
        for ax in range(3):
            if periodic[ax]:
                d[..., ax] -= box_len[ax] * np.round(d[..., ax] / box_len[ax])
        dist = np.sqrt(np.sum(d * d, axis=-1))
        idx = np.argmin(dist, axis=2)
        best = np.take_along_axis(dist, idx[..., None], axis=2)[..., 0]
        if np.any(best > tol):
            raise ValueError("face nodes do not match")
        out[s:s + chunk] = idx
    return out


class Mesh:
    """Volume mesh plus the derived surface/line/corner meshes."""

    def __init__(self, VX, EToV, N, P, face_bc=(BC_HABC,) * 6, periodic=(False, False, False),
                 box=None):
        VX = np.asarray(VX, dtype=np.float64)
        EToV = np.asarray(EToV, dtype=np.int64)
        self.N, self.P = N, P
        self.tet, self.tri, self.line = Tet(N), Tri(N), Line(N)
        self.K = K = EToV.shape[0]
        self.VX, self.EToV = VX, EToV
        if box is None:
            box = (VX.min(axis=0), VX.max(axis=0))
        self.lo, self.hi = np.asarray(box[0], float), np.asarray(box[1], float)
        self.box_len = self.hi - self.lo
        self.periodic = tuple(bool(p) for p in periodic)
        face_bc = list(face_bc)
        for ax in range(3):
            if self.periodic[ax]:
                face_bc[2 * ax] = face_bc[2 * ax + 1] = BC_PERIODIC
        self.face_bc = face_bc
        hmin = np.min(np.linalg.norm(VX[EToV[:, 1]] - VX[EToV[:, 0]], axis=1))
        self.tol = 1e-7 * hmin
        self._geometry3d()
        self._connect3d()
        self._surface()
        self._lines()
        self._corners()

    # ------------------------------------------------------------- 3D -----
    def _geometry3d(self):
        """Affine map x = v0 + (r+1)/2 (v1-v0) + (s+1)/2 (v2-v0) + (t+1)/2 (v3-v0);
        metric terms from the inverse Jacobian; normals -grad(xi) on xi = -1
        faces and grad(r+s+t) on the slanted face; Fscale = |grad(xi)|."""
        T = self.tet
        v = self.VX[self.EToV]                                  # (K, 4, 3)
        self.xn = (v[:, 0, None, :]
                   + 0.5 * (T.x[None, :, 0, None] + 1) * (v[:, 1] - v[:, 0])[:, None, :]
                   + 0.5 * (T.x[None, :, 1, None] + 1) * (v[:, 2] - v[:, 0])[:, None, :]
                   + 0.5 * (T.x[None, :, 2, None] + 1) * (v[:, 3] - v[:, 0])[:, None, :])
        Jm = np.stack([(v[:, 1] - v[:, 0]) / 2, (v[:, 2] - v[:, 0]) / 2, (v[:, 3] - v[:, 0]) / 2],
                      axis=2)                                   # columns x_r, x_s, x_t
        self.J = np.linalg.det(Jm)
        if np.any(self.J <= 0):
            raise ValueError("negatively oriented tetrahedron")
        G = np.linalg.inv(Jm)                                   # rows grad r, grad s, grad t
        self.rx, self.ry, self.rz = G[:, 0, 0], G[:, 0, 1], G[:, 0, 2]
        self.sx, self.sy, self.sz = G[:, 1, 0], G[:, 1, 1], G[:, 1, 2]
        self.tx, self.ty, self.tz = G[:, 2, 0], G[:, 2, 1], G[:, 2, 2]
        gr, gs, gt = G[:, 0, :], G[:, 1, :], G[:, 2, :]
        nraw = np.stack([-gt, -gs, gr + gs + gt, -gr], axis=1)  # (K, 4, 3)
        mag = np.linalg.norm(nraw, axis=2)
        self.nrm = nraw / mag[..., None]
        self.Fscale = mag                                       # sJ/J

    def _connect3d(self):
        K, T = self.K, self.tet
        # periodic vertex identification
        vid = np.arange(self.VX.shape[0])
        if any(self.periodic):
            key = self.VX.copy()
            for ax in range(3):
                if self.periodic[ax]:
                    top = np.abs(key[:, ax] - self.hi[ax]) < self.tol
                    key[top, ax] = self.lo[ax]
            q = np.round((key - self.lo) / self.tol).astype(np.int64)
            _, first, inv = np.unique(q, axis=0, return_index=True, return_inverse=True)
            vid = first[inv.ravel()]
        self.vcanon = vid
        faces = np.stack([np.sort(vid[self.EToV[:, list(fv)]], axis=1) for fv in FACE_VERTS],
                         axis=1)                                # (K, 4, 3)
        flat = faces.reshape(-1, 3)
        order = np.lexsort((flat[:, 2], flat[:, 1], flat[:, 0]))
        fs = flat[order]
        same = np.all(fs[1:] == fs[:-1], axis=1)
        self.EToE = np.full((K, 4), -1, dtype=np.int64)
        self.EToF = np.full((K, 4), -1, dtype=np.int64)
        i1 = order[:-1][same]
        i2 = order[1:][same]
        self.EToE.ravel()[i1] = i2 // 4
        self.EToF.ravel()[i1] = i2 % 4
        self.EToE.ravel()[i2] = i1 // 4
        self.EToF.ravel()[i2] = i1 % 4
        # node matching across interior faces: nbr_node[e, f, i] = node of EToE[e,f]
        Fm = T.Fmask
        xM = self.xn[:, Fm, :]                                  # (K, 4, Nfp, 3)
        self.nbr_node = np.full((K, 4, T.Nfp), -1, dtype=np.int64)
        e_int, f_int = np.nonzero(self.EToE >= 0)
        e2, f2 = self.EToE[e_int, f_int], self.EToF[e_int, f_int]
        idx = _match_nodes(xM[e_int, f_int], xM[e2, f2], self.box_len, self.periodic,
                           1e3 * self.tol)
        self.nbr_node[e_int, f_int] = Fm[f2][np.arange(len(f2))[:, None], idx]
        # boundary faces: domain face id from the face centroid
        self.bface = np.full((K, 4), -1, dtype=np.int64)
        e_b, f_b = np.nonzero(self.EToE < 0)
        cen = xM[e_b, f_b].mean(axis=1)
        dface = np.full(len(e_b), -1)
        for ax in range(3):
            dface[np.abs(cen[:, ax] - self.lo[ax]) < self.tol * 1e3] = 2 * ax
            dface[np.abs(cen[:, ax] - self.hi[ax]) < self.tol * 1e3] = 2 * ax + 1
        if np.any(dface < 0):
            raise ValueError("boundary face not on the box")
        self.bface[e_b, f_b] = dface

    # ------------------------------------------------------------- 2D -----
    def _surface(self):
        """Triangles = tet faces on HABC faces (Section 3.2)."""
        Tr = self.tri
        e_b, f_b = np.nonzero(self.bface >= 0)
        d_b = self.bface[e_b, f_b]
        habc = np.array([self.face_bc[d] == BC_HABC for d in d_b], dtype=bool)
        e_b, f_b, d_b = e_b[habc], f_b[habc], d_b[habc]
        order = np.lexsort((f_b, e_b, d_b))
        self.tri_elem, self.tri_face, self.tri_dface = e_b[order], f_b[order], d_b[order]
        Kt = self.Ktri = len(self.tri_elem)
        tv = np.sort(self.EToV[self.tri_elem[:, None], np.array(FACE_VERTS)[self.tri_face]], axis=1)
        self.tri_verts = tv                                     # (Kt, 3) global ids, sorted
        va, vb, vc = self.VX[tv[:, 0]], self.VX[tv[:, 1]], self.VX[tv[:, 2]]
        r, s = Tr.x[:, 0], Tr.x[:, 1]
        self.tri_xn = (va[:, None, :] + 0.5 * (r[None, :, None] + 1) * (vb - va)[:, None, :]
                       + 0.5 * (s[None, :, None] + 1) * (vc - va)[:, None, :])
        # in-plane axes
        ax = self.tri_dface // 2
        self.tri_axes = np.array([[a for a in range(3) if a != x] for x in ax],
                                 dtype=np.int64).reshape(-1, 2)  # (Kt, 2)
        rows = np.arange(Kt)
        d1, d2 = (vb - va) / 2, (vc - va) / 2
        ar, as_ = d1[rows, self.tri_axes[:, 0]], d2[rows, self.tri_axes[:, 0]]
        br, bs = d1[rows, self.tri_axes[:, 1]], d2[rows, self.tri_axes[:, 1]]
        J = ar * bs - as_ * br
        self.tri_J = J
        self.tri_rx, self.tri_ry = bs / J, -as_ / J
        self.tri_sx, self.tri_sy = -br / J, ar / J
        gr = np.stack([self.tri_rx, self.tri_ry], axis=1)
        gs = np.stack([self.tri_sx, self.tri_sy], axis=1)
        nraw = np.stack([-gs, gr + gs, -gr], axis=1)            # (Kt, 3, 2)
        mag = np.linalg.norm(nraw, axis=2)
        self.tri_nrm = nraw / mag[..., None]
        self.tri_Fscale = mag
        # triangle node -> node of the owning tet
        xt = self.xn[self.tri_elem[:, None], self.tet.Fmask[self.tri_face]]   # (Kt, Nfp, 3)
        idx = _match_nodes(self.tri_xn, xt, self.box_len, self.periodic, 1e3 * self.tol)
        self.tri_tetnode = self.tet.Fmask[self.tri_face][rows[:, None], idx]   # (Kt, Np2)
        # map (e, f) -> triangle id, and tet face node i -> triangle node
        self.face_tri = np.full((self.K, 4), -1, dtype=np.int64)
        self.face_tri[self.tri_elem, self.tri_face] = rows
        # for tet face node i (Fmask order) the triangle node holding it
        inv = np.empty((Kt, Tr.Np), dtype=np.int64)
        Fm = self.tet.Fmask[self.tri_face]                      # (Kt, Nfp)
        for i in range(Tr.Np):
            inv[:, i] = np.argmax(self.tri_tetnode == Fm[:, i:i + 1], axis=1)
        self.facenode_trinode = inv                             # (Kt, Nfp)
        # triangle edges: neighbours within the surface mesh
        vcan = self.vcanon
        ekeys = np.stack([np.sort(vcan[tv[:, list(ev)]], axis=1) for ev in TRI_EDGE_VERTS],
                         axis=1)                                # (Kt, 3, 2)
        self.tri_EToE = np.full((Kt, 3), -1, dtype=np.int64)
        self.tri_EToF = np.full((Kt, 3), -1, dtype=np.int64)
        flat = np.concatenate([ekeys.reshape(-1, 2), np.repeat(self.tri_dface, 3)[:, None]], axis=1)
        order = np.lexsort((flat[:, 1], flat[:, 0], flat[:, 2]))
        fsrt = flat[order]
        same = np.all(fsrt[1:] == fsrt[:-1], axis=1)
        i1, i2 = order[:-1][same], order[1:][same]
        self.tri_EToE.ravel()[i1] = i2 // 3
        self.tri_EToF.ravel()[i1] = i2 % 3
        self.tri_EToE.ravel()[i2] = i1 // 3
        self.tri_EToF.ravel()[i2] = i1 % 3
        Fm2 = Tr.Fmask
        xe = self.tri_xn[:, Fm2, :]                              # (Kt, 3, Nfp2, 3)
        self.tri_nbr_node = np.full((Kt, 3, Tr.Nfp), -1, dtype=np.int64)
        t_int, f_int = np.nonzero(self.tri_EToE >= 0)
        t2, f2 = self.tri_EToE[t_int, f_int], self.tri_EToF[t_int, f_int]
        if len(t_int):
            idx = _match_nodes(xe[t_int, f_int], xe[t2, f2], self.box_len, self.periodic,
                               1e3 * self.tol)
            self.tri_nbr_node[t_int, f_int] = Fm2[f2][np.arange(len(f2))[:, None], idx]
        # boundary edges of triangles: which other domain face holds them
        self.tri_bdface = np.full((Kt, 3), -1, dtype=np.int64)
        t_b, f_b = np.nonzero(self.tri_EToE < 0)
        cen = xe[t_b, f_b].mean(axis=1)
        other = np.full(len(t_b), -1)
        for k in range(len(t_b)):
            d = self.tri_dface[t_b[k]]
            for ax in range(3):
                if ax == d // 2 or self.periodic[ax]:
                    continue
                if abs(cen[k, ax] - self.lo[ax]) < 1e3 * self.tol:
                    other[k] = 2 * ax
                if abs(cen[k, ax] - self.hi[ax]) < 1e3 * self.tol:
                    other[k] = 2 * ax + 1
        if np.any(other < 0):
            raise ValueError("triangle boundary edge not on a domain edge")
        self.tri_bdface[t_b, f_b] = other

    # ------------------------------------------------------------- 1D -----
    def _lines(self):
        """Lines = triangle edges on domain edges between two HABC faces."""
        L = self.line
        recs = []
        for ei, (A, B) in enumerate(DOMAIN_EDGES):
            if self.face_bc[A] != BC_HABC or self.face_bc[B] != BC_HABC:
                continue
            tA, fA = np.nonzero((self.tri_bdface == B) & (self.tri_dface[:, None] == A))
            for t, f in zip(tA, fA):
                vs = np.sort(self.tri_verts[t, list(TRI_EDGE_VERTS[f])])
                recs.append((ei, vs[0], vs[1], t, f))
        recs.sort(key=lambda r: (r[0], r[1], r[2]))
        Kl = self.Klin = len(recs)
        self.lin_dedge = np.array([r[0] for r in recs], dtype=np.int64)
        self.lin_verts = np.array([[r[1], r[2]] for r in recs], dtype=np.int64).reshape(Kl, 2)
        # velocity axis = the axis of neither face
        self.lin_axis = np.array([3 - DOMAIN_EDGES[d][0] // 2 - DOMAIN_EDGES[d][1] // 2
                                  for d in self.lin_dedge], dtype=np.int64).reshape(-1)
        va, vb = self.VX[self.lin_verts[:, 0]], self.VX[self.lin_verts[:, 1]]
        self.lin_xn = va[:, None, :] + 0.5 * (L.x[None, :, None] + 1) * (vb - va)[:, None, :]
        rows = np.arange(Kl)
        dx = (vb - va)[rows, self.lin_axis] / 2                 # dx/dr along the axis
        self.lin_rx = 1.0 / dx
        self.lin_Fscale = np.abs(self.lin_rx)
        self.lin_nrm = np.stack([-np.sign(dx), np.sign(dx)], axis=1)   # (Kl, 2) at r=-1, r=+1
        # the two triangles (side 0 = face A, side 1 = face B) and node maps
        self.lin_tri = np.full((Kl, 2), -1, dtype=np.int64)
        self.lin_tri_edge = np.full((Kl, 2), -1, dtype=np.int64)
        self.lin_trinode = np.full((Kl, 2, L.Np), -1, dtype=np.int64)
        self.tri_edge_line = np.full((self.Ktri, 3), -1, dtype=np.int64)
        self.tri_edge_side = np.full((self.Ktri, 3), -1, dtype=np.int64)
        self.tri_edge_linenode = np.full((self.Ktri, 3, self.tri.Nfp), -1, dtype=np.int64)
        tri_edges = {}
        for t, f in zip(*np.nonzero(self.tri_bdface >= 0)):
            vs = np.sort(self.tri_verts[t, list(TRI_EDGE_VERTS[f])])
            tri_edges[(self.tri_dface[t], self.tri_bdface[t, f], vs[0], vs[1])] = (t, f)
        for l in range(Kl):
            A, B = DOMAIN_EDGES[self.lin_dedge[l]]
            for side, (face, other) in enumerate(((A, B), (B, A))):
                key = (face, other, self.lin_verts[l, 0], self.lin_verts[l, 1])
                if key not in tri_edges:
                    raise ValueError("line without adjacent triangle")
                t, f = tri_edges[key]
                self.lin_tri[l, side] = t
                self.lin_tri_edge[l, side] = f
                tn = self.tri.Fmask[f]
                xt = self.tri_xn[t, tn]                          # (Nfp2, 3)
                xl = self.lin_xn[l]                              # (Np1, 3)
                d = np.linalg.norm(xl[:, None, :] - xt[None, :, :], axis=2)
                if np.max(np.min(d, axis=1)) > 1e3 * self.tol:
                    raise ValueError("line nodes do not match triangle nodes")
                self.lin_trinode[l, side] = tn[np.argmin(d, axis=1)]
                self.tri_edge_line[t, f] = l
                self.tri_edge_side[t, f] = side
                self.tri_edge_linenode[t, f] = np.argmin(d, axis=0)
        # line neighbours along the edge (shared vertex), ends at corners
        self.lin_EToE = np.full((Kl, 2), -1, dtype=np.int64)
        self.lin_EToF = np.full((Kl, 2), -1, dtype=np.int64)
        ends = {}
        for l in range(Kl):
            for side in range(2):
                key = (self.lin_dedge[l], self.vcanon[self.lin_verts[l, side]])
                ends.setdefault(key, []).append((l, side))
        for key, lst in ends.items():
            if len(lst) == 2:
                (l1, s1), (l2, s2) = lst
                self.lin_EToE[l1, s1], self.lin_EToF[l1, s1] = l2, s2
                self.lin_EToE[l2, s2], self.lin_EToF[l2, s2] = l1, s1

    # ------------------------------------------------------------- 0D -----
    def _corners(self):
        """Corners where three HABC faces meet; slot a holds the line along
        axis a through the corner."""
        recs = []
        for c in range(8):
            bits = [(c >> a) & 1 for a in range(3)]
            faces = [2 * a + bits[a] for a in range(3)]
            if any(self.face_bc[f] != BC_HABC for f in faces):
                continue
            pos = np.array([self.hi[a] if bits[a] else self.lo[a] for a in range(3)])
            lines = []
            for a in range(3):
                found = None
                for l in np.nonzero(self.lin_axis == a)[0]:
                    A, B = DOMAIN_EDGES[self.lin_dedge[l]]
                    if set((A, B)) != set(f for f in faces if f // 2 != a):
                        continue
                    for end in range(2):
                        if np.linalg.norm(self.lin_xn[l, -1 if end else 0] - pos) < 1e3 * self.tol:
                            found = (l, end)
                if found is None:
                    raise ValueError("corner without line")
                lines.append(found)
            recs.append((c, lines, bits))
        self.Kpnt = len(recs)
        self.pnt_id = np.array([r[0] for r in recs], dtype=np.int64)
        self.pnt_line = np.array([[r[1][a][0] for a in range(3)] for r in recs],
                                 dtype=np.int64).reshape(-1, 3)
        self.pnt_end = np.array([[r[1][a][1] for a in range(3)] for r in recs],
                                dtype=np.int64).reshape(-1, 3)
        # outward normal along each slot's axis
        self.pnt_nrm = np.array([[1.0 if r[2][a] else -1.0 for a in range(3)] for r in recs]
                                ).reshape(-1, 3)
        # line end -> (corner, slot)
        self.lin_corner = np.full((self.Klin, 2), -1, dtype=np.int64)
        self.lin_corner_slot = np.full((self.Klin, 2), -1, dtype=np.int64)
        for p in range(self.Kpnt):
            for a in range(3):
                l, end = self.pnt_line[p, a], self.pnt_end[p, a]
                self.lin_corner[l, end] = p
                self.lin_corner_slot[l, end] = a
        # remaining open line ends: the third face is not HABC
        self.lin_bc = np.full((self.Klin, 2), "", dtype=object)
        for l in range(self.Klin):
            for end in range(2):
                if self.lin_EToE[l, end] >= 0 or self.lin_corner[l, end] >= 0:
                    continue
                x = self.lin_xn[l, -1 if end else 0]
                a = self.lin_axis[l]
                side = 1 if abs(x[a] - self.hi[a]) < 1e3 * self.tol else 0
                self.lin_bc[l, end] = self.face_bc[2 * a + side]
