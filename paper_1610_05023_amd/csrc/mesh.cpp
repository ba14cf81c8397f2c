// Affine geometry and four-level connectivity (see mesh.hpp).
#include "mesh.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>

namespace dgh {

const int kDomainEdges[12][2] = {{0, 2}, {0, 3}, {0, 4}, {0, 5}, {1, 2}, {1, 3},
                                 {1, 4}, {1, 5}, {2, 4}, {2, 5}, {3, 4}, {3, 5}};

static const int kPerms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
static const int kFaceOppV[4] = {3, 2, 0, 1};

void Mesh::node_xyz(int e, int n, double* x) const {
  const int* v = &EToV[4 * e];
  const double r = tet.r[n], s = tet.s[n], t = tet.t[n];
  const double w[4] = {-(1 + r + s + t) / 2, (1 + r) / 2, (1 + s) / 2, (1 + t) / 2};
  for (int d = 0; d < 3; ++d) {
    const double x0 = VX[3 * v[0] + d];
    x[d] = x0 + w[1] * (VX[3 * v[1] + d] - x0) + w[2] * (VX[3 * v[2] + d] - x0) +
           w[3] * (VX[3 * v[3] + d] - x0);
  }
}

void Mesh::tri_node_xyz(int t, int a, double* x) const {
  const int* v = &tri_verts[3 * t];
  const double r = tri.r[a], s = tri.s[a];
  for (int d = 0; d < 3; ++d) {
    const double x0 = VX[3 * v[0] + d];
    x[d] = x0 + 0.5 * (r + 1) * (VX[3 * v[1] + d] - x0) + 0.5 * (s + 1) * (VX[3 * v[2] + d] - x0);
  }
}

void Mesh::line_node_xyz(int l, int a, double* x) const {
  const int* v = &lin_verts[2 * l];
  for (int d = 0; d < 3; ++d) {
    const double x0 = VX[3 * v[0] + d];
    x[d] = x0 + 0.5 * (line.r[a] + 1) * (VX[3 * v[1] + d] - x0);
  }
}

namespace {

struct Ctx {
  Mesh& m;
  double tol;
  double len[3];
  std::vector<int> canon;  // periodic vertex identification
  explicit Ctx(Mesh& mm) : m(mm) {}
  double dist(const double* a, const double* b) const {
    double s = 0;
    for (int d = 0; d < 3; ++d) {
      double x = a[d] - b[d];
      if (m.periodic[d]) x -= len[d] * std::round(x / len[d]);
      s += x * x;
    }
    return std::sqrt(s);
  }
};

int lattice_node(const RefTet& T, const int ints[4]) {
  // node with barycentric ints (N-i-j-k, i, j, k)
  for (int n = 0; n < T.Np; ++n)
    if (T.lat[3 * n] == ints[1] && T.lat[3 * n + 1] == ints[2] && T.lat[3 * n + 2] == ints[3])
      return n;
  return -1;
}

}  // namespace

std::string build_mesh(Mesh& m) {
  if (m.N < 1 || m.N > 8) return "polynomial degree out of range";
  if (m.K <= 0 || m.Nv <= 0) return "empty mesh";
  build_tet(m.N, m.tet);
  build_tri(m.tet, m.tri);
  build_line(m.N, m.line);
  const RefTet& T = m.tet;
  const int K = m.K, Np = T.Np, Nfp = T.Nfp;
  Ctx c(m);
  for (int d = 0; d < 3; ++d) c.len[d] = m.hi[d] - m.lo[d];
  for (int d = 0; d < 3; ++d)
    if (m.periodic[d]) m.face_bc[2 * d] = m.face_bc[2 * d + 1] = BC_PERIODIC;
  for (int e = 0; e < K; ++e)
    for (int k = 0; k < 4; ++k)
      if (m.EToV[4 * e + k] < 0 || m.EToV[4 * e + k] >= m.Nv) return "vertex index out of range";

  // ---- geometry
  m.geo.assign(9 * K, 0.0);
  m.J.assign(K, 0.0);
  double hmin = 1e300;
  for (int e = 0; e < K; ++e) {
    const int* v = &m.EToV[4 * e];
    double A[3][3];  // columns x_r, x_s, x_t
    for (int d = 0; d < 3; ++d)
      for (int k = 0; k < 3; ++k) A[d][k] = 0.5 * (m.VX[3 * v[k + 1] + d] - m.VX[3 * v[0] + d]);
    const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                       A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                       A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    if (!(det > 0)) return "element " + std::to_string(e) + " is not positively oriented";
    m.J[e] = det;
    // inverse: rows grad r, grad s, grad t
    double I[3][3];
    I[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
    I[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
    I[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
    I[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
    I[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
    I[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
    I[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
    I[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
    I[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) m.geo[9 * e + 3 * i + j] = I[i][j];
    double ed = 0;
    for (int d = 0; d < 3; ++d) ed += 4 * A[d][0] * A[d][0];
    hmin = std::min(hmin, std::sqrt(ed));
  }
  c.tol = 1e-7 * hmin;
  const double mtol = 1e3 * c.tol;

  // ---- periodic vertex identification (canonical vertex ids)
  c.canon.resize(m.Nv);
  {
    std::map<std::tuple<long long, long long, long long>, int> seen;
    for (int v = 0; v < m.Nv; ++v) {
      double key[3];
      for (int d = 0; d < 3; ++d) {
        key[d] = m.VX[3 * v + d];
        if (m.periodic[d] && std::fabs(key[d] - m.hi[d]) < c.tol) key[d] = m.lo[d];
      }
      auto k = std::make_tuple(std::llround((key[0] - m.lo[0]) / c.tol),
                               std::llround((key[1] - m.lo[1]) / c.tol),
                               std::llround((key[2] - m.lo[2]) / c.tol));
      auto it = seen.find(k);
      if (it == seen.end()) {
        seen[k] = v;
        c.canon[v] = v;
      } else {
        c.canon[v] = it->second;
      }
    }
  }

  // ---- face-node maps for every (f, f', permutation)
  m.fmap.assign(4 * 4 * 6 * Nfp, -1);
  for (int f = 0; f < 4; ++f)
    for (int f2 = 0; f2 < 4; ++f2)
      for (int p = 0; p < 6; ++p)
        for (int i = 0; i < Nfp; ++i) {
          const int n = T.Fmask[f * Nfp + i];
          const int own[4] = {T.N - T.lat[3 * n] - T.lat[3 * n + 1] - T.lat[3 * n + 2],
                              T.lat[3 * n], T.lat[3 * n + 1], T.lat[3 * n + 2]};
          int nb[4] = {0, 0, 0, 0};
          // our face vertex k is the neighbour's face vertex kPerms[p][k]
          for (int k = 0; k < 3; ++k) nb[kFaceVerts[f2][kPerms[p][k]]] = own[kFaceVerts[f][k]];
          nb[kFaceOppV[f2]] = 0;
          m.fmap[((f * 4 + f2) * 6 + p) * Nfp + i] = lattice_node(T, nb);
        }

  // ---- 3D face matching
  m.EToE.assign(4 * K, -1);
  m.EToF.assign(4 * K, -1);
  m.perm.assign(4 * K, 0);
  m.bface.assign(4 * K, -1);
  {
    std::vector<std::tuple<int, int, int, int>> keys;  // sorted canon ids, e*4+f
    keys.reserve(4 * K);
    for (int e = 0; e < K; ++e)
      for (int f = 0; f < 4; ++f) {
        int a[3];
        for (int k = 0; k < 3; ++k) a[k] = c.canon[m.EToV[4 * e + kFaceVerts[f][k]]];
        std::sort(a, a + 3);
        keys.emplace_back(a[0], a[1], a[2], 4 * e + f);
      }
    std::sort(keys.begin(), keys.end());
    for (size_t i = 0; i < keys.size();) {
      size_t j = i + 1;
      while (j < keys.size() && std::get<0>(keys[j]) == std::get<0>(keys[i]) &&
             std::get<1>(keys[j]) == std::get<1>(keys[i]) &&
             std::get<2>(keys[j]) == std::get<2>(keys[i]))
        ++j;
      if (j - i > 2) return "non-manifold face";
      if (j - i == 2) {
        const int x = std::get<3>(keys[i]), y = std::get<3>(keys[i + 1]);
        m.EToE[x] = y / 4;
        m.EToF[x] = y % 4;
        m.EToE[y] = x / 4;
        m.EToF[y] = x % 4;
      }
      i = j;
    }
  }
  m.nbr_node.assign(4 * K * Nfp, -1);
  for (int e = 0; e < K; ++e)
    for (int f = 0; f < 4; ++f) {
      const int e2 = m.EToE[4 * e + f];
      if (e2 < 0) continue;
      const int f2 = m.EToF[4 * e + f];
      int a[3], b[3];
      for (int k = 0; k < 3; ++k) {
        a[k] = c.canon[m.EToV[4 * e + kFaceVerts[f][k]]];
        b[k] = c.canon[m.EToV[4 * e2 + kFaceVerts[f2][k]]];
      }
      int p = -1;
      for (int q = 0; q < 6 && p < 0; ++q)
        if (a[0] == b[kPerms[q][0]] && a[1] == b[kPerms[q][1]] && a[2] == b[kPerms[q][2]]) p = q;
      if (p < 0) return "face permutation not found";
      m.perm[4 * e + f] = p;
      for (int i = 0; i < Nfp; ++i) {
        const int n2 = m.fmap[((f * 4 + f2) * 6 + p) * Nfp + i];
        double x1[3], x2[3];
        m.node_xyz(e, T.Fmask[f * Nfp + i], x1);
        m.node_xyz(e2, n2, x2);
        if (c.dist(x1, x2) > mtol) return "face nodes do not coincide";
        m.nbr_node[(4 * e + f) * Nfp + i] = n2;
      }
    }
  // boundary faces -> domain face
  for (int e = 0; e < K; ++e)
    for (int f = 0; f < 4; ++f) {
      if (m.EToE[4 * e + f] >= 0) continue;
      double cen[3] = {0, 0, 0};
      for (int k = 0; k < 3; ++k)
        for (int d = 0; d < 3; ++d) cen[d] += m.VX[3 * m.EToV[4 * e + kFaceVerts[f][k]] + d] / 3;
      int df = -1;
      for (int d = 0; d < 3; ++d) {
        if (std::fabs(cen[d] - m.lo[d]) < mtol) df = 2 * d;
        if (std::fabs(cen[d] - m.hi[d]) < mtol) df = 2 * d + 1;
      }
      if (df < 0 || m.face_bc[df] == BC_PERIODIC) return "boundary face off the box";
      m.bface[4 * e + f] = df;
    }

  // ---- 2D: triangles on HABC faces
  {
    std::vector<std::tuple<int, int, int>> list;
    for (int e = 0; e < K; ++e)
      for (int f = 0; f < 4; ++f) {
        const int df = m.bface[4 * e + f];
        if (df >= 0 && m.face_bc[df] == BC_HABC) list.emplace_back(df, e, f);
      }
    std::sort(list.begin(), list.end());
    const int Kt = m.Ktri = (int)list.size();
    const int Np2 = m.tri.Np, Nfp2 = m.tri.Nfp;
    m.tri_elem.resize(Kt);
    m.tri_face.resize(Kt);
    m.tri_dface.resize(Kt);
    m.tri_verts.resize(3 * Kt);
    m.tri_axes.resize(2 * Kt);
    m.tri_geo.resize(4 * Kt);
    m.tri_tetnode.resize(Kt * Np2);
    m.face_tri.assign(4 * K, -1);
    m.facenode_trinode.resize(Kt * Nfp);
    for (int t = 0; t < Kt; ++t) {
      const int df = std::get<0>(list[t]), e = std::get<1>(list[t]), f = std::get<2>(list[t]);
      m.tri_dface[t] = df;
      m.tri_elem[t] = e;
      m.tri_face[t] = f;
      m.face_tri[4 * e + f] = t;
      int g[3];
      for (int k = 0; k < 3; ++k) g[k] = m.EToV[4 * e + kFaceVerts[f][k]];
      int sv[3] = {g[0], g[1], g[2]};
      std::sort(sv, sv + 3);
      for (int k = 0; k < 3; ++k) m.tri_verts[3 * t + k] = sv[k];
      const int ax = df / 2;
      int a0 = -1, a1 = -1;
      for (int d = 0; d < 3; ++d)
        if (d != ax) (a0 < 0 ? a0 : a1) = d;
      m.tri_axes[2 * t] = a0;
      m.tri_axes[2 * t + 1] = a1;
      const double ar = 0.5 * (m.VX[3 * sv[1] + a0] - m.VX[3 * sv[0] + a0]);
      const double as = 0.5 * (m.VX[3 * sv[2] + a0] - m.VX[3 * sv[0] + a0]);
      const double br = 0.5 * (m.VX[3 * sv[1] + a1] - m.VX[3 * sv[0] + a1]);
      const double bs = 0.5 * (m.VX[3 * sv[2] + a1] - m.VX[3 * sv[0] + a1]);
      const double Jt = ar * bs - as * br;
      if (Jt == 0.0) return "degenerate boundary triangle";
      m.tri_geo[4 * t + 0] = bs / Jt;    // rx (d r / d a0)
      m.tri_geo[4 * t + 1] = -as / Jt;   // ry (d r / d a1)
      m.tri_geo[4 * t + 2] = -br / Jt;   // sx
      m.tri_geo[4 * t + 3] = ar / Jt;    // sy
      // triangle node a <-> tet node: face vertex k is triangle vertex q[k]
      int q[3];
      for (int k = 0; k < 3; ++k) q[k] = (int)(std::find(sv, sv + 3, g[k]) - sv);
      for (int a = 0; a < Np2; ++a) {
        const int tri_ints[3] = {m.N - T.lat[3 * a] - T.lat[3 * a + 1], T.lat[3 * a],
                                 T.lat[3 * a + 1]};
        int ints[4] = {0, 0, 0, 0};
        for (int k = 0; k < 3; ++k) ints[kFaceVerts[f][k]] = tri_ints[q[k]];
        const int n = lattice_node(T, ints);
        double x1[3], x2[3];
        m.tri_node_xyz(t, a, x1);
        m.node_xyz(e, n, x2);
        if (c.dist(x1, x2) > mtol) return "triangle nodes do not match the tet face";
        m.tri_tetnode[t * Np2 + a] = n;
        for (int i = 0; i < Nfp; ++i)
          if (T.Fmask[f * Nfp + i] == n) m.facenode_trinode[t * Nfp + i] = a;
      }
    }
    // triangle neighbours within a domain face
    m.tri_EToE.assign(3 * Kt, -1);
    m.tri_nbr_node.assign(3 * Kt * Nfp2, -1);
    m.tri_bdface.assign(3 * Kt, -1);
    std::map<std::tuple<int, int, int>, std::vector<int>> ekeys;
    for (int t = 0; t < Kt; ++t)
      for (int f = 0; f < 3; ++f) {
        int a = c.canon[m.tri_verts[3 * t + kTriEdgeVerts[f][0]]];
        int b = c.canon[m.tri_verts[3 * t + kTriEdgeVerts[f][1]]];
        if (a > b) std::swap(a, b);
        ekeys[std::make_tuple(m.tri_dface[t], a, b)].push_back(3 * t + f);
      }
    for (auto& kv : ekeys) {
      auto& v = kv.second;
      if (v.size() > 2) return "non-manifold triangle edge";
      if (v.size() == 2) {
        for (int s = 0; s < 2; ++s) {
          const int x = v[s], y = v[1 - s];
          const int t = x / 3, f = x % 3, t2 = y / 3, f2 = y % 3;
          m.tri_EToE[x] = t2;
          for (int i = 0; i < Nfp2; ++i) {
            double x1[3];
            m.tri_node_xyz(t, m.tri.Fmask[f * Nfp2 + i], x1);
            int best = -1;
            for (int j = 0; j < Nfp2; ++j) {
              double x2[3];
              m.tri_node_xyz(t2, m.tri.Fmask[f2 * Nfp2 + j], x2);
              if (c.dist(x1, x2) < mtol) best = m.tri.Fmask[f2 * Nfp2 + j];
            }
            if (best < 0) return "triangle edge nodes do not match";
            m.tri_nbr_node[x * Nfp2 + i] = best;
          }
        }
      }
    }
    for (int t = 0; t < Kt; ++t)
      for (int f = 0; f < 3; ++f) {
        if (m.tri_EToE[3 * t + f] >= 0) continue;
        double cen[3];
        for (int d = 0; d < 3; ++d)
          cen[d] = 0.5 * (m.VX[3 * m.tri_verts[3 * t + kTriEdgeVerts[f][0]] + d] +
                          m.VX[3 * m.tri_verts[3 * t + kTriEdgeVerts[f][1]] + d]);
        int other = -1;
        for (int d = 0; d < 3; ++d) {
          if (d == m.tri_dface[t] / 2 || m.periodic[d]) continue;
          if (std::fabs(cen[d] - m.lo[d]) < mtol) other = 2 * d;
          if (std::fabs(cen[d] - m.hi[d]) < mtol) other = 2 * d + 1;
        }
        if (other < 0) return "triangle boundary edge not on a domain edge";
        m.tri_bdface[3 * t + f] = other;
      }
  }

  // ---- 1D: lines on edges between two HABC faces
  {
    const int Kt = m.Ktri, Nfp2 = m.tri.Nfp, Np1 = m.line.Np;
    std::map<std::tuple<int, int, int, int>, int> tri_edges;  // (face, other, lo, hi) -> 3t+f
    for (int t = 0; t < Kt; ++t)
      for (int f = 0; f < 3; ++f) {
        if (m.tri_bdface[3 * t + f] < 0) continue;
        int a = m.tri_verts[3 * t + kTriEdgeVerts[f][0]], b = m.tri_verts[3 * t + kTriEdgeVerts[f][1]];
        if (a > b) std::swap(a, b);
        tri_edges[std::make_tuple(m.tri_dface[t], m.tri_bdface[3 * t + f], a, b)] = 3 * t + f;
      }
    std::vector<std::tuple<int, int, int>> recs;
    for (int de = 0; de < 12; ++de) {
      const int A = kDomainEdges[de][0], B = kDomainEdges[de][1];
      if (m.face_bc[A] != BC_HABC || m.face_bc[B] != BC_HABC) continue;
      for (auto& kv : tri_edges)
        if (std::get<0>(kv.first) == A && std::get<1>(kv.first) == B)
          recs.emplace_back(de, std::get<2>(kv.first), std::get<3>(kv.first));
    }
    std::sort(recs.begin(), recs.end());
    const int Kl = m.Klin = (int)recs.size();
    m.lin_dedge.resize(Kl);
    m.lin_verts.resize(2 * Kl);
    m.lin_axis.resize(Kl);
    m.lin_rx.resize(Kl);
    m.lin_tri.resize(2 * Kl);
    m.lin_tri_edge.resize(2 * Kl);
    m.lin_trinode.resize(2 * Kl * Np1);
    m.tri_edge_line.assign(3 * Kt, -1);
    m.tri_edge_side.assign(3 * Kt, -1);
    m.tri_edge_linenode.assign(3 * Kt * Nfp2, -1);
    for (int l = 0; l < Kl; ++l) {
      const int de = std::get<0>(recs[l]);
      m.lin_dedge[l] = de;
      m.lin_verts[2 * l] = std::get<1>(recs[l]);
      m.lin_verts[2 * l + 1] = std::get<2>(recs[l]);
      const int A = kDomainEdges[de][0], B = kDomainEdges[de][1];
      const int ax = 3 - A / 2 - B / 2;
      m.lin_axis[l] = ax;
      const double dx = 0.5 * (m.VX[3 * m.lin_verts[2 * l + 1] + ax] - m.VX[3 * m.lin_verts[2 * l] + ax]);
      if (dx == 0.0) return "degenerate line";
      m.lin_rx[l] = 1.0 / dx;
      for (int side = 0; side < 2; ++side) {
        const int face = side == 0 ? A : B, other = side == 0 ? B : A;
        auto it = tri_edges.find(std::make_tuple(face, other, m.lin_verts[2 * l], m.lin_verts[2 * l + 1]));
        if (it == tri_edges.end()) return "line without adjacent triangle";
        const int t = it->second / 3, f = it->second % 3;
        m.lin_tri[2 * l + side] = t;
        m.lin_tri_edge[2 * l + side] = f;
        m.tri_edge_line[3 * t + f] = l;
        m.tri_edge_side[3 * t + f] = side;
        for (int a = 0; a < Np1; ++a) {
          double xl[3];
          m.line_node_xyz(l, a, xl);
          int found = -1, fi = -1;
          for (int i = 0; i < Nfp2; ++i) {
            double xt[3];
            m.tri_node_xyz(t, m.tri.Fmask[f * Nfp2 + i], xt);
            if (c.dist(xl, xt) < mtol) {
              found = m.tri.Fmask[f * Nfp2 + i];
              fi = i;
            }
          }
          if (found < 0) return "line nodes do not match triangle nodes";
          m.lin_trinode[(2 * l + side) * Np1 + a] = found;
          m.tri_edge_linenode[(3 * t + f) * Nfp2 + fi] = a;
        }
      }
    }
    // neighbours along the edge through the shared (canonical) vertex
    m.lin_EToE.assign(2 * Kl, -1);
    m.lin_EToF.assign(2 * Kl, -1);
    std::map<std::pair<int, int>, std::vector<int>> ends;
    for (int l = 0; l < Kl; ++l)
      for (int s = 0; s < 2; ++s) ends[{m.lin_dedge[l], c.canon[m.lin_verts[2 * l + s]]}].push_back(2 * l + s);
    for (auto& kv : ends) {
      if (kv.second.size() > 2) return "non-manifold line end";
      if (kv.second.size() == 2) {
        const int x = kv.second[0], y = kv.second[1];
        m.lin_EToE[x] = y / 2;
        m.lin_EToF[x] = y % 2;
        m.lin_EToE[y] = x / 2;
        m.lin_EToF[y] = x % 2;
      }
    }
  }

  // ---- 0D: corners of three HABC faces
  {
    const int Kl = m.Klin, Np1 = m.line.Np;
    m.pnt_id.clear();
    m.pnt_line.clear();
    m.pnt_end.clear();
    m.pnt_nrm.clear();
    m.lin_corner.assign(2 * Kl, -1);
    m.lin_corner_slot.assign(2 * Kl, -1);
    for (int cidx = 0; cidx < 8; ++cidx) {
      int bits[3], faces[3];
      for (int a = 0; a < 3; ++a) {
        bits[a] = (cidx >> a) & 1;
        faces[a] = 2 * a + bits[a];
      }
      if (m.face_bc[faces[0]] != BC_HABC || m.face_bc[faces[1]] != BC_HABC ||
          m.face_bc[faces[2]] != BC_HABC)
        continue;
      double pos[3];
      for (int a = 0; a < 3; ++a) pos[a] = bits[a] ? m.hi[a] : m.lo[a];
      int lines[3], endsl[3];
      for (int a = 0; a < 3; ++a) {
        lines[a] = -1;
        const int fA = faces[(a + 1) % 3], fB = faces[(a + 2) % 3];
        const int lo = std::min(fA, fB), hi = std::max(fA, fB);
        for (int l = 0; l < Kl; ++l) {
          const int de = m.lin_dedge[l];
          if (m.lin_axis[l] != a || kDomainEdges[de][0] != lo || kDomainEdges[de][1] != hi) continue;
          for (int end = 0; end < 2; ++end) {
            double x[3];
            m.line_node_xyz(l, end ? Np1 - 1 : 0, x);
            double d2 = 0;
            for (int d = 0; d < 3; ++d) d2 += (x[d] - pos[d]) * (x[d] - pos[d]);
            if (std::sqrt(d2) < mtol) {
              lines[a] = l;
              endsl[a] = end;
            }
          }
        }
        if (lines[a] < 0) return "corner without line";
      }
      const int p = (int)m.pnt_id.size();
      m.pnt_id.push_back(cidx);
      for (int a = 0; a < 3; ++a) {
        m.pnt_line.push_back(lines[a]);
        m.pnt_end.push_back(endsl[a]);
        m.pnt_nrm.push_back(bits[a] ? 1.0 : -1.0);
        m.lin_corner[2 * lines[a] + endsl[a]] = p;
        m.lin_corner_slot[2 * lines[a] + endsl[a]] = a;
      }
    }
    m.Kpnt = (int)m.pnt_id.size();
    m.lin_endbc.assign(2 * Kl, -1);
    for (int l = 0; l < Kl; ++l)
      for (int end = 0; end < 2; ++end) {
        if (m.lin_EToE[2 * l + end] >= 0 || m.lin_corner[2 * l + end] >= 0) continue;
        double x[3];
        m.line_node_xyz(l, end ? Np1 - 1 : 0, x);
        const int a = m.lin_axis[l];
        const int side = std::fabs(x[a] - m.hi[a]) < mtol ? 1 : 0;
        m.lin_endbc[2 * l + end] = m.face_bc[2 * a + side];
      }
  }
  return "";
}

}  // namespace dgh
