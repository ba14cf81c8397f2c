// Volume, surface and line meshes of a cuboid and the corners (Section 3.2):
// affine geometric factors and the four-level connectivity.
//
// Canonical orderings (part of the state layout of the C ABI):
//   domain faces  0..5 = x-, x+, y-, y+, z-, z+
//   triangles     HABC tet faces sorted by (domain face, tet, local face);
//                 vertices sorted by global id -> reference (-1,-1), (1,-1),
//                 (-1,1); in-plane axes = the two tangential axes, ascending
//   domain edges  face pairs (A, B), A < B on different axes, lexicographic
//   lines         sorted by (domain edge, low vertex id, high vertex id);
//                 node 0 at the low vertex id; velocity = +axis component
//   corners       c = xb + 2 yb + 4 zb; slot a = the line along axis a
#pragma once
#include <array>
#include <string>
#include <vector>

#include "refelem.hpp"

namespace dgh {

enum BcType { BC_HABC = 0, BC_ABC = 1, BC_DIRICHLET = 2, BC_PERIODIC = 3 };

struct Mesh {
  // inputs
  int K = 0, Nv = 0, N = 0;
  std::vector<double> VX;              // Nv x 3
  std::vector<int> EToV;               // K x 4
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  int periodic[3] = {0, 0, 0};
  int face_bc[6] = {0, 0, 0, 0, 0, 0};

  RefTet tet;
  RefTri tri;
  RefLine line;

  // 3D geometry (per element): metric terms rx..tz (9), J
  std::vector<double> geo;             // K x 9
  std::vector<double> J;
  // 3D connectivity
  std::vector<int> EToE, EToF, perm;   // K x 4 (perm: 0..5 face vertex permutation)
  std::vector<int> bface;              // K x 4 domain face of boundary faces, -1 interior
  std::vector<int> nbr_node;           // K x 4 x Nfp neighbour node (host check / tests)
  // face-node maps for each (face f, neighbour face f', permutation p): Nfp ints
  std::vector<int> fmap;               // 4*4*6*Nfp: node index (0..Np-1) in the neighbour

  // 2D
  int Ktri = 0;
  std::vector<int> tri_elem, tri_face, tri_dface, tri_verts;   // verts Ktri x 3
  std::vector<int> tri_axes;                                    // Ktri x 2
  std::vector<double> tri_geo;                                  // Ktri x 4: rx ry sx sy
  std::vector<int> tri_tetnode;                                 // Ktri x Np2
  std::vector<int> face_tri;                                    // K x 4 -> tri or -1
  std::vector<int> facenode_trinode;                            // Ktri x Nfp
  std::vector<int> tri_EToE, tri_nbr_node;                      // Ktri x 3, Ktri x 3 x Nfp2
  std::vector<int> tri_bdface;                                  // Ktri x 3 other domain face
  std::vector<int> tri_edge_line, tri_edge_side, tri_edge_linenode;  // Ktri x 3 (x Nfp2)

  // 1D
  int Klin = 0;
  std::vector<int> lin_dedge, lin_verts, lin_axis;             // verts Klin x 2
  std::vector<double> lin_rx;                                   // dr/dx along the axis
  std::vector<int> lin_tri, lin_tri_edge, lin_trinode;          // Klin x 2 (x Np1)
  std::vector<int> lin_EToE, lin_EToF;                          // Klin x 2
  std::vector<int> lin_corner, lin_corner_slot;                 // Klin x 2
  std::vector<int> lin_endbc;                                   // Klin x 2: BC of open ends

  // 0D
  int Kpnt = 0;
  std::vector<int> pnt_id, pnt_line, pnt_end;                   // Kpnt, Kpnt x 3
  std::vector<double> pnt_nrm;                                  // Kpnt x 3

  // node coordinates
  void node_xyz(int e, int n, double* x) const;
  void tri_node_xyz(int t, int a, double* x) const;
  void line_node_xyz(int l, int a, double* x) const;
};

extern const int kDomainEdges[12][2];

// Builds everything from VX/EToV/box/periodic/face_bc and the degree N.
// Returns an empty string on success, else the reason.
std::string build_mesh(Mesh& m);

}  // namespace dgh
