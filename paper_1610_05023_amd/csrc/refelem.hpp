// Reference elements of the nodal DG scheme (tetrahedron, triangle, line).
//
// Section 3.2 of the paper: Warp & Blend nodes on the tetrahedron; the
// triangle and line nodes are the tetrahedron's face and edge nodes.  Modal
// bases are orthonormal (Jacobi / collapsed-coordinate); differentiation and
// lifting matrices come from the Vandermonde matrices.
//
// Node order: lattice points (i, j, k), i + j + k <= N, k slowest, i fastest,
// barycentric coordinates (N-i-j-k, i, j, k)/N for the reference vertices
// (-1,-1,-1), (1,-1,-1), (-1,1,-1), (-1,-1,1).  Triangle nodes are the
// tetrahedron nodes with k = 0 (same order); line nodes are GLL points,
// ascending.  All matrices are dense, row-major, FP64.
#pragma once
#include <vector>

namespace dgh {

using Mat = std::vector<double>;  // row-major

struct RefTet {
  int N = 0, Np = 0, Nfp = 0;
  std::vector<int> lat;              // Np x 3 lattice indices (i, j, k)
  std::vector<double> r, s, t;       // nodes
  Mat V, Dr, Ds, Dt, Mass, LIFT;     // Np x Np, LIFT Np x 4Nfp
  std::vector<int> Fmask;            // 4 x Nfp, ascending node index per face
};

struct RefTri {
  int N = 0, Np = 0, Nfp = 0;
  std::vector<double> r, s;
  Mat Dr, Ds, LIFT;                  // LIFT Np x 3Nfp
  std::vector<int> Fmask;            // 3 x Nfp
};

struct RefLine {
  int N = 0, Np = 0;
  std::vector<double> r;
  Mat Dr, LIFT;                      // LIFT Np x 2
};

// Face vertex lists of the reference tetrahedron and triangle.
extern const int kFaceVerts[4][3];
extern const int kTriEdgeVerts[3][2];

double jacobi_p(double x, double alpha, double beta, int n);
double grad_jacobi_p(double x, double alpha, double beta, int n);
std::vector<double> gll_points(int N);

void build_tet(int N, RefTet& T);
void build_tri(const RefTet& T, RefTri& R);
void build_line(int N, RefLine& L);

// Orthonormal tetrahedron basis evaluated at (r, s, t): psi (Np values).
void tet_basis_at(int N, double r, double s, double t, double* psi);

bool invert(Mat& A, int n);          // in place, partial pivoting; false if singular
Mat matmul(const Mat& A, const Mat& B, int m, int k, int n);

}  // namespace dgh
