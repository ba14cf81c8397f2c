// Reference elements: nodes, modal bases, Vandermonde-based operators.
// See refelem.hpp for the node-order convention.
#include "refelem.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace dgh {

const int kFaceVerts[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {0, 2, 3}};
const int kTriEdgeVerts[3][2] = {{0, 1}, {1, 2}, {0, 2}};
static const int kFaceOpp[4] = {3, 2, 0, 1};
static const double kRefV[4][3] = {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};

// Optimised Warp & Blend parameters for the tetrahedron (Warburton 2006).
static const double kAlphaTet[15] = {0.0, 0.0, 0.0, 0.1002, 1.1332, 1.5608, 1.3413, 1.2577,
                                     1.1603, 1.10153, 0.6080, 0.4523, 0.8856, 0.8717, 0.9655};

// Orthonormal Jacobi polynomial: P_0 = 1/sqrt(h0), h0 the weight integral;
// three-term recurrence x P_n = a_{n+1} P_{n+1} + b_n P_n + a_n P_{n-1}.
double jacobi_p(double x, double a, double b, int n) {
  const double h0 = std::pow(2.0, a + b + 1) * std::tgamma(a + 1) * std::tgamma(b + 1) /
                    std::tgamma(a + b + 2);
  double pm = 1.0 / std::sqrt(h0);
  if (n == 0) return pm;
  const double h1 = (a + 1) * (b + 1) / (a + b + 3) * h0;
  double p = ((a + b + 2) * x / 2 + (a - b) / 2) / std::sqrt(h1);
  auto acoef = [&](int k) {  // a_k, k >= 1
    const double s = 2.0 * k + a + b;
    return 2.0 / s * std::sqrt(k * (k + a + b) * (k + a) * (k + b) / ((s - 1) * (s + 1)));
  };
  for (int k = 1; k < n; ++k) {
    const double s = 2.0 * k + a + b;
    const double bk = -(a * a - b * b) / (s * (s + 2));
    const double pn = ((x - bk) * p - acoef(k) * pm) / acoef(k + 1);
    pm = p;
    p = pn;
  }
  return p;
}

double grad_jacobi_p(double x, double a, double b, int n) {
  if (n == 0) return 0.0;
  return std::sqrt(n * (n + a + b + 1)) * jacobi_p(x, a + 1, b + 1, n - 1);
}

// GLL points: -1, the roots of P_{N-1}^{(1,1)} (Newton from Chebyshev-Lobatto
// guesses), +1; ascending.
std::vector<double> gll_points(int N) {
  std::vector<double> x(N + 1);
  x[0] = -1.0;
  x[N] = 1.0;
  for (int k = 1; k < N; ++k) {
    double z = -std::cos(M_PI * k / N);
    for (int it = 0; it < 100; ++it) {
      const double f = jacobi_p(z, 1, 1, N - 1);
      const double df = grad_jacobi_p(z, 1, 1, N - 1);
      const double dz = f / df;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    x[k] = z;
  }
  std::sort(x.begin(), x.end());
  return x;
}

// 1D warp of equispaced points toward GLL points divided by (1 - x^2).
static double warp_over(int N, const std::vector<double>& xg, double x) {
  std::vector<double> xe(N + 1);
  for (int i = 0; i <= N; ++i) xe[i] = -1.0 + 2.0 * i / N;
  double sum = 0.0;
  for (int i = 1; i < N; ++i) {
    // Lagrange polynomial of the equispaced node i divided by (x+1)(x-1)
    double term = (xg[i] - xe[i]) / ((xe[i] + 1.0) * (xe[i] - 1.0));
    for (int j = 1; j < N; ++j)
      if (j != i) term *= (x - xe[j]) / (xe[i] - xe[j]);
    sum += term;
  }
  return -sum;  // (x+1)(x-1) = -(1 - x^2)
}

static void tet_nodes(int N, std::vector<int>& lat, std::vector<double>& r,
                      std::vector<double>& s, std::vector<double>& t) {
  lat.clear();
  for (int k = 0; k <= N; ++k)
    for (int j = 0; j <= N - k; ++j)
      for (int i = 0; i <= N - k - j; ++i) {
        lat.push_back(i);
        lat.push_back(j);
        lat.push_back(k);
      }
  const int Np = (int)lat.size() / 3;
  const double alpha = N <= 15 ? kAlphaTet[N - 1] : 1.0;
  const std::vector<double> xg = gll_points(N);
  r.assign(Np, 0);
  s.assign(Np, 0);
  t.assign(Np, 0);
  for (int n = 0; n < Np; ++n) {
    const int li = lat[3 * n], lj = lat[3 * n + 1], lk = lat[3 * n + 2];
    const int ints[4] = {N - li - lj - lk, li, lj, lk};
    double lam[4];
    for (int v = 0; v < 4; ++v) lam[v] = (double)ints[v] / N;
    double X[3] = {0, 0, 0};
    for (int v = 0; v < 4; ++v)
      for (int d = 0; d < 3; ++d) X[d] += lam[v] * kRefV[v][d];
    int nzero = 0;
    for (int v = 0; v < 4; ++v) nzero += ints[v] == 0;
    double sh[3] = {0, 0, 0};
    if (nzero >= 2) {
      // edge node: pure 1D warp between its two nonzero vertices; vertex: none
      int vv[4], m = 0;
      for (int v = 0; v < 4; ++v)
        if (ints[v] != 0) vv[m++] = v;
      if (m == 2) {
        const int p = vv[0], q = vv[1];
        const double w = 4.0 * lam[p] * lam[q] * warp_over(N, xg, lam[q] - lam[p]);
        for (int d = 0; d < 3; ++d) sh[d] = 0.5 * w * (kRefV[q][d] - kRefV[p][d]);
      }
    } else {
      for (int f = 0; f < 4; ++f) {
        const int a = kFaceVerts[f][0], b = kFaceVerts[f][1], c = kFaceVerts[f][2];
        const double la = lam[kFaceOpp[f]];
        const double prod = lam[a] * lam[b] * lam[c];
        const double den = (lam[a] + 0.5 * la) * (lam[b] + 0.5 * la) * (lam[c] + 0.5 * la);
        if (prod == 0.0) continue;
        const double blend = (1.0 + (alpha * la) * (alpha * la)) * prod / den;
        const int edges[3][3] = {{a, b, c}, {b, c, a}, {c, a, b}};
        for (int e = 0; e < 3; ++e) {
          const int p = edges[e][0], q = edges[e][1], o = edges[e][2];
          const double w = 4.0 * lam[p] * lam[q] * warp_over(N, xg, lam[q] - lam[p]) *
                           (1.0 + (alpha * lam[o]) * (alpha * lam[o]));
          for (int d = 0; d < 3; ++d) sh[d] += blend * 0.5 * w * (kRefV[q][d] - kRefV[p][d]);
        }
      }
    }
    r[n] = X[0] + sh[0];
    s[n] = X[1] + sh[1];
    t[n] = X[2] + sh[2];
  }
}

// psi_ijk and its (r, s, t) derivatives at one point, all modes (i, j, k)
// ordered i slowest, k fastest.
static void tet_modes_at(int N, double r, double s, double t, double* V, double* Vr, double* Vs,
                         double* Vt) {
  double a = -1.0, b = -1.0;
  if (std::fabs(s + t) > 1e-14) a = 2.0 * (1.0 + r) / (-s - t) - 1.0;
  if (std::fabs(t - 1.0) > 1e-14) b = 2.0 * (1.0 + s) / (1.0 - t) - 1.0;
  const double c = t;
  const double C = 2.0 * std::sqrt(2.0);
  int m = 0;
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= N - i; ++j)
      for (int k = 0; k <= N - i - j; ++k, ++m) {
        const double fa = jacobi_p(a, 0, 0, i), dfa = grad_jacobi_p(a, 0, 0, i);
        const double gb = jacobi_p(b, 2 * i + 1, 0, j), dgb = grad_jacobi_p(b, 2 * i + 1, 0, j);
        const double hc = jacobi_p(c, 2 * i + 2 * j + 2, 0, k);
        const double dhc = grad_jacobi_p(c, 2 * i + 2 * j + 2, 0, k);
        const double ob = 1.0 - b, oc = 1.0 - c;
        auto pw = [](double x, int e) { return e <= 0 ? 1.0 : std::pow(x, e); };
        if (V) V[m] = C * fa * gb * pw(ob, i) * hc * pw(oc, i + j);
        if (!Vr) continue;
        // reduced powers remove the 1/(1-b), 1/(1-c) of the chain rule
        double dr = 0.0;
        if (i > 0) dr = 4.0 * dfa * gb * pw(ob, i - 1) * hc * pw(oc, i + j - 1);
        double fbp = dgb * pw(ob, i) - (i > 0 ? i * gb * pw(ob, i - 1) : 0.0);
        double tmp = fa * fbp * hc * pw(oc, i + j - 1);
        if (i + j == 0) tmp = 0.0;  // fbp = 0 then
        const double ds = 0.5 * (1.0 + a) * dr + 2.0 * tmp;
        double fcp = dhc * pw(oc, i + j) - (i + j > 0 ? (i + j) * hc * pw(oc, i + j - 1) : 0.0);
        const double dt = 0.5 * (1.0 + a) * dr + (1.0 + b) * tmp + fa * gb * pw(ob, i) * fcp;
        Vr[m] = C * dr;
        Vs[m] = C * ds;
        Vt[m] = C * dt;
      }
}

static void tri_modes_at(int N, double r, double s, double* V, double* Vr, double* Vs) {
  double a = -1.0;
  if (std::fabs(s - 1.0) > 1e-14) a = 2.0 * (1.0 + r) / (1.0 - s) - 1.0;
  const double b = s;
  const double C = std::sqrt(2.0);
  int m = 0;
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= N - i; ++j, ++m) {
      const double fa = jacobi_p(a, 0, 0, i), dfa = grad_jacobi_p(a, 0, 0, i);
      const double gb = jacobi_p(b, 2 * i + 1, 0, j), dgb = grad_jacobi_p(b, 2 * i + 1, 0, j);
      const double ob = 1.0 - b;
      auto pw = [](double x, int e) { return e <= 0 ? 1.0 : std::pow(x, e); };
      if (V) V[m] = C * fa * gb * pw(ob, i);
      if (!Vr) continue;
      const double dr = i > 0 ? 2.0 * dfa * gb * pw(ob, i - 1) : 0.0;
      const double fbp = dgb * pw(ob, i) - (i > 0 ? i * gb * pw(ob, i - 1) : 0.0);
      Vr[m] = C * dr;
      Vs[m] = C * (0.5 * (1.0 + a) * dr + fa * fbp);
    }
}

void tet_basis_at(int N, double r, double s, double t, double* psi) {
  tet_modes_at(N, r, s, t, psi, nullptr, nullptr, nullptr);
}

bool invert(Mat& A, int n) {
  std::vector<int> piv(n);
  Mat I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int col = 0; col < n; ++col) {
    int best = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(A[r * n + col]) > std::fabs(A[best * n + col])) best = r;
    if (A[best * n + col] == 0.0) return false;
    if (best != col)
      for (int k = 0; k < n; ++k) {
        std::swap(A[best * n + k], A[col * n + k]);
        std::swap(I[best * n + k], I[col * n + k]);
      }
    const double d = 1.0 / A[col * n + col];
    for (int k = 0; k < n; ++k) {
      A[col * n + k] *= d;
      I[col * n + k] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double f = A[r * n + col];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        A[r * n + k] -= f * A[col * n + k];
        I[r * n + k] -= f * I[col * n + k];
      }
    }
  }
  A = I;
  return true;
}

Mat matmul(const Mat& A, const Mat& B, int m, int k, int n) {
  Mat C(m * n, 0.0);
  for (int i = 0; i < m; ++i)
    for (int l = 0; l < k; ++l) {
      const double a = A[i * k + l];
      for (int j = 0; j < n; ++j) C[i * n + j] += a * B[l * n + j];
    }
  return C;
}

static Mat transpose(const Mat& A, int m, int n) {
  Mat T(m * n);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) T[j * m + i] = A[i * n + j];
  return T;
}

void build_tet(int N, RefTet& T) {
  if (N < 1) throw std::invalid_argument("N < 1");
  T.N = N;
  tet_nodes(N, T.lat, T.r, T.s, T.t);
  const int Np = T.Np = (int)T.r.size();
  T.Nfp = (N + 1) * (N + 2) / 2;
  Mat V(Np * Np), Vr(Np * Np), Vs(Np * Np), Vt(Np * Np);
  for (int n = 0; n < Np; ++n)
    tet_modes_at(N, T.r[n], T.s[n], T.t[n], &V[n * Np], &Vr[n * Np], &Vs[n * Np], &Vt[n * Np]);
  T.V = V;
  Mat Vi = V;
  if (!invert(Vi, Np)) throw std::runtime_error("singular tet Vandermonde");
  T.Dr = matmul(Vr, Vi, Np, Np, Np);
  T.Ds = matmul(Vs, Vi, Np, Np, Np);
  T.Dt = matmul(Vt, Vi, Np, Np, Np);
  Mat VVt = matmul(V, transpose(V, Np, Np), Np, Np, Np);
  T.Mass = VVt;
  invert(T.Mass, Np);
  // faces: k = 0, j = 0, i + j + k = N, i = 0
  T.Fmask.clear();
  for (int f = 0; f < 4; ++f)
    for (int n = 0; n < Np; ++n) {
      const int i = T.lat[3 * n], j = T.lat[3 * n + 1], k = T.lat[3 * n + 2];
      const bool on = f == 0 ? k == 0 : f == 1 ? j == 0 : f == 2 ? (i + j + k == N) : i == 0;
      if (on) T.Fmask.push_back(n);
    }
  const int Nfp = T.Nfp;
  // E: face mass matrices in each face's own two coordinates; LIFT = V V^T E
  Mat E(Np * 4 * Nfp, 0.0);
  for (int f = 0; f < 4; ++f) {
    Mat V2(Nfp * Nfp);
    for (int a = 0; a < Nfp; ++a) {
      const int n = T.Fmask[f * Nfp + a];
      double u, v;
      if (f == 0) { u = T.r[n]; v = T.s[n]; }
      else if (f == 1) { u = T.r[n]; v = T.t[n]; }
      else { u = T.s[n]; v = T.t[n]; }
      tri_modes_at(N, u, v, &V2[a * Nfp], nullptr, nullptr);
    }
    Mat Mf = matmul(V2, transpose(V2, Nfp, Nfp), Nfp, Nfp, Nfp);
    invert(Mf, Nfp);
    for (int a = 0; a < Nfp; ++a)
      for (int b = 0; b < Nfp; ++b)
        E[T.Fmask[f * Nfp + a] * 4 * Nfp + f * Nfp + b] = Mf[a * Nfp + b];
  }
  T.LIFT = matmul(VVt, E, Np, Np, 4 * Nfp);
}

void build_tri(const RefTet& T, RefTri& R) {
  const int N = T.N;
  R.N = N;
  R.Np = T.Nfp;
  R.Nfp = N + 1;
  const int Np = R.Np, Nfp = R.Nfp;
  R.r.resize(Np);
  R.s.resize(Np);
  std::vector<int> li(Np), lj(Np);
  for (int a = 0; a < Np; ++a) {  // face-0 nodes are the first Np tet nodes
    R.r[a] = T.r[a];
    R.s[a] = T.s[a];
    li[a] = T.lat[3 * a];
    lj[a] = T.lat[3 * a + 1];
  }
  Mat V(Np * Np), Vr(Np * Np), Vs(Np * Np);
  for (int a = 0; a < Np; ++a) tri_modes_at(N, R.r[a], R.s[a], &V[a * Np], &Vr[a * Np], &Vs[a * Np]);
  Mat Vi = V;
  if (!invert(Vi, Np)) throw std::runtime_error("singular tri Vandermonde");
  R.Dr = matmul(Vr, Vi, Np, Np, Np);
  R.Ds = matmul(Vs, Vi, Np, Np, Np);
  R.Fmask.clear();
  for (int f = 0; f < 3; ++f)
    for (int a = 0; a < Np; ++a) {
      const bool on = f == 0 ? lj[a] == 0 : f == 1 ? (li[a] + lj[a] == N) : li[a] == 0;
      if (on) R.Fmask.push_back(a);
    }
  Mat E(Np * 3 * Nfp, 0.0);
  for (int f = 0; f < 3; ++f) {
    Mat V1(Nfp * Nfp);
    for (int a = 0; a < Nfp; ++a) {
      const int n = R.Fmask[f * Nfp + a];
      const double x = f == 0 ? R.r[n] : R.s[n];
      for (int m = 0; m < Nfp; ++m) V1[a * Nfp + m] = jacobi_p(x, 0, 0, m);
    }
    Mat Mf = matmul(V1, transpose(V1, Nfp, Nfp), Nfp, Nfp, Nfp);
    invert(Mf, Nfp);
    for (int a = 0; a < Nfp; ++a)
      for (int b = 0; b < Nfp; ++b) E[R.Fmask[f * Nfp + a] * 3 * Nfp + f * Nfp + b] = Mf[a * Nfp + b];
  }
  Mat VVt = matmul(V, transpose(V, Np, Np), Np, Np, Np);
  R.LIFT = matmul(VVt, E, Np, Np, 3 * Nfp);
}

void build_line(int N, RefLine& L) {
  L.N = N;
  L.Np = N + 1;
  const int Np = L.Np;
  L.r = gll_points(N);
  Mat V(Np * Np), Vr(Np * Np);
  for (int a = 0; a < Np; ++a)
    for (int m = 0; m < Np; ++m) {
      V[a * Np + m] = jacobi_p(L.r[a], 0, 0, m);
      Vr[a * Np + m] = grad_jacobi_p(L.r[a], 0, 0, m);
    }
  Mat Vi = V;
  invert(Vi, Np);
  L.Dr = matmul(Vr, Vi, Np, Np, Np);
  Mat VVt = matmul(V, transpose(V, Np, Np), Np, Np, Np);
  L.LIFT.assign(Np * 2, 0.0);
  for (int a = 0; a < Np; ++a) {
    L.LIFT[a * 2 + 0] = VVt[a * Np + 0];
    L.LIFT[a * 2 + 1] = VVt[a * Np + Np - 1];
  }
}

}  // namespace dgh
