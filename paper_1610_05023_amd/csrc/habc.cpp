// HABC constants (see habc.hpp).
#include "habc.hpp"

#include <cmath>

#include "refelem.hpp"

namespace dgh {

bool build_habc(int P, const double* gin, HabcConsts& h) {
  h.P = P;
  const double M = 2.0 * P + 1.0;
  h.gamma.resize(P);
  for (int n = 0; n < P; ++n) {
    if (gin) {
      h.gamma[n] = gin[n];
    } else {
      const double tn = std::tan((n + 1) * M_PI / M);
      h.gamma[n] = tn * tn;
    }
    if (!(h.gamma[n] > 0.0)) return false;
  }
  const std::vector<double>& g = h.gamma;
  auto C = [&](int a, int b) { return (1.0 + g[a]) / (1.0 + g[a] + g[b]); };
  h.Cji.assign(P * P, 0.0);
  h.Cij.assign(P * P, 0.0);
  for (int i = 0; i < P; ++i)
    for (int j = 0; j < P; ++j) {
      h.Cji[i * P + j] = C(j, i);
      h.Cij[i * P + j] = C(i, j);
    }
  if (P == 0) {
    h.G.clear();
    h.H.clear();
    h.T.clear();
    return true;
  }
  // ---- edge: R from the equations for r-_{A,i} and r-_{B,j}
  const int n2 = 2 * P;
  Mat R(n2 * n2, 0.0);
  for (int i = 0; i < P; ++i)
    for (int j = 0; j < P; ++j) {
      R[i * n2 + i] += g[j] / M * (C(j, i) - 1.0);            // (C_ji - 1) S_A,i
      R[i * n2 + P + j] += g[j] / M * C(i, j);               // C_ij S_B,j
      R[(P + j) * n2 + i] += g[i] / M * C(j, i);             // C_ji S_A,i
      R[(P + j) * n2 + P + j] += g[i] / M * (C(i, j) - 1.0);  // (C_ij - 1) S_B,j
    }
  Mat L(n2 * n2, 0.0);
  for (int a = 0; a < n2 * n2; ++a) L[a] = -R[a];
  for (int a = 0; a < n2; ++a) L[a * n2 + a] += 1.0;
  if (!invert(L, n2)) return false;
  h.H = L;
  h.G = matmul(L, R, n2, n2, n2);
  // ---- corner
  const int PP = P * P, n3 = 3 * PP;
  Mat Rc(n3 * n3, 0.0);
  auto X = [&](int j, int k) { return j * P + k; };
  auto Y = [&](int i, int k) { return PP + i * P + k; };
  auto Z = [&](int i, int j) { return 2 * PP + i * P + j; };
  for (int i = 0; i < P; ++i)
    for (int j = 0; j < P; ++j)
      for (int k = 0; k < P; ++k) {
        const double D = 1.0 + g[i] + g[j] + g[k];
        const double ci = (1 + g[i]) / D, cj = (1 + g[j]) / D, ck = (1 + g[k]) / D;
        Rc[X(j, k) * n3 + X(j, k)] += g[i] / M * (ci - 1.0);
        Rc[X(j, k) * n3 + Y(i, k)] += g[i] / M * cj;
        Rc[X(j, k) * n3 + Z(i, j)] += g[i] / M * ck;
        Rc[Y(i, k) * n3 + X(j, k)] += g[j] / M * ci;
        Rc[Y(i, k) * n3 + Y(i, k)] += g[j] / M * (cj - 1.0);
        Rc[Y(i, k) * n3 + Z(i, j)] += g[j] / M * ck;
        Rc[Z(i, j) * n3 + X(j, k)] += g[k] / M * ci;
        Rc[Z(i, j) * n3 + Y(i, k)] += g[k] / M * cj;
        Rc[Z(i, j) * n3 + Z(i, j)] += g[k] / M * (ck - 1.0);
      }
  Mat Lc(n3 * n3, 0.0);
  for (int a = 0; a < n3 * n3; ++a) Lc[a] = -Rc[a];
  for (int a = 0; a < n3; ++a) Lc[a * n3 + a] += 1.0;
  if (!invert(Lc, n3)) return false;
  h.T = matmul(Lc, Rc, n3, n3, n3);
  return true;
}

}  // namespace dgh
