// HABC constants: Pade coefficients and the edge/corner compatibility maps.
//
// Section 2.1: gamma_n = tan^2(n pi / M), M = 2P + 1 (the paper's c_n).
// Section 3.1: the incoming characteristics at an edge solve a 2P system
// L r- = R r+ + b (b from the 1D temporaries p*), at a corner a 3P^2 system
// L r- = R r+; L = I - R in both cases.  The inverse is applied as two
// precomputed maps: edge r- = G r+ + H b with G = L^-1 R, H = L^-1;
// corner r- = T r+ with T = L^-1 R.
#pragma once
#include <vector>

namespace dgh {

struct HabcConsts {
  int P = 0;
  std::vector<double> gamma;    // P
  std::vector<double> Cji, Cij; // P x P: [i][j] = C_ji, C_ij; C_ab = (1+g_a)/(1+g_a+g_b)
  std::vector<double> G, H;     // 2P x 2P, row-major; unknowns ordered (A_1..A_P, B_1..B_P)
  std::vector<double> T;        // 3P^2 x 3P^2; unknowns (X_jk, Y_ik, Z_ij), index a*P + b
};

bool build_habc(int P, const double* gamma_or_null, HabcConsts& h);

}  // namespace dgh
