// Element order of the 3D layout (see order.hpp).
#include "order.hpp"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <numeric>

#include "levels.hpp"

namespace dgh {

namespace {

uint64_t spread3(uint64_t x) {  // 21 bits -> every third bit
  x &= 0x1fffff;
  x = (x | x << 32) & 0x1f00000000ffffULL;
  x = (x | x << 16) & 0x1f0000ff0000ffULL;
  x = (x | x << 8) & 0x100f00f00f00f00fULL;
  x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
  x = (x | x << 2) & 0x1249249249249249ULL;
  return x;
}

void morton_order(const Mesh& m, std::vector<int>& slot2elem) {
  const int K = m.K;
  std::vector<std::pair<uint64_t, int>> key(K);
  for (int e = 0; e < K; ++e) {
    double c[3] = {0, 0, 0};
    for (int k = 0; k < 4; ++k)
      for (int d = 0; d < 3; ++d) c[d] += 0.25 * m.VX[3 * m.EToV[4 * e + k] + d];
    uint64_t code = 0;
    for (int d = 0; d < 3; ++d) {
      const double u = (c[d] - m.lo[d]) / (m.hi[d] - m.lo[d]);
      const uint64_t q = (uint64_t)std::min(2097151.0, std::max(0.0, u * 2097152.0));
      code |= spread3(q) << d;
    }
    key[e] = {code, e};
  }
  std::sort(key.begin(), key.end());
  const int nslot = (K + kTile - 1) / kTile * kTile;
  slot2elem.assign(nslot, -1);
  for (int i = 0; i < K; ++i) slot2elem[i] = key[i].second;
}

}  // namespace

void element_order(const Mesh& m, std::vector<int>& slot2elem, bool* structured) {
  const int K = m.K;
  *structured = false;
  // bounding boxes; a structured mesh has one box size for all elements
  std::vector<double> bmin(3 * K);
  double h[3] = {-1, -1, -1};
  bool ok = true;
  for (int e = 0; e < K && ok; ++e) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int k = 0; k < 4; ++k)
      for (int d = 0; d < 3; ++d) {
        const double x = m.VX[3 * m.EToV[4 * e + k] + d];
        lo[d] = std::min(lo[d], x);
        hi[d] = std::max(hi[d], x);
      }
    for (int d = 0; d < 3; ++d) {
      const double ext = hi[d] - lo[d];
      if (h[d] < 0) h[d] = ext;
      if (!(ext > 0) || std::fabs(ext - h[d]) > 1e-9 * h[d]) ok = false;
      bmin[3 * e + d] = lo[d];
    }
  }
  int n[3] = {0, 0, 0};
  if (ok)
    for (int d = 0; d < 3; ++d) {
      const double r = (m.hi[d] - m.lo[d]) / h[d];
      n[d] = (int)std::llround(r);
      if (n[d] < 1 || std::fabs(r - n[d]) > 1e-6) ok = false;
    }
  // shape class = the ordered vertex offsets (0/1 per axis) within the box
  std::vector<int> cls(K), cell(K);
  std::map<int, int> classes;
  for (int e = 0; e < K && ok; ++e) {
    int code = 0;
    for (int k = 0; k < 4; ++k)
      for (int d = 0; d < 3; ++d) {
        const double o = (m.VX[3 * m.EToV[4 * e + k] + d] - bmin[3 * e + d]) / h[d];
        const long b = std::lround(o);
        if ((b != 0 && b != 1) || std::fabs(o - b) > 1e-6) ok = false;
        code = code * 2 + (int)b;
      }
    int ci[3];
    for (int d = 0; d < 3; ++d) {
      const double r = (bmin[3 * e + d] - m.lo[d]) / h[d];
      ci[d] = (int)std::llround(r);
      if (std::fabs(r - ci[d]) > 1e-6 || ci[d] < 0 || ci[d] >= n[d]) ok = false;
    }
    cls[e] = code;
    cell[e] = (ci[2] * n[1] + ci[1]) * n[0] + ci[0];
    classes.emplace(code, 0);
  }
  if (ok && (int)classes.size() > 24) ok = false;
  if (ok) {
    int r = 0;
    for (auto& kv : classes) kv.second = r++;
    const int nc = (int)classes.size();
    const long ncell = (long)n[0] * n[1] * n[2];
    const long nblock = (ncell + kTile - 1) / kTile;
    slot2elem.assign((size_t)nblock * nc * kTile, -1);
    for (int e = 0; e < K && ok; ++e) {
      const long c = cell[e];
      const size_t slot = ((size_t)(c / kTile) * nc + classes[cls[e]]) * kTile + c % kTile;
      if (slot2elem[slot] != -1) ok = false;  // two elements of one shape in a cell
      slot2elem[slot] = e;
    }
    if (ok) {
      *structured = true;
      return;
    }
  }
  morton_order(m, slot2elem);
}

}  // namespace dgh
