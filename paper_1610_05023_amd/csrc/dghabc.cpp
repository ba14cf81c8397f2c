// C ABI of the time stepper (include/dghabc.h): setup on the host, device
// data inside one caller-owned workspace, and the stage loop of Algorithm 1.
#include "dghabc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "habc.hpp"
#include "levels.hpp"
#include "mesh.hpp"
#include "order.hpp"

namespace {

// Carpenter & Kennedy (1994) five-stage fourth-order 2N-storage coefficients.
const double kA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                      -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
const double kB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                      1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                      2277821191437.0 / 14882151754819.0};
const double kC[5] = {0.0, 1432997174477.0 / 9575080441755.0, 2526269341429.0 / 6820363962896.0,
                      2006345519317.0 / 3224310063776.0, 2802321613138.0 / 2924317926251.0};

enum Stage { S_CREATED = 0, S_MESH, S_ORDER, S_HABC, S_MATERIAL, S_BOUND };

struct Region {
  size_t off = 0, bytes = 0;
};

struct Layout {
  size_t total = 0;
  Region q3[2], res3, geo3, zn3, nbr3, ops3, ops3f, ops3b, fmask3, fmap3, mass3, J3, esum;
  Region q2[2], res2, qb3, q03, geo2, edge2, info2, tetnode2, nbrnode2, ops2, fmask2, gamma;
  Region q1[2], res1, qb2, q02, geo1, info1, trinode1, ops1, cji, cij, G, H;
  Region qb1, info0, nrm0, T, srcw, srcp, flags, ops2f;
  Region mlpw, hist, csamp;   // learned closure: parameters, trace history, samples
  Region clk;                 // device clock of replayed stepping {t0, steps}
  Region grp;                 // member tables of a group step (two parities)
  // per-shot strides (doubles) of the state arrays
  size_t st3 = 0, st2 = 0, stb3 = 0, st1 = 0, stb2 = 0, stb1 = 0;
  size_t e3 = 8;   // bytes per element of the 3D state (8 FP64, 4 FP32)
  Region* add(Region& r, size_t bytes) {
    r.off = total;
    r.bytes = bytes;
    total += (bytes + 255) / 256 * 256;
    return &r;
  }
};

}  // namespace

struct dgh_ctx {
  int device = 0, precision = 0, n_shots = 1;
  int stage = S_CREATED;
  std::string err;
  dgh::Mesh mesh;
  int N = 0, P = 0;
  std::vector<double> gamma_in;
  bool gamma_given = false;
  dgh::HabcConsts habc;
  std::vector<double> rho, c;
  Layout lay;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int cur = 0;
  int ntile = 0;
  std::vector<int> slot2elem, elem2slot;  // element order of the 3D layout
  bool structured = false;
  // point source of each shot: slot of its element (-1: none)
  std::vector<int> src_slot;
  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev;   // pairs (start, stop) per timed launch
  size_t ev_used = 0;
  // host copies of device-layout constants (kept for tests and re-uploads)
  dgh::Lvl3 L3{};
  dgh::Lvl2 L2{};
  dgh::Lvl1 L1{};
  dgh::Lvl0 L0{};
  bool closure = false;               // learned closure replaces the face level
  bool record = false;                // keep the trace history for sampling
  double mem_tau[dgh::kMemScales] = {0, 0, 0, 0};   // closure time scales (0: default)
  dgh::LvlF LF{};
  // replayed stepping: one captured step per starting buffer parity, valid
  // for (gdt, gclosure, grecord); captured on a stream of the library's own
  bool graph = false;
  hipStream_t cap = nullptr;
  hipGraph_t g[2] = {nullptr, nullptr};
  hipGraphExec_t gx[2] = {nullptr, nullptr};
  double gdt = 0.0;
  bool gclosure = false, grecord = false;
};

namespace {

dgh_status fail(dgh_ctx* c, dgh_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

dgh_status hipfail(dgh_ctx* c, hipError_t e, const char* where) {
  return fail(c, DGH_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

void drop_graphs(dgh_ctx* c);

#define HIPCHECK(ctx, call)                                   \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return hipfail(ctx, e_, #call);     \
  } while (0)

template <class T>
T* dptr(dgh_ctx* c, const Region& r) {
  return reinterpret_cast<T*>(c->ws + r.off);
}

// Host-to-device copy and fill on the bound stream, each waited for before
// returning: work already queued on that stream (a step in flight) finishes
// first, and the host buffer may be reused at once.
hipError_t h2d(dgh_ctx* c, void* dst, const void* src, size_t bytes) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream);
  return e != hipSuccess ? e : hipStreamSynchronize(c->stream);
}

hipError_t d2h(dgh_ctx* c, void* dst, const void* src, size_t bytes) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c->stream);
  return e != hipSuccess ? e : hipStreamSynchronize(c->stream);
}

hipError_t dzero(dgh_ctx* c, void* dst, size_t bytes) {
  hipError_t e = hipMemsetAsync(dst, 0, bytes, c->stream);
  return e != hipSuccess ? e : hipStreamSynchronize(c->stream);
}

// Builds the device-layout arrays on the host.
struct HostArrays {
  std::vector<double> geo3, zn3, ops3, mass3, J3, ops2f;
  std::vector<float> ops3f;
  std::vector<unsigned short> ops3b;
  std::vector<int> nbr3, fmask3, fmap3;
  std::vector<double> geo2, edge2, ops2;
  std::vector<int> info2, tetnode2, nbrnode2, fmask2;
  std::vector<double> geo1, ops1;
  std::vector<int> info1, trinode1;
  std::vector<int> info0;
  std::vector<double> nrm0;
  bool map_ok = true;
};

void build_host_arrays(dgh_ctx* c, HostArrays& h) {
  const dgh::Mesh& m = c->mesh;
  const int Np = m.tet.Np, Nfp = m.tet.Nfp, nt = c->ntile;
  const int T = dgh::kTile;
  // ---- 3D
  h.geo3.assign((size_t)nt * 12 * T, 0.0);
  h.zn3.assign((size_t)nt * 4 * T, 1.0);
  h.nbr3.assign((size_t)nt * 4 * T, -1 - 1);  // padding: ABC boundary
  h.J3.assign((size_t)nt * T, 0.0);
  for (int slot = 0; slot < nt * T; ++slot) {
    const int tile = slot / T, es = slot % T;
    double* g = &h.geo3[(size_t)tile * 12 * T + es];
    const int e = c->slot2elem[slot];
    if (e < 0) {  // padding slot: benign geometry, 1/rho = 0 marks it, never written
      g[0] = g[4 * T] = g[8 * T] = 1.0;
      g[9 * T] = 0.0;
      g[10 * T] = g[11 * T] = 1.0;
      continue;
    }
    for (int k = 0; k < 9; ++k) g[k * T] = m.geo[9 * e + k];
    g[9 * T] = 1.0 / c->rho[e];
    g[10 * T] = c->rho[e] * c->c[e] * c->c[e];
    g[11 * T] = c->rho[e] * c->c[e];
    h.J3[slot] = m.J[e];
    for (int f = 0; f < 4; ++f) {
      const size_t o = ((size_t)tile * 4 + f) * T + es;
      const int e2 = m.EToE[4 * e + f];
      if (e2 >= 0) {
        h.nbr3[o] = (c->elem2slot[e2] << 5) | (m.EToF[4 * e + f] << 3) | m.perm[4 * e + f];
        h.zn3[o] = c->rho[e2] * c->c[e2];
      } else {
        const int df = m.bface[4 * e + f];
        const int bc = m.face_bc[df];
        int code = 0;
        if (bc == dgh::BC_HABC) {
          const int t = m.face_tri[4 * e + f];
          // permutation taking this face's vertices to the sorted triangle vertices
          const int* tv = &m.tri_verts[3 * t];
          int q[3];
          for (int k = 0; k < 3; ++k) {
            const int gv = m.EToV[4 * e + dgh::kFaceVerts[f][k]];
            q[k] = (int)(std::find(tv, tv + 3, gv) - tv);
          }
          static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                          {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
          int p = 0;
          for (int k = 0; k < 6; ++k)
            if (perms[k][0] == q[0] && perms[k][1] == q[1] && perms[k][2] == q[2]) p = k;
          code = (t << 5) | (p << 2) | 0;
          for (int i = 0; i < Nfp; ++i)
            if (m.fmap[((f * 4 + 0) * 6 + p) * Nfp + i] != m.facenode_trinode[t * Nfp + i])
              h.map_ok = false;
        } else {
          code = bc == dgh::BC_DIRICHLET ? 2 : 1;
        }
        h.nbr3[o] = -1 - code;
        h.zn3[o] = c->rho[e] * c->c[e];
      }
    }
  }
  {
    // MFMA A-fragments (see Lvl3::ops)
    const int RG = (Np + 3) / 4, FK = (Nfp + 3) / 4;
    h.ops3.assign(dgh::frag3_size(m.N), 0.0);
    const dgh::Mat* Ds[3] = {&m.tet.Dr, &m.tet.Ds, &m.tet.Dt};
    for (int d = 0; d < 3; ++d)
      for (int rg = 0; rg < RG; ++rg)
        for (int ks = 0; ks < RG; ++ks)
          for (int t = 0; t < 16; ++t) {
            const int row = 4 * rg + (t & 3), col = 4 * ks + (t >> 2);
            if (row < Np && col < Np)
              h.ops3[(((size_t)d * RG + rg) * RG + ks) * 16 + t] = (*Ds[d])[row * Np + col];
          }
    const size_t off = (size_t)3 * RG * RG * 16;
    for (int rg = 0; rg < RG; ++rg)
      for (int f = 0; f < 4; ++f)
        for (int jj = 0; jj < FK; ++jj)
          for (int t = 0; t < 16; ++t) {
            const int row = 4 * rg + (t & 3), k = 4 * jj + (t >> 2);
            if (row < Np && k < Nfp)
              h.ops3[off + (((size_t)rg * 4 + f) * FK + jj) * 16 + t] =
                  m.tet.LIFT[row * 4 * Nfp + f * Nfp + k];
          }
  }
  if (c->precision == DGH_FP32_MFMA) {
    // A-fragments of the FP32 16x16x4 MFMA (see Lvl3::ops32)
    const int RG = (Np + 3) / 4, RB = (Np + 15) / 16, FK = (Nfp + 3) / 4;
    h.ops3f.assign(dgh::frag3f_size(m.N), 0.0f);
    const dgh::Mat* Ds[3] = {&m.tet.Dr, &m.tet.Ds, &m.tet.Dt};
    for (int d = 0; d < 3; ++d)
      for (int rb = 0; rb < RB; ++rb)
        for (int j = 0; j < RG; ++j)
          for (int l = 0; l < 64; ++l) {
            const int row = 16 * rb + l % 16, col = 4 * j + l / 16;
            if (row < Np && col < Np)
              h.ops3f[(((size_t)d * RB + rb) * RG + j) * 64 + l] = (float)(*Ds[d])[row * Np + col];
          }
    const size_t off = (size_t)3 * RB * RG * 64;
    for (int rb = 0; rb < RB; ++rb)
      for (int f = 0; f < 4; ++f)
        for (int jj = 0; jj < FK; ++jj)
          for (int l = 0; l < 64; ++l) {
            const int row = 16 * rb + l % 16, k = 4 * jj + l / 16;
            if (row < Np && k < Nfp)
              h.ops3f[off + (((size_t)rb * 4 + f) * FK + jj) * 64 + l] =
                  (float)m.tet.LIFT[row * 4 * Nfp + f * Nfp + k];
          }
  }
  if (c->precision == DGH_BF16_MFMA) {
    // A-fragments of the BF16 16x16x16 MFMA (see Lvl3::opsb): operator
    // entries rounded to FP32, then to the nearest BF16 (ties to even)
    const int RB = (Np + 15) / 16, FK = (Nfp + 15) / 16;
    h.ops3b.assign(dgh::frag3b_size(m.N), 0);
    auto bf16 = [](double v) {
      const float f = (float)v;
      unsigned u;
      std::memcpy(&u, &f, 4);
      return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
    };
    const dgh::Mat* Ds[3] = {&m.tet.Dr, &m.tet.Ds, &m.tet.Dt};
    for (int d = 0; d < 3; ++d)
      for (int rb = 0; rb < RB; ++rb)
        for (int j = 0; j < RB; ++j)
          for (int l = 0; l < 64; ++l)
            for (int i = 0; i < 4; ++i) {
              const int row = 16 * rb + l % 16, col = 16 * j + 4 * (l / 16) + i;
              if (row < Np && col < Np)
                h.ops3b[((((size_t)d * RB + rb) * RB + j) * 64 + l) * 4 + i] =
                    bf16((*Ds[d])[row * Np + col]);
            }
    const size_t off = (size_t)3 * RB * RB * 64 * 4;
    for (int rb = 0; rb < RB; ++rb)
      for (int f = 0; f < 4; ++f)
        for (int jj = 0; jj < FK; ++jj)
          for (int l = 0; l < 64; ++l)
            for (int i = 0; i < 4; ++i) {
              const int row = 16 * rb + l % 16, k = 16 * jj + 4 * (l / 16) + i;
              if (row < Np && k < Nfp)
                h.ops3b[off + ((((size_t)rb * 4 + f) * FK + jj) * 64 + l) * 4 + i] =
                    bf16(m.tet.LIFT[row * 4 * Nfp + f * Nfp + k]);
            }
  }
  h.mass3 = m.tet.Mass;
  h.fmask3 = m.tet.Fmask;
  h.fmap3 = m.fmap;
  (void)Np;
  // ---- 2D
  const int Kt = m.Ktri, Np2 = m.tri.Np, Nfp2 = m.tri.Nfp;
  h.geo2.assign((size_t)Kt * 8, 0.0);
  h.info2.assign((size_t)Kt * 8, 0);
  h.tetnode2 = m.tri_tetnode;
  h.nbrnode2.assign((size_t)Kt * 3 * Nfp2, 0);
  for (int t = 0; t < Kt; ++t) {
    const int e = m.tri_elem[t];
    for (int k = 0; k < 4; ++k) h.geo2[t * 8 + k] = m.tri_geo[4 * t + k];
    h.geo2[t * 8 + 4] = 1.0 / c->rho[e];
    h.geo2[t * 8 + 5] = c->rho[e] * c->c[e] * c->c[e];
    h.geo2[t * 8 + 6] = c->rho[e] * c->c[e];
    h.info2[t * 8 + 0] = c->elem2slot[e];
    h.info2[t * 8 + 1] = m.tri_dface[t] / 2;
    h.info2[t * 8 + 2] = (m.tri_dface[t] % 2) ? 1 : -1;
    for (int f = 0; f < 3; ++f) {
      const int t2 = m.tri_EToE[3 * t + f];
      int code;
      if (t2 >= 0) {
        code = t2;
        for (int k = 0; k < Nfp2; ++k)
          h.nbrnode2[(t * 3 + f) * Nfp2 + k] = m.tri_nbr_node[(3 * t + f) * Nfp2 + k];
      } else {
        const int l = m.tri_edge_line[3 * t + f];
        if (l >= 0) {
          code = -1 - ((l << 3) | (m.tri_edge_side[3 * t + f] << 2) | 0);
          for (int k = 0; k < Nfp2; ++k)
            h.nbrnode2[(t * 3 + f) * Nfp2 + k] = m.tri_edge_linenode[(3 * t + f) * Nfp2 + k];
        } else {
          const int bc = m.face_bc[m.tri_bdface[3 * t + f]];
          code = -1 - (bc == dgh::BC_DIRICHLET ? 2 : 1);
        }
      }
      h.info2[t * 8 + 3 + f] = code;
    }
  }
  // per edge of each triangle (edges s = -1, r + s = 0, r = -1, whose
  // n fsc are -grad s, grad(r + s), -grad r): the unit in-plane normal, the
  // face scale, and the weights of the upwind flux against the exterior
  // state, whose impedance is the neighbour triangle's across an inner edge
  // and the own one on the boundary of the face
  h.edge2.assign((size_t)Kt * 24, 0.0);
  for (int t = 0; t < Kt; ++t) {
    const double rx = h.geo2[t * 8], ry = h.geo2[t * 8 + 1], sx = h.geo2[t * 8 + 2],
                 sy = h.geo2[t * 8 + 3], Z = h.geo2[t * 8 + 6];
    for (int f = 0; f < 3; ++f) {
      const double cr = f == 0 ? 0.0 : (f == 1 ? 1.0 : -1.0);
      const double cs = f == 2 ? 0.0 : (f == 1 ? 1.0 : -1.0);
      double na = cr * rx + cs * sx, nb = cr * ry + cs * sy;
      const double fsc = std::sqrt(na * na + nb * nb);
      na /= fsc;
      nb /= fsc;
      const int code = h.info2[t * 8 + 3 + f];
      const double ZP = code >= 0 ? h.geo2[(size_t)code * 8 + 6] : Z;
      const double iZ = 1.0 / (Z + ZP);
      double* o = &h.edge2[((size_t)t * 3 + f) * 8];
      o[0] = na;
      o[1] = nb;
      o[2] = fsc;
      o[3] = ZP * iZ;        // aM
      o[4] = Z * iZ;         // aP
      o[5] = iZ;
      o[6] = Z * (ZP * iZ);  // bZ
    }
  }
  {
    // MFMA A-fragments of the face kernel (see LvlF::ops)
    const int RG = (Np2 + 3) / 4, EK = (Nfp2 + 3) / 4;
    h.ops2f.assign(dgh::frag2_size(m.N), 0.0);
    const dgh::Mat* Ds[2] = {&m.tri.Dr, &m.tri.Ds};
    for (int d = 0; d < 2; ++d)
      for (int rg = 0; rg < RG; ++rg)
        for (int ks = 0; ks < RG; ++ks)
          for (int t = 0; t < 16; ++t) {
            const int row = 4 * rg + (t & 3), col = 4 * ks + (t >> 2);
            if (row < Np2 && col < Np2)
              h.ops2f[(((size_t)d * RG + rg) * RG + ks) * 16 + t] = (*Ds[d])[row * Np2 + col];
          }
    const size_t off = (size_t)2 * RG * RG * 16;
    for (int rg = 0; rg < RG; ++rg)
      for (int e = 0; e < 3; ++e)
        for (int jj = 0; jj < EK; ++jj)
          for (int t = 0; t < 16; ++t) {
            const int row = 4 * rg + (t & 3), k = 4 * jj + (t >> 2);
            if (row < Np2 && k < Nfp2)
              h.ops2f[off + (((size_t)rg * 3 + e) * EK + jj) * 16 + t] =
                  m.tri.LIFT[row * 3 * Nfp2 + e * Nfp2 + k];
          }
  }
  h.ops2.clear();
  h.ops2.insert(h.ops2.end(), m.tri.Dr.begin(), m.tri.Dr.end());
  h.ops2.insert(h.ops2.end(), m.tri.Ds.begin(), m.tri.Ds.end());
  h.ops2.insert(h.ops2.end(), m.tri.LIFT.begin(), m.tri.LIFT.end());
  h.fmask2 = m.tri.Fmask;
  (void)Np2;
  // ---- 1D
  const int Kl = m.Klin, Np1 = m.line.Np;
  h.geo1.assign((size_t)Kl * 4, 0.0);
  h.info1.assign((size_t)Kl * 8, 0);
  h.trinode1 = m.lin_trinode;
  for (int l = 0; l < Kl; ++l) {
    const int tA = m.lin_tri[2 * l];
    const int e = m.tri_elem[tA];
    h.geo1[l * 4 + 0] = m.lin_rx[l];
    h.geo1[l * 4 + 1] = 1.0 / c->rho[e];
    h.geo1[l * 4 + 2] = c->rho[e] * c->c[e] * c->c[e];
    h.geo1[l * 4 + 3] = c->rho[e] * c->c[e];
    const int de = m.lin_dedge[l];
    for (int side = 0; side < 2; ++side) {
      const int t = m.lin_tri[2 * l + side];
      const int other = dgh::kDomainEdges[de][1 - side];
      const int ax = other / 2;
      const int comp = 1 + (m.tri_axes[2 * t] == ax ? 0 : 1);
      h.info1[l * 8 + side] = t;
      h.info1[l * 8 + 2 + side] = (other % 2) ? comp : -comp;
    }
    const double sgn = m.lin_rx[l] > 0 ? 1.0 : -1.0;
    for (int end = 0; end < 2; ++end) {
      int code;
      const int l2 = m.lin_EToE[2 * l + end];
      if (l2 >= 0) {
        code = (l2 << 1) | m.lin_EToF[2 * l + end];
      } else if (m.lin_corner[2 * l + end] >= 0) {
        code = -1 - ((m.lin_corner[2 * l + end] << 4) | (m.lin_corner_slot[2 * l + end] << 2) | 0);
      } else {
        code = -1 - (m.lin_endbc[2 * l + end] == dgh::BC_DIRICHLET ? 2 : 1);
      }
      h.info1[l * 8 + 4 + end] = code;
      h.info1[l * 8 + 6 + end] = (int)(end ? sgn : -sgn);
    }
  }
  h.ops1 = m.line.Dr;
  h.ops1.insert(h.ops1.end(), m.line.LIFT.begin(), m.line.LIFT.end());
  (void)Np1;
  // ---- 0D
  h.info0.assign((size_t)m.Kpnt * 6, 0);
  h.nrm0 = m.pnt_nrm;
  for (int p = 0; p < m.Kpnt; ++p)
    for (int a = 0; a < 3; ++a) {
      h.info0[(p * 3 + a) * 2] = m.pnt_line[3 * p + a];
      h.info0[(p * 3 + a) * 2 + 1] = m.pnt_end[3 * p + a];
    }
}

size_t round32(size_t n) { return (std::max<size_t>(n, 1) + 31) / 32 * 32; }

void compute_layout(dgh_ctx* c) {
  const dgh::Mesh& m = c->mesh;
  Layout& L = c->lay;
  L = Layout{};
  const int Np = m.tet.Np, Nfp = m.tet.Nfp, nt = c->ntile, T = dgh::kTile, P = c->P;
  const size_t d = sizeof(double), i4 = sizeof(int), S = (size_t)c->n_shots;
  // every state array holds n_shots shots, each starting 256-byte aligned
  const int Kt = m.Ktri, Np2 = m.tri.Np, Nfp2 = m.tri.Nfp, Kl = m.Klin, Np1 = m.line.Np;
  L.e3 = c->precision == DGH_FP64 ? 8 : 4;   // FP32 state in both mixed forms
  L.st3 = ((size_t)nt * 4 * Np * T + 63) / 64 * 64;   // 256-byte aligned shots
  // at least one set of one triangle (read, unused, by the face kernel at P = 0)
  L.st2 = round32((size_t)Kt * std::max(P, 1) * 3 * Np2);
  L.stb3 = round32(std::max<size_t>(Nfp, (size_t)Kt * Np2));  // >= one triangle (read masked)
  L.st1 = round32((size_t)Kl * P * P * 2 * Np1);
  // at least one line, so that the face kernel may read line 0 of qb2
  L.stb2 = round32((size_t)std::max(Kl, 1) * 2 * std::max(P, 1) * Np1);
  L.stb1 = round32((size_t)m.Kpnt * 3 * P * P);
  L.add(L.q3[0], S * L.st3 * L.e3);
  L.add(L.q3[1], S * L.st3 * L.e3);
  L.add(L.res3, S * L.st3 * L.e3);
  L.add(L.geo3, (size_t)nt * 12 * T * d);
  L.add(L.zn3, (size_t)nt * 4 * T * d);
  L.add(L.nbr3, (size_t)nt * 4 * T * i4);
  L.add(L.ops3, (size_t)dgh::frag3_size(m.N) * d);
  L.add(L.ops3f, L.e3 == 4 ? (size_t)dgh::frag3f_size(m.N) * sizeof(float) : 1);
  L.add(L.ops3b, c->precision == DGH_BF16_MFMA ? (size_t)dgh::frag3b_size(m.N) * 2 : 1);
  L.add(L.fmask3, (size_t)4 * Nfp * i4);
  L.add(L.fmap3, (size_t)96 * Nfp * i4);
  L.add(L.mass3, (size_t)Np * Np * d);
  L.add(L.J3, (size_t)nt * T * d);
  L.add(L.esum, (size_t)nt * d);
  L.add(L.q2[0], S * L.st2 * d);
  L.add(L.q2[1], S * L.st2 * d);
  L.add(L.res2, S * L.st2 * d);
  L.add(L.qb3, S * L.stb3 * d);
  L.add(L.q03, S * L.stb3 * d);
  L.add(L.geo2, (size_t)std::max(1, Kt * 8) * d);
  L.add(L.edge2, (size_t)std::max(1, Kt * 24) * d);
  L.add(L.info2, (size_t)std::max(1, Kt * 8) * i4);
  L.add(L.tetnode2, (size_t)std::max(1, Kt * Np2) * i4);
  L.add(L.nbrnode2, (size_t)std::max(1, Kt * 3 * Nfp2) * i4);
  L.add(L.ops2, (size_t)(2 * Np2 * Np2 + Np2 * 3 * Nfp2) * d);
  L.add(L.fmask2, (size_t)3 * Nfp2 * i4);
  L.add(L.gamma, (size_t)std::max(1, P) * d);
  L.add(L.q1[0], S * L.st1 * d);
  L.add(L.q1[1], S * L.st1 * d);
  L.add(L.res1, S * L.st1 * d);
  L.add(L.qb2, S * L.stb2 * d);
  L.add(L.q02, S * L.stb2 * d);
  L.add(L.geo1, (size_t)std::max(1, Kl * 4) * d);
  L.add(L.info1, (size_t)std::max(1, Kl * 8) * i4);
  L.add(L.trinode1, (size_t)std::max(1, Kl * 2 * Np1) * i4);
  L.add(L.ops1, (size_t)(Np1 * Np1 + 2 * Np1) * d);
  L.add(L.cji, (size_t)std::max(1, P * P) * d);
  L.add(L.cij, (size_t)std::max(1, P * P) * d);
  L.add(L.G, (size_t)std::max(1, 4 * P * P) * d);
  L.add(L.H, (size_t)std::max(1, 4 * P * P) * d);
  L.add(L.qb1, S * L.stb1 * d);
  L.add(L.info0, (size_t)std::max(1, m.Kpnt * 6) * i4);
  L.add(L.nrm0, (size_t)std::max(1, m.Kpnt * 3) * d);
  L.add(L.T, (size_t)std::max(1, 9 * P * P * P * P) * d);
  L.add(L.srcw, S * Np * d);
  L.add(L.srcp, S * 4 * d);
  L.add(L.flags, (size_t)dgh::kScanMax * dgh::kScanBlocks * i4);
  L.add(L.ops2f, (size_t)dgh::frag2_size(m.N) * d);
  const size_t nnode = (size_t)std::max(1, Kt * Np2);
  L.add(L.mlpw, (size_t)dgh::kMlpParams * sizeof(float));
  L.add(L.hist, S * nnode * 10 * sizeof(float));
  L.add(L.csamp, nnode * 12 * sizeof(float));   // rows of 11, then targets
  L.add(L.clk, 2 * sizeof(double));
  L.add(L.grp, 2 * dgh::kMaxGroup * sizeof(dgh::Member3));
}

template <class V>
hipError_t upload(dgh_ctx* c, const Region& r, const V& v) {
  if (v.empty()) return hipSuccess;
  const size_t b = v.size() * sizeof(v[0]);
  if (b > r.bytes) return hipErrorInvalidValue;
  return h2d(c, c->ws + r.off, v.data(), b);
}

// register-streaming 3D kernel: 8 waves per workgroup where it is the
// default kernel with its operators in LDS (FP64 at N = 5, the FP32 and BF16
// variants at N = 6: two waves per SIMD share them), else 4
int default_waves(const dgh_ctx* c) {
  return (c->precision == DGH_FP64 ? c->N == 5 : c->N == 6) ? 8 : 4;
}

void fill_levels(dgh_ctx* c) {
  const dgh::Mesh& m = c->mesh;
  const Layout& L = c->lay;
  dgh::Lvl3& a = c->L3;
  a.K = m.K;
  a.ntile = c->ntile;
  if (a.eighths == 0) a.eighths = 8;   // the whole resident grid unless tuned
  if (a.waves == 0) a.waves = default_waves(c);
  a.N = m.N;
  a.Np = m.tet.Np;
  a.Nfp = m.tet.Nfp;
  a.nqb3 = std::max(m.tet.Nfp, m.Ktri * m.tri.Np);
  a.ops = dptr<double>(c, L.ops3);
  a.ops32 = dptr<float>(c, L.ops3f);
  a.opsb = dptr<unsigned short>(c, L.ops3b);
  a.fmask = dptr<int>(c, L.fmask3);
  a.fmap = dptr<int>(c, L.fmap3);
  a.geo = dptr<double>(c, L.geo3);
  a.zn = dptr<double>(c, L.zn3);
  a.nbr = dptr<int>(c, L.nbr3);
  dgh::Lvl2& b = c->L2;
  b.Kt = m.Ktri;
  b.P = c->P;
  b.Np = m.tri.Np;
  b.Nfp = m.tri.Nfp;
  b.invM = 1.0 / (2.0 * c->P + 1.0);
  b.ops = dptr<double>(c, L.ops2);
  b.fmask = dptr<int>(c, L.fmask2);
  b.geo = dptr<double>(c, L.geo2);
  b.edge = dptr<double>(c, L.edge2);
  b.info = dptr<int>(c, L.info2);
  b.tetnode = dptr<int>(c, L.tetnode2);
  b.nbrnode = dptr<int>(c, L.nbrnode2);
  b.gamma = dptr<double>(c, L.gamma);
  dgh::Lvl1& d = c->L1;
  d.Kl = m.Klin;
  d.P = c->P;
  d.Np = m.line.Np;
  d.invM = b.invM;
  d.ops = dptr<double>(c, L.ops1);
  d.geo = dptr<double>(c, L.geo1);
  d.info = dptr<int>(c, L.info1);
  d.trinode = dptr<int>(c, L.trinode1);
  d.gamma = b.gamma;
  d.Cji = dptr<double>(c, L.cji);
  d.Cij = dptr<double>(c, L.cij);
  d.G = dptr<double>(c, L.G);
  d.H = dptr<double>(c, L.H);
  dgh::Lvl0& z = c->L0;
  z.Kp = m.Kpnt;
  z.P = c->P;
  z.info = dptr<int>(c, L.info0);
  z.nrm = dptr<double>(c, L.nrm0);
  z.Tt = dptr<double>(c, L.T);
  c->LF.np3 = m.tet.Np;
  c->LF.ops = dptr<double>(c, L.ops2f);
}

// canonical [K][4][Np] <-> device [tile][4][Np][16] in slot order
void to_tiles(const double* src, double* dst, const std::vector<int>& slot2elem, int Np) {
  const int T = dgh::kTile;
  const size_t nslot = slot2elem.size();
  std::fill(dst, dst + nslot * 4 * Np, 0.0);
  for (size_t slot = 0; slot < nslot; ++slot) {
    const int e = slot2elem[slot];
    if (e < 0) continue;
    for (int f = 0; f < 4; ++f)
      for (int n = 0; n < Np; ++n)
        dst[(((slot / T) * 4 + f) * Np + n) * T + (slot % T)] = src[((size_t)e * 4 + f) * Np + n];
  }
}

void from_tiles(const double* src, double* dst, const std::vector<int>& slot2elem, int Np) {
  const int T = dgh::kTile;
  for (size_t slot = 0; slot < slot2elem.size(); ++slot) {
    const int e = slot2elem[slot];
    if (e < 0) continue;
    for (int f = 0; f < 4; ++f)
      for (int n = 0; n < Np; ++n)
        dst[((size_t)e * 4 + f) * Np + n] = src[(((slot / T) * 4 + f) * Np + n) * T + (slot % T)];
  }
}

}  // namespace

extern "C" {

dgh_status dgh_create(dgh_ctx** out, int device, int precision, int n_shots) {
  if (!out) return DGH_EINVAL;
  *out = nullptr;
  if ((precision != DGH_FP64 && precision != DGH_FP32_MFMA && precision != DGH_BF16_MFMA) ||
      n_shots < 1 || n_shots > 4096 ||
      device < 0)
    return DGH_EINVAL;
  dgh_ctx* c = new (std::nothrow) dgh_ctx();
  if (!c) return DGH_ENOMEM;
  c->device = device;
  c->precision = precision;
  c->n_shots = n_shots;
  *out = c;
  return DGH_OK;
}

dgh_status dgh_upload_mesh(dgh_ctx* c, int Nv, const double* VX, int K, const int* EToV,
                           const double* box, const int* periodic) {
  if (!c) return DGH_EINVAL;
  if (c->stage >= S_BOUND) return fail(c, DGH_ESTATE, "mesh after bind");
  if (Nv <= 0 || K <= 0 || !VX || !EToV || !box) return fail(c, DGH_EINVAL, "bad mesh arguments");
  if (K >= (1 << 26)) return fail(c, DGH_EINVAL, "too many elements");
  dgh::Mesh& m = c->mesh;
  m = dgh::Mesh{};
  m.Nv = Nv;
  m.K = K;
  m.VX.assign(VX, VX + 3 * (size_t)Nv);
  m.EToV.assign(EToV, EToV + 4 * (size_t)K);
  for (int d = 0; d < 3; ++d) {
    m.lo[d] = box[d];
    m.hi[d] = box[3 + d];
    if (!(m.hi[d] > m.lo[d])) return fail(c, DGH_EINVAL, "empty box");
    m.periodic[d] = periodic ? (periodic[d] != 0) : 0;
  }
  c->stage = S_MESH;
  return DGH_OK;
}

dgh_status dgh_set_order(dgh_ctx* c, int N) {
  if (!c) return DGH_EINVAL;
  if (c->stage < S_MESH || c->stage >= S_BOUND) return fail(c, DGH_ESTATE, "set_order out of order");
  if (N < 1 || N > 6) return fail(c, DGH_EINVAL, "N must be in 1..6");
  c->N = N;
  c->stage = S_ORDER;
  return DGH_OK;
}

dgh_status dgh_set_habc(dgh_ctx* c, int P, const double* gamma, const int* face_bc) {
  if (!c) return DGH_EINVAL;
  if (c->stage < S_ORDER || c->stage >= S_BOUND) return fail(c, DGH_ESTATE, "set_habc out of order");
  if (P < 0 || P > 12) return fail(c, DGH_EINVAL, "P must be in 0..12");
  dgh::Mesh& m = c->mesh;
  m.N = c->N;
  for (int f = 0; f < 6; ++f) {
    const int bc = face_bc ? face_bc[f] : DGH_BC_HABC;
    if (bc < 0 || bc > 3) return fail(c, DGH_EINVAL, "bad face_bc");
    m.face_bc[f] = bc;
  }
  for (int d = 0; d < 3; ++d)
    if ((m.face_bc[2 * d] == DGH_BC_PERIODIC) != (m.face_bc[2 * d + 1] == DGH_BC_PERIODIC))
      return fail(c, DGH_EINVAL, "periodic must pair both faces of an axis");
    else if (m.face_bc[2 * d] == DGH_BC_PERIODIC)
      m.periodic[d] = 1;
  const std::string r = dgh::build_mesh(m);
  if (!r.empty()) return fail(c, DGH_EINVAL, r);
  if (!dgh::build_habc(P, gamma, c->habc)) return fail(c, DGH_EINVAL, "bad HABC coefficients");
  c->P = P;
  dgh::element_order(m, c->slot2elem, &c->structured);
  c->ntile = (int)(c->slot2elem.size() / dgh::kTile);
  c->elem2slot.assign(m.K, -1);
  for (size_t i = 0; i < c->slot2elem.size(); ++i)
    if (c->slot2elem[i] >= 0) c->elem2slot[c->slot2elem[i]] = (int)i;
  c->stage = S_HABC;
  return DGH_OK;
}

dgh_status dgh_set_material(dgh_ctx* c, const double* rho, const double* cc) {
  if (!c) return DGH_EINVAL;
  if (c->stage < S_HABC || c->stage >= S_BOUND) return fail(c, DGH_ESTATE, "set_material out of order");
  if (!rho || !cc) return fail(c, DGH_EINVAL, "null material");
  const int K = c->mesh.K;
  for (int e = 0; e < K; ++e)
    if (!(rho[e] > 0) || !(cc[e] > 0) || !std::isfinite(rho[e]) || !std::isfinite(cc[e]))
      return fail(c, DGH_EINVAL, "materials must be positive and finite");
  c->rho.assign(rho, rho + K);
  c->c.assign(cc, cc + K);
  c->stage = S_MATERIAL;
  return DGH_OK;
}

dgh_status dgh_counts(const dgh_ctx* c, int* out) {
  if (!c || !out) return DGH_EINVAL;
  if (c->stage < S_HABC) return DGH_ESTATE;
  const dgh::Mesh& m = c->mesh;
  out[DGH_C_K] = m.K;
  out[DGH_C_KTRI] = m.Ktri;
  out[DGH_C_KLIN] = m.Klin;
  out[DGH_C_KPNT] = m.Kpnt;
  out[DGH_C_NP] = m.tet.Np;
  out[DGH_C_NP2] = m.tri.Np;
  out[DGH_C_NP1] = m.line.Np;
  out[DGH_C_P] = c->P;
  out[DGH_C_N] = c->N;
  out[DGH_C_NSHOTS] = c->n_shots;
  return DGH_OK;
}

dgh_status dgh_node_coords(const dgh_ctx* c, double* out) {
  if (!c || !out) return DGH_EINVAL;
  if (c->stage < S_HABC) return DGH_ESTATE;
  const dgh::Mesh& m = c->mesh;
  for (int e = 0; e < m.K; ++e)
    for (int n = 0; n < m.tet.Np; ++n) m.node_xyz(e, n, out + ((size_t)e * m.tet.Np + n) * 3);
  return DGH_OK;
}

dgh_status dgh_workspace_size(dgh_ctx* c, size_t* bytes) {
  if (!c || !bytes) return DGH_EINVAL;
  if (c->stage < S_MATERIAL) return fail(c, DGH_ESTATE, "workspace_size before set_material");
  compute_layout(c);
  if (c->lay.st3 * c->lay.e3 > 0xffffffffull)
    return fail(c, DGH_EINVAL, "3D state of a shot exceeds 4 GiB (32-bit buffer offsets)");
  *bytes = c->lay.total;
  return DGH_OK;
}

dgh_status dgh_bind_workspace(dgh_ctx* c, void* dev, size_t bytes, void* stream) {
  if (!c) return DGH_EINVAL;
  if (c->stage < S_MATERIAL) return fail(c, DGH_ESTATE, "bind before set_material");
  compute_layout(c);
  if (c->lay.st3 * c->lay.e3 > 0xffffffffull)
    return fail(c, DGH_EINVAL, "3D state of a shot exceeds 4 GiB (32-bit buffer offsets)");
  if (!dev || bytes < c->lay.total) return fail(c, DGH_ENOMEM, "workspace too small");
  if (reinterpret_cast<uintptr_t>(dev) % 256) return fail(c, DGH_EINVAL, "workspace not 256-byte aligned");
  HIPCHECK(c, hipSetDevice(c->device));
  drop_graphs(c);   // captured steps hold the old workspace's addresses
  c->ws = static_cast<char*>(dev);
  c->stream = static_cast<hipStream_t>(stream);
  HostArrays h;
  build_host_arrays(c, h);
  if (!h.map_ok) return fail(c, DGH_EINVAL, "tet face to triangle node map mismatch");
  const Layout& L = c->lay;
  HIPCHECK(c, hipMemsetAsync(c->ws, 0, L.total, c->stream));
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  HIPCHECK(c, upload(c, L.geo3, h.geo3));
  HIPCHECK(c, upload(c, L.zn3, h.zn3));
  HIPCHECK(c, upload(c, L.nbr3, h.nbr3));
  HIPCHECK(c, upload(c, L.ops3, h.ops3));
  HIPCHECK(c, upload(c, L.ops3f, h.ops3f));
  HIPCHECK(c, upload(c, L.ops3b, h.ops3b));
  HIPCHECK(c, upload(c, L.fmask3, h.fmask3));
  HIPCHECK(c, upload(c, L.fmap3, h.fmap3));
  HIPCHECK(c, upload(c, L.mass3, h.mass3));
  HIPCHECK(c, upload(c, L.J3, h.J3));
  HIPCHECK(c, upload(c, L.geo2, h.geo2));
  HIPCHECK(c, upload(c, L.edge2, h.edge2));
  HIPCHECK(c, upload(c, L.info2, h.info2));
  HIPCHECK(c, upload(c, L.tetnode2, h.tetnode2));
  HIPCHECK(c, upload(c, L.nbrnode2, h.nbrnode2));
  HIPCHECK(c, upload(c, L.ops2, h.ops2));
  HIPCHECK(c, upload(c, L.fmask2, h.fmask2));
  HIPCHECK(c, upload(c, L.gamma, c->habc.gamma));
  HIPCHECK(c, upload(c, L.geo1, h.geo1));
  HIPCHECK(c, upload(c, L.info1, h.info1));
  HIPCHECK(c, upload(c, L.trinode1, h.trinode1));
  HIPCHECK(c, upload(c, L.ops1, h.ops1));
  HIPCHECK(c, upload(c, L.cji, c->habc.Cji));
  HIPCHECK(c, upload(c, L.cij, c->habc.Cij));
  HIPCHECK(c, upload(c, L.G, c->habc.G));
  HIPCHECK(c, upload(c, L.H, c->habc.H));
  HIPCHECK(c, upload(c, L.info0, h.info0));
  HIPCHECK(c, upload(c, L.nrm0, h.nrm0));
  {
    const int n3 = 3 * c->P * c->P;
    std::vector<double> Tt((size_t)n3 * n3);
    for (int r = 0; r < n3; ++r)
      for (int k = 0; k < n3; ++k) Tt[(size_t)k * n3 + r] = c->habc.T[(size_t)r * n3 + k];
    HIPCHECK(c, upload(c, L.T, Tt));
  }
  HIPCHECK(c, upload(c, L.ops2f, h.ops2f));
  fill_levels(c);
  c->cur = 0;
  c->src_slot.assign(c->n_shots, -1);
  {
    std::vector<double> par((size_t)c->n_shots * 4, 0.0);
    for (int k = 0; k < c->n_shots; ++k) par[4 * k] = -1.0;
    HIPCHECK(c, upload(c, L.srcp, par));
  }
  c->stage = S_BOUND;
  return DGH_OK;
}

dgh_status dgh_set_state(dgh_ctx* c, int shot, const double* const* arr) {
  if (!c) return DGH_EINVAL;
  if (c->stage < S_BOUND) return fail(c, DGH_ESTATE, "set_state before bind");
  if (shot < 0 || shot >= c->n_shots) return fail(c, DGH_EINVAL, "shot out of range");
  const dgh::Mesh& m = c->mesh;
  const Layout& L = c->lay;
  const int Np = m.tet.Np;
  const int cur = c->cur;
  HIPCHECK(c, hipStreamSynchronize(c->stream));   // no step still reads or writes the state
  std::vector<double> buf((size_t)c->ntile * 4 * Np * dgh::kTile);
  for (int which : {DGH_Q3, DGH_RES3}) {
    if (arr && arr[which])
      to_tiles(arr[which], buf.data(), c->slot2elem, Np);
    else
      std::fill(buf.begin(), buf.end(), 0.0);   // a missing array is zero
    const Region& r = which == DGH_Q3 ? L.q3[cur] : L.res3;
    char* dst = c->ws + r.off + shot * L.st3 * L.e3;
    if (L.e3 == 4) {   // FP32 state: rounded on upload
      std::vector<float> f(buf.begin(), buf.end());
      HIPCHECK(c, h2d(c, dst, f.data(), f.size() * sizeof(float)));
    } else {
      HIPCHECK(c, h2d(c, dst, buf.data(), buf.size() * sizeof(double)));
    }
  }
  struct Item { int idx; const Region* r; size_t n, stride; };
  const int P = c->P;
  const Item items[] = {
      {DGH_Q2, &L.q2[cur], (size_t)m.Ktri * P * 3 * m.tri.Np, L.st2},
      {DGH_RES2, &L.res2, (size_t)m.Ktri * P * 3 * m.tri.Np, L.st2},
      {DGH_QB3, &L.qb3, (size_t)m.Ktri * m.tri.Np, L.stb3},
      {DGH_Q03, &L.q03, (size_t)m.Ktri * m.tri.Np, L.stb3},
      {DGH_Q1, &L.q1[cur], (size_t)m.Klin * P * P * 2 * m.line.Np, L.st1},
      {DGH_RES1, &L.res1, (size_t)m.Klin * P * P * 2 * m.line.Np, L.st1},
      {DGH_QB2, &L.qb2, (size_t)m.Klin * 2 * P * m.line.Np, L.stb2},
      {DGH_Q02, &L.q02, (size_t)m.Klin * 2 * P * m.line.Np, L.stb2},
      {DGH_QB1, &L.qb1, (size_t)m.Kpnt * 3 * P * P, L.stb1},
  };
  for (const Item& it : items) {
    if (it.n == 0) continue;
    char* dst = c->ws + it.r->off + shot * it.stride * sizeof(double);
    if (arr && arr[it.idx]) {
      HIPCHECK(c, h2d(c, dst, arr[it.idx], it.n * sizeof(double)));
    } else {
      HIPCHECK(c, dzero(c, dst, it.n * sizeof(double)));
    }
  }
  // a new state has no past: the closure's trace history starts at zero
  const size_t nn = (size_t)m.Ktri * m.tri.Np;
  if (nn > 0)
    HIPCHECK(c, dzero(c, c->ws + L.hist.off + shot * nn * 10 * sizeof(float),
                      nn * 10 * sizeof(float)));
  return DGH_OK;
}

dgh_status dgh_read_fields(dgh_ctx* c, int shot, double* const* arr) {
  if (!c || !arr) return DGH_EINVAL;
  if (c->stage < S_BOUND) return fail(c, DGH_ESTATE, "read before bind");
  if (shot < 0 || shot >= c->n_shots) return fail(c, DGH_EINVAL, "shot out of range");
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  const dgh::Mesh& m = c->mesh;
  const Layout& L = c->lay;
  const int Np = m.tet.Np, cur = c->cur, P = c->P;
  std::vector<double> buf((size_t)c->ntile * 4 * Np * dgh::kTile);
  for (int which : {DGH_Q3, DGH_RES3}) {
    if (!arr[which]) continue;
    const Region& r = which == DGH_Q3 ? L.q3[cur] : L.res3;
    const char* src = c->ws + r.off + shot * L.st3 * L.e3;
    if (L.e3 == 4) {
      std::vector<float> f(buf.size());
      HIPCHECK(c, d2h(c, f.data(), src, f.size() * sizeof(float)));
      std::copy(f.begin(), f.end(), buf.begin());
    } else {
      HIPCHECK(c, d2h(c, buf.data(), src, buf.size() * sizeof(double)));
    }
    from_tiles(buf.data(), arr[which], c->slot2elem, Np);
  }
  struct Item { int idx; const Region* r; size_t n, stride; };
  const Item items[] = {
      {DGH_Q2, &L.q2[cur], (size_t)m.Ktri * P * 3 * m.tri.Np, L.st2},
      {DGH_RES2, &L.res2, (size_t)m.Ktri * P * 3 * m.tri.Np, L.st2},
      {DGH_QB3, &L.qb3, (size_t)m.Ktri * m.tri.Np, L.stb3},
      {DGH_Q03, &L.q03, (size_t)m.Ktri * m.tri.Np, L.stb3},
      {DGH_Q1, &L.q1[cur], (size_t)m.Klin * P * P * 2 * m.line.Np, L.st1},
      {DGH_RES1, &L.res1, (size_t)m.Klin * P * P * 2 * m.line.Np, L.st1},
      {DGH_QB2, &L.qb2, (size_t)m.Klin * 2 * P * m.line.Np, L.stb2},
      {DGH_Q02, &L.q02, (size_t)m.Klin * 2 * P * m.line.Np, L.stb2},
      {DGH_QB1, &L.qb1, (size_t)m.Kpnt * 3 * P * P, L.stb1},
  };
  for (const Item& it : items)
    if (arr[it.idx] && it.n)
      HIPCHECK(c, d2h(c, arr[it.idx], c->ws + it.r->off + shot * it.stride * sizeof(double),
                      it.n * sizeof(double)));
  return DGH_OK;
}

dgh_status dgh_set_source(dgh_ctx* c, int shot, const double* xs, double f0, double t0, double amp) {
  if (!c || !xs) return DGH_EINVAL;
  if (c->stage < S_BOUND) return fail(c, DGH_ESTATE, "set_source before bind");
  if (shot < 0 || shot >= c->n_shots) return fail(c, DGH_EINVAL, "shot out of range");
  if (!std::isfinite(f0) || !std::isfinite(t0) || !std::isfinite(amp))
    return fail(c, DGH_EINVAL, "source parameters must be finite");
  HIPCHECK(c, hipStreamSynchronize(c->stream));   // no step still reads the source
  if (amp == 0.0) {
    c->src_slot[shot] = -1;
    const double par[4] = {-1.0, 0.0, 0.0, 0.0};
    HIPCHECK(c, h2d(c, c->ws + c->lay.srcp.off + (size_t)shot * 4 * sizeof(double), par,
                    sizeof(par)));
    return DGH_OK;
  }
  const dgh::Mesh& m = c->mesh;
  // the element whose smallest barycentric coordinate of xs is largest
  int best = -1;
  double bmin = -1e300, lam_best[3] = {0, 0, 0};
  for (int e = 0; e < m.K; ++e) {
    const double* g = &m.geo[9 * e];  // rows grad r, grad s, grad t
    const double* v0 = &m.VX[3 * m.EToV[4 * e]];
    double d[3] = {xs[0] - v0[0], xs[1] - v0[1], xs[2] - v0[2]};
    // (r+1)/2 = grad r . d / 2 ... since x - v0 = sum_k (xi_k + 1)/2 (v_k - v0)
    double lam[3];
    for (int k = 0; k < 3; ++k) lam[k] = 0.5 * (g[3 * k] * d[0] + g[3 * k + 1] * d[1] + g[3 * k + 2] * d[2]);
    const double l0 = 1.0 - lam[0] - lam[1] - lam[2];
    const double mn = std::min(std::min(l0, lam[0]), std::min(lam[1], lam[2]));
    if (mn > bmin) {
      bmin = mn;
      best = e;
      for (int k = 0; k < 3; ++k) lam_best[k] = lam[k];
    }
  }
  if (bmin < -1e-9) return fail(c, DGH_EINVAL, "source outside the mesh");
  const int Np = m.tet.Np;
  std::vector<double> psi(Np), w(Np, 0.0);
  dgh::tet_basis_at(m.N, 2 * lam_best[0] - 1, 2 * lam_best[1] - 1, 2 * lam_best[2] - 1, psi.data());
  for (int a = 0; a < Np; ++a) {
    for (int k = 0; k < Np; ++k) w[a] += m.tet.V[a * Np + k] * psi[k];
    w[a] /= m.J[best];
  }
  HIPCHECK(c, h2d(c, c->ws + c->lay.srcw.off + (size_t)shot * Np * sizeof(double), w.data(),
                  Np * sizeof(double)));
  c->src_slot[shot] = c->elem2slot[best];
  const double par[4] = {(double)c->src_slot[shot], f0, t0, amp};
  HIPCHECK(c, h2d(c, c->ws + c->lay.srcp.off + (size_t)shot * 4 * sizeof(double), par,
                  sizeof(par)));
  return DGH_OK;
}

}  // extern "C"

namespace {

// The 3D level of one stage in the context's arithmetic: reads q3[o],
// writes q3[n] and the residual `res` (which may alias q3[n] when timing).
hipError_t launch3d(dgh_ctx* c, int o, int n, const Region& res, double A, double B, double dt,
                    const dgh::Shots& sh, hipStream_t st) {
  const Layout& L = c->lay;
  if (c->precision == DGH_BF16_MFMA)
    return dgh::launch_level3_bf16(c->L3, dptr<float>(c, L.q3[o]), dptr<float>(c, L.q3[n]),
                                   dptr<float>(c, res), dptr<double>(c, L.qb3), A, B, dt, sh, st);
  if (c->precision == DGH_FP32_MFMA)
    return dgh::launch_level3_f32(c->L3, dptr<float>(c, L.q3[o]), dptr<float>(c, L.q3[n]),
                                  dptr<float>(c, res), dptr<double>(c, L.qb3), A, B, dt, sh, st);
  return dgh::launch_level3(c->L3, dptr<double>(c, L.q3[o]), dptr<double>(c, L.q3[n]),
                            dptr<double>(c, res), dptr<double>(c, L.qb3), A, B, dt, sh, st);
}

// The closure's time scales: as set, or by default 1.25, 2.5, 5 and 10
// times h / c_max, with h = (6 |Omega| / K)^(1/3) the edge of a cube cell of
// the mesh's mean element volume (the Kuhn cell size).
const double* memory_tau(dgh_ctx* c) {
  if (c->mem_tau[0] > 0.0) return c->mem_tau;
  static thread_local double tau[dgh::kMemScales];
  const dgh::Mesh& m = c->mesh;
  double vol = 0.0, cmax = 0.0;
  for (int e = 0; e < m.K; ++e) vol += m.J[e] * (4.0 / 3.0);
  for (double v : c->c) cmax = std::max(cmax, v);
  const double h = std::cbrt(6.0 * vol / std::max(1, m.K));
  for (int k = 0; k < dgh::kMemScales; ++k) tau[k] = 1.25 * (double)(1 << k) * h / cmax;
  return tau;
}

// One step (5 stages, Algorithm 1 order) on `st`.  Eager: the stage times
// come from t; replayed (clk non-null): from the device clock, which the
// step advances at its end.
dgh_status enqueue_step(dgh_ctx* c, double dt, double t, hipStream_t st, double* clk) {
  const Layout& L = c->lay;
  dgh::Shots sh{c->n_shots, L.st3, L.st2, L.stb3, L.st1, L.stb2, L.stb1,
                dptr<double>(c, L.srcw), dptr<double>(c, L.srcp), 0.0, clk, 0.0, dt};
  const bool timed = c->timing && !clk;
  for (int s = 0; s < 5; ++s) {
    const int o = c->cur, n = 1 - c->cur;
    sh.tau = t + kC[s] * dt;
    sh.cs = kC[s];
    if (timed) {
      if (c->ev_used + 2 > c->ev.size()) {
        for (int k = 0; k < 64; ++k) {
          hipEvent_t e;
          HIPCHECK(c, hipEventCreate(&e));
          c->ev.push_back(e);
        }
      }
      HIPCHECK(c, hipEventRecord(c->ev[c->ev_used], st));
    }
    HIPCHECK(c, launch3d(c, o, n, L.res3, kA[s], kB[s], dt, sh, st));
    if (timed) {
      HIPCHECK(c, hipEventRecord(c->ev[c->ev_used + 1], st));
      c->ev_used += 2;
    }
    if (!c->closure) {   // with the closure, qb3 holds from the last step end
      const dgh::FaceBufs fb{dptr<double>(c, L.q2[o]), dptr<double>(c, L.q2[n]),
                             dptr<double>(c, L.res2), dptr<double>(c, L.qb3),
                             dptr<double>(c, L.q03), c->ws + L.q3[n].off,
                             dptr<double>(c, L.qb2), L.e3 == 4 ? 1 : 0};
      HIPCHECK(c, dgh::launch_faces(c->LF, c->L2, fb, sh, kA[s], kB[s], dt, st));
    }
    HIPCHECK(c, dgh::launch_boundary(c->L2, c->L1, c->L0, c->L3, dptr<double>(c, L.q2[o]),
                                     dptr<double>(c, L.q2[n]), dptr<double>(c, L.res2),
                                     dptr<double>(c, L.qb2), dptr<double>(c, L.qb3),
                                     dptr<double>(c, L.q03), dptr<double>(c, L.q3[n]),
                                     dptr<double>(c, L.q1[o]), dptr<double>(c, L.q1[n]),
                                     dptr<double>(c, L.res1), dptr<double>(c, L.qb1),
                                     dptr<double>(c, L.q02), kA[s], kB[s], dt, sh, st));
    c->cur = n;
  }
  if (c->closure || c->record) {
    dgh::Memory mem;
    const double* tau = memory_tau(c);
    for (int k = 0; k < dgh::kMemScales; ++k) mem.decay[k] = (float)std::exp(-dt / tau[k]);
    if (c->closure)
      HIPCHECK(c, dgh::launch_closure(c->L2, dptr<float>(c, L.mlpw), c->ws + L.q3[c->cur].off,
                                      L.e3 == 4 ? 1 : 0, c->mesh.tet.Np, dptr<float>(c, L.hist),
                                      dptr<double>(c, L.qb3), dptr<double>(c, L.q03), sh, mem,
                                      st));
    else
      HIPCHECK(c, dgh::launch_hist_push(c->L2, c->ws + L.q3[c->cur].off, L.e3 == 4 ? 1 : 0,
                                        c->mesh.tet.Np, dptr<float>(c, L.hist), sh, mem, st));
  }
  if (clk) HIPCHECK(c, dgh::launch_clock_tick(clk, st));
  return DGH_OK;
}

void drop_graphs(dgh_ctx* c) {
  for (int p = 0; p < 2; ++p) {
    if (c->gx[p]) (void)hipGraphExecDestroy(c->gx[p]);
    if (c->g[p]) (void)hipGraphDestroy(c->g[p]);
    c->gx[p] = nullptr;
    c->g[p] = nullptr;
  }
}

// Captures one step for each starting buffer parity (5 stages flip the
// double buffers, so consecutive steps alternate between the two graphs).
dgh_status capture_steps(dgh_ctx* c, double dt) {
  drop_graphs(c);
  if (!c->cap) HIPCHECK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  const int saved = c->cur;
  double* clk = dptr<double>(c, c->lay.clk);
  for (int p = 0; p < 2; ++p) {
    c->cur = p;
    HIPCHECK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
    const dgh_status st = enqueue_step(c, dt, 0.0, c->cap, clk);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap, &g);
    c->g[p] = g;
    if (st != DGH_OK) {
      c->cur = saved;
      drop_graphs(c);
      return st;
    }
    if (e != hipSuccess) {
      c->cur = saved;
      drop_graphs(c);
      return hipfail(c, e, "hipStreamEndCapture");
    }
    const hipError_t ei = hipGraphInstantiate(&c->gx[p], g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      c->cur = saved;
      drop_graphs(c);
      return hipfail(c, ei, "hipGraphInstantiate");
    }
  }
  c->cur = saved;
  c->gdt = dt;
  c->gclosure = c->closure;
  c->grecord = c->record;
  return DGH_OK;
}

}  // namespace

extern "C" {

dgh_status dgh_step(dgh_ctx* c, int n_steps, double dt, double t_start) {
  if (!c) return DGH_EINVAL;
  if (c->stage < S_BOUND) return fail(c, DGH_ESTATE, "step before bind");
  if (n_steps < 0 || !(dt > 0) || !std::isfinite(dt) || !std::isfinite(t_start))
    return fail(c, DGH_EINVAL, "bad step arguments");
  if (n_steps == 0) return DGH_OK;
  if (c->graph && !c->timing) {
    if (!c->gx[0] || c->gdt != dt || c->gclosure != c->closure || c->grecord != c->record) {
      const dgh_status st = capture_steps(c, dt);
      if (st != DGH_OK) return st;
    }
    double* clk = dptr<double>(c, c->lay.clk);
    HIPCHECK(c, dgh::launch_clock_set(clk, t_start, c->stream));
    for (int it = 0; it < n_steps; ++it) {
      HIPCHECK(c, hipGraphLaunch(c->gx[c->cur], c->stream));
      c->cur = 1 - c->cur;
    }
    return DGH_OK;
  }
  for (int it = 0; it < n_steps; ++it) {
    const dgh_status st = enqueue_step(c, dt, t_start + it * dt, c->stream, nullptr);
    if (st != DGH_OK) return st;
  }
  return DGH_OK;
}

namespace {
// tuning candidates: three 3D kernels where the tile fits on chip (FP64
// N <= 4, FP32 and BF16 N <= 5): tile on chip, register streaming with 4
// and with 8 waves (64 or 128 elements) per workgroup; else the two
// register-streaming ones, the default first; x two item orders; x three
// persistent grid sizes (8, 6 or 4 eighths of the resident workgroups);
// candidate = (kernel * 2 + order) * 3 + grid
constexpr int kGrids[3] = {8, 6, 4};
bool tile_on_chip(const dgh_ctx* c) { return c->N <= (c->precision == DGH_FP64 ? 4 : 5); }
int tuning_count(const dgh_ctx* c) { return (tile_on_chip(c) ? 3 : 2) * 6; }
void apply_tuning(dgh_ctx* c, int candidate) {
  const int kern = candidate / 6, dw = default_waves(c);
  if (tile_on_chip(c)) {
    c->L3.kvar = kern == 0 ? 0 : 1;
    c->L3.waves = kern == 0 ? dw : (kern == 1 ? 4 : 8);
  } else {
    c->L3.kvar = 1;
    c->L3.waves = kern == 0 ? dw : 12 - dw;
  }
  c->L3.order = (candidate / 3) & 1;
  c->L3.eighths = kGrids[candidate % 3];
}
}  // namespace

dgh_status dgh_tuning_count(dgh_ctx* c, int* count) {
  if (!c || !count) return DGH_EINVAL;
  if (c->stage < S_BOUND) return fail(c, DGH_ESTATE, "tuning before bind");
  *count = tuning_count(c);
  return DGH_OK;
}

dgh_status dgh_set_tuning(dgh_ctx* c, int candidate) {
  if (!c) return DGH_EINVAL;
  if (c->stage < S_BOUND) return fail(c, DGH_ESTATE, "tuning before bind");
  if (candidate < 0 || candidate >= tuning_count(c)) return fail(c, DGH_EINVAL, "no such candidate");
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  apply_tuning(c, candidate);
  drop_graphs(c);   // captured launches carry the old choice
  return DGH_OK;
}

dgh_status dgh_autotune(dgh_ctx* c, int launches, int* best, double* ms) {
  if (!c || !best) return DGH_EINVAL;
  if (c->stage < S_BOUND) return fail(c, DGH_ESTATE, "autotune before bind");
  if (launches < 1 || launches > 10000) return fail(c, DGH_EINVAL, "launches out of range");
  const Layout& L = c->lay;
  const int nc = tuning_count(c), cur = c->cur;
  // the 3D level of the first stage, reading the current state and writing
  // only the other half of the double buffer (as its residual too), so the
  // state is left as it was
  dgh::Shots sh{c->n_shots, L.st3, L.st2, L.stb3, L.st1, L.stb2, L.stb1,
                dptr<double>(c, L.srcw), dptr<double>(c, L.srcp), 0.0, nullptr, 0.0, 1e-6};
  hipEvent_t e0, e1;
  HIPCHECK(c, hipEventCreate(&e0));
  HIPCHECK(c, hipEventCreate(&e1));
  const int keep_kvar = c->L3.kvar, keep_order = c->L3.order, keep_eighths = c->L3.eighths,
            keep_waves = c->L3.waves;
  double tbest = 0.0;
  int ibest = -1;
  hipError_t err = hipSuccess;
  for (int k = 0; k < nc && err == hipSuccess; ++k) {
    apply_tuning(c, k);
    auto launch = [&]() {
      return launch3d(c, cur, 1 - cur, L.q3[1 - cur], kA[0], kB[0], 1e-6, sh, c->stream);
    };
    for (int w = 0; w < 2 && err == hipSuccess; ++w) err = launch();
    if (err == hipSuccess) err = hipEventRecord(e0, c->stream);
    for (int r = 0; r < launches && err == hipSuccess; ++r) err = launch();
    if (err == hipSuccess) err = hipEventRecord(e1, c->stream);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float t = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
    if (err == hipSuccess) {
      const double per = (double)t / launches;
      if (ms) ms[k] = per;
      if (ibest < 0 || per < tbest) {
        tbest = per;
        ibest = k;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) {
    c->L3.kvar = keep_kvar;
    c->L3.order = keep_order;
    c->L3.eighths = keep_eighths;
    c->L3.waves = keep_waves;
    return hipfail(c, err, "autotune");
  }
  apply_tuning(c, ibest);
  drop_graphs(c);
  *best = ibest;
  return DGH_OK;
}

dgh_status dgh_step_group(dgh_ctx* const* ctxs, int n, int n_steps, double dt, double t_start) {
  if (!ctxs || n < 1 || n > dgh::kMaxGroup) return DGH_EINVAL;
  dgh_ctx* c0 = ctxs[0];
  if (!c0) return DGH_EINVAL;
  for (int i = 0; i < n; ++i) {
    dgh_ctx* c = ctxs[i];
    if (!c) return DGH_EINVAL;
    if (c->stage < S_BOUND) return fail(c0, DGH_ESTATE, "group member not bound");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) return fail(c0, DGH_EINVAL, "a context appears twice in the group");
    if (c->N > 4 || c->L3.kvar != 0)
      return fail(c0, DGH_EINVAL, "group steps need N <= 4 and the tile-on-chip kernel");
    if (c->N != c0->N || c->precision != c0->precision || c->device != c0->device ||
        c->stream != c0->stream)
      return fail(c0, DGH_EINVAL, "group members need the same N, precision, device and stream");
    if (c->closure || c->record) return fail(c0, DGH_EINVAL, "group steps run the plain method");
  }
  if (n_steps < 0 || !(dt > 0) || !std::isfinite(dt) || !std::isfinite(t_start))
    return fail(c0, DGH_EINVAL, "bad step arguments");
  if (n_steps == 0) return DGH_OK;
  hipStream_t st = c0->stream;
  // member tables for both parities of the double buffers; the previous
  // group step may still read them, so the stream drains first
  std::vector<dgh::Member3> hd(2 * n);
  long long first = 0;
  for (int i = 0; i < n; ++i) {
    dgh_ctx* c = ctxs[i];
    const Layout& L = c->lay;
    // work items of 4 tiles: one per wave of the tile-on-chip kernels'
    // workgroups (4 waves in both the FP64 and the FP32 kernel)
    const int ngrp = (c->ntile + 3) / 4;
    for (int p = 0; p < 2; ++p) {
      const int o = c->cur ^ p;
      dgh::Member3& m = hd[p * n + i];
      m.L = c->L3;
      m.qo = c->ws + L.q3[o].off;
      m.qn = c->ws + L.q3[1 - o].off;
      m.res = c->ws + L.res3.off;
      m.qb3 = dptr<double>(c, L.qb3);
      m.sh = dgh::Shots{c->n_shots, L.st3, L.st2, L.stb3, L.st1, L.stb2, L.stb1,
                        dptr<double>(c, L.srcw), dptr<double>(c, L.srcp), 0.0, nullptr, 0.0, dt};
      m.first = first;
      m.ngrp = ngrp;
    }
    first += (long long)ngrp * c->n_shots;
  }
  const long long total = first;
  dgh::Member3* dev = dptr<dgh::Member3>(c0, c0->lay.grp);
  HIPCHECK(c0, hipStreamSynchronize(st));
  HIPCHECK(c0, hipMemcpyAsync(dev, hd.data(), hd.size() * sizeof(dgh::Member3),
                              hipMemcpyHostToDevice, st));
  HIPCHECK(c0, hipStreamSynchronize(st));
  for (int it = 0; it < n_steps; ++it) {
    const double t = t_start + it * dt;
    for (int s = 0; s < 5; ++s) {
      const int par = (it * 5 + s) & 1;
      if (c0->precision == DGH_BF16_MFMA)
        HIPCHECK(c0, dgh::launch_level3_bf16_group(dev + par * n, n, total, c0->N, kA[s], kB[s],
                                                   dt, t + kC[s] * dt, kC[s], st));
      else if (c0->lay.e3 == 4)
        HIPCHECK(c0, dgh::launch_level3_f32_group(dev + par * n, n, total, c0->N, kA[s], kB[s],
                                                  dt, t + kC[s] * dt, kC[s], st));
      else
        HIPCHECK(c0, dgh::launch_level3_group(dev + par * n, n, total, c0->N, kA[s], kB[s], dt,
                                              t + kC[s] * dt, kC[s], st));
      for (int i = 0; i < n; ++i) {
        dgh_ctx* c = ctxs[i];
        const Layout& L = c->lay;
        const int o = c->cur, nn = 1 - c->cur;
        const dgh::Shots sh{c->n_shots, L.st3, L.st2, L.stb3, L.st1, L.stb2, L.stb1,
                            dptr<double>(c, L.srcw), dptr<double>(c, L.srcp),
                            t + kC[s] * dt, nullptr, kC[s], dt};
        const dgh::FaceBufs fb{dptr<double>(c, L.q2[o]), dptr<double>(c, L.q2[nn]),
                               dptr<double>(c, L.res2), dptr<double>(c, L.qb3),
                               dptr<double>(c, L.q03), c->ws + L.q3[nn].off,
                               dptr<double>(c, L.qb2), L.e3 == 4 ? 1 : 0};
        HIPCHECK(c0, dgh::launch_faces(c->LF, c->L2, fb, sh, kA[s], kB[s], dt, st));
        HIPCHECK(c0, dgh::launch_boundary(c->L2, c->L1, c->L0, c->L3,
                                          dptr<double>(c, L.q2[o]), dptr<double>(c, L.q2[nn]),
                                          dptr<double>(c, L.res2), dptr<double>(c, L.qb2),
                                          dptr<double>(c, L.qb3), dptr<double>(c, L.q03),
                                          dptr<double>(c, L.q3[nn]), dptr<double>(c, L.q1[o]),
                                          dptr<double>(c, L.q1[nn]), dptr<double>(c, L.res1),
                                          dptr<double>(c, L.qb1), dptr<double>(c, L.q02), kA[s],
                                          kB[s], dt, sh, st));
        c->cur = nn;
      }
    }
  }
  return DGH_OK;
}

dgh_status dgh_set_graph(dgh_ctx* c, int enable) {
  if (!c) return DGH_EINVAL;
  if (c->stage < S_BOUND) return fail(c, DGH_ESTATE, "set_graph before bind");
  c->graph = enable != 0;
  if (!c->graph) drop_graphs(c);
  return DGH_OK;
}

dgh_status dgh_energy(dgh_ctx* c, int shot, double* e) {
  if (!c || !e) return DGH_EINVAL;
  if (c->stage < S_BOUND) return fail(c, DGH_ESTATE, "energy before bind");
  if (shot < 0 || shot >= c->n_shots) return fail(c, DGH_EINVAL, "shot out of range");
  const Layout& L = c->lay;
  HIPCHECK(c, dgh::launch_energy(c->L3, c->ws + L.q3[c->cur].off + shot * L.st3 * L.e3,
                                 L.e3 == 4 ? 1 : 0, dptr<double>(c, L.mass3),
                                 dptr<double>(c, L.J3), dptr<double>(c, L.esum), c->stream));
  std::vector<double> part(c->ntile);
  HIPCHECK(c, hipMemcpyAsync(part.data(), c->ws + L.esum.off, c->ntile * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  double s = 0.0;
  for (double v : part) s += v;
  *e = s;
  return DGH_OK;
}

dgh_status dgh_check(dgh_ctx* c, int shot, double e_ref, double rel_tol, double* e_out) {
  if (!c) return DGH_EINVAL;
  if (c->stage < S_BOUND) return fail(c, DGH_ESTATE, "check before bind");
  if (shot < 0 || shot >= c->n_shots) return fail(c, DGH_EINVAL, "shot out of range");
  if (!(rel_tol >= 0.0)) return fail(c, DGH_EINVAL, "rel_tol must be >= 0");
  const dgh::Mesh& m = c->mesh;
  const Layout& L = c->lay;
  const int cur = c->cur, P = c->P, Np = m.tet.Np;
  const size_t n3 = (size_t)c->ntile * 4 * Np * dgh::kTile;
  const Region* regs[] = {&L.q3[cur], &L.res3, &L.q2[cur], &L.res2, &L.qb3, &L.q03,
                          &L.q1[cur], &L.res1, &L.qb2, &L.q02, &L.qb1};
  const size_t strides[] = {L.st3, L.st3, L.st2, L.st2, L.stb3, L.stb3,
                            L.st1, L.st1, L.stb2, L.stb2, L.stb1};
  const size_t ns[] = {n3, n3,
                       (size_t)m.Ktri * P * 3 * m.tri.Np, (size_t)m.Ktri * P * 3 * m.tri.Np,
                       (size_t)m.Ktri * m.tri.Np, (size_t)m.Ktri * m.tri.Np,
                       (size_t)m.Klin * P * P * 2 * m.line.Np,
                       (size_t)m.Klin * P * P * 2 * m.line.Np,
                       (size_t)m.Klin * 2 * P * m.line.Np, (size_t)m.Klin * 2 * P * m.line.Np,
                       (size_t)m.Kpnt * 3 * P * P};
  dgh::ScanList sl{};
  for (int a = 0; a < DGH_NARRAYS; ++a)
    if (ns[a] > 0) {
      const size_t eb = a < 2 ? L.e3 : sizeof(double);
      sl.ptr[sl.count] = c->ws + regs[a]->off + shot * strides[a] * eb;
      sl.f32[sl.count] = eb == 4 ? 1 : 0;
      sl.n[sl.count] = ns[a];
      ++sl.count;
    }
  HIPCHECK(c, dgh::launch_nonfinite(sl, dptr<int>(c, L.flags), c->stream));
  std::vector<int> fl((size_t)sl.count * dgh::kScanBlocks);
  if (!fl.empty())
    HIPCHECK(c, hipMemcpyAsync(fl.data(), c->ws + L.flags.off, fl.size() * sizeof(int),
                               hipMemcpyDeviceToHost, c->stream));
  double e = 0.0;
  const dgh_status st = dgh_energy(c, shot, &e);  // synchronises the stream
  if (st != DGH_OK) return st;
  if (e_out) *e_out = e;
  for (int f : fl)
    if (f) return fail(c, DGH_ENONFINITE, "non-finite value in the state");
  if (!std::isfinite(e)) return fail(c, DGH_ENONFINITE, "non-finite energy");
  if (e_ref > 0.0 && e > e_ref * (1.0 + rel_tol))
    return fail(c, DGH_EUNSTABLE, "energy grew beyond the reference");
  return DGH_OK;
}

dgh_status dgh_set_closure(dgh_ctx* c, const float* w, int n_w) {
  if (!c) return DGH_EINVAL;
  if (c->stage < S_BOUND) return fail(c, DGH_ESTATE, "set_closure before bind");
  if (n_w == 0) {
    c->closure = false;
    return DGH_OK;
  }
  if (!w || n_w != dgh::kMlpParams) return fail(c, DGH_EINVAL, "closure needs DGH_CLOSURE_PARAMS floats");
  if (c->P != 0) return fail(c, DGH_EINVAL, "the closure replaces the auxiliary fields: set P = 0");
  for (int i = 0; i < n_w; ++i)
    if (!std::isfinite(w[i])) return fail(c, DGH_EINVAL, "closure parameters must be finite");
  if (!(std::fabs(w[1]) <= 1.0f))
    return fail(c, DGH_EINVAL, "closure gain bound |g_max| must not exceed 1");
  HIPCHECK(c, hipStreamSynchronize(c->stream));   // no step still reads the weights
  HIPCHECK(c, h2d(c, c->ws + c->lay.mlpw.off, w, (size_t)n_w * sizeof(float)));
  c->closure = true;
  return DGH_OK;
}

dgh_status dgh_set_closure_memory(dgh_ctx* c, const double* tau) {
  if (!c) return DGH_EINVAL;
  if (c->stage < S_BOUND) return fail(c, DGH_ESTATE, "set_closure_memory before bind");
  if (tau)
    for (int k = 0; k < dgh::kMemScales; ++k)
      if (!(tau[k] > 0.0) || !std::isfinite(tau[k]))
        return fail(c, DGH_EINVAL, "closure time scales must be positive and finite");
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < dgh::kMemScales; ++k) c->mem_tau[k] = tau ? tau[k] : 0.0;
  drop_graphs(c);   // captured launches carry the old decay factors
  return DGH_OK;
}

dgh_status dgh_closure_record(dgh_ctx* c, int enable) {
  if (!c) return DGH_EINVAL;
  if (c->stage < S_BOUND) return fail(c, DGH_ESTATE, "closure_record before bind");
  c->record = enable != 0;
  return DGH_OK;
}

dgh_status dgh_closure_sample(dgh_ctx* c, int shot, float* x, float* y) {
  if (!c || !x || !y) return DGH_EINVAL;
  if (c->stage < S_BOUND) return fail(c, DGH_ESTATE, "closure_sample before bind");
  if (shot < 0 || shot >= c->n_shots) return fail(c, DGH_EINVAL, "shot out of range");
  const Layout& L = c->lay;
  const dgh::Mesh& m = c->mesh;
  const size_t nn = (size_t)m.Ktri * m.tri.Np;
  if (nn == 0) return DGH_OK;
  float* X = dptr<float>(c, L.csamp);
  float* Y = X + nn * 11;
  HIPCHECK(c, dgh::launch_closure_sample(
                  c->L2, c->ws + L.q3[c->cur].off + shot * L.st3 * L.e3, L.e3 == 4 ? 1 : 0,
                  m.tet.Np, dptr<float>(c, L.hist) + shot * nn * 10,
                  dptr<double>(c, L.qb3) + shot * L.stb3, X, Y, c->stream));
  HIPCHECK(c, hipMemcpyAsync(x, X, nn * 11 * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIPCHECK(c, hipMemcpyAsync(y, Y, nn * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  return DGH_OK;
}

dgh_status dgh_mlp_work_size(int batch, size_t* floats) {
  if (batch <= 0 || !floats) return DGH_EINVAL;
  *floats = dgh::mlp_work_floats(batch);
  return DGH_OK;
}

dgh_status dgh_mlp_forward(const float* W, const float* X, int n, float* Y, void* stream) {
  if (!W || (n > 0 && (!X || !Y)) || n < 0) return DGH_EINVAL;
  return dgh::mlp_forward(W, X, n, Y, static_cast<hipStream_t>(stream)) == hipSuccess ? DGH_OK
                                                                                    : DGH_EHIP;
}

dgh_status dgh_mlp_grad(const float* W, const float* X, const float* T, int n, float* G,
                        float* work, double* loss, void* stream) {
  if (!W || !X || !T || !G || !work || n <= 0) return DGH_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dgh::mlp_grad(W, X, T, n, G, work, st) != hipSuccess) return DGH_EHIP;
  if (loss) {
    const int nb = (n + 255) / 256;
    std::vector<float> part(nb);
    if (hipMemcpyAsync(part.data(), dgh::mlp_loss_partials(work, n), nb * sizeof(float),
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return DGH_EHIP;
    double sum = 0.0;
    for (float v : part) sum += v;
    *loss = sum / n;
  }
  return DGH_OK;
}

dgh_status dgh_mlp_grad_bf16(const float* W, const float* X, const float* T, int n, float* G,
                             float* work, double* loss, void* stream) {
  if (!W || !X || !T || !G || !work || n <= 0) return DGH_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dgh::mlp_grad_bf16(W, X, T, n, G, work, st) != hipSuccess) return DGH_EHIP;
  if (loss) {
    const int nb = (n + 63) / 64;
    std::vector<float> part(nb);
    if (hipMemcpyAsync(part.data(), dgh::mlp_loss_partials_bf16(work, n), nb * sizeof(float),
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return DGH_EHIP;
    double sum = 0.0;
    for (float v : part) sum += v;
    *loss = sum / n;
  }
  return DGH_OK;
}

dgh_status dgh_mlp_grad_static(const float* W, const float* X, const float* T, int n, float* G,
                               double* loss, void* stream) {
  static_assert(dgh::kMlpStaticBatch == DGH_MLP_STATIC_BATCH, "header and library agree");
  if (!W || !X || !T || !G || n <= 0 || n > DGH_MLP_STATIC_BATCH) return DGH_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* work = nullptr;
  if (dgh::mlp_static_work(st, &work) != hipSuccess) return DGH_EHIP;
  if (dgh::mlp_grad(W, X, T, n, G, work, st) != hipSuccess) return DGH_EHIP;
  if (loss) {
    constexpr int kParts = (DGH_MLP_STATIC_BATCH + 255) / 256;
    float part[kParts];
    const int nb = (n + 255) / 256;
    if (hipMemcpyAsync(part, dgh::mlp_loss_partials(work, n), nb * sizeof(float),
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return DGH_EHIP;
    double sum = 0.0;
    for (int b = 0; b < nb; ++b) sum += part[b];
    *loss = sum / n;
  }
  return DGH_OK;
}

dgh_status dgh_mlp_adam(float* W, const float* G, float* M, float* V, int t, float lr,
                        void* stream) {
  if (!W || !G || !M || !V || t < 1 || !(lr > 0)) return DGH_EINVAL;
  return dgh::mlp_adam(W, G, M, V, t, lr, 0.9f, 0.999f, 1e-8f, static_cast<hipStream_t>(stream)) ==
                 hipSuccess
             ? DGH_OK
             : DGH_EHIP;
}

dgh_status dgh_kernel_timing(dgh_ctx* c, int enable) {
  if (!c) return DGH_EINVAL;
  if (c->stage < S_BOUND) return fail(c, DGH_ESTATE, "timing before bind");
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  c->timing = enable != 0;
  if (enable) c->ev_used = 0;
  return DGH_OK;
}

dgh_status dgh_kernel_time(dgh_ctx* c, int level, double* total_ms, long long* launches) {
  if (!c || !total_ms || !launches) return DGH_EINVAL;
  if (level != 3) return fail(c, DGH_EINVAL, "only the 3D level is timed");
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  double t = 0.0;
  for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
    float ms = 0.f;
    HIPCHECK(c, hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]));
    t += ms;
  }
  *total_ms = t;
  *launches = (long long)(c->ev_used / 2);
  return DGH_OK;
}

const char* dgh_last_error(const dgh_ctx* c) { return c ? c->err.c_str() : "null context"; }

void dgh_destroy(dgh_ctx* c) {
  if (!c) return;
  drop_graphs(c);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"
