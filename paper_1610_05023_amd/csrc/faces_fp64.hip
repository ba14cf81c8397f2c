// FP64 face level (the 2D systems of the HABC faces, Section 2.3 and
// Algorithm 3) on the FP64 4x4x4 MFMA: one wave updates the P auxiliary
// sets of TW = 16 / P consecutive triangles (MFMA column es = local
// triangle * P + set), then applies the face rule.  Every load of a wave is
// issued before its first MFMA, in two dependent rounds: the wave's q2 and
// res2 spans (direct buffer-to-LDS loads) with the triangle data, then what
// the maps point to.
//
// Per triangle and set i, with K_i = rho c^2 / (1 + g_i) and the in-plane
// reference gradients (rx, ry), (sx, sy):
//   d p*_i/dt = -K_i div v_i + LIFT [fsc K_i (v.n^- - (v.n)*)]
//   d v_i/dt  = -(1/rho) grad p_i + LIFT [fsc (1/rho) (p^- - p*)] n
// with the upwind flux against the neighbouring triangle (same set), the
// characteristic condition r- = qb2 at an HABC edge, r- = 0 at a basic-ABC
// edge, or p = 0; then res = A res + dt rhs, p*_i = p_i - q0_3 + B res_p,
// v_i = v_i + B res_v, and from the new 3D trace: r+ = (p3 + Z n.u3)/2,
// r- = (1/M) sum_i g_i p*_i -> qb3, S = r+ + r- -> q0_3, p_i = p*_i + S.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"
#include "launch.hpp"
#include "levels.hpp"

namespace dgh {

namespace {

constexpr int kWaves2 = 4;   // waves per workgroup

template <int N>
struct Dims2 {
  static constexpr int Np = (N + 1) * (N + 2) / 2;
  static constexpr int Nfp = N + 1;
  static constexpr int RG = (Np + 3) / 4;    // row groups, also volume k-steps
  static constexpr int EK = (Nfp + 3) / 4;   // lifting k-steps per edge
  static constexpr int NFRAG = 2 * RG * RG + RG * 3 * EK;
  static constexpr int SPAN = 16 * 3 * Np;   // doubles of at most 16 (triangle, set) pairs
  // bytes of one LDS copy of a span (q2 or res2): whole 1 KB chunks of the
  // direct loads, with room for a span starting 8 bytes past a 16-byte boundary
  static constexpr int SB = ((SPAN + 1) * 8 + 1023) / 1024 * 1024;
  static constexpr int EB = 16 * 24 * 8;     // edge constants of at most 16 triangles
  static constexpr int STAGE = 2 * SB + EB;  // per wave: q2, res2, edge constants
};

typedef __attribute__((address_space(3))) void* lds_ptr;
using Rsrc = __amdgpu_buffer_rsrc_t;

// Raw buffer descriptor over [p, p + bytes): loads past the end read 0.
__device__ __forceinline__ Rsrc span_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           0x00020000);
}

// One work item: the kWaves2 wave slots of group bx of shot k (each wave
// its TW triangles).  T3: type of the 3D state (double, or float for the
// FP32 3D variant).
template <int N, class T3>
__device__ __forceinline__ void faces_item(const LvlF& F, const Lvl2& L2, FaceBufs b,
                                           const Shots& sh, double A, double B, double dt,
                                           int bx, int k, const double* sops, const double* sg,
                                           const int* smask, char* stage) {
  using D = Dims2<N>;
  constexpr int Np = D::Np, Nfp = D::Nfp, RG = D::RG, EK = D::EK;
  constexpr int KL = (D::SPAN + 63) / 64;    // 64-lane chunks of a span
  const int P = L2.P;
  {
    b.q2o += k * sh.st2;
    b.q2n += k * sh.st2;
    b.res2 += k * sh.st2;
    b.qb3 += k * sh.stb3;
    b.q03 += k * sh.stb3;
    b.q3n = static_cast<const T3*>(b.q3n) + k * sh.st3;
    b.qb2 += (size_t)k * sh.stb2;
  }
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int es = lane & 15, g = lane >> 4;
  const int ta = (lane & 3) + 4 * g;         // lane's entry of an A fragment
  const int Pc = P > 0 ? P : 1, TW = 16 / Pc;
  const int tl = es / Pc, i = es - tl * Pc;
  const int w0 = (bx * kWaves2 + wv) * TW;           // first triangle of this wave
  if (w0 >= L2.Kt) return;
  const int ntw = min(TW, L2.Kt - w0);               // triangles of this wave
  const bool col = tl < ntw;                         // column holds (triangle, set)
  const int t = w0 + min(tl, ntw - 1);
  const int ic = P > 0 ? i : 0;
  // ---- the wave's pairs are contiguous in q2 and res2: copied into this
  // wave's LDS stage by direct buffer-to-LDS loads (16 bytes per lane from
  // the 16-byte boundary at or before the span; the descriptors end with the
  // span) and, at the end, stored back with linear (coalesced) stores
  char* stq = stage + (size_t)wv * D::STAGE;
  char* str = stq + D::SB;
  char* ste = str + D::SB;
  const int cnt = ntw * P * 3 * Np;
  const size_t wbase = (size_t)w0 * P * 3 * Np;
  const int shq = (int)((reinterpret_cast<size_t>(b.q2o + wbase) >> 3) & 1);
  const int shr = (int)((reinterpret_cast<size_t>(b.res2 + wbase) >> 3) & 1);
  double* sq = reinterpret_cast<double*>(stq) + shq;
  double* sr = reinterpret_cast<double*>(str) + shr;
  if (P > 0) {
    const unsigned bq = (unsigned)(cnt + shq) * 8, br = (unsigned)(cnt + shr) * 8;
    const Rsrc Rq = span_rsrc(b.q2o + wbase - shq, bq), Rr = span_rsrc(b.res2 + wbase - shr, br);
    // the previous item's reads of this stage have returned before it is
    // overwritten (direct loads write LDS outside the LDS queue)
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0)
    const int chunks = (int)((std::max(bq, br) + 1023) >> 10);
    for (int c = 0; c < chunks; ++c) {
      __builtin_amdgcn_raw_ptr_buffer_load_lds(Rq, (lds_ptr)(stq + c * 1024), 16, lane * 16,
                                               c * 1024, 0, 0);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(Rr, (lds_ptr)(str + c * 1024), 16, lane * 16,
                                               c * 1024, 0, 0);
    }
    // the edge constants of the wave's triangles (192 bytes each, 16-byte
    // aligned), shared by every shot
    const unsigned be = (unsigned)ntw * 24 * 8;
    const Rsrc Re = span_rsrc(L2.edge + (size_t)w0 * 24, be);
    for (int c = 0; c < (int)((be + 1023) >> 10); ++c)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(Re, (lds_ptr)(ste + c * 1024), 16, lane * 16,
                                               c * 1024, 0, 0);
  }
  // ---- every other load that depends on the triangle only
  const double* gg = L2.geo + (size_t)t * 8;
  const double rx = gg[0], ry = gg[1], sx = gg[2], sy = gg[3], irho = gg[4], Kb = gg[5],
               Z = gg[6];
  const int* inf = L2.info + (size_t)t * 8;
  const int e3 = inf[0], ax = inf[1], sgn = inf[2];
  int code[3], nn[3][EK];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    code[e] = inf[3 + e];
#pragma unroll
    for (int jj = 0; jj < EK; ++jj)
      nn[e][jj] = L2.nbrnode[((size_t)t * 3 + e) * Nfp + min(4 * jj + g, Nfp - 1)];
  }
  int n3[RG];
  double S0[RG];
#pragma unroll
  for (int r = 0; r < RG; ++r) {
    const int n = min(4 * r + g, Np - 1);
    n3[r] = L2.tetnode[(size_t)t * Np + n];
    S0[r] = b.q03[(size_t)t * Np + n];
  }
  // the direct loads and the triangle data have landed (the compiler does not
  // order LDS reads after direct-to-LDS loads by itself; the map loads below
  // need the triangle data anyway)
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_sched_barrier(0);
  // ---- loads through the maps: new 3D trace, exterior values of the edges
  double p3[RG], u3[RG];
  {
    const T3* q3 = static_cast<const T3*>(b.q3n) + (size_t)(e3 >> 4) * 4 * F.np3 * kTile + (e3 & 15);
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      p3[r] = (double)q3[n3[r] * kTile];
      u3[r] = (double)q3[((1 + ax) * F.np3 + n3[r]) * kTile];
    }
  }
  // every load is issued at an address valid for any edge kind (own
  // triangle, line 0 of qb2) and the values are selected afterwards by bit
  // masks: a select on a loaded value lets the compiler move the load into
  // a branch, whose result then waits for every load in flight
  double xp[3][EK], xa[3][EK], xb[3][EK];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const bool inner = code[e] >= 0;
    const int c = -1 - code[e];
    const bool hb = !inner && (c & 3) == 0;
    const int tn = inner ? code[e] : t;
    const int lq = hb ? (c >> 3) : 0, sd = hb ? ((c >> 2) & 1) : 0;
    const double* qn = b.q2o + (P > 0 ? ((size_t)tn * P + i) * 3 * Np : 0);
    const double* qbl = b.qb2 + (((size_t)lq * 2 + sd) * Pc + ic) * Nfp;
#pragma unroll
    for (int jj = 0; jj < EK; ++jj) {
      const int m = min(nn[e][jj], Np - 1);
      const double a0 = qn[m], rb = qbl[min(nn[e][jj], Nfp - 1)];
      const long long bits = (__double_as_longlong(a0) & -(long long)inner) |
                             (__double_as_longlong(rb) & -(long long)hb);
      xp[e][jj] = __longlong_as_double(bits);
      xa[e][jj] = qn[Np + m];
      xb[e][jj] = qn[2 * Np + m];
    }
  }
  const int po = (tl < ntw ? es : (ntw * Pc - 1)) * 3 * Np;   // this pair in the stage
  double ps[RG];   // new p*_i at this lane's rows
#pragma unroll
  for (int r = 0; r < RG; ++r) ps[r] = 0.0;
  if (P > 0) {
    const double* fj = sops + ta;
    const double* fl = sops + 2 * RG * RG * 16 + ta;
    const double Ki = Kb / (1.0 + sg[i]);
    double vp[RG], va[RG], vb[RG];
#pragma unroll
    for (int j = 0; j < RG; ++j) {
      const int n = min(4 * j + g, Np - 1);
      vp[j] = sq[po + n];
      va[j] = sq[po + Np + n];
      vb[j] = sq[po + 2 * Np + n];
    }
    // ---- volume: Dr p, Ds p and div v = Dr (grad r . v) + Ds (grad s . v)
    double Gr[RG], Gs[RG], rp[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) Gr[r] = Gs[r] = rp[r] = 0.0;
#pragma unroll
    for (int j = 0; j < RG; ++j) {
      const double fr = rx * va[j] + ry * vb[j], fs = sx * va[j] + sy * vb[j];
#pragma unroll
      for (int r = 0; r < RG; ++r) {
        const double ar = fj[((0 * RG + r) * RG + j) * 16];
        const double as = fj[((1 * RG + r) * RG + j) * 16];
        Gr[r] = mfma4(ar, vp[j], Gr[r]);
        Gs[r] = mfma4(as, vp[j], Gs[r]);
        rp[r] = mfma4(ar, fr, rp[r]);
        rp[r] = mfma4(as, fs, rp[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < RG; ++r) rp[r] *= -Ki;
    // ---- surface: edges s = -1, r + s = 0, r = -1 with n fsc = -grad s,
    // grad(r+s), -grad r.  Upwind flux against the exterior state: the
    // neighbour's trace, p = 2 r- with v.n = 0 (characteristic condition,
    // r- = qb2 at an HABC edge, 0 at a basic-ABC edge), or the mirror
    // p = -p^-, v.n = v.n^- (p = 0).  The pressure jump is lifted into G
    // (Gs for edge 0, -Gr and -Gs for edge 1, Gr for edge 2).
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      // unit normal, face scale and flux weights of this edge (host-built)
      const double* ec = reinterpret_cast<const double*>(ste) + (t - w0) * 24 + e * 8;
      const double na = ec[0], nb = ec[1], fsc = ec[2];
      const double aM = ec[3], aP = ec[4], iZ = ec[5], bZ = ec[6], cP = fsc * Ki;
      const bool inner = code[e] >= 0;
      const int c = -1 - code[e];
      const bool hb = !inner && (c & 3) == 0, dir = !inner && (c & 3) == 2;
#pragma unroll
      for (int jj = 0; jj < EK; ++jj) {
        const int kc = min(4 * jj + g, Nfp - 1);   // rows beyond Nfp: LIFT columns are 0
        const int a = smask[e * Nfp + kc];
        const double pM = sq[po + a], vnM = na * sq[po + Np + a] + nb * sq[po + 2 * Np + a];
        const double vnP = na * xa[e][jj] + nb * xb[e][jj];
        const double pG = inner ? xp[e][jj] : (dir ? -pM : (hb ? 2.0 * xp[e][jj] : 0.0));
        const double uG = inner ? vnP : (dir ? vnM : 0.0);
        const double pF = aM * pM + aP * pG + bZ * (vnM - uG);
        const double vnF = iZ * (pM - pG) + aP * vnM + aM * uG;
        const double fp = cP * (vnM - vnF);
        const double fu = pM - pF;
        const double* fe = fl + (e * EK + jj) * 16;
#pragma unroll
        for (int r = 0; r < RG; ++r) {
          const double l = fe[r * 3 * EK * 16];
          rp[r] = mfma4(l, fp, rp[r]);
          if (e == 0) Gs[r] = mfma4(l, fu, Gs[r]);
          if (e == 1) {
            Gr[r] = mfma4(l, -fu, Gr[r]);
            Gs[r] = mfma4(l, -fu, Gs[r]);
          }
          if (e == 2) Gr[r] = mfma4(l, fu, Gr[r]);
        }
      }
    }
    // ---- LSRK update of the rows this lane holds, into the stage
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      const int n = 4 * r + g, nc = min(n, Np - 1);
      const double r0 = A * sr[po + nc] + dt * rp[r];
      const double r1 = A * sr[po + Np + nc] + dt * (-irho * (rx * Gr[r] + sx * Gs[r]));
      const double r2 = A * sr[po + 2 * Np + nc] + dt * (-irho * (ry * Gr[r] + sy * Gs[r]));
      ps[r] = vp[r] - S0[r] + B * r0;
      if (col && n < Np) {
        sr[po + n] = r0;
        sr[po + Np + n] = r1;
        sr[po + 2 * Np + n] = r2;
        sq[po + Np + n] = va[r] + B * r1;
        sq[po + 2 * Np + n] = vb[r] + B * r2;
      }
    }
  }
  // ---- face rule per row group: r- = (1/M) sum_i g_i p*_i over the P
  // columns of this triangle (lanes of the same row, gathered by shuffles)
#pragma unroll
  for (int r = 0; r < RG; ++r) {
    const int n = 4 * r + g;
    const double gp = P > 0 ? sg[ic] * ps[r] : 0.0;
    double rm = 0.0;
    for (int s2 = 0; s2 < P; ++s2) rm += __shfl(gp, (lane & ~15) + tl * Pc + s2);
    rm *= L2.invM;
    const double S = 0.5 * (p3[r] + Z * (double)sgn * u3[r]) + rm;
    if (col && n < Np) {
      if (i == 0) {
        b.qb3[(size_t)t * Np + n] = rm;
        b.q03[(size_t)t * Np + n] = S;
      }
      if (P > 0) sq[po + n] = ps[r] + S;
    }
  }
  // ---- linear stores of the new q2 and res2 of the wave's pairs
  if (P > 0) {
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const int x = lane + 64 * k;
      if (64 * k < cnt && x < cnt) {
        b.q2n[wbase + x] = sq[x];
        b.res2[wbase + x] = sr[x];
      }
    }
  }
}

// Persistent: each workgroup loads the operator fragments, face masks and
// gamma into LDS once, then takes (shot, group) items from its XCD's range.
template <int N, class T3>
__global__ void __launch_bounds__(kWaves2 * 64, 2) k_faces(LvlF F, Lvl2 L2, FaceBufs b, Shots sh,
                                                           double A, double B, double dt,
                                                           int ngrp) {
  using D = Dims2<N>;
  constexpr int Np = D::Np, Nfp = D::Nfp;
  __shared__ double sops[D::NFRAG * 16];
  __shared__ double sg[16];
  __shared__ int smask[3 * Nfp];
  __shared__ __attribute__((aligned(16))) char stage[kWaves2 * D::STAGE];
  fill_lds<kWaves2 * 64, D::NFRAG * 16>(sops, F.ops, threadIdx.x);
  fill_lds<kWaves2 * 64, 3 * Nfp>(smask, L2.fmask, threadIdx.x);
  if (threadIdx.x < L2.P) sg[threadIdx.x] = L2.gamma[threadIdx.x];
  __syncthreads();
  const XcdRange rg_((long long)ngrp * sh.n);
  for (long long it = rg_.lo; it < rg_.hi; it += rg_.step) {
    const int k = (int)(it / ngrp), bx = (int)(it - (long long)k * ngrp);
    faces_item<N, T3>(F, L2, b, sh, A, B, dt, bx, k, sops, sg, smask, stage);
  }
}

template <int N, class T3>
hipError_t launch_faces_t(const LvlF& F, const Lvl2& L2, const FaceBufs& b, const Shots& sh,
                          double A, double B, double dt, int ngrp, hipStream_t st) {
  // persistent grid: as many workgroups as fit on the device at once (a
  // multiple of 8, so that every XCD has blocks for its range)
  int resident = 0;
  {
    const hipError_t e = kernel_setup((const void*)(k_faces<N, T3>), kWaves2 * 64, 0, &resident);
    if (e != hipSuccess) return e;
  }
  const long long items = (long long)ngrp * sh.n;
  const int blocks = (int)std::max<long long>(8, std::min<long long>(resident, items) / 8 * 8);
  hipLaunchKernelGGL((k_faces<N, T3>), dim3(blocks), dim3(kWaves2 * 64), 0, st, F, L2, b, sh, A,
                     B, dt, ngrp);
  return hipGetLastError();
}

template <int N>
hipError_t launch_faces_n(const LvlF& F, const Lvl2& L2, const FaceBufs& b, const Shots& sh,
                          double A, double B, double dt, int ngrp, hipStream_t st) {
  if (b.q3f32) return launch_faces_t<N, float>(F, L2, b, sh, A, B, dt, ngrp, st);
  return launch_faces_t<N, double>(F, L2, b, sh, A, B, dt, ngrp, st);
}

}  // namespace

hipError_t launch_faces(const LvlF& F, const Lvl2& L2, const FaceBufs& b, const Shots& sh,
                        double A, double B, double dt, hipStream_t st) {
  if (L2.Kt == 0) return hipSuccess;
  if (L2.P > 16 || sh.n < 1 || sh.n > 65535) return hipErrorInvalidValue;
  const int TW = 16 / (L2.P > 0 ? L2.P : 1);
  const int waves = (L2.Kt + TW - 1) / TW;
  const int ngrp = (waves + kWaves2 - 1) / kWaves2;
  switch (L2.Np) {
    case 3: return launch_faces_n<1>(F, L2, b, sh, A, B, dt, ngrp, st);
    case 6: return launch_faces_n<2>(F, L2, b, sh, A, B, dt, ngrp, st);
    case 10: return launch_faces_n<3>(F, L2, b, sh, A, B, dt, ngrp, st);
    case 15: return launch_faces_n<4>(F, L2, b, sh, A, B, dt, ngrp, st);
    case 21: return launch_faces_n<5>(F, L2, b, sh, A, B, dt, ngrp, st);
    case 28: return launch_faces_n<6>(F, L2, b, sh, A, B, dt, ngrp, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dgh
