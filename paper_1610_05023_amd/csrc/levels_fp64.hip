// FP64 kernels of the four levels of one Runge-Kutta stage (Algorithm 1):
// the 3D volume level (volume term + upwind surface term + LSRK update in
// one kernel), the 2D face level (DG right-hand side of the P face systems,
// update, face rule), the 1D edge level (right-hand side of the P^2 edge
// systems, update, edge compatibility system) and the 0D corner systems.
//
// Discretisation (Section 3.2): strong-form nodal DG,
//   rhs_p = -rho c^2 div u + LIFT [Fscale rho c^2 (n.u^- - (n.u)*)]
//   rhs_u = -(1/rho) grad p + LIFT [Fscale (1/rho) (p^- - p*) n]
// with the exact-Riemann upwind flux between cells and the characteristic
// flux p* = r+ + r-_ext, (n.u)* = (r+ - r-_ext)/Z on boundaries, where
// r+- = (p +- Z n.u)/2; LSRK: res = A res + dt rhs, q = q + B res.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"
#include "launch.hpp"
#include "levels.hpp"

namespace dgh {

namespace {

// ------------------------------------------------------------------ 3D ---
// One wave per tile of 16 elements.  The volume and lifting contractions run
// on the FP64 4x4x4 MFMA (four 4x4x4 blocks per instruction; on gfx950 it
// issues at the full FP64 rate, unlike the 16x16x4 form).  Lane l holds
// element l%16 and the nodes n = 4 rg + l/16 of row group rg; the four
// blocks of an instruction are four groups of 4 elements sharing the same
// operator block:
//   A (operator rows 4rg..4rg+3, cols 4ks..4ks+3): lane l -> A[l%4][l/16]
//   B (fields at nodes 4ks + k of the 16 elements):  lane l -> B[l/16][l%16]
//   D (rows 4rg + k, elements):                       lane l -> D[l/16][l%16]
// so each instruction accumulates one double per lane.

template <int N>
struct Dims3 {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int RG = (Np + 3) / 4;     // row groups (also volume k-steps)
  static constexpr int FK = (Nfp + 3) / 4;    // lifting k-steps per face
  static constexpr int NFRAG = 3 * RG * RG + RG * 4 * FK;   // 16 doubles each
  // operator fragments in LDS up to 150 KB (N <= 6); above 64 KB the kernel
  // runs one workgroup per CU, with 512 registers per wave
  static constexpr bool kLds = NFRAG * 16 * 8 <= 150 * 1024;
};

// waves (tiles) per workgroup of the register-streaming 3D kernel: W = 4
// or 8 (Lvl3::waves; a tuning axis).  With the operators in LDS at N = 5
// eight waves share them, two per SIMD at 256 registers each: the second
// wave covers the first one's waits on memory (1,233 -> 910 us per launch
// at 40^3, although the compiler then spills 36 registers).
template <int N, int W>
struct Occ3 {   // workgroups per CU the registers are sized for
  static constexpr int value = W == 8 ? 1 : (Dims3<N>::NFRAG * 16 * 8 <= 64 * 1024 ? 2 : 1);
};

// Buffer-resource access: a 32-bit per-lane byte offset plus a uniform
// (scalar) offset, so the four fields of a node share one address register.
// The host keeps every 3D array below 4 GiB; an offset past the end of a
// resource reads 0 (never used: every index is in range by construction).
using Rsrc = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ Rsrc rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           0x00020000);
}
__device__ __forceinline__ double bld(Rsrc r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
// streaming load/store (non-temporal: read or written once per stage, so
// they leave the L2 to the state that is re-read within the stage)
__device__ __forceinline__ double bldn(Rsrc r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 2));
}
__device__ __forceinline__ void bstn(Rsrc r, unsigned voff, unsigned soff, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 2);
}

template <int N, int W>
__device__ __forceinline__ void tile_step(const Lvl3& L, const double* __restrict__ qo,
                                          double* __restrict__ qn, double* __restrict__ res,
                                          const double* __restrict__ qb3, double A, double B,
                                          double dt, const Shots& sh, long long item, int ngrp,
                                          const int* smap, const int* smask, const double* sops,
                                          int lane);

template <int N, int W>
__global__ void __launch_bounds__(W * 64, (Occ3<N, W>::value)) k_level3(Lvl3 L, const double* __restrict__ qo,
                                                   double* __restrict__ qn, double* __restrict__ res,
                                                   const double* __restrict__ qb3, double A, double B,
                                                   double dt, Shots sh) {
  using D = Dims3<N>;
  constexpr int Np = D::Np, Nfp = D::Nfp, RG = D::RG, FK = D::FK;
  constexpr unsigned FS = Np * kTile * 8;   // bytes between two fields of a tile
  constexpr unsigned TS = 4 * FS;           // bytes per tile
  extern __shared__ double sfrag[];
  // face-node tables in LDS (first), then the operator fragments
  int* smask = reinterpret_cast<int*>(sfrag);
  int* smap = smask + 4 * Nfp;
  constexpr int kTabDoubles = (4 * Nfp + 96 * Nfp + 1) / 2;
  fill_lds<W * 64, 4 * Nfp>(smask, L.fmask, threadIdx.x);
  fill_lds<W * 64, 96 * Nfp>(smap, L.fmap, threadIdx.x);
  double* sops = sfrag + kTabDoubles;
  if (D::kLds) fill_lds<W * 64, D::NFRAG * 16>(sops, L.ops, threadIdx.x);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  // persistent: the workgroup loads its tables once, then its waves take
  // (shot, group of W tiles) items from its XCD's range
  const int ngrp = (L.ntile + W - 1) / W;
  const XcdRange rg_(ngrp * (long long)sh.n, L.order);
  for (long long item = rg_.lo; item < rg_.hi; item += rg_.step)
    tile_step<N, W>(L, qo, qn, res, qb3, A, B, dt, sh, item, ngrp, smap, smask, sops, lane);
}

// One wave's share of one work item: tile (item mod ngrp) W + wave of
// shot item / ngrp.
template <int N, int W>
__device__ __forceinline__ void tile_step(const Lvl3& L, const double* __restrict__ qo,
                                          double* __restrict__ qn, double* __restrict__ res,
                                          const double* __restrict__ qb3, double A, double B,
                                          double dt, const Shots& sh, long long item, int ngrp,
                                          const int* smap, const int* smask, const double* sops,
                                          int lane) {
  using D = Dims3<N>;
  constexpr int Np = D::Np, Nfp = D::Nfp, RG = D::RG, FK = D::FK;
  constexpr unsigned FS = Np * kTile * 8;   // bytes between two fields of a tile
  constexpr unsigned TS = 4 * FS;           // bytes per tile
  const int shot = (int)(item / ngrp);
  const int tile = (int)(item - (long long)shot * ngrp) * W + (threadIdx.x >> 6);
  if (tile >= L.ntile) return;
  qo += shot * sh.st3;
  qn += shot * sh.st3;
  res += shot * sh.st3;
  qb3 += shot * sh.stb3;
  const int es = lane & 15, g = lane >> 4;
  const int ta = (lane & 3) + 4 * g;   // this lane's entry of a 16-value A fragment
  const double* frag = (D::kLds ? sops : L.ops) + ta;
  const double* fragL = frag + 3 * RG * RG * 16;
  const int e = tile * kTile + es;
  const unsigned nbytes = (unsigned)L.ntile * TS;
  const Rsrc Rq = rsrc(qo, nbytes), Rn = rsrc(qn, nbytes), Rr = rsrc(res, nbytes);
  const Rsrc Rb = rsrc(qb3, (unsigned)L.nqb3 * 8);
  const unsigned tb = (unsigned)tile * TS + (unsigned)es * 8;   // this lane's element
  const double* gt = L.geo + (size_t)tile * 12 * kTile + es;
  const double rx = gt[0 * kTile], ry = gt[1 * kTile], rz = gt[2 * kTile];
  const double sx = gt[3 * kTile], sy = gt[4 * kTile], sz = gt[5 * kTile];
  const double tx = gt[6 * kTile], ty = gt[7 * kTile], tz = gt[8 * kTile];
  const double irho = gt[9 * kTile], Kb = gt[10 * kTile], Z = gt[11 * kTile];
  // face codes and exterior impedances, loaded with the geometry
  const int* nbrt = L.nbr + tile * 4 * kTile + es;
  const double* znt = L.zn + tile * 4 * kTile + es;
  int fcode[4];
  double fz[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    fcode[f] = nbrt[f * kTile];
    fz[f] = znt[f * kTile];
  }

  // ---- volume: Dr p, Ds p, Dt p and div u = Dr fr + Ds fs + Dt ft with the
  // contravariant fluxes fr = grad r . u etc.  Rows beyond Np read the last
  // node (finite); the operator columns there are zero.
  double dpr[RG], dps[RG], dpt[RG], dv[RG];
#pragma unroll
  for (int i = 0; i < RG; ++i) dpr[i] = dps[i] = dpt[i] = dv[i] = 0.0;
  // fields of the lane's nodes 4 j + g, loaded PF k-steps ahead (fewer for
  // N > 4, where the accumulators leave no registers for it)
  constexpr int PF = N <= 4 ? 3 : 1;
  double bp[PF], bu[PF], bv[PF], bw[PF];
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    const unsigned o = tb + (unsigned)min(4 * k + g, Np - 1) * (kTile * 8);
    bp[k] = bld(Rq, o, 0);
    bu[k] = bld(Rq, o, FS);
    bv[k] = bld(Rq, o, 2 * FS);
    bw[k] = bld(Rq, o, 3 * FS);
  }
#pragma unroll 1
  for (int j0 = 0; j0 < RG; j0 += PF) {
#pragma unroll
    for (int sl = 0; sl < PF; ++sl) {
      const int j = j0 + sl;
      if (j < RG) {
        const double p = bp[sl], u = bu[sl], v = bv[sl], w = bw[sl];
        {
          const unsigned o = tb + (unsigned)min(4 * (j + PF) + g, Np - 1) * (kTile * 8);
          bp[sl] = bld(Rq, o, 0);
          bu[sl] = bld(Rq, o, FS);
          bv[sl] = bld(Rq, o, 2 * FS);
          bw[sl] = bld(Rq, o, 3 * FS);
        }
        const double fr = rx * u + ry * v + rz * w;
        const double fs = sx * u + sy * v + sz * w;
        const double ft = tx * u + ty * v + tz * w;
        const double* fj = frag + j * 16;
#pragma unroll
        for (int i = 0; i < RG; ++i) {
          if (i % 3 == 0) __builtin_amdgcn_sched_barrier(0);
          const double ar = fj[((0 * RG + i) * RG) * 16];
          const double as = fj[((1 * RG + i) * RG) * 16];
          const double at = fj[((2 * RG + i) * RG) * 16];
          dpr[i] = mfma4(ar, p, dpr[i]);
          dps[i] = mfma4(as, p, dps[i]);
          dpt[i] = mfma4(at, p, dpt[i]);
          dv[i] = mfma4(ar, fr, dv[i]);
          dv[i] = mfma4(as, fs, dv[i]);
          dv[i] = mfma4(at, ft, dv[i]);
        }
      }
    }
  }
  // rhs_p = -rho c^2 div u (+ the lifted surface term); the velocity rhs
  // stays the reference gradient G = (Dr p, Ds p, Dt p) plus the lifted
  // pressure jumps until the update maps it: rhs_u = -(1/rho) J^-T G
#pragma unroll
  for (int i = 0; i < RG; ++i) dv[i] *= -Kb;
  double* rp = dv;

  // ---- surface: fluxes at the face nodes in B-fragment order, then LIFT.
  // Every face uses the upwind flux against an exterior state: the
  // neighbour's trace (interior), p = 2 r- and n.u = 0 (characteristic
  // condition with incoming r-: HABC r- = qb3, basic ABC r- = 0), or the
  // mirror p = -p^-, n.u = n.u^- (p = 0); boundary faces carry their own
  // impedance, for which this reproduces the characteristic and Dirichlet
  // fluxes exactly.
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    __builtin_amdgcn_sched_barrier(0);
    // outward normal of face f: -grad t, -grad s, grad(r+s+t), -grad r
    const double cr = f == 2 ? 1.0 : (f == 3 ? -1.0 : 0.0);
    const double cs = f == 2 ? 1.0 : (f == 1 ? -1.0 : 0.0);
    const double ct = f == 2 ? 1.0 : (f == 0 ? -1.0 : 0.0);
    double nx = cr * rx + cs * sx + ct * tx;
    double ny = cr * ry + cs * sy + ct * ty;
    double nz = cr * rz + cs * sz + ct * tz;
    const double fsc = sqrt(nx * nx + ny * ny + nz * nz);
    const double inv = 1.0 / fsc;
    nx *= inv;
    ny *= inv;
    nz *= inv;
    const int code = fcode[f];
    const double ZP = fz[f];
    // interior faces gather from the neighbour; boundary faces read their own
    // element there (unused) and qb3 (triangle 0 unless HABC, unused) --
    // every load is issued, then the exterior state is selected
    const bool inner = code >= 0;
    const int cb = -1 - code;
    const bool hb = !inner && (cb & 3) == 0;
    const bool dir = !inner && (cb & 3) == 2;
    const int e2 = inner ? (code >> 5) : e;
    const unsigned nb = (unsigned)(e2 >> 4) * TS + (unsigned)(e2 & 15) * 8;
    const int mapbase = inner ? ((f * 4 + ((code >> 3) & 3)) * 6 + (code & 7)) * Nfp
                              : ((f * 4) * 6 + ((cb >> 2) & 7)) * Nfp;
    const unsigned qbo = (unsigned)(hb ? (cb >> 5) : 0) * (Nfp * 8);
    // upwind weights (exact-Riemann flux, Section 3.2)
    const double iZ = 1.0 / (Z + ZP);
    const double aM = ZP * iZ, aP = Z * iZ, bZ = Z * aM;
    const double cP = fsc * Kb;
#pragma unroll
    for (int jj = 0; jj < FK; ++jj) {
      const int kc = min(4 * jj + g, Nfp - 1);   // rows beyond Nfp: LIFT columns are 0
      const int n = smask[f * Nfp + kc];
      const int n2 = smap[mapbase + kc];
      const unsigned oM = tb + (unsigned)n * (kTile * 8);
      const unsigned oP = nb + (unsigned)n2 * (kTile * 8);
      const double pM = bld(Rq, oM, 0), uM = bld(Rq, oM, FS), vM = bld(Rq, oM, 2 * FS),
                   wM = bld(Rq, oM, 3 * FS);
      const double pP = bld(Rq, oP, 0), uP = bld(Rq, oP, FS), vP = bld(Rq, oP, 2 * FS),
                   wP = bld(Rq, oP, 3 * FS);
      const double rb = bld(Rb, qbo + (unsigned)min(n2, Nfp - 1) * 8, 0);
      const double unM = nx * uM + ny * vM + nz * wM;
      const double unP = nx * uP + ny * vP + nz * wP;
      const double pG = inner ? pP : (dir ? -pM : (hb ? 2.0 * rb : 0.0));
      const double uG = inner ? unP : (dir ? unM : 0.0);
      const double pF = aM * pM + aP * pG + bZ * (unM - uG);
      const double unF = iZ * (pM - pG) + aP * unM + aM * uG;
      const double fp = cP * (unM - unF);
      // pressure jump, lifted into G: with n fsc = -grad t, -grad s,
      // grad(r+s+t), -grad r on faces 0..3, the term fsc (1/rho) (p^- - p*) n
      // of rhs_u equals -(1/rho) J^-T (-c_f) L (p^- - p*)
      const double fu = pM - pF;
      const double* fl = fragL + (f * FK + jj) * 16;
      if (f == 2) {
#pragma unroll
        for (int i = 0; i < RG; ++i) {
          const double a = fl[i * 4 * FK * 16];
          rp[i] = mfma4(a, fp, rp[i]);
          dpr[i] = mfma4(a, -fu, dpr[i]);
          dps[i] = mfma4(a, -fu, dps[i]);
          dpt[i] = mfma4(a, -fu, dpt[i]);
        }
      } else {
        double* G = f == 0 ? dpt : (f == 1 ? dps : dpr);
#pragma unroll
        for (int i = 0; i < RG; ++i) {
          const double a = fl[i * 4 * FK * 16];
          rp[i] = mfma4(a, fp, rp[i]);
          G[i] = mfma4(a, fu, G[i]);
        }
      }
    }
  }

  // ---- LSRK update of the rows this lane holds (1/rho = 0 marks padding),
  // in chunks of row groups so that the loads in flight fit the registers;
  // loads at clamped rows, stores masked
  {
    const bool live = irho != 0.0;
    // point source S(tau) = amp (tau - t0) exp(-pi^2 f0^2 (tau - t0)^2)
    const double* sp = sh.srcp + 4 * shot;
    const bool src = (double)e == sp[0];
    const double tr = stage_time(sh) - sp[2], ar = M_PI * sp[1] * tr;
    const double src_s = sp[3] * tr * exp(-ar * ar);
    const double* src_w = sh.srcw + (size_t)shot * Np;
    constexpr int EC = 3;
#pragma unroll
    for (int i0 = 0; i0 < RG; i0 += EC) {
      __builtin_amdgcn_sched_barrier(0);
      double ro[EC][4], qo_[EC][4];
#pragma unroll
      for (int ii = 0; ii < EC; ++ii) {
        const unsigned o = tb + (unsigned)min(4 * (i0 + ii) + g, Np - 1) * (kTile * 8);
#pragma unroll
        for (int fl = 0; fl < 4; ++fl) {
          ro[ii][fl] = (i0 + ii < RG) ? bldn(Rr, o, fl * FS) : 0.0;
          qo_[ii][fl] = (i0 + ii < RG) ? bld(Rq, o, fl * FS) : 0.0;
        }
      }
#pragma unroll
      for (int ii = 0; ii < EC; ++ii) {
        const int i = i0 + ii;
        if (i >= RG) continue;
        const int n = 4 * i + g;
        const int nc = min(n, Np - 1);
        const unsigned o = tb + (unsigned)nc * (kTile * 8);
        const double sw = src_w[nc];
        const double a = dpr[i], bq = dps[i], c = dpt[i];
        const double rhs[4] = {rp[i] + (src ? sw * src_s : 0.0),
                               -irho * (rx * a + sx * bq + tx * c),
                               -irho * (ry * a + sy * bq + ty * c),
                               -irho * (rz * a + sz * bq + tz * c)};
        if (live && n < Np) {
#pragma unroll
          for (int fl = 0; fl < 4; ++fl) {
            const double rr = A * ro[ii][fl] + dt * rhs[fl];
            bstn(Rr, o, fl * FS, rr);
            bstn(Rn, o, fl * FS, qo_[ii][fl] + B * rr);
          }
        }
      }
    }
  }
}

// ---------------------------------------------- 3D, tile held on chip ---
// The same stage for N <= 4 with one wave per SIMD (one workgroup of four
// waves per CU).  Each wave owns an LDS buffer that receives its next tile
// (state, geometry, impedances, face codes) by direct buffer-to-LDS loads,
// issued as soon as the surface term no longer reads the current tile's
// copy (the own traces of the last face are taken into registers first), so
// the tile lands while the wave finishes the current one.  The wave holds
// the tile's q in registers (the B-fragment rows a lane holds for the volume
// term, nodes 4 j + g of element l%16, are the D-fragment rows it updates),
// reads the own traces from the LDS copy, and has the exterior traces of
// faces 0-2 in flight during the volume term (face 3's during face 0), so
// each value of q and res crosses HBM once; the neighbour traces are
// re-read, mostly from L2.
constexpr int kWavesR = 4;

template <int N>
struct BufR {
  static constexpr int Np = Dims3<N>::Np;
  static constexpr int QK = (Np + 1) / 2;           // 1 KB loads for the state (512 Np bytes)
  static constexpr int QB = QK * 1024;              // geometry, impedances, codes after it
  static constexpr int GEO = QB, ZN = QB + 2048, NBR = QB + 3072;
  static constexpr int BYTES = QB + 4096;
};

typedef __attribute__((address_space(3))) void* lds_ptr;

// direct loads of work item `item` (this wave's tile, shot) into buf; a tile
// past the end loads the last tile (never used).  Each instruction moves
// 16 bytes per lane to buf + 16 lane.
template <int N>
__device__ __forceinline__ void tile_dma(const Lvl3& L, const double* __restrict__ qo,
                                         const Shots& sh, long long item, int ngrp, char* buf,
                                         int lane) {
  using D = Dims3<N>;
  using BR = BufR<N>;
  constexpr unsigned TS = 4 * D::Np * kTile * 8;
  const int shot = (int)(item / ngrp);
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int tile = min((int)(item - (long long)shot * ngrp) * kWavesR + wv, L.ntile - 1);
  const Rsrc Rq = rsrc(qo + shot * sh.st3, (unsigned)L.ntile * TS);
  const Rsrc Rg = rsrc(L.geo, (unsigned)L.ntile * 12 * kTile * 8);
  const Rsrc Rz = rsrc(L.zn, (unsigned)L.ntile * 4 * kTile * 8);
  const Rsrc Rc = rsrc(L.nbr, (unsigned)L.ntile * 4 * kTile * 4);
  const int vo = lane * 16;
#pragma unroll
  for (int k = 0; k < BR::QK; ++k)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(Rq, (lds_ptr)(buf + k * 1024), 16, vo,
                                             (int)((unsigned)tile * TS + k * 1024), 0, 0);
#pragma unroll
  for (int k = 0; k < 2; ++k)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(Rg, (lds_ptr)(buf + BR::GEO + k * 1024), 16, vo,
                                             tile * 12 * kTile * 8 + k * 1024, 0, 0);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(Rz, (lds_ptr)(buf + BR::ZN), 16, vo,
                                           tile * 4 * kTile * 8, 0, 0);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(Rc, (lds_ptr)(buf + BR::NBR), 16, vo,
                                           tile * 4 * kTile * 4, 0, 0);
}

// exterior traces of one face at the lane's FK face-node rows
template <int N>
struct FaceIn {
  static constexpr int FK = Dims3<N>::FK;
  double p[FK], u[FK], v[FK], w[FK], rb[FK];
};

template <int N>
__device__ __forceinline__ void face_fetch(FaceIn<N>& x, int f, int code, int e, Rsrc Rq, Rsrc Rb,
                                           const int* smap, int g) {
  using D = Dims3<N>;
  constexpr int Np = D::Np, Nfp = D::Nfp, FK = D::FK;
  constexpr unsigned FS = Np * kTile * 8, TS = 4 * FS;
  const bool inner = code >= 0;
  const int cb = -1 - code;
  const bool hb = !inner && (cb & 3) == 0;
  const int e2 = inner ? (code >> 5) : e;
  const unsigned nb = (unsigned)(e2 >> 4) * TS + (unsigned)(e2 & 15) * 8;
  const int mapbase = inner ? ((f * 4 + ((code >> 3) & 3)) * 6 + (code & 7)) * Nfp
                            : ((f * 4) * 6 + ((cb >> 2) & 7)) * Nfp;
  const unsigned qbo = (unsigned)(hb ? (cb >> 5) : 0) * (Nfp * 8);
#pragma unroll
  for (int jj = 0; jj < FK; ++jj) {
    const int kc = min(4 * jj + g, Nfp - 1);
    const int n2 = smap[mapbase + kc];
    const unsigned oP = nb + (unsigned)n2 * (kTile * 8);
    x.p[jj] = bld(Rq, oP, 0);
    x.u[jj] = bld(Rq, oP, FS);
    x.v[jj] = bld(Rq, oP, 2 * FS);
    x.w[jj] = bld(Rq, oP, 3 * FS);
    x.rb[jj] = bld(Rb, qbo + (unsigned)min(n2, Nfp - 1) * 8, 0);
  }
}

// One work item whose tile is in buf; calls fetch_next() (which issues the
// direct loads of the next item, if any, into buf) once the tile's copy has
// been read.
template <int N, class Fetch>
__device__ __forceinline__ void tile_step_dma(const Lvl3& L, const double* __restrict__ qo,
                                              double* __restrict__ qn, double* __restrict__ res,
                                              const double* __restrict__ qb3, double A, double B,
                                              double dt, const Shots& sh, long long item,
                                              Fetch fetch_next, int ngrp, const int* smap,
                                              const int* smask, const double* sops, char* buf,
                                              int lane) {
  using D = Dims3<N>;
  using BR = BufR<N>;
  constexpr int Np = D::Np, Nfp = D::Nfp, RG = D::RG, FK = D::FK;
  constexpr unsigned FS = Np * kTile * 8;   // bytes between two fields of a tile
  constexpr unsigned TS = 4 * FS;           // bytes per tile
  const int shot = (int)(item / ngrp);
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int tile = (int)(item - (long long)shot * ngrp) * kWavesR + wv;
  // the tile's direct loads have landed: vector memory operations complete
  // in order and the previous tile issued 8 RG stores after them (the
  // compiler does not order LDS reads after direct-to-LDS loads by itself)
  constexpr int kVm = 8 * RG < 63 ? 8 * RG : 63;
  __builtin_amdgcn_s_waitcnt((kVm & 15) | ((kVm >> 4) << 14) | (7 << 4) | (15 << 8));
  if (tile >= L.ntile) {
    // no stores follow: wait for the next tile's direct loads here
    __builtin_amdgcn_s_waitcnt(0);
    fetch_next();
    __builtin_amdgcn_s_waitcnt(0);
    return;
  }
  const double* qos = qo + shot * sh.st3;
  double* qns = qn + shot * sh.st3;
  double* ress = res + shot * sh.st3;
  const double* qbs = qb3 + shot * sh.stb3;
  const int es = lane & 15, g = lane >> 4;
  const int ta = (lane & 3) + 4 * g;   // this lane's entry of a 16-value A fragment
  const double* frag = sops + ta;
  const double* fragL = frag + 3 * RG * RG * 16;
  const int e = tile * kTile + es;
  const unsigned nbytes = (unsigned)L.ntile * TS;
  const Rsrc Rq = rsrc(qos, nbytes), Rn = rsrc(qns, nbytes), Rr = rsrc(ress, nbytes);
  const Rsrc Rb = rsrc(qbs, (unsigned)L.nqb3 * 8);
  const unsigned tb = (unsigned)tile * TS + (unsigned)es * 8;   // this lane's element
  const double* bq = reinterpret_cast<const double*>(buf) + es;   // [field][node][16]
  const double* bg = reinterpret_cast<const double*>(buf + BR::GEO) + es;
  const double* bz = reinterpret_cast<const double*>(buf + BR::ZN) + es;
  const int* bc = reinterpret_cast<const int*>(buf + BR::NBR) + es;
  int fcode[4];
  double fz[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    fcode[f] = bc[f * kTile];
    fz[f] = bz[f * kTile];
  }
  // every face's exterior traces, in flight during the volume term
  FaceIn<N> fb[4];
#pragma unroll
  for (int f = 0; f < 3; ++f) face_fetch<N>(fb[f], f, fcode[f], e, Rq, Rb, smap, g);
  const double rx = bg[0 * kTile], ry = bg[1 * kTile], rz = bg[2 * kTile];
  const double sx = bg[3 * kTile], sy = bg[4 * kTile], sz = bg[5 * kTile];
  const double tx = bg[6 * kTile], ty = bg[7 * kTile], tz = bg[8 * kTile];
  const double irho = bg[9 * kTile], Kb = bg[10 * kTile], Z = bg[11 * kTile];
  double qv[RG][4];
#pragma unroll
  for (int j = 0; j < RG; ++j) {
    const int n = min(4 * j + g, Np - 1);
#pragma unroll
    for (int fl = 0; fl < 4; ++fl) qv[j][fl] = bq[(fl * Np + n) * kTile];
  }

  // ---- volume (as in tile_step), operands from registers
  double dpr[RG], dps[RG], dpt[RG], dv[RG];
#pragma unroll
  for (int i = 0; i < RG; ++i) dpr[i] = dps[i] = dpt[i] = dv[i] = 0.0;
#pragma unroll
  for (int j = 0; j < RG; ++j) {
    const double p = qv[j][0], u = qv[j][1], v = qv[j][2], w = qv[j][3];
    const double fr = rx * u + ry * v + rz * w;
    const double fs = sx * u + sy * v + sz * w;
    const double ft = tx * u + ty * v + tz * w;
    const double* fj = frag + j * 16;
#pragma unroll
    for (int i = 0; i < RG; ++i) {
      const double ar = fj[((0 * RG + i) * RG) * 16];
      const double as = fj[((1 * RG + i) * RG) * 16];
      const double at = fj[((2 * RG + i) * RG) * 16];
      dpr[i] = mfma4(ar, p, dpr[i]);
      dps[i] = mfma4(as, p, dps[i]);
      dpt[i] = mfma4(at, p, dpt[i]);
      dv[i] = mfma4(ar, fr, dv[i]);
      dv[i] = mfma4(as, fs, dv[i]);
      dv[i] = mfma4(at, ft, dv[i]);
    }
  }
#pragma unroll
  for (int i = 0; i < RG; ++i) dv[i] *= -Kb;
  double* rp = dv;

  // ---- surface (as in tile_step); own traces from the LDS copy
  double rv[RG][4];
  constexpr int kEarlyFace = 3;
  double ownr[4 - kEarlyFace][FK][4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    __builtin_amdgcn_sched_barrier(0);
    if (f == 1) {
      // the residual of this tile, needed by the update
#pragma unroll
      for (int j = 0; j < RG; ++j) {
        const unsigned o = tb + (unsigned)min(4 * j + g, Np - 1) * (kTile * 8);
#pragma unroll
        for (int fl = 0; fl < 4; ++fl) rv[j][fl] = bldn(Rr, o, fl * FS);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if (f == 0) {
      face_fetch<N>(fb[3], 3, fcode[3], e, Rq, Rb, smap, g);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (f == kEarlyFace) {
      // own traces of the remaining faces into registers; then the copy is
      // free and the next tile's direct loads go out
#pragma unroll
      for (int f2 = kEarlyFace; f2 < 4; ++f2)
#pragma unroll
        for (int jj = 0; jj < FK; ++jj) {
          const int n = smask[f2 * Nfp + min(4 * jj + g, Nfp - 1)];
#pragma unroll
          for (int fl = 0; fl < 4; ++fl) ownr[f2 - kEarlyFace][jj][fl] = bq[(fl * Np + n) * kTile];
        }
      __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): every LDS read returned
      __builtin_amdgcn_sched_barrier(0);
      fetch_next();
      __builtin_amdgcn_sched_barrier(0);
    }
    const FaceIn<N>& x = fb[f];
    const double cr = f == 2 ? 1.0 : (f == 3 ? -1.0 : 0.0);
    const double cs = f == 2 ? 1.0 : (f == 1 ? -1.0 : 0.0);
    const double ct = f == 2 ? 1.0 : (f == 0 ? -1.0 : 0.0);
    double nx = cr * rx + cs * sx + ct * tx;
    double ny = cr * ry + cs * sy + ct * ty;
    double nz = cr * rz + cs * sz + ct * tz;
    const double fsc = sqrt(nx * nx + ny * ny + nz * nz);
    const double inv = 1.0 / fsc;
    nx *= inv;
    ny *= inv;
    nz *= inv;
    const int code = fcode[f];
    const double ZP = fz[f];
    const bool inner = code >= 0;
    const int cb = -1 - code;
    const bool hb = !inner && (cb & 3) == 0;
    const bool dir = !inner && (cb & 3) == 2;
    const double iZ = 1.0 / (Z + ZP);
    const double aM = ZP * iZ, aP = Z * iZ, bZ = Z * aM;
    const double cP = fsc * Kb;
#pragma unroll
    for (int jj = 0; jj < FK; ++jj) {
      double pM, uM, vM, wM;
      if (f >= kEarlyFace) {
        pM = ownr[f - kEarlyFace][jj][0];
        uM = ownr[f - kEarlyFace][jj][1];
        vM = ownr[f - kEarlyFace][jj][2];
        wM = ownr[f - kEarlyFace][jj][3];
      } else {
        const int kc = min(4 * jj + g, Nfp - 1);
        const int n = smask[f * Nfp + kc];
        const double* sm = bq + n * kTile;
        pM = sm[0];
        uM = sm[Np * kTile];
        vM = sm[2 * Np * kTile];
        wM = sm[3 * Np * kTile];
      }
      const double pP = x.p[jj], uP = x.u[jj], vP = x.v[jj], wP = x.w[jj];
      const double unM = nx * uM + ny * vM + nz * wM;
      const double unP = nx * uP + ny * vP + nz * wP;
      const double pG = inner ? pP : (dir ? -pM : (hb ? 2.0 * x.rb[jj] : 0.0));
      const double uG = inner ? unP : (dir ? unM : 0.0);
      const double pF = aM * pM + aP * pG + bZ * (unM - uG);
      const double unF = iZ * (pM - pG) + aP * unM + aM * uG;
      const double fp = cP * (unM - unF);
      const double fu = pM - pF;
      const double* fl = fragL + (f * FK + jj) * 16;
      if (f == 2) {
#pragma unroll
        for (int i = 0; i < RG; ++i) {
          const double a = fl[i * 4 * FK * 16];
          rp[i] = mfma4(a, fp, rp[i]);
          dpr[i] = mfma4(a, -fu, dpr[i]);
          dps[i] = mfma4(a, -fu, dps[i]);
          dpt[i] = mfma4(a, -fu, dpt[i]);
        }
      } else {
        double* G = f == 0 ? dpt : (f == 1 ? dps : dpr);
#pragma unroll
        for (int i = 0; i < RG; ++i) {
          const double a = fl[i * 4 * FK * 16];
          rp[i] = mfma4(a, fp, rp[i]);
          G[i] = mfma4(a, fu, G[i]);
        }
      }
    }
  }
  // point source S(tau) = amp (tau - t0) exp(-pi^2 f0^2 (tau - t0)^2) on its
  // element (the branch is uniform: only the source's wave takes it)
  {
    const double* sp = sh.srcp + 4 * shot;
    const bool src = (double)e == sp[0];
    if (__builtin_amdgcn_read_exec() & __ballot(src)) {
      const double tr = stage_time(sh) - sp[2], ar = M_PI * sp[1] * tr;
      const double src_s = sp[3] * tr * exp(-ar * ar);
      const double* src_w = sh.srcw + (size_t)shot * Np;
#pragma unroll
      for (int i = 0; i < RG; ++i)
        if (src) rp[i] += src_w[min(4 * i + g, Np - 1)] * src_s;
    }
  }

  // ---- LSRK update from the registers: 8 RG stores, every lane issuing
  // them (a lane without a row stores past the end of the resource, which
  // the hardware drops), so the count after the direct loads is fixed
  const bool live = irho != 0.0;
#pragma unroll
  for (int i = 0; i < RG; ++i) {
    const int n = 4 * i + g;
    const int nc = min(n, Np - 1);
    const unsigned o = (live && n < Np) ? tb + (unsigned)nc * (kTile * 8) : 0xFFFFFFF8u;
    const double a = dpr[i], bq_ = dps[i], c = dpt[i];
    const double rhs[4] = {rp[i],
                           -irho * (rx * a + sx * bq_ + tx * c),
                           -irho * (ry * a + sy * bq_ + ty * c),
                           -irho * (rz * a + sz * bq_ + tz * c)};
#pragma unroll
    for (int fl = 0; fl < 4; ++fl) {
      const double rr = A * rv[i][fl] + dt * rhs[fl];
      bstn(Rr, o, fl * FS, rr);
      bstn(Rn, o, fl * FS, qv[i][fl] + B * rr);
    }
  }
}

template <int N>
__global__ void __launch_bounds__(kWavesR * 64, 1) k_level3_dma(Lvl3 L, const double* __restrict__ qo,
                                                       double* __restrict__ qn,
                                                       double* __restrict__ res,
                                                       const double* __restrict__ qb3, double A,
                                                       double B, double dt, Shots sh) {
  using D = Dims3<N>;
  constexpr int Nfp = D::Nfp;
  extern __shared__ double sfrag[];
  int* smask = reinterpret_cast<int*>(sfrag);
  int* smap = smask + 4 * Nfp;
  constexpr int kTabDoubles = (4 * Nfp + 96 * Nfp + 1) / 2;
  const int lane = threadIdx.x & 63;
  const int ngrp = (L.ntile + kWavesR - 1) / kWavesR;
  const XcdRange rg_(ngrp * (long long)sh.n, L.order);
  double* sops = sfrag + kTabDoubles;
  char* buf = reinterpret_cast<char*>(sops + D::NFRAG * 16) +
              __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * BufR<N>::BYTES;
  // the first tile's loads overlap the table fill
  if (rg_.lo < rg_.hi) tile_dma<N>(L, qo, sh, rg_.lo, ngrp, buf, lane);
  fill_lds<kWavesR * 64, 4 * Nfp>(smask, L.fmask, threadIdx.x);
  fill_lds<kWavesR * 64, 96 * Nfp>(smap, L.fmap, threadIdx.x);
  fill_lds<kWavesR * 64, D::NFRAG * 16>(sops, L.ops, threadIdx.x);
  __syncthreads();
  for (long long it = rg_.lo; it < rg_.hi; it += rg_.step) {
    const long long nx = it + rg_.step;
    auto fetch = [&]() {
      if (nx < rg_.hi) tile_dma<N>(L, qo, sh, nx, ngrp, buf, lane);
    };
    tile_step_dma<N>(L, qo, qn, res, qb3, A, B, dt, sh, it, fetch, ngrp, smap, smask, sops, buf,
                     lane);
  }
}

// The same kernel over a group of contexts (meshes of any size, same N):
// one work list, member c owning the items [first_c, first_c + items_c);
// the tables and operators in LDS depend on N only.  The next item's direct
// loads may come from another member.
template <int N>
__global__ void __launch_bounds__(kWavesR * 64, 1) k_level3_dma_group(
    const Member3* __restrict__ G, int nm, long long total, double A, double B, double dt,
    double tau, double cs) {
  using D = Dims3<N>;
  constexpr int Nfp = D::Nfp;
  extern __shared__ double sfrag[];
  int* smask = reinterpret_cast<int*>(sfrag);
  int* smap = smask + 4 * Nfp;
  constexpr int kTabDoubles = (4 * Nfp + 96 * Nfp + 1) / 2;
  const int lane = threadIdx.x & 63;
  const XcdRange rg_(total, G[0].L.order);
  double* sops = sfrag + kTabDoubles;
  char* buf = reinterpret_cast<char*>(sops + D::NFRAG * 16) +
              __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * BufR<N>::BYTES;
  auto member = [&](long long it) {
    int c = 0;
    while (c + 1 < nm && G[c + 1].first <= it) ++c;
    return c;
  };
  auto shots = [&](int c) {
    Shots sh = G[c].sh;
    sh.tau = tau;
    sh.cs = cs;
    sh.clk = nullptr;
    return sh;
  };
  if (rg_.lo < rg_.hi) {
    const int c = member(rg_.lo);
    const Shots sh = shots(c);
    tile_dma<N>(G[c].L, static_cast<const double*>(G[c].qo), sh, rg_.lo - G[c].first, G[c].ngrp,
                buf, lane);
  }
  fill_lds<kWavesR * 64, 4 * Nfp>(smask, G[0].L.fmask, threadIdx.x);
  fill_lds<kWavesR * 64, 96 * Nfp>(smap, G[0].L.fmap, threadIdx.x);
  fill_lds<kWavesR * 64, D::NFRAG * 16>(sops, G[0].L.ops, threadIdx.x);
  __syncthreads();
  for (long long it = rg_.lo; it < rg_.hi; it += rg_.step) {
    const long long nx = it + rg_.step;
    const int c = member(it);
    const Shots sh = shots(c);
    auto fetch = [&]() {
      if (nx < rg_.hi) {
        const int cn = member(nx);
        const Shots shn = shots(cn);
        tile_dma<N>(G[cn].L, static_cast<const double*>(G[cn].qo), shn, nx - G[cn].first,
                    G[cn].ngrp, buf, lane);
      }
    };
    tile_step_dma<N>(G[c].L, static_cast<const double*>(G[c].qo), static_cast<double*>(G[c].qn),
                     static_cast<double*>(G[c].res), G[c].qb3, A, B, dt, sh, it - G[c].first,
                     fetch, G[c].ngrp, smap, smask, sops, buf, lane);
  }
}

// -------------------------------------------------------------- energy ---
// One block per tile; partial sum of J/2 (p M p / (rho c^2) + rho u M u),
// accumulated in FP64 whatever the state's type.
template <class T>
__global__ void __launch_bounds__(256) k_energy(Lvl3 L, const T* __restrict__ q,
                                                const double* __restrict__ mass,
                                                const double* __restrict__ J,
                                                double* __restrict__ out) {
  // the mass matrix and the tile's four fields in LDS (sized at launch)
  extern __shared__ double sm[];
  const int Np = L.Np, tile = blockIdx.x, tid = threadIdx.x;
  double* sq = sm + Np * Np;
  for (int i = tid; i < Np * Np; i += 256) sm[i] = mass[i];
  const T* qt = q + (size_t)tile * 4 * Np * kTile;
  for (int i = tid; i < 4 * Np * kTile; i += 256) sq[i] = (double)qt[i];
  __syncthreads();
  const int es = tid & 15, g = tid >> 4;
  const double* gt = L.geo + (size_t)tile * 12 * kTile + es;
  const double irho = gt[9 * kTile], Kb = gt[10 * kTile];
  double acc = 0.0;
  if (irho != 0.0) {
    const double rho = 1.0 / irho;
    for (int a = g; a < Np; a += 16) {
      double mq[4] = {0, 0, 0, 0};
      for (int b = 0; b < Np; ++b) {
        const double m = sm[a * Np + b];
#pragma unroll
        for (int f = 0; f < 4; ++f) mq[f] += m * sq[(f * Np + b) * kTile + es];
      }
      acc += sq[a * kTile + es] * mq[0] / Kb +
             rho * (sq[(Np + a) * kTile + es] * mq[1] + sq[(2 * Np + a) * kTile + es] * mq[2] +
                    sq[(3 * Np + a) * kTile + es] * mq[3]);
    }
    acc *= 0.5 * J[tile * kTile + es];
  }
  double* red = sq + 4 * Np * kTile;
  red[tid] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  if (tid == 0) out[tile] = red[0];
}

template <int N>
hipError_t launch3_dma(const Lvl3& L, const double* qo, double* qn, double* res,
                       const double* qb3, double A, double B, double dt, const Shots& sh,
                       hipStream_t st) {
  using D = Dims3<N>;
  constexpr int Nfp = D::Nfp;
  const size_t lds = sizeof(double) * ((4 * Nfp + 96 * Nfp + 1) / 2 + D::NFRAG * 16) +
                     (size_t)kWavesR * BufR<N>::BYTES;
  const int ngrp = (L.ntile + kWavesR - 1) / kWavesR;
  if (sh.n < 1) return hipErrorInvalidValue;
  int resident = 0;
  {
    const hipError_t e = kernel_setup((const void*)(k_level3_dma<N>), kWavesR * 64, lds, &resident);
    if (e != hipSuccess) return e;
  }
  const long long items = (long long)ngrp * sh.n;
  const int blocks = grid3(resident, items, L.eighths);
  hipLaunchKernelGGL(k_level3_dma<N>, dim3(blocks), dim3(kWavesR * 64), lds, st, L, qo, qn, res,
                     qb3, A, B, dt, sh);
  return hipGetLastError();
}

template <int N>
hipError_t launch3_group(const Member3* G, int nm, long long total, double A, double B,
                         double dt, double tau, double cs, hipStream_t st) {
  using D = Dims3<N>;
  constexpr int Nfp = D::Nfp;
  const size_t lds = sizeof(double) * ((4 * Nfp + 96 * Nfp + 1) / 2 + D::NFRAG * 16) +
                     (size_t)kWavesR * BufR<N>::BYTES;
  int resident = 0;
  {
    const hipError_t e =
        kernel_setup((const void*)(k_level3_dma_group<N>), kWavesR * 64, lds, &resident);
    if (e != hipSuccess) return e;
  }
  const int blocks = (int)std::max<long long>(8, std::min<long long>(resident, total) / 8 * 8);
  hipLaunchKernelGGL(k_level3_dma_group<N>, dim3(blocks), dim3(kWavesR * 64), lds, st, G, nm,
                     total, A, B, dt, tau, cs);
  return hipGetLastError();
}

template <int N, int W>
hipError_t launch3_reg_w(const Lvl3& L, const double* qo, double* qn, double* res,
                         const double* qb3, double A, double B, double dt, const Shots& sh,
                         hipStream_t st) {
  using D = Dims3<N>;
  constexpr int Nfp = D::Nfp;
  const size_t lds = sizeof(double) * ((4 * Nfp + 96 * Nfp + 1) / 2 + (D::kLds ? D::NFRAG * 16 : 0));
  const int ngrp = (L.ntile + W - 1) / W;
  if (sh.n < 1) return hipErrorInvalidValue;
  // persistent grid: as many workgroups as fit on the device at once
  int resident = 0;
  {
    const hipError_t e = kernel_setup((const void*)(k_level3<N, W>), W * 64, lds, &resident);
    if (e != hipSuccess) return e;
  }
  const long long items = (long long)ngrp * sh.n;
  // a multiple of 8, so that every XCD has blocks for its range of items
  const int blocks = grid3(resident, items, L.eighths);
  hipLaunchKernelGGL((k_level3<N, W>), dim3(blocks), dim3(W * 64), lds, st, L, qo, qn, res, qb3,
                     A, B, dt, sh);
  return hipGetLastError();
}

template <int N>
hipError_t launch3_reg(const Lvl3& L, const double* qo, double* qn, double* res,
                       const double* qb3, double A, double B, double dt, const Shots& sh,
                       hipStream_t st) {
  if (L.waves == 8) return launch3_reg_w<N, 8>(L, qo, qn, res, qb3, A, B, dt, sh, st);
  return launch3_reg_w<N, 4>(L, qo, qn, res, qb3, A, B, dt, sh, st);
}

// N <= 4: the tile-on-chip kernel (its registers and LDS hold a whole
// tile) unless tuning chose the other; N = 5, 6: the register-streaming
// kernel
template <int N>
hipError_t launch3(const Lvl3& L, const double* qo, double* qn, double* res, const double* qb3,
                   double A, double B, double dt, const Shots& sh, hipStream_t st) {
  if constexpr (N <= 4) {
    if (L.kvar == 0) return launch3_dma<N>(L, qo, qn, res, qb3, A, B, dt, sh, st);
  }
  return launch3_reg<N>(L, qo, qn, res, qb3, A, B, dt, sh, st);
}

}  // namespace

hipError_t launch_level3(const Lvl3& L, const double* qo, double* qn, double* res,
                         const double* qb3, double A, double B, double dt, const Shots& sh,
                         hipStream_t st) {
  switch (L.N) {
    case 1: return launch3<1>(L, qo, qn, res, qb3, A, B, dt, sh, st);
    case 2: return launch3<2>(L, qo, qn, res, qb3, A, B, dt, sh, st);
    case 3: return launch3<3>(L, qo, qn, res, qb3, A, B, dt, sh, st);
    case 4: return launch3<4>(L, qo, qn, res, qb3, A, B, dt, sh, st);
    case 5: return launch3<5>(L, qo, qn, res, qb3, A, B, dt, sh, st);
    case 6: return launch3<6>(L, qo, qn, res, qb3, A, B, dt, sh, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_level3_group(const Member3* G, int nm, long long total, int N, double A,
                               double B, double dt, double tau, double cs, hipStream_t st) {
  switch (N) {
    case 1: return launch3_group<1>(G, nm, total, A, B, dt, tau, cs, st);
    case 2: return launch3_group<2>(G, nm, total, A, B, dt, tau, cs, st);
    case 3: return launch3_group<3>(G, nm, total, A, B, dt, tau, cs, st);
    case 4: return launch3_group<4>(G, nm, total, A, B, dt, tau, cs, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_energy(const Lvl3& L, const void* q, int q_f32, const double* mass,
                         const double* J, double* out, hipStream_t st) {
  const size_t lds = sizeof(double) * ((size_t)L.Np * L.Np + 4 * L.Np * kTile + 256);
  // N = 6 needs more than the default 64 KB
  const hipError_t e = kernel_setup(
      q_f32 ? (const void*)k_energy<float> : (const void*)k_energy<double>, 256, lds, nullptr);
  if (e != hipSuccess) return e;
  if (q_f32)
    hipLaunchKernelGGL(k_energy<float>, dim3(L.ntile), dim3(256), lds, st, L,
                       static_cast<const float*>(q), mass, J, out);
  else
    hipLaunchKernelGGL(k_energy<double>, dim3(L.ntile), dim3(256), lds, st, L,
                       static_cast<const double*>(q), mass, J, out);
  return hipGetLastError();
}

}  // namespace dgh
