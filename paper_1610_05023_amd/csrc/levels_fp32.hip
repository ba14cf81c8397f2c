// FP32 variant of the 3D level (volume term + upwind surface term + LSRK
// update, Section 3.2): FP32 state and residual, contractions on the FP32
// 16x16x4 MFMA with FP32 accumulation.  The face, edge and corner levels
// stay FP64 and read the new 3D trace from this FP32 state; the HABC
// characteristic qb3 they return is rounded to FP32 here.
//
// Lane l of a wave holds element l%16 of its tile.  Per instruction:
//   A (operator rows 16 rb..16 rb+15, cols 4 j..4 j+3): lane l -> A[l%16][l/16]
//   B (fields at nodes 4 j + k of the 16 elements):     lane l -> B[l/16][l%16]
//   D (rows 16 rb + 4 (l/16) + r, r = 0..3):             four floats per lane
// so a lane's B operand is the node 4 j + l/16 (as in the FP64 kernel) and
// its accumulator rows are the nodes 16 rb + 4 (l/16) + r.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"
#include "launch.hpp"
#include "levels.hpp"

namespace dgh {

namespace {

// waves (tiles) per workgroup of the register-streaming kernels: W = 4 or
// 8 (Lvl3::waves, a tuning axis); with 8 the registers are sized for two
// waves per SIMD (256 each)

typedef float f4 __attribute__((ext_vector_type(4)));

template <int N>
struct Dims3f {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int RG = (Np + 3) / 4;     // volume k-steps of 4 nodes
  static constexpr int RB = (Np + 15) / 16;   // row blocks of 16 nodes
  static constexpr int FK = (Nfp + 3) / 4;    // lifting k-steps per face
  static constexpr int NOPS = (3 * RB * RG + RB * 4 * FK) * 64;   // floats
  // operator fragments in LDS up to 150 KB (N <= 6); above 64 KB the
  // register-streaming kernel runs one workgroup per CU, with 512 registers
  // per wave
  static constexpr bool kLds = NOPS * 4 <= 150 * 1024;
  static constexpr int kOcc = NOPS * 4 <= 64 * 1024 ? 2 : 1;
};

__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

using Rsrc = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ Rsrc rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           0x00020000);
}
__device__ __forceinline__ float fld(Rsrc r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
// streaming (non-temporal) load: read once per stage
__device__ __forceinline__ float fldn(Rsrc r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 2));
}
// store of the new state and residual, without the streaming hint: an FP32
// node row of a tile is 64 bytes, half a cache line, and streaming stores
// of the two halves reached HBM as separate partial writes (1.40 times the
// bytes at N = 5; plain stores write each line once)
__device__ __forceinline__ void fst(Rsrc r, unsigned voff, unsigned soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}

template <int N, int W>
__device__ __forceinline__ void tile_f32(const Lvl3& L, const float* __restrict__ qo,
                                         float* __restrict__ qn, float* __restrict__ res,
                                         const double* __restrict__ qb3, float A, float B,
                                         float dt, const Shots& sh, long long item, int ngrp,
                                         const int* smap, const int* smask, const float* sops,
                                         int lane) {
  using D = Dims3f<N>;
  constexpr int Np = D::Np, Nfp = D::Nfp, RG = D::RG, RB = D::RB, FK = D::FK;
  constexpr unsigned FS = Np * kTile * 4;   // bytes between two fields of a tile
  constexpr unsigned TS = 4 * FS;           // bytes per tile
  const int shot = (int)(item / ngrp);
  const int tile = (int)(item - (long long)shot * ngrp) * W + (threadIdx.x >> 6);
  if (tile >= L.ntile) return;
  qo += shot * sh.st3;
  qn += shot * sh.st3;
  res += shot * sh.st3;
  qb3 += shot * sh.stb3;
  const int es = lane & 15, g = lane >> 4;
  const float* frag = (D::kLds ? sops : L.ops32) + lane;
  const float* fragL = frag + 3 * RB * RG * 64;
  const int e = tile * kTile + es;
  const unsigned nbytes = (unsigned)L.ntile * TS;
  const Rsrc Rq = rsrc(qo, nbytes), Rn = rsrc(qn, nbytes), Rr = rsrc(res, nbytes);
  const unsigned tb = (unsigned)tile * TS + (unsigned)es * 4;   // this lane's element
  const double* gt = L.geo + (size_t)tile * 12 * kTile + es;
  const float rx = (float)gt[0 * kTile], ry = (float)gt[1 * kTile], rz = (float)gt[2 * kTile];
  const float sx = (float)gt[3 * kTile], sy = (float)gt[4 * kTile], sz = (float)gt[5 * kTile];
  const float tx = (float)gt[6 * kTile], ty = (float)gt[7 * kTile], tz = (float)gt[8 * kTile];
  const float irho = (float)gt[9 * kTile], Kb = (float)gt[10 * kTile], Z = (float)gt[11 * kTile];
  const int* nbrt = L.nbr + tile * 4 * kTile + es;
  const double* znt = L.zn + tile * 4 * kTile + es;
  int fcode[4];
  float fz[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    fcode[f] = nbrt[f * kTile];
    fz[f] = (float)znt[f * kTile];
  }

  // ---- volume: Dr p, Ds p, Dt p and div u = Dr fr + Ds fs + Dt ft
  f4 dpr[RB], dps[RB], dpt[RB], dv[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) dpr[b] = dps[b] = dpt[b] = dv[b] = f4{0, 0, 0, 0};
  constexpr int PF = (N <= 4 || D::kOcc == 1) ? 3 : 1;   // k-steps of loads in flight
  float bp[PF], bu[PF], bv[PF], bw[PF];
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    const unsigned o = tb + (unsigned)min(4 * k + g, Np - 1) * (kTile * 4);
    bp[k] = fld(Rq, o, 0);
    bu[k] = fld(Rq, o, FS);
    bv[k] = fld(Rq, o, 2 * FS);
    bw[k] = fld(Rq, o, 3 * FS);
  }
#pragma unroll 1
  for (int j0 = 0; j0 < RG; j0 += PF) {
#pragma unroll
    for (int sl = 0; sl < PF; ++sl) {
      const int j = j0 + sl;
      if (j < RG) {
        const float p = bp[sl], u = bu[sl], v = bv[sl], w = bw[sl];
        {
          const unsigned o = tb + (unsigned)min(4 * (j + PF) + g, Np - 1) * (kTile * 4);
          bp[sl] = fld(Rq, o, 0);
          bu[sl] = fld(Rq, o, FS);
          bv[sl] = fld(Rq, o, 2 * FS);
          bw[sl] = fld(Rq, o, 3 * FS);
        }
        const float fr = rx * u + ry * v + rz * w;
        const float fs = sx * u + sy * v + sz * w;
        const float ft = tx * u + ty * v + tz * w;
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          const float ar = frag[((0 * RB + b) * RG + j) * 64];
          const float as = frag[((1 * RB + b) * RG + j) * 64];
          const float at = frag[((2 * RB + b) * RG + j) * 64];
          dpr[b] = mfma16(ar, p, dpr[b]);
          dps[b] = mfma16(as, p, dps[b]);
          dpt[b] = mfma16(at, p, dpt[b]);
          dv[b] = mfma16(ar, fr, dv[b]);
          dv[b] = mfma16(as, fs, dv[b]);
          dv[b] = mfma16(at, ft, dv[b]);
        }
      }
    }
  }
#pragma unroll
  for (int b = 0; b < RB; ++b) dv[b] *= -Kb;
  f4* rp = dv;

  // ---- surface (the FP64 kernel's scheme: one upwind flux against the
  // exterior state, the pressure jump lifted into the reference gradient)
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    __builtin_amdgcn_sched_barrier(0);
    const float cr = f == 2 ? 1.f : (f == 3 ? -1.f : 0.f);
    const float cs = f == 2 ? 1.f : (f == 1 ? -1.f : 0.f);
    const float ct = f == 2 ? 1.f : (f == 0 ? -1.f : 0.f);
    float nx = cr * rx + cs * sx + ct * tx;
    float ny = cr * ry + cs * sy + ct * ty;
    float nz = cr * rz + cs * sz + ct * tz;
    const float fsc = sqrtf(nx * nx + ny * ny + nz * nz);
    const float inv = 1.f / fsc;
    nx *= inv;
    ny *= inv;
    nz *= inv;
    const int code = fcode[f];
    const float ZP = fz[f];
    const bool inner = code >= 0;
    const int cb = -1 - code;
    const bool hb = !inner && (cb & 3) == 0;
    const bool dir = !inner && (cb & 3) == 2;
    const int e2 = inner ? (code >> 5) : e;
    const unsigned nb = (unsigned)(e2 >> 4) * TS + (unsigned)(e2 & 15) * 4;
    const int mapbase = inner ? ((f * 4 + ((code >> 3) & 3)) * 6 + (code & 7)) * Nfp
                              : ((f * 4) * 6 + ((cb >> 2) & 7)) * Nfp;
    const double* qbt = qb3 + (size_t)(hb ? (cb >> 5) : 0) * Nfp;
    const float iZ = 1.f / (Z + ZP);
    const float aM = ZP * iZ, aP = Z * iZ, bZ = Z * aM;
    const float cP = fsc * Kb;
#pragma unroll
    for (int jj = 0; jj < FK; ++jj) {
      const int kc = min(4 * jj + g, Nfp - 1);
      const int n = smask[f * Nfp + kc];
      const int n2 = smap[mapbase + kc];
      const unsigned oM = tb + (unsigned)n * (kTile * 4);
      const unsigned oP = nb + (unsigned)n2 * (kTile * 4);
      const float pM = fld(Rq, oM, 0), uM = fld(Rq, oM, FS), vM = fld(Rq, oM, 2 * FS),
                  wM = fld(Rq, oM, 3 * FS);
      const float pP = fld(Rq, oP, 0), uP = fld(Rq, oP, FS), vP = fld(Rq, oP, 2 * FS),
                  wP = fld(Rq, oP, 3 * FS);
      const float rb = (float)qbt[min(n2, Nfp - 1)];
      const float unM = nx * uM + ny * vM + nz * wM;
      const float unP = nx * uP + ny * vP + nz * wP;
      const float pG = inner ? pP : (dir ? -pM : (hb ? 2.f * rb : 0.f));
      const float uG = inner ? unP : (dir ? unM : 0.f);
      const float pF = aM * pM + aP * pG + bZ * (unM - uG);
      const float unF = iZ * (pM - pG) + aP * unM + aM * uG;
      const float fp = cP * (unM - unF);
      const float fu = pM - pF;
      const float* fl = fragL + (f * FK + jj) * 64;
      if (f == 2) {
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          const float a = fl[b * 4 * FK * 64];
          rp[b] = mfma16(a, fp, rp[b]);
          dpr[b] = mfma16(a, -fu, dpr[b]);
          dps[b] = mfma16(a, -fu, dps[b]);
          dpt[b] = mfma16(a, -fu, dpt[b]);
        }
      } else {
        f4* G = f == 0 ? dpt : (f == 1 ? dps : dpr);
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          const float a = fl[b * 4 * FK * 64];
          rp[b] = mfma16(a, fp, rp[b]);
          G[b] = mfma16(a, fu, G[b]);
        }
      }
    }
  }

  // ---- LSRK update of the four rows per row block this lane holds
  const bool live = irho != 0.f;
  const double* sp = sh.srcp + 4 * shot;
  const bool src = (double)e == sp[0];
  const double trr = stage_time(sh) - sp[2], arr = M_PI * sp[1] * trr;
  const float src_s = (float)(sp[3] * trr * exp(-arr * arr));
  const double* src_w = sh.srcw + (size_t)shot * Np;
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    __builtin_amdgcn_sched_barrier(0);
    float ro[4][4], qv[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const unsigned o = tb + (unsigned)min(16 * b + 4 * g + r, Np - 1) * (kTile * 4);
#pragma unroll
      for (int fl = 0; fl < 4; ++fl) {
        ro[r][fl] = fldn(Rr, o, fl * FS);
        qv[r][fl] = fld(Rq, o, fl * FS);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = 16 * b + 4 * g + r;
      const int nc = min(n, Np - 1);
      const unsigned o = tb + (unsigned)nc * (kTile * 4);
      const float sw = (float)src_w[nc];
      const float a = dpr[b][r], bq = dps[b][r], c = dpt[b][r];
      const float rhs[4] = {rp[b][r] + (src ? sw * src_s : 0.f),
                            -irho * (rx * a + sx * bq + tx * c),
                            -irho * (ry * a + sy * bq + ty * c),
                            -irho * (rz * a + sz * bq + tz * c)};
      if (live && n < Np) {
#pragma unroll
        for (int fl = 0; fl < 4; ++fl) {
          const float rr = A * ro[r][fl] + dt * rhs[fl];
          fst(Rr, o, fl * FS, rr);
          fst(Rn, o, fl * FS, qv[r][fl] + B * rr);
        }
      }
    }
  }
}

template <int N, int W>
__global__ void __launch_bounds__(W * 64, W == 8 ? 1 : Dims3f<N>::kOcc) k_level3_f32(Lvl3 L, const float* __restrict__ qo,
                                                        float* __restrict__ qn,
                                                        float* __restrict__ res,
                                                        const double* __restrict__ qb3, float A,
                                                        float B, float dt, Shots sh) {
  using D = Dims3f<N>;
  constexpr int Nfp = D::Nfp;
  extern __shared__ float sfl[];
  int* smask = reinterpret_cast<int*>(sfl);
  int* smap = smask + 4 * Nfp;
  float* sops = sfl + 4 * Nfp + 96 * Nfp;
  fill_lds<W * 64, 4 * Nfp>(smask, L.fmask, threadIdx.x);
  fill_lds<W * 64, 96 * Nfp>(smap, L.fmap, threadIdx.x);
  if (D::kLds) fill_lds<W * 64, D::NOPS>(sops, L.ops32, threadIdx.x);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int ngrp = (L.ntile + W - 1) / W;
  const XcdRange rg_(ngrp * (long long)sh.n, L.order);
  for (long long item = rg_.lo; item < rg_.hi; item += rg_.step)
    tile_f32<N, W>(L, qo, qn, res, qb3, A, B, dt, sh, item, ngrp, smap, smask, sops, lane);
}

// ------------------------------------------------- FP32, tile on chip ---
// N <= 5: one workgroup of four waves per CU (one per SIMD).  Each wave's
// LDS buffer receives its next tile (FP32 state, geometry, impedances, face
// codes) by direct buffer-to-LDS loads, issued once the current tile's copy
// has been read for the last time (before the last face), so every value
// of q and res crosses HBM once; the wait at the start of a tile leaves the
// previous update's stores in flight (they follow the direct loads).
constexpr int kWavesF = 4;

template <int N>
struct BufF {
  static constexpr int Np = Dims3f<N>::Np;
  static constexpr int QK = (Np * 256 + 1023) / 1024;   // 1 KB loads for the state
  static constexpr int QB = QK * 1024;
  static constexpr int GEO = QB, ZN = QB + 2048, NBR = QB + 3072;
  static constexpr int BYTES = QB + 4096;
};

typedef __attribute__((address_space(3))) void* lds_ptr_f;

template <int N>
__device__ __forceinline__ void tile_dma_f(const Lvl3& L, const float* __restrict__ qo,
                                           const Shots& sh, long long item, int ngrp, char* buf,
                                           int lane) {
  using D = Dims3f<N>;
  using BR = BufF<N>;
  constexpr unsigned TS = 4 * D::Np * kTile * 4;
  const int shot = (int)(item / ngrp);
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int tile = min((int)(item - (long long)shot * ngrp) * kWavesF + wv, L.ntile - 1);
  const Rsrc Rq = rsrc(qo + shot * sh.st3, (unsigned)L.ntile * TS);
  const Rsrc Rg = rsrc(L.geo, (unsigned)L.ntile * 12 * kTile * 8);
  const Rsrc Rz = rsrc(L.zn, (unsigned)L.ntile * 4 * kTile * 8);
  const Rsrc Rc = rsrc(L.nbr, (unsigned)L.ntile * 4 * kTile * 4);
  const int vo = lane * 16;
#pragma unroll
  for (int k = 0; k < BR::QK; ++k)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(Rq, (lds_ptr_f)(buf + k * 1024), 16, vo,
                                             (int)((unsigned)tile * TS + k * 1024), 0, 0);
#pragma unroll
  for (int k = 0; k < 2; ++k)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(Rg, (lds_ptr_f)(buf + BR::GEO + k * 1024), 16, vo,
                                             tile * 12 * kTile * 8 + k * 1024, 0, 0);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(Rz, (lds_ptr_f)(buf + BR::ZN), 16, vo,
                                           tile * 4 * kTile * 8, 0, 0);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(Rc, (lds_ptr_f)(buf + BR::NBR), 16, vo,
                                           tile * 4 * kTile * 4, 0, 0);
}

template <int N>
struct FaceInF {
  static constexpr int FK = Dims3f<N>::FK;
  float p[FK], u[FK], v[FK], w[FK], rb[FK];
};

template <int N>
__device__ __forceinline__ void face_fetch_f(FaceInF<N>& x, int f, int code, int e, Rsrc Rq,
                                             const double* __restrict__ qb3, const int* smap,
                                             int g) {
  using D = Dims3f<N>;
  constexpr int Np = D::Np, Nfp = D::Nfp, FK = D::FK;
  constexpr unsigned FS = Np * kTile * 4, TS = 4 * FS;
  const bool inner = code >= 0;
  const int cb = -1 - code;
  const bool hb = !inner && (cb & 3) == 0;
  const int e2 = inner ? (code >> 5) : e;
  const unsigned nb = (unsigned)(e2 >> 4) * TS + (unsigned)(e2 & 15) * 4;
  const int mapbase = inner ? ((f * 4 + ((code >> 3) & 3)) * 6 + (code & 7)) * Nfp
                            : ((f * 4) * 6 + ((cb >> 2) & 7)) * Nfp;
  const double* qbt = qb3 + (size_t)(hb ? (cb >> 5) : 0) * Nfp;
#pragma unroll
  for (int jj = 0; jj < FK; ++jj) {
    const int kc = min(4 * jj + g, Nfp - 1);
    const int n2 = smap[mapbase + kc];
    const unsigned oP = nb + (unsigned)n2 * (kTile * 4);
    x.p[jj] = fld(Rq, oP, 0);
    x.u[jj] = fld(Rq, oP, FS);
    x.v[jj] = fld(Rq, oP, 2 * FS);
    x.w[jj] = fld(Rq, oP, 3 * FS);
    x.rb[jj] = (float)qbt[min(n2, Nfp - 1)];
  }
}

// One work item whose tile is in buf; fetch_next() issues the direct loads
// of the next item (if any) once the tile's copy has been read.
template <int N, class Fetch>
__device__ __forceinline__ void tile_f32_dma(const Lvl3& L, const float* __restrict__ qo,
                                             float* __restrict__ qn, float* __restrict__ res,
                                             const double* __restrict__ qb3, float A, float B,
                                             float dt, const Shots& sh, long long item,
                                             Fetch fetch_next, int ngrp, const int* smap,
                                             const int* smask, const float* sops, char* buf,
                                             int lane) {
  using D = Dims3f<N>;
  using BR = BufF<N>;
  constexpr int Np = D::Np, Nfp = D::Nfp, RG = D::RG, RB = D::RB, FK = D::FK;
  constexpr unsigned FS = Np * kTile * 4;   // bytes between two fields of a tile
  constexpr unsigned TS = 4 * FS;           // bytes per tile
  const int shot = (int)(item / ngrp);
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int tile = (int)(item - (long long)shot * ngrp) * kWavesF + wv;
  // the tile's direct loads have landed: vector memory operations complete in
  // order and the previous tile issued 32 RB stores after them (the compiler
  // does not order LDS reads after direct-to-LDS loads by itself)
  constexpr int kVm = 32 * RB < 63 ? 32 * RB : 63;
  __builtin_amdgcn_s_waitcnt((kVm & 15) | ((kVm >> 4) << 14) | (7 << 4) | (15 << 8));
  if (tile >= L.ntile) {
    // no stores follow: wait for the next tile's direct loads here
    __builtin_amdgcn_s_waitcnt(0);
    fetch_next();
    __builtin_amdgcn_s_waitcnt(0);
    return;
  }
  const float* qos = qo + shot * sh.st3;
  float* qns = qn + shot * sh.st3;
  float* ress = res + shot * sh.st3;
  const double* qbs = qb3 + shot * sh.stb3;
  const int es = lane & 15, g = lane >> 4;
  const float* frag = sops + lane;
  const float* fragL = frag + 3 * RB * RG * 64;
  const int e = tile * kTile + es;
  const unsigned nbytes = (unsigned)L.ntile * TS;
  const Rsrc Rq = rsrc(qos, nbytes), Rn = rsrc(qns, nbytes), Rr = rsrc(ress, nbytes);
  const unsigned tb = (unsigned)tile * TS + (unsigned)es * 4;   // this lane's element
  const float* bq = reinterpret_cast<const float*>(buf) + es;    // [field][node][16]
  const double* bg = reinterpret_cast<const double*>(buf + BR::GEO) + es;
  const double* bz = reinterpret_cast<const double*>(buf + BR::ZN) + es;
  const int* bc = reinterpret_cast<const int*>(buf + BR::NBR) + es;
  int fcode[4];
  float fz[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    fcode[f] = bc[f * kTile];
    fz[f] = (float)bz[f * kTile];
  }
  FaceInF<N> fb[4];
#pragma unroll
  for (int f = 0; f < 3; ++f) face_fetch_f<N>(fb[f], f, fcode[f], e, Rq, qbs, smap, g);
  const float rx = (float)bg[0 * kTile], ry = (float)bg[1 * kTile], rz = (float)bg[2 * kTile];
  const float sx = (float)bg[3 * kTile], sy = (float)bg[4 * kTile], sz = (float)bg[5 * kTile];
  const float tx = (float)bg[6 * kTile], ty = (float)bg[7 * kTile], tz = (float)bg[8 * kTile];
  const float irho = (float)bg[9 * kTile], Kb = (float)bg[10 * kTile], Z = (float)bg[11 * kTile];

  // ---- volume (as in tile_f32), B operands from the LDS copy
  f4 dpr[RB], dps[RB], dpt[RB], dv[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) dpr[b] = dps[b] = dpt[b] = dv[b] = f4{0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < RG; ++j) {
    const int n = min(4 * j + g, Np - 1);
    const float p = bq[n * kTile], u = bq[(Np + n) * kTile], v = bq[(2 * Np + n) * kTile],
                w = bq[(3 * Np + n) * kTile];
    const float fr = rx * u + ry * v + rz * w;
    const float fs = sx * u + sy * v + sz * w;
    const float ft = tx * u + ty * v + tz * w;
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const float ar = frag[((0 * RB + b) * RG + j) * 64];
      const float as = frag[((1 * RB + b) * RG + j) * 64];
      const float at = frag[((2 * RB + b) * RG + j) * 64];
      dpr[b] = mfma16(ar, p, dpr[b]);
      dps[b] = mfma16(as, p, dps[b]);
      dpt[b] = mfma16(at, p, dpt[b]);
      dv[b] = mfma16(ar, fr, dv[b]);
      dv[b] = mfma16(as, fs, dv[b]);
      dv[b] = mfma16(at, ft, dv[b]);
    }
  }
#pragma unroll
  for (int b = 0; b < RB; ++b) dv[b] *= -Kb;
  f4* rp = dv;

  // ---- surface (as in tile_f32); own traces from the LDS copy
  float rv[RB][4][4], qd[RB][4][4], own3[FK][4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    __builtin_amdgcn_sched_barrier(0);
    if (f == 0) {
      face_fetch_f<N>(fb[3], 3, fcode[3], e, Rq, qbs, smap, g);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (f == 1) {
      // the residual of this tile at the update's rows
#pragma unroll
      for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const unsigned o = tb + (unsigned)min(16 * b + 4 * g + r, Np - 1) * (kTile * 4);
#pragma unroll
          for (int fl = 0; fl < 4; ++fl) rv[b][r][fl] = fldn(Rr, o, fl * FS);
        }
      __builtin_amdgcn_sched_barrier(0);
    }
    if (f == 3) {
      // the last reads of the copy (face 3's own traces, the update's q),
      // then the next tile's direct loads
#pragma unroll
      for (int jj = 0; jj < FK; ++jj) {
        const int n = smask[3 * Nfp + min(4 * jj + g, Nfp - 1)];
#pragma unroll
        for (int fl = 0; fl < 4; ++fl) own3[jj][fl] = bq[(fl * Np + n) * kTile];
      }
#pragma unroll
      for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int n = min(16 * b + 4 * g + r, Np - 1);
#pragma unroll
          for (int fl = 0; fl < 4; ++fl) qd[b][r][fl] = bq[(fl * Np + n) * kTile];
        }
      __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): every LDS read returned
      __builtin_amdgcn_sched_barrier(0);
      fetch_next();
      __builtin_amdgcn_sched_barrier(0);
    }
    const FaceInF<N>& x = fb[f];
    const float cr = f == 2 ? 1.f : (f == 3 ? -1.f : 0.f);
    const float cs = f == 2 ? 1.f : (f == 1 ? -1.f : 0.f);
    const float ct = f == 2 ? 1.f : (f == 0 ? -1.f : 0.f);
    float nx = cr * rx + cs * sx + ct * tx;
    float ny = cr * ry + cs * sy + ct * ty;
    float nz = cr * rz + cs * sz + ct * tz;
    const float fsc = sqrtf(nx * nx + ny * ny + nz * nz);
    const float inv = 1.f / fsc;
    nx *= inv;
    ny *= inv;
    nz *= inv;
    const int code = fcode[f];
    const float ZP = fz[f];
    const bool inner = code >= 0;
    const int cb = -1 - code;
    const bool hb = !inner && (cb & 3) == 0;
    const bool dir = !inner && (cb & 3) == 2;
    const float iZ = 1.f / (Z + ZP);
    const float aM = ZP * iZ, aP = Z * iZ, bZ = Z * aM;
    const float cP = fsc * Kb;
#pragma unroll
    for (int jj = 0; jj < FK; ++jj) {
      float pM, uM, vM, wM;
      if (f == 3) {
        pM = own3[jj][0];
        uM = own3[jj][1];
        vM = own3[jj][2];
        wM = own3[jj][3];
      } else {
        const int n = smask[f * Nfp + min(4 * jj + g, Nfp - 1)];
        pM = bq[n * kTile];
        uM = bq[(Np + n) * kTile];
        vM = bq[(2 * Np + n) * kTile];
        wM = bq[(3 * Np + n) * kTile];
      }
      const float pP = x.p[jj], uP = x.u[jj], vP = x.v[jj], wP = x.w[jj];
      const float unM = nx * uM + ny * vM + nz * wM;
      const float unP = nx * uP + ny * vP + nz * wP;
      const float pG = inner ? pP : (dir ? -pM : (hb ? 2.f * x.rb[jj] : 0.f));
      const float uG = inner ? unP : (dir ? unM : 0.f);
      const float pF = aM * pM + aP * pG + bZ * (unM - uG);
      const float unF = iZ * (pM - pG) + aP * unM + aM * uG;
      const float fp = cP * (unM - unF);
      const float fu = pM - pF;
      const float* fl = fragL + (f * FK + jj) * 64;
      if (f == 2) {
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          const float a = fl[b * 4 * FK * 64];
          rp[b] = mfma16(a, fp, rp[b]);
          dpr[b] = mfma16(a, -fu, dpr[b]);
          dps[b] = mfma16(a, -fu, dps[b]);
          dpt[b] = mfma16(a, -fu, dpt[b]);
        }
      } else {
        f4* G = f == 0 ? dpt : (f == 1 ? dps : dpr);
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          const float a = fl[b * 4 * FK * 64];
          rp[b] = mfma16(a, fp, rp[b]);
          G[b] = mfma16(a, fu, G[b]);
        }
      }
    }
  }

  // point source on its element (a uniform branch only that wave takes)
  {
    const double* sp = sh.srcp + 4 * shot;
    const bool src = (double)e == sp[0];
    if (__builtin_amdgcn_read_exec() & __ballot(src)) {
      const double trr = stage_time(sh) - sp[2], arr = M_PI * sp[1] * trr;
      const float src_s = (float)(sp[3] * trr * exp(-arr * arr));
      const double* src_w = sh.srcw + (size_t)shot * Np;
#pragma unroll
      for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (src) rp[b][r] += (float)src_w[min(16 * b + 4 * g + r, Np - 1)] * src_s;
    }
  }

  // ---- LSRK update: 32 RB stores, every lane issuing them (a lane without
  // a row stores past the end of the resource, which the hardware drops)
  __builtin_amdgcn_sched_barrier(0);
  const bool live = irho != 0.f;
#pragma unroll
  for (int b = 0; b < RB; ++b) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = 16 * b + 4 * g + r;
      const unsigned o = (live && n < Np) ? tb + (unsigned)n * (kTile * 4) : 0xFFFFFFF8u;
      const float a = dpr[b][r], bq_ = dps[b][r], c = dpt[b][r];
      const float rhs[4] = {rp[b][r],
                            -irho * (rx * a + sx * bq_ + tx * c),
                            -irho * (ry * a + sy * bq_ + ty * c),
                            -irho * (rz * a + sz * bq_ + tz * c)};
#pragma unroll
      for (int fl = 0; fl < 4; ++fl) {
        const float rr = A * rv[b][r][fl] + dt * rhs[fl];
        fst(Rr, o, fl * FS, rr);
        fst(Rn, o, fl * FS, qd[b][r][fl] + B * rr);
      }
    }
  }
}

template <int N>
__global__ void __launch_bounds__(kWavesF * 64, 1) k_level3_f32_dma(
    Lvl3 L, const float* __restrict__ qo, float* __restrict__ qn, float* __restrict__ res,
    const double* __restrict__ qb3, float A, float B, float dt, Shots sh) {
  using D = Dims3f<N>;
  constexpr int Nfp = D::Nfp;
  extern __shared__ float sfl[];
  int* smask = reinterpret_cast<int*>(sfl);
  int* smap = smask + 4 * Nfp;
  float* sops = sfl + 4 * Nfp + 96 * Nfp;
  const int lane = threadIdx.x & 63;
  const int ngrp = (L.ntile + kWavesF - 1) / kWavesF;
  const XcdRange rg_(ngrp * (long long)sh.n, L.order);
  char* buf = reinterpret_cast<char*>(sops + D::NOPS) +
              __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * BufF<N>::BYTES;
  if (rg_.lo < rg_.hi) tile_dma_f<N>(L, qo, sh, rg_.lo, ngrp, buf, lane);
  fill_lds<kWavesF * 64, 4 * Nfp>(smask, L.fmask, threadIdx.x);
  fill_lds<kWavesF * 64, 96 * Nfp>(smap, L.fmap, threadIdx.x);
  fill_lds<kWavesF * 64, D::NOPS>(sops, L.ops32, threadIdx.x);
  __syncthreads();
  for (long long it = rg_.lo; it < rg_.hi; it += rg_.step) {
    const long long nx = it + rg_.step;
    auto fetch = [&]() {
      if (nx < rg_.hi) tile_dma_f<N>(L, qo, sh, nx, ngrp, buf, lane);
    };
    tile_f32_dma<N>(L, qo, qn, res, qb3, A, B, dt, sh, it, fetch, ngrp, smap, smask, sops, buf,
                    lane);
  }
}

// The same kernel over a group of contexts (any mesh sizes, same N): one
// work list, member c owning [first_c, first_c + items_c); the LDS tables
// and operators depend on N only.
template <int N>
__global__ void __launch_bounds__(kWavesF * 64, 1) k_level3_f32_dma_group(
    const Member3* __restrict__ G, int nm, long long total, float A, float B, float dt,
    double tau, double cs) {
  using D = Dims3f<N>;
  constexpr int Nfp = D::Nfp;
  extern __shared__ float sfl[];
  int* smask = reinterpret_cast<int*>(sfl);
  int* smap = smask + 4 * Nfp;
  float* sops = sfl + 4 * Nfp + 96 * Nfp;
  const int lane = threadIdx.x & 63;
  const XcdRange rg_(total, G[0].L.order);
  char* buf = reinterpret_cast<char*>(sops + D::NOPS) +
              __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * BufF<N>::BYTES;
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
    tile_dma_f<N>(G[c].L, static_cast<const float*>(G[c].qo), shots(c), rg_.lo - G[c].first,
                  G[c].ngrp, buf, lane);
  }
  fill_lds<kWavesF * 64, 4 * Nfp>(smask, G[0].L.fmask, threadIdx.x);
  fill_lds<kWavesF * 64, 96 * Nfp>(smap, G[0].L.fmap, threadIdx.x);
  fill_lds<kWavesF * 64, D::NOPS>(sops, G[0].L.ops32, threadIdx.x);
  __syncthreads();
  for (long long it = rg_.lo; it < rg_.hi; it += rg_.step) {
    const long long nx = it + rg_.step;
    const int c = member(it);
    const Shots sh = shots(c);
    auto fetch = [&]() {
      if (nx < rg_.hi) {
        const int cn = member(nx);
        tile_dma_f<N>(G[cn].L, static_cast<const float*>(G[cn].qo), shots(cn),
                      nx - G[cn].first, G[cn].ngrp, buf, lane);
      }
    };
    tile_f32_dma<N>(G[c].L, static_cast<const float*>(G[c].qo), static_cast<float*>(G[c].qn),
                    static_cast<float*>(G[c].res), G[c].qb3, A, B, dt, sh, it - G[c].first,
                    fetch, G[c].ngrp, smap, smask, sops, buf, lane);
  }
}

template <int N>
hipError_t launch3f_group(const Member3* G, int nm, long long total, double A, double B,
                          double dt, double tau, double cs, hipStream_t st) {
  using D = Dims3f<N>;
  constexpr int Nfp = D::Nfp;
  const size_t lds = sizeof(float) * (4 * Nfp + 96 * Nfp + D::NOPS) +
                     (size_t)kWavesF * BufF<N>::BYTES;
  int resident = 0;
  {
    const hipError_t e =
        kernel_setup((const void*)(k_level3_f32_dma_group<N>), kWavesF * 64, lds, &resident);
    if (e != hipSuccess) return e;
  }
  const int blocks = (int)std::max<long long>(8, std::min<long long>(resident, total) / 8 * 8);
  hipLaunchKernelGGL(k_level3_f32_dma_group<N>, dim3(blocks), dim3(kWavesF * 64), lds, st, G, nm,
                     total, (float)A, (float)B, (float)dt, tau, cs);
  return hipGetLastError();
}

template <int N>
hipError_t launch3f_dma(const Lvl3& L, const float* qo, float* qn, float* res, const double* qb3,
                        double A, double B, double dt, const Shots& sh, hipStream_t st) {
  using D = Dims3f<N>;
  constexpr int Nfp = D::Nfp;
  const size_t lds = sizeof(float) * (4 * Nfp + 96 * Nfp + D::NOPS) +
                     (size_t)kWavesF * BufF<N>::BYTES;
  if (sh.n < 1) return hipErrorInvalidValue;
  const int ngrp = (L.ntile + kWavesF - 1) / kWavesF;
  int resident = 0;
  {
    const hipError_t e =
        kernel_setup((const void*)(k_level3_f32_dma<N>), kWavesF * 64, lds, &resident);
    if (e != hipSuccess) return e;
  }
  const long long items = (long long)ngrp * sh.n;
  const int blocks = grid3(resident, items, L.eighths);
  hipLaunchKernelGGL(k_level3_f32_dma<N>, dim3(blocks), dim3(kWavesF * 64), lds, st, L, qo, qn,
                     res, qb3, (float)A, (float)B, (float)dt, sh);
  return hipGetLastError();
}

template <int N, int W>
hipError_t launch3f_reg(const Lvl3& L, const float* qo, float* qn, float* res, const double* qb3,
                        double A, double B, double dt, const Shots& sh, hipStream_t st) {
  using D = Dims3f<N>;
  constexpr int Nfp = D::Nfp;
  const size_t lds = sizeof(float) * (4 * Nfp + 96 * Nfp + (D::kLds ? D::NOPS : 0));
  const int ngrp = (L.ntile + W - 1) / W;
  if (sh.n < 1) return hipErrorInvalidValue;
  int resident = 0;
  {
    const hipError_t e = kernel_setup((const void*)(k_level3_f32<N, W>), W * 64, lds, &resident);
    if (e != hipSuccess) return e;
  }
  const long long items = (long long)ngrp * sh.n;
  const int blocks = grid3(resident, items, L.eighths);
  hipLaunchKernelGGL((k_level3_f32<N, W>), dim3(blocks), dim3(W * 64), lds, st, L, qo, qn, res,
                     qb3, (float)A, (float)B, (float)dt, sh);
  return hipGetLastError();
}

template <int N>
hipError_t launch3f(const Lvl3& L, const float* qo, float* qn, float* res, const double* qb3,
                    double A, double B, double dt, const Shots& sh, hipStream_t st) {
  if constexpr (N <= 5) {   // the tile buffers and fragments fit the LDS up to N = 5
    if (L.kvar == 0) return launch3f_dma<N>(L, qo, qn, res, qb3, A, B, dt, sh, st);
  }
  if (L.waves == 8) return launch3f_reg<N, 8>(L, qo, qn, res, qb3, A, B, dt, sh, st);
  return launch3f_reg<N, 4>(L, qo, qn, res, qb3, A, B, dt, sh, st);
}

// ------------------------------------------------ BF16 contractions ---
// The FP32-state kernel with the volume and LIFT contractions on the BF16
// 16x16x16 MFMA (FP32 accumulation): the operator fragments are BF16 (from
// the host), the field values and fluxes are rounded to BF16 as they enter
// an instruction; the state, the residual, the fluxes and the update stay
// FP32.  Per instruction (K = 16):
//   A: lane l -> A[l%16][4 (l/16) + i], i = 0..3 (four BF16 in 8 bytes)
//   B: lane l -> B[4 (l/16) + i][l%16]
//   D: rows 4 (l/16) + r of column l%16 (as the FP32 instruction)
// so a lane's B operand of k-step j is the nodes 16 j + 4 (l/16) + i of its
// element, and its accumulator rows 16 b + 4 (l/16) + r.
typedef short s4 __attribute__((ext_vector_type(4)));

template <int N>
struct Dims3b {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int RB = (Np + 15) / 16;   // row blocks (and volume k-steps) of 16 nodes
  static constexpr int FK = (Nfp + 15) / 16;  // lifting k-steps per face
  static constexpr int NFR = 3 * RB * RB + RB * 4 * FK;   // fragments of 64 lanes x 8 bytes
  static constexpr int kOcc = NFR * 512 <= 64 * 1024 ? 2 : 1;
};

__device__ __forceinline__ f4 mfma_bf16(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// four FP32 -> BF16, round to nearest even: two v_cvt_pk_bf16_f32
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float fl2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ s4 pack4(const float* v) {
  const bf2 lo = __builtin_convertvector(fl2{v[0], v[1]}, bf2);
  const bf2 hi = __builtin_convertvector(fl2{v[2], v[3]}, bf2);
  return __builtin_bit_cast(
      s4, u32x2f{__builtin_bit_cast(unsigned, lo), __builtin_bit_cast(unsigned, hi)});
}

template <int N, int W>
__device__ __forceinline__ void tile_bf16(const Lvl3& L, const float* __restrict__ qo,
                                          float* __restrict__ qn, float* __restrict__ res,
                                          const double* __restrict__ qb3, float A, float B,
                                          float dt, const Shots& sh, long long item, int ngrp,
                                          const int* smap, const int* smask, const s4* sops,
                                          int lane) {
  using D = Dims3b<N>;
  constexpr int Np = D::Np, Nfp = D::Nfp, RB = D::RB, FK = D::FK;
  constexpr unsigned FS = Np * kTile * 4;   // bytes between two fields of a tile
  constexpr unsigned TS = 4 * FS;           // bytes per tile
  const int shot = (int)(item / ngrp);
  const int tile = (int)(item - (long long)shot * ngrp) * W + (threadIdx.x >> 6);
  if (tile >= L.ntile) return;
  qo += shot * sh.st3;
  qn += shot * sh.st3;
  res += shot * sh.st3;
  qb3 += shot * sh.stb3;
  const int es = lane & 15, g = lane >> 4;
  const s4* frag = sops + lane;
  const s4* fragL = frag + 3 * RB * RB * 64;
  const int e = tile * kTile + es;
  const unsigned nbytes = (unsigned)L.ntile * TS;
  const Rsrc Rq = rsrc(qo, nbytes), Rn = rsrc(qn, nbytes), Rr = rsrc(res, nbytes);
  const unsigned tb = (unsigned)tile * TS + (unsigned)es * 4;   // this lane's element
  const double* gt = L.geo + (size_t)tile * 12 * kTile + es;
  const float rx = (float)gt[0 * kTile], ry = (float)gt[1 * kTile], rz = (float)gt[2 * kTile];
  const float sx = (float)gt[3 * kTile], sy = (float)gt[4 * kTile], sz = (float)gt[5 * kTile];
  const float tx = (float)gt[6 * kTile], ty = (float)gt[7 * kTile], tz = (float)gt[8 * kTile];
  const float irho = (float)gt[9 * kTile], Kb = (float)gt[10 * kTile], Z = (float)gt[11 * kTile];
  const int* nbrt = L.nbr + tile * 4 * kTile + es;
  const double* znt = L.zn + tile * 4 * kTile + es;
  int fcode[4];
  float fz[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    fcode[f] = nbrt[f * kTile];
    fz[f] = (float)znt[f * kTile];
  }

  // ---- volume: Dr p, Ds p, Dt p and div u = Dr fr + Ds fs + Dt ft, one
  // k-step of 16 nodes at a time (this lane: nodes 16 j + 4 g + i)
  f4 dpr[RB], dps[RB], dpt[RB], dv[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) dpr[b] = dps[b] = dpt[b] = dv[b] = f4{0, 0, 0, 0};
#pragma unroll 1
  for (int j = 0; j < RB; ++j) {
    float p[4], fr[4], fs[4], ft[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const unsigned o = tb + (unsigned)min(16 * j + 4 * g + i, Np - 1) * (kTile * 4);
      const float u = fld(Rq, o, FS), v = fld(Rq, o, 2 * FS), w = fld(Rq, o, 3 * FS);
      p[i] = fld(Rq, o, 0);
      fr[i] = rx * u + ry * v + rz * w;
      fs[i] = sx * u + sy * v + sz * w;
      ft[i] = tx * u + ty * v + tz * w;
    }
    const s4 bp = pack4(p), br = pack4(fr), bs = pack4(fs), bt = pack4(ft);
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const s4 ar = frag[((0 * RB + b) * RB + j) * 64];
      const s4 as = frag[((1 * RB + b) * RB + j) * 64];
      const s4 at = frag[((2 * RB + b) * RB + j) * 64];
      dpr[b] = mfma_bf16(ar, bp, dpr[b]);
      dps[b] = mfma_bf16(as, bp, dps[b]);
      dpt[b] = mfma_bf16(at, bp, dpt[b]);
      dv[b] = mfma_bf16(ar, br, dv[b]);
      dv[b] = mfma_bf16(as, bs, dv[b]);
      dv[b] = mfma_bf16(at, bt, dv[b]);
    }
  }
#pragma unroll
  for (int b = 0; b < RB; ++b) dv[b] *= -Kb;
  f4* rp = dv;

  // ---- surface: one upwind flux against the exterior state per face node
  // (FP32), the pressure jump lifted into the reference gradient; a lane
  // computes the fluxes of face nodes 16 jj + 4 g + i
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    __builtin_amdgcn_sched_barrier(0);
    const float cr = f == 2 ? 1.f : (f == 3 ? -1.f : 0.f);
    const float cs = f == 2 ? 1.f : (f == 1 ? -1.f : 0.f);
    const float ct = f == 2 ? 1.f : (f == 0 ? -1.f : 0.f);
    float nx = cr * rx + cs * sx + ct * tx;
    float ny = cr * ry + cs * sy + ct * ty;
    float nz = cr * rz + cs * sz + ct * tz;
    const float fsc = sqrtf(nx * nx + ny * ny + nz * nz);
    const float inv = 1.f / fsc;
    nx *= inv;
    ny *= inv;
    nz *= inv;
    const int code = fcode[f];
    const float ZP = fz[f];
    const bool inner = code >= 0;
    const int cb = -1 - code;
    const bool hb = !inner && (cb & 3) == 0;
    const bool dir = !inner && (cb & 3) == 2;
    const int e2 = inner ? (code >> 5) : e;
    const unsigned nb = (unsigned)(e2 >> 4) * TS + (unsigned)(e2 & 15) * 4;
    const int mapbase = inner ? ((f * 4 + ((code >> 3) & 3)) * 6 + (code & 7)) * Nfp
                              : ((f * 4) * 6 + ((cb >> 2) & 7)) * Nfp;
    const double* qbt = qb3 + (size_t)(hb ? (cb >> 5) : 0) * Nfp;
    const float iZ = 1.f / (Z + ZP);
    const float aM = ZP * iZ, aP = Z * iZ, bZ = Z * aM;
    const float cP = fsc * Kb;
#pragma unroll
    for (int jj = 0; jj < FK; ++jj) {
      float fp[4], fu[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int kc = min(16 * jj + 4 * g + i, Nfp - 1);
        const int n = smask[f * Nfp + kc];
        const int n2 = smap[mapbase + kc];
        const unsigned oM = tb + (unsigned)n * (kTile * 4);
        const unsigned oP = nb + (unsigned)n2 * (kTile * 4);
        const float pM = fld(Rq, oM, 0), uM = fld(Rq, oM, FS), vM = fld(Rq, oM, 2 * FS),
                    wM = fld(Rq, oM, 3 * FS);
        const float pP = fld(Rq, oP, 0), uP = fld(Rq, oP, FS), vP = fld(Rq, oP, 2 * FS),
                    wP = fld(Rq, oP, 3 * FS);
        const float rb = (float)qbt[min(n2, Nfp - 1)];
        const float unM = nx * uM + ny * vM + nz * wM;
        const float unP = nx * uP + ny * vP + nz * wP;
        const float pG = inner ? pP : (dir ? -pM : (hb ? 2.f * rb : 0.f));
        const float uG = inner ? unP : (dir ? unM : 0.f);
        const float pF = aM * pM + aP * pG + bZ * (unM - uG);
        const float unF = iZ * (pM - pG) + aP * unM + aM * uG;
        fp[i] = cP * (unM - unF);
        fu[i] = pM - pF;
      }
      const s4 bfp = pack4(fp), bfu = pack4(fu);
      const s4* fl = fragL + (f * FK + jj) * 64;
      if (f == 2) {
        float nfu[4] = {-fu[0], -fu[1], -fu[2], -fu[3]};
        const s4 bnu = pack4(nfu);
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          const s4 a = fl[b * 4 * FK * 64];
          rp[b] = mfma_bf16(a, bfp, rp[b]);
          dpr[b] = mfma_bf16(a, bnu, dpr[b]);
          dps[b] = mfma_bf16(a, bnu, dps[b]);
          dpt[b] = mfma_bf16(a, bnu, dpt[b]);
        }
      } else {
        f4* G = f == 0 ? dpt : (f == 1 ? dps : dpr);
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          const s4 a = fl[b * 4 * FK * 64];
          rp[b] = mfma_bf16(a, bfp, rp[b]);
          G[b] = mfma_bf16(a, bfu, G[b]);
        }
      }
    }
  }

  // ---- LSRK update of the four rows per row block this lane holds (FP32)
  const bool live = irho != 0.f;
  const double* sp = sh.srcp + 4 * shot;
  const bool src = (double)e == sp[0];
  const double trr = stage_time(sh) - sp[2], arr = M_PI * sp[1] * trr;
  const float src_s = (float)(sp[3] * trr * exp(-arr * arr));
  const double* src_w = sh.srcw + (size_t)shot * Np;
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    __builtin_amdgcn_sched_barrier(0);
    float ro[4][4], qv[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const unsigned o = tb + (unsigned)min(16 * b + 4 * g + r, Np - 1) * (kTile * 4);
#pragma unroll
      for (int fl = 0; fl < 4; ++fl) {
        ro[r][fl] = fldn(Rr, o, fl * FS);
        qv[r][fl] = fld(Rq, o, fl * FS);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = 16 * b + 4 * g + r;
      const int nc = min(n, Np - 1);
      const unsigned o = tb + (unsigned)nc * (kTile * 4);
      const float sw = (float)src_w[nc];
      const float a = dpr[b][r], bq = dps[b][r], c = dpt[b][r];
      const float rhs[4] = {rp[b][r] + (src ? sw * src_s : 0.f),
                            -irho * (rx * a + sx * bq + tx * c),
                            -irho * (ry * a + sy * bq + ty * c),
                            -irho * (rz * a + sz * bq + tz * c)};
      if (live && n < Np) {
#pragma unroll
        for (int fl = 0; fl < 4; ++fl) {
          const float rr = A * ro[r][fl] + dt * rhs[fl];
          fst(Rr, o, fl * FS, rr);
          fst(Rn, o, fl * FS, qv[r][fl] + B * rr);
        }
      }
    }
  }
}

template <int N, int W>
__global__ void __launch_bounds__(W * 64, W == 8 ? 1 : Dims3b<N>::kOcc) k_level3_bf16(
    Lvl3 L, const float* __restrict__ qo, float* __restrict__ qn, float* __restrict__ res,
    const double* __restrict__ qb3, float A, float B, float dt, Shots sh) {
  using D = Dims3b<N>;
  constexpr int Nfp = D::Nfp;
  extern __shared__ float sfl[];
  int* smask = reinterpret_cast<int*>(sfl);
  int* smap = smask + 4 * Nfp;
  // fragments after the maps, at an 8-byte boundary
  s4* sops = reinterpret_cast<s4*>(sfl + ((4 * Nfp + 96 * Nfp + 1) & ~1));
  fill_lds<W * 64, 4 * Nfp>(smask, L.fmask, threadIdx.x);
  fill_lds<W * 64, 96 * Nfp>(smap, L.fmap, threadIdx.x);
  fill_lds<W * 64, D::NFR * 64>(reinterpret_cast<unsigned long long*>(sops),
                                       reinterpret_cast<const unsigned long long*>(L.opsb),
                                       threadIdx.x);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int ngrp = (L.ntile + W - 1) / W;
  const XcdRange rg_(ngrp * (long long)sh.n, L.order);
  for (long long item = rg_.lo; item < rg_.hi; item += rg_.step)
    tile_bf16<N, W>(L, qo, qn, res, qb3, A, B, dt, sh, item, ngrp, smap, smask, sops, lane);
}

// ------------------------------------------ BF16 contractions, tile on chip ---
// N <= 5: the BF16 contractions over the tile-on-chip scheme of the FP32
// kernel (one workgroup of four waves per CU, each wave's next FP32 tile
// arriving in its LDS buffer by direct loads while it finishes the current
// one).  With K = 16 a lane's B operand of k-step j is the nodes
// 16 j + 4 (l/16) + i of its element, read from the LDS copy and rounded to
// BF16; the exterior traces of faces 0-2 are in flight during the volume
// term, face 3's during face 0.
template <int N>
struct FaceInB {
  static constexpr int FK = Dims3b<N>::FK;
  float p[FK][4], u[FK][4], v[FK][4], w[FK][4], rb[FK][4];
};

template <int N>
__device__ __forceinline__ void face_fetch_b(FaceInB<N>& x, int f, int code, int e, Rsrc Rq,
                                             const double* __restrict__ qb3, const int* smap,
                                             int g) {
  using D = Dims3b<N>;
  constexpr int Np = D::Np, Nfp = D::Nfp, FK = D::FK;
  constexpr unsigned FS = Np * kTile * 4, TS = 4 * FS;
  const bool inner = code >= 0;
  const int cb = -1 - code;
  const bool hb = !inner && (cb & 3) == 0;
  const int e2 = inner ? (code >> 5) : e;
  const unsigned nb = (unsigned)(e2 >> 4) * TS + (unsigned)(e2 & 15) * 4;
  const int mapbase = inner ? ((f * 4 + ((code >> 3) & 3)) * 6 + (code & 7)) * Nfp
                            : ((f * 4) * 6 + ((cb >> 2) & 7)) * Nfp;
  const double* qbt = qb3 + (size_t)(hb ? (cb >> 5) : 0) * Nfp;
#pragma unroll
  for (int jj = 0; jj < FK; ++jj)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int kc = min(16 * jj + 4 * g + i, Nfp - 1);
      const int n2 = smap[mapbase + kc];
      const unsigned oP = nb + (unsigned)n2 * (kTile * 4);
      x.p[jj][i] = fld(Rq, oP, 0);
      x.u[jj][i] = fld(Rq, oP, FS);
      x.v[jj][i] = fld(Rq, oP, 2 * FS);
      x.w[jj][i] = fld(Rq, oP, 3 * FS);
      x.rb[jj][i] = (float)qbt[min(n2, Nfp - 1)];
    }
}

// One work item whose tile is in buf; fetch_next() issues the direct loads
// of the next item (if any) once the tile's copy has been read.
template <int N, class Fetch>
__device__ __forceinline__ void tile_bf16_dma(const Lvl3& L, const float* __restrict__ qo,
                                              float* __restrict__ qn, float* __restrict__ res,
                                              const double* __restrict__ qb3, float A, float B,
                                              float dt, const Shots& sh, long long item,
                                              Fetch fetch_next, int ngrp, const int* smap,
                                              const int* smask, const s4* sops, char* buf,
                                              int lane) {
  using D = Dims3b<N>;
  using BR = BufF<N>;
  constexpr int Np = D::Np, Nfp = D::Nfp, RB = D::RB, FK = D::FK;
  constexpr unsigned FS = Np * kTile * 4;   // bytes between two fields of a tile
  constexpr unsigned TS = 4 * FS;           // bytes per tile
  const int shot = (int)(item / ngrp);
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int tile = (int)(item - (long long)shot * ngrp) * kWavesF + wv;
  // the tile's direct loads have landed: vector memory operations complete in
  // order and the previous tile issued 32 RB stores after them
  constexpr int kVm = 32 * RB < 63 ? 32 * RB : 63;
  __builtin_amdgcn_s_waitcnt((kVm & 15) | ((kVm >> 4) << 14) | (7 << 4) | (15 << 8));
  if (tile >= L.ntile) {
    __builtin_amdgcn_s_waitcnt(0);
    fetch_next();
    __builtin_amdgcn_s_waitcnt(0);
    return;
  }
  const float* qos = qo + shot * sh.st3;
  float* qns = qn + shot * sh.st3;
  float* ress = res + shot * sh.st3;
  const double* qbs = qb3 + shot * sh.stb3;
  const int es = lane & 15, g = lane >> 4;
  const s4* frag = sops + lane;
  const s4* fragL = frag + 3 * RB * RB * 64;
  const int e = tile * kTile + es;
  const unsigned nbytes = (unsigned)L.ntile * TS;
  const Rsrc Rq = rsrc(qos, nbytes), Rn = rsrc(qns, nbytes), Rr = rsrc(ress, nbytes);
  const unsigned tb = (unsigned)tile * TS + (unsigned)es * 4;   // this lane's element
  const float* bq = reinterpret_cast<const float*>(buf) + es;    // [field][node][16]
  const double* bg = reinterpret_cast<const double*>(buf + BR::GEO) + es;
  const double* bz = reinterpret_cast<const double*>(buf + BR::ZN) + es;
  const int* bc = reinterpret_cast<const int*>(buf + BR::NBR) + es;
  int fcode[4];
  float fz[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    fcode[f] = bc[f * kTile];
    fz[f] = (float)bz[f * kTile];
  }
  FaceInB<N> fb[4];
#pragma unroll
  for (int f = 0; f < 3; ++f) face_fetch_b<N>(fb[f], f, fcode[f], e, Rq, qbs, smap, g);
  const float rx = (float)bg[0 * kTile], ry = (float)bg[1 * kTile], rz = (float)bg[2 * kTile];
  const float sx = (float)bg[3 * kTile], sy = (float)bg[4 * kTile], sz = (float)bg[5 * kTile];
  const float tx = (float)bg[6 * kTile], ty = (float)bg[7 * kTile], tz = (float)bg[8 * kTile];
  const float irho = (float)bg[9 * kTile], Kb = (float)bg[10 * kTile], Z = (float)bg[11 * kTile];

  // ---- volume: one k-step of 16 nodes at a time, B operands from the copy
  f4 dpr[RB], dps[RB], dpt[RB], dv[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) dpr[b] = dps[b] = dpt[b] = dv[b] = f4{0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    float p[4], fr[4], fs[4], ft[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int n = min(16 * j + 4 * g + i, Np - 1);
      const float u = bq[(Np + n) * kTile], v = bq[(2 * Np + n) * kTile],
                  w = bq[(3 * Np + n) * kTile];
      p[i] = bq[n * kTile];
      fr[i] = rx * u + ry * v + rz * w;
      fs[i] = sx * u + sy * v + sz * w;
      ft[i] = tx * u + ty * v + tz * w;
    }
    const s4 bp = pack4(p), br = pack4(fr), bs = pack4(fs), bt = pack4(ft);
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const s4 ar = frag[((0 * RB + b) * RB + j) * 64];
      const s4 as = frag[((1 * RB + b) * RB + j) * 64];
      const s4 at = frag[((2 * RB + b) * RB + j) * 64];
      dpr[b] = mfma_bf16(ar, bp, dpr[b]);
      dps[b] = mfma_bf16(as, bp, dps[b]);
      dpt[b] = mfma_bf16(at, bp, dpt[b]);
      dv[b] = mfma_bf16(ar, br, dv[b]);
      dv[b] = mfma_bf16(as, bs, dv[b]);
      dv[b] = mfma_bf16(at, bt, dv[b]);
    }
  }
#pragma unroll
  for (int b = 0; b < RB; ++b) dv[b] *= -Kb;
  f4* rp = dv;

  // ---- surface (as in tile_bf16); own traces from the LDS copy
  float rv[RB][4][4], qd[RB][4][4], own3[FK][4][4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    __builtin_amdgcn_sched_barrier(0);
    if (f == 0) {
      face_fetch_b<N>(fb[3], 3, fcode[3], e, Rq, qbs, smap, g);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (f == 1) {
      // the residual of this tile at the update's rows
#pragma unroll
      for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const unsigned o = tb + (unsigned)min(16 * b + 4 * g + r, Np - 1) * (kTile * 4);
#pragma unroll
          for (int fl = 0; fl < 4; ++fl) rv[b][r][fl] = fldn(Rr, o, fl * FS);
        }
      __builtin_amdgcn_sched_barrier(0);
    }
    if (f == 3) {
      // the last reads of the copy (face 3's own traces, the update's q),
      // then the next tile's direct loads
#pragma unroll
      for (int jj = 0; jj < FK; ++jj)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int n = smask[3 * Nfp + min(16 * jj + 4 * g + i, Nfp - 1)];
#pragma unroll
          for (int fl = 0; fl < 4; ++fl) own3[jj][i][fl] = bq[(fl * Np + n) * kTile];
        }
#pragma unroll
      for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int n = min(16 * b + 4 * g + r, Np - 1);
#pragma unroll
          for (int fl = 0; fl < 4; ++fl) qd[b][r][fl] = bq[(fl * Np + n) * kTile];
        }
      __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): every LDS read returned
      __builtin_amdgcn_sched_barrier(0);
      fetch_next();
      __builtin_amdgcn_sched_barrier(0);
    }
    const FaceInB<N>& x = fb[f];
    const float cr = f == 2 ? 1.f : (f == 3 ? -1.f : 0.f);
    const float cs = f == 2 ? 1.f : (f == 1 ? -1.f : 0.f);
    const float ct = f == 2 ? 1.f : (f == 0 ? -1.f : 0.f);
    float nx = cr * rx + cs * sx + ct * tx;
    float ny = cr * ry + cs * sy + ct * ty;
    float nz = cr * rz + cs * sz + ct * tz;
    const float fsc = sqrtf(nx * nx + ny * ny + nz * nz);
    const float inv = 1.f / fsc;
    nx *= inv;
    ny *= inv;
    nz *= inv;
    const int code = fcode[f];
    const float ZP = fz[f];
    const bool inner = code >= 0;
    const int cb = -1 - code;
    const bool hb = !inner && (cb & 3) == 0;
    const bool dir = !inner && (cb & 3) == 2;
    const float iZ = 1.f / (Z + ZP);
    const float aM = ZP * iZ, aP = Z * iZ, bZ = Z * aM;
    const float cP = fsc * Kb;
#pragma unroll
    for (int jj = 0; jj < FK; ++jj) {
      float fp[4], fu[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float pM, uM, vM, wM;
        if (f == 3) {
          pM = own3[jj][i][0];
          uM = own3[jj][i][1];
          vM = own3[jj][i][2];
          wM = own3[jj][i][3];
        } else {
          const int n = smask[f * Nfp + min(16 * jj + 4 * g + i, Nfp - 1)];
          pM = bq[n * kTile];
          uM = bq[(Np + n) * kTile];
          vM = bq[(2 * Np + n) * kTile];
          wM = bq[(3 * Np + n) * kTile];
        }
        const float pP = x.p[jj][i], uP = x.u[jj][i], vP = x.v[jj][i], wP = x.w[jj][i];
        const float unM = nx * uM + ny * vM + nz * wM;
        const float unP = nx * uP + ny * vP + nz * wP;
        const float pG = inner ? pP : (dir ? -pM : (hb ? 2.f * x.rb[jj][i] : 0.f));
        const float uG = inner ? unP : (dir ? unM : 0.f);
        const float pF = aM * pM + aP * pG + bZ * (unM - uG);
        const float unF = iZ * (pM - pG) + aP * unM + aM * uG;
        fp[i] = cP * (unM - unF);
        fu[i] = pM - pF;
      }
      const s4 bfp = pack4(fp), bfu = pack4(fu);
      const s4* fl = fragL + (f * FK + jj) * 64;
      if (f == 2) {
        float nfu[4] = {-fu[0], -fu[1], -fu[2], -fu[3]};
        const s4 bnu = pack4(nfu);
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          const s4 a = fl[b * 4 * FK * 64];
          rp[b] = mfma_bf16(a, bfp, rp[b]);
          dpr[b] = mfma_bf16(a, bnu, dpr[b]);
          dps[b] = mfma_bf16(a, bnu, dps[b]);
          dpt[b] = mfma_bf16(a, bnu, dpt[b]);
        }
      } else {
        f4* G = f == 0 ? dpt : (f == 1 ? dps : dpr);
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          const s4 a = fl[b * 4 * FK * 64];
          rp[b] = mfma_bf16(a, bfp, rp[b]);
          G[b] = mfma_bf16(a, bfu, G[b]);
        }
      }
    }
  }

  // point source on its element (a uniform branch only that wave takes)
  {
    const double* sp = sh.srcp + 4 * shot;
    const bool src = (double)e == sp[0];
    if (__builtin_amdgcn_read_exec() & __ballot(src)) {
      const double trr = stage_time(sh) - sp[2], arr = M_PI * sp[1] * trr;
      const float src_s = (float)(sp[3] * trr * exp(-arr * arr));
      const double* src_w = sh.srcw + (size_t)shot * Np;
#pragma unroll
      for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (src) rp[b][r] += (float)src_w[min(16 * b + 4 * g + r, Np - 1)] * src_s;
    }
  }

  // ---- LSRK update: 32 RB stores, every lane issuing them (a lane without
  // a row stores past the end of the resource, which the hardware drops)
  __builtin_amdgcn_sched_barrier(0);
  const bool live = irho != 0.f;
#pragma unroll
  for (int b = 0; b < RB; ++b) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = 16 * b + 4 * g + r;
      const unsigned o = (live && n < Np) ? tb + (unsigned)n * (kTile * 4) : 0xFFFFFFF8u;
      const float a = dpr[b][r], bq_ = dps[b][r], c = dpt[b][r];
      const float rhs[4] = {rp[b][r],
                            -irho * (rx * a + sx * bq_ + tx * c),
                            -irho * (ry * a + sy * bq_ + ty * c),
                            -irho * (rz * a + sz * bq_ + tz * c)};
#pragma unroll
      for (int fl = 0; fl < 4; ++fl) {
        const float rr = A * rv[b][r][fl] + dt * rhs[fl];
        fst(Rr, o, fl * FS, rr);
        fst(Rn, o, fl * FS, qd[b][r][fl] + B * rr);
      }
    }
  }
}

// LDS of the tile-on-chip BF16 kernel: face-node tables, the BF16 operator
// fragments (8-byte aligned), then the four tile buffers (16-byte aligned)
template <int N>
struct LdsB {
  static constexpr size_t TAB = sizeof(float) * ((4 * Dims3b<N>::Nfp + 96 * Dims3b<N>::Nfp + 1) & ~1);
  static constexpr size_t BUF = (TAB + (size_t)Dims3b<N>::NFR * 512 + 15) / 16 * 16;
  static constexpr size_t BYTES = BUF + (size_t)kWavesF * BufF<N>::BYTES;
};

template <int N>
__global__ void __launch_bounds__(kWavesF * 64, 1) k_level3_bf16_dma(
    Lvl3 L, const float* __restrict__ qo, float* __restrict__ qn, float* __restrict__ res,
    const double* __restrict__ qb3, float A, float B, float dt, Shots sh) {
  using D = Dims3b<N>;
  using LB = LdsB<N>;
  constexpr int Nfp = D::Nfp;
  extern __shared__ float sfl[];
  int* smask = reinterpret_cast<int*>(sfl);
  int* smap = smask + 4 * Nfp;
  s4* sops = reinterpret_cast<s4*>(reinterpret_cast<char*>(sfl) + LB::TAB);
  const int lane = threadIdx.x & 63;
  const int ngrp = (L.ntile + kWavesF - 1) / kWavesF;
  const XcdRange rg_(ngrp * (long long)sh.n, L.order);
  char* buf = reinterpret_cast<char*>(sfl) + LB::BUF +
              __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * BufF<N>::BYTES;
  if (rg_.lo < rg_.hi) tile_dma_f<N>(L, qo, sh, rg_.lo, ngrp, buf, lane);
  fill_lds<kWavesF * 64, 4 * Nfp>(smask, L.fmask, threadIdx.x);
  fill_lds<kWavesF * 64, 96 * Nfp>(smap, L.fmap, threadIdx.x);
  fill_lds<kWavesF * 64, D::NFR * 64>(reinterpret_cast<unsigned long long*>(sops),
                                      reinterpret_cast<const unsigned long long*>(L.opsb),
                                      threadIdx.x);
  __syncthreads();
  for (long long it = rg_.lo; it < rg_.hi; it += rg_.step) {
    const long long nx = it + rg_.step;
    auto fetch = [&]() {
      if (nx < rg_.hi) tile_dma_f<N>(L, qo, sh, nx, ngrp, buf, lane);
    };
    tile_bf16_dma<N>(L, qo, qn, res, qb3, A, B, dt, sh, it, fetch, ngrp, smap, smask, sops, buf,
                     lane);
  }
}

// The same kernel over a group of contexts (any mesh sizes, same N), as
// the FP32 group kernel: one work list, member c owning
// [first_c, first_c + items_c).
template <int N>
__global__ void __launch_bounds__(kWavesF * 64, 1) k_level3_bf16_dma_group(
    const Member3* __restrict__ G, int nm, long long total, float A, float B, float dt,
    double tau, double cs) {
  using D = Dims3b<N>;
  using LB = LdsB<N>;
  constexpr int Nfp = D::Nfp;
  extern __shared__ float sfl[];
  int* smask = reinterpret_cast<int*>(sfl);
  int* smap = smask + 4 * Nfp;
  s4* sops = reinterpret_cast<s4*>(reinterpret_cast<char*>(sfl) + LB::TAB);
  const int lane = threadIdx.x & 63;
  const XcdRange rg_(total, G[0].L.order);
  char* buf = reinterpret_cast<char*>(sfl) + LB::BUF +
              __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * BufF<N>::BYTES;
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
    tile_dma_f<N>(G[c].L, static_cast<const float*>(G[c].qo), shots(c), rg_.lo - G[c].first,
                  G[c].ngrp, buf, lane);
  }
  fill_lds<kWavesF * 64, 4 * Nfp>(smask, G[0].L.fmask, threadIdx.x);
  fill_lds<kWavesF * 64, 96 * Nfp>(smap, G[0].L.fmap, threadIdx.x);
  fill_lds<kWavesF * 64, D::NFR * 64>(reinterpret_cast<unsigned long long*>(sops),
                                      reinterpret_cast<const unsigned long long*>(G[0].L.opsb),
                                      threadIdx.x);
  __syncthreads();
  for (long long it = rg_.lo; it < rg_.hi; it += rg_.step) {
    const long long nx = it + rg_.step;
    const int c = member(it);
    const Shots sh = shots(c);
    auto fetch = [&]() {
      if (nx < rg_.hi) {
        const int cn = member(nx);
        tile_dma_f<N>(G[cn].L, static_cast<const float*>(G[cn].qo), shots(cn),
                      nx - G[cn].first, G[cn].ngrp, buf, lane);
      }
    };
    tile_bf16_dma<N>(G[c].L, static_cast<const float*>(G[c].qo), static_cast<float*>(G[c].qn),
                     static_cast<float*>(G[c].res), G[c].qb3, A, B, dt, sh, it - G[c].first,
                     fetch, G[c].ngrp, smap, smask, sops, buf, lane);
  }
}

template <int N>
hipError_t launch3b_group(const Member3* G, int nm, long long total, double A, double B,
                          double dt, double tau, double cs, hipStream_t st) {
  const size_t lds = LdsB<N>::BYTES;
  int resident = 0;
  {
    const hipError_t e =
        kernel_setup((const void*)(k_level3_bf16_dma_group<N>), kWavesF * 64, lds, &resident);
    if (e != hipSuccess) return e;
  }
  const int blocks = (int)std::max<long long>(8, std::min<long long>(resident, total) / 8 * 8);
  hipLaunchKernelGGL(k_level3_bf16_dma_group<N>, dim3(blocks), dim3(kWavesF * 64), lds, st, G,
                     nm, total, (float)A, (float)B, (float)dt, tau, cs);
  return hipGetLastError();
}

template <int N>
hipError_t launch3b_dma(const Lvl3& L, const float* qo, float* qn, float* res, const double* qb3,
                        double A, double B, double dt, const Shots& sh, hipStream_t st) {
  const size_t lds = LdsB<N>::BYTES;
  if (sh.n < 1) return hipErrorInvalidValue;
  const int ngrp = (L.ntile + kWavesF - 1) / kWavesF;
  int resident = 0;
  {
    const hipError_t e =
        kernel_setup((const void*)(k_level3_bf16_dma<N>), kWavesF * 64, lds, &resident);
    if (e != hipSuccess) return e;
  }
  const long long items = (long long)ngrp * sh.n;
  const int blocks = grid3(resident, items, L.eighths);
  hipLaunchKernelGGL(k_level3_bf16_dma<N>, dim3(blocks), dim3(kWavesF * 64), lds, st, L, qo, qn,
                     res, qb3, (float)A, (float)B, (float)dt, sh);
  return hipGetLastError();
}

template <int N, int W>
hipError_t launch3b_reg(const Lvl3& L, const float* qo, float* qn, float* res, const double* qb3,
                        double A, double B, double dt, const Shots& sh, hipStream_t st) {
  using D = Dims3b<N>;
  constexpr int Nfp = D::Nfp;
  const size_t lds = sizeof(float) * ((4 * Nfp + 96 * Nfp + 1) & ~1) + (size_t)D::NFR * 512;
  const int ngrp = (L.ntile + W - 1) / W;
  if (sh.n < 1) return hipErrorInvalidValue;
  int resident = 0;
  {
    const hipError_t e = kernel_setup((const void*)(k_level3_bf16<N, W>), W * 64, lds, &resident);
    if (e != hipSuccess) return e;
  }
  const long long items = (long long)ngrp * sh.n;
  const int blocks = grid3(resident, items, L.eighths);
  hipLaunchKernelGGL((k_level3_bf16<N, W>), dim3(blocks), dim3(W * 64), lds, st, L, qo, qn, res,
                     qb3, (float)A, (float)B, (float)dt, sh);
  return hipGetLastError();
}

template <int N>
hipError_t launch3b(const Lvl3& L, const float* qo, float* qn, float* res, const double* qb3,
                    double A, double B, double dt, const Shots& sh, hipStream_t st) {
  if constexpr (N <= 5) {   // the tile buffers and fragments fit the LDS up to N = 5
    if (L.kvar == 0) return launch3b_dma<N>(L, qo, qn, res, qb3, A, B, dt, sh, st);
  }
  if (L.waves == 8) return launch3b_reg<N, 8>(L, qo, qn, res, qb3, A, B, dt, sh, st);
  return launch3b_reg<N, 4>(L, qo, qn, res, qb3, A, B, dt, sh, st);
}

}  // namespace

hipError_t launch_level3_f32_group(const Member3* G, int nm, long long total, int N, double A,
                                   double B, double dt, double tau, double cs, hipStream_t st) {
  switch (N) {
    case 1: return launch3f_group<1>(G, nm, total, A, B, dt, tau, cs, st);
    case 2: return launch3f_group<2>(G, nm, total, A, B, dt, tau, cs, st);
    case 3: return launch3f_group<3>(G, nm, total, A, B, dt, tau, cs, st);
    case 4: return launch3f_group<4>(G, nm, total, A, B, dt, tau, cs, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_level3_f32(const Lvl3& L, const float* qo, float* qn, float* res,
                             const double* qb3, double A, double B, double dt, const Shots& sh,
                             hipStream_t st) {
  switch (L.N) {
    case 1: return launch3f<1>(L, qo, qn, res, qb3, A, B, dt, sh, st);
    case 2: return launch3f<2>(L, qo, qn, res, qb3, A, B, dt, sh, st);
    case 3: return launch3f<3>(L, qo, qn, res, qb3, A, B, dt, sh, st);
    case 4: return launch3f<4>(L, qo, qn, res, qb3, A, B, dt, sh, st);
    case 5: return launch3f<5>(L, qo, qn, res, qb3, A, B, dt, sh, st);
    case 6: return launch3f<6>(L, qo, qn, res, qb3, A, B, dt, sh, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_level3_bf16_group(const Member3* G, int nm, long long total, int N, double A,
                                    double B, double dt, double tau, double cs, hipStream_t st) {
  switch (N) {
    case 1: return launch3b_group<1>(G, nm, total, A, B, dt, tau, cs, st);
    case 2: return launch3b_group<2>(G, nm, total, A, B, dt, tau, cs, st);
    case 3: return launch3b_group<3>(G, nm, total, A, B, dt, tau, cs, st);
    case 4: return launch3b_group<4>(G, nm, total, A, B, dt, tau, cs, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_level3_bf16(const Lvl3& L, const float* qo, float* qn, float* res,
                              const double* qb3, double A, double B, double dt, const Shots& sh,
                              hipStream_t st) {
  switch (L.N) {
    case 1: return launch3b<1>(L, qo, qn, res, qb3, A, B, dt, sh, st);
    case 2: return launch3b<2>(L, qo, qn, res, qb3, A, B, dt, sh, st);
    case 3: return launch3b<3>(L, qo, qn, res, qb3, A, B, dt, sh, st);
    case 4: return launch3b<4>(L, qo, qn, res, qb3, A, B, dt, sh, st);
    case 5: return launch3b<5>(L, qo, qn, res, qb3, A, B, dt, sh, st);
    case 6: return launch3b<6>(L, qo, qn, res, qb3, A, B, dt, sh, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dgh
