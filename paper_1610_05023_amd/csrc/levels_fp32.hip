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
#include "levels.hpp"

namespace dgh {

namespace {

constexpr int kWaves3f = 4;   // waves (tiles) per workgroup

typedef float f4 __attribute__((ext_vector_type(4)));

template <int N>
struct Dims3f {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int RG = (Np + 3) / 4;     // volume k-steps of 4 nodes
  static constexpr int RB = (Np + 15) / 16;   // row blocks of 16 nodes
  static constexpr int FK = (Nfp + 3) / 4;    // lifting k-steps per face
  static constexpr int NOPS = (3 * RB * RG + RB * 4 * FK) * 64;   // floats
  static constexpr bool kLds = NOPS * 4 <= 64 * 1024;
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
// streaming (non-temporal) load and store: read or written once per stage
__device__ __forceinline__ float fldn(Rsrc r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 2));
}
__device__ __forceinline__ void fstn(Rsrc r, unsigned voff, unsigned soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 2);
}

template <int N>
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
  const int tile = (int)(item - (long long)shot * ngrp) * kWaves3f + (threadIdx.x >> 6);
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
  constexpr int PF = N <= 4 ? 3 : 1;   // fewer registers left at N > 4
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
          fstn(Rr, o, fl * FS, rr);
          fstn(Rn, o, fl * FS, qv[r][fl] + B * rr);
        }
      }
    }
  }
}

template <int N>
__global__ void __launch_bounds__(kWaves3f * 64, 2) k_level3_f32(Lvl3 L, const float* __restrict__ qo,
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
  fill_lds<kWaves3f * 64, 4 * Nfp>(smask, L.fmask, threadIdx.x);
  fill_lds<kWaves3f * 64, 96 * Nfp>(smap, L.fmap, threadIdx.x);
  if (D::kLds) fill_lds<kWaves3f * 64, D::NOPS>(sops, L.ops32, threadIdx.x);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int ngrp = (L.ntile + kWaves3f - 1) / kWaves3f;
  const XcdRange rg_(ngrp * (long long)sh.n, L.order);
  for (long long item = rg_.lo; item < rg_.hi; item += rg_.step)
    tile_f32<N>(L, qo, qn, res, qb3, A, B, dt, sh, item, ngrp, smap, smask, sops, lane);
}

template <int N>
hipError_t launch3f(const Lvl3& L, const float* qo, float* qn, float* res, const double* qb3,
                    double A, double B, double dt, const Shots& sh, hipStream_t st) {
  using D = Dims3f<N>;
  constexpr int Nfp = D::Nfp;
  const size_t lds = sizeof(float) * (4 * Nfp + 96 * Nfp + (D::kLds ? D::NOPS : 0));
  static bool attr = false;
  if (!attr) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_level3_f32<N>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int ngrp = (L.ntile + kWaves3f - 1) / kWaves3f;
  if (sh.n < 1) return hipErrorInvalidValue;
  static int resident = 0;
  if (!resident) {
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_level3_f32<N>, kWaves3f * 64,
                                                       lds);
    if (e != hipSuccess) return e;
    resident = std::max(1, per_cu) * prop.multiProcessorCount;
  }
  const long long items = (long long)ngrp * sh.n;
  const int blocks = (int)std::max<long long>(8, std::min<long long>(resident, items) / 8 * 8);
  hipLaunchKernelGGL(k_level3_f32<N>, dim3(blocks), dim3(kWaves3f * 64), lds, st, L, qo, qn, res,
                     qb3, (float)A, (float)B, (float)dt, sh);
  return hipGetLastError();
}

}  // namespace

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

}  // namespace dgh
