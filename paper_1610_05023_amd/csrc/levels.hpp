// Device-side descriptions of the four levels of the multidimensional step
// (volume, faces, edges, corners; Algorithm 1) and the launchers of their
// kernels.  All pointers point into the caller-owned workspace.
#pragma once
#include <hip/hip_runtime.h>

namespace dgh {

constexpr int kTile = 16;  // elements per tile of the 3D node-major layout

// Number of floats of the FP32 3D operator fragments for degree N.
inline int frag3f_size(int N) {
  const int Np = (N + 1) * (N + 2) * (N + 3) / 6, Nfp = (N + 1) * (N + 2) / 2;
  const int RG = (Np + 3) / 4, RB = (Np + 15) / 16, FK = (Nfp + 3) / 4;
  return (3 * RB * RG + RB * 4 * FK) * 64;
}

// Number of BF16 values of the BF16 variant's fragments for degree N.
inline int frag3b_size(int N) {
  const int Np = (N + 1) * (N + 2) * (N + 3) / 6, Nfp = (N + 1) * (N + 2) / 2;
  const int RB = (Np + 15) / 16, FK = (Nfp + 15) / 16;
  return (3 * RB * RB + RB * 4 * FK) * 64 * 4;
}

// Number of doubles of the 3D operator fragments for degree N.
inline int frag3_size(int N) {
  const int Np = (N + 1) * (N + 2) * (N + 3) / 6, Nfp = (N + 1) * (N + 2) / 2;
  const int RG = (Np + 3) / 4, FK = (Nfp + 3) / 4;
  return (3 * RG * RG + RG * 4 * FK) * 16;
}

// 3D level.  State layout [tile][field][node][16]; geometry [tile][12][16]:
// rx ry rz sx sy sz tx ty tz 1/rho rho*c^2 rho*c; zn [tile][4][16] impedance
// of the neighbour across each face (the element's own on boundary faces); nbr [tile][4][16] face codes:
//   >= 0 : (e2 << 5) | (f2 << 3) | perm      interior face
//   <  0 : -1 - ((t << 5) | (perm << 2) | bc) boundary; bc 0 = HABC
//          (t = triangle, perm = vertex permutation to it), 1 = ABC,
//          2 = Dirichlet
struct Lvl3 {
  int K, ntile, N, Np, Nfp;
  int nqb3;            // doubles in qb3 (>= Nfp)
  // A-fragments of the FP64 4x4x4 MFMA: Dr, Ds, Dt as [3][RG][RG][16] with
  // entry t = i + 4 k holding D[4 rg + i][4 ks + k], then LIFT as
  // [RG][4 faces][FK][16] with entry t holding LIFT[4 rg + i][f Nfp + 4 jj + k];
  // zero outside the matrix.  RG = ceil(Np/4), FK = ceil(Nfp/4).
  const double* ops;
  // FP32 variant: A-fragments of the FP32 16x16x4 MFMA, Dr, Ds, Dt as
  // [3][RB][RG][64] with lane l holding D[16 rb + l%16][4 j + l/16], then
  // LIFT as [RB][4][FK][64] with lane l holding LIFT[16 rb + l%16][f Nfp +
  // 4 jj + l/16]; zero outside the matrix.  RB = ceil(Np/16).
  const float* ops32;
  // BF16 variant: A-fragments of the BF16 16x16x16 MFMA, Dr, Ds, Dt as
  // [3][RB][RB][64] with lane l holding the four BF16 values D[16 rb + l%16]
  // [16 j + 4 (l/16) + i], i = 0..3, then LIFT as [RB][4][FKB][64] with lane
  // l holding LIFT[16 rb + l%16][f Nfp + 16 jj + 4 (l/16) + i]; zero outside
  // the matrix.  FKB = ceil(Nfp/16).
  const unsigned short* opsb;
  const int* fmask;    // 4 x Nfp
  const int* fmap;     // 4 x 4 x 6 x Nfp
  const double* geo;
  const double* zn;
  const int* nbr;
  int kvar;    // 3D kernel where the tile fits on chip: 0 tile on chip, 1 register-streaming
  int waves;   // register-streaming kernels: waves (tiles of 16 elements) per workgroup, 4 or 8
  int order;   // work items: 0 XCD-contiguous ranges, 1 round-robin over blocks
  int eighths; // persistent grid: this many eighths of the resident workgroups
};

// Persistent grid of a 3D launch: the resident workgroups (fewer when there
// are fewer items) times eighths/8, a multiple of 8 so that every XCD has
// blocks for its range.
inline int grid3(long long resident, long long items, int eighths) {
  const long long b = (resident < items ? resident : items) * eighths / 8;
  return (int)(b < 8 ? 8 : b / 8 * 8);
}

// 2D level (faces).  q2 [Ktri][P][3][Np2]; geo [Ktri][8]: rx ry sx sy 1/rho
// rho*c^2 rho*c (pad); info [Ktri][8]: owning tet, axis of the domain face,
// sign of its outward normal (+-1), edge codes x3, (pad x2); edge code >= 0:
// neighbour triangle; < 0: -1 - ((line << 3) | (side << 2) | bc), bc 0 =
// HABC edge (a line), 1 = ABC, 2 = Dirichlet.  nbrnode [Ktri][3][Nfp2]: the
// neighbour's node (interior edges) or the line node (HABC edges).
struct Lvl2 {
  int Kt, P, Np, Nfp;
  double invM;
  const double* ops;   // Dr2 | Ds2 | LIFT2 (Np x 3Nfp)
  const int* fmask;    // 3 x Nfp
  const double* geo;
  // [Ktri][3 edges][8]: unit in-plane normal (2), face scale, upwind-flux
  // weights aM = ZP/(Z+ZP), aP = Z/(Z+ZP), iZ = 1/(Z+ZP), bZ = Z aM, pad
  const double* edge;
  const int* info;
  const int* tetnode;  // [Ktri][Np2] node of the owning tet
  const int* nbrnode;
  const double* gamma; // P
};

// 1D level (edges).  q1 [Klin][P*P][2][Np1]; geo [Klin][4]: rx 1/rho
// rho*c^2 rho*c; info [Klin][8]: tri side0, tri side1, velocity component of
// the side-0 triangle along the side-1 face normal (1 or 2), same for side 1,
// end codes x2, normal signs x2 (+-1 as int); end code >= 0: (l2 << 1) | end2;
// < 0: -1 - ((corner << 4) | (slot << 2) | bc), bc 0 = corner, 1 = ABC,
// 2 = Dirichlet.  trinode [Klin][2][Np1].
struct Lvl1 {
  int Kl, P, Np;
  double invM;
  const double* ops;   // Dr1 (Np x Np) | LIFT1 (Np x 2)
  const double* geo;
  const int* info;
  const int* trinode;
  const double* gamma;
  const double* Cji;   // P x P
  const double* Cij;
  const double* G;     // 2P x 2P
  const double* H;
};

// 0D level (corners).  info [Kpnt][3][2]: line, end; nrm [Kpnt][3].
struct Lvl0 {
  int Kp, P;
  const int* info;
  const double* nrm;
  const double* Tt;    // transposed corner map: Tt[k][row] = T[row][k], 3P^2 x 3P^2
};

// Shots stepped together: every state array holds n shots, shot k of an
// array at k times its stride (in doubles).  Point sources per shot: w[k][Np]
// weights, par[k][4] = (slot of the element or -1, f0, t0, amp); tau = the
// stage time.
struct Shots {
  int n;
  size_t st3;    // q3, res3
  size_t st2;    // q2, res2
  size_t stb3;   // qb3, q0_3
  size_t st1;    // q1, res1
  size_t stb2;   // qb2, q0_2
  size_t stb1;   // qb1
  const double* srcw;
  const double* srcp;
  double tau;          // stage time (eager stepping)
  // replayed stepping: the stage time is clk[0] + clk[1] dt + cs dt, with
  // clk = {t_start, steps done} on the device (null: use tau)
  const double* clk;
  double cs;
  double dt;
};

// One member of a group step (several contexts with the same N in one 3D
// launch): its level, buffers and shots, and its range of the work list.
struct Member3 {
  Lvl3 L;
  const void* qo;
  void* qn;
  void* res;
  const double* qb3;
  Shots sh;
  long long first;   // first item of the group's work list owned by this member
  int ngrp;          // tile groups per shot
};
constexpr int kMaxGroup = 8;
// N <= 4 (the tile-on-chip kernels), FP64 or FP32 state; G in device memory
hipError_t launch_level3_group(const Member3* G, int nm, long long total, int N, double A,
                               double B, double dt, double tau, double cs, hipStream_t st);
hipError_t launch_level3_f32_group(const Member3* G, int nm, long long total, int N, double A,
                                   double B, double dt, double tau, double cs, hipStream_t st);
hipError_t launch_level3_bf16_group(const Member3* G, int nm, long long total, int N, double A,
                                   double B, double dt, double tau, double cs, hipStream_t st);

// the device clock of replayed stepping: clk = {t0, 0}; clk[1] += 1
hipError_t launch_clock_set(double* clk, double t0, hipStream_t st);
hipError_t launch_clock_tick(double* clk, hipStream_t st);

hipError_t launch_level3(const Lvl3& L, const double* qo, double* qn, double* res,
                         const double* qb3, double A, double B, double dt, const Shots& sh,
                         hipStream_t st);
// FP32 state, FP32 MFMA (levels_fp32.hip); qb3 and the rest of the step FP64.
hipError_t launch_level3_f32(const Lvl3& L, const float* qo, float* qn, float* res,
                             const double* qb3, double A, double B, double dt, const Shots& sh,
                             hipStream_t st);
hipError_t launch_level3_bf16(const Lvl3& L, const float* qo, float* qn, float* res,
                              const double* qb3, double A, double B, double dt, const Shots& sh,
                              hipStream_t st);
// Work list of the line-group kernel: block b updates the lines
// lines[b][*] (each with its edge system), then the corners corners[b][*];
// -1 ends a list.  A block holds every line of its corners.

// 1D and 0D levels of one stage (after the 3D and 2D updates).
hipError_t launch_boundary(const Lvl2& L2, const Lvl1& L1, const Lvl0& L0,
                           const Lvl3& L3, const double* q2o, double* q2n, double* res2,
                           double* qb2, double* qb3, double* q03, const double* q3n,
                           const double* q1o, double* q1n, double* res1, double* qb1,
                           double* q02, double A, double B, double dt, const Shots& sh,
                           hipStream_t st);
// Face level on MFMA (all triangles, TW = 16 / P per wave): ops holds Dr2,
// Ds2 as [2][RG][RG][16] and LIFT2 as [RG][3][EK][16] 4x4x4 A-fragments
// (entry t = i + 4 k), RG = ceil(Np2/4), EK = ceil(Nfp2/4).
struct LvlF {
  int np3;             // nodes of the 3D element (q3 layout)
  const double* ops;
};
struct FaceBufs {
  const double* q2o;
  double *q2n, *res2, *qb3, *q03;
  const void* q3n;     // new 3D state: double, or float for the FP32 variant
  const double* qb2;
  int q3f32;           // 1 if q3n holds floats
};
hipError_t launch_faces(const LvlF& F, const Lvl2& L2, const FaceBufs& b, const Shots& sh,
                        double A, double B, double dt, hipStream_t st);
inline int frag2_size(int N) {
  const int Np = (N + 1) * (N + 2) / 2, Nfp = N + 1, RG = (Np + 3) / 4, EK = (Nfp + 3) / 4;
  return (2 * RG * RG + RG * 3 * EK) * 16;
}

// Learned closure (closure.hip): the decay per step exp(-dt/tau_k) of the
// averages of p^2 and (Z |u_t|)^2 at the closure's time scales tau_k.
constexpr int kMemScales = 4;
struct Memory {
  float decay[kMemScales];
};

// Learned closure (closure.hip): MLP parameters, flat, FP32.
constexpr int kMlpParams = 9091;
size_t mlp_work_floats(int n);
// largest batch of the no-allocation gradient (its work array's size)
constexpr int kMlpStaticBatch = 4096;
// The no-allocation gradient's work array on the device of `st` (the
// current device for the null stream), resolved once per device.
hipError_t mlp_static_work(hipStream_t st, float** work);
const float* mlp_loss_partials(const float* work, int n);
hipError_t mlp_forward(const float* W, const float* X, int n, float* Y, hipStream_t st);
hipError_t mlp_grad(const float* W, const float* X, const float* T, int n, float* G, float* work,
                    hipStream_t st);
hipError_t mlp_grad_bf16(const float* W, const float* X, const float* T, int n, float* G,
                         float* work, hipStream_t st);
const float* mlp_loss_partials_bf16(const float* work, int n);
hipError_t mlp_adam(float* W, const float* G, float* M, float* V, int t, float lr, float b1,
                    float b2, float eps, hipStream_t st);
hipError_t launch_closure(const Lvl2& L2, const float* W, const void* q3, int q3f32, int np3,
                          float* hist, double* qb3, double* q03, const Shots& sh,
                          const Memory& mem, hipStream_t st);
hipError_t launch_hist_push(const Lvl2& L2, const void* q3, int q3f32, int np3, float* hist,
                            const Shots& sh, const Memory& mem, hipStream_t st);
hipError_t launch_closure_sample(const Lvl2& L2, const void* q3, int q3f32, int np3,
                                 const float* hist, const double* qb3, float* X, float* Y,
                                 hipStream_t st);

// Arrays scanned by the finiteness check (at most kScanMax of them); the
// kernel writes one int per (array, block): 1 if a non-finite value was seen.
constexpr int kScanMax = 12;
constexpr int kScanBlocks = 256;
struct ScanList {
  const void* ptr[kScanMax];
  size_t n[kScanMax];
  int f32[kScanMax];   // 1: the array holds floats, 0: doubles
  int count;
};
hipError_t launch_nonfinite(const ScanList& s, int* flags, hipStream_t st);

// FP64 energy partial sums: one value per tile written to out[ntile]; q
// holds doubles, or floats if q_f32.
hipError_t launch_energy(const Lvl3& L, const void* q, int q_f32, const double* mass,
                         const double* J, double* out, hipStream_t st);

}  // namespace dgh
