// FP64 edge and corner levels of one Runge-Kutta stage (Algorithm 1 after
// the volume and face updates): the 1D edge systems with the edge
// compatibility systems, and the corner systems.
//
// One block per line (the lines of a stage are independent: each reads the
// stage-start states of its neighbours and the corner r- of the previous
// stage), then one block per corner in a second launch, which reads the new
// line-end values; the new 2D traces the edge systems need come from the
// face kernel launched before.
//
// Discretisation as for the volume (Section 3.2), with the face system
//   (1+g_i) dp*_i/dt + rho c^2 div v_i = 0, rho dv_i/dt + grad p_i = 0,
// the edge system
//   (1+g_i+g_j) dp*_ij/dt + rho c^2 dw_ij/dx = 0, rho dw_ij/dt + dp_ij/dx = 0,
// the stored pressures p_i = p*_i + S and p_ij = p*_ij + C_ji S_A,i + C_ij S_B,j
// (Section 3.1), and the characteristic fluxes with Z = rho c.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "launch.hpp"
#include "levels.hpp"

namespace dgh {

namespace {

__device__ __forceinline__ void upwind2(double pM, double unM, double ZM, double pP, double unP,
                                        double ZP, double& pF, double& unF) {
  const double iZ = 1.0 / (ZM + ZP);
  pF = (ZP * pM + ZM * pP + ZM * ZP * (unM - unP)) * iZ;
  unF = (pM - pP + ZM * unM + ZP * unP) * iZ;
}

__device__ __forceinline__ void bcflux2(int bc, double pM, double unM, double Z, double rm,
                                        double& pF, double& unF) {
  if (bc == 2) {  // p = 0
    pF = 0.0;
    unF = unM + pM / Z;
  } else {
    const double rp = 0.5 * (pM + Z * unM);
    const double r = bc == 0 ? rm : 0.0;
    pF = rp + r;
    unF = (rp - r) / Z;
  }
}

// Per-node inputs of the 1D update, loaded before any store of the phase.
struct LineNode {
  bool on;
  int s, a;
  double ro0, ro1, SA, SB;
  double xp[2], xw[2], xz[2], xr[2];
};

struct Bufs {
  const double* q2o;
  double *q2n, *res2, *qb2, *qb3, *q03;
  const double* q3n;
  const double* q1o;
  double *q1n, *res1, *qb1, *q02;
};

// One block per line.  NPT edge nodes per thread (NPT 512 >= P^2 Np1).
template <int NPT>
__global__ void __launch_bounds__(512, 4) k_boundary(Lvl2 L2, Lvl1 L1, int np3, Bufs b, Shots sh,
                                                     double A, double B, double dt) {
  extern __shared__ double smem[];
  {
    // this block's shot
    const size_t k = blockIdx.y;
    b.q2o += k * sh.st2;
    b.q2n += k * sh.st2;
    b.res2 += k * sh.st2;
    b.qb3 += k * sh.stb3;
    b.q03 += k * sh.stb3;
    b.q1o += k * sh.st1;
    b.q1n += k * sh.st1;
    b.res1 += k * sh.st1;
    b.qb2 += k * sh.stb2;
    b.q02 += k * sh.stb2;
    b.qb1 += k * sh.stb1;
  }
  const int P = L2.P;
  const int tid = threadIdx.x, nth = blockDim.x, blk = blockIdx.x;
  // Every phase issues all of a thread's global loads before its first
  // global store, so that they are in flight together (the state arrays may
  // alias as far as the compiler knows); small constant tables sit in LDS.
  if (blk >= L1.Kl || P == 0) return;
  // ---------------------------------------------------------------- 1D ----
  const int PP = P * P, Np = L1.Np, n2 = 2 * P;
  double* cDr = smem;                  // Np x Np
  double* cLF = cDr + Np * Np;         // Np x 2
  double* cG = cLF + 2 * Np;           // 2P x 2P
  double* cH = cG + n2 * n2;           // 2P x 2P
  double* cCji = cH + n2 * n2;         // P x P
  double* cCij = cCji + PP;            // P x P
  double* cg = cCij + PP;              // P
  double* sq = cg + P;                 // PP x 2 x Np  (this line, old)
  double* sps = sq + PP * 2 * Np;      // PP x Np      (new p*)
  double* sw = sps + PP * Np;          // PP x Np      (new w)
  double* srp = sw + PP * Np;          // 2P x Np
  double* sb = srp + n2 * Np;          // 2P x Np
  double* sS = sb + n2 * Np;           // 2P x Np
  // The constant tables and this line's old state go to LDS, each thread's
  // entries loaded into registers first (at most one of Dr|LIFT, two of G
  // and of H, one of Cji, Cij and gamma, four of the state: the launcher
  // checks the sizes), so that they are in flight with the loads below and
  // the line costs two rounds of loads, not three.
  const int nops = Np * Np + 2 * Np, ng = n2 * n2, nq = PP * 2 * Np;
  double vo = 0.0, vG[2] = {0.0, 0.0}, vH[2] = {0.0, 0.0}, vCji = 0.0, vCij = 0.0, vg = 0.0;
  double vq[4];
  if (tid < nops) vo = L1.ops[tid];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int x = tid + h * nth;
    if (x < ng) {
      vG[h] = L1.G[x];
      vH[h] = L1.H[x];
    }
  }
  if (tid < PP) {
    vCji = L1.Cji[tid];
    vCij = L1.Cij[tid];
  }
  if (tid < P) vg = L1.gamma[tid];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int x = tid + h * nth;
    vq[h] = x < nq ? b.q1o[(size_t)blk * nq + x] : 0.0;
  }
  {
    const int l = blk;
    const double rx = L1.geo[l * 4 + 0], irho = L1.geo[l * 4 + 1], Kb = L1.geo[l * 4 + 2],
                 Z = L1.geo[l * 4 + 3];
    int info[8];
    for (int k = 0; k < 8; ++k) info[k] = L1.info[l * 8 + k];
    // this thread's entry (row, node) of the 2P x Np table of outgoing 2D
    // characteristics: the new face traces (written by the face kernel,
    // never by this one) are loaded now, in flight with the loads below
    // (2P Np <= 168 < 512 threads: one entry per thread)
    const bool yon = tid < n2 * Np;
    double ypv = 0.0, yuv = 0.0, yzt = 1.0;
    if (yon) {
      const int row = tid / Np, cy = tid - row * Np;
      const int side = row / P, ii = row - side * P;
      const int t = info[side], comp = info[2 + side];
      const int node = L1.trinode[((size_t)l * 2 + side) * Np + cy];
      const double* q = b.q2n + ((size_t)t * P + ii) * 3 * L2.Np;
      const int cc = comp > 0 ? comp : -comp;
      yzt = L2.geo[(size_t)t * 8 + 6];
      ypv = q[node];
      yuv = q[cc * L2.Np + node];
    }
    // loads of this thread's nodes (x = tid + h nth, h < NPT: NPT nth >=
    // P^2 Np1): old residuals, q0 of both faces, and the exterior values at
    // both line ends (neighbour line or corner r-)
    LineNode nd[NPT];
#pragma unroll
    for (int h = 0; h < NPT; ++h) {
      LineNode& v = nd[h];
      const int x = tid + h * nth;
      v.on = x < PP * Np;
      v.s = v.on ? x / Np : 0;
      v.a = v.on ? x - v.s * Np : 0;
      if (v.on) {
        const int i = v.s / P, j = v.s - i * P;
        const size_t base = (((size_t)l * PP + v.s) * 2) * Np + v.a;
        v.ro0 = b.res1[base];
        v.ro1 = b.res1[base + Np];
        v.SA = b.q02[(((size_t)l * 2 + 0) * P + i) * Np + v.a];
        v.SB = b.q02[(((size_t)l * 2 + 1) * P + j) * Np + v.a];
        for (int end = 0; end < 2; ++end) {
          const int code = info[4 + end];
          v.xp[end] = v.xw[end] = v.xr[end] = 0.0;
          v.xz[end] = 1.0;
          if (code >= 0) {
            const int l2 = code >> 1, node2 = (code & 1) ? Np - 1 : 0;
            const double* q = b.q1o + (((size_t)l2 * PP + v.s) * 2) * Np;
            v.xp[end] = q[node2];
            v.xw[end] = q[Np + node2];
            v.xz[end] = L1.geo[l2 * 4 + 3];
          } else {
            const int c = -1 - code, cs = (c >> 2) & 3, corner = c >> 4;
            if ((c & 3) == 0) v.xr[end] = b.qb1[((size_t)corner * 3 + cs) * PP + v.s];
          }
        }
      }
    }
    if (tid < nops) cDr[tid] = vo;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int x = tid + h * nth;
      if (x < ng) {
        cG[x] = vG[h];
        cH[x] = vH[h];
      }
    }
    if (tid < PP) {
      cCji[tid] = vCji;
      cCij[tid] = vCij;
    }
    if (tid < P) cg[tid] = vg;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int x = tid + h * nth;
      if (x < nq) sq[x] = vq[h];
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < NPT; ++h) {
      const LineNode& v = nd[h];
      if (!v.on) continue;
      const int s = v.s, a = v.a, i = s / P, j = s - i * P;
      const double Kij = Kb / (1.0 + cg[i] + cg[j]);
      double px = 0, wx = 0;
      for (int m = 0; m < Np; ++m) {
        px += cDr[a * Np + m] * sq[(s * 2) * Np + m];
        wx += cDr[a * Np + m] * sq[(s * 2 + 1) * Np + m];
      }
      px *= rx;
      wx *= rx;
      double rhs0 = -Kij * wx, rhs1 = -irho * px;
      const double fsc = fabs(rx);
      for (int end = 0; end < 2; ++end) {
        const int node = end ? Np - 1 : 0;
        const double n = (double)info[6 + end];
        const double pM = sq[(s * 2) * Np + node];
        const double wnM = n * sq[(s * 2 + 1) * Np + node];
        const int code = info[4 + end];
        double pF, wnF;
        if (code >= 0)
          upwind2(pM, wnM, Z, v.xp[end], n * v.xw[end], v.xz[end], pF, wnF);
        else
          bcflux2((-1 - code) & 3, pM, wnM, Z, v.xr[end], pF, wnF);
        rhs0 += cLF[a * 2 + end] * fsc * Kij * (wnM - wnF);
        rhs1 += cLF[a * 2 + end] * fsc * irho * (pM - pF) * n;
      }
      const size_t base = (((size_t)l * PP + s) * 2) * Np + a;
      const double r0 = A * v.ro0 + dt * rhs0, r1 = A * v.ro1 + dt * rhs1;
      b.res1[base] = r0;
      b.res1[base + Np] = r1;
      sps[s * Np + a] = sq[(s * 2) * Np + a] - cCji[i * P + j] * v.SA - cCij[i * P + j] * v.SB + B * r0;
      const double wn = sq[(s * 2 + 1) * Np + a] + B * r1;
      b.q1n[base + Np] = wn;
      sw[s * Np + a] = wn;
    }
    __syncthreads();
    // outgoing 2D characteristics (from the new 2D traces loaded above) and b
    if (yon) {
      const int row = tid / Np, c = tid - row * Np;
      const int side = row / P, ii = row - side * P;
      const double sgn = info[2 + side] > 0 ? 1.0 : -1.0;
      double bb = 0.0;
      if (side == 0)
        for (int jj = 0; jj < P; ++jj) bb += cg[jj] * sps[(ii * P + jj) * Np + c];
      else
        for (int i2 = 0; i2 < P; ++i2) bb += cg[i2] * sps[(i2 * P + ii) * Np + c];
      sb[row * Np + c] = bb * L1.invM;
      srp[row * Np + c] = 0.5 * (ypv + yzt * sgn * yuv);
    }
    __syncthreads();
    // edge system r- = G r+ + H b
    for (int y = tid; y < n2 * Np; y += nth) {
      const int row = y / Np, c = y - row * Np;
      double rm = 0.0;
      for (int k = 0; k < n2; ++k)
        rm += cG[row * n2 + k] * srp[k * Np + c] + cH[row * n2 + k] * sb[k * Np + c];
      const int side = row / P, ii = row - side * P;
      const size_t o = (((size_t)l * 2 + side) * P + ii) * Np + c;
      b.qb2[o] = rm;
      const double S = srp[row * Np + c] + rm;
      b.q02[o] = S;
      sS[row * Np + c] = S;
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < NPT; ++h) {
      const LineNode& v = nd[h];
      if (!v.on) continue;
      const int s = v.s, a = v.a, i = s / P, j = s - i * P;
      const double p = sps[s * Np + a] + cCji[i * P + j] * sS[i * Np + a] +
                       cCij[i * P + j] * sS[(P + j) * Np + a];
      b.q1n[(((size_t)l * PP + s) * 2) * Np + a] = p;
    }
  }
}

// ---------------------------------------------------------------- 0D ----
// One block per corner: r+ from the new ends of its three lines, then
// r- = T r+ with the 3P^2 x 3P^2 corner map; the products are split over
// the block (nparts partial sums per output) and reduced in LDS.
__global__ void __launch_bounds__(512) k_corners(Lvl1 L1, Lvl0 L0, Bufs b, Shots sh) {
  extern __shared__ double smem[];
  {
    const size_t k = blockIdx.y;   // this block's shot
    b.q1n += k * sh.st1;
    b.qb1 += k * sh.stb1;
  }
  const int P = L1.P, PP = P * P, n3 = 3 * PP, Np = L1.Np;
  const int tid = threadIdx.x, nth = blockDim.x, c = blockIdx.x;
  double* srp0 = smem;         // 3 PP
  double* sred = srp0 + n3;    // max(nth, n3) partial sums
  const int nparts = nth / n3 > 0 ? nth / n3 : 1;
  {
    for (int y = tid; y < n3; y += nth) {
      const int cs = y / PP, s = y - cs * PP;
      const int l = L0.info[(c * 3 + cs) * 2], end = L0.info[(c * 3 + cs) * 2 + 1];
      const int node = end ? Np - 1 : 0;
      const double* q = b.q1n + (((size_t)l * PP + s) * 2) * Np;
      srp0[y] = 0.5 * (q[node] + L1.geo[l * 4 + 3] * L0.nrm[c * 3 + cs] * q[Np + node]);
    }
    __syncthreads();
    for (int y = tid; y < n3 * nparts; y += nth) {
      const int part = y / n3, xo = y - part * n3;
      double acc = 0.0;
#pragma unroll 8
      for (int k = part; k < n3; k += nparts) acc += L0.Tt[(size_t)k * n3 + xo] * srp0[k];
      sred[y] = acc;
    }
    __syncthreads();
    for (int y = tid; y < n3; y += nth) {
      double rm = 0.0;
      for (int part = 0; part < nparts; ++part) rm += sred[part * n3 + y];
      b.qb1[(size_t)c * n3 + y] = rm;
    }
  }
}

}  // namespace

hipError_t launch_boundary(const Lvl2& L2, const Lvl1& L1, const Lvl0& L0,
                           const Lvl3& L3, const double* q2o, double* q2n, double* res2,
                           double* qb2, double* qb3, double* q03, const double* q3n,
                           const double* q1o, double* q1n, double* res1, double* qb1,
                           double* q02, double A, double B, double dt, const Shots& sh,
                           hipStream_t st) {
  if (L1.Kl == 0) return hipSuccess;
  if (sh.n < 1 || sh.n > 65535) return hipErrorInvalidValue;
  const int P = L2.P, Np1 = L1.Np, PP = P * P;
  if (P == 0) return hipSuccess;   // no edge or corner systems
  const int n2 = 2 * P, n3 = 3 * PP;
  const size_t a1 = Np1 * Np1 + 2 * Np1 + 2 * n2 * n2 + 2 * PP + P + PP * 2 * Np1 +
                    2 * PP * Np1 + 3 * n2 * Np1;
  Bufs b{q2o, q2n, res2, qb2, qb3, q03, q3n, q1o, q1n, res1, qb1, q02};
  // edge nodes at most two per thread; the 2P x Np1 table of outgoing 2D
  // characteristics one entry per thread; the tables and the line state at
  // most as many entries per thread as k_boundary loads
  if (PP * Np1 > 1024 || n2 * Np1 > 512 || Np1 * Np1 + 2 * Np1 > 512 || n2 * n2 > 1024 ||
      PP > 512 || 2 * PP * Np1 > 2048)
    return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * a1;
  // one edge node per thread unless P^2 Np1 exceeds the block (P > 10)
  if (PP * Np1 <= 512) {
    hipError_t e = kernel_setup((const void*)k_boundary<1>, 512, lds, nullptr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_boundary<1>, dim3(L1.Kl, sh.n), dim3(512), lds, st, L2, L1, L3.Np, b,
                       sh, A, B, dt);
  } else {
    hipError_t e = kernel_setup((const void*)k_boundary<2>, 512, lds, nullptr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_boundary<2>, dim3(L1.Kl, sh.n), dim3(512), lds, st, L2, L1, L3.Np, b,
                       sh, A, B, dt);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || L0.Kp == 0) return e;
  // srp0, then the partial sums: nparts n3 <= 512 entries, or n3 when a
  // corner system is larger than the block (nparts = 1)
  const size_t lds0 = sizeof(double) * (n3 + std::max(512, n3));
  e = kernel_setup((const void*)k_corners, 512, lds0, nullptr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_corners, dim3(L0.Kp, sh.n), dim3(512), lds0, st, L1, L0, b, sh);
  return hipGetLastError();
}

}  // namespace dgh
