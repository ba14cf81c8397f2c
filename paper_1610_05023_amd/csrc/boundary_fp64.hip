// FP64 boundary levels of one Runge-Kutta stage in one launch (Algorithm 1
// after the volume update): the 2D face systems with the face rule, the 1D
// edge systems with the edge compatibility systems, and the corner systems.
//
// Every block works from its entry in the work list: first its triangles
// (P sets in parallel: thread = triangle x set x node), then its lines one
// after the other, then its corners.  A block that owns a line also owns the
// triangles next to it and, if the line ends at a corner, the corner's three
// lines, so the new 2D traces the edge system needs and the new 1D traces
// the corner system needs are produced by the same block.  Blocks without
// lines (most of them) only update triangles.
//
// Discretisation as for the volume (Section 3.2), with the face system
//   (1+g_i) dp*_i/dt + rho c^2 div v_i = 0, rho dv_i/dt + grad p_i = 0,
// the edge system
//   (1+g_i+g_j) dp*_ij/dt + rho c^2 dw_ij/dx = 0, rho dw_ij/dt + dp_ij/dx = 0,
// the stored pressures p_i = p*_i + S and p_ij = p*_ij + C_ji S_A,i + C_ij S_B,j
// (Section 3.1), and the characteristic fluxes with Z = rho c.
#include <hip/hip_runtime.h>

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

struct Bufs {
  const double* q2o;
  double *q2n, *res2, *qb2, *qb3, *q03;
  const double* q3n;
  const double* q1o;
  double *q1n, *res1, *qb1, *q02;
};

__global__ void __launch_bounds__(512) k_boundary(LvlB W, Lvl2 L2, Lvl1 L1, Lvl0 L0, Lvl3 L3,
                                                  Bufs b, double A, double B, double dt) {
  extern __shared__ double smem[];
  const int P = L2.P, Pe = P > 0 ? P : 1;
  const int tid = threadIdx.x, nth = blockDim.x, blk = blockIdx.x;
  // ---------------------------------------------------------------- 2D ----
  {
    const int Np = L2.Np, Nfp = L2.Nfp, NE = 3 * Nfp, NS = W.NS, TPB = W.TPB;
    double* sDr = smem;
    double* sDs = sDr + Np * Np;
    double* sL = sDs + Np * Np;                 // Np x NE
    double* sq = sL + Np * NE;                  // TPB x P x 3 x Np
    double* sf = sq + TPB * P * 3 * Np;         // TPB x P x 2 x NE
    double* sps = sf + TPB * P * 2 * NE;        // TPB x P x Np
    double* sS = sps + TPB * P * Np;            // TPB x Np
    for (int x = tid; x < 2 * Np * Np + Np * NE; x += nth) sDr[x] = L2.ops[x];
    const int per = Pe * NS;
    const int tl = tid / per, rem = tid - tl * per, i = rem / NS, slot = rem - i * NS;
    const int ntri = W.ntri[blk];
    for (int c0 = 0; c0 < ntri; c0 += TPB) {
      const int t = (tl < TPB && c0 + tl < ntri) ? W.tris[blk * W.maxtri + c0 + tl] : -1;
      __syncthreads();
      if (t >= 0)
        for (int x = rem; x < P * 3 * Np; x += per)
          sq[tl * P * 3 * Np + x] = b.q2o[(size_t)t * P * 3 * Np + x];
      double rx = 0, ry = 0, sx = 0, sy = 0, irho = 0, Kb = 0, Z = 1;
      int info[6] = {0, 0, 0, 0, 0, 0};
      if (t >= 0) {
        const double* gg = L2.geo + (size_t)t * 8;
        rx = gg[0]; ry = gg[1]; sx = gg[2]; sy = gg[3]; irho = gg[4]; Kb = gg[5]; Z = gg[6];
        for (int k = 0; k < 6; ++k) info[k] = L2.info[t * 8 + k];
      }
      const bool act = t >= 0 && i < P;
      // loads of this thread that do not depend on the tile: the previous
      // residual and q0 of its node, the new 3D trace for the face rule, and
      // the neighbour's trace (or the edge characteristic) of its edge node
      double r0 = 0, r1 = 0, r2 = 0, S0 = 0, p3 = 0, u3 = 0;
      if (act && slot < Np) {
        const size_t base = ((size_t)t * P + i) * 3 * Np + slot;
        r0 = b.res2[base];
        r1 = b.res2[base + Np];
        r2 = b.res2[base + 2 * Np];
        S0 = b.q03[(size_t)t * Np + slot];
      }
      if (t >= 0 && i == 0 && slot < Np) {
        const int e = info[0], n3 = L2.tetnode[(size_t)t * Np + slot];
        const double* q3 = b.q3n + (size_t)(e >> 4) * 4 * L3.Np * kTile + (e & 15);
        p3 = q3[n3 * kTile];
        u3 = q3[((1 + info[1]) * L3.Np + n3) * kTile];
      }
      int ef = 0, ek = 0, code = 0, nn = 0;
      double gP = 0, gA = 0, gB = 0, gZ = 1, grm = 0;
      if (act && slot < NE) {
        ef = slot / Nfp;
        ek = slot - ef * Nfp;
        code = info[3 + ef];
        nn = L2.nbrnode[(t * 3 + ef) * Nfp + ek];
        if (code >= 0) {
          const double* q = b.q2o + ((size_t)code * P + i) * 3 * Np;
          gP = q[nn];
          gA = q[Np + nn];
          gB = q[2 * Np + nn];
          gZ = L2.geo[(size_t)code * 8 + 6];
        } else {
          const int c = -1 - code;
          if ((c & 3) == 0) grm = b.qb2[(((size_t)(c >> 3) * 2 + ((c >> 2) & 1)) * P + i) * Nfp + nn];
        }
      }
      __syncthreads();
      const double* sqt = sq + (tl * P + i) * 3 * Np;
      // edge normals (a, b) of the edges s = -1, r + s = 0, r = -1 and Fscale
      double en[3][3];
      {
        const double v[3][2] = {{-sx, -sy}, {rx + sx, ry + sy}, {-rx, -ry}};
        for (int f = 0; f < 3; ++f) {
          const double m = sqrt(v[f][0] * v[f][0] + v[f][1] * v[f][1]);
          en[f][2] = m;
          en[f][0] = t >= 0 ? v[f][0] / m : 0.0;
          en[f][1] = t >= 0 ? v[f][1] / m : 0.0;
        }
      }
      const double Ki = act ? Kb / (1.0 + L2.gamma[i]) : 0.0;
      // ---- fluxes on the 3 edges
      if (act && slot < NE) {
        const int a = L2.fmask[ef * Nfp + ek];
        const double na = en[ef][0], nb = en[ef][1];
        const double pM = sqt[a];
        const double vnM = na * sqt[Np + a] + nb * sqt[2 * Np + a];
        double pF, vnF;
        if (code >= 0)
          upwind2(pM, vnM, Z, gP, na * gA + nb * gB, gZ, pF, vnF);
        else
          bcflux2((-1 - code) & 3, pM, vnM, Z, grm, pF, vnF);
        double* sft = sf + (tl * P + i) * 2 * NE;
        sft[slot] = en[ef][2] * Ki * (vnM - vnF);
        sft[NE + slot] = en[ef][2] * irho * (pM - pF);
      }
      __syncthreads();
      // ---- volume, lift, update of set i
      if (act && slot < Np) {
        const int a = slot;
        const double* sft = sf + (tl * P + i) * 2 * NE;
        double pr_ = 0, ps_ = 0, div = 0;
        for (int m = 0; m < Np; ++m) {
          const double dr = sDr[a * Np + m], ds = sDs[a * Np + m];
          const double p = sqt[m], va = sqt[Np + m], vb = sqt[2 * Np + m];
          pr_ += dr * p;
          ps_ += ds * p;
          div += dr * (rx * va + ry * vb) + ds * (sx * va + sy * vb);
        }
        double lp = 0, lv[3] = {0, 0, 0};
        for (int f = 0; f < 3; ++f)
          for (int k = 0; k < Nfp; ++k) {
            const int j = f * Nfp + k;
            const double l = sL[a * NE + j];
            lp += l * sft[j];
            lv[f] += l * sft[NE + j];
          }
        double rhs1 = -irho * (rx * pr_ + sx * ps_), rhs2 = -irho * (ry * pr_ + sy * ps_);
        for (int f = 0; f < 3; ++f) {
          rhs1 += en[f][0] * lv[f];
          rhs2 += en[f][1] * lv[f];
        }
        const size_t base = ((size_t)t * P + i) * 3 * Np + a;
        r0 = A * r0 + dt * (-Ki * div + lp);
        r1 = A * r1 + dt * rhs1;
        r2 = A * r2 + dt * rhs2;
        b.res2[base] = r0;
        b.res2[base + Np] = r1;
        b.res2[base + 2 * Np] = r2;
        sps[(tl * P + i) * Np + a] = sqt[a] - S0 + B * r0;
        b.q2n[base + Np] = sqt[Np + a] + B * r1;
        b.q2n[base + 2 * Np] = sqt[2 * Np + a] + B * r2;
      }
      __syncthreads();
      // ---- face rule: r+ from the new 3D trace, r- = (1/M) sum g_i p*_i
      if (t >= 0 && i == 0 && slot < Np) {
        const int a = slot;
        const double rp = 0.5 * (p3 + Z * (double)info[2] * u3);
        double rm = 0.0;
        for (int s = 0; s < P; ++s) rm += L2.gamma[s] * sps[(tl * P + s) * Np + a];
        rm *= L2.invM;
        const double S = rp + rm;
        b.qb3[(size_t)t * Np + a] = rm;
        b.q03[(size_t)t * Np + a] = S;
        sS[tl * Np + a] = S;
      }
      __syncthreads();
      if (act && slot < Np)
        b.q2n[((size_t)t * P + i) * 3 * Np + slot] = sps[(tl * P + i) * Np + slot] + sS[tl * Np + slot];
    }
  }
  if (W.maxlin == 0 || W.lines[blk * W.maxlin] < 0 || P == 0) return;
  // ---------------------------------------------------------------- 1D ----
  const int PP = P * P, Np = L1.Np;
  double* sq = smem;                   // PP x 2 x Np  (this line, old)
  double* sps = sq + PP * 2 * Np;      // PP x Np      (new p*)
  double* sw = sps + PP * Np;          // PP x Np      (new w)
  double* srp = sw + PP * Np;          // 2P x Np
  double* sb = srp + 2 * P * Np;       // 2P x Np
  double* sS = sb + 2 * P * Np;        // 2P x Np
  double* sC = sS + 2 * P * Np;        // maxcor x 3 x PP x 2 (corner ends: p, w)
  const double* Dr = L1.ops;
  const double* LF = L1.ops + Np * Np;
  for (int li = 0; li < W.maxlin; ++li) {
    const int l = W.lines[blk * W.maxlin + li];
    if (l < 0) break;
    __syncthreads();
    for (int x = tid; x < PP * 2 * Np; x += nth) sq[x] = b.q1o[(size_t)l * PP * 2 * Np + x];
    const double rx = L1.geo[l * 4 + 0], irho = L1.geo[l * 4 + 1], Kb = L1.geo[l * 4 + 2],
                 Z = L1.geo[l * 4 + 3];
    const int* info = L1.info + l * 8;
    __syncthreads();
    for (int x = tid; x < PP * Np; x += nth) {
      const int s = x / Np, a = x - s * Np;
      const int i = s / P, j = s - i * P;
      const double Kij = Kb / (1.0 + L1.gamma[i] + L1.gamma[j]);
      double px = 0, wx = 0;
      for (int m = 0; m < Np; ++m) {
        px += Dr[a * Np + m] * sq[(s * 2) * Np + m];
        wx += Dr[a * Np + m] * sq[(s * 2 + 1) * Np + m];
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
        if (code >= 0) {
          const int l2 = code >> 1, node2 = (code & 1) ? Np - 1 : 0;
          const double* q = b.q1o + (((size_t)l2 * PP + s) * 2) * Np;
          upwind2(pM, wnM, Z, q[node2], n * q[Np + node2], L1.geo[l2 * 4 + 3], pF, wnF);
        } else {
          const int c = -1 - code, bc = c & 3, cs = (c >> 2) & 3, corner = c >> 4;
          const double rm = bc == 0 ? b.qb1[((size_t)corner * 3 + cs) * PP + s] : 0.0;
          bcflux2(bc, pM, wnM, Z, rm, pF, wnF);
        }
        rhs0 += LF[a * 2 + end] * fsc * Kij * (wnM - wnF);
        rhs1 += LF[a * 2 + end] * fsc * irho * (pM - pF) * n;
      }
      const size_t base = (((size_t)l * PP + s) * 2) * Np + a;
      double r = A * b.res1[base] + dt * rhs0;
      b.res1[base] = r;
      const double SA = b.q02[(((size_t)l * 2 + 0) * P + i) * Np + a];
      const double SB = b.q02[(((size_t)l * 2 + 1) * P + j) * Np + a];
      sps[s * Np + a] = sq[(s * 2) * Np + a] - L1.Cji[i * P + j] * SA - L1.Cij[i * P + j] * SB + B * r;
      r = A * b.res1[base + Np] + dt * rhs1;
      b.res1[base + Np] = r;
      const double wn = sq[(s * 2 + 1) * Np + a] + B * r;
      b.q1n[base + Np] = wn;
      sw[s * Np + a] = wn;
    }
    __syncthreads();
    // outgoing 2D characteristics (new 2D traces, written by this block) and b
    for (int x = tid; x < 2 * P * Np; x += nth) {
      const int row = x / Np, a = x - row * Np;
      const int side = row / P, i = row - side * P;
      const int t = info[side], comp = info[2 + side];
      const int node = L1.trinode[((size_t)l * 2 + side) * Np + a];
      const double* q = b.q2n + ((size_t)t * P + i) * 3 * L2.Np;
      const double sgn = comp > 0 ? 1.0 : -1.0;
      const int cc = comp > 0 ? comp : -comp;
      srp[row * Np + a] = 0.5 * (q[node] + L2.geo[(size_t)t * 8 + 6] * sgn * q[cc * L2.Np + node]);
      double bb = 0.0;
      if (side == 0)
        for (int j = 0; j < P; ++j) bb += L1.gamma[j] * sps[(i * P + j) * Np + a];
      else
        for (int ii = 0; ii < P; ++ii) bb += L1.gamma[ii] * sps[(ii * P + i) * Np + a];
      sb[row * Np + a] = bb * L1.invM;
    }
    __syncthreads();
    // edge system r- = G r+ + H b
    for (int x = tid; x < 2 * P * Np; x += nth) {
      const int row = x / Np, a = x - row * Np;
      const int n2 = 2 * P;
      double rm = 0.0;
      for (int k = 0; k < n2; ++k)
        rm += L1.G[row * n2 + k] * srp[k * Np + a] + L1.H[row * n2 + k] * sb[k * Np + a];
      const int side = row / P, i = row - side * P;
      const size_t o = (((size_t)l * 2 + side) * P + i) * Np + a;
      b.qb2[o] = rm;
      const double S = srp[row * Np + a] + rm;
      b.q02[o] = S;
      sS[row * Np + a] = S;
    }
    __syncthreads();
    for (int x = tid; x < PP * Np; x += nth) {
      const int s = x / Np, a = x - s * Np;
      const int i = s / P, j = s - i * P;
      const double p = sps[s * Np + a] + L1.Cji[i * P + j] * sS[i * Np + a] +
                       L1.Cij[i * P + j] * sS[(P + j) * Np + a];
      b.q1n[(((size_t)l * PP + s) * 2) * Np + a] = p;
      // keep the corner-end values for the corner systems of this block
      if (a == 0 || a == Np - 1)
        for (int ci = 0; ci < W.maxcor; ++ci) {
          const int c = W.corners[blk * W.maxcor + ci];
          if (c < 0) break;
          for (int cs = 0; cs < 3; ++cs)
            if (L0.info[(c * 3 + cs) * 2] == l && (L0.info[(c * 3 + cs) * 2 + 1] ? Np - 1 : 0) == a) {
              sC[((ci * 3 + cs) * PP + s) * 2] = p;
              sC[((ci * 3 + cs) * PP + s) * 2 + 1] = sw[s * Np + a];
            }
        }
    }
  }
  // ---------------------------------------------------------------- 0D ----
  double* srp0 = sC + W.maxcor * 3 * PP * 2;   // 3 PP
  const int n3 = 3 * PP;
  for (int ci = 0; ci < W.maxcor; ++ci) {
    const int c = W.corners[blk * W.maxcor + ci];
    if (c < 0) break;
    __syncthreads();
    for (int x = tid; x < n3; x += nth) {
      const int cs = x / PP;
      const int l = L0.info[(c * 3 + cs) * 2];
      srp0[x] = 0.5 * (sC[(ci * 3 * PP + x) * 2] +
                       L1.geo[l * 4 + 3] * L0.nrm[c * 3 + cs] * sC[(ci * 3 * PP + x) * 2 + 1]);
    }
    __syncthreads();
    for (int x = tid; x < n3; x += nth) {
      double rm = 0.0;
      for (int k = 0; k < n3; ++k) rm += L0.Tt[(size_t)k * n3 + x] * srp0[k];
      b.qb1[(size_t)c * n3 + x] = rm;
    }
  }
}

}  // namespace

hipError_t launch_boundary(const LvlB& W, const Lvl2& L2, const Lvl1& L1, const Lvl0& L0,
                           const Lvl3& L3, const double* q2o, double* q2n, double* res2,
                           double* qb2, double* qb3, double* q03, const double* q3n,
                           const double* q1o, double* q1n, double* res1, double* qb1,
                           double* q02, double A, double B, double dt, hipStream_t st) {
  if (W.nblocks == 0) return hipSuccess;
  const int P = L2.P, Np2 = L2.Np, NE = 3 * L2.Nfp, TPB = W.TPB, Np1 = L1.Np, PP = P * P;
  const size_t a2 = 2 * Np2 * Np2 + Np2 * NE + TPB * P * 3 * Np2 + TPB * P * 2 * NE +
                    TPB * P * Np2 + TPB * Np2;
  const size_t a1 = PP * 2 * Np1 + 2 * PP * Np1 + 6 * P * Np1 + W.maxcor * 3 * PP * 2 + 3 * PP;
  const size_t lds = sizeof(double) * (a2 > a1 ? a2 : a1);
  static size_t attr = 0;
  if (lds > attr) {
    hipFuncSetAttribute((const void*)k_boundary, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    attr = lds;
  }
  Bufs b{q2o, q2n, res2, qb2, qb3, q03, q3n, q1o, q1n, res1, qb1, q02};
  hipLaunchKernelGGL(k_boundary, dim3(W.nblocks), dim3(512), lds, st, W, L2, L1, L0, L3, b, A, B,
                     dt);
  return hipGetLastError();
}

}  // namespace dgh
