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

#include "levels.hpp"

namespace dgh {

namespace {

__device__ __forceinline__ void upwind(double pM, double unM, double ZM, double pP, double unP,
                                       double ZP, double& pF, double& unF) {
  // p* = ({p/Z} - n.[[u]]) / {1/Z}, (n.u)* = (n.{Z u} - [[p]]) / {Z}
  const double iZ = 1.0 / (ZM + ZP);
  pF = (ZP * pM + ZM * pP + ZM * ZP * (unM - unP)) * iZ;
  unF = (pM - pP + ZM * unM + ZP * unP) * iZ;
}

__device__ __forceinline__ void charflux(double pM, double unM, double Z, double rm, double& pF,
                                         double& unF) {
  const double rp = 0.5 * (pM + Z * unM);
  pF = rp + rm;
  unF = (rp - rm) / Z;
}

__device__ __forceinline__ void bcflux(int bc, double pM, double unM, double Z, double rm,
                                       double& pF, double& unF) {
  if (bc == 2) {  // p = 0
    pF = 0.0;
    unF = unM + pM / Z;
  } else {
    charflux(pM, unM, Z, bc == 0 ? rm : 0.0, pF, unF);
  }
}

// ------------------------------------------------------------------ 3D ---
// One workgroup per tile of 16 elements, 256 threads: lane (es, g) with
// es = element slot, g = 0..15 a node group.  Operators and the tile's
// fields are staged in LDS; neighbour traces are gathered from the previous
// stage's buffer qo, so the kernel writes qn without races.
template <int N>
__global__ void __launch_bounds__(256) k_level3(Lvl3 L, const double* __restrict__ qo,
                                                double* __restrict__ qn, double* __restrict__ res,
                                                const double* __restrict__ qb3, double A, double B,
                                                double dt, int src_e,
                                                const double* __restrict__ src_w, double src_s) {
  constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  constexpr int Nfp = (N + 1) * (N + 2) / 2;
  constexpr int NF = 4 * Nfp;
  // operators in LDS when they fit beside the tile (N <= 4), else read
  // through the caches
  constexpr bool kOpsLds = (3 * Np * Np + Np * NF) * 8 <= 64 * 1024;
  extern __shared__ double smem[];
  double* sq = smem;                  // 4 Np 16
  double* sf = sq + 4 * Np * kTile;   // 2 NF 16
  double* sops = sf + 2 * NF * kTile; // 3 Np^2 + Np NF (if kOpsLds)
  const int tile = blockIdx.x, tid = threadIdx.x;
  const int es = tid & 15, g = tid >> 4;
  const int e = tile * kTile + es;
  if (kOpsLds)
    for (int i = tid; i < 3 * Np * Np + Np * NF; i += 256) sops[i] = L.ops[i];
  const double* sD = kOpsLds ? sops : L.ops;
  const double* sL = sD + 3 * Np * Np;
  const double* qt = qo + (size_t)tile * 4 * Np * kTile;
  for (int i = tid; i < 4 * Np * kTile; i += 256) sq[i] = qt[i];
  const double* gt = L.geo + (size_t)tile * 12 * kTile + es;
  const double rx = gt[0 * kTile], ry = gt[1 * kTile], rz = gt[2 * kTile];
  const double sx = gt[3 * kTile], sy = gt[4 * kTile], sz = gt[5 * kTile];
  const double tx = gt[6 * kTile], ty = gt[7 * kTile], tz = gt[8 * kTile];
  const double irho = gt[9 * kTile], Kb = gt[10 * kTile], Z = gt[11 * kTile];
  // outward normals -grad(xi) of the faces xi = -1 and grad(r+s+t) of the
  // slanted face; Fscale = |grad xi|
  double nv[4][3] = {{-tx, -ty, -tz}, {-sx, -sy, -sz},
                     {rx + sx + tx, ry + sy + ty, rz + sz + tz}, {-rx, -ry, -rz}};
  double fs[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    fs[f] = sqrt(nv[f][0] * nv[f][0] + nv[f][1] * nv[f][1] + nv[f][2] * nv[f][2]);
    const double inv = 1.0 / fs[f];
    nv[f][0] *= inv;
    nv[f][1] *= inv;
    nv[f][2] *= inv;
  }
  __syncthreads();
  // ---- surface fluxes at the 4 Nfp face nodes
  for (int j = g; j < NF; j += 16) {
    const int f = j / Nfp, i = j - f * Nfp;
    const int n = L.fmask[f * Nfp + i];
    const double nx = nv[f][0], ny = nv[f][1], nz = nv[f][2];
    const double pM = sq[n * kTile + es];
    const double unM = nx * sq[(Np + n) * kTile + es] + ny * sq[(2 * Np + n) * kTile + es] +
                       nz * sq[(3 * Np + n) * kTile + es];
    const int code = L.nbr[(tile * 4 + f) * kTile + es];
    double pF, unF;
    if (code >= 0) {
      const int e2 = code >> 5, f2 = (code >> 3) & 3, pr = code & 7;
      const int n2 = L.fmap[((f * 4 + f2) * 6 + pr) * Nfp + i];
      const double* q2 = qo + (size_t)(e2 >> 4) * 4 * Np * kTile + (e2 & 15);
      const double pP = q2[n2 * kTile];
      const double unP = nx * q2[(Np + n2) * kTile] + ny * q2[(2 * Np + n2) * kTile] +
                         nz * q2[(3 * Np + n2) * kTile];
      upwind(pM, unM, Z, pP, unP, L.zn[(tile * 4 + f) * kTile + es], pF, unF);
    } else {
      const int c = -1 - code;
      const int bc = c & 3;
      double rm = 0.0;
      if (bc == 0) {
        const int pr = (c >> 2) & 7, t = c >> 5;
        rm = qb3[(size_t)t * Nfp + L.fmap[((f * 4 + 0) * 6 + pr) * Nfp + i]];
      }
      bcflux(bc, pM, unM, Z, rm, pF, unF);
    }
    sf[j * kTile + es] = fs[f] * Kb * (unM - unF);
    sf[(NF + j) * kTile + es] = fs[f] * irho * (pM - pF);
  }
  __syncthreads();
  // ---- volume term, lift, update
  for (int n = g; n < Np; n += 16) {
    double pr_ = 0, ps_ = 0, pt_ = 0, div = 0;
    for (int m = 0; m < Np; ++m) {
      const double a = sD[n * Np + m], b = sD[Np * Np + n * Np + m],
                   c = sD[2 * Np * Np + n * Np + m];
      const double p = sq[m * kTile + es], u = sq[(Np + m) * kTile + es],
                   v = sq[(2 * Np + m) * kTile + es], w = sq[(3 * Np + m) * kTile + es];
      pr_ += a * p;
      ps_ += b * p;
      pt_ += c * p;
      div += a * (rx * u + ry * v + rz * w) + b * (sx * u + sy * v + sz * w) +
             c * (tx * u + ty * v + tz * w);
    }
    double lp = 0, la[4] = {0, 0, 0, 0};
#pragma unroll
    for (int f = 0; f < 4; ++f)
      for (int i = 0; i < Nfp; ++i) {
        const int j = f * Nfp + i;
        const double l = sL[n * NF + j];
        lp += l * sf[j * kTile + es];
        la[f] += l * sf[(NF + j) * kTile + es];
      }
    double rhs[4];
    rhs[0] = -Kb * div + lp;
    if (e == src_e) rhs[0] += src_w[n] * src_s;
    rhs[1] = -irho * (rx * pr_ + sx * ps_ + tx * pt_);
    rhs[2] = -irho * (ry * pr_ + sy * ps_ + ty * pt_);
    rhs[3] = -irho * (rz * pr_ + sz * ps_ + tz * pt_);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      rhs[1] += nv[f][0] * la[f];
      rhs[2] += nv[f][1] * la[f];
      rhs[3] += nv[f][2] * la[f];
    }
    if (e < L.K) {
#pragma unroll
      for (int fl = 0; fl < 4; ++fl) {
        const size_t idx = ((size_t)(tile * 4 + fl) * Np + n) * kTile + es;
        const double r = A * res[idx] + dt * rhs[fl];
        res[idx] = r;
        qn[idx] = sq[(fl * Np + n) * kTile + es] + B * r;
      }
    }
  }
}

// ------------------------------------------------------------------ 2D ---
// Block: TPB triangles x NS slots (NS = max(Np2, 3 Nfp2)); sets serial.
__global__ void k_level2(Lvl2 L, Lvl3 L3, const double* __restrict__ q2o,
                         double* __restrict__ q2n, double* __restrict__ res2,
                         const double* __restrict__ qb2, double* __restrict__ qb3,
                         double* __restrict__ q03, const double* __restrict__ q3n, double A,
                         double B, double dt, int TPB, int NS) {
  const int P = L.P, Np = L.Np, Nfp = L.Nfp, NE = 3 * Nfp;
  extern __shared__ double smem[];
  double* sDr = smem;
  double* sDs = sDr + Np * Np;
  double* sL = sDs + Np * Np;              // Np x NE
  double* sq = sL + Np * NE;               // TPB x P x 3 x Np
  double* sf = sq + TPB * P * 3 * Np;      // TPB x 2 x NE
  double* sps = sf + TPB * 2 * NE;         // TPB x P x Np  (new p*)
  const int tid = threadIdx.x;
  const int tl = tid / NS, slot = tid - tl * NS;
  const int t = blockIdx.x * TPB + tl;
  const bool act = tl < TPB && t < L.Kt;
  for (int i = tid; i < 2 * Np * Np + Np * NE; i += blockDim.x) sDr[i] = L.ops[i];
  const int tfirst = blockIdx.x * TPB;
  const int nt = min(TPB, L.Kt - tfirst);
  for (int i = tid; i < nt * P * 3 * Np; i += blockDim.x)
    sq[i] = q2o[(size_t)tfirst * P * 3 * Np + i];
  double rx = 0, ry = 0, sx = 0, sy = 0, irho = 0, Kb = 0, Z = 1;
  int info[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (act) {
    const double* gg = L.geo + (size_t)t * 8;
    rx = gg[0]; ry = gg[1]; sx = gg[2]; sy = gg[3]; irho = gg[4]; Kb = gg[5]; Z = gg[6];
    for (int k = 0; k < 8; ++k) info[k] = L.info[t * 8 + k];
  }
  double en[3][3];  // edge normals (a, b) and Fscale
  {
    const double v[3][2] = {{-sx, -sy}, {rx + sx, ry + sy}, {-rx, -ry}};
    for (int f = 0; f < 3; ++f) {
      const double m = sqrt(v[f][0] * v[f][0] + v[f][1] * v[f][1]);
      en[f][2] = m;
      en[f][0] = act ? v[f][0] / m : 0.0;
      en[f][1] = act ? v[f][1] / m : 0.0;
    }
  }
  __syncthreads();
  const double* sqt = sq + tl * P * 3 * Np;
  for (int i = 0; i < P; ++i) {
    const double Ki = Kb / (1.0 + L.gamma[i]);
    // ---- fluxes on the 3 edges
    if (act && slot < NE) {
      const int f = slot / Nfp, k = slot - f * Nfp;
      const int a = L.fmask[f * Nfp + k];
      const double na = en[f][0], nb = en[f][1];
      const double pM = sqt[(i * 3 + 0) * Np + a];
      const double vnM = na * sqt[(i * 3 + 1) * Np + a] + nb * sqt[(i * 3 + 2) * Np + a];
      const int code = info[3 + f];
      const int nn = L.nbrnode[(t * 3 + f) * Nfp + k];
      double pF, vnF;
      if (code >= 0) {
        const double* q = q2o + ((size_t)code * P + i) * 3 * Np;
        const double pP = q[nn];
        const double vnP = na * q[Np + nn] + nb * q[2 * Np + nn];
        upwind(pM, vnM, Z, pP, vnP, L.geo[(size_t)code * 8 + 6], pF, vnF);
      } else {
        const int c = -1 - code, bc = c & 3, side = (c >> 2) & 1, l = c >> 3;
        double rm = 0.0;
        if (bc == 0) rm = qb2[(((size_t)l * 2 + side) * P + i) * (L.Nfp) + nn];
        bcflux(bc, pM, vnM, Z, rm, pF, vnF);
      }
      sf[(tl * 2 + 0) * NE + slot] = en[f][2] * Ki * (vnM - vnF);
      sf[(tl * 2 + 1) * NE + slot] = en[f][2] * irho * (pM - pF);
    }
    __syncthreads();
    // ---- volume, lift, update of set i
    if (act && slot < Np) {
      const int a = slot;
      double pr_ = 0, ps_ = 0, div = 0;
      for (int m = 0; m < Np; ++m) {
        const double dr = sDr[a * Np + m], ds = sDs[a * Np + m];
        const double p = sqt[(i * 3) * Np + m], va = sqt[(i * 3 + 1) * Np + m],
                     vb = sqt[(i * 3 + 2) * Np + m];
        pr_ += dr * p;
        ps_ += ds * p;
        div += dr * (rx * va + ry * vb) + ds * (sx * va + sy * vb);
      }
      double lp = 0, lv[3] = {0, 0, 0};
      for (int f = 0; f < 3; ++f)
        for (int k = 0; k < Nfp; ++k) {
          const int j = f * Nfp + k;
          const double l = sL[a * NE + j];
          lp += l * sf[(tl * 2) * NE + j];
          lv[f] += l * sf[(tl * 2 + 1) * NE + j];
        }
      double rhs[3];
      rhs[0] = -Ki * div + lp;
      rhs[1] = -irho * (rx * pr_ + sx * ps_);
      rhs[2] = -irho * (ry * pr_ + sy * ps_);
      for (int f = 0; f < 3; ++f) {
        rhs[1] += en[f][0] * lv[f];
        rhs[2] += en[f][1] * lv[f];
      }
      const size_t base = ((size_t)t * P + i) * 3 * Np + a;
      const double S0 = q03[(size_t)t * Np + a];
      double r = A * res2[base] + dt * rhs[0];
      res2[base] = r;
      sps[(tl * P + i) * Np + a] = sqt[(i * 3) * Np + a] - S0 + B * r;
      for (int fl = 1; fl < 3; ++fl) {
        r = A * res2[base + fl * Np] + dt * rhs[fl];
        res2[base + fl * Np] = r;
        q2n[base + fl * Np] = sqt[(i * 3 + fl) * Np + a] + B * r;
      }
    }
    __syncthreads();
  }
  // ---- face rule: r+ from the new 3D trace, r- = (1/M) sum gamma_i p*_i
  if (act && slot < Np) {
    const int a = slot;
    const int e = info[0], ax = info[1];
    const double sgn = (double)info[2];
    const int n3 = L.tetnode[(size_t)t * Np + a];
    const double* q3 = q3n + (size_t)(e >> 4) * 4 * L3.Np * kTile + (e & 15);
    const double p3 = q3[n3 * kTile];
    const double un = sgn * q3[((1 + ax) * L3.Np + n3) * kTile];
    const double rp = 0.5 * (p3 + Z * un);
    double rm = 0.0;
    for (int i = 0; i < P; ++i) rm += L.gamma[i] * sps[(tl * P + i) * Np + a];
    rm *= L.invM;
    const double S = rp + rm;
    qb3[(size_t)t * Np + a] = rm;
    q03[(size_t)t * Np + a] = S;
    for (int i = 0; i < P; ++i)
      q2n[((size_t)t * P + i) * 3 * Np + a] = sps[(tl * P + i) * Np + a] + S;
  }
}

// ------------------------------------------------------------------ 1D ---
// One block per line; threads (set s, node a) then (row, node a).
__global__ void k_level1(Lvl1 L, Lvl2 L2, const double* __restrict__ q1o,
                         double* __restrict__ q1n, double* __restrict__ res1,
                         const double* __restrict__ qb1, double* __restrict__ qb2,
                         double* __restrict__ q02, const double* __restrict__ q2n, double A,
                         double B, double dt) {
  const int P = L.P, PP = P * P, Np = L.Np, l = blockIdx.x, tid = threadIdx.x;
  extern __shared__ double smem[];
  double* sq = smem;                 // PP x 2 x Np
  double* sps = sq + PP * 2 * Np;    // PP x Np
  double* srp = sps + PP * Np;       // 2P x Np
  double* sb = srp + 2 * P * Np;     // 2P x Np
  double* sS = sb + 2 * P * Np;      // 2P x Np
  for (int i = tid; i < PP * 2 * Np; i += blockDim.x) sq[i] = q1o[(size_t)l * PP * 2 * Np + i];
  const double rx = L.geo[l * 4 + 0], irho = L.geo[l * 4 + 1], Kb = L.geo[l * 4 + 2],
               Z = L.geo[l * 4 + 3];
  const int* info = L.info + l * 8;
  __syncthreads();
  const double* Dr = L.ops;
  const double* LF = L.ops + Np * Np;
  if (tid < PP * Np) {
    const int s = tid / Np, a = tid - s * Np;
    const int i = s / P, j = s - i * P;
    const double Kij = Kb / (1.0 + L.gamma[i] + L.gamma[j]);
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
        const double pP = q1o[(((size_t)l2 * PP + s) * 2) * Np + node2];
        const double wnP = n * q1o[(((size_t)l2 * PP + s) * 2 + 1) * Np + node2];
        upwind(pM, wnM, Z, pP, wnP, L.geo[l2 * 4 + 3], pF, wnF);
      } else {
        const int c = -1 - code, bc = c & 3, slot = (c >> 2) & 3, corner = c >> 4;
        double rm = 0.0;
        if (bc == 0) rm = qb1[((size_t)corner * 3 + slot) * PP + s];
        bcflux(bc, pM, wnM, Z, rm, pF, wnF);
      }
      rhs0 += LF[a * 2 + end] * fsc * Kij * (wnM - wnF);
      rhs1 += LF[a * 2 + end] * fsc * irho * (pM - pF) * n;
    }
    const size_t base = (((size_t)l * PP + s) * 2) * Np + a;
    double r = A * res1[base] + dt * rhs0;
    res1[base] = r;
    const double SA = q02[(((size_t)l * 2 + 0) * P + i) * Np + a];
    const double SB = q02[(((size_t)l * 2 + 1) * P + j) * Np + a];
    sps[s * Np + a] = sq[(s * 2) * Np + a] - L.Cji[i * P + j] * SA - L.Cij[i * P + j] * SB + B * r;
    r = A * res1[base + Np] + dt * rhs1;
    res1[base + Np] = r;
    q1n[base + Np] = sq[(s * 2 + 1) * Np + a] + B * r;
  }
  __syncthreads();
  // ---- outgoing 2D characteristics and the b vector at every line node
  if (tid < 2 * P * Np) {
    const int row = tid / Np, a = tid - row * Np;
    const int side = row / P, i = row - side * P;
    const int t = info[side], comp = info[2 + side];
    const int node = L.trinode[((size_t)l * 2 + side) * Np + a];
    const double* q = q2n + ((size_t)t * L2.P + i) * 3 * L2.Np;
    // the normal of the other face: stored sign folded into comp's sign
    const double sgn = comp > 0 ? 1.0 : -1.0;
    const int cc = comp > 0 ? comp : -comp;
    const double Zt = L2.geo[(size_t)t * 8 + 6];
    srp[row * Np + a] = 0.5 * (q[node] + Zt * sgn * q[cc * L2.Np + node]);
    double b = 0.0;
    if (side == 0)
      for (int j = 0; j < P; ++j) b += L.gamma[j] * sps[(i * P + j) * Np + a];
    else
      for (int ii = 0; ii < P; ++ii) b += L.gamma[ii] * sps[(ii * P + i) * Np + a];
    sb[row * Np + a] = b * L.invM;
  }
  __syncthreads();
  // ---- edge system r- = G r+ + H b
  if (tid < 2 * P * Np) {
    const int row = tid / Np, a = tid - row * Np;
    const int n2 = 2 * P;
    double rm = 0.0;
    for (int k = 0; k < n2; ++k) rm += L.G[row * n2 + k] * srp[k * Np + a] + L.H[row * n2 + k] * sb[k * Np + a];
    const int side = row / P, i = row - side * P;
    const size_t o = (((size_t)l * 2 + side) * P + i) * Np + a;
    qb2[o] = rm;
    const double S = srp[row * Np + a] + rm;
    q02[o] = S;
    sS[row * Np + a] = S;
  }
  __syncthreads();
  if (tid < PP * Np) {
    const int s = tid / Np, a = tid - s * Np;
    const int i = s / P, j = s - i * P;
    q1n[(((size_t)l * PP + s) * 2) * Np + a] =
        sps[s * Np + a] + L.Cji[i * P + j] * sS[i * Np + a] + L.Cij[i * P + j] * sS[(P + j) * Np + a];
  }
}

// ------------------------------------------------------------------ 0D ---
__global__ void k_level0(Lvl0 L, Lvl1 L1, const double* __restrict__ q1n,
                         double* __restrict__ qb1) {
  const int P = L.P, PP = P * P, n3 = 3 * PP, c = blockIdx.x, tid = threadIdx.x;
  extern __shared__ double smem[];  // n3
  if (tid < n3) {
    const int slot = tid / PP, s = tid - slot * PP;
    const int l = L.info[(c * 3 + slot) * 2], end = L.info[(c * 3 + slot) * 2 + 1];
    const int node = end ? L1.Np - 1 : 0;
    const double* q = q1n + (((size_t)l * PP + s) * 2) * L1.Np;
    const double Z = L1.geo[l * 4 + 3];
    smem[tid] = 0.5 * (q[node] + Z * L.nrm[c * 3 + slot] * q[L1.Np + node]);
  }
  __syncthreads();
  if (tid < n3) {
    double rm = 0.0;
    for (int k = 0; k < n3; ++k) rm += L.T[(size_t)tid * n3 + k] * smem[k];
    qb1[(size_t)c * n3 + tid] = rm;
  }
}

// -------------------------------------------------------------- energy ---
// One block per tile; partial sum of J/2 (p M p / (rho c^2) + rho u M u).
__global__ void k_energy(Lvl3 L, const double* __restrict__ q, const double* __restrict__ mass,
                         const double* __restrict__ J, double* __restrict__ out) {
  const int Np = L.Np, tile = blockIdx.x, tid = threadIdx.x, es = tid & 15, g = tid >> 4;
  const int e = tile * kTile + es;
  __shared__ double red[256];
  double acc = 0.0;
  if (e < L.K) {
    const double* qt = q + (size_t)tile * 4 * Np * kTile + es;
    const double* gt = L.geo + (size_t)tile * 12 * kTile + es;
    const double irho = gt[9 * kTile], Kb = gt[10 * kTile];
    const double rho = 1.0 / irho;
    for (int a = g; a < Np; a += 16) {
      double mq[4] = {0, 0, 0, 0};
      for (int b = 0; b < Np; ++b) {
        const double m = mass[a * Np + b];
        for (int f = 0; f < 4; ++f) mq[f] += m * qt[(f * Np + b) * kTile];
      }
      acc += qt[a * kTile] * mq[0] / Kb +
             rho * (qt[(Np + a) * kTile] * mq[1] + qt[(2 * Np + a) * kTile] * mq[2] +
                    qt[(3 * Np + a) * kTile] * mq[3]);
    }
    acc *= 0.5 * J[e];
  }
  red[tid] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) out[tile] = red[0];
}

template <int N>
hipError_t launch3(const Lvl3& L, const double* qo, double* qn, double* res, const double* qb3,
                   double A, double B, double dt, int src_e, const double* src_w, double src_s,
                   hipStream_t st) {
  constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  constexpr int Nfp = (N + 1) * (N + 2) / 2;
  constexpr bool kOpsLds = (3 * Np * Np + Np * 4 * Nfp) * 8 <= 64 * 1024;
  const size_t lds = sizeof(double) * (4 * Np * kTile + 2 * 4 * Nfp * kTile +
                                       (kOpsLds ? 3 * Np * Np + Np * 4 * Nfp : 0));
  static bool attr = false;
  if (!attr) {
    hipFuncSetAttribute((const void*)k_level3<N>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    attr = true;
  }
  hipLaunchKernelGGL(k_level3<N>, dim3(L.ntile), dim3(256), lds, st, L, qo, qn, res, qb3, A, B,
                     dt, src_e, src_w, src_s);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_level3(const Lvl3& L, const double* qo, double* qn, double* res,
                         const double* qb3, double A, double B, double dt, int src_e,
                         const double* src_w, double src_s, hipStream_t st) {
  switch (L.N) {
    case 1: return launch3<1>(L, qo, qn, res, qb3, A, B, dt, src_e, src_w, src_s, st);
    case 2: return launch3<2>(L, qo, qn, res, qb3, A, B, dt, src_e, src_w, src_s, st);
    case 3: return launch3<3>(L, qo, qn, res, qb3, A, B, dt, src_e, src_w, src_s, st);
    case 4: return launch3<4>(L, qo, qn, res, qb3, A, B, dt, src_e, src_w, src_s, st);
    case 5: return launch3<5>(L, qo, qn, res, qb3, A, B, dt, src_e, src_w, src_s, st);
    case 6: return launch3<6>(L, qo, qn, res, qb3, A, B, dt, src_e, src_w, src_s, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_level2(const Lvl2& L, const Lvl3& L3, const double* q2o, double* q2n,
                         double* res2, const double* qb2, double* qb3, double* q03,
                         const double* q3n, double A, double B, double dt, hipStream_t st) {
  if (L.Kt == 0) return hipSuccess;
  const int NS = L.Np > 3 * L.Nfp ? L.Np : 3 * L.Nfp;
  int TPB = 256 / NS;
  if (TPB < 1) TPB = 1;
  const int threads = ((TPB * NS + 63) / 64) * 64;
  const int NE = 3 * L.Nfp;
  const size_t lds = sizeof(double) * (2 * L.Np * L.Np + L.Np * NE + TPB * L.P * 3 * L.Np +
                                       TPB * 2 * NE + TPB * L.P * L.Np);
  static size_t attr = 0;
  if (lds > attr) {
    hipFuncSetAttribute((const void*)k_level2, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    attr = lds;
  }
  const int blocks = (L.Kt + TPB - 1) / TPB;
  hipLaunchKernelGGL(k_level2, dim3(blocks), dim3(threads), lds, st, L, L3, q2o, q2n, res2, qb2,
                     qb3, q03, q3n, A, B, dt, TPB, NS);
  return hipGetLastError();
}

hipError_t launch_level1(const Lvl1& L, const Lvl2& L2, const double* q1o, double* q1n,
                         double* res1, const double* qb1, double* qb2, double* q02,
                         const double* q2n, double A, double B, double dt, hipStream_t st) {
  if (L.Kl == 0 || L.P == 0) return hipSuccess;
  const int PP = L.P * L.P;
  int need = PP * L.Np;
  if (2 * L.P * L.Np > need) need = 2 * L.P * L.Np;
  const int threads = ((need + 63) / 64) * 64;
  const size_t lds = sizeof(double) * (PP * 2 * L.Np + PP * L.Np + 3 * 2 * L.P * L.Np);
  hipLaunchKernelGGL(k_level1, dim3(L.Kl), dim3(threads), lds, st, L, L2, q1o, q1n, res1, qb1,
                     qb2, q02, q2n, A, B, dt);
  return hipGetLastError();
}

hipError_t launch_level0(const Lvl0& L, const Lvl1& L1, const double* q1n, double* qb1,
                         hipStream_t st) {
  if (L.Kp == 0 || L.P == 0) return hipSuccess;
  const int n3 = 3 * L.P * L.P;
  const int threads = ((n3 + 63) / 64) * 64;
  hipLaunchKernelGGL(k_level0, dim3(L.Kp), dim3(threads), sizeof(double) * n3, st, L, L1, q1n,
                     qb1);
  return hipGetLastError();
}

hipError_t launch_energy(const Lvl3& L, const double* q, const double* mass, const double* J,
                         double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_energy, dim3(L.ntile), dim3(256), 0, st, L, q, mass, J, out);
  return hipGetLastError();
}

}  // namespace dgh
