// Learned boundary closure: a small MLP that maps the recent history of the
// traces at an absorbing-face node to the incoming characteristic r- the 3D
// flux needs there (the quantity the order-P auxiliary recursion of
// Sections 2-3 produces), with hand-written training kernels.
//
// Inputs: p and Z |u_t| (u_t the velocity tangential to the face) at the
// node now, and the root mean squares of p and of Z |u_t| over the recent
// past at four time scales tau_1..tau_4 (exponential averages of their
// squares, updated at every step end with the weight 1 - exp(-dt/tau_k) of
// the new value), 10 values, divided by their own root mean square (a
// linear boundary's reflection gain does not depend on the amplitude) and
// times in_scale.  For a plane wave, p and Z |u_t| carry the same factor
// whatever part of it the boundary reflects, so their ratio (sin of the
// incidence angle) does not feed back on the closure's own output, and the
// averages over a fixed physical time keep that ratio where p itself
// passes through zero; Z n.u is left out on purpose, as it would let the
// network copy the interior's incoming characteristic, a map that in the
// continuum imposes no condition at all.
// Network (FP32): 10 -> 64 -> 64 -> 64 (tanh) -> y, and r- = g_max tanh(y)
// r+ with r+ = (p + Z n.u)/2 the current outgoing characteristic.  The
// network thus picks a reflection gain in (-g_max, g_max); with g_max <= 1
// every node has |r-| <= |r+|, so the boundary never feeds energy back into
// the domain whatever the weights (the energy flux through a face with the
// upwind flux goes as r+^2 - r-^2).
// Parameters, flat: in_scale, g_max, W1[64][10], b1[64], W2[64][64], b2[64],
// W3[64][64], b3[64], W4[64], b4 (9091 floats; the first two are fixed, the
// rest trained with Adam on the mean squared error of r-).  A sample row
// holds the 10 raw inputs and r+ (11 floats).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "kernels.hpp"
#include "launch.hpp"
#include "levels.hpp"

namespace dgh {

namespace {

constexpr int kH = 64;              // hidden width
constexpr int kIn = 10;             // inputs
constexpr int kRow = kIn + 1;       // sample row: the raw inputs, then r+
constexpr int oW1 = 2, ob1 = oW1 + kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH,
              oW3 = ob2 + kH, ob3 = oW3 + kH * kH, oW4 = ob3 + kH, ob4 = oW4 + kH;
constexpr int kNW = ob4 + 1;        // 9091
constexpr int kThreads = 256;
// memory per node: p, Z |u_t| at the last step end, then the averages of
// p^2 and (Z |u_t|)^2 at the four time scales
constexpr int kHist = 10;
static_assert(kHist == kIn, "one input per memory value");
static_assert(kHist == 2 + 2 * kMemScales, "memory layout");

// Updates a node's memory h[kHist] with the traces p, zut of a step end
// and writes the inputs f[kIn]: p, zut and the square roots of the averages.
__device__ __forceinline__ void memory_update(float* h, float p, float zut, const Memory& mem,
                                              float* f) {
  h[0] = p;
  h[1] = zut;
  f[0] = p;
  f[1] = zut;
#pragma unroll
  for (int k = 0; k < kMemScales; ++k) {
    const float a = mem.decay[k];
    h[2 + 2 * k] = a * h[2 + 2 * k] + (1.f - a) * p * p;
    h[3 + 2 * k] = a * h[3 + 2 * k] + (1.f - a) * zut * zut;
    f[2 + 2 * k] = sqrtf(h[2 + 2 * k]);
    f[3 + 2 * k] = sqrtf(h[3 + 2 * k]);
  }
}
static_assert(kNW == kMlpParams, "parameter layout");

// 1 / root mean square of the raw inputs (0 inputs stay 0)
__device__ __forceinline__ float input_inv_rms(const float* xin) {
  float q = 0.f;
#pragma unroll
  for (int k = 0; k < kIn; ++k) q += xin[k] * xin[k];
  return 1.0f / sqrtf(q * (1.0f / kIn) + 1e-30f);
}

// forward of one sample; h receives the three hidden layers if non-null
__device__ __forceinline__ float mlp_eval(const float* __restrict__ w, const float* xin,
                                          float inv, float* __restrict__ hout, int hstride) {
  float x[kIn];
#pragma unroll
  for (int k = 0; k < kIn; ++k) x[k] = w[0] * inv * xin[k];
  float a[kH], b[kH];
#pragma unroll
  for (int i = 0; i < kH; ++i) {
    float s = w[ob1 + i];
#pragma unroll
    for (int k = 0; k < kIn; ++k) s += w[oW1 + i * kIn + k] * x[k];
    a[i] = tanhf(s);
    if (hout) hout[i * hstride] = a[i];
  }
#pragma unroll
  for (int i = 0; i < kH; ++i) {
    float s = w[ob2 + i];
#pragma unroll
    for (int k = 0; k < kH; ++k) s += w[oW2 + i * kH + k] * a[k];
    b[i] = tanhf(s);
    if (hout) hout[(kH + i) * hstride] = b[i];
  }
#pragma unroll
  for (int i = 0; i < kH; ++i) {
    float s = w[ob3 + i];
#pragma unroll
    for (int k = 0; k < kH; ++k) s += w[oW3 + i * kH + k] * b[k];
    a[i] = tanhf(s);
    if (hout) hout[(2 * kH + i) * hstride] = a[i];
  }
  float y = w[ob4];
#pragma unroll
  for (int k = 0; k < kH; ++k) y += w[oW4 + k] * a[k];
  return y;
}

// Forward over n sample rows X[n][11]: Y[n] = r-; H (if non-null) gets the
// hidden layers column-major, H[l][s] for l < 192, Th[s] = tanh(y) and
// Inv[s] = 1 / rms of the raw inputs.
__global__ void __launch_bounds__(kThreads) k_mlp_fwd(const float* __restrict__ W,
                                                      const float* __restrict__ X, int n,
                                                      float* __restrict__ H,
                                                      float* __restrict__ Th,
                                                      float* __restrict__ Inv,
                                                      float* __restrict__ Y) {
  __shared__ float w[kNW];
  for (int i = threadIdx.x; i < kNW; i += blockDim.x) w[i] = W[i];
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float x[kIn];
#pragma unroll
  for (int k = 0; k < kIn; ++k) x[k] = X[(size_t)s * kRow + k];
  const float inv = input_inv_rms(x);
  const float th = tanhf(mlp_eval(w, x, inv, H ? H + s : nullptr, n));
  if (H) {
    Th[s] = th;
    Inv[s] = inv;
  }
  Y[s] = w[1] * th * X[(size_t)s * kRow + kIn];
}

// Backward through the activations of one batch: with the loss
// L = (1/n) sum_s (Y_s - T_s)^2, dY = dL/dy (y the output layer's value)
// and dH[l][s] = dL/d(pre-activation of hidden unit l).  lossp[block] gets
// the block's partial sum of squared errors.
__global__ void __launch_bounds__(kThreads) k_mlp_bwd(const float* __restrict__ W,
                                                      const float* __restrict__ X,
                                                      const float* __restrict__ T, int n,
                                                      const float* __restrict__ H,
                                                      const float* __restrict__ Th,
                                                      const float* __restrict__ Y,
                                                      float* __restrict__ dY,
                                                      float* __restrict__ dH,
                                                      float* __restrict__ lossp) {
  __shared__ float w[kNW];
  __shared__ float red[kThreads];
  for (int i = threadIdx.x; i < kNW; i += blockDim.x) w[i] = W[i];
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  float sq = 0.f;
  if (s < n) {
    const float e = Y[s] - T[s];
    sq = e * e;
    const float th = Th[s];
    const float rp = X[(size_t)s * kRow + kIn];
    const float dy = 2.f * e / (float)n * w[1] * rp * (1.f - th * th);
    dY[s] = dy;
    float g3[kH], g2[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
      const float h = H[(size_t)(2 * kH + j) * n + s];
      g3[j] = w[oW4 + j] * dy * (1.f - h * h);
      dH[(size_t)(2 * kH + j) * n + s] = g3[j];
    }
#pragma unroll
    for (int i = 0; i < kH; ++i) {
      float acc = 0.f;
#pragma unroll
      for (int j = 0; j < kH; ++j) acc += w[oW3 + j * kH + i] * g3[j];
      const float h = H[(size_t)(kH + i) * n + s];
      g2[i] = acc * (1.f - h * h);
      dH[(size_t)(kH + i) * n + s] = g2[i];
    }
#pragma unroll
    for (int i = 0; i < kH; ++i) {
      float acc = 0.f;
#pragma unroll
      for (int j = 0; j < kH; ++j) acc += w[oW2 + j * kH + i] * g2[j];
      const float h = H[(size_t)i * n + s];
      dH[(size_t)i * n + s] = acc * (1.f - h * h);
    }
  }
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int k = kThreads / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) lossp[blockIdx.x] = red[0];
}

// Parameter gradients: one thread per parameter, summed over the batch
// (dW = dH^T * previous layer, db = sum dH).  G[0], G[1] (scales) = 0.
__global__ void __launch_bounds__(kThreads) k_mlp_wgrad(const float* __restrict__ W,
                                                        const float* __restrict__ X, int n,
                                                        const float* __restrict__ H,
                                                        const float* __restrict__ Inv,
                                                        const float* __restrict__ dY,
                                                        const float* __restrict__ dH,
                                                        float* __restrict__ G) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNW) return;
  const float sin_ = W[0];
  float acc = 0.f;
  if (p < oW1) {
    acc = 0.f;
  } else if (p < ob1) {                       // W1[i][k]: dH1[i] x[k] in_scale / rms
    const int i = (p - oW1) / kIn, k = (p - oW1) % kIn;
    for (int s = 0; s < n; ++s)
      acc += dH[(size_t)i * n + s] * (X[(size_t)s * kRow + k] * Inv[s]);
    acc *= sin_;
  } else if (p < oW2) {                       // b1
    const int i = p - ob1;
    for (int s = 0; s < n; ++s) acc += dH[(size_t)i * n + s];
  } else if (p < ob2) {                       // W2[i][k]: dH2[i] h1[k]
    const int i = (p - oW2) / kH, k = (p - oW2) % kH;
    for (int s = 0; s < n; ++s) acc += dH[(size_t)(kH + i) * n + s] * H[(size_t)k * n + s];
  } else if (p < oW3) {                       // b2
    const int i = p - ob2;
    for (int s = 0; s < n; ++s) acc += dH[(size_t)(kH + i) * n + s];
  } else if (p < ob3) {                       // W3[i][k]: dH3[i] h2[k]
    const int i = (p - oW3) / kH, k = (p - oW3) % kH;
    for (int s = 0; s < n; ++s)
      acc += dH[(size_t)(2 * kH + i) * n + s] * H[(size_t)(kH + k) * n + s];
  } else if (p < oW4) {                       // b3
    const int i = p - ob3;
    for (int s = 0; s < n; ++s) acc += dH[(size_t)(2 * kH + i) * n + s];
  } else if (p < ob4) {                       // W4[k]: dY h3[k]
    const int k = p - oW4;
    for (int s = 0; s < n; ++s) acc += dY[s] * H[(size_t)(2 * kH + k) * n + s];
  } else {                                    // b4
    for (int s = 0; s < n; ++s) acc += dY[s];
  }
  G[p] = acc;
}

// Adam (Kingma & Ba) on the trained parameters (index >= 2), step t >= 1.
__global__ void k_adam(float* __restrict__ W, const float* __restrict__ G, float* __restrict__ M,
                       float* __restrict__ V, int t, float lr, float b1, float b2, float eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < oW1 || p >= kNW) return;
  const float g = G[p];
  const float m = b1 * M[p] + (1.f - b1) * g;
  const float v = b2 * V[p] + (1.f - b2) * g * g;
  M[p] = m;
  V[p] = v;
  const float mh = m / (1.f - powf(b1, (float)t)), vh = v / (1.f - powf(b2, (float)t));
  W[p] -= lr * mh / (sqrtf(vh) + eps);
}

// Traces of the new 3D state at triangle node (t, a): p, Z n.u and Z |u_t|
// (the face normal is the axis ax with sign sgn).
template <class T3>
__device__ __forceinline__ void node_trace(const Lvl2& L2, const T3* __restrict__ q3, int np3,
                                           int t, int a, float& p, float& zun, float& zut) {
  const int* inf = L2.info + (size_t)t * 8;
  const int e3 = inf[0], ax = inf[1], sgn = inf[2];
  const int n3 = L2.tetnode[(size_t)t * L2.Np + a];
  const T3* q = q3 + (size_t)(e3 >> 4) * 4 * np3 * kTile + (e3 & 15);
  const double Z = L2.geo[(size_t)t * 8 + 6];
  const double un = (double)q[((1 + ax) * np3 + n3) * kTile];
  const double ua = (double)q[((1 + (ax + 1) % 3) * np3 + n3) * kTile];
  const double ub = (double)q[((1 + (ax + 2) % 3) * np3 + n3) * kTile];
  p = (float)q[n3 * kTile];
  zun = (float)(Z * (double)sgn * un);
  zut = (float)(Z * sqrt(ua * ua + ub * ub));
}

// End of a step with the closure on: the history moves one step back and
// takes the current traces first (as k_hist_push), then r- at every
// absorbing-face node comes from the current traces and the 4 step ends
// before them -> qb3, which every stage of the next step reads; q0_3 =
// r+ + r- (kept for symmetry with the face rule).  The inputs are those
// k_closure_sample records after a step of the plain method.
//
// The network runs on the FP32 16x16x4 MFMA, 16 nodes per wave: a layer is
// H_out[64][16] = W[64][K] H_in[K][16] with the weights as A fragments (lane
// l: W[16 rb + l%16][4 ks + l/16], arranged in LDS in that order, in_scale
// folded into W1) and the activations as B fragments (lane l: H_in[4 ks +
// l/16][node l%16]).  The accumulator rows a lane holds (16 rb + 4 (l/16) +
// r) are not the B rows of the next layer, so each hidden layer goes
// through a per-wave LDS tile [64][16] between layers.  The output row W4
// is a dot product: partial sums over a lane's 16 rows, then across the 4
// lane groups of a node.
typedef float cf4 __attribute__((ext_vector_type(4)));
constexpr int kCW = 4;                       // waves per workgroup
constexpr int kA1 = 4 * 3 * 64;              // W1 fragments (K = 10 padded to 12)
constexpr int kA2 = 4 * 16 * 64;             // W2 (and W3) fragments
constexpr int kCF = kA1 + 2 * kA2 + 4 * kH + 2;   // + b1, b2, b3, W4, b4, g_max

__device__ __forceinline__ cf4 mfma_c(float a, float b, cf4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <class T3>
__global__ void __launch_bounds__(kCW * 64) k_closure(Lvl2 L2, const float* __restrict__ W,
                                                      const T3* __restrict__ q3, int np3,
                                                      float* __restrict__ hist,
                                                      double* __restrict__ qb3,
                                                      double* __restrict__ q03, Shots sh,
                                                      Memory mem) {
  __shared__ float cw[kCF];
  __shared__ float tl[kCW][kH * 16];        // per wave: a hidden layer, [row][node]
  // weights in fragment order
  for (int i = threadIdx.x; i < kA1; i += blockDim.x) {
    const int rb = i / 192, ks = (i / 64) % 3, l = i & 63;
    const int row = 16 * rb + (l & 15), col = 4 * ks + (l >> 4);
    cw[i] = col < kIn ? W[0] * W[oW1 + row * kIn + col] : 0.f;
  }
  for (int i = threadIdx.x; i < kA2; i += blockDim.x) {
    const int rb = i / 1024, ks = (i / 64) % 16, l = i & 63;
    const int rc = (16 * rb + (l & 15)) * kH + 4 * ks + (l >> 4);
    cw[kA1 + i] = W[oW2 + rc];
    cw[kA1 + kA2 + i] = W[oW3 + rc];
  }
  float* cb1 = cw + kA1 + 2 * kA2;
  float* cb2 = cb1 + kH;
  float* cb3 = cb2 + kH;
  float* cw4 = cb3 + kH;
  for (int i = threadIdx.x; i < kH; i += blockDim.x) {
    cb1[i] = W[ob1 + i];
    cb2[i] = W[ob2 + i];
    cb3[i] = W[ob3 + i];
    cw4[i] = W[oW4 + i];
  }
  if (threadIdx.x == 0) {
    cw4[kH] = W[ob4];
    cw4[kH + 1] = W[1];
  }
  __syncthreads();
  const size_t k = blockIdx.y;
  q3 += k * sh.st3;
  qb3 += k * sh.stb3;
  q03 += k * sh.stb3;
  const int nn = L2.Kt * L2.Np;
  hist += k * (size_t)nn * kHist;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, q = lane >> 4, nd = lane & 15;
  // persistent: the workgroup staged the weights once; its waves walk the
  // 16-node tiles
  for (int x0 = (blockIdx.x * kCW + wv) * 16; x0 < nn; x0 += gridDim.x * kCW * 16) {
  const int x = x0 + nd;                     // this lane's node
  const bool valid = x < nn;
  const int xc = valid ? x : nn - 1;
  const int t = xc / L2.Np, a = xc - t * L2.Np;
  float f[kIn], h[kHist], p, zun, zut;
  node_trace(L2, q3, np3, t, a, p, zun, zut);
#pragma unroll
  for (int j = 0; j < kHist; ++j) h[j] = hist[(size_t)xc * kHist + j];
  memory_update(h, p, zut, mem, f);
  if (valid && q == 0) {
    float* o = hist + (size_t)x * kHist;
#pragma unroll
    for (int j = 0; j < kHist; ++j) o[j] = h[j];
  }
  const float inv = input_inv_rms(f);
  float* T = tl[wv];
  const float* A1 = cw + lane;
  const float* A2 = cw + kA1 + lane;
  const float* A3 = cw + kA1 + kA2 + lane;
  // layer 1: B = the lane group's inputs (feature 4 ks + q of node nd)
  cf4 acc[4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) acc[rb] = cf4{0, 0, 0, 0};
#pragma unroll
  for (int ks = 0; ks < 3; ++ks) {
    const int c0 = 4 * ks;
    float v = q == 0 ? f[c0] : (q == 1 ? f[c0 + 1] : 0.f);
    if (c0 + 2 < kIn && q == 2) v = f[c0 + 2];
    if (c0 + 3 < kIn && q == 3) v = f[c0 + 3];
    v *= inv;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[rb] = mfma_c(A1[(rb * 3 + ks) * 64], v, acc[rb]);
  }
  // hidden layers 2 and 3 through the LDS tile
#pragma unroll
  for (int layer = 0; layer < 2; ++layer) {
    const float* bias = layer == 0 ? cb1 : cb2;
    const float* A = layer == 0 ? A2 : A3;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * rb + 4 * q + r;
        T[row * 16 + nd] = tanhf(acc[rb][r] + bias[row]);
      }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[rb] = cf4{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      const float v = T[(4 * ks + q) * 16 + nd];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) acc[rb] = mfma_c(A[(rb * 16 + ks) * 64], v, acc[rb]);
    }
  }
  // output: y = W4 . tanh(acc + b3) + b4, summed over the node's 4 lane groups
  float y = 0.f;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * rb + 4 * q + r;
      y += cw4[row] * tanhf(acc[rb][r] + cb3[row]);
    }
  y += __shfl_xor(y, 16, 64);
  y += __shfl_xor(y, 32, 64);
  y += cw4[kH];
  if (valid && q == 0) {
    const float rpf = 0.5f * (f[0] + zun);
    const double rm = (double)(cw4[kH + 1] * tanhf(y) * rpf);
    qb3[x] = rm;
    q03[x] = (double)rpf + rm;
  }
  }
}

// End of a step: every node's memory takes the current traces (as
// k_closure does before it evaluates the network).
template <class T3>
__global__ void __launch_bounds__(kThreads) k_hist_push(Lvl2 L2, const T3* __restrict__ q3,
                                                        int np3, float* __restrict__ hist,
                                                        Shots sh, Memory mem) {
  const size_t k = blockIdx.y;
  q3 += k * sh.st3;
  const int nn = L2.Kt * L2.Np;
  hist += k * (size_t)nn * kHist;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nn) return;
  const int t = x / L2.Np, a = x - t * L2.Np;
  float p, zun, zut;
  node_trace(L2, q3, np3, t, a, p, zun, zut);
  float h[kHist], f[kIn];
#pragma unroll
  for (int j = 0; j < kHist; ++j) h[j] = hist[(size_t)x * kHist + j];
  memory_update(h, p, zut, mem, f);
  float* o = hist + (size_t)x * kHist;
#pragma unroll
  for (int j = 0; j < kHist; ++j) o[j] = h[j];
}

// Training samples of one shot, taken after a step end (whose traces the
// memory already holds): X[node][11] = the raw inputs (the current p,
// Z |u_t| and the root mean squares at the four time scales) and r+,
// Y[node] = the current qb3 -- the r- the face rule produced at the step's
// last stage.
template <class T3>
__global__ void __launch_bounds__(kThreads) k_closure_sample(Lvl2 L2, const T3* __restrict__ q3,
                                                             int np3, const float* __restrict__ hist,
                                                             const double* __restrict__ qb3,
                                                             float* __restrict__ X,
                                                             float* __restrict__ Y) {
  const int nn = L2.Kt * L2.Np;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nn) return;
  const int t = x / L2.Np, a = x - t * L2.Np;
  float p, zun, zut;
  node_trace(L2, q3, np3, t, a, p, zun, zut);
  float* r = X + (size_t)x * kRow;
  r[0] = p;
  r[1] = zut;
#pragma unroll
  for (int j = 0; j < 8; ++j) r[2 + j] = sqrtf(hist[(size_t)x * kHist + 2 + j]);
  r[kIn] = 0.5f * (p + zun);
  Y[x] = (float)qb3[x];
}

// ---- BF16 training step on the MFMA (FP32 master weights) ----
// One workgroup of four waves takes 64 samples, a wave 16 of them as the
// columns of the BF16 16x16x16 instruction (lane l: A[l%16][4(l/16) + i],
// B[4(l/16) + i][l%16], accumulator rows 4(l/16) + r of column l%16).  The
// weights enter as BF16 A fragments (W for the forward pass, W^T for the
// backward one), the activations and their gradients as BF16 B fragments,
// every sum in FP32.  A layer's accumulator rows 16 b + 4(l/16) + r are the
// B rows 16 ks + 4(l/16) + i of the next layer's k-step ks = b, so the
// forward and backward passes stay in registers; the weight gradients
// (sums over the samples) take the activations and gradients of a wave
// through an LDS tile, as A = dH [unit][sample] and B = H [sample][unit].
// The four waves' sums are added in a fixed order in LDS and each
// workgroup writes its partial gradient; k_mlp_grad_reduce adds the
// partials of all workgroups in a fixed order (no atomics).
typedef short bs4 __attribute__((ext_vector_type(4)));

// four FP32 -> BF16, round to nearest even: two v_cvt_pk_bf16_f32
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float fl2 __attribute__((ext_vector_type(2)));
typedef unsigned u2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ bs4 bpack(float a, float b, float c, float d) {
  const bf2 lo = __builtin_convertvector(fl2{a, b}, bf2);
  const bf2 hi = __builtin_convertvector(fl2{c, d}, bf2);
  return __builtin_bit_cast(bs4,
                            u2{__builtin_bit_cast(unsigned, lo), __builtin_bit_cast(unsigned, hi)});
}
__device__ __forceinline__ cf4 mfma_b(bs4 a, bs4 b, cf4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

constexpr int kTW = 4;                     // waves per workgroup
constexpr int kTS = kTW * 16;              // samples per workgroup

struct TrainLds {
  bs4 w1[4][64];                           // W1 s (rows 16 rb + l%16, inputs 4 g + i)
  bs4 w2[4][4][64], w3[4][4][64];          // W [row block][k-step][lane]
  bs4 w2t[4][4][64], w3t[4][4][64];        // W^T
  float tile[kTW][2][64][17];              // per wave: a gradient and an activation [unit][sample]
  float acc[64][65];                       // the workgroup's sum of one weight matrix
  float vec[8][64];                        // sums of b1, b2, b3, W4, then b4, loss
};

__global__ void __launch_bounds__(kTW * 64) k_mlp_grad_bf16(const float* __restrict__ W,
                                                            const float* __restrict__ X,
                                                            const float* __restrict__ T, int n,
                                                            float* __restrict__ part,
                                                            float* __restrict__ lossp) {
  extern __shared__ char lds_raw[];
  TrainLds& S = *reinterpret_cast<TrainLds*>(lds_raw);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g = lane >> 4, col = lane & 15;
  const float sc = W[0], gmax = W[1];
  // weight fragments, BF16
  for (int x = tid; x < 4 * 64; x += blockDim.x) {
    const int rb = x >> 6, l = x & 63, row = 16 * rb + (l & 15);
    float v[4];
    for (int i = 0; i < 4; ++i) {
      const int k = 4 * (l >> 4) + i;
      v[i] = k < kIn ? sc * W[oW1 + row * kIn + k] : 0.f;
    }
    S.w1[rb][l] = bpack(v[0], v[1], v[2], v[3]);
  }
  for (int x = tid; x < 16 * 64; x += blockDim.x) {
    const int rb = x >> 8, ks = (x >> 6) & 3, l = x & 63;
    const int row = 16 * rb + (l & 15), k0 = 16 * ks + 4 * (l >> 4);
    const float* w2 = W + oW2;
    const float* w3 = W + oW3;
    S.w2[rb][ks][l] = bpack(w2[row * kH + k0], w2[row * kH + k0 + 1], w2[row * kH + k0 + 2],
                            w2[row * kH + k0 + 3]);
    S.w3[rb][ks][l] = bpack(w3[row * kH + k0], w3[row * kH + k0 + 1], w3[row * kH + k0 + 2],
                            w3[row * kH + k0 + 3]);
    S.w2t[rb][ks][l] = bpack(w2[k0 * kH + row], w2[(k0 + 1) * kH + row], w2[(k0 + 2) * kH + row],
                             w2[(k0 + 3) * kH + row]);
    S.w3t[rb][ks][l] = bpack(w3[k0 * kH + row], w3[(k0 + 1) * kH + row], w3[(k0 + 2) * kH + row],
                             w3[(k0 + 3) * kH + row]);
  }
  for (int x = tid; x < 8 * 64; x += blockDim.x) (&S.vec[0][0])[x] = 0.f;
  __syncthreads();
  // this lane's sample (lanes past n compute on the last one and add nothing)
  const int s = blockIdx.x * kTS + wv * 16 + col;
  const bool live = s < n;
  const int sc_ = live ? s : n - 1;
  float xin[kIn];
#pragma unroll
  for (int k = 0; k < kIn; ++k) xin[k] = X[(size_t)sc_ * kRow + k];
  const float inv = input_inv_rms(xin);
  const float rp = X[(size_t)sc_ * kRow + kIn];
  float xs[16];                              // the scaled inputs (sc folded into W1)
#pragma unroll
  for (int k = 0; k < 16; ++k) xs[k] = k < kIn ? inv * xin[k] : 0.f;
  // ---- forward
  cf4 h1[4], h2[4], h3[4];
  {
    const bs4 bx = bpack(xs[4 * g], xs[4 * g + 1], xs[4 * g + 2], xs[4 * g + 3]);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      cf4 a = mfma_b(S.w1[rb][lane], bx, cf4{0, 0, 0, 0});
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = tanhf(a[r] + W[ob1 + 16 * rb + 4 * g + r]);
      h1[rb] = a;
    }
  }
#pragma unroll
  for (int layer = 0; layer < 2; ++layer) {
    const cf4* hin = layer == 0 ? h1 : h2;
    cf4* hout = layer == 0 ? h2 : h3;
    const float* bias = W + (layer == 0 ? ob2 : ob3);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      cf4 a = cf4{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const bs4 b = bpack(hin[ks][0], hin[ks][1], hin[ks][2], hin[ks][3]);
        a = mfma_b(layer == 0 ? S.w2[rb][ks][lane] : S.w3[rb][ks][lane], b, a);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = tanhf(a[r] + bias[16 * rb + 4 * g + r]);
      hout[rb] = a;
    }
  }
  float y = 0.f;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int r = 0; r < 4; ++r) y += W[oW4 + 16 * rb + 4 * g + r] * h3[rb][r];
  y += __shfl_xor(y, 16, 64);
  y += __shfl_xor(y, 32, 64);
  y += W[ob4];
  const float th = tanhf(y);
  const float e = live ? gmax * th * rp - T[sc_] : 0.f;
  const float dy = live ? 2.f * e / (float)n * gmax * rp * (1.f - th * th) : 0.f;
  // ---- backward through the activations
  cf4 d3[4], d2[4], d1[4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      d3[rb][r] = W[oW4 + 16 * rb + 4 * g + r] * dy * (1.f - h3[rb][r] * h3[rb][r]);
#pragma unroll
  for (int layer = 0; layer < 2; ++layer) {
    const cf4* dout = layer == 0 ? d3 : d2;
    const cf4* hact = layer == 0 ? h2 : h1;
    cf4* din = layer == 0 ? d2 : d1;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      cf4 a = cf4{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const bs4 b = bpack(dout[ks][0], dout[ks][1], dout[ks][2], dout[ks][3]);
        a = mfma_b(layer == 0 ? S.w3t[rb][ks][lane] : S.w2t[rb][ks][lane], b, a);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] *= 1.f - hact[rb][r] * hact[rb][r];
      din[rb] = a;
    }
  }
  // ---- vector sums over the wave's samples: b1, b2, b3 (the gradients),
  // W4 (dy h3), b4 (dy) and the squared error; lanes of one group hold the
  // same rows for 16 samples
  auto wave_sum16 = [&](float v) {
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 8, 64);
    return v;
  };
  float bsum[4][4][4];   // [vector][rb][r]
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      bsum[0][rb][r] = wave_sum16(d1[rb][r]);
      bsum[1][rb][r] = wave_sum16(d2[rb][r]);
      bsum[2][rb][r] = wave_sum16(d3[rb][r]);
      bsum[3][rb][r] = wave_sum16(dy * h3[rb][r]);
    }
  const float dysum = wave_sum16(g == 0 ? dy : 0.f);
  const float esum = wave_sum16(g == 0 ? e * e : 0.f);
  for (int w = 0; w < kTW; ++w) {            // fixed order over the waves
    if (wv == w && col == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int r = 0; r < 4; ++r) S.vec[v][16 * rb + 4 * g + r] += bsum[v][rb][r];
      if (g == 0) {
        S.vec[4][0] += dysum;
        S.vec[5][0] += esum;
      }
    }
    __syncthreads();
  }
  // ---- weight matrices: dW = sum over samples of dH (unit) x H (unit)
  float* part_blk = part + (size_t)blockIdx.x * kNW;
  float (*Tg)[17] = S.tile[wv][0];
  float (*Th)[17] = S.tile[wv][1];
#pragma unroll 1
  for (int m = 0; m < 3; ++m) {              // W3 (d3, h2), W2 (d2, h1), W1 (d1, x)
    const cf4* dg = m == 0 ? d3 : (m == 1 ? d2 : d1);
    const cf4* ha = m == 0 ? h2 : h1;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int u = 16 * rb + 4 * g + r;
        Tg[u][col] = dg[rb][r];
        Th[u][col] = m == 2 ? (u < 16 ? xs[u] : 0.f) : ha[rb][r];
      }
    __syncthreads();
    // A[row = unit o][k = sample], B[k = sample][col = unit i]
    cf4 acc[4][4];
    const int ncb = m == 2 ? 1 : 4;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const bs4 a = bpack(Tg[16 * rb + col][4 * g], Tg[16 * rb + col][4 * g + 1],
                          Tg[16 * rb + col][4 * g + 2], Tg[16 * rb + col][4 * g + 3]);
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        if (cb >= ncb) break;
        const bs4 b = bpack(Th[16 * cb + col][4 * g], Th[16 * cb + col][4 * g + 1],
                            Th[16 * cb + col][4 * g + 2], Th[16 * cb + col][4 * g + 3]);
        acc[rb][cb] = mfma_b(a, b, cf4{0, 0, 0, 0});
      }
    }
    for (int x = tid; x < 64 * 65; x += blockDim.x) (&S.acc[0][0])[x] = 0.f;
    __syncthreads();
    for (int w = 0; w < kTW; ++w) {
      if (wv == w) {
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) {
            if (cb >= ncb) break;
#pragma unroll
            for (int r = 0; r < 4; ++r) S.acc[16 * rb + 4 * g + r][16 * cb + col] += acc[rb][cb][r];
          }
      }
      __syncthreads();
    }
    if (m == 0) {
      for (int x = tid; x < kH * kH; x += blockDim.x) part_blk[oW3 + x] = S.acc[x / kH][x % kH];
    } else if (m == 1) {
      for (int x = tid; x < kH * kH; x += blockDim.x) part_blk[oW2 + x] = S.acc[x / kH][x % kH];
    } else {
      for (int x = tid; x < kH * kIn; x += blockDim.x)
        part_blk[oW1 + x] = sc * S.acc[x / kIn][x % kIn];
    }
    __syncthreads();
  }
  for (int x = tid; x < kH; x += blockDim.x) {
    part_blk[ob1 + x] = S.vec[0][x];
    part_blk[ob2 + x] = S.vec[1][x];
    part_blk[ob3 + x] = S.vec[2][x];
    part_blk[oW4 + x] = S.vec[3][x];
  }
  if (tid == 0) {
    part_blk[ob4] = S.vec[4][0];
    part_blk[0] = part_blk[1] = 0.f;
    lossp[blockIdx.x] = S.vec[5][0];
  }
}

// G[p] = sum over the workgroups' partial gradients, in workgroup order.
__global__ void __launch_bounds__(kThreads) k_mlp_grad_reduce(const float* __restrict__ part,
                                                              int nb, float* __restrict__ G) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNW) return;
  float acc = 0.f;
  for (int b = 0; b < nb; ++b) acc += part[(size_t)b * kNW + p];
  G[p] = acc;
}

}  // namespace

// work of the FP32 step: H[192][n], dH[192][n], Y[n], dY[n], Th[n], Inv[n],
// then the loss partials; of the BF16 step: the workgroups' partial
// gradients and loss partials.  The buffer serves either.
constexpr size_t work_floats(int n) {
  const size_t f32 = (size_t)n * (2 * 3 * kH + 4) + (n + kThreads - 1) / kThreads;
  const size_t b16 = (size_t)((n + 63) / 64) * (kNW + 1);
  return f32 > b16 ? f32 : b16;
}
size_t mlp_work_floats(int n) { return work_floats(n); }

// The gradient's work buffer for callers that cannot allocate: one
// file-scope array per GPU, sized for kMlpStaticBatch samples (6.4 MB),
// held until the process ends.  Host code reaches it only through the
// address hipGetSymbolAddress returns on that device.
static_assert(kMlpStaticBatch % kThreads == 0, "static batch");
static __device__ __align__(256) float scratch[work_floats(kMlpStaticBatch)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t mlp_static_work(hipStream_t st, float** work) {
  int dev = 0;
  hipError_t e = st ? hipStreamGetDevice(st, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int prev = 0;
    e = hipGetDevice(&prev);
    if (e != hipSuccess) return e;
    if (prev != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    const hipError_t back = prev != dev ? hipSetDevice(prev) : hipSuccess;
    if (e != hipSuccess) return e;
    if (back != hipSuccess) return back;
    g_scratch_ptr[dev] = static_cast<float*>(ptr);
  }
  *work = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t mlp_forward(const float* W, const float* X, int n, float* Y, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_fwd, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, st, W, X,
                     n, nullptr, nullptr, nullptr, Y);
  return hipGetLastError();
}

hipError_t mlp_grad(const float* W, const float* X, const float* T, int n, float* G, float* work,
                    hipStream_t st) {
  if (n <= 0) return hipErrorInvalidValue;
  float* H = work;
  float* dH = H + (size_t)n * 3 * kH;
  float* Y = dH + (size_t)n * 3 * kH;
  float* dY = Y + n;
  float* Th = dY + n;
  float* Inv = Th + n;
  float* lossp = Inv + n;
  const dim3 gs((n + kThreads - 1) / kThreads), bs(kThreads);
  hipLaunchKernelGGL(k_mlp_fwd, gs, bs, 0, st, W, X, n, H, Th, Inv, Y);
  hipLaunchKernelGGL(k_mlp_bwd, gs, bs, 0, st, W, X, T, n, H, Th, Y, dY, dH, lossp);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3((kNW + kThreads - 1) / kThreads), bs, 0, st, W, X, n, H, Inv,
                     dY, dH, G);
  return hipGetLastError();
}

hipError_t mlp_adam(float* W, const float* G, float* M, float* V, int t, float lr, float b1,
                    float b2, float eps, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((kNW + kThreads - 1) / kThreads), dim3(kThreads), 0, st, W, G, M,
                     V, t, lr, b1, b2, eps);
  return hipGetLastError();
}

// BF16 training step: the workgroups' partial gradients [nb][kNW], then
// the loss partials [nb], at the start of the work buffer (nb = n / 64
// rounded up; fewer floats than the FP32 step's work for any n >= 1).
hipError_t mlp_grad_bf16(const float* W, const float* X, const float* T, int n, float* G,
                         float* work, hipStream_t st) {
  if (n <= 0) return hipErrorInvalidValue;
  const int nb = (n + kTS - 1) / kTS;
  static_assert(kTS == 64, "work_floats counts 64 samples per workgroup");
  float* part = work;
  float* lossp = work + (size_t)nb * kNW;
  const size_t lds = sizeof(TrainLds);
  static_assert(sizeof(TrainLds) <= 160 * 1024, "LDS");
  hipError_t e = kernel_setup((const void*)k_mlp_grad_bf16, kTW * 64, lds, nullptr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_grad_bf16, dim3(nb), dim3(kTW * 64), lds, st, W, X, T, n, part, lossp);
  hipLaunchKernelGGL(k_mlp_grad_reduce, dim3((kNW + kThreads - 1) / kThreads), dim3(kThreads), 0,
                     st, part, nb, G);
  return hipGetLastError();
}

const float* mlp_loss_partials_bf16(const float* work, int n) {
  return work + (size_t)((n + kTS - 1) / kTS) * kNW;
}

const float* mlp_loss_partials(const float* work, int n) {
  return work + (size_t)n * (2 * 3 * kH + 4);
}

hipError_t launch_closure(const Lvl2& L2, const float* W, const void* q3, int q3f32, int np3,
                          float* hist, double* qb3, double* q03, const Shots& sh,
                          const Memory& mem, hipStream_t st) {
  const int nn = L2.Kt * L2.Np;
  if (nn == 0) return hipSuccess;
  const int tiles = (nn + 15) / 16;
  // persistent over the tiles of each shot: about 3 workgroups per CU in all
  int cus = 0;
  {
    const hipError_t e = device_cus(&cus);
    if (e != hipSuccess) return e;
  }
  const int per_shot = std::max(1, 3 * cus / std::max(1, sh.n));
  const dim3 g(std::min((tiles + kCW - 1) / kCW, per_shot), sh.n), b(kCW * 64);
  if (q3f32)
    hipLaunchKernelGGL(k_closure<float>, g, b, 0, st, L2, W, static_cast<const float*>(q3), np3,
                       hist, qb3, q03, sh, mem);
  else
    hipLaunchKernelGGL(k_closure<double>, g, b, 0, st, L2, W, static_cast<const double*>(q3), np3,
                       hist, qb3, q03, sh, mem);
  return hipGetLastError();
}

hipError_t launch_hist_push(const Lvl2& L2, const void* q3, int q3f32, int np3, float* hist,
                            const Shots& sh, const Memory& mem, hipStream_t st) {
  const int nn = L2.Kt * L2.Np;
  if (nn == 0) return hipSuccess;
  const dim3 g((nn + kThreads - 1) / kThreads, sh.n), b(kThreads);
  if (q3f32)
    hipLaunchKernelGGL(k_hist_push<float>, g, b, 0, st, L2, static_cast<const float*>(q3), np3,
                       hist, sh, mem);
  else
    hipLaunchKernelGGL(k_hist_push<double>, g, b, 0, st, L2, static_cast<const double*>(q3), np3,
                       hist, sh, mem);
  return hipGetLastError();
}

hipError_t launch_closure_sample(const Lvl2& L2, const void* q3, int q3f32, int np3,
                                 const float* hist, const double* qb3, float* X, float* Y,
                                 hipStream_t st) {
  const int nn = L2.Kt * L2.Np;
  if (nn == 0) return hipSuccess;
  const dim3 g((nn + kThreads - 1) / kThreads), b(kThreads);
  if (q3f32)
    hipLaunchKernelGGL(k_closure_sample<float>, g, b, 0, st, L2, static_cast<const float*>(q3),
                       np3, hist, qb3, X, Y);
  else
    hipLaunchKernelGGL(k_closure_sample<double>, g, b, 0, st, L2, static_cast<const double*>(q3),
                       np3, hist, qb3, X, Y);
  return hipGetLastError();
}

}  // namespace dgh
