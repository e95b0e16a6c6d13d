// lbm_closure.hip -- the learned boundary closure (include/lbm_closure.h):
// training-sample gathering on lattices and ensembles, and the network
// trainer (fused forward + backward per 64-row tile on BF16 MFMA with FP32
// accumulation, deterministic gradient reduction, Adam on FP32 masters).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstring>
#include <vector>

#include "lbm.h"
#include "lbm_closure.h"
#include "lbm_device.h"
#include "lbm_host.h"
#include "lbm_launch.h"
#include "lbm_mlp.h"
#include "lbm_sweep.h"

namespace lbm {

using mlp::bf16;
using mlp::bf16x8;
using mlp::f32x4;

// ------------------------------------------------------------------ sampling
__device__ inline void edge_normal(int edge, int& nx_, int& ny_) {
  nx_ = edge == E_LEFT ? -1 : (edge == E_RIGHT ? 1 : 0);
  ny_ = edge == E_BOTTOM ? -1 : (edge == E_TOP ? 1 : 0);
}

template <int S>
__device__ inline void load_node(const LatDesc& L, int parity, int x, int y, typename Codec<S>::R g[9]) {
  using C = Codec<S>;
  const typename C::T* A = static_cast<const typename C::T*>(buf_of(L, parity));
  const int idx = y * L.pitch + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) g[i] = C::dec(A[i * L.plane + idx], L.ds[i]);
}

template <int S>
__device__ void site_features_body(const LatDesc& L, int parity, int x, int y, int edge, float* feat, float* mc) {
  using R = typename Codec<S>::R;
  int enx, eny;
  edge_normal(edge, enx, eny);
  const R rho0 = R(L.rho0);
  const Base<R> base(L);
  const R ref[3] = {R(L.m0[0]), R(L.m0[1]), R(L.m0[2])};
  R mom[3][3];  // depth 0..2 at k = 0
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int k = -1; k <= 1; ++k) {
      const int sx = x - d * enx - k * eny, sy = y - d * eny + k * enx;
      R g[9];
      load_node<S>(L, parity, sx, sy, g);
      float f[NODE_FEAT];
      strip_node_features<R>(g, rho0, base, ref, enx, eny, f);
#pragma unroll
      for (int q = 0; q < NODE_FEAT; ++q) feat[(3 * d + k + 1) * NODE_FEAT + q] = f[q];
      if (k == 0) moments<R>(g, rho0, base, mom[d][0], mom[d][1], mom[d][2]);
    }
  }
  // NSBC's m_c with a single normal (eqs. nes_2, nes_3)
  R m[3];
  const R gam = R(L.gamma), beta = R(L.beta);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const R mp = mom[0][c] - gam * normal_diff(mom[0][c], mom[1][c], mom[2][c], L.grad_order);
    m[c] = (R(1) - beta) * mp + beta * ref[c];
  }
  float rn[3], dn[3];
  to_normal_frame<R>(ref, base, enx, eny, rn);
  normal_frame_diff<R>(m, ref, enx, eny, dn);
  const float A = finish_inputs(feat, float(L.rho0), float(L.omega), dn, rn);
  mc[0] = dn[0];
  mc[1] = dn[1];
  mc[2] = dn[2];
  mc[3] = A;
}

// Moments of a site in the (n, t) frame; with `sub` (m_c - m0 and A of the
// previous step) the training residual ((m - m0) - (m_c - m0)) / A, the first
// difference formed at the lattice's precision.
template <int S>
__device__ void site_moments_body(const LatDesc& L, int parity, int x, int y, int edge, const float* sub, float* out) {
  using R = typename Codec<S>::R;
  int enx, eny;
  edge_normal(edge, enx, eny);
  R g[9], m[3];
  load_node<S>(L, parity, x, y, g);
  const Base<R> base(L);
  moments<R>(g, R(L.rho0), base, m[0], m[1], m[2]);
  if (sub) {
    const R ref[3] = {R(L.m0[0]), R(L.m0[1]), R(L.m0[2])};
    float d[3];
    normal_frame_diff<R>(m, ref, enx, eny, d);
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] = (d[c] - sub[c]) / sub[3];
  } else {
    to_normal_frame<R>(m, base, enx, eny, out);
  }
}

// Decode a site row; false when the strip (depth 0..2, tangential +-1) leaves the lattice.
__device__ inline bool site_of(const int32_t* s, int ens, int count, const LatDesc& single, const LatDesc* descs,
                               const LatDesc*& D, int& x, int& y, int& edge) {
  if (ens) {
    if (s[0] < 0 || s[0] >= count) return false;
    D = descs + s[0];
    x = s[1];
    y = s[2];
    edge = s[3];
  } else {
    D = &single;
    x = s[0];
    y = s[1];
    edge = s[2];
  }
  if (edge < 0 || edge > 3) return false;
  int enx, eny;
  edge_normal(edge, enx, eny);
  for (int d = 0; d < 3; ++d)
    for (int k = -1; k <= 1; ++k) {
      const int sx = x - d * enx - k * eny, sy = y - d * eny + k * enx;
      if (sx < 0 || sx >= D->nx || sy < 0 || sy >= D->ny) return false;
    }
  return true;
}

__global__ void k_site_features(LatDesc single, const LatDesc* __restrict__ descs, int ens, int count, int parity,
                                const int32_t* __restrict__ sites, int n, float* __restrict__ feat,
                                float* __restrict__ mc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const LatDesc* D;
  int x, y, edge;
  float* f = feat + (size_t)i * mlp::IN;
  float* m = mc + (size_t)i * 4;
  if (!site_of(sites + 4 * i, ens, count, single, descs, D, x, y, edge)) {
    for (int q = 0; q < mlp::IN; ++q) f[q] = NAN;
    m[0] = m[1] = m[2] = m[3] = NAN;
    return;
  }
  const LatDesc L = *D;
  switch (L.store) {
    case ST_F64: site_features_body<ST_F64>(L, parity, x, y, edge, f, m); break;
    case ST_F32: site_features_body<ST_F32>(L, parity, x, y, edge, f, m); break;
    case ST_F16: site_features_body<ST_F16>(L, parity, x, y, edge, f, m); break;
    default: site_features_body<ST_BF16>(L, parity, x, y, edge, f, m); break;
  }
}

__global__ void k_site_moments(LatDesc single, const LatDesc* __restrict__ descs, int ens, int count, int parity,
                               const int32_t* __restrict__ sites, int n, const float* __restrict__ sub,
                               float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const LatDesc* D;
  int x, y, edge;
  float* o = out + (size_t)i * 3;
  if (!site_of(sites + 4 * i, ens, count, single, descs, D, x, y, edge)) {
    o[0] = o[1] = o[2] = NAN;
    return;
  }
  const LatDesc L = *D;
  const float* sb = sub ? sub + (size_t)i * 4 : nullptr;
  switch (L.store) {
    case ST_F64: site_moments_body<ST_F64>(L, parity, x, y, edge, sb, o); break;
    case ST_F32: site_moments_body<ST_F32>(L, parity, x, y, edge, sb, o); break;
    case ST_F16: site_moments_body<ST_F16>(L, parity, x, y, edge, sb, o); break;
    default: site_moments_body<ST_BF16>(L, parity, x, y, edge, sb, o); break;
  }
}

hipError_t launch_site_features(const LatDesc* single, const LatDesc* descs, int count, int parity,
                                const int32_t* sites, int n, float* feat, float* mc, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LatDesc dummy;
  std::memset(&dummy, 0, sizeof(dummy));
  k_site_features<<<dim3((n + 127) / 128), dim3(128), 0, s>>>(single ? *single : dummy, descs, single ? 0 : 1,
                                                              count, parity, sites, n, feat, mc);
  return hipGetLastError();
}

hipError_t launch_site_moments(const LatDesc* single, const LatDesc* descs, int count, int parity,
                               const int32_t* sites, int n, const float* sub, float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LatDesc dummy;
  std::memset(&dummy, 0, sizeof(dummy));
  k_site_moments<<<dim3((n + 127) / 128), dim3(128), 0, s>>>(single ? *single : dummy, descs, single ? 0 : 1,
                                                             count, parity, sites, n, sub, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ trainer
constexpr int NP_PAD = 10624;  // per-block stride of the partial-gradient buffer
constexpr int TB = 64;         // rows per training block
constexpr int TTHREADS = 256;  // 4 wavefronts of 16 rows
constexpr int STAT_BLOCKS = 256;
constexpr int STAT_COLS = mlp::IN + mlp::OUT;

// Fused forward + backward of one 64-row tile; writes this tile's gradient
// contributions (partial[blockIdx.x][NPARAM]) and its summed squared error.
__global__ __launch_bounds__(TTHREADS) void k_mlp_train(const mlp::Net* __restrict__ net, const bf16* __restrict__ W3p,
                                                       const bf16* __restrict__ X, const float* __restrict__ T,
                                                       int64_t nsrc, const int32_t* __restrict__ rows, int batch,
                                                       float* __restrict__ partial, float* __restrict__ ploss) {
  using namespace mlp;
  __shared__ __attribute__((aligned(16))) bf16 sX[TB * XS];
  __shared__ __attribute__((aligned(16))) bf16 sH1[TB * HS];
  __shared__ __attribute__((aligned(16))) bf16 sH2[TB * HS];
  __shared__ __attribute__((aligned(16))) bf16 sdY[TB * YS];
  __shared__ __attribute__((aligned(16))) bf16 sdZ2[TB * HS];
  __shared__ __attribute__((aligned(16))) bf16 sdZ1[TB * HS];
  __shared__ float sdYf[TB][4];
  __shared__ float sZf[TB][HID + 1];
  __shared__ float sloss[TTHREADS];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int base = blockIdx.x * TB;
  float* P = partial + (size_t)blockIdx.x * NP_PAD;

  for (int e = tid; e < TB * (IN / 8); e += TTHREADS) {
    const int r = e / (IN / 8), c = e - r * (IN / 8);
    const int gr = base + r;
    const int64_t src = gr < batch ? (rows ? (int64_t)rows[gr] : (int64_t)gr) : -1;
    bf16x8 v;
    if (src >= 0 && src < nsrc) {
      v = *reinterpret_cast<const bf16x8*>(X + (size_t)src * IN + 8 * c);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = (bf16)0.f;
    }
    *reinterpret_cast<bf16x8*>(sX + r * XS + 8 * c) = v;
  }
  for (int e = tid; e < TB * YS; e += TTHREADS) sdY[e] = (bf16)0.f;
  __syncthreads();

  // forward, rows 16 w .. 16 w + 15
  f32x4 a1[4], a2[4], a3[1];
  layer<IN, 4>(sX + 16 * w * XS, XS, net->W1, a1);
  bias_tanh_store<4>(a1, net->b1, sH1 + 16 * w * HS, HS);
  __builtin_amdgcn_s_waitcnt(0);
  layer<HID, 4>(sH1 + 16 * w * HS, HS, net->W2, a2);
  bias_tanh_store<4>(a2, net->b2, sH2 + 16 * w * HS, HS);
  __builtin_amdgcn_s_waitcnt(0);
  layer<HID, 1>(sH2 + 16 * w * HS, HS, net->W3, a3);

  // loss and dY = 2 (y - t) / (3 batch)
  float lsum = 0.f;
  const int col = l & 15;
  if (col < OUT) {
    const float inv = 2.f / (3.f * (float)batch);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * w + 4 * (l >> 4) + r, gr = base + row;
      const int64_t src = gr < batch ? (rows ? (int64_t)rows[gr] : (int64_t)gr) : -1;
      float dy = 0.f;
      if (src >= 0 && src < nsrc) {
        const float e = a3[0][r] + net->b3[col] - T[(size_t)src * OUT + col];
        lsum += e * e;
        dy = e * inv;
      }
      sdYf[row][col] = dy;
      sdY[row * YS + col] = (bf16)dy;
    }
  }
  sloss[tid] = lsum;
  __syncthreads();

  // dZ2 = (dYb W3) * (1 - H2b^2): K = 32 (outputs, zero padded), N = 64
  f32x4 d2[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) d2[n] = f32x4{0.f, 0.f, 0.f, 0.f};
  {
    const bf16x8 a = frag_k1(sdY + 16 * w * YS, YS, 0, 0);
#pragma unroll
    for (int n = 0; n < 4; ++n) d2[n] = mfma(a, frag_gather(W3p, 1, HID, 16 * n, 0), d2[n]);
  }
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * w + 4 * (l >> 4) + r, c = 16 * n + col;
      const float h = (float)sH2[row * HS + c];
      const float z = d2[n][r] * (1.f - h * h);
      sZf[row][c] = z;
      sdZ2[row * HS + c] = (bf16)z;
    }
  __builtin_amdgcn_s_waitcnt(0);
  // dZ1 = (dZ2b W2) * (1 - H1b^2): K = 64, N = 64
  f32x4 d1[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) d1[n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kt = 0; kt < 2; ++kt) {
    const bf16x8 a = frag_k1(sdZ2 + 16 * w * HS, HS, 0, 32 * kt);
#pragma unroll
    for (int n = 0; n < 4; ++n) d1[n] = mfma(a, frag_gather(net->W2, 1, HID, 16 * n, 32 * kt), d1[n]);
  }
  __syncthreads();
  if (tid < HID) {  // db2: column sums of dZ2 in row order
    float s = 0.f;
    for (int r = 0; r < TB; ++r) s += sZf[r][tid];
    P[OFF_B2 + tid] = s;
  }
  __syncthreads();
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * w + 4 * (l >> 4) + r, c = 16 * n + col;
      const float h = (float)sH1[row * HS + c];
      const float z = d1[n][r] * (1.f - h * h);
      sZf[row][c] = z;
      sdZ1[row * HS + c] = (bf16)z;
    }
  __syncthreads();
  if (tid < HID) {  // db1
    float s = 0.f;
    for (int r = 0; r < TB; ++r) s += sZf[r][tid];
    P[OFF_B1 + tid] = s;
  } else if (tid < HID + OUT) {  // db3
    const int c = tid - HID;
    float s = 0.f;
    for (int r = 0; r < TB; ++r) s += sdYf[r][c];
    P[OFF_B3 + c] = s;
  } else if (tid == 128) {
    float s = 0.f;
    for (int k = 0; k < TTHREADS; ++k) s += sloss[k];
    ploss[blockIdx.x] = s;
  }

  // weight gradients of this tile, K = the tile's 64 rows
  // dW1 [64][96] = dZ1b^T Xb: 4 x 6 tiles of 16 x 16
  for (int q = w; q < 24; q += 4) {
    const int mt = q / 6, nt = q - mt * 6;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
      acc = mfma(frag_gather(sdZ1, 1, HS, 16 * mt, 32 * kt), frag_gather(sX, 1, XS, 16 * nt, 32 * kt), acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) P[OFF_W1 + (16 * mt + 4 * (l >> 4) + r) * IN + 16 * nt + col] = acc[r];
  }
  // dW2 [64][64] = dZ2b^T H1b
  for (int q = w; q < 16; q += 4) {
    const int mt = q >> 2, nt = q & 3;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
      acc = mfma(frag_gather(sdZ2, 1, HS, 16 * mt, 32 * kt), frag_gather(sH1, 1, HS, 16 * nt, 32 * kt), acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) P[OFF_W2 + (16 * mt + 4 * (l >> 4) + r) * HID + 16 * nt + col] = acc[r];
  }
  // dW3 [3][64] = dYb^T H2b (first 3 rows of a 16-row tile)
  {
    const int nt = w;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
      acc = mfma(frag_gather(sdY, 1, YS, 0, 32 * kt), frag_gather(sH2, 1, HS, 16 * nt, 32 * kt), acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = 4 * (l >> 4) + r;
      if (o < OUT) P[OFF_W3 + o * HID + 16 * nt + col] = acc[r];
    }
  }
}

// Sum the per-tile gradients in tile order; optionally return them, and
// optionally take an Adam step; refresh the BF16 copies and biases of the net.
__global__ void k_mlp_apply(const float* __restrict__ partial, int nblocks, float* __restrict__ master,
                            float* __restrict__ am, float* __restrict__ av, int adam, float lr, float bc1, float bc2,
                            float* __restrict__ grads_out, mlp::Net* __restrict__ net, bf16* __restrict__ W3p) {
  using namespace mlp;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  float w = master[p];
  if (nblocks > 0) {
    float g = 0.f;
    for (int b = 0; b < nblocks; ++b) g += partial[(size_t)b * NP_PAD + p];
    if (grads_out) grads_out[p] = g;
    if (adam) {
      const float m = 0.9f * am[p] + 0.1f * g;
      const float v = 0.999f * av[p] + 0.001f * g * g;
      am[p] = m;
      av[p] = v;
      w -= lr * (m / bc1) / (sqrtf(v / bc2) + 1e-8f);
      master[p] = w;
    }
  }
  if (p < OFF_B1) net->W1[p - OFF_W1] = (bf16)w;
  else if (p < OFF_W2) net->b1[p - OFF_B1] = w;
  else if (p < OFF_B2) net->W2[p - OFF_W2] = (bf16)w;
  else if (p < OFF_W3) net->b2[p - OFF_B2] = w;
  else if (p < OFF_B3) {
    net->W3[p - OFF_W3] = (bf16)w;
    W3p[p - OFF_W3] = (bf16)w;
  } else {
    net->b3[p - OFF_B3] = w;
  }
}

__global__ void k_mlp_loss(const float* __restrict__ ploss, int nblocks, int batch, float* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float s = 0.f;
  for (int b = 0; b < nblocks; ++b) s += ploss[b];
  *out = s / (3.f * (float)batch);
}

__global__ __launch_bounds__(TTHREADS) void k_mlp_forward(const mlp::Net* __restrict__ net,
                                                         const bf16* __restrict__ X, int64_t n,
                                                         float* __restrict__ Y) {
  using namespace mlp;
  __shared__ __attribute__((aligned(16))) bf16 sX[TB * XS];
  __shared__ __attribute__((aligned(16))) bf16 sH1[TB * HS];
  __shared__ __attribute__((aligned(16))) bf16 sH2[TB * HS];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int64_t base = (int64_t)blockIdx.x * TB;
  for (int e = tid; e < TB * (IN / 8); e += TTHREADS) {
    const int r = e / (IN / 8), c = e - r * (IN / 8);
    bf16x8 v;
    if (base + r < n) {
      v = *reinterpret_cast<const bf16x8*>(X + (size_t)(base + r) * IN + 8 * c);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = (bf16)0.f;
    }
    *reinterpret_cast<bf16x8*>(sX + r * XS + 8 * c) = v;
  }
  __syncthreads();
  f32x4 y;
  forward16(*net, sX + 16 * w * XS, sH1 + 16 * w * HS, sH2 + 16 * w * HS, y);
  const int col = l & 15;
  if (col < OUT) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = base + 16 * w + 4 * (l >> 4) + r;
      if (row < n) Y[row * OUT + col] = y[r];
    }
  }
}

// Column sums and sums of squares (fp64) of the raw inputs and the residuals.
__global__ void k_stats_partial(const float* __restrict__ feat, const float* __restrict__ resid, int64_t n,
                                double* __restrict__ part) {
  const int c = threadIdx.x;
  if (c >= STAT_COLS) return;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = r0 + per < n ? r0 + per : n;
  double s = 0.0, q = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    const double v = c < mlp::IN ? (double)feat[r * mlp::IN + c] : (double)resid[r * mlp::OUT + (c - mlp::IN)];
    s += v;
    q += v * v;
  }
  part[((size_t)blockIdx.x * STAT_COLS + c) * 2] = s;
  part[((size_t)blockIdx.x * STAT_COLS + c) * 2 + 1] = q;
}

// Mean, 1/std and output scales from the partial sums.  A strip-node input
// whose spread is below kNoiseFloor of the largest spread of the same moment
// over the nine strip nodes is dropped (weight 0): moments that vanish in
// exact arithmetic at the boundary row (e.g. the odd ones NSBC's
// non-equilibrium bounce-back cancels) hold only rounding noise there, and
// normalising that noise to unit spread would feed the network a
// precision-dependent random input.
constexpr double kNoiseFloor = 1e-3;

__global__ void k_stats_final(const double* __restrict__ part, int nblocks, int64_t n, mlp::Net* __restrict__ net) {
  __shared__ double sd_s[mlp::IN];
  const int c = threadIdx.x;
  double mean = 0.0, sd = 0.0, q = 0.0;
  if (c < STAT_COLS) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) {
      s += part[((size_t)b * STAT_COLS + c) * 2];
      q += part[((size_t)b * STAT_COLS + c) * 2 + 1];
    }
    mean = s / (double)n;
    const double var = q / (double)n - mean * mean;
    sd = var > 0.0 ? sqrt(var) : 0.0;
  }
  if (c < mlp::IN) sd_s[c] = sd;
  __syncthreads();
  if (c >= STAT_COLS) return;
  if (c < mlp::IN) {
    // constant inputs (a spread at the fp64 rounding level of the mean) carry nothing
    bool used = c < mlp::NFEAT && sd > 1e-30 && sd > 1e-7 * fabs(mean);
    if (used && c < 9 * NODE_FEAT) {
      const int kind = c % NODE_FEAT;
      double top = 0.0;
      for (int j = 0; j < 9; ++j) top = fmax(top, sd_s[NODE_FEAT * j + kind]);
      used = sd > kNoiseFloor * top;
    }
    net->feat_mean[c] = used ? (float)mean : 0.f;
    net->feat_inv_std[c] = used ? (float)(1.0 / sd) : 0.f;
  } else {
    const double rms = sqrt(q / (double)n);
    net->out_scale[c - mlp::IN] = (float)(rms > 1e-30 ? rms : 1e-30);
  }
}

__global__ void k_pack(const mlp::Net* __restrict__ net, const float* __restrict__ feat,
                       const float* __restrict__ resid, int64_t n, bf16* __restrict__ x, float* __restrict__ t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * mlp::IN) return;
  const int c = (int)(i % mlp::IN);
  const int64_t r = i / mlp::IN;
  x[i] = (bf16)((feat[i] - net->feat_mean[c]) * net->feat_inv_std[c]);
  if (resid && t && c < mlp::OUT) t[r * mlp::OUT + c] = resid[r * mlp::OUT + c] / net->out_scale[c];
}

__global__ void k_init_net(mlp::Net* __restrict__ net, bf16* __restrict__ W3p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 32 * mlp::HID) W3p[i] = (bf16)0.f;
  if (i < mlp::OUT_PAD * mlp::HID) net->W3[i] = (bf16)0.f;
  if (i < mlp::OUT_PAD) net->b3[i] = 0.f;
  if (i < mlp::IN) {
    net->feat_mean[i] = 0.f;
    net->feat_inv_std[i] = i < mlp::NFEAT ? 1.f : 0.f;
  }
  if (i < 4) net->out_scale[i] = 1.f;
  if (i == 0) {
    net->trust = 0.f;
    net->kmin = 0.f;
  }
}

// Trust bound and gain of an exported blob: the gain scales the output scales
// (an under-relaxed correction for gain < 1).
__global__ void k_export_finish(mlp::Net* __restrict__ net, float trust, float gain, float kmin) {
  const int i = threadIdx.x;
  if (i < mlp::OUT) net->out_scale[i] *= gain;
  if (i == 0) {
    net->trust = trust;
    net->kmin = kmin;
  }
}

}  // namespace lbm

// ---------------------------------------------------------------------- C ABI
namespace {

using lbm::host::fail;

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(LBM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct MlpLayout {
  size_t off_master, off_m, off_v, off_net, off_w3p, off_partial, off_ploss, off_stats, off_grads, total;
};

MlpLayout mlp_layout(int32_t max_batch) {
  using lbm::host::round_up;
  MlpLayout L;
  size_t o = 0;
  const size_t np = sizeof(float) * lbm::NP_PAD;
  L.off_master = o;
  o = round_up(o + np, 256);
  L.off_m = o;
  o = round_up(o + np, 256);
  L.off_v = o;
  o = round_up(o + np, 256);
  L.off_net = o;
  o = round_up(o + sizeof(lbm::mlp::Net), 256);
  L.off_w3p = o;
  o = round_up(o + sizeof(lbm::mlp::bf16) * 32 * lbm::mlp::HID, 256);
  L.off_partial = o;
  o = round_up(o + np * (size_t)(max_batch / lbm::TB), 256);
  L.off_ploss = o;
  o = round_up(o + sizeof(float) * (size_t)(max_batch / lbm::TB), 256);
  L.off_stats = o;
  o = round_up(o + sizeof(double) * 2 * lbm::STAT_COLS * lbm::STAT_BLOCKS, 256);
  L.off_grads = o;
  o = round_up(o + np, 256);
  L.total = o;
  return L;
}

}  // namespace

struct lbm_mlp {
  int32_t max_batch = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  MlpLayout lay;
  int64_t step = 0;
  float* master() { return reinterpret_cast<float*>(ws + lay.off_master); }
  float* am() { return reinterpret_cast<float*>(ws + lay.off_m); }
  float* av() { return reinterpret_cast<float*>(ws + lay.off_v); }
  lbm::mlp::Net* net() { return reinterpret_cast<lbm::mlp::Net*>(ws + lay.off_net); }
  lbm::mlp::bf16* w3p() { return reinterpret_cast<lbm::mlp::bf16*>(ws + lay.off_w3p); }
  float* partial() { return reinterpret_cast<float*>(ws + lay.off_partial); }
  float* ploss() { return reinterpret_cast<float*>(ws + lay.off_ploss); }
  double* stats() { return reinterpret_cast<double*>(ws + lay.off_stats); }
  float* grads() { return reinterpret_cast<float*>(ws + lay.off_grads); }
};

namespace {

int check_batch(const lbm_mlp* m, int32_t batch) {
  if (!m) return fail(LBM_ERR_ARG, "trainer is NULL");
  if (batch < 1 || batch > m->max_batch) return fail(LBM_ERR_ARG, "batch %d outside [1, %d]", batch, m->max_batch);
  return LBM_OK;
}

int run_train(lbm_mlp* m, const uint16_t* x, const float* t, int64_t nsamples, const int32_t* rows, int32_t batch,
              int adam, float lr, float* grads_out, float* loss_out) {
  int rc = check_batch(m, batch);
  if (rc) return rc;
  if (!x || !t) return fail(LBM_ERR_ARG, "x and t must not be NULL");
  if (nsamples < 1) return fail(LBM_ERR_ARG, "nsamples %lld < 1", (long long)nsamples);
  if (!rows && nsamples < batch) return fail(LBM_ERR_ARG, "batch %d > nsamples %lld", batch, (long long)nsamples);
  if (adam && !(lr > 0.f && std::isfinite(lr))) return fail(LBM_ERR_ARG, "learning rate %g", (double)lr);
  const int nb = (batch + lbm::TB - 1) / lbm::TB;
  lbm::k_mlp_train<<<dim3(nb), dim3(lbm::TTHREADS), 0, m->stream>>>(
      m->net(), m->w3p(), reinterpret_cast<const lbm::mlp::bf16*>(x), t, nsamples, rows, batch, m->partial(),
      m->ploss());
  HIPCHK(hipGetLastError());
  if (loss_out) {
    lbm::k_mlp_loss<<<dim3(1), dim3(64), 0, m->stream>>>(m->ploss(), nb, batch, loss_out);
    HIPCHK(hipGetLastError());
  }
  float bc1 = 1.f, bc2 = 1.f;
  if (adam) {
    m->step += 1;
    bc1 = (float)(1.0 - std::pow(0.9, (double)m->step));
    bc2 = (float)(1.0 - std::pow(0.999, (double)m->step));
  }
  lbm::k_mlp_apply<<<dim3((lbm::mlp::NPARAM + 255) / 256), dim3(256), 0, m->stream>>>(
      m->partial(), nb, m->master(), m->am(), m->av(), adam, lr, bc1, bc2, grads_out, m->net(), m->w3p());
  HIPCHK(hipGetLastError());
  return LBM_OK;
}

}  // namespace

namespace lbm {
namespace host {
// used by lbm_api.hip / lbm_ensemble.hip
hipError_t closure_features(const LatDesc* single, const LatDesc* descs, int count, int parity, const int32_t* sites,
                            int n, float* feat, float* mc, hipStream_t s) {
  return launch_site_features(single, descs, count, parity, sites, n, feat, mc, s);
}
hipError_t closure_moments(const LatDesc* single, const LatDesc* descs, int count, int parity, const int32_t* sites,
                           int n, const float* sub, float* out, hipStream_t s) {
  return launch_site_moments(single, descs, count, parity, sites, n, sub, out, s);
}
}  // namespace host
}  // namespace lbm

extern "C" {

int lbm_closure_net_bytes(size_t* bytes) {
  if (!bytes) return fail(LBM_ERR_ARG, "bytes is NULL");
  *bytes = sizeof(lbm::mlp::Net);
  return LBM_OK;
}

int lbm_mlp_workspace_bytes(int32_t max_batch, size_t* bytes) {
  if (!bytes) return fail(LBM_ERR_ARG, "bytes is NULL");
  if (max_batch < lbm::TB || max_batch > 65536 || max_batch % lbm::TB)
    return fail(LBM_ERR_ARG, "max_batch %d must be a multiple of %d in [%d, 65536]", max_batch, lbm::TB, lbm::TB);
  *bytes = mlp_layout(max_batch).total;
  return LBM_OK;
}

void lbm_mlp_destroy(lbm_mlp* m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->stream);
  delete m;
}

int lbm_mlp_init(lbm_mlp** out, int32_t max_batch, void* workspace, size_t bytes, const float* params,
                 void* hip_stream) {
  if (!out) return fail(LBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  int rc = lbm_mlp_workspace_bytes(max_batch, &need);
  if (rc) return rc;
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(LBM_ERR_ARG, "workspace NULL or not 256-byte aligned");
  if (bytes < need) return fail(LBM_ERR_ARG, "workspace of %zu bytes < %zu required", bytes, need);
  if (!params) return fail(LBM_ERR_ARG, "params is NULL");
  lbm_mlp* m = new lbm_mlp();
  m->max_batch = max_batch;
  m->stream = static_cast<hipStream_t>(hip_stream);
  m->ws = static_cast<char*>(workspace);
  m->lay = mlp_layout(max_batch);
  hipError_t e = hipMemcpyAsync(m->master(), params, sizeof(float) * lbm::mlp::NPARAM, hipMemcpyDeviceToDevice,
                                m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->am(), 0, sizeof(float) * lbm::NP_PAD, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->av(), 0, sizeof(float) * lbm::NP_PAD, m->stream);
  if (e == hipSuccess) {
    lbm::k_init_net<<<dim3(8), dim3(256), 0, m->stream>>>(m->net(), m->w3p());
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    lbm::k_mlp_apply<<<dim3((lbm::mlp::NPARAM + 255) / 256), dim3(256), 0, m->stream>>>(
        m->partial(), 0, m->master(), m->am(), m->av(), 0, 0.f, 1.f, 1.f, nullptr, m->net(), m->w3p());
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) {
    delete m;
    return fail(LBM_ERR_HIP, "trainer init: %s", hipGetErrorString(e));
  }
  *out = m;
  return LBM_OK;
}

int lbm_mlp_fit_normalization(lbm_mlp* m, const float* feat, const float* resid, int64_t n) {
  if (!m || !feat || !resid) return fail(LBM_ERR_ARG, "NULL argument");
  if (n < 2) return fail(LBM_ERR_ARG, "need at least 2 samples");
  lbm::k_stats_partial<<<dim3(lbm::STAT_BLOCKS), dim3(128), 0, m->stream>>>(feat, resid, n, m->stats());
  HIPCHK(hipGetLastError());
  lbm::k_stats_final<<<dim3(1), dim3(128), 0, m->stream>>>(m->stats(), lbm::STAT_BLOCKS, n, m->net());
  HIPCHK(hipGetLastError());
  return LBM_OK;
}

int lbm_mlp_pack(lbm_mlp* m, const float* feat, const float* resid, int64_t n, uint16_t* x_out, float* t_out) {
  if (!m || !feat || !x_out) return fail(LBM_ERR_ARG, "NULL argument");
  if (n < 0) return fail(LBM_ERR_ARG, "n < 0");
  if (n == 0) return LBM_OK;
  const int64_t total = n * lbm::mlp::IN;
  lbm::k_pack<<<dim3((unsigned)((total + 255) / 256)), dim3(256), 0, m->stream>>>(
      m->net(), feat, resid, n, reinterpret_cast<lbm::mlp::bf16*>(x_out), t_out);
  HIPCHK(hipGetLastError());
  return LBM_OK;
}

int lbm_mlp_train_step(lbm_mlp* m, const uint16_t* x, const float* t, int64_t nsamples, const int32_t* rows,
                       int32_t batch, float lr, float* loss_out) {
  return run_train(m, x, t, nsamples, rows, batch, 1, lr, nullptr, loss_out);
}

int lbm_mlp_grads(lbm_mlp* m, const uint16_t* x, const float* t, int64_t nsamples, const int32_t* rows,
                  int32_t batch, float* grads_out, float* loss_out) {
  if (!grads_out) return fail(LBM_ERR_ARG, "grads_out is NULL");
  return run_train(m, x, t, nsamples, rows, batch, 0, 0.f, grads_out, loss_out);
}

int lbm_mlp_forward(lbm_mlp* m, const uint16_t* x, int64_t n, float* y_out) {
  if (!m || !x || !y_out) return fail(LBM_ERR_ARG, "NULL argument");
  if (n <= 0) return n == 0 ? LBM_OK : fail(LBM_ERR_ARG, "n < 0");
  lbm::k_mlp_forward<<<dim3((unsigned)((n + lbm::TB - 1) / lbm::TB)), dim3(lbm::TTHREADS), 0, m->stream>>>(
      m->net(), reinterpret_cast<const lbm::mlp::bf16*>(x), n, y_out);
  HIPCHK(hipGetLastError());
  return LBM_OK;
}

int lbm_mlp_params(lbm_mlp* m, float* params_out) {
  if (!m || !params_out) return fail(LBM_ERR_ARG, "NULL argument");
  HIPCHK(hipMemcpyAsync(params_out, m->master(), sizeof(float) * lbm::mlp::NPARAM, hipMemcpyDeviceToDevice,
                        m->stream));
  return LBM_OK;
}

int lbm_mlp_normalization(lbm_mlp* m, float* mean_out, float* inv_std_out, float* scale_out) {
  if (!m) return fail(LBM_ERR_ARG, "trainer is NULL");
  lbm::mlp::Net* net = m->net();
  if (mean_out) HIPCHK(hipMemcpyAsync(mean_out, net->feat_mean, sizeof(float) * 96, hipMemcpyDeviceToDevice, m->stream));
  if (inv_std_out)
    HIPCHK(hipMemcpyAsync(inv_std_out, net->feat_inv_std, sizeof(float) * 96, hipMemcpyDeviceToDevice, m->stream));
  if (scale_out) HIPCHK(hipMemcpyAsync(scale_out, net->out_scale, sizeof(float) * 3, hipMemcpyDeviceToDevice, m->stream));
  return LBM_OK;
}

int lbm_mlp_set_normalization(lbm_mlp* m, const float* mean, const float* inv_std, const float* scale) {
  if (!m || !mean || !inv_std || !scale) return fail(LBM_ERR_ARG, "NULL argument");
  lbm::mlp::Net* net = m->net();
  HIPCHK(hipMemcpyAsync(net->feat_mean, mean, sizeof(float) * 96, hipMemcpyDeviceToDevice, m->stream));
  HIPCHK(hipMemcpyAsync(net->feat_inv_std, inv_std, sizeof(float) * 96, hipMemcpyDeviceToDevice, m->stream));
  HIPCHK(hipMemcpyAsync(net->out_scale, scale, sizeof(float) * 3, hipMemcpyDeviceToDevice, m->stream));
  return LBM_OK;
}

int lbm_mlp_export(lbm_mlp* m, float trust, float gain, float kmin, void* net_out) {
  if (!m || !net_out) return fail(LBM_ERR_ARG, "NULL argument");
  if (!(trust > 0.f)) return fail(LBM_ERR_ARG, "trust bound %g must be > 0", (double)trust);
  if (!(gain > 0.f) || !std::isfinite(gain)) return fail(LBM_ERR_ARG, "gain %g must be finite and > 0", (double)gain);
  if (!(kmin >= 0.f) || !std::isfinite(kmin)) return fail(LBM_ERR_ARG, "kmin %g must be finite and >= 0", (double)kmin);
  HIPCHK(hipMemcpyAsync(net_out, m->net(), sizeof(lbm::mlp::Net), hipMemcpyDeviceToDevice, m->stream));
  lbm::k_export_finish<<<dim3(1), dim3(32), 0, m->stream>>>(static_cast<lbm::mlp::Net*>(net_out), trust, gain,
                                                             kmin);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(m->stream));
  return LBM_OK;
}

}  // extern "C"
