// lbm_mlp.h -- device building blocks of the boundary-closure network:
// BF16 MFMA tiles for gfx950 (v_mfma_f32_16x16x32_bf16, FP32 accumulate),
// one wavefront per 16 rows.
//
// Network: 96 inputs (87 used) -> 64 (tanh) -> 64 (tanh) -> 3 outputs (padded to 16),
// BF16 weights and layer inputs, FP32 accumulation, bias and tanh in FP32.
//
// MFMA lane layout (16x16x32): lane l holds A[l % 16][8 (l / 16) + j] and
// B[8 (l / 16) + j][l % 16] for j = 0..7, and accumulates
// D[4 (l / 16) + r][l % 16] for r = 0..3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {
namespace mlp {

constexpr int IN = 96, HID = 64, OUT = 3, OUT_PAD = 16, NFEAT = 87;
constexpr int XS = 104;  // LDS row stride (bf16) of a 96-wide tile: 16-byte rows, no bank conflicts
constexpr int HS = 72;   // LDS row stride (bf16) of a 64-wide tile
constexpr int YS = 40;   // LDS row stride (bf16) of the output-gradient tile (K padded to 32)

// Packed fp32 parameter vector: W1 [64][96], b1 [64], W2 [64][64], b2 [64], W3 [3][64], b3 [3].
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + HID * IN;
constexpr int OFF_W2 = OFF_B1 + HID;
constexpr int OFF_B2 = OFF_W2 + HID * HID;
constexpr int OFF_W3 = OFF_B2 + HID;
constexpr int OFF_B3 = OFF_W3 + OUT * HID;
constexpr int NPARAM = OFF_B3 + OUT;  // 10563

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Network as the edge kernel reads it (device memory).  Weights in BF16,
// row-major [out][in]; W3 rows 3..15 are zero.
struct Net {
  bf16 W1[HID * IN];
  bf16 W2[HID * HID];
  bf16 W3[OUT_PAD * HID];
  float b1[HID];
  float b2[HID];
  float b3[OUT_PAD];
  float feat_mean[IN];
  float feat_inv_std[IN];
  float out_scale[4];  // physical units of one normalised output (drho, u_n, u_t)
  float trust;         // largest |normalised output| accepted
  float kmin;          // regime gate: the correction applies where the strip's kinetic disturbance
                       // sum |du|^2 exceeds kmin times its acoustic part sum c_s^2 drho^2 / rho0^2
  int32_t pad[2];
};

__device__ inline int lane() { return threadIdx.x & 63; }

// Fragment with 8 consecutive k-elements contiguous in memory (16-byte aligned).
__device__ inline bf16x8 frag_k1(const bf16* base, int ld, int mn0, int k0) {
  const int l = lane();
  return *reinterpret_cast<const bf16x8*>(base + (mn0 + (l & 15)) * ld + k0 + 8 * (l >> 4));
}

// Fragment with the k-elements `ldk` apart and rows/columns `ld` apart.
__device__ inline bf16x8 frag_gather(const bf16* base, int ld, int ldk, int mn0, int k0) {
  const int l = lane();
  const bf16* p = base + (mn0 + (l & 15)) * ld + (k0 + 8 * (l >> 4)) * ldk;
  bf16x8 v;
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = p[j * ldk];
  return v;
}

__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// One dense layer for the 16 rows of this wavefront:
//   out[16 x 16 NT] = X[16 x K] W^T, X in LDS (row stride xs), W global [NT*16][K] (row-major).
template <int K, int NT>
__device__ inline void layer(const bf16* X, int xs, const bf16* W, f32x4 acc[NT]) {
#pragma unroll
  for (int n = 0; n < NT; ++n) acc[n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kt = 0; kt < K / 32; ++kt) {
    const bf16x8 a = frag_k1(X, xs, 0, 32 * kt);
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[n] = mfma(a, frag_k1(W, K, 16 * n, 32 * kt), acc[n]);
  }
}

// acc (16 x 16 NT) + bias -> tanh -> BF16 into LDS rows H (stride hs).
template <int NT>
__device__ inline void bias_tanh_store(const f32x4 acc[NT], const float* bias, bf16* H, int hs) {
  const int l = lane();
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    const int col = 16 * n + (l & 15);
    const float b = bias[col];
#pragma unroll
    for (int r = 0; r < 4; ++r) H[(4 * (l >> 4) + r) * hs + col] = (bf16)tanhf(acc[n][r] + b);
  }
}

// Where a forward pass reads the parameters: the Net itself, or a copy of
// its weights and biases in LDS (same values, same instruction sequence).
struct Params {
  const bf16* W1;
  const bf16* W2;
  const bf16* W3;
  const float* b1;
  const float* b2;
  const float* b3;
  const float* mean;     // input normalisation (feat_mean, feat_inv_std)
  const float* inv_std;
};
__device__ inline Params params_of(const Net& net) {
  return {net.W1, net.W2, net.W3, net.b1, net.b2, net.b3, net.feat_mean, net.feat_inv_std};
}

// The biases and input normalisation as one block (b1, b2, b3, feat_mean,
// feat_inv_std; fp32), for an LDS copy beside the weights in device memory.
constexpr int PARAM_BYTES = (HID + HID + OUT_PAD + 2 * IN) * 4;

// Copies the biases and the input normalisation into `dst` (16-byte aligned,
// PARAM_BYTES) with the threads of a block (tid of nt) and returns the
// parameters with those read from there; the caller synchronises before use.
__device__ inline Params stage_params(const Net& net, char* dst, int tid, int nt) {
  constexpr int ob2 = HID * 4, ob3 = ob2 + HID * 4, om = ob3 + OUT_PAD * 4, os = om + IN * 4;
  auto copy = [&](const float* src, int off, int n) {
    float* d = reinterpret_cast<float*>(dst + off);
    for (int k = tid; k < n; k += nt) d[k] = src[k];
  };
  copy(net.b1, 0, HID);
  copy(net.b2, ob2, HID);
  copy(net.b3, ob3, OUT_PAD);
  copy(net.feat_mean, om, IN);
  copy(net.feat_inv_std, os, IN);
  return {net.W1,
          net.W2,
          net.W3,
          reinterpret_cast<const float*>(dst),
          reinterpret_cast<const float*>(dst + ob2),
          reinterpret_cast<const float*>(dst + ob3),
          reinterpret_cast<const float*>(dst + om),
          reinterpret_cast<const float*>(dst + os)};
}

// Forward pass of 16 rows (this wavefront): X (LDS, stride XS) -> H1, H2 (LDS,
// stride HS) -> y (lane l, r: row 4 (l / 16) + r, output column l % 16).
__device__ inline void forward16(const Params& p, const bf16* X, bf16* H1, bf16* H2, f32x4& y) {
  f32x4 a1[4], a2[4], a3[1];
  layer<IN, 4>(X, XS, p.W1, a1);
  bias_tanh_store<4>(a1, p.b1, H1, HS);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_s_waitcnt(0);
  layer<HID, 4>(H1, HS, p.W2, a2);
  bias_tanh_store<4>(a2, p.b2, H2, HS);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_s_waitcnt(0);
  layer<HID, 1>(H2, HS, p.W3, a3);
  const float b = p.b3[lane() & 15];
  y = a3[0] + f32x4{b, b, b, b};
}
__device__ inline void forward16(const Net& net, const bf16* X, bf16* H1, bf16* H2, f32x4& y) {
  forward16(params_of(net), X, H1, H2, y);
}

}  // namespace mlp
}  // namespace lbm
