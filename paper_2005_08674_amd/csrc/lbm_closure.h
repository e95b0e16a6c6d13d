// lbm_closure.h -- input features of the learned boundary closure.
//
// For a boundary node b with outward unit normal n (an axis direction) and
// tangent t = (-n_y, n_x), the network sees the nine strip nodes
// s(d, k) = b - d n + k t, d = 0, 1, 2 (depth), k = -1, 0, 1 (tangential),
// at time t, each described in the (n, t) frame by
//   [rho - rho_ref, (u - u_ref).n, (u - u_ref).t, P_nn, P_nt, P_tt, Q_nnt, Q_ntt, R_nntt]
// where (rho_ref, u_ref) is the lattice's far-field state m0 and P, Q, R are
// the 2nd/3rd/4th moments of the non-equilibrium part f_i - f_i^eq (its 0th
// and 1st moments vanish); strip node j = 3 d + k + 1 fills inputs 9 j .. 9 j + 8.
// These 81 values and NSBC's m_c - m0 (inputs 82..84, same frame) are divided
// by the strip amplitude
//   A = sqrt( (1/9) sum_j [c_s^2 (rho_j - rho_ref)^2 / rho0^2 + |u_j - u_ref|^2] ),
// so the inputs describe the shape of the disturbance, not its size; input 81
// is omega = 1/tau and inputs 85, 86 are u_ref.n, u_ref.t; 87..95 are zero.
// The network's 3 outputs, times the output scales and A, correct m_c in the
// (n, t) frame: the closure is homogeneous of degree one in the disturbance
// and vanishes with it.
#pragma once

#include "lbm_device.h"
#include "lbm_mlp.h"

namespace lbm {

constexpr int NODE_FEAT = 9;
constexpr int F_STRIP = 9 * NODE_FEAT;  // 81
constexpr int F_OMEGA = 81, F_MC = 82, F_UREF = 85;

// Unscaled features of one strip node from its 9 decoded deviations; ref =
// m0 in the deviation form (rho_ref - rho0, u_ref - u_b).
template <class R>
__device__ inline void strip_node_features(const R g[9], R rho0, const Base<R>& b, const R ref[3], int nx_, int ny_,
                                           float f[NODE_FEAT]) {
  R dr, dux, duy, geq[9];
  moments<R>(g, rho0, b, dr, dux, duy);
  equilibrium<R>(rho0, b, dr, dux, duy, geq);
  const R px = dux - ref[1], py = duy - ref[2];
  R pnn = 0, pnt = 0, ptt = 0, qnnt = 0, qntt = 0, rnntt = 0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const R q = g[i] - geq[i];
    const R cn = R(kCx[i] * nx_ + kCy[i] * ny_);
    const R ct = R(-kCx[i] * ny_ + kCy[i] * nx_);
    pnn += q * cn * cn;
    pnt += q * cn * ct;
    ptt += q * ct * ct;
    qnnt += q * cn * cn * ct;
    qntt += q * cn * ct * ct;
    rnntt += q * cn * cn * ct * ct;
  }
  f[0] = float(dr - ref[0]);
  f[1] = float(px * R(nx_) + py * R(ny_));
  f[2] = float(-px * R(ny_) + py * R(nx_));
  f[3] = float(pnn);
  f[4] = float(pnt);
  f[5] = float(ptt);
  f[6] = float(qnnt);
  f[7] = float(qntt);
  f[8] = float(rnntt);
}

// (drho, u_n, u_t) of a moment triple (drho, du_x, du_y) about base velocity u_b.
template <class R>
__device__ inline void to_normal_frame(const R m[3], const Base<R>& b, int nx_, int ny_, float out[3]) {
  const R ux = m[1] + b.ubx, uy = m[2] + b.uby;
  out[0] = float(m[0]);
  out[1] = float(ux * R(nx_) + uy * R(ny_));
  out[2] = float(-ux * R(ny_) + uy * R(nx_));
}

// (a - b) in the (n, t) frame for two moment triples in the deviation form;
// the difference is formed at the lattice's precision before rounding.
template <class R>
__device__ inline void normal_frame_diff(const R a[3], const R b[3], int nx_, int ny_, float out[3]) {
  const R dx = a[1] - b[1], dy = a[2] - b[2];
  out[0] = float(a[0] - b[0]);
  out[1] = float(dx * R(nx_) + dy * R(ny_));
  out[2] = float(-dx * R(ny_) + dy * R(nx_));
}

// Strip amplitude of an input row,
//   A = sqrt( (1/9) sum_j [c_s^2 (rho_j - rho_ref)^2 / rho0^2 + |u_j - u_ref|^2] ),
// from the unscaled strip features feat(j, q) (strip node j, feature q).
template <class F>
__device__ inline float strip_amplitude(F feat, float rho0) {
  constexpr float cs2 = 1.f / 3.f;
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    const float r = feat(j, 0) / rho0, un = feat(j, 1), ut = feat(j, 2);
    s += cs2 * r * r + un * un + ut * ut;
  }
  return sqrtf(s / 9.f);
}

__device__ inline float amplitude_inverse(float A) { return A > 0.f ? 1.f / A : 0.f; }

// Input q of a finished row: the strip part scaled by 1/A (inv), omega,
// (m_c - m0)/A, u_ref and zeros.  dmc: m_c - m0 and refn: m0, both as
// (drho, u_n, u_t) in the edge frame.
template <class F>
__device__ inline float input_value(int q, F feat, float inv, float omega, const float dmc[3], const float refn[3]) {
  if (q < F_STRIP) return feat(q / NODE_FEAT, q % NODE_FEAT) * inv;
  if (q == F_OMEGA) return omega;
  if (q < F_UREF) return dmc[q - F_MC] * inv;
  if (q < mlp::NFEAT) return refn[1 + q - F_UREF];
  return 0.f;
}

// Regime gate of a finished row, given as scaled(j, q) = feat(j, q) / A: true
// when the strip's kinetic disturbance sum_j |u_j - u_ref|^2 exceeds kmin
// times its acoustic part sum_j c_s^2 (rho_j - rho_ref)^2 / rho0^2.  A sound
// wave carries the two in equal measure (ratio 1 at normal incidence), a
// convected vortex almost only the first; kmin = 0 accepts every node.  The
// ratio does not depend on the 1/A scaling of the row.
template <class F>
__device__ inline bool vortical_row(F scaled, float rho0, float kmin) {
  constexpr float cs2 = 1.f / 3.f;
  float su = 0.f, sr = 0.f;
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    const float r = scaled(j, 0) / rho0, un = scaled(j, 1), ut = scaled(j, 2);
    su += un * un + ut * ut;
    sr += cs2 * r * r;
  }
  return su > kmin * sr;
}

// Completes an input row x[0..86] whose strip part x[0..80] holds the
// unscaled node features: appends omega, (m_c - m0)/A and u_ref, scales the
// strip part by 1/A, zeroes 87..95 and returns A.  dmc: m_c - m0 and refn:
// m0, both as (drho, u_n, u_t) in the edge frame.
__device__ inline float finish_inputs(float* x, float rho0, float omega, const float dmc[3], const float refn[3]) {
  auto unscaled = [&](int j, int q) { return x[NODE_FEAT * j + q]; };
  const float A = strip_amplitude(unscaled, rho0);
  const float inv = amplitude_inverse(A);
  float row[mlp::IN];
#pragma unroll
  for (int q = 0; q < mlp::IN; ++q) row[q] = input_value(q, unscaled, inv, omega, dmc, refn);
#pragma unroll
  for (int q = 0; q < mlp::IN; ++q) x[q] = row[q];
  return A;
}

// Regime gate of a finished row x (see vortical_row).
__device__ inline bool vortical(const float* x, float rho0, float kmin) {
  return vortical_row([&](int j, int q) { return x[NODE_FEAT * j + q]; }, rho0, kmin);
}

// Normalised network input q of value v (BF16), as the network was trained.
__device__ inline mlp::bf16 normalised_input(const float* mean, const float* inv_std, int q, float v) {
  return (mlp::bf16)((v - mean[q]) * inv_std[q]);
}
__device__ inline mlp::bf16 normalised_input(const mlp::Net& net, int q, float v) {
  return normalised_input(net.feat_mean, net.feat_inv_std, q, v);
}

// The closure's correction of m_c for network outputs o (normalised) and
// strip amplitude amp > 0, in the lattice frame: false (NSBC's m_c stays)
// when an output is not finite or leaves the trust bound (fmaxf would drop a
// NaN operand, so finiteness is tested first).
__device__ inline bool closure_delta(const mlp::Net& net, float o0, float o1, float o2, float amp, int enx, int eny,
                                     float d[3]) {
  const bool finite = isfinite(o0) && isfinite(o1) && isfinite(o2);
  if (!(finite && fmaxf(fabsf(o0), fmaxf(fabsf(o1), fabsf(o2))) <= net.trust)) return false;
  const float cr = amp * (o0 * net.out_scale[0]);
  const float cn = amp * (o1 * net.out_scale[1]);
  const float ct = amp * (o2 * net.out_scale[2]);
  // back to the lattice frame: du = c_n n + c_t t, t = (-n_y, n_x)
  d[0] = cr;
  d[1] = cn * float(enx) - ct * float(eny);
  d[2] = cn * float(eny) + ct * float(enx);
  return true;
}

}  // namespace lbm
