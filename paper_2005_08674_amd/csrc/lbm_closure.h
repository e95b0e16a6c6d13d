// lbm_closure.h -- input features of the learned boundary closure.
//
// For a boundary node b with outward unit normal n (an axis direction) and
// tangent t = (-n_y, n_x), the network sees the nine strip nodes
// s(d, k) = b - d n + k t, d = 0, 1, 2 (depth), k = -1, 0, 1 (tangential),
// at time t, each described in the (n, t) frame by
//   [drho, u.n, u.t, P_nn, P_nt, P_tt, Q_nnt, Q_ntt, R_nntt]
// where P, Q, R are the 2nd/3rd/4th moments of the non-equilibrium part
// f_i - f_i^eq (its 0th and 1st moments vanish), strip node j = 3 d + k + 1
// filling features 9 j .. 9 j + 8; then omega = 1/tau (feature 81) and NSBC's
// m_c = (drho_c, u_c.n, u_c.t) (features 82..84); 85..95 are zero.
// The network's 3 outputs correct m_c in the same frame.
#pragma once

#include "lbm_device.h"
#include "lbm_mlp.h"

namespace lbm {

constexpr int NODE_FEAT = 9;

// Features of one strip node from its 9 decoded deviations.
template <class R>
__device__ inline void strip_node_features(const R g[9], R rho0, const Base<R>& b, int nx_, int ny_,
                                           float f[NODE_FEAT]) {
  R dr, dux, duy, geq[9];
  moments<R>(g, rho0, b, dr, dux, duy);
  equilibrium<R>(rho0, b, dr, dux, duy, geq);
  const R ux = dux + b.ubx, uy = duy + b.uby;
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
  f[0] = float(dr);
  f[1] = float(ux * R(nx_) + uy * R(ny_));
  f[2] = float(-ux * R(ny_) + uy * R(nx_));
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

}  // namespace lbm
