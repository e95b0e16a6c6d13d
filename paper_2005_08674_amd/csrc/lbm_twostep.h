// lbm_twostep.h -- two lattice steps per launch (t -> t + 2) for lattices
// with NSBC on all four edges (eqs. lbe_0, lbe_1, feq_1 in the bulk;
// eqs. nes_0..nes_4 on the edges).
//
// The single-step path reads and writes every population once per step.
// Here the intermediate level t + 1 never leaves the registers, so one launch
// moves the state through HBM once for two steps.
//
// Layout of the work: a wavefront owns 64 consecutive columns
// x = X0 - 2 .. X0 + 61 and sweeps a band of rows upward, one row per
// iteration.  Populations shifted along x come from the neighbouring lanes
// (lane shuffles); shifts along y come from the rows already swept, held in
// a rolling register window.  Level t + 1 is exact on lanes 1..62 and level
// t + 2 on lanes 2..61, which are the 60 columns X0 .. X0 + 59 the wavefront
// writes.  Rows are swept in bands of H output rows; a band re-reads at most
// four rows of its neighbours (two more at the lattice's top and bottom
// edges, for the NSBC normal differences).
//
// Per node the arithmetic is the single-step path's, in the same order
// (pull, NSBC assignment and correction with the same m_c, BGK), and the
// intermediate level is rounded through the storage codec exactly as if it
// had been stored, so results are bit-identical to two single steps.
#pragma once

#include "lbm_device.h"
#include "lbm_sweep.h"

namespace lbm {

constexpr int TS_COLS = 60;   // columns written per wavefront
constexpr int TS_WAVES = 4;   // wavefronts per block

__device__ inline float ts_shfl(float v, int src) { return __shfl(v, src, 64); }
__device__ inline double ts_shfl(double v, int src) { return __shfl(v, src, 64); }

// Value of lane l - dx (dx = +1 or -1) by a whole-wavefront DPP shift
// (wave_shr:1 / wave_shl:1, a VALU operand modifier; no LDS round trip).  The
// lane that has no source keeps 0; the sweep never uses it.
template <int DX>
__device__ inline float ts_shift(float v) {
  static_assert(DX == 1 || DX == -1, "unit shifts only");
  constexpr int ctrl = DX == 1 ? 0x138 : 0x130;  // wave_shr:1, wave_shl:1
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xf, 0xf, false));
}

// Rolling state of one level of the sweep: the rows that source rows of the
// previous level have been streamed into.  Before source row s is streamed,
// `full` holds row s - 2 complete; streaming s then
//   completes row s - 1 with the c_y = -1 populations of s,
//   adds the c_y = 0 populations of s to row s,
//   starts row s + 1 with the c_y = +1 populations of s.
template <class R>
struct TsLevel {
  R full[9];    // row s - 2, complete
  R pa[6];      // row s - 1: populations 3, 5, 7 (from s - 2) and 0, 1, 2 (from s - 1)
  R pb[3];      // row s: populations 3, 5, 7 (from s - 1)
  R mom[5][3];  // moments of the source rows s - 4 .. s (after ts_push_moments)
};

template <class R>
__device__ inline void ts_init(TsLevel<R>& L) {
#pragma unroll
  for (int i = 0; i < 9; ++i) L.full[i] = R(0);
#pragma unroll
  for (int k = 0; k < 6; ++k) L.pa[k] = R(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) L.pb[k] = R(0);
#pragma unroll
  for (int j = 0; j < 5; ++j) L.mom[j][0] = L.mom[j][1] = L.mom[j][2] = R(0);
}

// Slide the moment window by source row s (values v of this lane's column).
template <class R>
__device__ inline void ts_push_moments(TsLevel<R>& L, const R v[9], R rho0, const Base<R>& b, bool valid) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    L.mom[j][0] = L.mom[j + 1][0];
    L.mom[j][1] = L.mom[j + 1][1];
    L.mom[j][2] = L.mom[j + 1][2];
  }
  if (valid) {
    moments<R>(v, rho0, b, L.mom[4][0], L.mom[4][1], L.mom[4][2]);
  } else {
    L.mom[4][0] = L.mom[4][1] = L.mom[4][2] = R(0);
  }
}

// Stream source row s into the level (after row s - 2 has been taken from
// `full`): population i of column x comes from column x - c_x.
template <class R>
__device__ inline void ts_stream(TsLevel<R>& L, const R v[9], int lane) {
  R sh[9];
  // c_x = +1: populations 1, 5, 8; c_x = -1: 2, 6, 7
  sh[0] = v[0];
  sh[3] = v[3];
  sh[4] = v[4];
  sh[1] = ts_shift<1>(v[1]);
  sh[5] = ts_shift<1>(v[5]);
  sh[8] = ts_shift<1>(v[8]);
  sh[2] = ts_shift<-1>(v[2]);
  sh[6] = ts_shift<-1>(v[6]);
  sh[7] = ts_shift<-1>(v[7]);
  (void)lane;
  L.full[3] = L.pa[0];
  L.full[5] = L.pa[1];
  L.full[7] = L.pa[2];
  L.full[0] = L.pa[3];
  L.full[1] = L.pa[4];
  L.full[2] = L.pa[5];
  L.full[4] = sh[4];
  L.full[6] = sh[6];
  L.full[8] = sh[8];
  L.pa[0] = L.pb[0];
  L.pa[1] = L.pb[1];
  L.pa[2] = L.pb[2];
  L.pa[3] = sh[0];
  L.pa[4] = sh[1];
  L.pa[5] = sh[2];
  L.pb[0] = sh[3];
  L.pb[1] = sh[5];
  L.pb[2] = sh[7];
}

// Finalise node (x, q) of a level: `g` holds its streamed populations
// (L.full), the source-row moments of rows q - 2 .. q + 2 are L.mom[0..4].
// Boundary nodes get NSBC (unknown populations rebuilt from m_c), then BGK.
// mxn[d][c]: moments of row q at column x + d * dir (d = 1, 2) towards the
// interior for a node on the left (dir +1) or right (dir -1) edge.
template <class R>
__device__ inline void ts_finalise(const LatDesc& Ld, R g[9], const R (&mom)[5][3], const R (&mxn)[2][3], int x,
                                   int q, R rho0, const Base<R>& b, R omega) {
  const int nx = Ld.nx, ny = Ld.ny;
  const bool onL = x == 0, onR = x == nx - 1, onB = q == 0, onT = q == ny - 1;
  if (onL || onR || onB || onT) {
    uint32_t unknown = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int sx = x - kCx[i], sy = q - kCy[i];
      if (sx < 0 || sx >= nx || sy < 0 || sy >= ny) {
        unknown |= 1u << i;
        g[i] = R(0);
      }
    }
    // eq. nes_2: one-sided normal differences at time t, the x normal first
    // (the vertical edges own the corners), then the y normal
    R dsum[3] = {R(0), R(0), R(0)};
    int nn = 0;
    if (onL || onR) {
      ++nn;
#pragma unroll
      for (int c = 0; c < 3; ++c) dsum[c] += normal_diff(mom[2][c], mxn[0][c], mxn[1][c], Ld.grad_order);
    }
    if (onB || onT) {
      ++nn;
#pragma unroll
      for (int c = 0; c < 3; ++c)
        dsum[c] += onB ? normal_diff(mom[2][c], mom[3][c], mom[4][c], Ld.grad_order)
                       : normal_diff(mom[2][c], mom[1][c], mom[0][c], Ld.grad_order);
    }
    R fac = R(Ld.gamma);
    if (nn == 2) fac *= Ld.corner_mode == 0 ? R(0.70710678118654752440) : R(0.5);
    const R beta = R(Ld.beta);
    M3<R> mc;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const R mp = mom[2][c] - fac * dsum[c];
      mc.v[c] = (R(1) - beta) * mp + beta * R(Ld.m0[c]);  // eq. nes_3
    }
    nsbc_assign_correct<R>(g, unknown, mc, rho0, b, Ld.corr_mode);
  }
  bgk<R>(g, rho0, b, omega);
}

// Moments of row q (window slot 2) at the two interior neighbours of an
// edge column, taken from the neighbouring lanes.
template <class R>
__device__ inline void ts_edge_moments(const R (&mom)[5][3], int lane, int dir, R (&mxn)[2][3]) {
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int c = 0; c < 3; ++c) mxn[d][c] = ts_shfl(mom[2][c], lane + (d + 1) * dir);
}

// One wavefront of the two-step sweep over output rows [y0, y0 + H), for
// wavefronts and bands that reach the lattice edges.
template <int S, int H, bool NTS>
__device__ inline void two_step_edge(const LatDesc& Ld, int parity, int X0) {
  using C = Codec<S>;
  using T = typename C::T;
  using R = typename C::R;
  const int nx = Ld.nx, ny = Ld.ny;
  const int lane = threadIdx.x & 63;
  const int x = X0 - 2 + lane;
  const bool xin = x >= 0 && x < nx;
  const bool out_lane = lane >= 2 && lane < 2 + TS_COLS && xin;

  // rows written (a2..b2), rows of level t + 1 and of level t they need
  const int a2 = blockIdx.y * H;
  const int b2 = min(a2 + H, ny);
  int a1 = a2 - 1, b1 = b2 + 1;
  if (b2 == ny) a1 = min(a1, ny - 3);
  if (a2 == 0) b1 = max(b1, 3);
  a1 = max(a1, 0);
  b1 = min(b1, ny);
  int a0 = a1 - 1, b0 = b1 + 1;
  if (b1 == ny) a0 = min(a0, ny - 3);
  if (a1 == 0) b0 = max(b0, 3);
  a0 = max(a0, 0);
  b0 = min(b0, ny);

  const T* __restrict__ A = static_cast<const T*>(buf_of(Ld, parity));
  T* __restrict__ B = static_cast<T*>(buf_of(Ld, parity ^ 1));
  const int pitch = Ld.pitch;
  const int64_t plane = Ld.plane;
  const R rho0 = R(Ld.rho0), omega = R(Ld.omega);
  const Base<R> base(Ld);
  // wavefronts whose level t + 1 columns (X0 - 1 .. X0 + 60) include an edge
  // column gather interior-neighbour moments
  const bool has_left = X0 == 0;
  const bool has_right = X0 - 1 <= nx - 1 && nx - 1 <= X0 + TS_COLS;

  const bool edge_wave = has_left || has_right;

  TsLevel<R> L1, L2;
  ts_init(L1);
  ts_init(L2);

  // row r of level t, loaded one iteration ahead (its loads are in flight
  // while row r - 1 is processed)
  T nxt[9];
  auto fetch = [&](int r, T (&dst)[9]) {
    if (xin && r < b0) {
      const int64_t idx = (int64_t)r * pitch + x;
#pragma unroll
      for (int i = 0; i < 9; ++i) dst[i] = A[i * plane + idx];
    }
  };
  fetch(a0, nxt);

  // iteration r takes source row r of level t; level t + 1 finalises row
  // r - 2, level t + 2 row r - 4
  for (int r = a0; r <= b2 + 3; ++r) {
    R v[9];
    const bool lv = xin && r < b0;
#pragma unroll
    for (int i = 0; i < 9; ++i) v[i] = lv ? C::dec(nxt[i], Ld.ds[i]) : R(0);
    fetch(r + 1, nxt);
    // the NSBC normal differences need source-row moments only near the
    // lattice edges
    ts_push_moments<R>(L1, v, rho0, base, lv && (edge_wave || r <= 2 || r >= ny - 3));

    // level t + 1, row q = r - 2
    const int q = r - 2;
    const bool v1 = xin && q >= a1 && q < b1;
    R u[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) u[i] = L1.full[i];
    ts_stream<R>(L1, v, lane);
    R mxn[2][3] = {{R(0), R(0), R(0)}, {R(0), R(0), R(0)}};
    if (has_left) ts_edge_moments<R>(L1.mom, lane, 1, mxn);
    if (has_right) {
      R mr[2][3];
      ts_edge_moments<R>(L1.mom, lane, -1, mr);
      if (x == nx - 1) {
#pragma unroll
        for (int d = 0; d < 2; ++d)
#pragma unroll
          for (int c = 0; c < 3; ++c) mxn[d][c] = mr[d][c];
      }
    }
    if (v1) {
      ts_finalise<R>(Ld, u, L1.mom, mxn, x, q, rho0, base, omega);
      // round through the codec as the single-step path's store and load do
#pragma unroll
      for (int i = 0; i < 9; ++i) u[i] = C::dec(C::enc(u[i], Ld.es[i]), Ld.ds[i]);
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) u[i] = R(0);
    }
    ts_push_moments<R>(L2, u, rho0, base, v1 && (edge_wave || q <= 2 || q >= ny - 3));

    // level t + 2, row p = r - 4
    const int p = r - 4;
    R w[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) w[i] = L2.full[i];
    ts_stream<R>(L2, u, lane);
    if (p >= a2 && p < b2) {
      R mxn2[2][3] = {{R(0), R(0), R(0)}, {R(0), R(0), R(0)}};
      if (has_left) ts_edge_moments<R>(L2.mom, lane, 1, mxn2);
      if (has_right) {
        R mr[2][3];
        ts_edge_moments<R>(L2.mom, lane, -1, mr);
        if (x == nx - 1) {
#pragma unroll
          for (int d = 0; d < 2; ++d)
#pragma unroll
            for (int c = 0; c < 3; ++c) mxn2[d][c] = mr[d][c];
        }
      }
      if (out_lane) {
        ts_finalise<R>(Ld, w, L2.mom, mxn2, x, p, rho0, base, omega);
        const int64_t idx = (int64_t)p * pitch + x;
#pragma unroll
        for (int i = 0; i < 9; ++i) put<NTS>(B + i * plane + idx, C::enc(w[i], Ld.es[i]));
      }
    }
  }
}

// Interior wavefront-band: every column X0 - 2 .. X0 + 61 and every row the
// band touches lie inside the lattice, at least one node away from the edges
// for level t + 1, so no NSBC node, edge test or moment window is needed.
template <int S, int H, bool NTS>
__device__ inline void two_step_interior(const LatDesc& Ld, int parity, int X0, int a2, int b2) {
  using C = Codec<S>;
  using T = typename C::T;
  using R = typename C::R;
  const int lane = threadIdx.x & 63;
  const int x = X0 - 2 + lane;
  const bool out_lane = lane >= 2 && lane < 2 + TS_COLS;
  const int a1 = a2 - 1, b1 = b2 + 1, a0 = a2 - 2, b0 = b2 + 2;
  const int last = b2 + 3;
  const T* __restrict__ A = static_cast<const T*>(buf_of(Ld, parity));
  T* __restrict__ B = static_cast<T*>(buf_of(Ld, parity ^ 1));
  const int pitch = Ld.pitch;
  const int64_t plane = Ld.plane;
  const R rho0 = R(Ld.rho0), omega = R(Ld.omega);
  const Base<R> base(Ld);

  TsLevel<R> L1, L2;
  ts_init(L1);
  ts_init(L2);
  // three rows of level t in flight: buffer k holds the rows r = a0 + k (mod 3)
  T buf[3][9];
  auto fetch = [&](int r, T (&dst)[9]) {
    if (r < b0) {
      const int64_t idx = (int64_t)r * pitch + x;
#pragma unroll
      for (int i = 0; i < 9; ++i) dst[i] = A[i * plane + idx];
    }
  };
  fetch(a0, buf[0]);
  fetch(a0 + 1, buf[1]);
  fetch(a0 + 2, buf[2]);
  auto row = [&](int r, T (&cur)[9]) {
    R v[9];
    const bool lv = r < b0;
#pragma unroll
    for (int i = 0; i < 9; ++i) v[i] = lv ? C::dec(cur[i], Ld.ds[i]) : R(0);
    fetch(r + 3, cur);
    const int q = r - 2;
    R u[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) u[i] = L1.full[i];
    ts_stream<R>(L1, v, lane);
    if (q >= a1 && q < b1) {
      bgk<R>(u, rho0, base, omega);
#pragma unroll
      for (int i = 0; i < 9; ++i) u[i] = C::dec(C::enc(u[i], Ld.es[i]), Ld.ds[i]);
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) u[i] = R(0);
    }
    const int p = r - 4;
    R w[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) w[i] = L2.full[i];
    ts_stream<R>(L2, u, lane);
    if (p >= a2 && p < b2 && out_lane) {
      bgk<R>(w, rho0, base, omega);
      const int64_t idx = (int64_t)p * pitch + x;
#pragma unroll
      for (int i = 0; i < 9; ++i) put<NTS>(B + i * plane + idx, C::enc(w[i], Ld.es[i]));
    }
  };
  for (int r = a0; r <= last; r += 3) {
    row(r, buf[0]);
    if (r + 1 <= last) row(r + 1, buf[1]);
    if (r + 2 <= last) row(r + 2, buf[2]);
  }
}

template <int S, int H, bool NTS>
__device__ inline void two_step_body(const LatDesc& Ld, int parity) {
  const int nx = Ld.nx, ny = Ld.ny;
  const int X0 = (blockIdx.x * TS_WAVES + (threadIdx.x >> 6)) * TS_COLS;
  if (X0 >= nx) return;  // the whole wavefront is past the lattice (no block-wide barrier follows)
  const int a2 = blockIdx.y * H;
  const int b2 = min(a2 + H, ny);
  const bool interior = X0 >= 2 && X0 + TS_COLS + 2 <= nx - 1 && a2 >= 2 && b2 <= ny - 2;
  if (interior) two_step_interior<S, H, NTS>(Ld, parity, X0, a2, b2);
  else two_step_edge<S, H, NTS>(Ld, parity, X0);
}

}  // namespace lbm
