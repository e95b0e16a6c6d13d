// lbm_twostep_lds.h -- two lattice steps per launch (t -> t + 2) with the
// intermediate level in LDS, for lattices with NSBC on all four edges
// (eqs. lbe_0, lbe_1, feq_1 in the bulk; eqs. nes_0..nes_4 on the edges).
//
// A block owns an output tile of 64 x TY nodes.  It first computes level
// t + 1 on the tile widened by a margin (2 columns each side; 1 row, or 2
// rows where the tile holds a lattice edge), pulling level t straight from
// HBM, and keeps those post-collision values in LDS; after one barrier it
// computes level t + 2 on the tile from LDS and stores it.  Only the tile is
// written, so the state crosses HBM about once per two steps (the margin is
// re-read from L2 by the neighbouring tiles).
//
// Per node the arithmetic is the single-step path's, in the same order, and
// level t + 1 is rounded through the storage codec exactly as a store and
// reload would: results are bit-identical to two single steps.
#pragma once

#include <type_traits>

#include "lbm_device.h"
#include "lbm_sweep.h"

namespace lbm {

constexpr int TL_TX = 64;             // output columns per tile
constexpr int TL_W = TL_TX + 4;       // LDS row: 2 margin columns each side

// Moments of lattice node (x, y) of level t (stored, decoded).
template <int S>
__device__ inline void tl_moments_global(const LatDesc& Ld, const typename Codec<S>::T* A, int x, int y,
                                         const Base<typename Codec<S>::R>& b, typename Codec<S>::R m[3]) {
  using C = Codec<S>;
  using R = typename C::R;
  R g[9];
  const int64_t idx = (int64_t)y * Ld.pitch + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) g[i] = C::dec(ldg(A + i * Ld.plane, (uint32_t)idx * (uint32_t)sizeof(typename C::T)), Ld.ds[i]);
  moments<R>(g, R(Ld.rho0), b, m[0], m[1], m[2]);
}

// Populations of node (x, y) whose pull source x - c_i lies outside the
// lattice (all four edges non-periodic): c_x = +1 at x = 0, c_x = -1 at
// x = nx - 1, and the same in y.  Non-zero exactly on boundary nodes.
__device__ inline uint32_t tl_unknown(int x, int y, int nx, int ny) {
  uint32_t u = 0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const bool out = (x == 0 && kCx[i] > 0) || (x == nx - 1 && kCx[i] < 0) || (y == 0 && kCy[i] > 0) ||
                     (y == ny - 1 && kCy[i] < 0);
    u |= out ? (1u << i) : 0u;
  }
  return u;
}

// NSBC's vector m_c of boundary node (x, y) (eqs. nes_2, nes_3); `mom(xx,
// yy, m)` returns the previous level's moments of any lattice node.  Same
// order as the edge kernel: the x normal first (the vertical edges own the
// corners), then the y normal.
template <class R, class MomFn>
__device__ inline M3<R> tl_predict(const LatDesc& Ld, int x, int y, const Base<R>& b, MomFn mom) {
  const int nx = Ld.nx, ny = Ld.ny;
  const bool onL = x == 0, onR = x == nx - 1, onB = y == 0, onT = y == ny - 1;
  R mb[3];
  mom(x, y, mb);
  R dsum[3] = {R(0), R(0), R(0)};
  int nn = 0;
  if (onL || onR) {
    const int d = onL ? 1 : -1;
    R m1[3], m2[3];
    mom(x + d, y, m1);
    mom(x + 2 * d, y, m2);
    ++nn;
#pragma unroll
    for (int c = 0; c < 3; ++c) dsum[c] += normal_diff(mb[c], m1[c], m2[c], Ld.grad_order);
  }
  if (onB || onT) {
    const int d = onB ? 1 : -1;
    R m1[3], m2[3];
    mom(x, y + d, m1);
    mom(x, y + 2 * d, m2);
    ++nn;
#pragma unroll
    for (int c = 0; c < 3; ++c) dsum[c] += normal_diff(mb[c], m1[c], m2[c], Ld.grad_order);
  }
  R fac = R(Ld.gamma);
  if (nn == 2) fac *= Ld.corner_mode == 0 ? R(0.70710678118654752440) : R(0.5);
  const R beta = R(Ld.beta);
  M3<R> mc;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const R mp = mb[c] - fac * dsum[c];
    mc.v[c] = (R(1) - beta) * mp + beta * R(Ld.m0[c]);
  }
  return mc;
}

// NSBC of boundary node (x, y): unknown populations already zeroed and
// flagged in `unknown`; m_c as tl_predict, then assignment and correction
// (eqs. nes_0, nes_1, nes_4).
template <class R, class MomFn>
__device__ inline void tl_nsbc(const LatDesc& Ld, R g[9], uint32_t unknown, int x, int y, R rho0, const Base<R>& b,
                               MomFn mom) {
  const M3<R> mc = tl_predict<R>(Ld, x, y, b, mom);
  nsbc_assign_correct<R>(g, unknown, mc, rho0, b, Ld.corr_mode);
}

// NT threads per block.  Level t + 1 is kept in LDS in the storage format
// (encoded exactly as a store would write it, decoded on every read), which
// halves the LDS of the 16-bit formats.  CM is the collision model, fixed at
// compile time (COLL_BGK or COLL_MRT).
// The level array of a two-step block, one allocation per kernel whichever
// path (tile or column march) takes it.
template <int S, int TY>
__device__ inline auto two_lds() -> typename Codec<S>::T (&)[9][TY + 4][TL_W] {
  __shared__ __attribute__((aligned(16))) typename Codec<S>::T a[9][TY + 4][TL_W];
  return a;
}

// part 2: only an edge tile (an inner tile's block leaves at once).
template <int S, int TY, int NT, bool NTS, int CM>
__device__ inline void two_step_tile(const LatDesc& Ld, int parity, int txi, int tyi, int part = 0) {
  using C = Codec<S>;
  using T = typename C::T;
  using R = typename C::R;
  constexpr int TH = TY + 4;  // LDS rows (margin of up to 2 each side)
  auto& lds = two_lds<S, TY>();

  const int nx = Ld.nx, ny = Ld.ny;
  const int x0 = txi * TL_TX, y0 = tyi * TY;
  const int tid = threadIdx.x;
  const bool edge_tile = x0 == 0 || x0 + TL_TX >= nx || y0 == 0 || y0 + TY >= ny;
  const int my = edge_tile ? 2 : 1;        // row margin of level t + 1
  const int ly0 = 2 - my;                  // first LDS row used
  const int rows1 = TY + 2 * my;           // level t + 1 rows computed
  const T* __restrict__ A = static_cast<const T*>(buf_of(Ld, parity));
  T* __restrict__ B = static_cast<T*>(buf_of(Ld, parity ^ 1));
  const int pitch = Ld.pitch;
  const int64_t plane = Ld.plane;
  const R rho0 = R(Ld.rho0), omega = R(Ld.omega);
  const Base<R> base(Ld);
  const OutPlanes<T> out(B, plane);

  // Inner tile: every level t + 1 node (rows y0 - 1 .. y0 + TY, columns
  // x0 - 2 .. x0 + 65) is an interior lattice node, so no pull leaves the
  // lattice and no NSBC node occurs: the loops drop those checks (same
  // arithmetic, same bits) and have trip counts known at compile time.
  const bool inner = x0 >= 3 && x0 + TL_TX + 3 <= nx && y0 >= 2 && y0 + TY + 2 <= ny;
  if (part == 2 && inner) return;
  // Inlined twice, with the base state's u_b = 0 flag a known constant in
  // each copy (the per-node arithmetic keeps only the branch that runs).
  auto inner_sweep = [&](const Base<R>& base) __attribute__((always_inline)) {
    constexpr int N1 = (TY + 2) * TL_W, N2 = TY * TL_TX;
    // per-plane base pointers (uniform) and 32-bit unsigned byte offsets (a
    // plane is below 4 GiB), so each access is a scalar base plus one vector
    // offset
#pragma unroll
    for (int it = 0; it < (N1 + NT - 1) / NT; ++it) {
      const int k = tid + it * NT;
      if (k < N1) {
        const int r = k / TL_W, cx = k - r * TL_W;
        const uint32_t idx = (uint32_t)((y0 - 1 + r) * pitch + (x0 - 2 + cx));
        // byte offsets of the source rows y + 1, y, y - 1; the x shift is a constant
        const uint32_t ro[3] = {(idx + (uint32_t)pitch) * (uint32_t)sizeof(T), idx * (uint32_t)sizeof(T),
                                (idx - (uint32_t)pitch) * (uint32_t)sizeof(T)};
        R g[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = C::raw(ldg(A + i * plane, ro[1 + kCy[i]] - kCx[i] * (int)sizeof(T)));
        collide_stored<S, CM>(Ld, g, rho0, base, omega);
#pragma unroll
        for (int i = 0; i < 9; ++i) lds[i][1 + r][cx] = C::raw_enc(g[i]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < (N2 + NT - 1) / NT; ++it) {
      const int k = tid + it * NT;
      if (k < N2) {
        const int r = k / TL_TX, cx = k - r * TL_TX;
        R g[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = C::raw(lds[i][r + 2 - kCy[i]][cx + 2 - kCx[i]]);
        collide_stored<S, CM>(Ld, g, rho0, base, omega);
        const uint32_t off = (uint32_t)((y0 + r) * pitch + (x0 + cx)) * (uint32_t)sizeof(T);
#pragma unroll
        for (int i = 0; i < 9; ++i) out.template put<NTS>(i, off, C::raw_enc(g[i]));
      }
    }
  };
  if (inner) {
    Base<R> b = base;
    if (base.zero) {
      b.zero = true;
      inner_sweep(b);
    } else {
      b.zero = false;
      inner_sweep(b);
    }
    return;
  }

  // ---- level t + 1 on lattice rows y0 - my .. y0 + TY + my - 1, columns x0 - 2 .. x0 + 65.
  // A population whose pull source lies outside the lattice is unknown (set
  // by the node's position alone); the others are pulled from sources clamped
  // into the lattice (a clamped source is only ever an unknown one), so every
  // lane runs the same loads and selects instead of branching per population.
  for (int k = tid; k < rows1 * TL_W; k += NT) {
    const int r = k / TL_W, cx = k - r * TL_W;
    const int x = x0 - 2 + cx, y = y0 - my + r;
    if (x < 0 || x >= nx || y < 0 || y >= ny) continue;
    const uint32_t unknown = tl_unknown(x, y, nx, ny);
    // source column for c_x = -1, 0, +1 and byte offset of the source row for c_y = -1, 0, +1
    const int sxs[3] = {min(x + 1, nx - 1), x, max(x - 1, 0)};
    const uint32_t srow[3] = {(uint32_t)(min(y + 1, ny - 1) * pitch), (uint32_t)(y * pitch),
                              (uint32_t)(max(y - 1, 0) * pitch)};
    R g[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const R v = C::raw(ldg(A + i * plane, (srow[1 + kCy[i]] + (uint32_t)sxs[1 + kCx[i]]) * (uint32_t)sizeof(T)));
      g[i] = (unknown >> i) & 1u ? R(0) : v;
    }
    // a boundary node decodes, takes NSBC and collide, and encodes; an
    // interior one collides on its values as stored (as the single-step
    // edge and bulk kernels do)
    if (unknown) {
      if constexpr (C::scaled) {
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] *= Ld.ds[i];
      }
      auto mom = [&](int xx, int yy, R m[3]) { tl_moments_global<S>(Ld, A, xx, yy, base, m); };
      tl_nsbc<R>(Ld, g, unknown, x, y, rho0, base, mom);
      collide<R, CM>(Ld, g, rho0, base, omega);
      if constexpr (C::scaled) {
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] *= Ld.es[i];
      }
    } else {
      collide_stored<S, CM>(Ld, g, rho0, base, omega);
    }
    // encoded as the single-step path's store would write it
#pragma unroll
    for (int i = 0; i < 9; ++i) lds[i][ly0 + r][cx] = C::raw_enc(g[i]);
  }
  __syncthreads();

  // ---- level t + 2 on the tile, from LDS (lattice node (x, y) at lds[.][y - y0 + 2][x - x0 + 2])
  auto mom1 = [&](int xx, int yy, R m[3]) {
    R q[9];
    const int lx = xx - x0 + 2, ly = yy - y0 + 2;
#pragma unroll
    for (int i = 0; i < 9; ++i) q[i] = C::dec(lds[i][ly][lx], Ld.ds[i]);
    moments<R>(q, rho0, base, m[0], m[1], m[2]);
  };
  for (int k = tid; k < TY * TL_TX; k += NT) {
    const int r = k / TL_TX, cx = k - r * TL_TX;
    const int x = x0 + cx, y = y0 + r;
    if (x >= nx || y >= ny) continue;
    const uint32_t unknown = tl_unknown(x, y, nx, ny);
    const int lxs[3] = {min(x + 1, nx - 1) - x0 + 2, cx + 2, max(x - 1, 0) - x0 + 2};
    const int lys[3] = {min(y + 1, ny - 1) - y0 + 2, r + 2, max(y - 1, 0) - y0 + 2};
    R g[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const R v = C::raw(lds[i][lys[1 + kCy[i]]][lxs[1 + kCx[i]]]);
      g[i] = (unknown >> i) & 1u ? R(0) : v;
    }
    if (unknown) {
      if constexpr (C::scaled) {
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] *= Ld.ds[i];
      }
      tl_nsbc<R>(Ld, g, unknown, x, y, rho0, base, mom1);
      collide<R, CM>(Ld, g, rho0, base, omega);
      if constexpr (C::scaled) {
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] *= Ld.es[i];
      }
    } else {
      collide_stored<S, CM>(Ld, g, rho0, base, omega);
    }
    const uint32_t off = (uint32_t)(y * pitch + x) * (uint32_t)sizeof(T);
#pragma unroll
    for (int i = 0; i < 9; ++i) out.template put<NTS>(i, off, C::raw_enc(g[i]));
  }
}

}  // namespace lbm

namespace lbm {

// ------------------------------------------------------------------ three steps per launch
// t -> t + 3 with levels t + 1 and t + 2 in LDS.  The output tile is 64 x TY
// at (x0, y0) = (min(64 txi, nx - 64), min(TY tyi, ny - TY)): every tile is
// whole (the last tile of a row or column overlaps its neighbour and writes
// the same values), so a lattice edge that crosses a level's region has the
// two nodes NSBC reads inward of it inside the previous level's region.
// Level t + 1 covers columns x0 - 2 .. x0 + 65 and rows y0 - 2 .. y0 + TY + 1
// (lds1), level t + 2 columns x0 - 1 .. x0 + 64 and rows y0 - 1 .. y0 + TY
// (lds2), level t + 3 the tile.  Per node the arithmetic is the single-step
// path's and each level is rounded through the storage codec: bit-identical
// to three single steps.
constexpr int T3_W1 = TL_TX + 4;
constexpr int T3_W2 = TL_TX + 2;

// First thread of the waves that run one iteration fewer of a sweep over n
// nodes by nt threads (0 when every wave runs the same number).
__host__ __device__ constexpr int light_waves_start(int n, int nt) {
  return n % nt == 0 ? 0 : ((n % nt + 63) / 64 * 64) % nt;
}

// The two level arrays of a three-step block, one allocation per kernel
// whichever path (tile or column march) takes them.
template <int S, int TY>
__device__ inline auto three_lds1() -> typename Codec<S>::T (&)[9][TY + 4][T3_W1] {
  __shared__ __attribute__((aligned(16))) typename Codec<S>::T a[9][TY + 4][T3_W1];
  return a;
}
template <int S, int TY>
__device__ inline auto three_lds2() -> typename Codec<S>::T (&)[9][TY + 2][T3_W2] {
  __shared__ __attribute__((aligned(16))) typename Codec<S>::T a[9][TY + 2][T3_W2];
  return a;
}

template <int S, int TY>
constexpr int three_step_lds_bytes() {
  return 9 * ((TY + 4) * T3_W1 + (TY + 2) * T3_W2) * (int)sizeof(typename Codec<S>::T);
}

// LDS of the closure phases of an edge tile (CL), one edge segment at a
// time: the segment's strip features [3][CL_STRIP][9] (fp32), then per
// network wave its 16 input rows [16][XS] (reused for the second hidden
// layer) and first hidden layer [16][HS] (bf16).  They reuse a level array
// not in use at the time when at least two waves' worth fits in the
// smaller one, else take LDS of their own; the outputs and amplitudes of a
// level's edge nodes, [edge nodes][4] fp32, have LDS of their own.
constexpr int CL_STRIP = TL_TX + 6;  // a segment's nodes plus one beyond each end, at most
constexpr int CL_FEAT_BYTES = (3 * CL_STRIP * NODE_FEAT * 4 + 15) / 16 * 16;
constexpr int CL_WAVE_BYTES = 16 * (mlp::XS + mlp::HS) * 2;

template <int S, int TY, int NT>
constexpr int cl_fit_waves() {
  constexpr int w = (9 * (TY + 2) * T3_W2 * (int)sizeof(typename Codec<S>::T) - CL_FEAT_BYTES) / CL_WAVE_BYTES;
  return w < 0 ? 0 : (w > 4 ? 4 : (w > NT / 64 ? NT / 64 : w));
}
template <int S, int TY, int NT>
constexpr bool cl_own_lds() {
  return cl_fit_waves<S, TY, NT>() < 2;
}
template <int S, int TY, int NT>
constexpr int cl_waves() {
  return cl_own_lds<S, TY, NT>() ? (NT / 64 < 4 ? NT / 64 : 4) : cl_fit_waves<S, TY, NT>();
}
// lattice-edge nodes of a level's region, at most (both columns and both rows of level t + 1's)
template <int TY>
constexpr int cl_max_edge() {
  return 2 * (TY + 4) + 2 * T3_W1;
}
// (plus the network's biases and input normalisation, staged once per tile)
template <int S, int TY, int NT, bool CL>
constexpr int three_step_cl_lds_bytes() {
  return !CL ? 0
             : cl_max_edge<TY>() * 16 + mlp::PARAM_BYTES +
                   (cl_own_lds<S, TY, NT>() ? CL_FEAT_BYTES + cl_waves<S, TY, NT>() * CL_WAVE_BYTES : 0);
}

// Lattice-edge node region of a level (rows ry0 .. ry0 + rh - 1, columns
// rx0 .. rx0 + rw - 1, clipped to the lattice): bounds and the counts of
// column nodes (x = 0 and x = nx - 1) and of the remaining row nodes.
__device__ inline void tl_edge_count(int nx, int ny, int rx0, int ry0, int rw, int rh, int& xl, int& xh, int& yl,
                                     int& yh, int& ncol, int& nrow) {
  xl = max(rx0, 0);
  xh = min(rx0 + rw - 1, nx - 1);
  yl = max(ry0, 0);
  yh = min(ry0 + rh - 1, ny - 1);
  const int left = xl == 0, right = xh == nx - 1;
  ncol = (left + right) * (yh - yl + 1);        // nodes of the x = 0 and x = nx - 1 columns
  const int cx0 = xl + left, cx1 = xh - right;  // row nodes not already in those columns
  nrow = ((yl == 0) + (yh == ny - 1)) * max(0, cx1 - cx0 + 1);
}

// The learned closure for one level of a multi-step edge tile: the
// network's correction of m_c for every lattice-edge node of the level's
// region with a single normal, from the previous level (the edge kernel's
// closure applied per level: same inputs, same arithmetic).  The previous
// level's population i of node (x, y) is prev[i ps_i + (y - oy) ps_y + (x -
// ox)] (the state in HBM, or a level array in LDS).  One edge segment of the
// region at a time (left column, right column, bottom row, top row, numbered
// as the edge pass numbers its nodes): the strip features of the segment
// (depth 0..2 along the inward normal, one node beyond each end) into LDS,
// then waves 0..CLW-1 each build the input rows of 16 nodes and run the
// network on them.  Outputs land in cl_y[4 e + 0..2] and the amplitude (0:
// NSBC's m_c stays) in cl_y[4 e + 3] for edge node e.  Called by the whole
// block.  An edge tile runs this code once per level and tile, not in a hot
// loop, so it is kept compact (one copy for the three levels, loops rolled):
// its instructions come from L2 on every tile, and their count, not the
// arithmetic, sets its time.
template <int S, int CLW>
__device__ inline __attribute__((always_inline)) void closure_level(const LatDesc& Ld, int rx0, int ry0, int rw, int rh,
                                           const typename Codec<S>::T* prev, int64_t ps_i, int ps_y, int ox, int oy,
                                           char* scr, float* cl_y, int nt, const mlp::Params& par) {
  using C = Codec<S>;
  using R = typename C::R;
  const int nx = Ld.nx, ny = Ld.ny;
  const int tid = threadIdx.x;
  const mlp::Net& net = *static_cast<const mlp::Net*>(Ld.net);
  const Base<R> b(Ld);
  const R rho0 = R(Ld.rho0);
  const R ref[3] = {R(Ld.m0[0]), R(Ld.m0[1]), R(Ld.m0[2])};
  const float rho0f = float(Ld.rho0), omegaf = float(Ld.omega);
  auto pops = [&](int x, int y, R g[9]) {
    const int64_t idx = (int64_t)(y - oy) * ps_y + (x - ox);
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i] = C::dec(prev[i * ps_i + idx], Ld.ds[i]);
  };
  int xl, xh, yl, yh, ncol, nrow;
  tl_edge_count(nx, ny, rx0, ry0, rw, rh, xl, xh, yl, yh, ncol, nrow);
  const int left = xl == 0, right = xh == nx - 1, hcol = yh - yl + 1;
  const int cx0 = xl + left, cw = max(0, (xh - right) - cx0 + 1);
  float* feat = reinterpret_cast<float*>(scr);
  const int w = tid >> 6, l = tid & 63;
  mlp::bf16* X = reinterpret_cast<mlp::bf16*>(scr + CL_FEAT_BYTES + w * CL_WAVE_BYTES);
  mlp::bf16* H1 = X + 16 * mlp::XS;
  for (int sg = 0; sg < 4; ++sg) {
    // segment sg: left column, right column, bottom row, top row
    const bool vert = sg < 2;
    const bool present = sg == 0 ? left : (sg == 1 ? right : (sg == 2 ? yl == 0 && cw > 0 : yh == ny - 1 && cw > 0));
    if (!present) continue;
    const int base_e = sg == 0 ? 0 : (sg == 1 ? left * hcol : (sg == 2 ? ncol : ncol + (yl == 0) * cw));
    const int len = vert ? hcol : cw, ta = vert ? yl : cx0, ntan = vert ? ny : nx;
    const int enx = sg == 0 ? -1 : (sg == 1 ? 1 : 0), eny = sg == 2 ? -1 : (sg == 3 ? 1 : 0);
    // node of the segment's strip at depth d and tangential coordinate tc
    auto strip_xy = [&](int d, int tc, int& x, int& y) {
      x = vert ? (enx < 0 ? d : nx - 1 - d) : tc;
      y = vert ? tc : (eny < 0 ? d : ny - 1 - d);
    };
    // strip features: feat[(d CL_STRIP + j) 9 + q] at tangential coordinate ta - 1 + j
    for (int i = tid; i < 3 * (len + 2); i += nt) {
      const int d = i / (len + 2), j = i - d * (len + 2), tc = ta - 1 + j;
      if (tc < 0 || tc >= ntan) continue;
      int x, y;
      strip_xy(d, tc, x, y);
      R g[9];
      pops(x, y, g);
      float f[NODE_FEAT];
      strip_node_features<R>(g, rho0, b, ref, enx, eny, f);
#pragma unroll
      for (int q = 0; q < NODE_FEAT; ++q) feat[(d * CL_STRIP + j) * NODE_FEAT + q] = f[q];
    }
    __syncthreads();
    if (w < CLW) {
      // lane l: node r = l % 16 of the group and inputs q = 4 qq + c of its row (c = l / 16), so
      // that every lane takes the same path through the row; the node's amplitude and m_c are
      // formed by each of its four lanes
      const int r = l & 15, c = l >> 4;
      // the tangent t = (-n_y, n_x) runs along increasing tc on the right and bottom edges
      const int tsign = (sg == 1 || sg == 2) ? 1 : -1;
      for (int g0 = 16 * w; g0 < len; g0 += 16 * CLW) {
        const int i = g0 + r, tc = ta + i;
        const bool valid = i < len;
        const bool eligible = valid && (!vert || (tc >= 1 && tc <= ny - 2));
        const int ic = min(i, len - 1);  // a strip position inside the segment for idle lanes
        // unscaled features of strip node j = 3 d + k + 1, s(d, k) = b - d n + k t
        auto fv = [&](int jj, int q) {
          const int d = jj / 3, k = jj - 3 * d - 1;
          return feat[(d * CL_STRIP + ic + 1 + tsign * k) * NODE_FEAT + q];
        };
        // amplitude and regime gate first: a group without a gated node keeps NSBC's m_c for all
        // of its nodes (amplitude 0) and skips the network
        float A = 0.f, inv = 0.f;
        bool gated = false;
        if (eligible) {
          A = strip_amplitude(fv, rho0f);
          inv = amplitude_inverse(A);
          auto scaled = [&](int jj, int q) { return fv(jj, q) * inv; };
          gated = vortical_row(scaled, rho0f, net.kmin);
        }
        if (c == 0 && valid) cl_y[4 * (base_e + i) + 3] = gated ? A : 0.f;
        if (__ballot(gated) == 0) continue;              // wave-uniform
        float dmc[3] = {0.f, 0.f, 0.f}, refn[3] = {0.f, 0.f, 0.f};
        if (eligible) {
          // inputs 82..86: m_c - m0 and m0 in the edge frame
          int x, y;
          strip_xy(0, tc, x, y);
          auto mom = [&](int xx, int yy, R m[3]) {
            R q[9];
            pops(xx, yy, q);
            moments<R>(q, rho0, b, m[0], m[1], m[2]);
          };
          const M3<R> mc = tl_predict<R>(Ld, x, y, b, mom);
          normal_frame_diff<R>(mc.v, ref, enx, eny, dmc);
          to_normal_frame<R>(ref, b, enx, eny, refn);
        }
        mlp::bf16* row = X + r * mlp::XS;
#pragma unroll 4
        for (int qq = 0; qq < mlp::IN / 4; ++qq) {
          const int q = 4 * qq + c;
          // input_value(q, ...) with the choice made by selects
          const int qs = min(q, F_STRIP - 1);
          const float strip = fv(qs / NODE_FEAT, qs % NODE_FEAT) * inv;
          const int m = min(max(q - F_MC, 0), 2), u = min(max(q - F_UREF, 0), 1);
          const float dm = (m == 0 ? dmc[0] : (m == 1 ? dmc[1] : dmc[2])) * inv;
          const float ur = u == 0 ? refn[1] : refn[2];
          const float v = q < F_STRIP ? strip : (q == F_OMEGA ? omegaf : (q < F_UREF ? dm : (q < mlp::NFEAT ? ur : 0.f)));
          row[q] = eligible ? normalised_input(par.mean, par.inv_std, q, v) : (mlp::bf16)0.f;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_s_waitcnt(0);
        mlp::f32x4 yv;
        mlp::forward16(par, X, H1, X, yv);
        const int col = l & 15;
        if (col < 3) {
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int node = g0 + 4 * (l >> 4) + rr;
            if (node < len) cl_y[4 * (base_e + node) + col] = yv[rr];
          }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_s_waitcnt(0);
      }
    }
    __syncthreads();
  }
}

// `part` selects the tiles a launch updates: 0 every tile, 1 the inner tiles
// only, 2 the edge tiles only (a tile of the other kind returns before any
// barrier); a lattice on the learned closure runs its edge tiles with CL in
// one launch and its inner tiles without in another.
// part: 0 the tile, 1 only an inner tile, 2 only an edge tile.
template <int S, int TY, int NT, bool NTS, int CM, bool CL = false>
__device__ inline void three_step_tile(const LatDesc& Ld, int parity, int txi, int tyi, int part = 0) {
  using C = Codec<S>;
  using T = typename C::T;
  using R = typename C::R;
  auto& lds1 = three_lds1<S, TY>();
  auto& lds2 = three_lds2<S, TY>();
  constexpr int CLW = cl_waves<S, TY, NT>();
  constexpr bool CL_OWN = CL && cl_own_lds<S, TY, NT>();
  __shared__ __attribute__((aligned(16))) char cl_own[CL_OWN ? CL_FEAT_BYTES + CLW * CL_WAVE_BYTES : 16];
  __shared__ float cl_y[CL ? cl_max_edge<TY>() : 1][4];
  __shared__ __attribute__((aligned(16))) char cl_par[CL ? mlp::PARAM_BYTES : 16];

  const int nx = Ld.nx, ny = Ld.ny;
  const int x0 = min(txi * TL_TX, nx - TL_TX), y0 = min(tyi * TY, ny - TY);
  // a last tile moved back to end at the lattice edge stores only the nodes
  // its neighbour does not (the overlap holds the same values in both)
  const int xo = txi * TL_TX, yo = tyi * TY;
  const int tid = threadIdx.x;
  const T* __restrict__ A = static_cast<const T*>(buf_of(Ld, parity));
  T* __restrict__ B = static_cast<T*>(buf_of(Ld, parity ^ 1));
  const int pitch = Ld.pitch;
  const int64_t plane = Ld.plane;
  const R rho0 = R(Ld.rho0), omega = R(Ld.omega);
  const Base<R> base(Ld);

  // Inner tile: every level t + 1 node and its pull sources lie inside the
  // lattice and away from its edges: no clamps, no NSBC.
  const bool inner = x0 >= 3 && x0 + TL_TX + 3 <= nx && y0 >= 3 && y0 + TY + 3 <= ny;
  if ((part == 1 && !inner) || (part == 2 && inner)) return;
  auto interior_node = [&](int x, int y) { return x >= 1 && x <= nx - 2 && y >= 1 && y <= ny - 2; };

  // One sweep per level over the level's whole region, its iterations
  // unrolled.  In an edge tile (edge = true) every node of the region runs the
  // interior update, a node off the lattice or on its edge on sources clamped
  // into the lattice, and only the lattice's interior nodes keep their result;
  // the lattice-edge nodes follow in edge_pass.  Every lane thus issues the
  // same unconditional loads, as in an inner tile.
  auto level1 = [&](const Base<R>& b, auto edge) __attribute__((always_inline)) {
    constexpr bool E = decltype(edge)::value;
    constexpr int N1 = (TY + 4) * T3_W1;
#pragma unroll
    for (int it = 0; it < (N1 + NT - 1) / NT; ++it) {
      const int k = tid + it * NT;
      if (k < N1) {
        const int r = k / T3_W1, cx = k - r * T3_W1;
        int x = x0 - 2 + cx, y = y0 - 2 + r;
        bool keep = true;
        if constexpr (E) {
          keep = interior_node(x, y);
          x = min(max(x, 1), nx - 2);
          y = min(max(y, 1), ny - 2);
        }
        // per-plane base pointers (uniform) and 32-bit unsigned byte offsets
        // (a plane is below 4 GiB): a scalar base plus one vector offset
        const uint32_t idx = (uint32_t)(y * pitch + x);
        const uint32_t ro[3] = {(idx + (uint32_t)pitch) * (uint32_t)sizeof(T), idx * (uint32_t)sizeof(T),
                                (idx - (uint32_t)pitch) * (uint32_t)sizeof(T)};
        R g[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = C::raw(ldg(A + i * plane, ro[1 + kCy[i]] - kCx[i] * (int)sizeof(T)));
        collide_stored<S, CM>(Ld, g, rho0, b, omega);
        if (keep) {
#pragma unroll
          for (int i = 0; i < 9; ++i) lds1[i][r][cx] = C::raw_enc(g[i]);
        }
      }
    }
  };
  // (LDS reads of a dropped node stay inside the arrays; its values are unused.)
  auto level2 = [&](const Base<R>& b, auto edge) __attribute__((always_inline)) {
    constexpr bool E = decltype(edge)::value;
    constexpr int N2 = (TY + 2) * T3_W2;
#pragma unroll
    for (int it = 0; it < (N2 + NT - 1) / NT; ++it) {
      const int k = tid + it * NT;
      if (k < N2) {
        const int r = k / T3_W2, cx = k - r * T3_W2;
        R g[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = C::raw(lds1[i][r + 1 - kCy[i]][cx + 1 - kCx[i]]);
        collide_stored<S, CM>(Ld, g, rho0, b, omega);
        if (!E || interior_node(x0 - 1 + cx, y0 - 1 + r)) {
#pragma unroll
          for (int i = 0; i < 9; ++i) lds2[i][r][cx] = C::raw_enc(g[i]);
        }
      }
    }
  };
  const OutPlanes<T> out(B, plane);
  // store of decoded values (an edge node's) and of values as stored (an interior node's)
  auto store = [&](int x, int y, const R g[9]) {
    const uint32_t off = (uint32_t)(y * pitch + x) * (uint32_t)sizeof(T);
#pragma unroll
    for (int i = 0; i < 9; ++i) out.template put<NTS>(i, off, C::enc(g[i], Ld.es[i]));
  };
  auto store_raw = [&](int x, int y, const R s[9]) {
    const uint32_t off = (uint32_t)(y * pitch + x) * (uint32_t)sizeof(T);
#pragma unroll
    for (int i = 0; i < 9; ++i) out.template put<NTS>(i, off, C::raw_enc(s[i]));
  };
  auto level3 = [&](const Base<R>& b, auto edge) __attribute__((always_inline)) {
    constexpr bool E = decltype(edge)::value;
    constexpr int N3 = TY * TL_TX;
#pragma unroll
    for (int it = 0; it < (N3 + NT - 1) / NT; ++it) {
      const int k = tid + it * NT;
      if (k < N3) {
        const int r = k / TL_TX, cx = k - r * TL_TX;
        R g[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = C::raw(lds2[i][r + 1 - kCy[i]][cx + 1 - kCx[i]]);
        collide_stored<S, CM>(Ld, g, rho0, b, omega);
        if (!E || (interior_node(x0 + cx, y0 + r) && x0 + cx >= xo && y0 + r >= yo)) store_raw(x0 + cx, y0 + r, g);
      }
    }
  };
  if (inner) {
    // inlined twice, with the base state's u_b = 0 flag a known constant in
    // each copy, so the per-node arithmetic carries only the branch that runs
    // (the operations and their order are unchanged)
    auto sweep = [&](const Base<R>& b) __attribute__((always_inline)) {
      level1(b, std::false_type{});
      __syncthreads();
      level2(b, std::false_type{});
      __syncthreads();
      level3(b, std::false_type{});
    };
    Base<R> b = base;
    if (base.zero) {
      b.zero = true;
      sweep(b);
    } else {
      b.zero = false;
      sweep(b);
    }
    return;
  }

  // ---- edge tiles.  After each level's sweep, the region's lattice-edge
  // nodes are gathered into consecutive lanes, so that NSBC runs on full
  // wavefronts instead of one lane per row, starting at the first wave that
  // ran one iteration fewer of the sweep.  The per-node arithmetic is the
  // single-step path's, so the results do not change.
  const Base<R>& b = base;
  // region of a level: lattice rows ry0 .. ry0 + rh - 1, columns rx0 .. rx0 + rw - 1
  auto edge_count = [&](int rx0, int ry0, int rw, int rh, int& xl, int& xh, int& yl, int& yh, int& ncol, int& nrow) {
    tl_edge_count(nx, ny, rx0, ry0, rw, rh, xl, xh, yl, yh, ncol, nrow);
  };
  // lattice-edge node number e of a region (left column, right column, then bottom row, top row)
  auto edge_node = [&](int e, int xl, int xh, int yl, int yh, int ncol, int& x, int& y) {
    const int hcol = yh - yl + 1;
    const int left = xl == 0, right = xh == nx - 1;
    if (e < ncol) {
      const bool first = left && e < hcol;
      x = first ? 0 : nx - 1;
      y = yl + (first ? e : e - left * hcol);
      return;
    }
    e -= ncol;
    const int cx0 = xl + left, cw = (xh - right) - cx0 + 1;
    const bool bottom = yl == 0 && e < cw;
    y = bottom ? 0 : ny - 1;
    x = cx0 + (bottom ? e : e - (yl == 0) * cw);
  };
  // edge-pass lane of this thread for a sweep over N nodes
  auto edge_lane = [&](int N) { return (tid + NT - light_waves_start(N, NT)) % NT; };

  // m_c of edge node e at (x, y), with the closure's correction (CL)
  auto edge_mc = [&](int e, int x, int y, auto mom) __attribute__((always_inline)) {
    M3<R> mc = tl_predict<R>(Ld, x, y, b, mom);
    if constexpr (CL) {
      const float amp = cl_y[e][3];
      float dl[3];
      const int enx = x == 0 ? -1 : (x == nx - 1 ? 1 : 0), eny = y == 0 ? -1 : (y == ny - 1 ? 1 : 0);
      if (amp > 0.f &&
          closure_delta(*static_cast<const mlp::Net*>(Ld.net), cl_y[e][0], cl_y[e][1], cl_y[e][2], amp, enx, eny, dl)) {
#pragma unroll
        for (int c = 0; c < 3; ++c) mc.v[c] += R(dl[c]);
      }
    }
    return mc;
  };
  // the network's parameters in LDS (CL; read after the first closure phase's barrier)
  mlp::Params par{};
  if constexpr (CL) par = mlp::stage_params(*static_cast<const mlp::Net*>(Ld.net), cl_par, tid, NT);
  // the closure phases of a level (CL): region, previous level (base,
  // strides, origin) and scratch (the level arrays not in use, or LDS of
  // their own)
  auto closure = [&](int rx0, int ry0, int rw, int rh, const T* prev, int64_t ps_i, int ps_y, int ox, int oy,
                     int level) __attribute__((always_inline)) {
    if constexpr (CL) {
      char* scr = CL_OWN ? cl_own
                         : (level == 3 ? reinterpret_cast<char*>(&lds1[0][0][0]) : reinterpret_cast<char*>(&lds2[0][0][0]));
      closure_level<S, CLW>(Ld, rx0, ry0, rw, rh, prev, ps_i, ps_y, ox, oy, scr, &cl_y[0][0], NT, par);
    }
  };

  // ---- level t + 1 from HBM
  auto mom0 = [&](int xx, int yy, R m[3]) { tl_moments_global<S>(Ld, A, xx, yy, b, m); };
  closure(x0 - 2, y0 - 2, T3_W1, TY + 4, A, plane, pitch, 0, 0, 1);
  level1(b, std::true_type{});
  {
    int xl, xh, yl, yh, ncol, nrow;
    edge_count(x0 - 2, y0 - 2, T3_W1, TY + 4, xl, xh, yl, yh, ncol, nrow);
    for (int e = edge_lane((TY + 4) * T3_W1); e < ncol + nrow; e += NT) {
      int x, y;
      edge_node(e, xl, xh, yl, yh, ncol, x, y);
      // sources clamped into the lattice (a clamped source is only ever an unknown population's)
      const uint32_t unknown = tl_unknown(x, y, nx, ny);
      const int sxs[3] = {min(x + 1, nx - 1), x, max(x - 1, 0)};
      const uint32_t srow[3] = {(uint32_t)(min(y + 1, ny - 1) * pitch), (uint32_t)(y * pitch),
                                (uint32_t)(max(y - 1, 0) * pitch)};
      R g[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const R v = C::dec(ldg(A + i * plane, (srow[1 + kCy[i]] + (uint32_t)sxs[1 + kCx[i]]) * (uint32_t)sizeof(T)), Ld.ds[i]);
        g[i] = (unknown >> i) & 1u ? R(0) : v;
      }
      nsbc_assign_correct<R>(g, unknown, edge_mc(e, x, y, mom0), rho0, b, Ld.corr_mode);
      collide<R, CM>(Ld, g, rho0, b, omega);
#pragma unroll
      for (int i = 0; i < 9; ++i) lds1[i][y - y0 + 2][x - x0 + 2] = C::enc(g[i], Ld.es[i]);
    }
  }
  __syncthreads();

  // ---- level t + 2 from lds1 (lattice node (x, y) at lds1[.][y - y0 + 2][x - x0 + 2])
  {
    auto pops1 = [&](int xx, int yy, R q[9]) {
      const int lx = xx - x0 + 2, ly = yy - y0 + 2;
#pragma unroll
      for (int i = 0; i < 9; ++i) q[i] = C::dec(lds1[i][ly][lx], Ld.ds[i]);
    };
    auto mom1 = [&](int xx, int yy, R m[3]) {
      R q[9];
      pops1(xx, yy, q);
      moments<R>(q, rho0, b, m[0], m[1], m[2]);
    };
    closure(x0 - 1, y0 - 1, T3_W2, TY + 2, &lds1[0][0][0], (TY + 4) * T3_W1, T3_W1, x0 - 2, y0 - 2, 2);
    level2(b, std::true_type{});
    int xl, xh, yl, yh, ncol, nrow;
    edge_count(x0 - 1, y0 - 1, T3_W2, TY + 2, xl, xh, yl, yh, ncol, nrow);
    for (int e = edge_lane((TY + 2) * T3_W2); e < ncol + nrow; e += NT) {
      int x, y;
      edge_node(e, xl, xh, yl, yh, ncol, x, y);
      const uint32_t unknown = tl_unknown(x, y, nx, ny);
      const int lxs[3] = {min(x + 1, nx - 1) - x0 + 2, x - x0 + 2, max(x - 1, 0) - x0 + 2};
      const int lys[3] = {min(y + 1, ny - 1) - y0 + 2, y - y0 + 2, max(y - 1, 0) - y0 + 2};
      R g[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const R v = C::dec(lds1[i][lys[1 + kCy[i]]][lxs[1 + kCx[i]]], Ld.ds[i]);
        g[i] = (unknown >> i) & 1u ? R(0) : v;
      }
      nsbc_assign_correct<R>(g, unknown, edge_mc(e, x, y, mom1), rho0, b, Ld.corr_mode);
      collide<R, CM>(Ld, g, rho0, b, omega);
#pragma unroll
      for (int i = 0; i < 9; ++i) lds2[i][y - y0 + 1][x - x0 + 1] = C::enc(g[i], Ld.es[i]);
    }
  }
  __syncthreads();

  // ---- level t + 3 on the tile from lds2 (lattice node (x, y) at lds2[.][y - y0 + 1][x - x0 + 1])
  {
    auto pops2 = [&](int xx, int yy, R q[9]) {
      const int lx = xx - x0 + 1, ly = yy - y0 + 1;
#pragma unroll
      for (int i = 0; i < 9; ++i) q[i] = C::dec(lds2[i][ly][lx], Ld.ds[i]);
    };
    auto mom2 = [&](int xx, int yy, R m[3]) {
      R q[9];
      pops2(xx, yy, q);
      moments<R>(q, rho0, b, m[0], m[1], m[2]);
    };
    closure(x0, y0, TL_TX, TY, &lds2[0][0][0], (TY + 2) * T3_W2, T3_W2, x0 - 1, y0 - 1, 3);
    level3(b, std::true_type{});
    int xl, xh, yl, yh, ncol, nrow;
    edge_count(x0, y0, TL_TX, TY, xl, xh, yl, yh, ncol, nrow);
    for (int e = edge_lane(TY * TL_TX); e < ncol + nrow; e += NT) {
      int x, y;
      edge_node(e, xl, xh, yl, yh, ncol, x, y);
      const uint32_t unknown = tl_unknown(x, y, nx, ny);
      const int lxs[3] = {min(x + 1, nx - 1) - x0 + 1, x - x0 + 1, max(x - 1, 0) - x0 + 1};
      const int lys[3] = {min(y + 1, ny - 1) - y0 + 1, y - y0 + 1, max(y - 1, 0) - y0 + 1};
      R g[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const R v = C::dec(lds2[i][lys[1 + kCy[i]]][lxs[1 + kCx[i]]], Ld.ds[i]);
        g[i] = (unknown >> i) & 1u ? R(0) : v;
      }
      nsbc_assign_correct<R>(g, unknown, edge_mc(e, x, y, mom2), rho0, b, Ld.corr_mode);
      collide<R, CM>(Ld, g, rho0, b, omega);
      if (x >= xo && y >= yo) store(x, y, g);
    }
  }
}

}  // namespace lbm
