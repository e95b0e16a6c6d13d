// lbm3d.hip -- the D3Q19 / D3Q27 sweep for gfx950: one launch per step, every node
// pulled (eq. lbe_0), collided with BGK (eqs. lbe_1, feq_1) and, on NSBC
// faces, rebuilt and corrected first (eqs. nes_0..nes_4 with the normal of
// the faces the node lies on); plus the C ABI of include/lbm3d.h.
//
// Pull streaming reads every stored value exactly once, so the sweep moves
// 2 x q x s bytes per node (D3Q19 FP32: 152 B) and is bound by HBM bandwidth.
// Threads map to consecutive x (64-wide wavefronts, coalesced); each access
// is a per-plane (uniform) base pointer plus a 32-bit byte offset, one offset
// per source row (y, z shift) plus the lane's x shift.  The only
// lines fetched twice are those a row's x-shifted pulls straddle at a block
// edge; the block order keeps x-neighbouring blocks on one XCD so that the
// second fetch hits its L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lbm.h"
#include "lbm_trace.h"
#include "lbm3d.h"
#include "lbm_device.h"
#include "lbm_host.h"

namespace lbm {
namespace d3 {

// Velocities: D3Q19 is the first 19 rows (rest, the six axis directions,
// the twelve face diagonals), D3Q27 all 27 (then the eight cube diagonals).
// Opposite directions are the pairs (2k - 1, 2k).
constexpr int kC[27][3] = {{0, 0, 0},   {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                           {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
                           {-1, 0, 1},  {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}, {1, 1, 1},  {-1, -1, -1},
                           {1, 1, -1},  {-1, -1, 1}, {1, -1, 1},  {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};

// Weights by speed: D3Q19 1/3, 1/18, 1/36; D3Q27 8/27, 2/27, 1/54, 1/216.
template <int NQ, class R>
__host__ __device__ constexpr R w3(int i) {
  return NQ == 19 ? (i == 0 ? R(1) / R(3) : (i <= 6 ? R(1) / R(18) : R(1) / R(36)))
                  : (i == 0 ? R(8) / R(27) : (i <= 6 ? R(2) / R(27) : (i <= 18 ? R(1) / R(54) : R(1) / R(216))));
}

// Everything a kernel needs about one lattice.
struct Lat3 {
  void* buf[2];
  // Moments (rho - rho0, ux, uy, uz) at time t of the nodes x = 0, 1,
  // nx - 2, nx - 1, for NSBC on the x faces: mx[p] goes with buf[p], element
  // ((side * 2 + layer) * 4 + c) * mxs + z * ny + y, side 0 at x = 0 and 1
  // at x = nx - 1, layer 0 the face node and 1 its inner neighbour.
  void* mx[2];
  int64_t mxs;
  int32_t nx, ny, nz, pitch;
  int64_t slab;   // elements per z-slab (ny * pitch)
  int64_t plane;  // elements per population plane
  int32_t bc[6];
  int32_t store, q;  // q: velocity set, 19 or 27
  double omega, rho0, gamma, beta;
  double m0[4];   // far field (rho - rho0, ux, uy, uz)
  // storage codec scales per population: a stored value is enc(g_i, es[i])
  // and decodes as dec(v, ds[i]) (1 for FP64/FP32; 2^k / w_i and w_i 2^-k for
  // FP16, k chosen at init; 1 / w_i and w_i for BF16)
  float es[27], ds[27];
};

template <int NQ, class R>
__device__ inline void moments3(const R g[NQ], R rho0, R m[4]) {
  R s = R(0), j[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    s += g[i];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (kC[i][a]) j[a] += kC[i][a] > 0 ? g[i] : -g[i];
  }
  const R ir = recip(rho0 + s);
  m[0] = s;
#pragma unroll
  for (int a = 0; a < 3; ++a) m[1 + a] = j[a] * ir;
}

// g^eq_i - w_i rho0 = w_i [drho + rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)]
template <int NQ, class R>
__device__ inline void equilibrium3(R rho0, const R m[4], R geq[NQ]) {
  const R rho = rho0 + m[0];
  const R q = R(1.5) * (m[1] * m[1] + m[2] * m[2] + m[3] * m[3]);
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    R a = R(0);
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (kC[i][k]) a += kC[i][k] > 0 ? m[1 + k] : -m[1 + k];
    geq[i] = w3<NQ, R>(i) * (m[0] + rho * fma(a, fma(R(4.5), a, R(3)), -q));
  }
}

// BGK in place, written per pair of opposite directions (2i-1, 2i): the even
// part E + 9/2 rho a^2 is shared, w_i is folded into omega.
template <int NQ, class R>
__device__ inline void bgk3(R g[NQ], R rho0, R omega, R m[4]) {
  moments3<NQ, R>(g, rho0, m);
  const R rho = rho0 + m[0];
  const R e = fma(-rho, R(1.5) * (m[1] * m[1] + m[2] * m[2] + m[3] * m[3]), m[0]);
  const R r45 = R(4.5) * rho, r3 = R(3) * rho, om1 = R(1) - omega;
  g[0] = fma(omega * w3<NQ, R>(0), e, om1 * g[0]);
#pragma unroll
  for (int p = 1; p < NQ; p += 2) {
    R a = R(0);
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (kC[p][k]) a += kC[p][k] > 0 ? m[1 + k] : -m[1 + k];
    const R ow = omega * w3<NQ, R>(p);
    const R even = fma(r45 * a, a, e), odd = r3 * a;
    g[p] = fma(ow, even + odd, om1 * g[p]);
    g[p + 1] = fma(ow, even - odd, om1 * g[p + 1]);
  }
}

template <int NQ, class R>
__device__ inline void bgk3(R g[NQ], R rho0, R omega) {
  R m[4];
  bgk3<NQ, R>(g, rho0, omega, m);
}

// Moments of the stored node at byte offset `off` of each plane.
template <int S, int NQ>
__device__ inline void node_moments3(const Lat3& L, const typename Codec<S>::T* A, uint32_t off,
                                     typename Codec<S>::R m[4]) {
  using C = Codec<S>;
  using T = typename C::T;
  using R = typename C::R;
  R s = R(0), j[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const R v = C::dec(*reinterpret_cast<const T*>(reinterpret_cast<const char*>(A + i * L.plane) + off), L.ds[i]);
    s += v;
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (kC[i][a]) j[a] += kC[i][a] > 0 ? v : -v;
  }
  const R ir = recip(R(L.rho0) + s);
  m[0] = s;
#pragma unroll
  for (int a = 0; a < 3; ++a) m[1 + a] = j[a] * ir;
}

// Node on the lattice's outer shell: pulls wrap across periodic faces; a
// population whose source lies beyond an NSBC face is unknown and rebuilt.
// Written to keep few values live (no equilibrium or copy arrays: rebuilt
// populations are formed in place from their opposites), so that the sweep
// that carries it keeps the occupancy of its interior path.
template <int S, int NQ>
__device__ inline void boundary_node3(const Lat3& L, const typename Codec<S>::T* A, int x, int y, int z,
                                      typename Codec<S>::R g[NQ]) {
  using C = Codec<S>;
  using T = typename C::T;
  using R = typename C::R;
  const int n[3] = {L.nx, L.ny, L.nz}, p[3] = {x, y, z};
  const uint32_t stride[3] = {1u, (uint32_t)L.pitch, (uint32_t)L.slab};
  uint32_t unknown = 0;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    uint32_t src = 0;
    bool out = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      int s = p[a] - kC[i][a];
      if (s < 0 || s >= n[a]) {
        if (L.bc[2 * a] == BC_PERIODIC) {
          s = s < 0 ? s + n[a] : s - n[a];
        } else {
          out = true;
          s = p[a];  // any node in range: the value is replaced below
        }
      }
      src += (uint32_t)s * stride[a];
    }
    unknown |= (uint32_t)out << i;
    g[i] = C::dec(*reinterpret_cast<const T*>(reinterpret_cast<const char*>(A + i * L.plane) + src * sizeof(T)),
                  L.ds[i]);
  }
  if (!unknown) return;
  // eq. nes_2 with the normalised normal of the k NSBC faces the node is on
  const uint32_t own = ((uint32_t)z * stride[2] + (uint32_t)y * stride[1] + (uint32_t)x) * (uint32_t)sizeof(T);
  R mb[4], d[4] = {R(0), R(0), R(0), R(0)};
  node_moments3<S, NQ>(L, A, own, mb);
  int k = 0;
#pragma unroll 1
  for (int a = 0; a < 3; ++a) {
    if (L.bc[2 * a] != BC_NSBC) continue;
    const int step = p[a] == 0 ? 1 : (p[a] == n[a] - 1 ? -1 : 0);
    if (!step) continue;
    R mn[4];
    node_moments3<S, NQ>(L, A, own + (uint32_t)(step * (int)sizeof(T)) * stride[a], mn);
#pragma unroll
    for (int c = 0; c < 4; ++c) d[c] += mb[c] - mn[c];
    ++k;
  }
  const R fac = R(L.gamma) * (k == 1 ? R(1) : (k == 2 ? R(0.70710678118654752440) : R(0.57735026918962576451)));
  const R beta = R(L.beta);
  R mc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) mc[c] = (R(1) - beta) * (mb[c] - fac * d[c]) + beta * R(L.m0[c]);  // eq. nes_3
  // eqs. nes_0/nes_1: f_i = f^eq_i + (f_o - f^eq_o) = f_o + 6 w_i rho_c (c_i . u_c) when the opposite o is
  // known, f^eq_i(m_c) when it is not
  const R rc = R(L.rho0) + mc[0];
  const R uu = R(1.5) * (mc[1] * mc[1] + mc[2] * mc[2] + mc[3] * mc[3]);
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    if (!((unknown >> i) & 1u)) continue;
    const int o = i & 1 ? i + 1 : i - 1;
    R cu = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (kC[i][a]) cu += kC[i][a] > 0 ? mc[1 + a] : -mc[1 + a];
    g[i] = (unknown >> o) & 1u ? w3<NQ, R>(i) * (mc[0] + rc * fma(cu, fma(R(4.5), cu, R(3)), -uu))
                               : fma(R(6) * w3<NQ, R>(i) * rc, cu, g[o]);
  }
  // eq. nes_4 with 1/c_s^2 = 3: shift all populations so the node carries m_c
  R s = R(0), j[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    s += g[i];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (kC[i][a]) j[a] += kC[i][a] > 0 ? g[i] : -g[i];
  }
  const R dr = s - mc[0];
  R dj[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) dj[a] = R(3) * (j[a] - rc * mc[1 + a]);
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    R cd = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (kC[i][a]) cd += kC[i][a] > 0 ? dj[a] : -dj[a];
    g[i] -= w3<NQ, R>(i) * (dr + cd);
  }
}

// NSBC on an x face, for a node whose y and z neighbours all lie inside: `g`
// holds its pulls with the unknown ones (c_x = side, side = +1 at x = 0 and
// -1 at x = nx - 1) loaded from any node in range; mb and mn are the moments
// at time t of the node and of its inner x neighbour.  Same arithmetic as
// boundary_node3 with k = 1.
template <int S, int NQ>
__device__ inline void xface_nsbc3(const Lat3& L, const typename Codec<S>::R mb[4],
                                   const typename Codec<S>::R mn[4], int side, typename Codec<S>::R g[NQ]) {
  using R = typename Codec<S>::R;
  const R fac = R(L.gamma), beta = R(L.beta);
  R mc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) mc[c] = (R(1) - beta) * (mb[c] - fac * (mb[c] - mn[c])) + beta * R(L.m0[c]);
  const R rc = R(L.rho0) + mc[0];
#pragma unroll
  for (int p = 1; p < NQ; p += 2) {
    if (!kC[p][0]) continue;
    R cu = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (kC[p][a]) cu += kC[p][a] > 0 ? mc[1 + a] : -mc[1 + a];
    const R t = R(6) * w3<NQ, R>(p) * rc;
    const bool p_unknown = kC[p][0] == side;
    const R gp = fma(t, cu, g[p + 1]), go = fma(t, -cu, g[p]);
    g[p] = p_unknown ? gp : g[p];
    g[p + 1] = p_unknown ? g[p + 1] : go;
  }
  R s = R(0), j[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    s += g[i];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (kC[i][a]) j[a] += kC[i][a] > 0 ? g[i] : -g[i];
  }
  const R dr = s - mc[0];
  R dj[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) dj[a] = R(3) * (j[a] - rc * mc[1 + a]);
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    R cd = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (kC[i][a]) cd += kC[i][a] > 0 ? dj[a] : -dj[a];
    g[i] -= w3<NQ, R>(i) * (dr + cd);
  }
}

// Register budget: the shell paths would otherwise take more registers than
// the interior path and cost every node occupancy.  Without spills D3Q19 fits
// 6 waves per SIMD in FP32, 5 with a 16-bit format (its per-population
// scales take registers) and 4 in FP64; D3Q27 5, 4 and 3.
template <int S, int NQ>
constexpr int k3_waves() {
  return S == ST_F64 ? (NQ == 19 ? 4 : 3) : S == ST_F32 ? (NQ == 19 ? 6 : 5) : (NQ == 19 ? 5 : 4);
}

// Pulls of a node whose y and z neighbours all lie inside.  `idx` is its
// element index; sxm and sxp are the byte shifts of the pulls with c_x = +1
// (source x - 1) and c_x = -1 (source x + 1).
template <int S, int NQ, bool NTL = false>
__device__ __forceinline__ void pull_row3(const Lat3& L, const typename Codec<S>::T* A, uint32_t idx, int sxm,
                                          int sxp, typename Codec<S>::R g[NQ]) {
  using C = Codec<S>;
  using T = typename C::T;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const char* Ai = reinterpret_cast<const char*>(A + i * L.plane);
    const uint32_t row = (idx - (uint32_t)(kC[i][2] * L.slab + kC[i][1] * L.pitch)) * (uint32_t)sizeof(T);
    const int sh = kC[i][0] > 0 ? sxm : (kC[i][0] < 0 ? sxp : 0);
    const T* src = reinterpret_cast<const T*>(Ai + (row + (uint32_t)sh));
    g[i] = C::dec(NTL ? __builtin_nontemporal_load(src) : *src, L.ds[i]);
  }
}

// One launch per step.  Block b takes item (b mod 8) * per + b / 8 of the
// list of (z chunk, tile row, tile column) in that order, so XCD k (blocks
// b = k mod 8) works through the k-th contiguous stretch: x-neighbouring
// tiles, which share the lines their shifted pulls straddle, run on one XCD.
// Rows on a y or z face are left to a second launch (k3_faces, node by node
// with boundary_node3), so that their registers do not weigh on this kernel.
// In the other rows an x-face node is one lane of
// a wavefront: it pulls with the others (the x shift adjusted), and on a NSBC
// face it takes the moments at time t of itself and of its inner neighbour
// from Lat3::mx instead of loading 2 q stored populations: the lanes of those
// nodes in the previous step summed the populations they stored (the same
// sums node_moments3 would form from memory) and wrote them there.  Nodes
// with y and z
// inside are written by the wavefront that holds their whole row segment:
// no cache line of the output is written in parts by different blocks.
template <int S, int NQ, int BX, int BY, int ZC, bool NTL>
__global__ __launch_bounds__(BX* BY, (k3_waves<S, NQ>())) void k3_step(Lat3 L, int parity, int tiles_x, int tiles_y,
                                                                int nitems, int per) {
  using C = Codec<S>;
  using T = typename C::T;
  using R = typename C::R;
  const int b = blockIdx.x;
  const int item = (b & 7) * per + (b >> 3);
  if (item >= nitems) return;  // no barrier in this kernel
  const int ntile = tiles_x * tiles_y;
  const int zc = item / ntile, t = item - zc * ntile;
  const int ty = t / tiles_x, tx = t - ty * tiles_x;
  const int x = tx * BX + threadIdx.x, y = ty * BY + threadIdx.y;
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  if (x >= nx || y >= ny) return;
  const T* __restrict__ A = static_cast<const T*>(parity ? L.buf[1] : L.buf[0]);
  T* __restrict__ B = static_cast<T*>(parity ? L.buf[0] : L.buf[1]);
  const R* __restrict__ MA = static_cast<const R*>(parity ? L.mx[1] : L.mx[0]);
  R* __restrict__ MB = static_cast<R*>(parity ? L.mx[0] : L.mx[1]);
  const R rho0 = R(L.rho0), omega = R(L.omega);
  const bool y_inner = y >= 1 && y <= ny - 2;
  // Byte shifts of the pulls with c_x = +1 (source x - 1) and c_x = -1
  // (source x + 1).  Beyond an x face the source wraps (periodic) or is a node
  // in range whose value xface_nsbc3 replaces (NSBC).
  const bool xper = L.bc[0] == BC_PERIODIC;
  const int sxm = (x > 0 ? -1 : (xper ? nx - 1 : 0)) * (int)sizeof(T);
  const int sxp = (x < nx - 1 ? 1 : (xper ? 1 - nx : 0)) * (int)sizeof(T);
  const int xside = xper ? 0 : (x == 0 ? 1 : (x == nx - 1 ? -1 : 0));
  // does this lane write slots of Lat3::mx (x = 0, 1, nx - 2, nx - 1)?
  const bool mwrite = !xper && (x <= 1 || x >= nx - 2);
  const uint32_t mxs = (uint32_t)L.mxs;
  const int z1 = min(nz, (zc + 1) * ZC);
  for (int z = zc * ZC; z < z1; ++z) {
    R g[NQ];
    const uint32_t idx = (uint32_t)((int64_t)z * L.slab + (int64_t)y * L.pitch + x);
    const bool inner_row = y_inner && z >= 1 && z <= nz - 2;
    if (!inner_row) continue;  // rows on a y or z face: k3_faces
    {
      pull_row3<S, NQ, NTL>(L, A, idx, sxm, sxp, g);
      if (xside) {
        const uint32_t mo = (uint32_t)z * (uint32_t)ny + (uint32_t)y;
        const R* Mb = MA + (x == 0 ? 0 : 8 * mxs);  // slots 0, 1 (x = 0) or 2, 3
        R mb[4], mn[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          mb[c] = R(Mb[c * mxs + mo]);
          mn[c] = R(Mb[(4 + c) * mxs + mo]);
        }
        xface_nsbc3<S, NQ>(L, mb, mn, xside, g);
      }
    }
    bgk3<NQ, R>(g, rho0, omega);
    if (mwrite) {
      // moments of the populations stored below, as they decode; slot 0:
      // x = 0, 1: x = 1, 2: x = nx - 1, 3: x = nx - 2 (both 1 and 3 when nx = 3)
      R gs[NQ], m[4];
#pragma unroll
      for (int i = 0; i < NQ; ++i) gs[i] = C::dec(C::enc(g[i], L.es[i]), L.ds[i]);
      moments3<NQ, R>(gs, rho0, m);
      const uint32_t mo = (uint32_t)z * (uint32_t)ny + (uint32_t)y;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (x == 0) MB[c * mxs + mo] = m[c];
        if (x == 1) MB[(4 + c) * mxs + mo] = m[c];
        if (x == nx - 1) MB[(8 + c) * mxs + mo] = m[c];
        if (x == nx - 2) MB[(12 + c) * mxs + mo] = m[c];
      }
    }
    const uint32_t off = idx * (uint32_t)sizeof(T);
#pragma unroll
    for (int i = 0; i < NQ; ++i)
      __builtin_nontemporal_store(C::enc(g[i], L.es[i]),
                                  reinterpret_cast<T*>(reinterpret_cast<char*>(B + i * L.plane) + off));
  }
}

// ------------------------------------------------------------------ pair sweep (16-bit formats)
// The same step with two x-neighbouring nodes (x0, x0 + 1; x0 even) per lane,
// for the 16-bit storage formats.  Each pull is one 32-bit load of the two
// values the pair needs: at element x0 for c_x = 0, at x0 - 1 for c_x = +1
// and at x0 + 1 for c_x = -1 (2-byte aligned: the GPU serves such loads),
// and each store one 32-bit store of both results.  The one-node sweep
// issues a load per 2 bytes; this one per 4, so every wave keeps twice the
// bytes in flight.  Per node the pulls, the functions and their order are the
// one-node sweep's (an x-face node takes its unknown pulls from itself, as
// there), so the results are bit-identical.  The rows on a y or z face go to
// a second, node-by-node launch (k3_faces).  Lattices with periodic x faces or
// an odd nx take the one-node sweep.
template <class T>
__device__ inline T from_bits16(uint32_t h) {
  return __builtin_bit_cast(T, (uint16_t)h);
}
template <class T>
__device__ inline uint32_t to_bits16(T v) {
  return (uint32_t)__builtin_bit_cast(uint16_t, v);
}

// (a wave per SIMD fewer than the one-node sweep: each holds two nodes' pulls)
template <int NQ>
constexpr int k3_pair_waves() {
  return NQ == 19 ? 4 : 3;
}

template <int S, int NQ, int BX, int BY, int ZC>
__global__ __launch_bounds__(BX* BY, (k3_pair_waves<NQ>())) void k3_pair(Lat3 L, int parity, int tiles_x, int tiles_y,
                                                                int nitems, int per) {
  using C = Codec<S>;
  using T = typename C::T;
  using R = typename C::R;
  static_assert(sizeof(T) == 2, "the pair sweep is for the 16-bit formats");
  const int b = blockIdx.x;
  const int item = (b & 7) * per + (b >> 3);
  if (item >= nitems) return;  // no barrier in this kernel
  const int ntile = tiles_x * tiles_y;
  const int zc = item / ntile, t = item - zc * ntile;
  const int ty = t / tiles_x, tx = t - ty * tiles_x;
  const int x0 = 2 * (tx * BX + threadIdx.x), y = ty * BY + threadIdx.y;
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  if (x0 >= nx || y >= ny) return;  // nx is even: x0 + 1 < nx
  const int xb = x0 + 1;
  const T* __restrict__ A = static_cast<const T*>(parity ? L.buf[1] : L.buf[0]);
  T* __restrict__ B = static_cast<T*>(parity ? L.buf[0] : L.buf[1]);
  const R* __restrict__ MA = static_cast<const R*>(parity ? L.mx[1] : L.mx[0]);
  R* __restrict__ MB = static_cast<R*>(parity ? L.mx[0] : L.mx[1]);
  const R rho0 = R(L.rho0), omega = R(L.omega);
  const bool y_inner = y >= 1 && y <= ny - 2;
  const uint32_t mxs = (uint32_t)L.mxs;
  // moments at time t + 1 of a node on or next to an x face, as its stored values decode (slot k
  // of Lat3::mx), from the encoded values in half `shift` (0 or 16) of w
  auto write_slot = [&](const uint32_t w[NQ], int shift, int slot, uint32_t mo) {
    R gs[NQ], m[4];
#pragma unroll
    for (int i = 0; i < NQ; ++i) gs[i] = C::dec(from_bits16<T>(w[i] >> shift), L.ds[i]);
    moments3<NQ, R>(gs, rho0, m);
#pragma unroll
    for (int c = 0; c < 4; ++c) MB[(4 * slot + c) * mxs + mo] = m[c];
  };
  // NSBC on an x face from the moments at time t of the face node and its inner neighbour
  auto xface = [&](R g[NQ], int side, uint32_t mo) {
    const R* Mb = MA + (side > 0 ? 0 : 8 * mxs);  // slots 0, 1 (x = 0) or 2, 3 (x = nx - 1)
    R mb[4], mn[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      mb[c] = R(Mb[c * mxs + mo]);
      mn[c] = R(Mb[(4 + c) * mxs + mo]);
    }
    xface_nsbc3<S, NQ>(L, mb, mn, side, g);
  };
  const int z1 = min(nz, (zc + 1) * ZC);
  for (int z = zc * ZC; z < z1; ++z) {
    const uint32_t idx = (uint32_t)((int64_t)z * L.slab + (int64_t)y * L.pitch + x0);
    const uint32_t mo = (uint32_t)z * (uint32_t)ny + (uint32_t)y;
    if (y_inner && z >= 1 && z <= nz - 2) {
      // pulls: the low half of w[i] is node x0's, the high half node x0 + 1's.  Every load
      // stays inside its source row (elements 0 .. nx - 1): on an x face the pair loads its
      // own aligned word, whose halves hold what both nodes pull there (the face node pulls
      // its unknown population from itself, as in the one-node sweep; the value is replaced)
      const bool left_face = x0 == 0, right_face = xb == nx - 1;
      uint32_t w[NQ];
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        const char* Ai = reinterpret_cast<const char*>(A + i * L.plane);
        // element offset of (x0, y - c_y, z - c_z): >= 0 in an inner row
        const uint32_t row = (idx - (uint32_t)(kC[i][2] * L.slab + kC[i][1] * L.pitch)) * 2u;
        const int cx = kC[i][0];
        const int sh = cx > 0 ? (left_face ? 0 : -2) : (cx < 0 ? (right_face ? 0 : 2) : 0);
        const uint32_t v = *reinterpret_cast<const uint32_t*>(Ai + (int64_t)row + sh);
        uint32_t lo = v & 0xffffu, hi = v >> 16;
        if (cx > 0 && left_face) hi = lo;   // node 1 pulls element 0
        if (cx < 0 && right_face) lo = hi;  // node nx - 2 pulls element nx - 1
        w[i] = lo | (hi << 16);
      }
      {
        R g[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i) g[i] = C::dec(from_bits16<T>(w[i]), L.ds[i]);
        if (x0 == 0) xface(g, 1, mo);
        bgk3<NQ, R>(g, rho0, omega);
#pragma unroll
        for (int i = 0; i < NQ; ++i) w[i] = (w[i] & 0xffff0000u) | to_bits16<T>(C::enc(g[i], L.es[i]));
      }
      if (x0 == 0) write_slot(w, 0, 0, mo);
      if (x0 == nx - 2) write_slot(w, 0, 3, mo);
      {
        R g[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i) g[i] = C::dec(from_bits16<T>(w[i] >> 16), L.ds[i]);
        if (xb == nx - 1) xface(g, -1, mo);
        bgk3<NQ, R>(g, rho0, omega);
#pragma unroll
        for (int i = 0; i < NQ; ++i) w[i] = (w[i] & 0xffffu) | (to_bits16<T>(C::enc(g[i], L.es[i])) << 16);
      }
      if (xb == 1) write_slot(w, 16, 1, mo);
      if (xb == nx - 1) write_slot(w, 16, 2, mo);
      const uint32_t off = idx * 2u;
#pragma unroll
      for (int i = 0; i < NQ; ++i)
        __builtin_nontemporal_store(w[i], reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(B + i * L.plane) + off));
    }
    // (rows on a y or z face: k3_faces)
  }
}

// The rows on a y or z face (y = 0, ny - 1 for every z; z = 0, nz - 1 for the
// other y), node by node with boundary_node3, one block per row segment of
// 256 nodes; launched after k3_step or k3_pair, which leave them out so that
// their registers do not weigh on them.
template <int S, int NQ>
__global__ __launch_bounds__(256) void k3_faces(Lat3 L, int parity) {
  using C = Codec<S>;
  using T = typename C::T;
  using R = typename C::R;
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const int r = blockIdx.y;  // face row: 0 .. 2 nz - 1 on the y faces, then 2 (ny - 2) on the z faces
  int y, z;
  if (r < 2 * nz) {
    z = r >> 1;
    y = r & 1 ? ny - 1 : 0;
  } else {
    const int k = r - 2 * nz;
    y = 1 + (k >> 1);
    z = k & 1 ? nz - 1 : 0;
  }
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= nx) return;
  const T* __restrict__ A = static_cast<const T*>(parity ? L.buf[1] : L.buf[0]);
  T* __restrict__ B = static_cast<T*>(parity ? L.buf[0] : L.buf[1]);
  R g[NQ];
  boundary_node3<S, NQ>(L, A, x, y, z, g);
  bgk3<NQ, R>(g, R(L.rho0), R(L.omega));
  const uint32_t off = (uint32_t)((int64_t)z * L.slab + (int64_t)y * L.pitch + x) * (uint32_t)sizeof(T);
#pragma unroll
  for (int i = 0; i < NQ; ++i)
    __builtin_nontemporal_store(C::enc(g[i], L.es[i]), reinterpret_cast<T*>(reinterpret_cast<char*>(B + i * L.plane) + off));
}

// Launch shapes: block BX x BY, ZC z-planes per block, non-temporal pull
// loads (NTL; every stored value is read once, so caching it only displaces
// the lines that x-neighbouring blocks share).
struct Shape3 {
  int bx, by, zc;
  bool ntl;
};
#define LBM3D_SHAPES(X) \
  X(64, 4, 1, false)    \
  X(64, 4, 2, false)    \
  X(64, 4, 4, false)    \
  X(64, 2, 1, false)    \
  X(128, 1, 1, false)   \
  X(128, 2, 4, false)   \
  X(256, 1, 4, false)   \
  X(64, 4, 1, true)     \
  X(64, 2, 1, true)     \
  X(128, 1, 1, true)
static const Shape3 kShapes3[] = {
#define X(a, b, c, d) {a, b, c, d},
    LBM3D_SHAPES(X)
#undef X
};
static constexpr int kNumShapes3 = sizeof(kShapes3) / sizeof(kShapes3[0]);

// Pair-sweep shapes (ids from kNumShapes3 on): BX lanes (2 BX nodes) x BY rows, ZC z-planes.
#define LBM3D_PAIR_SHAPES(X) \
  X(64, 4, 1)                \
  X(64, 2, 1)                \
  X(64, 4, 2)                \
  X(128, 1, 1)               \
  X(128, 2, 2)               \
  X(64, 1, 4)
struct ShapePair {
  int bx, by, zc;
};
static const ShapePair kPairs3[] = {
#define X(a, b, c) {a, b, c},
    LBM3D_PAIR_SHAPES(X)
#undef X
};
static constexpr int kNumPairs3 = sizeof(kPairs3) / sizeof(kPairs3[0]);
static constexpr int kNumAll3 = kNumShapes3 + kNumPairs3;

// Whether launch shape `id` takes lattice L: the pair shapes need a 16-bit
// format, non-periodic x faces and an even nx.
static bool shape3_supported(const Lat3& L, int id) {
  if (id < 0 || id >= kNumAll3) return false;
  if (id < kNumShapes3) return true;
  return (L.store == ST_F16 || L.store == ST_BF16) && L.bc[0] != BC_PERIODIC && L.nx % 2 == 0;
}

template <int S, int NQ, int BX, int BY, int ZC, bool NTL>
static hipError_t launch3_t(const Lat3& L, int parity, hipStream_t s) {
  const int tiles_x = (L.nx + BX - 1) / BX, tiles_y = (L.ny + BY - 1) / BY, zch = (L.nz + ZC - 1) / ZC;
  const int nitems = tiles_x * tiles_y * zch, per = (nitems + 7) / 8;
  k3_step<S, NQ, BX, BY, ZC, NTL><<<dim3(8 * per), dim3(BX, BY), 0, s>>>(L, parity, tiles_x, tiles_y, nitems, per);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k3_faces<S, NQ><<<dim3((L.nx + 255) / 256, 2 * L.nz + 2 * (L.ny - 2)), dim3(256), 0, s>>>(L, parity);
  return hipGetLastError();
}

template <int S, int NQ, int BX, int BY, int ZC>
static hipError_t launch3_pair_t(const Lat3& L, int parity, hipStream_t s) {
  if constexpr (S == ST_F16 || S == ST_BF16) {
    const int tiles_x = (L.nx / 2 + BX - 1) / BX, tiles_y = (L.ny + BY - 1) / BY, zch = (L.nz + ZC - 1) / ZC;
    const int nitems = tiles_x * tiles_y * zch, per = (nitems + 7) / 8;
    k3_pair<S, NQ, BX, BY, ZC><<<dim3(8 * per), dim3(BX, BY), 0, s>>>(L, parity, tiles_x, tiles_y, nitems, per);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k3_faces<S, NQ><<<dim3((L.nx + 255) / 256, 2 * L.nz + 2 * (L.ny - 2)), dim3(256), 0, s>>>(L, parity);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int S, int NQ>
static hipError_t launch3_s(const Lat3& L, int parity, int shape, hipStream_t s) {
  if (!shape3_supported(L, shape)) return hipErrorInvalidValue;
  int k = 0;
#define X(a, b, c, d)                                                    \
  if (shape == k) return launch3_t<S, NQ, a, b, c, d>(L, parity, s);    \
  ++k;
  LBM3D_SHAPES(X)
#undef X
#define X(a, b, c)                                                       \
  if (shape == k) return launch3_pair_t<S, NQ, a, b, c>(L, parity, s);  \
  ++k;
  LBM3D_PAIR_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

template <int NQ>
static hipError_t launch3_q(const Lat3& L, int parity, int shape, hipStream_t s) {
  switch (L.store) {
    case ST_F64: return launch3_s<ST_F64, NQ>(L, parity, shape, s);
    case ST_F32: return launch3_s<ST_F32, NQ>(L, parity, shape, s);
    case ST_F16: return launch3_s<ST_F16, NQ>(L, parity, shape, s);
    case ST_BF16: return launch3_s<ST_BF16, NQ>(L, parity, shape, s);
  }
  return hipErrorInvalidValue;
}

static hipError_t launch3(const Lat3& L, int parity, int shape, hipStream_t s) {
  return L.q == 27 ? launch3_q<27>(L, parity, shape, s) : launch3_q<19>(L, parity, shape, s);
}

// The x-face slots of Lat3::mx[parity] for node (x, y, z) (x = 0, 1, nx - 2,
// nx - 1 only), from the values `v` just stored at the node: the moments of
// the populations as they decode.
template <int S, int NQ>
__device__ inline void mx_from_stored(const Lat3& L, int parity, int x, int y, int z,
                                      const typename Codec<S>::T v[NQ]) {
  using C = Codec<S>;
  using R = typename C::R;
  const int nx = L.nx;
  if (x > 1 && x < nx - 2) return;
  R g[NQ], ms[4];
#pragma unroll
  for (int i = 0; i < NQ; ++i) g[i] = C::dec(v[i], L.ds[i]);
  moments3<NQ, R>(g, R(L.rho0), ms);
  R* M = static_cast<R*>(L.mx[parity]);
  const int64_t mo = (int64_t)z * L.ny + y;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (x == 0) M[(0 * 4 + c) * L.mxs + mo] = ms[c];
    if (x == 1) M[(1 * 4 + c) * L.mxs + mo] = ms[c];
    if (x == nx - 2) M[(3 * 4 + c) * L.mxs + mo] = ms[c];
    if (x == nx - 1) M[(2 * 4 + c) * L.mxs + mo] = ms[c];
  }
}

// Largest |g^eq_i / w_i| of the initial state (deviation form), one partial
// per block of a fixed 256 x 256 grid (a fixed-order tree in each block): the
// host picks the FP16 scale exponent from it.
template <int NQ>
__global__ __launch_bounds__(256) void k3_absmax(Lat3 L, const double* __restrict__ drho,
                                                 const double* __restrict__ ux, const double* __restrict__ uy,
                                                 const double* __restrict__ uz, float* __restrict__ part) {
  __shared__ float red[256];
  const int64_t n = (int64_t)L.nx * L.ny * L.nz;
  float mx = 0.f;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += 256 * 256) {
    const double m[4] = {drho[k], ux[k], uy[k], uz[k]};
    double geq[NQ];
    equilibrium3<NQ, double>(L.rho0, m, geq);
#pragma unroll
    for (int i = 0; i < NQ; ++i) mx = fmaxf(mx, (float)fabs(geq[i] / w3<NQ, double>(i)));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// f = f^eq(rho, u) of the initial fields, as deviations
template <int S, int NQ>
__global__ void k3_init(Lat3 L, const double* __restrict__ drho, const double* __restrict__ ux,
                        const double* __restrict__ uy, const double* __restrict__ uz) {
  using T = typename Codec<S>::T;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= L.nx) return;
  const int64_t k = ((int64_t)z * L.ny + y) * L.nx + x;
  const double m[4] = {drho[k], ux[k], uy[k], uz[k]};
  double geq[NQ];
  equilibrium3<NQ, double>(L.rho0, m, geq);
  using C = Codec<S>;
  T* B = static_cast<T*>(L.buf[0]);
  const int64_t idx = (int64_t)z * L.slab + (int64_t)y * L.pitch + x;
  T v[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    v[i] = C::enc(typename C::R(geq[i] * (double)L.es[i]), 1.0f);
    B[i * L.plane + idx] = v[i];
  }
  mx_from_stored<S, NQ>(L, 0, x, y, z, v);
}

template <int S, int NQ>
__global__ void k3_moments(Lat3 L, int parity, double* __restrict__ out) {
  using T = typename Codec<S>::T;
  using R = typename Codec<S>::R;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= L.nx) return;
  R m[4];
  const uint32_t off = (uint32_t)((int64_t)z * L.slab + (int64_t)y * L.pitch + x) * (uint32_t)sizeof(T);
  node_moments3<S, NQ>(L, static_cast<const T*>(parity ? L.buf[1] : L.buf[0]), off, m);
  const int64_t n = (int64_t)L.nx * L.ny * L.nz, k = ((int64_t)z * L.ny + y) * L.nx + x;
#pragma unroll
  for (int c = 0; c < 4; ++c) out[c * n + k] = (double)m[c];
}

// Stored populations (f_i - w_i rho0) of buffer `parity` into out[q][nz][ny][nx].
template <int S, int NQ>
__global__ void k3_get_pops(Lat3 L, int parity, double* __restrict__ out) {
  using T = typename Codec<S>::T;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= L.nx) return;
  const T* A = static_cast<const T*>(parity ? L.buf[1] : L.buf[0]);
  const int64_t idx = (int64_t)z * L.slab + (int64_t)y * L.pitch + x;
  const int64_t n = (int64_t)L.nx * L.ny * L.nz, k = ((int64_t)z * L.ny + y) * L.nx + x;
#pragma unroll
  for (int i = 0; i < NQ; ++i) out[i * n + k] = (double)Codec<S>::dec(A[i * L.plane + idx], L.ds[i]);
}

// Overwrite buffer `parity` (and its x-face moments) with in[q][nz][ny][nx].
template <int S, int NQ>
__global__ void k3_set_pops(Lat3 L, int parity, const double* __restrict__ in) {
  using T = typename Codec<S>::T;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= L.nx) return;
  T* A = static_cast<T*>(parity ? L.buf[1] : L.buf[0]);
  const int64_t idx = (int64_t)z * L.slab + (int64_t)y * L.pitch + x;
  const int64_t n = (int64_t)L.nx * L.ny * L.nz, k = ((int64_t)z * L.ny + y) * L.nx + x;
  using C = Codec<S>;
  T v[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    v[i] = C::enc(typename C::R(in[i * n + k] * (double)L.es[i]), 1.0f);
    A[i * L.plane + idx] = v[i];
  }
  mx_from_stored<S, NQ>(L, parity, x, y, z, v);
}

// *bad = 1 if a stored population of buffer `parity` is not finite.
template <int S, int NQ>
__global__ void k3_finite(Lat3 L, int parity, int* bad) {
  using T = typename Codec<S>::T;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= L.nx) return;
  const T* A = static_cast<const T*>(parity ? L.buf[1] : L.buf[0]);
  const int64_t idx = (int64_t)z * L.slab + (int64_t)y * L.pitch + x;
  bool ok = true;
#pragma unroll
  for (int i = 0; i < NQ; ++i) ok = ok && isfinite((double)Codec<S>::dec(A[i * L.plane + idx], L.ds[i]));
  if (!ok) *bad = 1;
}

// Launch one of the per-node kernels above for the context's store and q.
#define LBM3D_NODE_LAUNCH_S(KERNEL, NQ, L, s, ...)                                   \
  do {                                                                             \
    const dim3 grid_((L.nx + 255) / 256, L.ny, L.nz);                                \
    switch (L.store) {                                                             \
      case ST_F64: KERNEL<ST_F64, NQ><<<grid_, dim3(256), 0, s>>>(L, __VA_ARGS__); break;   \
      case ST_F32: KERNEL<ST_F32, NQ><<<grid_, dim3(256), 0, s>>>(L, __VA_ARGS__); break;   \
      case ST_F16: KERNEL<ST_F16, NQ><<<grid_, dim3(256), 0, s>>>(L, __VA_ARGS__); break;   \
      case ST_BF16: KERNEL<ST_BF16, NQ><<<grid_, dim3(256), 0, s>>>(L, __VA_ARGS__); break; \
      default: return hipErrorInvalidValue;                                        \
    }                                                                              \
  } while (0)
#define LBM3D_NODE_LAUNCH(KERNEL, L, s, ...)                  \
  do {                                                      \
    if (L.q == 27) LBM3D_NODE_LAUNCH_S(KERNEL, 27, L, s, __VA_ARGS__); \
    else LBM3D_NODE_LAUNCH_S(KERNEL, 19, L, s, __VA_ARGS__);           \
  } while (0)

static hipError_t launch_get_pops3(const Lat3& L, int parity, double* out, hipStream_t s) {
  LBM3D_NODE_LAUNCH(k3_get_pops, L, s, parity, out);
  return hipGetLastError();
}

static hipError_t launch_set_pops3(const Lat3& L, int parity, const double* in, hipStream_t s) {
  LBM3D_NODE_LAUNCH(k3_set_pops, L, s, parity, in);
  return hipGetLastError();
}

static hipError_t launch_finite3(const Lat3& L, int parity, int* bad, hipStream_t s) {
  LBM3D_NODE_LAUNCH(k3_finite, L, s, parity, bad);
  return hipGetLastError();
}

static hipError_t launch_init3(const Lat3& L, const double* drho, const double* ux, const double* uy,
                               const double* uz, hipStream_t s) {
  LBM3D_NODE_LAUNCH(k3_init, L, s, drho, ux, uy, uz);
  return hipGetLastError();
}

static hipError_t launch_moments3(const Lat3& L, int parity, double* out, hipStream_t s) {
  LBM3D_NODE_LAUNCH(k3_moments, L, s, parity, out);
  return hipGetLastError();
}

static hipError_t launch_absmax3(const Lat3& L, const double* drho, const double* ux, const double* uy,
                                 const double* uz, float* part, hipStream_t s) {
  if (L.q == 27) k3_absmax<27><<<dim3(256), dim3(256), 0, s>>>(L, drho, ux, uy, uz, part);
  else k3_absmax<19><<<dim3(256), dim3(256), 0, s>>>(L, drho, ux, uy, uz, part);
  return hipGetLastError();
}

}  // namespace d3
}  // namespace lbm

// ------------------------------------------------------------------ C ABI
using lbm::host::fail;

#define HIPCHK3(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(LBM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct lbm3d_ctx {
  lbm::d3::Lat3 L;
  int parity = 0;
  int64_t t = 0;
  int shape = 4;  // 128x1xz1, the fastest on 256^3 in both formats
  hipStream_t stream = nullptr;
  int* flag = nullptr;    // device int in the workspace (lbm3d_check_finite)
  float* part = nullptr;  // 256 device floats in the workspace (FP16 exponent at init)
  int f16_exp = 0;
};

namespace {

struct Layout3 {
  size_t esize, rsize;  // stored and arithmetic element sizes
  int32_t pitch;
  int64_t slab, plane;
  int q;
  size_t buf_bytes, mx_bytes, total;
};

int check3(const lbm3d_params* p) {
  if (!p) return fail(LBM_ERR_ARG, "params is NULL");
  if (p->nx < 3 || p->ny < 3 || p->nz < 3) return fail(LBM_ERR_ARG, "lattice %dx%dx%d: each side must be >= 3", p->nx, p->ny, p->nz);
  if ((int64_t)p->nx * p->ny * p->nz > (int64_t)1 << 28) return fail(LBM_ERR_ARG, "lattice exceeds 2^28 nodes");
  {
    // the kernels address a plane with 32-bit byte offsets
    const int64_t es = p->store == LBM_STORE_F64 ? 8 : (p->store == LBM_STORE_F32 ? 4 : 2);
    const int64_t row = ((int64_t)p->nx * es + 255) / 256 * 256;
    if (row * p->ny * p->nz > ((int64_t)1 << 32) - 65536)
      return fail(LBM_ERR_ARG, "lattice %dx%dx%d: a plane with rows padded to 256 bytes exceeds 4 GiB", p->nx,
                  p->ny, p->nz);
  }
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail(LBM_ERR_ARG, "tau = %g: BGK needs tau > 0.5", p->tau);
  if (!(p->rho0 > 0) || !std::isfinite(p->rho0)) return fail(LBM_ERR_ARG, "rho0 = %g must be > 0", p->rho0);
  for (int f = 0; f < 6; ++f)
    if (p->bc[f] != LBM_BC_PERIODIC && p->bc[f] != LBM_BC_NSBC)
      return fail(LBM_ERR_ARG, "bc[%d] = %d is not LBM_BC_PERIODIC or LBM_BC_NSBC", f, p->bc[f]);
  for (int a = 0; a < 3; ++a)
    if ((p->bc[2 * a] == LBM_BC_PERIODIC) != (p->bc[2 * a + 1] == LBM_BC_PERIODIC))
      return fail(LBM_ERR_ARG, "periodic faces must come in pairs");
  if (!std::isfinite(p->gamma)) return fail(LBM_ERR_ARG, "gamma must be finite");
  if (p->store != LBM_STORE_F64 && p->store != LBM_STORE_F32 && p->store != LBM_STORE_F16DEV &&
      p->store != LBM_STORE_BF16DEV)
    return fail(LBM_ERR_ARG, "store = %d is not an LBM_STORE_* format", p->store);
  if (p->velocity_set != LBM3D_D3Q19 && p->velocity_set != LBM3D_D3Q27)
    return fail(LBM_ERR_ARG, "velocity_set = %d is not LBM3D_D3Q19 or LBM3D_D3Q27", p->velocity_set);
  return LBM_OK;
}

Layout3 layout3(const lbm3d_params* p) {
  using lbm::host::round_up;
  Layout3 l;
  l.esize = p->store == LBM_STORE_F64 ? 8 : (p->store == LBM_STORE_F32 ? 4 : 2);
  l.rsize = p->store == LBM_STORE_F64 ? 8 : 4;
  const size_t row = round_up((size_t)p->nx * l.esize, 256);
  l.pitch = (int32_t)(row / l.esize);
  l.slab = (int64_t)l.pitch * p->ny;
  size_t plane_bytes = round_up(row * (size_t)p->ny * p->nz, 4096);
  if (plane_bytes % 65536 == 0) plane_bytes += 4096;  // planes not a large power of two apart
  l.plane = (int64_t)(plane_bytes / l.esize);
  l.q = p->velocity_set == LBM3D_D3Q27 ? 27 : 19;
  l.buf_bytes = round_up((size_t)l.q * plane_bytes, (size_t)2 << 20);
  l.mx_bytes = round_up((size_t)16 * p->ny * p->nz * l.rsize, 4096);
  l.total = 2 * l.buf_bytes + 2 * l.mx_bytes + 256 + 1024;  // + the check_finite flag, the FP16 partials
  return l;
}

}  // namespace

extern "C" {

int lbm3d_params_default(lbm3d_params* p) {
  if (!p) return fail(LBM_ERR_ARG, "params is NULL");
  std::memset(p, 0, sizeof(*p));
  p->nx = p->ny = p->nz = 3;
  p->tau = 0.6;
  p->rho0 = 1.0;
  for (int f = 0; f < 6; ++f) p->bc[f] = LBM_BC_NSBC;
  p->gamma = 0.6;
  p->store = LBM_STORE_F32;
  return LBM_OK;
}

int lbm3d_workspace_bytes(const lbm3d_params* p, size_t* bytes) {
  if (!bytes) return fail(LBM_ERR_ARG, "bytes is NULL");
  int rc = check3(p);
  if (rc) return rc;
  *bytes = layout3(p).total;
  return LBM_OK;
}

int lbm3d_init(lbm3d_ctx** out, const lbm3d_params* p, void* workspace, size_t bytes, const double* drho,
               const double* ux, const double* uy, const double* uz, void* hip_stream) {
  if (!out) return fail(LBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  int rc = check3(p);
  if (rc) return rc;
  const Layout3 lay = layout3(p);
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(LBM_ERR_ARG, "workspace NULL or not 256-byte aligned");
  if (bytes < lay.total) return fail(LBM_ERR_ARG, "workspace of %zu bytes < %zu required", bytes, lay.total);
  if (!drho || !ux || !uy || !uz) return fail(LBM_ERR_ARG, "initial fields must not be NULL");
  lbm3d_ctx* c = new lbm3d_ctx();
  lbm::d3::Lat3& L = c->L;
  std::memset(&L, 0, sizeof(L));
  L.buf[0] = workspace;
  L.buf[1] = static_cast<char*>(workspace) + lay.buf_bytes;
  L.mx[0] = static_cast<char*>(workspace) + 2 * lay.buf_bytes;
  L.mx[1] = static_cast<char*>(workspace) + 2 * lay.buf_bytes + lay.mx_bytes;
  c->flag = reinterpret_cast<int*>(static_cast<char*>(workspace) + 2 * lay.buf_bytes + 2 * lay.mx_bytes);
  c->part = reinterpret_cast<float*>(static_cast<char*>(workspace) + 2 * lay.buf_bytes + 2 * lay.mx_bytes + 256);
  L.mxs = (int64_t)p->ny * p->nz;
  L.nx = p->nx;
  L.ny = p->ny;
  L.nz = p->nz;
  L.pitch = lay.pitch;
  L.slab = lay.slab;
  L.plane = lay.plane;
  for (int f = 0; f < 6; ++f) L.bc[f] = p->bc[f];
  L.store = p->store == LBM_STORE_F64   ? lbm::ST_F64
            : p->store == LBM_STORE_F32 ? lbm::ST_F32
            : p->store == LBM_STORE_F16DEV ? lbm::ST_F16
                                           : lbm::ST_BF16;
  L.q = lay.q;
  L.omega = 1.0 / p->tau;
  L.rho0 = p->rho0;
  L.gamma = p->gamma;
  c->stream = static_cast<hipStream_t>(hip_stream);
  // codec scales: FP16 stores g_i / w_i * 2^k with k chosen so that the
  // largest initial |g_i / w_i| 2^k is about 2^12; BF16 stores g_i / w_i
  int k = 0;
  if (p->store == LBM_STORE_F16DEV) {
    float host[256];
    hipError_t e = lbm::d3::launch_absmax3(L, drho, ux, uy, uz, c->part, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host, c->part, sizeof(host), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      delete c;
      return fail(LBM_ERR_HIP, "f16 exponent reduction: %s", hipGetErrorString(e));
    }
    float mx = 0.f;
    for (float v : host) mx = std::max(mx, v);
    if (!std::isfinite(mx)) {
      delete c;
      return fail(LBM_ERR_ARG, "initial fields are not finite");
    }
    k = lbm::host::f16_exp_from_max(mx);
  }
  c->f16_exp = k;
  for (int i = 0; i < 27; ++i) {
    const double w = L.q == 27 ? lbm::d3::w3<27, double>(i) : (i < 19 ? lbm::d3::w3<19, double>(i) : 1.0);
    const bool scaled = p->store == LBM_STORE_F16DEV || p->store == LBM_STORE_BF16DEV;
    L.es[i] = scaled ? (float)std::ldexp(1.0 / w, k) : 1.0f;  // 1/w_i: 3, 18, 36, 13.5, 54, 216 times 2^k, exact
    L.ds[i] = scaled ? (float)std::ldexp(w, -k) : 1.0f;
  }
  hipError_t e = lbm::d3::launch_init3(L, drho, ux, uy, uz, c->stream);
  if (e != hipSuccess) {
    delete c;
    return fail(LBM_ERR_HIP, "init: %s", hipGetErrorString(e));
  }
  *out = c;
  return LBM_OK;
}

int lbm3d_set_farfield(lbm3d_ctx* c, double beta, double rho, double ux, double uy, double uz) {
  if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
  if (!(beta >= 0.0 && beta <= 1.0)) return fail(LBM_ERR_ARG, "beta = %g outside [0, 1]", beta);
  if (!std::isfinite(rho) || !std::isfinite(ux) || !std::isfinite(uy) || !std::isfinite(uz))
    return fail(LBM_ERR_ARG, "reference vector must be finite");
  c->L.beta = beta;
  c->L.m0[0] = rho - c->L.rho0;
  c->L.m0[1] = ux;
  c->L.m0[2] = uy;
  c->L.m0[3] = uz;
  return LBM_OK;
}

int lbm3d_step(lbm3d_ctx* c, int32_t n) {
  const lbm::TraceRange trace_range("lbm3d_step");
  if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
  if (n < 0) return fail(LBM_ERR_ARG, "n = %d < 0", n);
  for (int32_t s = 0; s < n; ++s) {
    HIPCHK3(lbm::d3::launch3(c->L, c->parity, c->shape, c->stream));
    c->parity ^= 1;
    c->t += 1;
  }
  return LBM_OK;
}

int lbm3d_moments(lbm3d_ctx* c, double* out) {
  if (!c || !out) return fail(LBM_ERR_ARG, "NULL argument");
  HIPCHK3(lbm::d3::launch_moments3(c->L, c->parity, out, c->stream));
  return LBM_OK;
}

int lbm3d_get_populations(lbm3d_ctx* c, double* out) {
  if (!c || !out) return fail(LBM_ERR_ARG, "NULL argument");
  HIPCHK3(lbm::d3::launch_get_pops3(c->L, c->parity, out, c->stream));
  return LBM_OK;
}

int lbm3d_set_populations(lbm3d_ctx* c, const double* in) {
  if (!c || !in) return fail(LBM_ERR_ARG, "NULL argument");
  HIPCHK3(lbm::d3::launch_set_pops3(c->L, c->parity, in, c->stream));
  return LBM_OK;
}

int lbm3d_check_finite(lbm3d_ctx* c, int* ok) {
  if (!c || !ok) return fail(LBM_ERR_ARG, "NULL argument");
  int host = 0;
  HIPCHK3(hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
  HIPCHK3(lbm::d3::launch_finite3(c->L, c->parity, c->flag, c->stream));
  HIPCHK3(hipMemcpyAsync(&host, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK3(hipStreamSynchronize(c->stream));
  *ok = host ? 0 : 1;
  return host ? fail(LBM_ERR_NONFINITE, "populations hold a non-finite value at t = %lld", (long long)c->t) : LBM_OK;
}

int lbm3d_f16_exp(const lbm3d_ctx* c, int32_t* k) {
  if (!c || !k) return fail(LBM_ERR_ARG, "NULL argument");
  *k = c->f16_exp;
  return LBM_OK;
}

int lbm3d_time(const lbm3d_ctx* c, int64_t* t) {
  if (!c || !t) return fail(LBM_ERR_ARG, "NULL argument");
  *t = c->t;
  return LBM_OK;
}

int lbm3d_shape_count(void) { return lbm::d3::kNumAll3; }

int lbm3d_shape_describe(int32_t id, char* buf, size_t len) {
  if (!buf || len == 0) return fail(LBM_ERR_ARG, "NULL buffer");
  if (id < 0 || id >= lbm::d3::kNumAll3) return fail(LBM_ERR_ARG, "shape id %d out of range", id);
  if (id >= lbm::d3::kNumShapes3) {
    const lbm::d3::ShapePair& s = lbm::d3::kPairs3[id - lbm::d3::kNumShapes3];
    snprintf(buf, len, "pair:%dx%dxz%d", s.bx, s.by, s.zc);
    return LBM_OK;
  }
  const lbm::d3::Shape3& s = lbm::d3::kShapes3[id];
  snprintf(buf, len, "%dx%dxz%d%s", s.bx, s.by, s.zc, s.ntl ? "+ntl" : "");
  return LBM_OK;
}

int lbm3d_set_shape(lbm3d_ctx* c, int32_t id) {
  if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
  if (id < 0 || id >= lbm::d3::kNumAll3) return fail(LBM_ERR_ARG, "shape id %d out of range", id);
  if (!lbm::d3::shape3_supported(c->L, id))
    return fail(LBM_ERR_ARG, "shape %d: the pair shapes need FP16 or BF16 storage, non-periodic x faces and an even nx",
                id);
  c->shape = id;
  return LBM_OK;
}

int lbm3d_autotune(lbm3d_ctx* c, int32_t reps, int32_t* best, float* times_ms) {
  const lbm::TraceRange trace_range("lbm3d_autotune");
  if (!c || !best) return fail(LBM_ERR_ARG, "NULL argument");
  if (reps < 1 || reps > 1000) return fail(LBM_ERR_ARG, "reps = %d outside [1, 1000]", reps);
  std::vector<hipEvent_t> ev(2 * reps);
  for (auto& x : ev) HIPCHK3(hipEventCreate(&x));
  float best_t = 1e30f;
  int best_id = c->shape, rc = LBM_OK;
  for (int id = 0; id < lbm::d3::kNumAll3 && rc == LBM_OK; ++id) {
    if (!lbm::d3::shape3_supported(c->L, id)) {
      if (times_ms) times_ms[id] = -1.f;
      continue;
    }
    // a step reads buffer `parity` and writes only the other: the state is not advanced
    hipError_t e = lbm::d3::launch3(c->L, c->parity, id, c->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
      e = hipEventRecord(ev[2 * r], c->stream);
      if (e == hipSuccess) e = lbm::d3::launch3(c->L, c->parity, id, c->stream);
      if (e == hipSuccess) e = hipEventRecord(ev[2 * r + 1], c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    std::vector<float> ts(reps);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = hipEventElapsedTime(&ts[r], ev[2 * r], ev[2 * r + 1]);
    if (e != hipSuccess) {
      rc = fail(LBM_ERR_HIP, "3-D shape %d: %s", id, hipGetErrorString(e));
      break;
    }
    std::sort(ts.begin(), ts.end());
    if (times_ms) times_ms[id] = ts[reps / 2];
    if (ts[reps / 2] < best_t) {
      best_t = ts[reps / 2];
      best_id = id;
    }
  }
  for (auto& x : ev) (void)hipEventDestroy(x);
  if (rc) return rc;
  c->shape = best_id;
  *best = best_id;
  return LBM_OK;
}

void lbm3d_destroy(lbm3d_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  delete c;
}

}  // extern "C"
