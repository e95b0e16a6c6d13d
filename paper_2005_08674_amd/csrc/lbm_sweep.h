// lbm_sweep.h -- the per-tile bodies of the two sweep kernels, shared by
// the single-lattice kernels (lbm_kernels.hip) and the ensemble kernels
// (lbm_ensemble.hip): the bulk collide-stream tile and the NSBC edge segment.
#pragma once

#include "lbm_closure.h"
#include "lbm_device.h"
#include "lbm_mlp.h"

namespace lbm {

// Store of one population; NTS selects a non-temporal store (the written
// buffer is not read again before the next step streams it back in, so it
// should not displace the lines the shifted loads share).
template <bool NTS, class T>
__device__ inline void put(T* p, T v) {
  if (NTS) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Load of a population at byte offset `off` from plane base `base`, as a
// global-memory access: a buffer pointer read from a descriptor in memory
// (the ensemble's) is otherwise a generic one, whose FLAT loads also count
// against the LDS counter and so wait on the LDS traffic around them.
template <class T>
__device__ inline T ldg(const T* base, uint32_t off) {
  using GC = const __attribute__((address_space(1))) char;
  using GT = const __attribute__((address_space(1))) T;
  return *(GT*)((GC*)reinterpret_cast<const char*>(base) + off);
}

// The nine planes of an output buffer as global-memory bases, each held
// opaque in scalar registers: a store is then a scalar base plus the lane's
// 32-bit byte offset, instead of a 64-bit address formed per plane on every
// lane.
template <class T>
struct OutPlanes {
  using GC = __attribute__((address_space(1))) char;
  using GT = __attribute__((address_space(1))) T;
  GC* p[9];
  __device__ inline OutPlanes(T* B, int64_t plane) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      p[i] = (GC*)(reinterpret_cast<char*>(B + i * plane));
      asm volatile("" : "+s"(p[i]));
    }
  }
  template <bool NTS>
  __device__ inline void put(int i, uint32_t off, T v) const {
    GT* q = (GT*)(p[i] + off);
    if constexpr (NTS)
      __builtin_nontemporal_store(v, q);
    else
      *q = v;
  }
};

// Load of one population; NTL selects a non-temporal load, used only for the
// populations with c_x = 0, whose cache lines no other wavefront reads.
template <class T>
__device__ inline T get(const T* p, bool nt) {
  if (nt) return __builtin_nontemporal_load(p);
  return *p;
}

// One bulk tile: BX x (BY * NYT) interior nodes starting at tile (txi, tyi)
// of lattice L -- pull, collide on the values as stored (collide_stored),
// store (eqs. lbe_0, lbe_1, feq_1).
template <int S, int BX, int BY, int NYT, bool NTS, bool NTL>
__device__ inline void bulk_tile_body(const LatDesc& L, int parity, int txi, int tyi) {
  using C = Codec<S>;
  using T = typename C::T;
  using R = typename C::R;
  const int x = txi * BX + threadIdx.x;
  if (x < 1 || x > L.nx - 2) return;
  const int y0 = 1 + tyi * (BY * NYT) + threadIdx.y;
  const int pitch = L.pitch;
  const T* __restrict__ A = static_cast<const T*>(buf_of(L, parity));
  T* __restrict__ B = static_cast<T*>(buf_of(L, parity ^ 1));
  const int64_t plane = L.plane;
  const R rho0 = R(L.rho0), omega = R(L.omega);
  const Base<R> base(L);

  // Interior nodes pull from inside the lattice: every access is a per-plane
  // (uniform) base pointer plus a 32-bit unsigned byte offset (a plane is
  // below 4 GiB), one per source row, with the x shift as a constant.
  R g[NYT][9];
#pragma unroll
  for (int j = 0; j < NYT; ++j) {
    const int y = y0 + j * BY;
    if (y <= L.ny - 2) {
      const uint32_t idx = (uint32_t)(y * pitch + x);
      const uint32_t ro[3] = {(idx + (uint32_t)pitch) * (uint32_t)sizeof(T), idx * (uint32_t)sizeof(T),
                              (idx - (uint32_t)pitch) * (uint32_t)sizeof(T)};
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const char* Ai = reinterpret_cast<const char*>(A + i * plane);
        g[j][i] = C::raw(get(reinterpret_cast<const T*>(Ai + ro[1 + kCy[i]] - kCx[i] * (int)sizeof(T)),
                             NTL && kCx[i] == 0));
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NYT; ++j) {
    const int y = y0 + j * BY;
    if (y <= L.ny - 2) {
      collide_stored<S, -1>(L, g[j], rho0, base, omega);
      const uint32_t off = (uint32_t)(y * pitch + x) * (uint32_t)sizeof(T);
#pragma unroll
      for (int i = 0; i < 9; ++i)
        put<NTS>(reinterpret_cast<T*>(reinterpret_cast<char*>(B + i * plane) + off), C::raw_enc(g[j][i]));
    }
  }
}

constexpr int SEG = 64;    // boundary nodes per block (one wavefront)
constexpr int HALO = 2;    // tangential halo of the staged strip
constexpr int DEPTH = 3;   // staged depths 0..2 along the inward normal
constexpr int STRIP = SEG + 2 * HALO;

__host__ __device__ inline int edge_segments_v(int ny) { return (ny + SEG - 1) / SEG; }
__host__ __device__ inline int edge_segments_h(int nx) { return (nx - 2 + SEG - 1) / SEG; }

// Node of edge `edge` at depth d (along the inward normal) and tangential
// coordinate t (y for left/right, x for bottom/top).
__device__ inline void edge_node(const LatDesc& L, int edge, int d, int t, int& x, int& y) {
  switch (edge) {
    case E_LEFT: x = d; y = t; break;
    case E_RIGHT: x = L.nx - 1 - d; y = t; break;
    case E_BOTTOM: x = t; y = d; break;
    default: x = t; y = L.ny - 1 - d; break;
  }
}

template <class R>
__device__ inline R normal_diff(R mb, R m1, R m2, int order) {
  return order == 1 ? mb - m1 : (R(3) * mb - R(4) * m1 + m2) * R(0.5);
}

constexpr int EDGE_THREADS = 256;  // >= DEPTH * STRIP: one staged strip node per thread
static_assert(EDGE_THREADS >= DEPTH * STRIP, "edge block must cover the staged strip");

// Block index -> (edge, segment) of a lattice: left segments first, then
// right, bottom, top.  Left/right segments cover y = 0..ny-1 (corners
// included), bottom/top segments cover x = 1..nx-2.
__host__ __device__ inline void edge_of_block(int nx, int ny, int& b, int& edge) {
  const int nsv = edge_segments_v(ny), nsh = edge_segments_h(nx);
  if (b < nsv) {
    edge = E_LEFT;
  } else if (b < 2 * nsv) {
    edge = E_RIGHT;
    b -= nsv;
  } else if (b < 2 * nsv + nsh) {
    edge = E_BOTTOM;
    b -= 2 * nsv;
  } else {
    edge = E_TOP;
    b -= 2 * nsv + nsh;
  }
}

// LDS of the closure path of the edge kernel: strip features, the 64 x 96
// network input tile, the two hidden tiles and the outputs.
struct ClosureLds {
  float feat[NODE_FEAT][DEPTH][STRIP];
  __attribute__((aligned(16))) mlp::bf16 X[SEG * mlp::XS];
  __attribute__((aligned(16))) mlp::bf16 H1[SEG * mlp::HS];
  __attribute__((aligned(16))) mlp::bf16 H2[SEG * mlp::HS];
  float Y[SEG][4];
  int gate[SEG];  // 1 where the correction may apply (eligible node, amplitude > 0 after the gate)
};

// One 64-node segment `b` of edge `edge` of lattice L, computed by a block of
// EDGE_THREADS threads: lanes 0..SEG-1 own one boundary node each.  With
// CLOSURE the NSBC vector m_c of every node with a single NSBC normal is
// corrected by the closure network (NSBC stays the fallback when the output
// is not finite or leaves the trust bound); corners keep NSBC.
template <int S, bool CLOSURE>
__device__ inline void edge_segment_body(const LatDesc& L, int parity, int edge, int b,
                                         typename Codec<S>::R (&mom)[3][DEPTH][STRIP], ClosureLds* cl) {
  using C = Codec<S>;
  using T = typename C::T;
  using R = typename C::R;
  const int nx = L.nx, ny = L.ny;
  const bool vertical = edge == E_LEFT || edge == E_RIGHT;
  const int ntan = vertical ? ny : nx;
  const int t0 = vertical ? b * SEG : 1 + b * SEG;
  const int tend = vertical ? ny : nx - 1;
  const bool xper = L.bc[E_LEFT] == BC_PERIODIC;
  const bool yper = L.bc[E_BOTTOM] == BC_PERIODIC;
  const bool tan_per = vertical ? yper : xper;
  const bool any_nsbc = !(xper && yper);
  // outward normal of this edge and the sign taking the tangent t = (-n_y, n_x)
  // to increasing tangential coordinate
  const int enx = edge == E_LEFT ? -1 : (edge == E_RIGHT ? 1 : 0);
  const int eny = edge == E_BOTTOM ? -1 : (edge == E_TOP ? 1 : 0);
  const int tsign = (edge == E_RIGHT || edge == E_BOTTOM) ? 1 : -1;

  const T* __restrict__ A = static_cast<const T*>(buf_of(L, parity));
  T* __restrict__ B = static_cast<T*>(buf_of(L, parity ^ 1));
  const int pitch = L.pitch;
  const int64_t plane = L.plane;
  const R rho0 = R(L.rho0);
  const Base<R> base(L);
  // linear thread index: the edge body also runs in the fused step kernels,
  // whose blocks are 2-D and may hold more than EDGE_THREADS threads (the
  // extra ones only pass the barriers)
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;

  // Lanes 0..SEG-1 own one boundary node each: pull its known populations
  // (wrapping across periodic edges) and mark those whose source lies
  // outside the domain.  Issued before the strip staging so both sets of
  // loads are in flight together.
  const int t = t0 + tid;
  const bool owner = tid < SEG && t < tend;
  int x = 0, y = 0;
  R g[9];
  uint32_t unknown = 0;
  if (owner) {
    edge_node(L, edge, 0, t, x, y);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      int sx = x - kCx[i], sy = y - kCy[i];
      const bool outx = sx < 0 || sx >= nx;
      const bool outy = sy < 0 || sy >= ny;
      if ((outx && !xper) || (outy && !yper)) {
        unknown |= 1u << i;
        g[i] = R(0);
      } else {
        if (outx) sx = sx < 0 ? sx + nx : sx - nx;
        if (outy) sy = sy < 0 ? sy + ny : sy - ny;
        g[i] = C::dec(A[i * plane + (sy * pitch + sx)], L.ds[i]);
      }
    }
  }

  // Stage the time-t moments (and, with CLOSURE, the strip features) of the
  // strip (depth 0..2, tangential halo 2), one strip node per thread.
  if (any_nsbc && tid < DEPTH * STRIP) {
    const int d = tid / STRIP, tt = tid - d * STRIP;
    int ts = t0 - HALO + tt;
    bool inside = true;
    if (ts < 0 || ts >= ntan) {
      if (tan_per) ts = ts < 0 ? ts + ntan : ts - ntan;
      else inside = false;
    }
    R m[3] = {R(0), R(0), R(0)};
    float f[NODE_FEAT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (inside) {
      int sx, sy;
      edge_node(L, edge, d, ts, sx, sy);
      R gs[9];
      const int idx = sy * pitch + sx;
#pragma unroll
      for (int i = 0; i < 9; ++i) gs[i] = C::dec(A[i * plane + idx], L.ds[i]);
      moments<R>(gs, rho0, base, m[0], m[1], m[2]);
      if (CLOSURE) {
        const R ref[3] = {R(L.m0[0]), R(L.m0[1]), R(L.m0[2])};
        strip_node_features<R>(gs, rho0, base, ref, enx, eny, f);
      }
    }
    mom[0][d][tt] = m[0];
    mom[1][d][tt] = m[1];
    mom[2][d][tt] = m[2];
    if (CLOSURE) {
#pragma unroll
      for (int q = 0; q < NODE_FEAT; ++q) cl->feat[q][d][tt] = f[q];
    }
  }
  __syncthreads();

  const bool onL = owner && x == 0 && L.bc[E_LEFT] == BC_NSBC;
  const bool onR = owner && x == nx - 1 && L.bc[E_RIGHT] == BC_NSBC;
  const bool onB = owner && y == 0 && L.bc[E_BOTTOM] == BC_NSBC;
  const bool onT = owner && y == ny - 1 && L.bc[E_TOP] == BC_NSBC;
  const bool nsbc_node = onL || onR || onB || onT;
  const int tt = tid + HALO;
  const bool own = (edge == E_LEFT && onL) || (edge == E_RIGHT && onR) || (edge == E_BOTTOM && onB) ||
                   (edge == E_TOP && onT);
  int nn = 0;
  M3<R> mc;
  if (nsbc_node) {
    R dsum[3] = {R(0), R(0), R(0)};
    // eq. nes_2: outward normal derivative by a one-sided difference, time t
    if (own) {
      ++nn;
#pragma unroll
      for (int c = 0; c < 3; ++c) dsum[c] += normal_diff(mom[c][0][tt], mom[c][1][tt], mom[c][2][tt], L.grad_order);
    }
    if (vertical && (onB || onT)) {  // corner node: second normal runs along this strip
      const int sgn = onB ? 1 : -1;
      ++nn;
#pragma unroll
      for (int c = 0; c < 3; ++c)
        dsum[c] += normal_diff(mom[c][0][tt], mom[c][0][tt + sgn], mom[c][0][tt + 2 * sgn], L.grad_order);
    }
    R fac = R(L.gamma);
    if (nn == 2) fac *= L.corner_mode == 0 ? R(0.70710678118654752440) : R(0.5);
    const R beta = R(L.beta);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const R mp = mom[c][0][tt] - fac * dsum[c];
      mc.v[c] = (R(1) - beta) * mp + beta * R(L.m0[c]);  // eq. nes_3
    }
  }

  if (CLOSURE) {
    const mlp::Net& net = *static_cast<const mlp::Net*>(L.net);
    const bool eligible = nsbc_node && own && nn == 1;
    float amp = 0.f;
    if (tid < SEG) {
      // network input row of this lane: strip features, omega, m_c and m0 in the (n, t) frame
      float xin[mlp::IN];
      if (eligible) {
#pragma unroll
        for (int d = 0; d < DEPTH; ++d)
#pragma unroll
          for (int k = -1; k <= 1; ++k)
#pragma unroll
            for (int q = 0; q < NODE_FEAT; ++q) xin[(3 * d + k + 1) * NODE_FEAT + q] = cl->feat[q][d][tt + tsign * k];
        const R mcv[3] = {mc.v[0], mc.v[1], mc.v[2]};
        const R ref[3] = {R(L.m0[0]), R(L.m0[1]), R(L.m0[2])};
        float refn[3], dmc[3];
        to_normal_frame<R>(ref, base, enx, eny, refn);
        normal_frame_diff<R>(mcv, ref, enx, eny, dmc);
        amp = finish_inputs(xin, float(L.rho0), float(L.omega), dmc, refn);
        if (!vortical(xin, float(L.rho0), net.kmin)) amp = 0.f;  // outside the gated regime: NSBC's m_c
      }
      mlp::bf16* row = cl->X + tid * mlp::XS;
#pragma unroll
      for (int q = 0; q < mlp::IN; ++q) row[q] = eligible ? normalised_input(net, q, xin[q]) : (mlp::bf16)0.f;
      cl->gate[tid] = eligible && amp > 0.f;
    }
    __syncthreads();
    {
      const int w = tid >> 6;  // wavefront w runs rows 16 w .. 16 w + 15
      // (a group with no row the correction may apply to skips the network: its outputs are unused)
      int any = 0;
#pragma unroll
      for (int r = 0; r < 16; ++r) any |= cl->gate[16 * w + r];
      if (any) {
        mlp::f32x4 yv;
        mlp::forward16(net, cl->X + 16 * w * mlp::XS, cl->H1 + 16 * w * mlp::HS, cl->H2 + 16 * w * mlp::HS, yv);
        const int l = tid & 63, col = l & 15;
        if (col < 3) {
#pragma unroll
          for (int r = 0; r < 4; ++r) cl->Y[16 * w + 4 * (l >> 4) + r][col] = yv[r];
        }
      }
    }
    __syncthreads();
    float dl[3];
    if (eligible && amp > 0.f && closure_delta(net, cl->Y[tid][0], cl->Y[tid][1], cl->Y[tid][2], amp, enx, eny, dl)) {
#pragma unroll
      for (int c = 0; c < 3; ++c) mc.v[c] += R(dl[c]);
    }
  }
  if (!owner) return;
  // Dirichlet velocity edge (left or right, bottom and top periodic): the
  // prescribed velocity and the density the known populations fix, then the
  // same assignment and correction as NSBC
  const int vel_nx = (x == 0 && L.bc[E_LEFT] == BC_VELOCITY) ? -1 : ((x == nx - 1 && L.bc[E_RIGHT] == BC_VELOCITY) ? 1 : 0);
  if (vel_nx) {
    mc = velocity_edge_moments<R>(g, vel_nx, rho0, in_type<R>(L.uw[0], L.uwf[0]), in_type<R>(L.duw[0], L.duwf[0]),
                                  in_type<R>(L.duw[1], L.duwf[1]));
  }
  if (nsbc_node || vel_nx) nsbc_assign_correct<R>(g, unknown, mc, rho0, base, L.corr_mode);
  collide<R>(L, g, rho0, base, R(L.omega));
  const int idx = y * pitch + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) put<true>(B + i * plane + idx, C::enc(g[i], L.es[i]));
}

}  // namespace lbm
