// lbm_kernels.hip -- gfx950 kernels of the D2Q9 BGK + NSBC sweep and its
// helpers (initialisation, moments, population export/import, finiteness,
// fp64 energy reduction) plus their host-side launchers.
//
// Bulk kernel: fused pull-streaming + BGK collision (eqs. lbe_0, lbe_1,
// feq_1) over the interior nodes 1 <= x <= nx-2, 1 <= y <= ny-2.  Pure
// streaming work: 9 loads and 9 stores per node, no data reuse except the
// +-1 shifted cache lines of neighbouring wavefronts, so it is bound by HBM
// bandwidth.  Threads map to consecutive x (coalesced, 64-wide wavefronts);
// stores are aligned, the x-shifted loads straddle one extra line per
// wavefront which the same CU / XCD L2 serves.  An optional block remap
// gives every XCD a contiguous band of tiles so that those shared lines stay
// in one L2.
//
// Edge kernel: the perimeter nodes.  One 64-lane block per segment of an
// edge stages the moments of a 3-deep, (64 + 4)-wide strip of the previous
// step in LDS, then each lane pulls its known populations (wrapping across
// periodic edges), rebuilds the unknown ones with NSBC (Sec. 5) and collides.
#include <hip/hip_runtime.h>

#include <cmath>

#include "lbm_device.h"
#include "lbm_launch.h"
#include "lbm_sweep.h"

namespace lbm {

// ------------------------------------------------------------------ bulk kernel
// Block -> tile maps.  Workgroups are dispatched to the 8 XCDs round-robin
// (workgroup b runs on XCD b mod 8), and each XCD has its own L2.
//   REMAP 0: tile = b (row-major tiles, consecutive tiles on different XCDs).
//   REMAP 1: XCD k takes the k-th contiguous eighth of the tiles.
//   REMAP 2: XCD k takes the tile rows r = k (mod 8) and walks each row in x,
//            so the x-neighbours that share the shifted loads' straddling
//            cache lines run back to back on one XCD, while the eight XCDs
//            still work on eight adjacent rows.
//   REMAP 3: block b sweeps the whole tile row b in x (a loop over the
//            tiles), so every straddling cache line of the x-shifted loads is
//            shared inside one workgroup and fetched from HBM once.
//   REMAP 4: in each run of 64 blocks, XCD k takes 8 consecutive tiles
//            (tiles 64 g + 8 k .. 64 g + 8 k + 7), so only one tile boundary
//            in 8 crosses XCDs, while the 64 blocks in flight still cover one
//            contiguous stretch of tiles as in REMAP 0.
template <int REMAP>
__device__ inline bool bulk_tile(int b, int tiles_x, int tiles_y, int& txi, int& tyi) {
  if (REMAP == 2) {
    const int seq = b >> 3;
    const int grp = seq / tiles_x;
    txi = seq - grp * tiles_x;
    tyi = grp * 8 + (b & 7);
    return tyi < tiles_y;
  }
  const int ntiles = tiles_x * tiles_y;
  int tile = b;
  if (REMAP == 4) tile = (b & ~63) + ((b & 7) << 3) + ((b >> 3) & 7);
  if (REMAP == 1) {
    const int per = (ntiles + 7) >> 3;
    tile = (b & 7) * per + (b >> 3);
  }
  if (tile >= ntiles) return false;
  tyi = tile / tiles_x;
  txi = tile - tyi * tiles_x;
  return true;
}

// Bulk block b (in the launch's own numbering) of the tile grid.
template <int S, int BX, int BY, int NYT, int REMAP, bool NTS, bool NTL>
__device__ inline void bulk_block(const LatDesc& L, int parity, int b, int tiles_x, int tiles_y) {
  if (REMAP == 3) {
    const int tyi = b;
    if (tyi >= tiles_y) return;
    for (int txi = 0; txi < tiles_x; ++txi) bulk_tile_body<S, BX, BY, NYT, NTS, NTL>(L, parity, txi, tyi);
    return;
  }
  int txi, tyi;
  if (!bulk_tile<REMAP>(b, tiles_x, tiles_y, txi, tyi)) return;
  bulk_tile_body<S, BX, BY, NYT, NTS, NTL>(L, parity, txi, tyi);
}

template <int S, int BX, int BY, int NYT, int REMAP, bool NTS, bool NTL>
__global__ __launch_bounds__(BX* BY) void k_bulk(LatDesc L, int parity, int tiles_x, int tiles_y) {
  bulk_block<S, BX, BY, NYT, REMAP, NTS, NTL>(L, parity, blockIdx.x, tiles_x, tiles_y);
}

// One launch per step: blocks [0, eblocks) run the edge kernel's segments,
// the rest the bulk tiles (numbered from a multiple of 8, so the XCD-aware
// block maps keep their meaning).  Both halves read buffer `parity` and write
// disjoint nodes of the other buffer, exactly as the two separate launches.
template <int S, int BX, int BY, int NYT, int REMAP, bool NTS, bool NTL>
__global__ __launch_bounds__(BX* BY) void k_step(LatDesc L, int parity, int tiles_x, int tiles_y, int eblocks,
                                                 int eoffset) {
  __shared__ typename Codec<S>::R mom[3][DEPTH][STRIP];
  const int b = blockIdx.x;
  if (b < eoffset) {
    if (b >= eblocks) return;  // padding to the multiple of 8 (uniform per block)
    int seg = b, edge;
    edge_of_block(L.nx, L.ny, seg, edge);
    edge_segment_body<S, false>(L, parity, edge, seg, mom, nullptr);
    return;
  }
  bulk_block<S, BX, BY, NYT, REMAP, NTS, NTL>(L, parity, b - eoffset, tiles_x, tiles_y);
}

struct TileShape {
  int bx, by, nyt, remap;
  bool nts, ntl;
};

// Candidate launch shapes of the bulk kernel: block (BX x BY), nodes per
// thread along y (NYT), block -> tile map (REMAP), non-temporal stores (NTS),
// non-temporal loads of the unshifted populations (NTL).
#define LBM_TILES(X)                   \
  X(256, 1, 1, 0, true, false)         \
  X(256, 1, 2, 0, true, false)         \
  X(256, 1, 4, 0, true, false)         \
  X(128, 2, 1, 0, true, false)         \
  X(128, 2, 2, 0, true, false)         \
  X(64, 4, 1, 0, true, false)          \
  X(64, 4, 2, 0, true, false)          \
  X(64, 8, 1, 0, true, false)          \
  X(128, 4, 1, 0, true, false)         \
  X(512, 1, 1, 0, true, false)         \
  X(1024, 1, 1, 0, true, false)        \
  X(256, 1, 1, 1, true, false)         \
  X(128, 2, 1, 1, true, false)         \
  X(256, 1, 1, 2, true, false)         \
  X(256, 1, 2, 2, true, false)         \
  X(512, 1, 1, 2, true, false)         \
  X(128, 2, 1, 2, true, false)         \
  X(64, 4, 1, 2, true, false)          \
  X(256, 1, 1, 2, true, true)          \
  X(512, 1, 1, 2, true, true)          \
  X(256, 1, 1, 0, true, true)          \
  X(512, 1, 1, 0, true, true)          \
  X(256, 1, 1, 0, false, false)        \
  X(256, 1, 2, 0, false, false)        \
  X(128, 2, 1, 0, false, false)        \
  X(64, 4, 1, 0, false, false)         \
  X(256, 1, 1, 3, true, true)          \
  X(256, 1, 1, 3, true, false)         \
  X(512, 1, 1, 3, true, true)          \
  X(1024, 1, 1, 3, true, true)         \
  X(256, 1, 2, 3, true, true)          \
  X(128, 2, 1, 3, true, true)          \
  X(256, 1, 2, 3, true, false)        \
  X(256, 1, 1, 4, true, true)          \
  X(256, 1, 1, 4, true, false)         \
  X(512, 1, 1, 4, true, true)          \
  X(128, 2, 1, 4, true, false)         \
  X(256, 1, 2, 4, true, false)

static const TileShape kTiles[] = {
#define X(a, b, c, d, e, f) {a, b, c, d, e, f},
    LBM_TILES(X)
#undef X
};
static constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

int num_tiles() { return kNumTiles; }

void tile_name(int id, char* buf, size_t len) {
  if (id < 0 || id >= kNumTiles) {
    snprintf(buf, len, "invalid");
    return;
  }
  const TileShape& t = kTiles[id];
  snprintf(buf, len, "%dx%dx%d%s%s%s", t.bx, t.by, t.nyt,
           t.remap == 1 ? "+xcdband"
                        : (t.remap == 2 ? "+xcdrow" : (t.remap == 3 ? "+rowsweep" : (t.remap == 4 ? "+xcd8" : ""))),
           t.nts ? "+nts" : "", t.ntl ? "+ntl" : "");
}

int edge_blocks(int nx, int ny);

template <int S, int BX, int BY, int NYT, int REMAP, bool NTS, bool NTL>
static hipError_t launch_step_t(const LatDesc& L, int parity, hipStream_t s) {
  const int tiles_x = (L.nx + BX - 1) / BX;
  const int tiles_y = (L.ny - 2 + BY * NYT - 1) / (BY * NYT);
  int grid;
  if (REMAP == 0) grid = tiles_x * tiles_y;
  else if (REMAP == 1) grid = ((tiles_x * tiles_y + 7) >> 3) * 8;
  else if (REMAP == 2) grid = tiles_x * ((tiles_y + 7) >> 3) * 8;
  else if (REMAP == 4) grid = ((tiles_x * tiles_y + 63) >> 6) * 64;
  else grid = tiles_y;
  const int eb = edge_blocks(L.nx, L.ny);
  const int eo = (eb + 7) & ~7;
  k_step<S, BX, BY, NYT, REMAP, NTS, NTL><<<dim3(eo + grid), dim3(BX, BY), 0, s>>>(L, parity, tiles_x, tiles_y,
                                                                                   eb, eo);
  return hipGetLastError();
}

template <int S>
static hipError_t launch_step_s(const LatDesc& L, int parity, int tile, hipStream_t s) {
  int id = 0;
#define X(a, b, c, d, e, f)                                                \
  if (tile == id) return launch_step_t<S, a, b, c, d, e, f>(L, parity, s); \
  ++id;
  LBM_TILES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_step(const LatDesc& L, int parity, int tile, hipStream_t s) {
  if (L.closure && L.net) return hipErrorInvalidValue;
  switch (L.store) {
    case ST_F64: return launch_step_s<ST_F64>(L, parity, tile, s);
    case ST_F32: return launch_step_s<ST_F32>(L, parity, tile, s);
    case ST_F16: return launch_step_s<ST_F16>(L, parity, tile, s);
    case ST_BF16: return launch_step_s<ST_BF16>(L, parity, tile, s);
  }
  return hipErrorInvalidValue;
}

template <int S, int BX, int BY, int NYT, int REMAP, bool NTS, bool NTL>
static hipError_t launch_bulk_t(const LatDesc& L, int parity, hipStream_t s) {
  const int tiles_x = (L.nx + BX - 1) / BX;
  const int tiles_y = (L.ny - 2 + BY * NYT - 1) / (BY * NYT);
  if (tiles_x <= 0 || tiles_y <= 0) return hipSuccess;
  int grid;
  if (REMAP == 0) grid = tiles_x * tiles_y;
  else if (REMAP == 1) grid = ((tiles_x * tiles_y + 7) >> 3) * 8;
  else if (REMAP == 2) grid = tiles_x * ((tiles_y + 7) >> 3) * 8;
  else if (REMAP == 4) grid = ((tiles_x * tiles_y + 63) >> 6) * 64;
  else grid = tiles_y;
  k_bulk<S, BX, BY, NYT, REMAP, NTS, NTL><<<dim3(grid), dim3(BX, BY), 0, s>>>(L, parity, tiles_x, tiles_y);
  return hipGetLastError();
}

template <int S>
static hipError_t launch_bulk_s(const LatDesc& L, int parity, int tile, hipStream_t s) {
  int id = 0;
#define X(a, b, c, d, e, f)                                                \
  if (tile == id) return launch_bulk_t<S, a, b, c, d, e, f>(L, parity, s); \
  ++id;
  LBM_TILES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_bulk(const LatDesc& L, int parity, int tile, hipStream_t s) {
  switch (L.store) {
    case ST_F64: return launch_bulk_s<ST_F64>(L, parity, tile, s);
    case ST_F32: return launch_bulk_s<ST_F32>(L, parity, tile, s);
    case ST_F16: return launch_bulk_s<ST_F16>(L, parity, tile, s);
    case ST_BF16: return launch_bulk_s<ST_BF16>(L, parity, tile, s);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ edge kernel
template <int S>
__global__ __launch_bounds__(EDGE_THREADS) void k_edge(LatDesc L, int parity) {
  __shared__ typename Codec<S>::R mom[3][DEPTH][STRIP];
  int b = blockIdx.x, edge;
  edge_of_block(L.nx, L.ny, b, edge);
  edge_segment_body<S, false>(L, parity, edge, b, mom, nullptr);
}

// The edge kernel with the learned closure (NSBC fallback).
template <int S>
__global__ __launch_bounds__(EDGE_THREADS) void k_edge_closure(LatDesc L, int parity) {
  __shared__ typename Codec<S>::R mom[3][DEPTH][STRIP];
  __shared__ ClosureLds cl;
  int b = blockIdx.x, edge;
  edge_of_block(L.nx, L.ny, b, edge);
  edge_segment_body<S, true>(L, parity, edge, b, mom, &cl);
}

int edge_blocks(int nx, int ny) { return 2 * edge_segments_v(ny) + 2 * edge_segments_h(nx); }

hipError_t launch_edge(const LatDesc& L, int parity, hipStream_t s) {
  const dim3 grid(edge_blocks(L.nx, L.ny)), block(EDGE_THREADS);
  const bool cl = L.closure && L.net;
#define LBM_EDGE(ST)                                                            \
  if (cl) k_edge_closure<ST><<<grid, block, 0, s>>>(L, parity);                \
  else k_edge<ST><<<grid, block, 0, s>>>(L, parity);
  switch (L.store) {
    case ST_F64: LBM_EDGE(ST_F64) break;
    case ST_F32: LBM_EDGE(ST_F32) break;
    case ST_F16: LBM_EDGE(ST_F16) break;
    case ST_BF16: LBM_EDGE(ST_BF16) break;
    default: return hipErrorInvalidValue;
  }
#undef LBM_EDGE
  return hipGetLastError();
}

// ------------------------------------------------------------------ helpers
// Equilibrium deviations in fp64 for the initial state, encoded to the store.
template <int S>
__global__ void k_init(LatDesc L, int parity, const double* __restrict__ drho, const double* __restrict__ ux,
                       const double* __restrict__ uy) {
  using C = Codec<S>;
  using T = typename C::T;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= L.nx) return;
  const int64_t k = (int64_t)y * L.nx + x;
  double geq[9];
  const Base<double> base(L);
  equilibrium<double>(L.rho0, base, drho[k], ux[k] - L.ub[0], uy[k] - L.ub[1], geq);
  T* B = static_cast<T*>(buf_of(L, parity));
  const int idx = y * L.pitch + x;
  // scale in fp64 (the encode scales are exact powers of two over w_i), then
  // round once to the stored type
#pragma unroll
  for (int i = 0; i < 9; ++i)
    B[i * L.plane + idx] = C::enc(typename C::R(geq[i] * (double)L.es[i]), 1.0f);
}

// Per-block maximum of |geq_i / w_i| over the initial fields (FP16 exponent choice).
__global__ void k_absmax_init(LatDesc L, const double* __restrict__ drho, const double* __restrict__ ux,
                              const double* __restrict__ uy, float* partial) {
  __shared__ float red[256];
  float mx = 0.f;
  const int64_t n = (int64_t)L.nx * L.ny;
  const Base<double> base(L);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    double geq[9];
    equilibrium<double>(L.rho0, base, drho[k], ux[k] - L.ub[0], uy[k] - L.ub[1], geq);
#pragma unroll
    for (int i = 0; i < 9; ++i) mx = fmaxf(mx, (float)fabs(geq[i] / wgt<double>(i)));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Decoded populations of node (x, y) in fp64, for any store (runtime switch).
__device__ inline void load_node_f64(const LatDesc& L, int parity, int x, int y, double g[9]) {
  const int idx = y * L.pitch + x;
  switch (L.store) {
    case ST_F64: {
      const double* A = static_cast<const double*>(buf_of(L, parity));
#pragma unroll
      for (int i = 0; i < 9; ++i) g[i] = A[i * L.plane + idx];
      break;
    }
    case ST_F32: {
      const float* A = static_cast<const float*>(buf_of(L, parity));
#pragma unroll
      for (int i = 0; i < 9; ++i) g[i] = A[i * L.plane + idx];
      break;
    }
    case ST_F16: {
      const _Float16* A = static_cast<const _Float16*>(buf_of(L, parity));
#pragma unroll
      for (int i = 0; i < 9; ++i) g[i] = (double)Codec<ST_F16>::dec(A[i * L.plane + idx], L.ds[i]);
      break;
    }
    default: {
      const uint16_t* A = static_cast<const uint16_t*>(buf_of(L, parity));
#pragma unroll
      for (int i = 0; i < 9; ++i) g[i] = (double)Codec<ST_BF16>::dec(A[i * L.plane + idx], L.ds[i]);
      break;
    }
  }
}

// rho - rho0 and the absolute velocity of node (x, y), in fp64.
__device__ inline void node_moments_f64(const LatDesc& L, int parity, int x, int y, double& dr, double& ux,
                                        double& uy) {
  double g[9];
  load_node_f64(L, parity, x, y, g);
  const Base<double> base(L);
  moments<double>(g, L.rho0, base, dr, ux, uy);
  ux += L.ub[0];
  uy += L.ub[1];
}

__global__ void k_moments(LatDesc L, int parity, void* out_r, void* out_u, void* out_v, int f64, int deviation) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= L.nx) return;
  double dr, ux, uy;
  node_moments_f64(L, parity, x, y, dr, ux, uy);
  const double r = deviation ? dr : L.rho0 + dr;
  const int64_t k = (int64_t)y * L.nx + x;
  if (f64) {
    if (out_r) static_cast<double*>(out_r)[k] = r;
    if (out_u) static_cast<double*>(out_u)[k] = ux;
    if (out_v) static_cast<double*>(out_v)[k] = uy;
  } else {
    if (out_r) static_cast<float*>(out_r)[k] = (float)r;
    if (out_u) static_cast<float*>(out_u)[k] = (float)ux;
    if (out_v) static_cast<float*>(out_v)[k] = (float)uy;
  }
}

__global__ void k_get_pops(LatDesc L, int parity, double* out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= L.nx) return;
  double g[9];
  load_node_f64(L, parity, x, y, g);
  const int64_t n = (int64_t)L.nx * L.ny, k = (int64_t)y * L.nx + x;
  // f_i - w_i rho0 = g_i + w_i rho0 (P_i(u_b) - 1)
#pragma unroll
  for (int i = 0; i < 9; ++i) out[i * n + k] = g[i] + wgt<double>(i) * L.rho0 * (L.pb[i] - 1.0);
}

template <int S>
__global__ void k_set_pops(LatDesc L, int parity, const double* __restrict__ in) {
  using C = Codec<S>;
  using T = typename C::T;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= L.nx) return;
  const int64_t n = (int64_t)L.nx * L.ny, k = (int64_t)y * L.nx + x;
  T* B = static_cast<T*>(buf_of(L, parity));
  const int idx = y * L.pitch + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double g = in[i * n + k] - wgt<double>(i) * L.rho0 * (L.pb[i] - 1.0);
    B[i * L.plane + idx] = C::enc(typename C::R(g * (double)L.es[i]), 1.0f);
  }
}

__global__ void k_finite(LatDesc L, int parity, int* bad) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= L.nx) return;
  double g[9];
  load_node_f64(L, parity, x, y, g);
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 9; ++i) ok = ok && isfinite(g[i]);
  if (!ok) *bad = 1;
}

// Acoustic-energy reduction in fp64, fixed order: a fixed grid strides over
// the test nodes, every block reduces in a fixed tree and writes one partial;
// k_sum_partials adds the partials in a fixed tree.
constexpr int EN_BLOCK = 256;
constexpr int EN_GRID = 1024;

__global__ __launch_bounds__(EN_BLOCK) void k_energy(LatDesc T_, int pt, LatDesc R_, int pr, int has_ref, int xo,
                                                    int yo, double ux_ref, double uy_ref, double* partial) {
  __shared__ double red[EN_BLOCK];
  double acc = 0.0;
  const int64_t n = (int64_t)T_.nx * T_.ny;
  const double cs2 = 1.0 / 3.0, rho0 = T_.rho0;
  for (int64_t k = (int64_t)blockIdx.x * EN_BLOCK + threadIdx.x; k < n; k += (int64_t)EN_GRID * EN_BLOCK) {
    const int y = (int)(k / T_.nx), x = (int)(k - (int64_t)y * T_.nx);
    double dr, ux, uy;
    node_moments_f64(T_, pt, x, y, dr, ux, uy);
    double rr = 0.0, ru = ux_ref, rv = uy_ref;
    if (has_ref) node_moments_f64(R_, pr, x + xo, y + yo, rr, ru, rv);
    const double a = dr - rr, b = ux - ru, c = uy - rv;
    acc += 0.5 * (cs2 * a * a / rho0 + rho0 * (b * b + c * c));
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = EN_BLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(EN_BLOCK) void k_sum_partials(const double* partial, int n, double* out) {
  __shared__ double red[EN_BLOCK];
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += EN_BLOCK) acc += partial[k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = EN_BLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// Plain device copy: one 16-byte element per thread, non-temporal loads and
// stores, one block per 4 KiB.  The bandwidth reference the bulk kernel is
// compared with.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy16(const u32x4* __restrict__ a, u32x4* __restrict__ b, size_t n16) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

__global__ void k_copy1(const unsigned char* __restrict__ a, unsigned char* __restrict__ b, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  for (size_t done = 0; done < n16;) {  // chunks keep a launch below 2^31 work-items
    const size_t chunk = n16 - done < ((size_t)1 << 31) ? n16 - done : ((size_t)1 << 31);
    const unsigned grid = (unsigned)((chunk + 255) / 256);
    k_copy16<<<dim3(grid), dim3(256), 0, s>>>(static_cast<const u32x4*>(src) + done,
                                               static_cast<u32x4*>(dst) + done, chunk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    done += chunk;
  }
  const size_t tail = bytes - n16 * 16;
  if (tail) {
    k_copy1<<<dim3(1), dim3(16), 0, s>>>(static_cast<const unsigned char*>(src) + n16 * 16,
                                         static_cast<unsigned char*>(dst) + n16 * 16, tail);
    return hipGetLastError();
  }
  return hipSuccess;
}

// ------------------------------------------------------------------ launchers
static inline dim3 node_grid(const LatDesc& L, int bs) { return dim3((L.nx + bs - 1) / bs, L.ny); }

hipError_t launch_init(const LatDesc& L, int parity, const double* drho, const double* ux, const double* uy,
                       hipStream_t s) {
  const dim3 grid = node_grid(L, 256), block(256);
  switch (L.store) {
    case ST_F64: k_init<ST_F64><<<grid, block, 0, s>>>(L, parity, drho, ux, uy); break;
    case ST_F32: k_init<ST_F32><<<grid, block, 0, s>>>(L, parity, drho, ux, uy); break;
    case ST_F16: k_init<ST_F16><<<grid, block, 0, s>>>(L, parity, drho, ux, uy); break;
    case ST_BF16: k_init<ST_BF16><<<grid, block, 0, s>>>(L, parity, drho, ux, uy); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int absmax_blocks() { return 256; }

hipError_t launch_absmax_init(const LatDesc& L, const double* drho, const double* ux, const double* uy,
                              float* partial, hipStream_t s) {
  k_absmax_init<<<dim3(absmax_blocks()), dim3(256), 0, s>>>(L, drho, ux, uy, partial);
  return hipGetLastError();
}

hipError_t launch_moments(const LatDesc& L, int parity, void* r, void* u, void* v, int f64, int deviation,
                          hipStream_t s) {
  k_moments<<<node_grid(L, 256), dim3(256), 0, s>>>(L, parity, r, u, v, f64, deviation);
  return hipGetLastError();
}

hipError_t launch_get_pops(const LatDesc& L, int parity, double* out, hipStream_t s) {
  k_get_pops<<<node_grid(L, 256), dim3(256), 0, s>>>(L, parity, out);
  return hipGetLastError();
}

hipError_t launch_set_pops(const LatDesc& L, int parity, const double* in, hipStream_t s) {
  const dim3 grid = node_grid(L, 256), block(256);
  switch (L.store) {
    case ST_F64: k_set_pops<ST_F64><<<grid, block, 0, s>>>(L, parity, in); break;
    case ST_F32: k_set_pops<ST_F32><<<grid, block, 0, s>>>(L, parity, in); break;
    case ST_F16: k_set_pops<ST_F16><<<grid, block, 0, s>>>(L, parity, in); break;
    case ST_BF16: k_set_pops<ST_BF16><<<grid, block, 0, s>>>(L, parity, in); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finite(const LatDesc& L, int parity, int* bad, hipStream_t s) {
  k_finite<<<node_grid(L, 256), dim3(256), 0, s>>>(L, parity, bad);
  return hipGetLastError();
}

int energy_partials() { return EN_GRID; }

hipError_t launch_energy(const LatDesc& T_, int pt, const LatDesc* R_, int pr, int xo, int yo, double ux_ref,
                         double uy_ref, double* partial, double* out, hipStream_t s) {
  k_energy<<<dim3(EN_GRID), dim3(EN_BLOCK), 0, s>>>(T_, pt, R_ ? *R_ : T_, pr, R_ != nullptr, xo, yo, ux_ref,
                                                     uy_ref, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_sum_partials<<<dim3(1), dim3(EN_BLOCK), 0, s>>>(partial, EN_GRID, out);
  return hipGetLastError();
}

}  // namespace lbm
