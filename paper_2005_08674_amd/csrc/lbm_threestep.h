// lbm_threestep.h -- the single-lattice three-step kernel (three_step_tile,
// t -> t + 3 in one launch) and its compile-time shapes, shared by the
// translation units that instantiate it without and with the learned
// closure (lbm_twostep.hip, lbm_twostep_cl.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_device.h"
#include "lbm_twostep_lds.h"

namespace lbm {

// Register budget of the multi-step kernels: the 32-bit arithmetic formats
// are held to 80 VGPRs, which lets 6 waves share a SIMD (the LDS of the larger
// tiles allows no more); the boundary-tile path would otherwise take a few
// more and cost every tile that occupancy.
template <int S>
constexpr int two_step_waves() {
  return S == ST_F64 ? 1 : 6;
}

// Candidate shapes of the three-step sweep (three_step_tile): output tile
// 64 x TY, NT threads, non-temporal stores (NTS); tiles in XCD bands (XCD k
// takes the k-th contiguous eighth of the row-major tiles).  A shape whose
// LDS exceeds a workgroup's 160 KiB for a storage format is not built for it
// (FP64 at TY >= 16).
#define LBM_THREE_STEP(X) \
  X(8, 512, true)         \
  X(12, 512, true)        \
  X(12, 768, true)        \
  X(16, 512, true)        \
  X(16, 768, true)        \
  X(20, 768, true)

// ------------------------------------------------------------------ column march
// Candidate shapes of the marched three-step sweep, one launch of NT-thread
// blocks: the edge tiles (the ring around the inner tiles' rectangle) as
// three-step tiles of 64 x TY, then the rectangle as 64-column strips cut
// into chunks of about H rows, each walked down in rounds of MR rows
// (three_step_march) with PF rounds of loads in flight; the march's level
// rings take the tiles' level arrays.  NT threads cover a round's MR x 68
// level-(t + 1) nodes in one pass; NTS: non-temporal stores (plain stores
// and chunks of 160 rows measured slower at 4096^2 in every format).
#define LBM_THREE_MARCH(X)       \
  X(12, 11, 768, 128, 1, true)   \
  X(12, 11, 768, 96, 1, true)    \
  X(12, 11, 768, 64, 1, true)    \
  X(12, 11, 768, 128, 2, true)   \
  X(8, 7, 512, 128, 1, true)     \
  X(8, 7, 512, 64, 1, true)

template <int S, int TY>
constexpr bool three_step_fits() {
  return three_step_lds_bytes<S, TY>() <= 160 * 1024;
}

// Threads of the closure's edge-tile kernel: four waves, so that one of its
// blocks (a wave per SIMD) shares a CU with a block of the inner-tile kernel
// running beside it.
constexpr int CL_THREADS = 256;

template <int S, int TY>
constexpr bool three_step_fits_closure() {
  return three_step_lds_bytes<S, TY>() + three_step_cl_lds_bytes<S, TY, CL_THREADS, true>() <= 160 * 1024;
}

// Blocks per SIMD the register allocation is held to: the sweep kernels as
// two_step_waves; the closure's edge-tile kernel runs few blocks and takes
// the registers the network wants.
template <int S, bool CL>
constexpr int three_step_waves() {
  return CL ? 2 : two_step_waves<S>();
}

// The inner tiles of a lattice form the rectangle txi in [1, ix], tyi in
// [1, iy] (tile x0 = 64 txi >= 3 with x0 + 67 <= nx, and the same in y);
// the edge tiles the ring around it.  Edge tile number b of that ring (row 0,
// the rows above iy, then per middle row the tile at txi = 0 and those
// beyond ix); false past the last.
__host__ __device__ inline bool ring_tile(int b, int tiles_x, int tiles_y, int ix, int iy, int& txi, int& tyi) {
  if (ix <= 0 || iy <= 0) {
    if (b >= tiles_x * tiles_y) return false;
    tyi = b / tiles_x;
    txi = b - tyi * tiles_x;
    return true;
  }
  const int top = (tiles_y - 1 - iy) * tiles_x;
  if (b < tiles_x + top) {
    tyi = b < tiles_x ? 0 : iy + 1 + (b - tiles_x) / tiles_x;
    txi = b < tiles_x ? b : (b - tiles_x) % tiles_x;
    return true;
  }
  b -= tiles_x + top;
  const int cells = 1 + (tiles_x - 1 - ix);
  if (b >= iy * cells) return false;
  tyi = 1 + b / cells;
  const int k = b - (tyi - 1) * cells;
  txi = k == 0 ? 0 : ix + k;
  return true;
}
__host__ __device__ inline int inner_cols(int nx) { return nx >= 67 ? (nx - 67) / TL_TX : 0; }
__host__ __device__ inline int inner_rows(int ny, int ty) { return ny >= ty + 3 ? (ny - ty - 3) / ty : 0; }

// The march items of a launch part (strip sx of ix, chunk c of chunks):
// part 0 all of them, part 1 those whose neighbours are all march items
// (1 <= sx <= ix - 2 and 1 <= c <= chunks - 2: a level-t read or a write of
// theirs stays 3 nodes or more from every edge tile), part 2 the others (the
// border of the rectangle).  Part 1 is chunk-major; part 2 is row c = 0, then
// the two ends of each middle row, then row chunks - 1.  Block m takes item
// (m mod 8) * per + m / 8 of its part, so each XCD works through a
// contiguous stretch; false past the part's last item.
__host__ __device__ inline int march_part_items(int ix, int chunks, int part) {
  const int inner = ix > 2 && chunks > 2 ? (ix - 2) * (chunks - 2) : 0;
  return part == 0 ? ix * chunks : (part == 1 ? inner : ix * chunks - inner);
}
__host__ __device__ inline bool march_item(int m, int ix, int chunks, int part, int& c, int& sx) {
  const int items = march_part_items(ix, chunks, part), per = (items + 7) >> 3;
  const int item = (m & 7) * per + (m >> 3);
  if (item >= items) return false;
  const int fx = ix - 2, fc = chunks - 2;
  if (part == 1) {
    c = 1 + item / fx;
    sx = 1 + item % fx;
  } else if (part == 0 || fx <= 0 || fc <= 0) {  // part 2 without inner items is every item
    c = item / ix;
    sx = item - c * ix;
  } else if (item < ix) {
    c = 0;
    sx = item;
  } else if (item < ix + 2 * fc) {
    const int k = item - ix;
    c = 1 + (k >> 1);
    sx = (k & 1) ? ix - 1 : 0;
  } else {
    c = chunks - 1;
    sx = item - ix - 2 * fc;
  }
  return true;
}

// `part` as three_step_tile, or 3 and 4: the inner tiles away from the edge
// tiles and the others (a closure lattice's two launches of its inner tiles).
// The closure kernel (CL) runs one block per
// edge tile (the ring); the others one block per tile in XCD bands.
template <int S, int TY, int NT, bool NTS, int CM, bool CL>
__global__ __launch_bounds__(NT, (three_step_waves<S, CL>())) void k_three_step(LatDesc L, int parity, int tiles_x,
                                                                            int tiles_y, int part) {
  int txi, tyi;
  if (CL) {
    if (!ring_tile(blockIdx.x, tiles_x, tiles_y, inner_cols(L.nx), inner_rows(L.ny, TY), txi, tyi)) return;
  } else if (part >= 3) {
    // part 3: the inner tiles whose neighbours are all inner tiles, part 4
    // the other inner tiles (march_item over the inner rectangle)
    int c, sx;
    if (!march_item(blockIdx.x, inner_cols(L.nx), inner_rows(L.ny, TY), part - 2, c, sx)) return;
    tyi = 1 + c;
    txi = 1 + sx;
  } else {
    const int b = blockIdx.x, ntiles = tiles_x * tiles_y;
    const int per = (ntiles + 7) >> 3;
    const int tile = (b & 7) * per + (b >> 3);
    if (tile >= ntiles) return;  // padding blocks: the whole block leaves before any barrier
    tyi = tile / tiles_x;
    txi = tile - tyi * tiles_x;
  }
  three_step_tile<S, TY, NT, NTS, CM, CL>(L, parity, txi, tyi, CL ? 2 : (part >= 3 ? 1 : part));
}

template <int S, int TY, int NT, bool NTS, bool CL>
inline hipError_t launch_three_t(const LatDesc& L, int parity, hipStream_t s, int part) {
  constexpr bool fits = CL ? three_step_fits_closure<S, TY>() : three_step_fits<S, TY>();
  if constexpr (!fits) {
    return hipErrorInvalidValue;
  } else {
    const int tiles_x = (L.nx + TL_TX - 1) / TL_TX, tiles_y = (L.ny + TY - 1) / TY;
    const int n = CL ? tiles_x * tiles_y - inner_cols(L.nx) * inner_rows(L.ny, TY)
                     : (part >= 3 ? (march_part_items(inner_cols(L.nx), inner_rows(L.ny, TY), part - 2) + 7) >> 3 << 3
                                  : ((tiles_x * tiles_y + 7) >> 3) * 8);
    if (n == 0) return hipSuccess;
    const dim3 grid(n);
    if (L.coll == COLL_MRT)
      k_three_step<S, TY, NT, NTS, COLL_MRT, CL><<<grid, dim3(NT), 0, s>>>(L, parity, tiles_x, tiles_y, part);
    else
      k_three_step<S, TY, NT, NTS, COLL_BGK, CL><<<grid, dim3(NT), 0, s>>>(L, parity, tiles_x, tiles_y, part);
    return hipGetLastError();
  }
}

template <int S, bool CL>
inline hipError_t launch_three_s(const LatDesc& L, int parity, int id, hipStream_t s, int part) {
  int k = 0;
#define X(a, b, c)                                                           \
  if (id == k) {                                                             \
    if constexpr (CL)                                                        \
      return launch_three_t<S, a, CL_THREADS, c, true>(L, parity, s, part);  \
    else                                                                     \
      return launch_three_t<S, a, b, c, false>(L, parity, s, part);          \
  }                                                                          \
  ++k;
  LBM_THREE_STEP(X)
#undef X
  return hipErrorInvalidValue;
}

// Whether three-step shape `id` fits the LDS in storage format `store`, with
// the closure's LDS when `closure`.
inline bool three_step_fits_store(int store, int id, bool closure) {
  int k = 0;
#define X(a, b, c)                                                                                             \
  if (id == k) {                                                                                               \
    switch (store) {                                                                                           \
      case ST_F64: return closure ? three_step_fits_closure<ST_F64, a>() : three_step_fits<ST_F64, a>();    \
      case ST_F32: return closure ? three_step_fits_closure<ST_F32, a>() : three_step_fits<ST_F32, a>();    \
      case ST_F16: return closure ? three_step_fits_closure<ST_F16, a>() : three_step_fits<ST_F16, a>();    \
      case ST_BF16: return closure ? three_step_fits_closure<ST_BF16, a>() : three_step_fits<ST_BF16, a>(); \
    }                                                                                                          \
    return false;                                                                                              \
  }                                                                                                            \
  ++k;
  LBM_THREE_STEP(X)
#undef X
#define X(a, m, b, h, p, n)                                                                                    \
  if (id == k) {                                                                                            \
    switch (store) {                                                                                        \
      case ST_F64: return three_step_fits<ST_F64, a>() && (!closure || three_step_fits_closure<ST_F64, a>()); \
      case ST_F32: return three_step_fits<ST_F32, a>() && (!closure || three_step_fits_closure<ST_F32, a>()); \
      case ST_F16: return three_step_fits<ST_F16, a>() && (!closure || three_step_fits_closure<ST_F16, a>()); \
      case ST_BF16: return three_step_fits<ST_BF16, a>() && (!closure || three_step_fits_closure<ST_BF16, a>()); \
    }                                                                                                       \
    return false;                                                                                           \
  }                                                                                                         \
  ++k;
  LBM_THREE_MARCH(X)
#undef X
  return false;
}

// Chunk rows of a march over an inner rectangle of `rows` rows in chunks of
// about h: the count, and the height of all but the last.
__host__ __device__ inline void march_chunks(int rows, int h, int& chunks, int& height) {
  chunks = rows > 0 ? (rows + h - 1) / h : 0;
  height = chunks > 0 ? (rows + chunks - 1) / chunks : 0;
}

// Column march (TY: the level arrays' tile rows): the block owns the 64
// columns xs .. xs + 63 of output rows ya .. yb - 1, all inside the inner
// tiles' rectangle (no clamp, no NSBC), and walks down them in rounds of MR
// rows: round j computes level t + 1 on rows ya - 2 + j MR + [0, MR) (68
// columns, pulled from HBM), level t + 2 one row behind (66 columns) and
// level t + 3 one row behind that (the 64 output columns, stored).  Each
// level keeps its last MR + 2 rows in a ring in the tile's level arrays (row
// y of level t + 1 in slot (y - ya + 2) mod (MR + 2) of lds1, of level t + 2
// in (y - ya + 1) mod (MR + 2) of lds2), so apart from the two ends of the
// strip no row is computed twice.  The loads of level t + 1 run PF rounds
// ahead of their use: those of round j + PF are issued before round j's
// levels t + 2 and t + 3.  Per node the arithmetic and the codec rounding
// are the tiles': bit-identical to single steps.
template <int S, int TY, int MR, int NT, bool NTS, int CM, int PF>
__device__ inline void three_step_march(const LatDesc& Ld, int parity, int xs, int ya, int yb) {
  static_assert(MR >= 5 && MR <= TY && (PF == 1 || PF == 2), "march shape");
  using C = Codec<S>;
  using T = typename C::T;
  using R = typename C::R;
  constexpr int RR = MR + 2;
  constexpr int NI = (MR * T3_W1 + NT - 1) / NT;
  auto& r1 = three_lds1<S, TY>();
  auto& r2 = three_lds2<S, TY>();
  const int tid = threadIdx.x;
  const T* __restrict__ A = static_cast<const T*>(buf_of(Ld, parity));
  T* __restrict__ B = static_cast<T*>(buf_of(Ld, parity ^ 1));
  const int pitch = Ld.pitch;
  const int64_t plane = Ld.plane;
  const R rho0 = R(Ld.rho0), omega = R(Ld.omega);
  const int rounds = (yb - ya + 4 + MR - 1) / MR;
  T raw[PF][NI][9];
  // loads of level t + 1's rows of round j (ya - 2 + j MR + r, r < n) into raw[u]
  auto fetch = [&](int j, int u) __attribute__((always_inline)) {
    const int q = ya - 2 + j * MR, n = min(MR, yb + 2 - q);
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int k = tid + it * NT;
      if (k < n * T3_W1) {
        const int r = k / T3_W1, cx = k - r * T3_W1;
        const uint32_t idx = (uint32_t)((q + r) * pitch + (xs - 2 + cx));
        const uint32_t ro[3] = {(idx + (uint32_t)pitch) * (uint32_t)sizeof(T), idx * (uint32_t)sizeof(T),
                                (idx - (uint32_t)pitch) * (uint32_t)sizeof(T)};
#pragma unroll
        for (int i = 0; i < 9; ++i) raw[u][it][i] = ldg(A + i * plane, ro[1 + kCy[i]] - kCx[i] * (int)sizeof(T));
      }
    }
  };
  // LDS as element offsets from the arrays' first element (32-bit
  // arithmetic; population i's plane of a level array at a constant offset)
  T* const l1 = &r1[0][0][0];
  T* const l2 = &r2[0][0][0];
  constexpr int P1 = (TY + 4) * T3_W1, P2 = (TY + 2) * T3_W2;
  const OutPlanes<T> out(B, plane);
  // ring slot of a row: su (the round's first row's slot, uniform) + r, wrapped once
  auto wrap = [](int v) { return v >= RR ? v - RR : v; };
  auto level1 = [&](const Base<R>& b, int j, int u) __attribute__((always_inline)) {
    const int q = ya - 2 + j * MR, n = min(MR, yb + 2 - q);
    const int su = (j * MR) % RR;
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int k = tid + it * NT;
      if (k < n * T3_W1) {
        const int r = k / T3_W1, cx = k - r * T3_W1;
        R g[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = C::raw(raw[u][it][i]);
        collide_stored<S, CM>(Ld, g, rho0, b, omega);
        const uint32_t o = (uint32_t)(wrap(su + r) * T3_W1 + cx);
#pragma unroll
        for (int i = 0; i < 9; ++i) l1[o + i * P1] = C::raw_enc(g[i]);
      }
    }
  };
  auto level2 = [&](const Base<R>& b, int j) __attribute__((always_inline)) {
    const int lo = max(ya - 3 + j * MR, ya - 1), hi = min(ya - 3 + (j + 1) * MR, yb + 1);
    const int su = (lo - ya + 2) % RR;
    constexpr int N2 = MR * T3_W2;
#pragma unroll
    for (int it = 0; it < (N2 + NT - 1) / NT; ++it) {
      const int k = tid + it * NT;
      if (k < (hi - lo) * T3_W2) {
        const int r = k / T3_W2, cx = k - r * T3_W2;
        // level t + 1 slots of rows y - 1, y, y + 1 (y = lo + r); row y of level t + 2 goes to slot sm
        const int s0 = wrap(su + r);
        const int sm = s0 == 0 ? RR - 1 : s0 - 1, sp = s0 == RR - 1 ? 0 : s0 + 1;
        const uint32_t om = (uint32_t)(sm * T3_W1 + cx + 1), o0 = (uint32_t)(s0 * T3_W1 + cx + 1),
                       op = (uint32_t)(sp * T3_W1 + cx + 1);
        R g[9];
#pragma unroll
        for (int i = 0; i < 9; ++i)
          g[i] = C::raw(l1[(kCy[i] > 0 ? om : (kCy[i] < 0 ? op : o0)) + i * P1 - kCx[i]]);
        collide_stored<S, CM>(Ld, g, rho0, b, omega);
        const uint32_t ow = (uint32_t)(sm * T3_W2 + cx);
#pragma unroll
        for (int i = 0; i < 9; ++i) l2[ow + i * P2] = C::raw_enc(g[i]);
      }
    }
  };
  auto level3 = [&](const Base<R>& b, int j) __attribute__((always_inline)) {
    const int lo = max(ya - 4 + j * MR, ya), hi = min(ya - 4 + (j + 1) * MR, yb);
    const int su = (lo - ya + 1) % RR;
    constexpr int N3 = MR * TL_TX;
#pragma unroll
    for (int it = 0; it < (N3 + NT - 1) / NT; ++it) {
      const int k = tid + it * NT;
      if (k < (hi - lo) * TL_TX) {
        const int r = k / TL_TX, cx = k - r * TL_TX;
        const int s0 = wrap(su + r);
        const int sm = s0 == 0 ? RR - 1 : s0 - 1, sp = s0 == RR - 1 ? 0 : s0 + 1;
        const uint32_t om = (uint32_t)(sm * T3_W2 + cx + 1), o0 = (uint32_t)(s0 * T3_W2 + cx + 1),
                       op = (uint32_t)(sp * T3_W2 + cx + 1);
        R g[9];
#pragma unroll
        for (int i = 0; i < 9; ++i)
          g[i] = C::raw(l2[(kCy[i] > 0 ? om : (kCy[i] < 0 ? op : o0)) + i * P2 - kCx[i]]);
        collide_stored<S, CM>(Ld, g, rho0, b, omega);
        const uint32_t off = (uint32_t)((lo + r) * pitch + xs + cx) * (uint32_t)sizeof(T);
#pragma unroll
        for (int i = 0; i < 9; ++i) out.template put<NTS>(i, off, C::raw_enc(g[i]));
      }
    }
  };
  // One round (its level t + 1 already in r1): round j + 1's level t + 1
  // overwrites ring rows that round j's level t + 2 has read (a barrier lies
  // between them), round j + 1's level t + 2 those that round j's level
  // t + 3 has read (the barrier closing round j).  raw[u] holds round
  // j + 1's loads; round j + PF's go to the buffer round j's level t + 1
  // emptied.
  auto round = [&](const Base<R>& b, int j, int u) __attribute__((always_inline)) {
    if (PF == 2 && j + 2 < rounds) fetch(j + 2, u ^ 1);
    if (PF == 1 && j + 1 < rounds) fetch(j + 1, 0);
    level2(b, j);
    __syncthreads();
    level3(b, j);
    if (j + 1 < rounds) level1(b, j + 1, PF == 2 ? u : 0);
    __syncthreads();
  };
  auto run = [&](const Base<R>& b) __attribute__((always_inline)) {
    fetch(0, 0);
    if (PF == 2 && rounds > 1) fetch(1, 1);
    level1(b, 0, 0);
    __syncthreads();
    // with PF = 2, round j's successor's loads sit in raw[(j + 1) & 1]; the
    // loop is unrolled by two so that every register index is a constant
    for (int j = 0; j < rounds; j += 2) {
      round(b, j, 1);
      if (j + 1 < rounds) round(b, j + 1, 0);
    }
  };
  const Base<R> base(Ld);
  Base<R> b = base;
  if (base.zero) {
    b.zero = true;
    run(b);
  } else {
    b.zero = false;
    run(b);
  }
}

// Blocks below ring8 take the edge tiles (ring_tile order, padded to a
// multiple of 8), the others the strips' chunks in XCD bands: XCD k takes
// the k-th contiguous eighth of the chunk-major list, so neighbouring strips
// share its L2.  The edge tiles come first: they are the slower blocks.
template <int S, int TY, int MR, int NT, bool NTS, int CM, int PF>
__global__ __launch_bounds__(NT, two_step_waves<S>()) void k_three_march(LatDesc L, int parity, int tiles_x,
                                                                       int tiles_y, int ring8, int height,
                                                                       int chunks, int part) {
  const int ix = inner_cols(L.nx), iy = inner_rows(L.ny, TY);
  const int b = blockIdx.x;
  if (b < ring8) {
    int txi, tyi;
    if (!ring_tile(b, tiles_x, tiles_y, ix, iy, txi, tyi)) return;  // padding: the block leaves before any barrier
    three_step_tile<S, TY, NT, NTS, CM, false>(L, parity, txi, tyi, 2);
    return;
  }
  // (ring8 is a multiple of 8, so m and b run on the same XCD)
  int c, sx;
  if (!march_item(b - ring8, ix, chunks, part, c, sx)) return;
  const int ya = TY + c * height, yb = min(ya + height, TY * (iy + 1));
  three_step_march<S, TY, MR, NT, NTS, CM, PF>(L, parity, TL_TX * (1 + sx), ya, yb);
}

// One launch: the edge tiles (unless !ring: a closure lattice's run in the
// closure kernel) and part `part` of the march over the inner rectangle in
// chunks of about h rows (march_item).
template <int S, int TY, int MR, int NT, bool NTS, int PF>
inline hipError_t launch_march_t(const LatDesc& L, int parity, hipStream_t s, int h, bool ring, int part) {
  if constexpr (!three_step_fits<S, TY>()) {
    return hipErrorInvalidValue;
  } else {
    const int tiles_x = (L.nx + TL_TX - 1) / TL_TX, tiles_y = (L.ny + TY - 1) / TY;
    const int ix = inner_cols(L.nx), iy = inner_rows(L.ny, TY);
    const int ring8 = ring ? (tiles_x * tiles_y - ix * iy + 7) / 8 * 8 : 0;
    int chunks, height;
    march_chunks(ix > 0 ? TY * iy : 0, h, chunks, height);
    const int items = march_part_items(ix, chunks, part);
    if (ring8 + items == 0) return hipSuccess;
    const dim3 grid(ring8 + (items + 7) / 8 * 8);
    if (L.coll == COLL_MRT)
      k_three_march<S, TY, MR, NT, NTS, COLL_MRT, PF>
          <<<grid, dim3(NT), 0, s>>>(L, parity, tiles_x, tiles_y, ring8, height, chunks, part);
    else
      k_three_march<S, TY, MR, NT, NTS, COLL_BGK, PF>
          <<<grid, dim3(NT), 0, s>>>(L, parity, tiles_x, tiles_y, ring8, height, chunks, part);
    return hipGetLastError();
  }
}

// march shape `id` (among the march shapes) on one lattice, with its edge
// tiles when `ring`, over part `part` of the march items (lbm_march.hip)
hipError_t launch_three_march(const LatDesc& L, int parity, int id, hipStream_t s, bool ring, int part = 0);

// ------------------------------------------------------------------ two-step column march
// Candidate shapes of the marched two-step sweep (t -> t + 2), one launch of
// NT-thread blocks: the edge tiles as two-step tiles of 64 x TY
// (two_step_tile, part 2), then the inner rectangle of the two-step tiling
// (tiles 1 .. (nx - 67) / 64 across, 1 .. (ny - TY - 2) / TY up) as
// 64-column strips in chunks of about H rows, walked down in rounds of MR
// rows (two_step_march) whose level ring takes the tile's level array.
#define LBM_TWO_MARCH(X)      \
  X(12, 11, 768, 96, true)    \
  X(12, 11, 768, 128, true)   \
  X(8, 7, 512, 96, true)

__host__ __device__ inline int inner_rows2(int ny, int ty) { return ny >= ty + 2 ? (ny - ty - 2) / ty : 0; }

// Two-step column march over output rows ya .. yb - 1 of the 64 columns xs
// .. xs + 63 (all inside the two-step tiling's inner rectangle): round j
// computes level t + 1 on rows ya - 1 + j MR + [0, MR) (66 columns, pulled
// from HBM) into a ring of MR + 2 rows (row y in slot (y - ya + 1) mod
// (MR + 2)) and level t + 2 one row behind, stored.  The loads of round
// j + 1 are issued before round j's level t + 2.  Same per-node arithmetic
// and codec rounding as the tiles: bit-identical to single steps.
template <int S, int TY, int MR, int NT, bool NTS, int CM>
__device__ inline void two_step_march(const LatDesc& Ld, int parity, int xs, int ya, int yb) {
  static_assert(MR >= 3 && MR + 2 <= TY + 4, "march shape");
  using C = Codec<S>;
  using T = typename C::T;
  using R = typename C::R;
  constexpr int RR = MR + 2, W1 = TL_TX + 2;
  constexpr int NI = (MR * W1 + NT - 1) / NT;
  auto& r1 = two_lds<S, TY>();
  T* const l1 = &r1[0][0][0];
  constexpr int P1 = (TY + 4) * TL_W;
  const int tid = threadIdx.x;
  const T* __restrict__ A = static_cast<const T*>(buf_of(Ld, parity));
  const OutPlanes<T> out(static_cast<T*>(buf_of(Ld, parity ^ 1)), Ld.plane);
  const int pitch = Ld.pitch;
  const int64_t plane = Ld.plane;
  const R rho0 = R(Ld.rho0), omega = R(Ld.omega);
  const int rounds = (yb - ya + 2 + MR - 1) / MR;
  auto wrap = [](int v) { return v >= RR ? v - RR : v; };
  T raw[NI][9];
  auto fetch = [&](int j) __attribute__((always_inline)) {
    const int q = ya - 1 + j * MR, n = min(MR, yb + 1 - q);
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int k = tid + it * NT;
      if (k < n * W1) {
        const int r = k / W1, cx = k - r * W1;
        const uint32_t idx = (uint32_t)((q + r) * pitch + (xs - 1 + cx));
        const uint32_t ro[3] = {(idx + (uint32_t)pitch) * (uint32_t)sizeof(T), idx * (uint32_t)sizeof(T),
                                (idx - (uint32_t)pitch) * (uint32_t)sizeof(T)};
#pragma unroll
        for (int i = 0; i < 9; ++i) raw[it][i] = ldg(A + i * plane, ro[1 + kCy[i]] - kCx[i] * (int)sizeof(T));
      }
    }
  };
  auto level1 = [&](const Base<R>& b, int j) __attribute__((always_inline)) {
    const int q = ya - 1 + j * MR, n = min(MR, yb + 1 - q);
    const int su = (j * MR) % RR;
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int k = tid + it * NT;
      if (k < n * W1) {
        const int r = k / W1, cx = k - r * W1;
        R g[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = C::raw(raw[it][i]);
        collide_stored<S, CM>(Ld, g, rho0, b, omega);
        const uint32_t o = (uint32_t)(wrap(su + r) * TL_W + cx);
#pragma unroll
        for (int i = 0; i < 9; ++i) l1[o + i * P1] = C::raw_enc(g[i]);
      }
    }
  };
  auto level2 = [&](const Base<R>& b, int j) __attribute__((always_inline)) {
    const int lo = max(ya - 2 + j * MR, ya), hi = min(ya - 2 + (j + 1) * MR, yb);
    const int su = (lo - ya + 1) % RR;
    constexpr int N2 = MR * TL_TX;
#pragma unroll
    for (int it = 0; it < (N2 + NT - 1) / NT; ++it) {
      const int k = tid + it * NT;
      if (k < (hi - lo) * TL_TX) {
        const int r = k / TL_TX, cx = k - r * TL_TX;
        const int s0 = wrap(su + r);
        const int sm = s0 == 0 ? RR - 1 : s0 - 1, sp = s0 == RR - 1 ? 0 : s0 + 1;
        const uint32_t om = (uint32_t)(sm * TL_W + cx + 1), o0 = (uint32_t)(s0 * TL_W + cx + 1),
                       op = (uint32_t)(sp * TL_W + cx + 1);
        R g[9];
#pragma unroll
        for (int i = 0; i < 9; ++i)
          g[i] = C::raw(l1[(kCy[i] > 0 ? om : (kCy[i] < 0 ? op : o0)) + i * P1 - kCx[i]]);
        collide_stored<S, CM>(Ld, g, rho0, b, omega);
        const uint32_t off = (uint32_t)((lo + r) * pitch + xs + cx) * (uint32_t)sizeof(T);
#pragma unroll
        for (int i = 0; i < 9; ++i) out.template put<NTS>(i, off, C::raw_enc(g[i]));
      }
    }
  };
  // round j + 1's level t + 1 overwrites ring rows round j's level t + 2 has
  // read: a barrier between them, and one before the next level t + 2
  auto run = [&](const Base<R>& b) __attribute__((always_inline)) {
    fetch(0);
    level1(b, 0);
    __syncthreads();
    for (int j = 0; j < rounds; ++j) {
      const bool more = j + 1 < rounds;
      if (more) fetch(j + 1);
      level2(b, j);
      __syncthreads();
      if (more) level1(b, j + 1);
      __syncthreads();
    }
  };
  const Base<R> base(Ld);
  Base<R> b = base;
  if (base.zero) {
    b.zero = true;
    run(b);
  } else {
    b.zero = false;
    run(b);
  }
}

// Blocks below ring8 take the two-step tiling's edge tiles (ring_tile order,
// padded to a multiple of 8), the others the strips' chunks in XCD bands.
template <int S, int TY, int MR, int NT, bool NTS, int CM>
__global__ __launch_bounds__(NT, two_step_waves<S>()) void k_two_march(LatDesc L, int parity, int tiles_x,
                                                                     int tiles_y, int ring8, int height,
                                                                     int chunks) {
  const int ix = inner_cols(L.nx), iy = inner_rows2(L.ny, TY);
  const int b = blockIdx.x;
  if (b < ring8) {
    int txi, tyi;
    if (!ring_tile(b, tiles_x, tiles_y, ix, iy, txi, tyi)) return;  // padding: the block leaves before any barrier
    two_step_tile<S, TY, NT, NTS, CM>(L, parity, txi, tyi, 2);
    return;
  }
  const int m = b - ring8, items = ix * chunks, per = (items + 7) >> 3;
  const int item = (m & 7) * per + (m >> 3);
  if (item >= items) return;
  const int c = item / ix, sx = item - c * ix;
  const int ya = TY + c * height, yb = min(ya + height, TY * (iy + 1));
  two_step_march<S, TY, MR, NT, NTS, CM>(L, parity, TL_TX * (1 + sx), ya, yb);
}

template <int S, int TY, int MR, int NT, bool NTS>
inline hipError_t launch_two_march_t(const LatDesc& L, int parity, hipStream_t s, int h) {
  const int tiles_x = (L.nx + TL_TX - 1) / TL_TX, tiles_y = (L.ny + TY - 1) / TY;
  const int ix = inner_cols(L.nx), iy = inner_rows2(L.ny, TY);
  const int ring8 = (tiles_x * tiles_y - ix * iy + 7) / 8 * 8;
  int chunks, height;
  march_chunks(ix > 0 ? TY * iy : 0, h, chunks, height);
  const dim3 grid(ring8 + (ix * chunks + 7) / 8 * 8);
  if (L.coll == COLL_MRT)
    k_two_march<S, TY, MR, NT, NTS, COLL_MRT><<<grid, dim3(NT), 0, s>>>(L, parity, tiles_x, tiles_y, ring8, height, chunks);
  else
    k_two_march<S, TY, MR, NT, NTS, COLL_BGK><<<grid, dim3(NT), 0, s>>>(L, parity, tiles_x, tiles_y, ring8, height, chunks);
  return hipGetLastError();
}

// two-step march shape `id` (among the two-step march shapes) on one lattice (lbm_march.hip)
hipError_t launch_two_march(const LatDesc& L, int parity, int id, hipStream_t s);

// three-step launch of a lattice with the learned closure (lbm_twostep_cl.hip)
hipError_t launch_three_step_closure(const LatDesc& L, int parity, int id, hipStream_t s);

}  // namespace lbm
