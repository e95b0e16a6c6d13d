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

// `part` as three_step_tile.  The closure kernel (CL) runs one block per
// edge tile (the ring); the others one block per tile in XCD bands.
template <int S, int TY, int NT, bool NTS, int CM, bool CL>
__global__ __launch_bounds__(NT, (three_step_waves<S, CL>())) void k_three_step(LatDesc L, int parity, int tiles_x,
                                                                            int tiles_y, int part) {
  int txi, tyi;
  if (CL) {
    if (!ring_tile(blockIdx.x, tiles_x, tiles_y, inner_cols(L.nx), inner_rows(L.ny, TY), txi, tyi)) return;
  } else {
    const int b = blockIdx.x, ntiles = tiles_x * tiles_y;
    const int per = (ntiles + 7) >> 3;
    const int tile = (b & 7) * per + (b >> 3);
    if (tile >= ntiles) return;  // padding blocks: the whole block leaves before any barrier
    tyi = tile / tiles_x;
    txi = tile - tyi * tiles_x;
  }
  three_step_tile<S, TY, NT, NTS, CM, CL>(L, parity, txi, tyi, CL ? 2 : part);
}

template <int S, int TY, int NT, bool NTS, bool CL>
inline hipError_t launch_three_t(const LatDesc& L, int parity, hipStream_t s, int part) {
  constexpr bool fits = CL ? three_step_fits_closure<S, TY>() : three_step_fits<S, TY>();
  if constexpr (!fits) {
    return hipErrorInvalidValue;
  } else {
    const int tiles_x = (L.nx + TL_TX - 1) / TL_TX, tiles_y = (L.ny + TY - 1) / TY;
    const dim3 grid(CL ? tiles_x * tiles_y - inner_cols(L.nx) * inner_rows(L.ny, TY)
                       : ((tiles_x * tiles_y + 7) >> 3) * 8);
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
  return false;
}

// three-step launch of a lattice with the learned closure (lbm_twostep_cl.hip)
hipError_t launch_three_step_closure(const LatDesc& L, int parity, int id, hipStream_t s);

}  // namespace lbm
