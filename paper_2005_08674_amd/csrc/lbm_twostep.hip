// lbm_twostep.hip -- the two-step sweep (t -> t + 2 in one launch, level
// t + 1 in LDS) and the three-step sweep (t -> t + 3, levels t + 1 and t + 2
// in LDS; lbm_twostep_lds.h) for lattices with NSBC on all four edges: their
// compile-time shapes, one instance per storage format and collision model,
// and their host-side launchers.
#include <hip/hip_runtime.h>

#include <cstdio>

#include "lbm_device.h"
#include "lbm_launch.h"
#include "lbm_threestep.h"
#include "lbm_twostep_lds.h"

namespace lbm {

// ------------------------------------------------------------------ two-step kernel
// Candidate shapes of the two-step sweep (lbm_twostep_lds.h): output tile
// 64 x TY, NT threads per block, non-temporal stores (NTS), block -> tile map
// (MAP).  Workgroups go to the 8 XCDs round-robin (block b on XCD b mod 8),
// each XCD with its own L2, and a tile re-reads its neighbours' edge cache
// lines for its margin:
//   MAP 0: a 2-D grid, tile = (blockIdx.x, blockIdx.y); horizontal
//          neighbours run on different XCDs.
//   MAP 1: a 1-D grid over the row-major tiles in runs of 64 blocks; XCD k
//          takes 8 consecutive tiles of each run, so 7 of 8 horizontal
//          neighbours share an L2.
//   MAP 2: XCD k takes the k-th contiguous eighth of the row-major tiles, so
//          horizontal and vertical neighbours share an L2 except at the
//          eight band boundaries.
// TY and NT trade the margin's share of the work, the idle lanes of the last
// pass over the (TY + 2) x 68 and TY x 64 nodes, and the blocks that fit in
// a CU's LDS.
#define LBM_TWO_STEP(X)  \
  X(12, 512, true, 0)    \
  X(16, 512, true, 0)    \
  X(16, 512, true, 1)    \
  X(12, 512, true, 2)    \
  X(16, 512, true, 2)    \
  X(20, 512, true, 2)    \
  X(8, 256, true, 2)     \
  X(12, 384, true, 2)    \
  X(24, 768, true, 2)    \
  X(20, 768, true, 2)

template <int S, int TY, int NT, bool NTS, int CM, int MAP>
__global__ __launch_bounds__(NT, two_step_waves<S>()) void k_two_step(LatDesc L, int parity, int tiles_x,
                                                                    int tiles_y) {
  int txi, tyi;
  if (MAP == 0) {
    txi = blockIdx.x;
    tyi = blockIdx.y;
  } else {
    const int b = blockIdx.x, ntiles = tiles_x * tiles_y;
    int tile;
    if (MAP == 1) {
      tile = (b & ~63) + ((b & 7) << 3) + ((b >> 3) & 7);
    } else {
      const int per = (ntiles + 7) >> 3;
      tile = (b & 7) * per + (b >> 3);
    }
    if (tile >= ntiles) return;  // padding blocks: the whole block leaves before any barrier
    tyi = tile / tiles_x;
    txi = tile - tyi * tiles_x;
  }
  two_step_tile<S, TY, NT, NTS, CM>(L, parity, txi, tyi);
}

// the tile shapes first, then the marched ones (mr > 0: rows per round, h:
// chunk rows)
struct TwoStepShape {
  int ty, nt;
  bool nts;
  int map, mr, h;
};
static const TwoStepShape kTwo[] = {
#define X(a, b, c, d) {a, b, c, d, 0, 0},
    LBM_TWO_STEP(X)
#undef X
#define X(a, m, b, h, n) {a, b, n, 2, m, h},
    LBM_TWO_MARCH(X)
#undef X
};
static constexpr int kNumTwo = sizeof(kTwo) / sizeof(kTwo[0]);
static constexpr int kNumTwoMarch = 0
#define X(a, m, b, h, n) +1
    LBM_TWO_MARCH(X)
#undef X
    ;

bool two_step_is_march(int id) { return id >= 0 && id < kNumTwo && kTwo[id].mr > 0; }

int num_two_step() { return kNumTwo; }

void two_step_name(int id, char* buf, size_t len) {
  if (id < 0 || id >= kNumTwo) {
    snprintf(buf, len, "invalid");
    return;
  }
  const TwoStepShape& t = kTwo[id];
  if (t.mr > 0)
    snprintf(buf, len, "2step:64x%d/%d+march%dxh%d+xcdband%s", t.ty, t.nt, t.mr, t.h, t.nts ? "+nts" : "");
  else
    snprintf(buf, len, "2step:64x%d/%d%s%s", t.ty, t.nt, t.map == 1 ? "+xcd8" : (t.map == 2 ? "+xcdband" : ""),
             t.nts ? "+nts" : "");
}

bool two_step_supported(const LatDesc& L) {
  return L.bc[E_LEFT] == BC_NSBC && L.bc[E_RIGHT] == BC_NSBC && L.bc[E_BOTTOM] == BC_NSBC &&
         L.bc[E_TOP] == BC_NSBC && L.nx >= 3 && L.ny >= 3;
}

template <int S, int TY, int NT, bool NTS, int MAP>
static hipError_t launch_two_t(const LatDesc& L, int parity, hipStream_t s) {
  const int tiles_x = (L.nx + TL_TX - 1) / TL_TX, tiles_y = (L.ny + TY - 1) / TY;
  dim3 grid(tiles_x, tiles_y);
  if (MAP == 1) grid = dim3(((tiles_x * tiles_y + 63) >> 6) * 64);
  if (MAP == 2) grid = dim3(((tiles_x * tiles_y + 7) >> 3) * 8);
  if (L.coll == COLL_MRT)
    k_two_step<S, TY, NT, NTS, COLL_MRT, MAP><<<grid, dim3(NT), 0, s>>>(L, parity, tiles_x, tiles_y);
  else
    k_two_step<S, TY, NT, NTS, COLL_BGK, MAP><<<grid, dim3(NT), 0, s>>>(L, parity, tiles_x, tiles_y);
  return hipGetLastError();
}

template <int S>
static hipError_t launch_two_s(const LatDesc& L, int parity, int id, hipStream_t s) {
  int k = 0;
#define X(a, b, c, d)                                               \
  if (id == k) return launch_two_t<S, a, b, c, d>(L, parity, s);   \
  ++k;
  LBM_TWO_STEP(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_two_step(const LatDesc& L, int parity, int id, hipStream_t s) {
  // the two-step sweep has no closure path
  if (!two_step_supported(L) || (L.closure && L.net)) return hipErrorInvalidValue;
  if (id >= 0 && id < kNumTwo && kTwo[id].mr > 0) return launch_two_march(L, parity, id - (kNumTwo - kNumTwoMarch), s);
  switch (L.store) {
    case ST_F64: return launch_two_s<ST_F64>(L, parity, id, s);
    case ST_F32: return launch_two_s<ST_F32>(L, parity, id, s);
    case ST_F16: return launch_two_s<ST_F16>(L, parity, id, s);
    case ST_BF16: return launch_two_s<ST_BF16>(L, parity, id, s);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ three-step kernel
// (shapes and kernel in lbm_threestep.h)
// the tile shapes first, then the marched ones (mr > 0: rows per round, h:
// chunk rows; non-temporal stores)
struct ThreeStepShape {
  int ty, nt;
  bool nts;
  int mr, h, pf;
};
static const ThreeStepShape kThree[] = {
#define X(a, b, c) {a, b, c, 0, 0, 0},
    LBM_THREE_STEP(X)
#undef X
#define X(a, m, b, h, p, n) {a, b, n, m, h, p},
    LBM_THREE_MARCH(X)
#undef X
};
static constexpr int kNumThree = sizeof(kThree) / sizeof(kThree[0]);
static constexpr int kNumMarch = 0
#define X(a, m, b, h, p, n) +1
    LBM_THREE_MARCH(X)
#undef X
    ;

bool three_step_is_march(int id) { return id >= 0 && id < kNumThree && kThree[id].mr > 0; }

int num_three_step() { return kNumThree; }

void three_step_name(int id, char* buf, size_t len) {
  if (id < 0 || id >= kNumThree) {
    snprintf(buf, len, "invalid");
    return;
  }
  const ThreeStepShape& t = kThree[id];
  if (t.mr > 0)
    snprintf(buf, len, "3step:64x%d/%d+march%dxh%d%s+xcdband%s", t.ty, t.nt, t.mr, t.h, t.pf == 2 ? "+pf2" : "",
             t.nts ? "+nts" : "");
  else
    snprintf(buf, len, "3step:64x%d/%d+xcdband%s", t.ty, t.nt, t.nts ? "+nts" : "");
}

bool three_step_supported(const LatDesc& L, int id) {
  return id >= 0 && id < kNumThree && two_step_supported(L) && L.nx >= TL_TX && L.ny >= kThree[id].ty &&
         three_step_fits_store(L.store, id, L.closure && L.net);
}

// The tile shape whose edge tiles a march shape's closure lattice runs in
// the closure kernel: the first tile shape with the march's tile rows.
static int closure_tile_of(int id) {
  for (int k = 0; k < kNumThree; ++k)
    if (kThree[k].mr == 0 && kThree[k].ty == kThree[id].ty) return k;
  return -1;
}

// One launch of a tile or march shape, except on the learned closure, which
// takes two: its edge tiles with the network and its inner tiles (tile
// shapes) or inner strips (march shapes) with the plain sweep (both read
// buffer `parity` and write disjoint parts of the other).  With a second stream
// `side` the edge-tile kernel runs there, forked from `s` after the work
// already on it (event `fork`) and joined back before what follows (event
// `join`), so the two kernels share the GPU; without one they run in turn
// on `s`.
// A closure launch on two streams: the edge-tile kernel on `side` after
// everything already on s (the fork), the inner part on s.  Launch n's
// edge-tile kernel needs launch n - 1's inner part done (it reads that
// part's output and overwrites the buffer that part read) and launch n's
// inner part needs launch n - 1's edge-tile kernel done (the same, the other
// way); with kJoinDefer on every launch but the last and kJoinPrev on every
// launch but the first, those are the only waits, so the edge-tile kernels,
// the longer of the two, follow one another on `side` without a round trip
// through s.  The inner part splits further: its march items or inner tiles
// away from the edge tiles depend on neither edge-tile kernel and run before
// the wait.
hipError_t launch_three_step(const LatDesc& L, int parity, int id, hipStream_t s, hipStream_t side, hipEvent_t fork,
                             hipEvent_t join, int flags) {
  if (!three_step_supported(L, id)) return hipErrorInvalidValue;
  const bool march = kThree[id].mr > 0;
  const int mid = id - (kNumThree - kNumMarch);
  if (march && !(L.closure && L.net)) return launch_three_march(L, parity, mid, s, true);
  int part = 0;
  const bool forked = L.closure && L.net && side && fork && join;
  if (L.closure && L.net) {
    hipError_t e = hipSuccess;
    if (forked) {
      e = hipEventRecord(fork, s);
      if (e == hipSuccess) e = hipStreamWaitEvent(side, fork, 0);
    }
    const int cid = march ? closure_tile_of(id) : id;
    if (e == hipSuccess) e = cid >= 0 ? launch_three_step_closure(L, parity, cid, forked ? side : s) : hipErrorInvalidValue;
    // the march items (inner tiles) whose reads and writes stay 3 nodes or
    // more from every edge tile touch nothing an edge-tile kernel reads or
    // writes: they go before the wait for the previous launch's edge-tile
    // kernel
    if (forked && march && e == hipSuccess) e = launch_three_march(L, parity, mid, s, false, 1);
    if (forked && !march && e == hipSuccess) {
      switch (L.store) {
        case ST_F64: e = launch_three_s<ST_F64, false>(L, parity, id, s, 3); break;
        case ST_F32: e = launch_three_s<ST_F32, false>(L, parity, id, s, 3); break;
        case ST_F16: e = launch_three_s<ST_F16, false>(L, parity, id, s, 3); break;
        case ST_BF16: e = launch_three_s<ST_BF16, false>(L, parity, id, s, 3); break;
      }
    }
    // s waits for the previous launch's edge-tile kernel before join is recorded anew
    if (forked && (flags & kJoinPrev) && e == hipSuccess) e = hipStreamWaitEvent(s, join, 0);
    if (forked && e == hipSuccess) e = hipEventRecord(join, side);
    if (e != hipSuccess) return e;
    part = forked ? 4 : 1;
  }
  const bool wait_end = forked && !(flags & kJoinDefer);
  hipError_t e = hipErrorInvalidValue;
  if (march) {
    // the closure kernel took the edge tiles: the march covers the inner
    // rectangle (on two streams, the items bordering the edge tiles here)
    e = launch_three_march(L, parity, mid, s, false, forked ? 2 : 0);
    if (wait_end && e == hipSuccess) e = hipStreamWaitEvent(s, join, 0);
    return e;
  }
  switch (L.store) {
    case ST_F64: e = launch_three_s<ST_F64, false>(L, parity, id, s, part); break;
    case ST_F32: e = launch_three_s<ST_F32, false>(L, parity, id, s, part); break;
    case ST_F16: e = launch_three_s<ST_F16, false>(L, parity, id, s, part); break;
    case ST_BF16: e = launch_three_s<ST_BF16, false>(L, parity, id, s, part); break;
  }
  if (wait_end && e == hipSuccess) e = hipStreamWaitEvent(s, join, 0);
  return e;
}

// ------------------------------------------------------------------ ensemble
// One block per entry of a device list of (member, tile) in block order (the
// host lays the list out so that each XCD takes a contiguous stretch of it);
// entries with lat < 0 pad the grid.  The member's descriptor carries its
// collision model, read at run time.
template <int S, int TY, int NT, bool NTS>
__global__ __launch_bounds__(NT, two_step_waves<S>()) void k_ens_two_step(const LatDesc* __restrict__ descs,
                                                     const TwoTile* __restrict__ list, int parity) {
  const TwoTile t = list[blockIdx.x];
  if (t.lat < 0) return;  // padding: the whole block leaves before any barrier
  const LatDesc L = descs[t.lat];
  two_step_tile<S, TY, NT, NTS, -1>(L, parity, t.txi, t.tyi);
}

int two_step_tile_rows(int id) { return id >= 0 && id < kNumTwo ? kTwo[id].ty : 0; }

int two_step_min_rows() {
  int m = kTwo[0].ty;
  for (int i = 1; i < kNumTwo; ++i) m = kTwo[i].ty < m ? kTwo[i].ty : m;
  return m;
}

// Three-step sweep over an ensemble's tile list (as k_ens_two_step).
template <int S, int TY, int NT, bool NTS>
__global__ __launch_bounds__(NT, two_step_waves<S>()) void k_ens_three_step(const LatDesc* __restrict__ descs,
                                                       const TwoTile* __restrict__ list, int parity) {
  const TwoTile t = list[blockIdx.x];
  if (t.lat < 0) return;  // padding: the whole block leaves before any barrier
  const LatDesc L = descs[t.lat];
  three_step_tile<S, TY, NT, NTS, -1>(L, parity, t.txi, t.tyi);
}

int three_step_tile_rows(int id) { return id >= 0 && id < kNumThree ? kThree[id].ty : 0; }

int three_step_min_rows() {
  int m = kThree[0].ty;
  for (int i = 1; i < kNumThree; ++i) m = kThree[i].ty < m ? kThree[i].ty : m;
  return m;
}

template <int S>
static hipError_t launch_ens_three_s(int id, const LatDesc* d, const TwoTile* list, int n, int parity,
                                     hipStream_t s) {
  int k = 0;
#define X(a, b, c)                                                                        \
  if (id == k) {                                                                          \
    if constexpr (three_step_fits<S, a>()) {                                              \
      k_ens_three_step<S, a, b, c><<<dim3(n), dim3(b), 0, s>>>(d, list, parity);          \
      return hipGetLastError();                                                           \
    } else {                                                                              \
      return hipErrorInvalidValue;                                                        \
    }                                                                                     \
  }                                                                                       \
  ++k;
  LBM_THREE_STEP(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_ens_three_step(int store, int id, const LatDesc* d, const TwoTile* list, int n, int parity,
                                 hipStream_t s) {
  if (n <= 0) return hipSuccess;
  switch (store) {
    case ST_F64: return launch_ens_three_s<ST_F64>(id, d, list, n, parity, s);
    case ST_F32: return launch_ens_three_s<ST_F32>(id, d, list, n, parity, s);
    case ST_F16: return launch_ens_three_s<ST_F16>(id, d, list, n, parity, s);
    case ST_BF16: return launch_ens_three_s<ST_BF16>(id, d, list, n, parity, s);
  }
  return hipErrorInvalidValue;
}

template <int S>
static hipError_t launch_ens_two_s(int id, const LatDesc* d, const TwoTile* list, int n, int parity,
                                   hipStream_t s) {
  int k = 0;
#define X(a, b, c, m)                                                                   \
  if (id == k) {                                                                        \
    k_ens_two_step<S, a, b, c><<<dim3(n), dim3(b), 0, s>>>(d, list, parity);            \
    return hipGetLastError();                                                           \
  }                                                                                     \
  ++k;
  LBM_TWO_STEP(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_ens_two_step(int store, int id, const LatDesc* d, const TwoTile* list, int n, int parity,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  switch (store) {
    case ST_F64: return launch_ens_two_s<ST_F64>(id, d, list, n, parity, s);
    case ST_F32: return launch_ens_two_s<ST_F32>(id, d, list, n, parity, s);
    case ST_F16: return launch_ens_two_s<ST_F16>(id, d, list, n, parity, s);
    case ST_BF16: return launch_ens_two_s<ST_BF16>(id, d, list, n, parity, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbm
