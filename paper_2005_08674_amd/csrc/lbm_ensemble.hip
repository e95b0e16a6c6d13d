// lbm_ensemble.hip -- batched ensemble of independent lattices (include/lbm_ensemble.h).
//
// Every member keeps the single-lattice layout (two 9-plane buffers) inside
// one workspace arena.  A device table lists, for one launch of the bulk
// kernel, the (member, tile) of every block, and another lists the (member,
// edge, segment) of every block of the edge kernel, so a whole ensemble step
// is two launches whatever the member count.  Each block copies its member's
// descriptor from device memory and runs exactly the per-tile bodies of the
// single-lattice kernels, so results are bit-identical to lattices run alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <tuple>
#include <utility>
#include <vector>

#include "lbm.h"
#include "lbm_trace.h"
#include "lbm_closure.h"
#include "lbm_ensemble.h"
#include "lbm_device.h"
#include "lbm_host.h"
#include "lbm_launch.h"
#include "lbm_sweep.h"
#include "lbm_twostep_lds.h"

namespace lbm {

struct EnsTile {
  int32_t lat, txi, tyi, pad;
};
struct EnsSeg {
  int32_t lat, edge, seg, pad;
};

template <int S, int BX, int BY, int NYT>
__global__ __launch_bounds__(BX* BY) void k_ens_bulk(const LatDesc* __restrict__ descs,
                                                     const EnsTile* __restrict__ tiles, int parity) {
  const EnsTile t = tiles[blockIdx.x];
  const LatDesc L = descs[t.lat];
  bulk_tile_body<S, BX, BY, NYT, true, false>(L, parity, t.txi, t.tyi);
}

template <int S>
__global__ __launch_bounds__(EDGE_THREADS) void k_ens_edge(const LatDesc* __restrict__ descs,
                                                          const EnsSeg* __restrict__ segs, int parity) {
  __shared__ typename Codec<S>::R mom[3][DEPTH][STRIP];
  const EnsSeg sg = segs[blockIdx.x];
  const LatDesc L = descs[sg.lat];
  edge_segment_body<S, false>(L, parity, sg.edge, sg.seg, mom, nullptr);
}

// Edge kernel of an ensemble in which some members use the learned closure;
// a block of a member without it runs the plain NSBC path (uniform branch).
template <int S>
__global__ __launch_bounds__(EDGE_THREADS) void k_ens_edge_closure(const LatDesc* __restrict__ descs,
                                                                  const EnsSeg* __restrict__ segs, int parity) {
  __shared__ typename Codec<S>::R mom[3][DEPTH][STRIP];
  __shared__ ClosureLds cl;
  const EnsSeg sg = segs[blockIdx.x];
  const LatDesc L = descs[sg.lat];
  if (L.closure && L.net) edge_segment_body<S, true>(L, parity, sg.edge, sg.seg, mom, &cl);
  else edge_segment_body<S, false>(L, parity, sg.edge, sg.seg, mom, nullptr);
}

// Entry of the fused step's work list: a bulk tile (lat, txi, tyi), an edge
// segment (lat, edge, seg) or padding.
enum EnsWorkKind : int32_t { W_TILE = 0, W_SEG = 1, W_NONE = 2 };
struct EnsWork {
  int32_t lat, a, b, kind;
};

// One launch per ensemble step (no member on the closure).  Block i takes
// work item i, and runs on XCD i mod 8: the host orders the list so that each
// band of 64 rows of a member -- its bulk tiles, then the left and right edge
// segments of those rows -- sits on one XCD back to back, so the edge blocks'
// strided column reads find the lines the band's bulk tiles just pulled
// through that XCD's L2.  Identical results to the separate launches.
template <int S, int BX, int BY, int NYT>
__global__ __launch_bounds__(BX* BY) void k_ens_step(const LatDesc* __restrict__ descs,
                                                     const EnsWork* __restrict__ work, int parity) {
  __shared__ typename Codec<S>::R mom[3][DEPTH][STRIP];
  const EnsWork w = work[blockIdx.x];
  if (w.kind == W_NONE) return;
  const LatDesc L = descs[w.lat];
  if (w.kind == W_SEG) {
    edge_segment_body<S, false>(L, parity, w.a, w.b, mom, nullptr);
    return;
  }
  bulk_tile_body<S, BX, BY, NYT, true, false>(L, parity, w.a, w.b);
}

struct EnsShape {
  int bx, by, nyt;
};

#define LBM_ENS_SHAPES(X) \
  X(64, 4, 1)             \
  X(128, 2, 1)            \
  X(256, 1, 1)            \
  X(64, 4, 2)             \
  X(128, 2, 2)            \
  X(64, 8, 1)             \
  X(64, 4, 4)             \
  X(128, 2, 4)            \
  X(256, 1, 4)            \
  X(64, 8, 2)             \
  X(32, 8, 2)             \
  X(128, 4, 2)

static const EnsShape kEnsShapes[] = {
#define X(a, b, c) {a, b, c},
    LBM_ENS_SHAPES(X)
#undef X
};
static constexpr int kNumEnsShapes = sizeof(kEnsShapes) / sizeof(kEnsShapes[0]);

template <int S>
static hipError_t launch_ens_bulk_s(int shape, const LatDesc* d, const EnsTile* t, int n, int parity,
                                    hipStream_t s) {
  int id = 0;
#define X(a, b, c)                                                              \
  if (shape == id) {                                                            \
    k_ens_bulk<S, a, b, c><<<dim3(n), dim3(a, b), 0, s>>>(d, t, parity);        \
    return hipGetLastError();                                                   \
  }                                                                             \
  ++id;
  LBM_ENS_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

static hipError_t launch_ens_bulk(int store, int shape, const LatDesc* d, const EnsTile* t, int n, int parity,
                                  hipStream_t s) {
  if (n <= 0) return hipSuccess;
  switch (store) {
    case ST_F64: return launch_ens_bulk_s<ST_F64>(shape, d, t, n, parity, s);
    case ST_F32: return launch_ens_bulk_s<ST_F32>(shape, d, t, n, parity, s);
    case ST_F16: return launch_ens_bulk_s<ST_F16>(shape, d, t, n, parity, s);
    case ST_BF16: return launch_ens_bulk_s<ST_BF16>(shape, d, t, n, parity, s);
  }
  return hipErrorInvalidValue;
}

template <int S>
static hipError_t launch_ens_step_s(int shape, const LatDesc* d, const EnsWork* w, int nw, int parity,
                                   hipStream_t s) {
  int id = 0;
#define X(a, b, c)                                                                 \
  if (shape == id) {                                                               \
    k_ens_step<S, a, b, c><<<dim3(nw), dim3(a, b), 0, s>>>(d, w, parity);          \
    return hipGetLastError();                                                      \
  }                                                                                \
  ++id;
  LBM_ENS_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

static hipError_t launch_ens_step(int store, int shape, const LatDesc* d, const EnsWork* w, int nw, int parity,
                                  hipStream_t s) {
  if (nw <= 0) return hipSuccess;
  switch (store) {
    case ST_F64: return launch_ens_step_s<ST_F64>(shape, d, w, nw, parity, s);
    case ST_F32: return launch_ens_step_s<ST_F32>(shape, d, w, nw, parity, s);
    case ST_F16: return launch_ens_step_s<ST_F16>(shape, d, w, nw, parity, s);
    case ST_BF16: return launch_ens_step_s<ST_BF16>(shape, d, w, nw, parity, s);
  }
  return hipErrorInvalidValue;
}

static hipError_t launch_ens_edge(int store, bool closure, const LatDesc* d, const EnsSeg* sg, int n, int parity,
                                  hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid(n), block(EDGE_THREADS);
#define LBM_ENS_EDGE(ST)                                                             \
  if (closure) k_ens_edge_closure<ST><<<grid, block, 0, s>>>(d, sg, parity);         \
  else k_ens_edge<ST><<<grid, block, 0, s>>>(d, sg, parity);
  switch (store) {
    case ST_F64: LBM_ENS_EDGE(ST_F64) break;
    case ST_F32: LBM_ENS_EDGE(ST_F32) break;
    case ST_F16: LBM_ENS_EDGE(ST_F16) break;
    case ST_BF16: LBM_ENS_EDGE(ST_BF16) break;
    default: return hipErrorInvalidValue;
  }
#undef LBM_ENS_EDGE
  return hipGetLastError();
}

}  // namespace lbm

namespace {

using lbm::host::fail;

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(LBM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 4096;

struct EnsLayout {
  size_t off_descs, off_tiles, off_segs, off_work, off_two, off_scratch, off_lattices, total;
  size_t max_tiles, nsegs, max_work, max_two;
  std::vector<size_t> lat_off;  // member buffers, relative to the workspace
  std::vector<lbm::host::Layout> lat;
};

size_t tiles_for(const lbm_params& p, const lbm::EnsShape& s) {
  const size_t tx = (p.nx + s.bx - 1) / s.bx;
  const size_t ty = (p.ny - 2 + s.by * s.nyt - 1) / (s.by * s.nyt);
  return tx * ty;
}

int ens_layout(const lbm_params* m, int32_t count, EnsLayout& L) {
  if (!m || count < 1) return fail(LBM_ERR_ARG, "need at least one member");
  for (int32_t k = 0; k < count; ++k) {
    int rc = lbm::host::check_params(&m[k]);
    if (rc) return fail(rc, "member %d: %s", k, lbm::host::last_error());
    if (m[k].store != m[0].store) return fail(LBM_ERR_ARG, "member %d: all members must share one store", k);
  }
  using lbm::host::round_up;
  L.max_tiles = 0;
  L.nsegs = 0;
  for (int s = 0; s < lbm::kNumEnsShapes; ++s) {
    size_t n = 0;
    for (int32_t k = 0; k < count; ++k) n += tiles_for(m[k], lbm::kEnsShapes[s]);
    L.max_tiles = std::max(L.max_tiles, n);
  }
  for (int32_t k = 0; k < count; ++k) L.nsegs += lbm::edge_blocks(m[k].nx, m[k].ny);
  if (L.max_tiles > (size_t)INT32_MAX || L.nsegs > (size_t)INT32_MAX) return fail(LBM_ERR_ARG, "ensemble too large");
  size_t off = 0;
  L.off_descs = off;
  off = round_up(off + sizeof(lbm::LatDesc) * count, kAlign);
  L.off_tiles = off;
  off = round_up(off + sizeof(lbm::EnsTile) * L.max_tiles, kAlign);
  L.off_segs = off;
  off = round_up(off + sizeof(lbm::EnsSeg) * L.nsegs, kAlign);
  // work list of the fused step: every tile and segment plus the padding that
  // evens out the eight per-XCD lists (at most 7 entries per list item)
  L.max_work = 8 * (L.max_tiles + L.nsegs) + 64;
  L.off_work = off;
  off = round_up(off + sizeof(lbm::EnsWork) * L.max_work, kAlign);
  // tile list of the two-step sweep at its shortest tiles, padded to a multiple of 8
  L.max_two = 8;
  const int tymin = std::min(lbm::two_step_min_rows(), lbm::three_step_min_rows());
  for (int32_t k = 0; k < count; ++k)
    L.max_two += (size_t)((m[k].nx + lbm::TL_TX - 1) / lbm::TL_TX) * ((m[k].ny + tymin - 1) / tymin);
  if (L.max_two > (size_t)INT32_MAX) return fail(LBM_ERR_ARG, "ensemble too large");
  L.off_two = off;
  off = round_up(off + sizeof(lbm::TwoTile) * L.max_two, kAlign);
  L.off_scratch = off;
  off = round_up(off + lbm::host::kScratchBytes, (size_t)2 << 20);
  L.off_lattices = off;
  L.lat.resize(count);
  L.lat_off.resize(count);
  for (int32_t k = 0; k < count; ++k) {
    L.lat[k] = lbm::host::layout(&m[k]);
    L.lat_off[k] = off;
    off += 2 * L.lat[k].buf_bytes;
  }
  L.total = off;
  return LBM_OK;
}

}  // namespace

struct lbm_ens {
  int32_t count = 0;
  int store = 0;
  std::vector<lbm_params> p;
  std::vector<lbm::LatDesc> descs;
  EnsLayout lay;
  char* ws = nullptr;
  lbm::LatDesc* d_descs = nullptr;
  lbm::EnsTile* d_tiles = nullptr;
  lbm::EnsSeg* d_segs = nullptr;
  lbm::EnsWork* d_work = nullptr;
  int32_t ntiles = 0, nsegs = 0, nwork = 0;
  int shape = 0;
  int parity = 0;
  int64_t t = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;  // private stream used for graph capture
  // captured graphs by (n, parity, log_every, log buffer, log sites)
  std::map<std::tuple<int, int, int, uintptr_t, uintptr_t, uintptr_t, int>, hipGraphExec_t> graphs;
  // training-data sites logged by lbm_ens_step_graph (device arrays, borrowed)
  const int32_t* log_ms = nullptr;
  const int32_t* log_ts = nullptr;
  int32_t log_n = 0;
  bool any_closure = false;
  bool fused = true;  // one launch per step when no member runs the closure
  int two = -1;       // two-step shape, or -1 (single steps)
  lbm::TwoTile* d_two = nullptr;
  int32_t ntwo = 0;
};

namespace {

void drop_graphs(lbm_ens* e) {
  for (auto& kv : e->graphs) (void)hipGraphExecDestroy(kv.second);
  e->graphs.clear();
}

int upload_descs(lbm_ens* e) {
  HIPCHK(hipMemcpyAsync(e->d_descs, e->descs.data(), sizeof(lbm::LatDesc) * e->count, hipMemcpyHostToDevice,
                        e->stream));
  HIPCHK(hipStreamSynchronize(e->stream));
  return LBM_OK;
}

int build_tiles(lbm_ens* e, int shape) {
  const lbm::EnsShape& s = lbm::kEnsShapes[shape];
  // per member, its bulk tiles with the interior row on which each starts
  std::vector<lbm::EnsTile> tiles;
  std::vector<std::vector<std::pair<lbm::EnsTile, int>>> mtiles(e->count);
  for (int32_t k = 0; k < e->count; ++k) {
    const int nx = e->p[k].nx, ny = e->p[k].ny;
    const int tx = (nx + s.bx - 1) / s.bx;
    const int ty = (ny - 2 + s.by * s.nyt - 1) / (s.by * s.nyt);
    for (int j = 0; j < ty; ++j)
      for (int i = 0; i < tx; ++i) mtiles[k].push_back({{k, i, j, 0}, j * s.by * s.nyt});
    for (const auto& t : mtiles[k]) tiles.push_back(t.first);
  }
  if (tiles.size() > e->lay.max_tiles) return fail(LBM_ERR_STATE, "tile table overflow");
  // Work list of the fused step: bands of SEG rows per member, each holding
  // the bulk tiles whose first row lies in it, then that band's left and
  // right edge segments (the bottom/top segments join the first/last band);
  // bands go whole to the least loaded of the 8 XCD lists, which are then
  // interleaved (entry 8 j + k is item j of list k) and padded to one length.
  std::vector<std::vector<lbm::EnsWork>> xcd(8);
  std::vector<size_t> load(8, 0);
  for (int32_t k = 0; k < e->count; ++k) {
    const int nx = e->p[k].nx, ny = e->p[k].ny;
    const int nsv = lbm::edge_segments_v(ny), nsh = lbm::edge_segments_h(nx);
    std::vector<std::vector<lbm::EnsWork>> bands(nsv);
    for (const auto& t : mtiles[k]) {
      const int band = std::min((1 + t.second) / lbm::SEG, nsv - 1);  // lattice row = 1 + interior row
      bands[band].push_back({k, t.first.txi, t.first.tyi, lbm::W_TILE});
    }
    for (int b = 0; b < nsv; ++b) {
      bands[b].push_back({k, lbm::E_LEFT, b, lbm::W_SEG});
      bands[b].push_back({k, lbm::E_RIGHT, b, lbm::W_SEG});
    }
    for (int b = 0; b < nsh; ++b) {
      bands[0].push_back({k, lbm::E_BOTTOM, b, lbm::W_SEG});
      bands[nsv - 1].push_back({k, lbm::E_TOP, b, lbm::W_SEG});
    }
    for (auto& band : bands) {
      const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      xcd[x].insert(xcd[x].end(), band.begin(), band.end());
      load[x] += band.size();
    }
  }
  const size_t len = *std::max_element(load.begin(), load.end());
  std::vector<lbm::EnsWork> work(8 * len, lbm::EnsWork{0, 0, 0, lbm::W_NONE});
  for (int x = 0; x < 8; ++x)
    for (size_t j = 0; j < xcd[x].size(); ++j) work[8 * j + x] = xcd[x][j];
  if (work.size() > e->lay.max_work) return fail(LBM_ERR_STATE, "work list overflow");
  HIPCHK(hipMemcpyAsync(e->d_tiles, tiles.data(), sizeof(lbm::EnsTile) * tiles.size(), hipMemcpyHostToDevice,
                        e->stream));
  HIPCHK(hipMemcpyAsync(e->d_work, work.data(), sizeof(lbm::EnsWork) * work.size(), hipMemcpyHostToDevice,
                        e->stream));
  HIPCHK(hipStreamSynchronize(e->stream));
  e->ntiles = (int32_t)tiles.size();
  e->nwork = (int32_t)work.size();
  e->shape = shape;
  drop_graphs(e);
  return LBM_OK;
}

// Two-step tile list in block order: the member-major, row-major list of
// 64 x TY tiles is cut into 8 contiguous stretches and block b takes item
// (b mod 8) * per + b / 8, so XCD k (block b runs on XCD b mod 8) works through
// stretch k and neighbouring tiles share its L2; the tail pads with lat = -1.
// Multi-step shapes: ids below num_two_step() are two-step shapes, the next
// num_three_step() three-step shapes (as in the single-lattice API).
int ens_multi_count() { return lbm::num_two_step() + lbm::num_three_step(); }
int ens_multi_steps(int id) { return id < lbm::num_two_step() ? 2 : 3; }

int build_two(lbm_ens* e, int id) {
  const int n2 = lbm::num_two_step();
  const int ty = id < n2 ? lbm::two_step_tile_rows(id) : lbm::three_step_tile_rows(id - n2);
  if (ty <= 0) return fail(LBM_ERR_ARG, "multi-step shape %d out of range", id);
  std::vector<lbm::TwoTile> items;
  for (int32_t k = 0; k < e->count; ++k) {
    const int tx = (e->p[k].nx + lbm::TL_TX - 1) / lbm::TL_TX, tyn = (e->p[k].ny + ty - 1) / ty;
    for (int j = 0; j < tyn; ++j)
      for (int i = 0; i < tx; ++i) items.push_back({k, i, j, 0});
  }
  const size_t n = items.size(), per = (n + 7) / 8;
  std::vector<lbm::TwoTile> list(8 * per, lbm::TwoTile{-1, 0, 0, 0});
  for (size_t b = 0; b < list.size(); ++b) {
    const size_t item = (b & 7) * per + (b >> 3);
    if (item < n) list[b] = items[item];
  }
  if (list.size() > e->lay.max_two) return fail(LBM_ERR_STATE, "two-step list overflow");
  HIPCHK(hipMemcpyAsync(e->d_two, list.data(), sizeof(lbm::TwoTile) * list.size(), hipMemcpyHostToDevice,
                        e->stream));
  HIPCHK(hipStreamSynchronize(e->stream));
  e->ntwo = (int32_t)list.size();
  e->two = id;
  drop_graphs(e);
  return LBM_OK;
}

// every member takes the sweep (id -1: the two-step sweeps' common condition)
bool two_supported(const lbm_ens* e, int id = -1) {
  const int n2 = lbm::num_two_step();
  for (const auto& d : e->descs) {
    if (!lbm::two_step_supported(d)) return false;
    if (id >= 0 && id < n2 && lbm::two_step_is_march(id)) return false;
    if (id >= n2 && (lbm::three_step_is_march(id - n2) || !lbm::three_step_supported(d, id - n2))) return false;
  }
  return true;
}

// Members on the learned closure need the separate edge launch, so they step singly.
bool use_two(const lbm_ens* e) { return e->two >= 0 && !e->any_closure; }

hipError_t ens_launch_multi(const lbm_ens* e, int id, int parity, hipStream_t s) {
  const int n2 = lbm::num_two_step();
  return id < n2 ? lbm::launch_ens_two_step(e->store, id, e->d_descs, e->d_two, e->ntwo, parity, s)
                 : lbm::launch_ens_three_step(e->store, id - n2, e->d_descs, e->d_two, e->ntwo, parity, s);
}

int ens_launch_two(lbm_ens* e, int parity, hipStream_t s) {
  HIPCHK(ens_launch_multi(e, e->two, parity, s));
  return LBM_OK;
}

int ens_launch_step(lbm_ens* e, int parity, hipStream_t s) {
  if (!e->any_closure && e->fused) {
    HIPCHK(lbm::launch_ens_step(e->store, e->shape, e->d_descs, e->d_work, e->nwork, parity, s));
    return LBM_OK;
  }
  HIPCHK(lbm::launch_ens_bulk(e->store, e->shape, e->d_descs, e->d_tiles, e->ntiles, parity, s));
  HIPCHK(lbm::launch_ens_edge(e->store, e->any_closure, e->d_descs, e->d_segs, e->nsegs, parity, s));
  return LBM_OK;
}

int check_member(const lbm_ens* e, int32_t m) {
  if (!e) return fail(LBM_ERR_ARG, "ensemble is NULL");
  if (m < 0 || m >= e->count) return fail(LBM_ERR_ARG, "member %d out of range [0, %d)", m, e->count);
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_ens_workspace_bytes(const lbm_params* members, int32_t count, size_t* bytes) {
  if (!bytes) return fail(LBM_ERR_ARG, "bytes is NULL");
  EnsLayout L;
  int rc = ens_layout(members, count, L);
  if (rc) return rc;
  *bytes = L.total;
  return LBM_OK;
}

void lbm_ens_destroy(lbm_ens* e) {
  if (!e) return;
  (void)hipStreamSynchronize(e->stream);
  drop_graphs(e);
  if (e->cap) (void)hipStreamDestroy(e->cap);
  delete e;
}

int lbm_ens_init(lbm_ens** out, const lbm_params* members, int32_t count, void* workspace, size_t bytes,
                 const double* drho, const double* ux, const double* uy, void* hip_stream) {
  if (!out) return fail(LBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  EnsLayout lay;
  int rc = ens_layout(members, count, lay);
  if (rc) return rc;
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(LBM_ERR_ARG, "workspace NULL or not 256-byte aligned");
  if (bytes < lay.total) return fail(LBM_ERR_ARG, "workspace of %zu bytes < %zu required", bytes, lay.total);
  if (!drho || !ux || !uy) return fail(LBM_ERR_ARG, "initial fields must not be NULL");

  lbm_ens* e = new lbm_ens();
  e->count = count;
  e->store = members[0].store;
  e->p.assign(members, members + count);
  e->lay = lay;
  e->ws = static_cast<char*>(workspace);
  e->stream = static_cast<hipStream_t>(hip_stream);
  e->d_descs = reinterpret_cast<lbm::LatDesc*>(e->ws + lay.off_descs);
  e->d_tiles = reinterpret_cast<lbm::EnsTile*>(e->ws + lay.off_tiles);
  e->d_segs = reinterpret_cast<lbm::EnsSeg*>(e->ws + lay.off_segs);
  e->d_work = reinterpret_cast<lbm::EnsWork*>(e->ws + lay.off_work);
  e->d_two = reinterpret_cast<lbm::TwoTile*>(e->ws + lay.off_two);
  if (hipStreamCreateWithFlags(&e->cap, hipStreamNonBlocking) != hipSuccess) {
    lbm_ens_destroy(e);
    return fail(LBM_ERR_HIP, "capture stream creation failed");
  }
  e->descs.resize(count);
  float* part = reinterpret_cast<float*>(e->ws + lay.off_scratch);
  std::vector<float> host(lbm::absmax_blocks());
  size_t foff = 0;
  for (int32_t k = 0; k < count; ++k) {
    const lbm_params& p = members[k];
    char* base = e->ws + lay.lat_off[k];
    lbm::host::fill_desc(e->descs[k], &p, lay.lat[k], base, base + lay.lat[k].buf_bytes);
    int kexp = 0;
    if (p.store == LBM_STORE_F16DEV) {
      if (p.f16_exp == LBM_F16_EXP_AUTO) {
        hipError_t he = lbm::launch_absmax_init(e->descs[k], drho + foff, ux + foff, uy + foff, part, e->stream);
        if (he == hipSuccess)
          he = hipMemcpyAsync(host.data(), part, host.size() * sizeof(float), hipMemcpyDeviceToHost, e->stream);
        if (he == hipSuccess) he = hipStreamSynchronize(e->stream);
        if (he != hipSuccess) {
          lbm_ens_destroy(e);
          return fail(LBM_ERR_HIP, "member %d f16 exponent: %s", k, hipGetErrorString(he));
        }
        float mx = 0.f;
        for (float v : host) mx = std::max(mx, v);
        kexp = lbm::host::f16_exp_from_max(mx);
      } else {
        kexp = p.f16_exp;
      }
    }
    lbm::host::set_scales(e->descs[k], p.store, kexp);
    hipError_t he = lbm::launch_init(e->descs[k], 0, drho + foff, ux + foff, uy + foff, e->stream);
    if (he != hipSuccess) {
      lbm_ens_destroy(e);
      return fail(LBM_ERR_HIP, "member %d init: %s", k, hipGetErrorString(he));
    }
    foff += (size_t)p.nx * p.ny;
  }
  std::vector<lbm::EnsSeg> segs;
  for (int32_t k = 0; k < count; ++k) {
    const int nb = lbm::edge_blocks(members[k].nx, members[k].ny);
    for (int b = 0; b < nb; ++b) {
      int bb = b, edge = 0;
      lbm::edge_of_block(members[k].nx, members[k].ny, bb, edge);
      segs.push_back({k, edge, bb, 0});
    }
  }
  e->nsegs = (int32_t)segs.size();
  hipError_t he = hipMemcpyAsync(e->d_segs, segs.data(), sizeof(lbm::EnsSeg) * segs.size(), hipMemcpyHostToDevice,
                                 e->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(e->stream);
  if (he != hipSuccess) {
    lbm_ens_destroy(e);
    return fail(LBM_ERR_HIP, "segment table: %s", hipGetErrorString(he));
  }
  if ((rc = upload_descs(e)) || (rc = build_tiles(e, 0))) {
    lbm_ens_destroy(e);
    return rc;
  }
  *out = e;
  return LBM_OK;
}

int lbm_ens_set_farfield(lbm_ens* e, int32_t member, double beta, double rho_ref, double ux_ref, double uy_ref) {
  int rc = check_member(e, member);
  if (rc) return rc;
  lbm::LatDesc L = e->descs[member];
  rc = lbm::host::set_farfield(L, beta, rho_ref, ux_ref, uy_ref);
  if (rc) return rc;
  e->descs[member] = L;
  return upload_descs(e);
}

int lbm_ens_set_velocity_edge(lbm_ens* e, int32_t member, double ux, double uy) {
  int rc = check_member(e, member);
  if (rc) return rc;
  lbm::LatDesc L = e->descs[member];
  rc = lbm::host::set_velocity_edge(L, ux, uy);
  if (rc) return rc;
  e->descs[member] = L;
  return upload_descs(e);
}

int lbm_ens_step(lbm_ens* e, int32_t n) {
  const lbm::TraceRange trace_range("lbm_ens_step");
  if (!e) return fail(LBM_ERR_ARG, "ensemble is NULL");
  if (n < 0) return fail(LBM_ERR_ARG, "n = %d < 0", n);
  const int k = use_two(e) ? ens_multi_steps(e->two) : 1;
  for (int32_t s = 0; s < n;) {
    const bool multi = k > 1 && n - s >= k;
    int rc = multi ? ens_launch_two(e, e->parity, e->stream) : ens_launch_step(e, e->parity, e->stream);
    if (rc) return rc;
    e->parity ^= 1;  // a multi-step launch writes t + k into the other buffer
    e->t += multi ? k : 1;
    s += multi ? k : 1;
  }
  return LBM_OK;
}

static_assert(LBM_ENS_LOG_FLOATS == lbm::mlp::IN + (lbm::mlp::OUT + 1) + lbm::mlp::OUT, "log record layout");

int lbm_ens_set_log_sites(lbm_ens* e, const int32_t* member_sites, const int32_t* twin_sites, int32_t n) {
  if (!e) return fail(LBM_ERR_ARG, "ensemble is NULL");
  if (n < 0 || (n > 0 && (!member_sites || !twin_sites))) return fail(LBM_ERR_ARG, "bad log sites (n = %d)", n);
  if (n > (1 << 24)) return fail(LBM_ERR_ARG, "%d log sites exceed 2^24", n);
  e->log_ms = n ? member_sites : nullptr;
  e->log_ts = n ? twin_sites : nullptr;
  e->log_n = n;
  return LBM_OK;
}

int lbm_ens_log_bytes(const lbm_ens* e, int32_t n, int32_t log_every, size_t* bytes) {
  if (!e || !bytes) return fail(LBM_ERR_ARG, "NULL argument");
  if (n < 1 || log_every < 1) return fail(LBM_ERR_ARG, "n = %d and log_every = %d must be >= 1", n, log_every);
  const size_t logs = (size_t)((n + log_every - 1) / log_every);
  *bytes = logs * (size_t)e->log_n * LBM_ENS_LOG_FLOATS * sizeof(float);
  return LBM_OK;
}

int lbm_ens_step_graph(lbm_ens* e, int32_t n, void* log_buf, size_t log_bytes, int32_t log_every) {
  const lbm::TraceRange trace_range("lbm_ens_step_graph");
  if (!e) return fail(LBM_ERR_ARG, "ensemble is NULL");
  if (n < 1 || n > 100000) return fail(LBM_ERR_ARG, "n = %d outside [1, 100000]", n);
  const bool logging = log_buf != nullptr;
  if (logging) {
    if (log_every < 1) return fail(LBM_ERR_ARG, "log_every = %d must be >= 1", log_every);
    if (e->log_n <= 0) return fail(LBM_ERR_STATE, "no log sites set (lbm_ens_set_log_sites)");
    size_t need = 0;
    int rc = lbm_ens_log_bytes(e, n, log_every, &need);
    if (rc) return rc;
    if (log_bytes < need) return fail(LBM_ERR_ARG, "log buffer of %zu bytes < %zu required", log_bytes, need);
    if ((uintptr_t)log_buf & 15) return fail(LBM_ERR_ARG, "log buffer not 16-byte aligned");
  } else {
    log_every = 0;
  }
  const bool two = use_two(e);
  const int k = two ? ens_multi_steps(e->two) : 1;
  // launches of s steps from parity p: multi-step launches while they fit, then single steps
  auto run = [&](int steps, int& p, hipStream_t st) -> int {
    for (int32_t s = 0; s < steps;) {
      const bool multi = k > 1 && steps - s >= k;
      int rc = multi ? ens_launch_two(e, p, st) : ens_launch_step(e, p, st);
      if (rc) return rc;
      p ^= 1;
      s += multi ? k : 1;
    }
    return LBM_OK;
  };
  const auto key = std::make_tuple(n, e->parity, log_every, (uintptr_t)log_buf, (uintptr_t)e->log_ms,
                                   (uintptr_t)e->log_ts, logging ? e->log_n : 0);
  auto it = e->graphs.find(key);
  int end_parity = e->parity;
  {
    // parity after the n steps (the same launches as the capture below)
    int p = e->parity;
    if (!logging) {
      for (int32_t s = 0; s < n;) {
        const bool multi = k > 1 && n - s >= k;
        p ^= 1;
        s += multi ? k : 1;
      }
    } else {
      for (int32_t s = 0; s < n; s += log_every) {
        p ^= 1;  // the logged step
        const int rest = std::min(log_every - 1, n - s - 1);
        for (int32_t q = 0; q < rest;) {
          const bool multi = k > 1 && rest - q >= k;
          p ^= 1;
          q += multi ? k : 1;
        }
      }
    }
    end_parity = p;
  }
  if (it == e->graphs.end()) {
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(e->cap, hipStreamCaptureModeThreadLocal));
    int rc = LBM_OK;
    int p = e->parity;
    if (!logging) {
      rc = run(n, p, e->cap);
    } else {
      // record j (step s = j * log_every): inputs at time s at the member sites, one step, then the
      // twin's moments at s + 1 at the twin sites minus m_c (the residual target), then the rest
      const size_t rec = (size_t)e->log_n * LBM_ENS_LOG_FLOATS;
      float* base = static_cast<float*>(log_buf);
      for (int32_t s = 0, j = 0; s < n && rc == LBM_OK; s += log_every, ++j) {
        float* feat = base + (size_t)j * rec;
        float* mc = feat + (size_t)e->log_n * lbm::mlp::IN;
        float* res = mc + (size_t)e->log_n * (lbm::mlp::OUT + 1);
        hipError_t he = lbm::host::closure_features(nullptr, e->d_descs, e->count, p, e->log_ms, e->log_n, feat, mc,
                                                    e->cap);
        if (he != hipSuccess) {
          rc = fail(LBM_ERR_HIP, "log features: %s", hipGetErrorString(he));
          break;
        }
        rc = ens_launch_step(e, p, e->cap);
        if (rc) break;
        p ^= 1;
        he = lbm::host::closure_moments(nullptr, e->d_descs, e->count, p, e->log_ts, e->log_n, mc, res, e->cap);
        if (he != hipSuccess) {
          rc = fail(LBM_ERR_HIP, "log moments: %s", hipGetErrorString(he));
          break;
        }
        rc = run(std::min(log_every - 1, n - s - 1), p, e->cap);
      }
    }
    hipError_t he = hipStreamEndCapture(e->cap, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (he != hipSuccess) return fail(LBM_ERR_HIP, "graph capture: %s", hipGetErrorString(he));
    if (p != end_parity) {
      (void)hipGraphDestroy(g);
      return fail(LBM_ERR_STATE, "internal: captured parity %d != %d", p, end_parity);
    }
    hipGraphExec_t x = nullptr;
    he = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (he != hipSuccess) return fail(LBM_ERR_HIP, "graph instantiate: %s", hipGetErrorString(he));
    it = e->graphs.emplace(key, x).first;
  }
  HIPCHK(hipGraphLaunch(it->second, e->stream));
  e->parity = end_parity;
  e->t += n;
  return lbm::host::debug_sync(e->stream, "lbm_ens_step_graph");
}

int lbm_ens_moments(lbm_ens* e, int32_t member, void* r, void* u, void* v, int out_f64, int deviation) {
  int rc = check_member(e, member);
  if (rc) return rc;
  HIPCHK(lbm::launch_moments(e->descs[member], e->parity, r, u, v, out_f64 ? 1 : 0, deviation ? 1 : 0, e->stream));
  return LBM_OK;
}

int lbm_ens_get_populations(lbm_ens* e, int32_t member, double* g_out) {
  int rc = check_member(e, member);
  if (rc) return rc;
  if (!g_out) return fail(LBM_ERR_ARG, "g_out is NULL");
  HIPCHK(lbm::launch_get_pops(e->descs[member], e->parity, g_out, e->stream));
  return LBM_OK;
}

int lbm_ens_time(const lbm_ens* e, int64_t* t) {
  if (!e || !t) return fail(LBM_ERR_ARG, "NULL argument");
  *t = e->t;
  return LBM_OK;
}

int lbm_ens_info(const lbm_ens* e, int64_t* nodes, int32_t* bulk_blocks, int32_t* edge_blocks) {
  if (!e) return fail(LBM_ERR_ARG, "ensemble is NULL");
  if (nodes) {
    int64_t n = 0;
    for (const auto& p : e->p) n += (int64_t)p.nx * p.ny;
    *nodes = n;
  }
  if (bulk_blocks) *bulk_blocks = e->ntiles;
  if (edge_blocks) *edge_blocks = e->nsegs;
  return LBM_OK;
}

int lbm_ens_set_closure(lbm_ens* e, int32_t member, const void* net, int mode) {
  if (!e) return fail(LBM_ERR_ARG, "ensemble is NULL");
  if (member < -1 || member >= e->count) return fail(LBM_ERR_ARG, "member %d out of range", member);
  if (mode != 0 && mode != 1) return fail(LBM_ERR_ARG, "closure mode %d", mode);
  if (mode == 1 && !net) return fail(LBM_ERR_ARG, "closure mode 1 needs a network");
  if (net && ((uintptr_t)net & 15)) return fail(LBM_ERR_ARG, "network blob not 16-byte aligned");
  for (int32_t k = (member < 0 ? 0 : member); k < (member < 0 ? e->count : member + 1); ++k) {
    e->descs[k].net = mode ? net : nullptr;
    e->descs[k].closure = mode;
  }
  bool any = false;
  for (const auto& d : e->descs) any = any || (d.closure && d.net);
  if (any != e->any_closure) drop_graphs(e);  // captured launches name the kernel variant
  e->any_closure = any;
  return upload_descs(e);
}

int lbm_ens_set_fused(lbm_ens* e, int on) {
  if (!e) return fail(LBM_ERR_ARG, "ensemble is NULL");
  if ((on != 0) != e->fused) drop_graphs(e);  // captured launches name the kernels
  e->fused = on != 0;
  return LBM_OK;
}

int lbm_ens_closure_features(lbm_ens* e, const int32_t* sites, int32_t n, float* feat_out, float* mc_out) {
  if (!e || (n > 0 && (!sites || !feat_out || !mc_out))) return fail(LBM_ERR_ARG, "NULL argument");
  if (n < 0) return fail(LBM_ERR_ARG, "n < 0");
  HIPCHK(lbm::host::closure_features(nullptr, e->d_descs, e->count, e->parity, sites, n, feat_out, mc_out, e->stream));
  return LBM_OK;
}

int lbm_ens_closure_moments(lbm_ens* e, const int32_t* sites, int32_t n, const float* sub, float* m_out) {
  if (!e || (n > 0 && (!sites || !m_out))) return fail(LBM_ERR_ARG, "NULL argument");
  if (n < 0) return fail(LBM_ERR_ARG, "n < 0");
  HIPCHK(lbm::host::closure_moments(nullptr, e->d_descs, e->count, e->parity, sites, n, sub, m_out, e->stream));
  return LBM_OK;
}

int lbm_ens_shape_count(void) { return lbm::kNumEnsShapes; }

int lbm_ens_shape_describe(int32_t id, char* buf, size_t len) {
  if (!buf || len == 0) return fail(LBM_ERR_ARG, "NULL buffer");
  if (id < 0 || id >= lbm::kNumEnsShapes) return fail(LBM_ERR_ARG, "shape id %d out of range", id);
  const lbm::EnsShape& s = lbm::kEnsShapes[id];
  snprintf(buf, len, "%dx%dx%d", s.bx, s.by, s.nyt);
  return LBM_OK;
}

int lbm_ens_set_shape(lbm_ens* e, int32_t id) {
  if (!e) return fail(LBM_ERR_ARG, "ensemble is NULL");
  if (id < 0 || id >= lbm::kNumEnsShapes) return fail(LBM_ERR_ARG, "shape id %d out of range", id);
  return build_tiles(e, id);
}

int lbm_ens_autotune(lbm_ens* e, int32_t reps, int32_t* best, float* times_ms) {
  const lbm::TraceRange trace_range("lbm_ens_autotune");
  if (!e || !best) return fail(LBM_ERR_ARG, "NULL argument");
  if (reps < 1 || reps > 1000) return fail(LBM_ERR_ARG, "reps = %d outside [1, 1000]", reps);
  std::vector<hipEvent_t> ev(2 * reps);
  for (auto& x : ev) HIPCHK(hipEventCreate(&x));
  float best_t = 1e30f;
  int best_id = e->shape;
  int rc = LBM_OK;
  for (int id = 0; id < lbm::kNumEnsShapes && rc == LBM_OK; ++id) {
    rc = build_tiles(e, id);
    if (rc) break;
    // timed: the launch a step uses (the fused step, or the bulk kernel when
    // fusion is off or a member runs the closure); both read buffer `parity`
    // and write only the other one
    const bool fused = e->fused && !e->any_closure;
    auto launch = [&]() {
      return fused ? lbm::launch_ens_step(e->store, id, e->d_descs, e->d_work, e->nwork, e->parity, e->stream)
                   : lbm::launch_ens_bulk(e->store, id, e->d_descs, e->d_tiles, e->ntiles, e->parity, e->stream);
    };
    hipError_t he = launch();
    for (int r = 0; r < reps && he == hipSuccess; ++r) {
      he = hipEventRecord(ev[2 * r], e->stream);
      if (he == hipSuccess) he = launch();
      if (he == hipSuccess) he = hipEventRecord(ev[2 * r + 1], e->stream);
    }
    if (he == hipSuccess) he = hipStreamSynchronize(e->stream);
    std::vector<float> ts(reps);
    for (int r = 0; r < reps && he == hipSuccess; ++r) he = hipEventElapsedTime(&ts[r], ev[2 * r], ev[2 * r + 1]);
    if (he != hipSuccess) {
      rc = fail(LBM_ERR_HIP, "ensemble autotune shape %d: %s", id, hipGetErrorString(he));
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
  rc = build_tiles(e, best_id);
  if (rc) return rc;
  *best = best_id;
  return LBM_OK;
}

int lbm_ens_set_two_step(lbm_ens* e, int32_t id) {
  if (!e) return fail(LBM_ERR_ARG, "ensemble is NULL");
  if (id == -1) {
    if (e->two != -1) drop_graphs(e);
    e->two = -1;
    return LBM_OK;
  }
  if (id < 0 || id >= ens_multi_count()) return fail(LBM_ERR_ARG, "multi-step shape %d out of range", id);
  if (!two_supported(e)) return fail(LBM_ERR_UNSUPPORTED, "the multi-step sweeps need NSBC on all four edges of every member");
  if (!two_supported(e, id))
    return fail(LBM_ERR_UNSUPPORTED, "three-step shape %d needs every member >= 64 x its tile rows (and LDS for the format)", id);
  return build_two(e, id);
}

int lbm_ens_get_two_step(const lbm_ens* e, int32_t* id) {
  if (!e || !id) return fail(LBM_ERR_ARG, "NULL argument");
  *id = e->two;
  return LBM_OK;
}

int lbm_ens_autotune_two_step(lbm_ens* e, int32_t reps, int32_t* best, float* times_ms) {
  const lbm::TraceRange trace_range("lbm_ens_autotune_two_step");
  if (!e || !best) return fail(LBM_ERR_ARG, "NULL argument");
  if (reps < 1 || reps > 1000) return fail(LBM_ERR_ARG, "reps = %d outside [1, 1000]", reps);
  if (!two_supported(e)) return fail(LBM_ERR_UNSUPPORTED, "the multi-step sweeps need NSBC on all four edges of every member");
  std::vector<hipEvent_t> ev(2 * reps);
  for (auto& x : ev) HIPCHK(hipEventCreate(&x));
  float best_t = 1e30f;
  int best_id = 0;
  int rc = LBM_OK;
  for (int id = 0; id < ens_multi_count() && rc == LBM_OK; ++id) {
    if (!two_supported(e, id)) {
      if (times_ms) times_ms[id] = -1.f;
      continue;
    }
    rc = build_two(e, id);
    if (rc) break;
    // the sweep reads buffer `parity` and writes only the other one: the state is not advanced
    hipError_t he = ens_launch_multi(e, id, e->parity, e->stream);
    for (int r = 0; r < reps && he == hipSuccess; ++r) {
      he = hipEventRecord(ev[2 * r], e->stream);
      if (he == hipSuccess) he = ens_launch_multi(e, id, e->parity, e->stream);
      if (he == hipSuccess) he = hipEventRecord(ev[2 * r + 1], e->stream);
    }
    if (he == hipSuccess) he = hipStreamSynchronize(e->stream);
    std::vector<float> ts(reps);
    for (int r = 0; r < reps && he == hipSuccess; ++r) he = hipEventElapsedTime(&ts[r], ev[2 * r], ev[2 * r + 1]);
    if (he != hipSuccess) {
      rc = fail(LBM_ERR_HIP, "ensemble two-step shape %d: %s", id, hipGetErrorString(he));
      break;
    }
    std::sort(ts.begin(), ts.end());
    // shapes advance 2 or 3 steps per launch: compare time per step
    const float per_step = ts[reps / 2] / (float)ens_multi_steps(id);
    if (times_ms) times_ms[id] = per_step;
    if (per_step < best_t) {
      best_t = per_step;
      best_id = id;
    }
  }
  for (auto& x : ev) (void)hipEventDestroy(x);
  if (rc) return rc;
  rc = build_two(e, best_id);
  if (rc) return rc;
  *best = best_id;
  return LBM_OK;
}

}  // extern "C"
