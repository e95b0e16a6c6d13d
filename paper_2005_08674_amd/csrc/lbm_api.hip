// lbm_api.hip -- the C ABI declared in include/lbm.h: context lifetime,
// workspace layout, parameter checking, step loop, timing and autotuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_trace.h"
#include "lbm_closure.h"
#include "lbm_device.h"
#include "lbm_host.h"
#include "lbm_launch.h"

namespace lbm {
namespace host {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

const char* last_error() { return g_err.c_str(); }

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_bytes(int store) {
  switch (store) {
    case LBM_STORE_F64: return 8;
    case LBM_STORE_F32: return 4;
    default: return 2;
  }
}

Layout layout(const lbm_params* p) {
  Layout l;
  l.esize = elem_bytes(p->store);
  const size_t row = round_up((size_t)p->nx * l.esize, 256);
  l.pitch = (int32_t)(row / l.esize);
  size_t plane_bytes = round_up(row * (size_t)p->ny, 4096);
  // keep the nine planes from sitting a large power of two apart, so the 18
  // concurrent streams of one step do not start on the same HBM channel
  if (plane_bytes % 65536 == 0) plane_bytes += 4096;
  l.plane = (int64_t)(plane_bytes / l.esize);
  l.buf_bytes = round_up(9 * plane_bytes, (size_t)2 << 20);
  l.total = 2 * l.buf_bytes + kScratchBytes;
  return l;
}

int check_params(const lbm_params* p) {
  if (!p) return fail(LBM_ERR_ARG, "params is NULL");
  if (p->nx < 3 || p->ny < 3) return fail(LBM_ERR_ARG, "lattice %dx%d: each side must be >= 3", p->nx, p->ny);
  if ((int64_t)p->nx * p->ny > (int64_t)1 << 28)
    return fail(LBM_ERR_ARG, "lattice %dx%d exceeds 2^28 nodes", p->nx, p->ny);
  if (p->store >= LBM_STORE_F64 && p->store <= LBM_STORE_BF16DEV) {
    // the sweeps address a plane with 32-bit byte offsets (row * pitch + x)
    const int64_t row = ((int64_t)p->nx * (int64_t)elem_bytes(p->store) + 255) / 256 * 256;
    if (row * p->ny > ((int64_t)1 << 32) - 65536)
      return fail(LBM_ERR_ARG, "lattice %dx%d: a plane with rows padded to 256 bytes exceeds 4 GiB", p->nx, p->ny);
  }
  if (p->collision != LBM_COLL_BGK && p->collision != LBM_COLL_MRT)
    return fail(LBM_ERR_ARG, "collision = %d is not LBM_COLL_BGK or LBM_COLL_MRT", p->collision);
  if (p->collision == LBM_COLL_BGK && (!(p->tau > 0.5) || !std::isfinite(p->tau)))
    return fail(LBM_ERR_ARG, "tau = %g: BGK needs tau > 0.5", p->tau);
  if (p->collision == LBM_COLL_MRT) {
    if (!(p->tau >= 0.5) || !std::isfinite(p->tau))
      return fail(LBM_ERR_ARG, "tau = %g: MRT needs tau >= 0.5 (omega_nu <= 2)", p->tau);
    const double r[3] = {p->omega_e, p->omega_eps, p->omega_q};
    for (int k = 0; k < 3; ++k)
      if (!(r[k] > 0.0 && r[k] <= 2.0))
        return fail(LBM_ERR_ARG, "MRT rates (%g, %g, %g) must lie in (0, 2]", r[0], r[1], r[2]);
  }
  if (!(p->rho0 > 0) || !std::isfinite(p->rho0)) return fail(LBM_ERR_ARG, "rho0 = %g must be > 0", p->rho0);
  for (int e = 0; e < 4; ++e)
    if (p->bc[e] != LBM_BC_PERIODIC && p->bc[e] != LBM_BC_NSBC && p->bc[e] != LBM_BC_VELOCITY)
      return fail(LBM_ERR_ARG, "bc[%d] = %d is not LBM_BC_PERIODIC, LBM_BC_NSBC or LBM_BC_VELOCITY", e, p->bc[e]);
  if (p->bc[2] == LBM_BC_VELOCITY || p->bc[3] == LBM_BC_VELOCITY)
    return fail(LBM_ERR_ARG, "velocity edges are supported on the left and right edges only");
  if ((p->bc[0] == LBM_BC_VELOCITY || p->bc[1] == LBM_BC_VELOCITY) && p->bc[2] != LBM_BC_PERIODIC)
    return fail(LBM_ERR_ARG, "a velocity edge needs periodic bottom and top edges");
  if ((p->bc[0] == LBM_BC_PERIODIC) != (p->bc[1] == LBM_BC_PERIODIC) ||
      (p->bc[2] == LBM_BC_PERIODIC) != (p->bc[3] == LBM_BC_PERIODIC))
    return fail(LBM_ERR_ARG, "periodic edges must come in pairs (left+right, bottom+top)");
  if (!std::isfinite(p->gamma)) return fail(LBM_ERR_ARG, "gamma must be finite");
  if (!std::isfinite(p->ubase[0]) || !std::isfinite(p->ubase[1]) ||
      p->ubase[0] * p->ubase[0] + p->ubase[1] * p->ubase[1] > 0.25)
    return fail(LBM_ERR_ARG, "base velocity (%g, %g) must be finite with |u_b| <= 0.5", p->ubase[0], p->ubase[1]);
  if (p->store < LBM_STORE_F64 || p->store > LBM_STORE_BF16DEV) return fail(LBM_ERR_ARG, "store = %d", p->store);
  if (p->corr_mode != 0 && p->corr_mode != 1) return fail(LBM_ERR_ARG, "corr_mode = %d", p->corr_mode);
  if (p->grad_order != 1 && p->grad_order != 2) return fail(LBM_ERR_ARG, "grad_order = %d", p->grad_order);
  if (p->corner_mode != 0 && p->corner_mode != 1) return fail(LBM_ERR_ARG, "corner_mode = %d", p->corner_mode);
  if (p->store == LBM_STORE_F16DEV && p->f16_exp != LBM_F16_EXP_AUTO && (p->f16_exp < -30 || p->f16_exp > 60))
    return fail(LBM_ERR_ARG, "f16_exp = %d outside [-30, 60]", p->f16_exp);
  return LBM_OK;
}

void set_scales(LatDesc& L, int store, int k) {
  L.sc = (store == LBM_STORE_F64 || store == LBM_STORE_F32) ? 1.0f : (float)std::ldexp(1.0, k);
  for (int i = 0; i < 9; ++i) {
    if (store == LBM_STORE_F64 || store == LBM_STORE_F32) {
      L.ds[i] = 1.0f;
      L.es[i] = 1.0f;
    } else {
      const double w = wgt<double>(i);
      L.ds[i] = (float)std::ldexp(w, -k);
      L.es[i] = (float)std::ldexp(1.0 / w, k);  // 2.25, 9, 36 times 2^k: exact
    }
  }
}

void fill_desc(LatDesc& L, const lbm_params* p, const Layout& lay, void* buf0, void* buf1) {
  std::memset(&L, 0, sizeof(L));
  L.buf[0] = buf0;
  L.buf[1] = buf1;
  L.nx = p->nx;
  L.ny = p->ny;
  L.pitch = lay.pitch;
  L.store = p->store;
  L.plane = lay.plane;
  for (int e = 0; e < 4; ++e) L.bc[e] = p->bc[e];
  L.corr_mode = p->corr_mode;
  L.grad_order = p->grad_order;
  L.corner_mode = p->corner_mode;
  L.omega = 1.0 / p->tau;
  L.coll = p->collision == LBM_COLL_MRT ? COLL_MRT : COLL_BGK;
  if (L.coll == COLL_MRT) {
    // s_k / |row_k|^2 for the e, eps, q and stress rows (lbm_device.h, mrt())
    L.mk[0] = p->omega_e / 36.0;
    L.mk[1] = p->omega_eps / 36.0;
    L.mk[2] = p->omega_q / 12.0;
    L.mk[3] = L.omega / 4.0;
    for (int k = 0; k < 4; ++k) L.mkf[k] = static_cast<float>(L.mk[k]);
  }
  L.rho0 = p->rho0;
  L.gamma = p->gamma;
  L.beta = 0.0;
  L.ub[0] = p->ubase[0];
  L.ub[1] = p->ubase[1];
  for (int i = 0; i < 9; ++i) {
    const double cu = kCx[i] * p->ubase[0] + kCy[i] * p->ubase[1];
    L.pb[i] = 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (p->ubase[0] * p->ubase[0] + p->ubase[1] * p->ubase[1]);
    L.pbf[i] = static_cast<float>(L.pb[i]);
  }
  L.ubf[0] = static_cast<float>(L.ub[0]);
  L.ubf[1] = static_cast<float>(L.ub[1]);
  L.ub_zero = p->ubase[0] == 0.0 && p->ubase[1] == 0.0;
  // far field m0 = (rho0, 0, 0) until set
  L.m0[0] = 0.0;
  L.m0[1] = -p->ubase[0];
  L.m0[2] = -p->ubase[1];
  set_scales(L, p->store, 0);
  set_velocity_edge(L, 0.0, 0.0);
}

int set_velocity_edge(LatDesc& L, double ux, double uy) {
  if (!std::isfinite(ux) || !std::isfinite(uy) || ux * ux + uy * uy > 0.25)
    return fail(LBM_ERR_ARG, "velocity (%g, %g) must be finite with |u| <= 0.5", ux, uy);
  L.uw[0] = ux;
  L.uw[1] = uy;
  L.duw[0] = ux - L.ub[0];
  L.duw[1] = uy - L.ub[1];
  for (int k = 0; k < 2; ++k) {
    L.uwf[k] = static_cast<float>(L.uw[k]);
    L.duwf[k] = static_cast<float>(L.duw[k]);
  }
  return LBM_OK;
}

int set_farfield(LatDesc& L, double beta, double rho_ref, double ux_ref, double uy_ref) {
  if (!(beta >= 0.0 && beta <= 1.0)) return fail(LBM_ERR_ARG, "beta = %g outside [0, 1]", beta);
  if (!std::isfinite(rho_ref) || !std::isfinite(ux_ref) || !std::isfinite(uy_ref))
    return fail(LBM_ERR_ARG, "reference vector must be finite");
  L.beta = beta;
  L.m0[0] = rho_ref - L.rho0;
  L.m0[1] = ux_ref - L.ub[0];
  L.m0[2] = uy_ref - L.ub[1];
  return LBM_OK;
}

namespace {
int g_debug = -1;  // -1: not read from the environment yet
}

int debug_level() {
  if (g_debug < 0) {
    const char* e = std::getenv("LBM_DEBUG");
    g_debug = e ? std::max(0, std::min(2, std::atoi(e))) : 0;
  }
  return g_debug;
}

void set_debug_level(int level) { g_debug = std::max(0, std::min(2, level)); }

int debug_sync(hipStream_t s, const char* call) {
  if (debug_level() == 0) return LBM_OK;
  hipError_t e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return fail(LBM_ERR_HIP, "%s (LBM_DEBUG): %s", call, hipGetErrorString(e));
  return LBM_OK;
}

uint64_t fnv1a(const void* p, size_t n, uint64_t h) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

int f16_exp_from_max(float mx) {
  int k = mx > 1e-30f ? (int)std::floor(std::log2(4096.0 / (double)mx)) : 12;
  return std::min(60, std::max(-30, k));
}

}  // namespace host
}  // namespace lbm

namespace {

using lbm::host::fail;
using lbm::host::Layout;
using lbm::host::layout;
using lbm::host::check_params;
using lbm::host::kScratchBytes;

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(LBM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kOffEnergy = 0;            // energy partials (double)
constexpr size_t kOffAbsmax = 64 << 10;     // absmax partials (float)
constexpr size_t kOffFlag = 128 << 10;      // finiteness flag (int)

int default_tile(const lbm_params*) { return 0; }

}  // namespace

// Scratch of lbm_energy_noalloc: the block partials of the fixed-grid fp64
// energy reduction.  Each GPU holds its own copy for the life of the process;
// host code reaches it only through the device address looked up per device.
constexpr int kNoAllocPartials = 1024;  // 8 KiB
static __device__ __align__(256) double scratch[kNoAllocPartials];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's `scratch`, looked up on the first call
// on that device (the symbol's host-side name is not a device address).
int scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(LBM_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(LBM_ERR_UNSUPPORTED, "device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(LBM_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}
}  // namespace

struct lbm_ctx {
  int device = -1;  // GPU current at lbm_init
  lbm_params p;
  lbm::LatDesc L;
  Layout lay;
  int parity = 0;
  hipStream_t stream = nullptr;
  int64_t t = 0;
  char* ws = nullptr;
  char* scratch = nullptr;
  int tile = 0;
  int f16_exp = 0;
  // edge kernel on a second stream, overlapped with the bulk kernel
  bool overlap = false;
  hipStream_t side = nullptr;
  hipEvent_t ev_bulk = nullptr, ev_edge = nullptr;
  // per-kernel timing
  bool timing = false;
  std::vector<hipEvent_t> events;
  size_t ev_used = 0;
  double bulk_ms = 0, edge_ms = 0;
  int64_t bulk_n = 0, edge_n = 0;
  std::vector<char> ev_two;  // per 4-event group: 1 = a two-step launch (events 0, 1)
  double two_ms = 0;
  int64_t two_n = 0;
  // multi-step sweep shape (-1: off)
  int two_step = -1;
  // a closure launch's wait of the stream for its edge-tile kernel (on the
  // second stream) deferred to the next launch or to the end of lbm_step
  bool join_pending = false;
  // shape per steps-per-launch k (2..4) that runs a remainder of k steps
  // after launches of the selected shape (the autotuner's best shape with
  // that many steps, else a default)
  int rem_best[5] = {-1, -1, -1, -1, -1};
  // edge segments and bulk tiles of a step in one launch
  bool fused = true;
};

namespace {

int flush_timing(lbm_ctx* c) {
  if (c->ev_used == 0) return LBM_OK;
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipStreamSynchronize(c->side));
  for (size_t k = 0; k + 3 < c->ev_used; k += 4) {
    float a = 0, b = 0;
    HIPCHK(hipEventElapsedTime(&a, c->events[k], c->events[k + 1]));
    if (c->ev_two[k / 4] == 1) {
      c->two_ms += a;
      c->two_n += 1;
      continue;
    }
    if (c->ev_two[k / 4] == 2) {  // fused step launch
      c->bulk_ms += a;
      c->bulk_n += 1;
      continue;
    }
    HIPCHK(hipEventElapsedTime(&b, c->events[k + 2], c->events[k + 3]));
    c->bulk_ms += a;
    c->edge_ms += b;
    c->bulk_n += 1;
    c->edge_n += 1;
  }
  c->ev_used = 0;
  c->ev_two.clear();
  return LBM_OK;
}

int next_event(lbm_ctx* c, hipEvent_t* ev) {
  if (c->ev_used == c->events.size()) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    c->events.push_back(e);
  }
  *ev = c->events[c->ev_used++];
  return LBM_OK;
}

// Launch one step.  The bulk kernel goes on the context's stream; the edge
// kernel goes on the side stream when overlapping (else on the same stream).
// Both read buffer `parity` and write disjoint node sets of the other one, so
// within a step they are independent; across steps each waits for both
// kernels of the previous step (events ev_bulk / ev_edge).
bool use_fused(const lbm_ctx* c) { return c->fused && !c->overlap && !(c->L.closure && c->L.net); }

int step_once(lbm_ctx* c) {
  if (use_fused(c)) {
    // one launch; timed as the step's bulk kernel (events 0, 1)
    hipEvent_t t[4] = {nullptr, nullptr, nullptr, nullptr};
    if (c->timing) {
      if (c->ev_used + 4 > 4 * 4096) {
        int rc = flush_timing(c);
        if (rc) return rc;
      }
      for (int k = 0; k < 4; ++k) {
        int rc = next_event(c, &t[k]);
        if (rc) return rc;
      }
      c->ev_two.push_back(2);
    }
    if (t[0]) HIPCHK(hipEventRecord(t[0], c->stream));
    HIPCHK(lbm::launch_step(c->L, c->parity, c->tile, c->stream));
    if (t[1]) HIPCHK(hipEventRecord(t[1], c->stream));
    c->parity ^= 1;
    c->t += 1;
    return LBM_OK;
  }
  hipStream_t es = c->overlap ? c->side : c->stream;
  hipEvent_t t[4] = {nullptr, nullptr, nullptr, nullptr};
  if (c->timing) {
    if (c->ev_used + 4 > 4 * 4096) {
      int rc = flush_timing(c);
      if (rc) return rc;
    }
    for (int k = 0; k < 4; ++k) {
      int rc = next_event(c, &t[k]);
      if (rc) return rc;
    }
    c->ev_two.push_back(0);
  }
  if (c->overlap) {
    HIPCHK(hipStreamWaitEvent(c->side, c->ev_bulk, 0));    // bulk kernel of the previous step
    HIPCHK(hipStreamWaitEvent(c->stream, c->ev_edge, 0));  // edge kernel of the previous step
  }
  if (t[2]) HIPCHK(hipEventRecord(t[2], es));
  HIPCHK(lbm::launch_edge(c->L, c->parity, es));
  if (t[3]) HIPCHK(hipEventRecord(t[3], es));
  if (c->overlap) HIPCHK(hipEventRecord(c->ev_edge, es));
  if (t[0]) HIPCHK(hipEventRecord(t[0], c->stream));
  HIPCHK(lbm::launch_bulk(c->L, c->parity, c->tile, c->stream));
  if (t[1]) HIPCHK(hipEventRecord(t[1], c->stream));
  if (c->overlap) HIPCHK(hipEventRecord(c->ev_bulk, c->stream));
  c->parity ^= 1;
  c->t += 1;
  return LBM_OK;
}

// Multi-step sweep shapes: ids below num_two_step() are two-step shapes,
// the next num_three_step() are three-step shapes.
int multi_count() { return lbm::num_two_step() + lbm::num_three_step(); }
int multi_steps(int id) { return id < lbm::num_two_step() ? 2 : 3; }
// (with the learned closure only the three-step shapes: the two-step sweep has no closure path)
bool multi_supported(const lbm::LatDesc& L, int id) {
  if (id < 0 || id >= multi_count()) return false;
  return id < lbm::num_two_step() ? lbm::two_step_supported(L) && !(L.closure && L.net)
                                  : lbm::three_step_supported(L, id - lbm::num_two_step());
}
// (a closure lattice's edge-tile kernel runs on the context's second stream)
hipError_t launch_multi(const lbm_ctx* c, int parity, int id, int flags = 0) {
  return id < lbm::num_two_step()
             ? lbm::launch_two_step(c->L, parity, id, c->stream)
             : lbm::launch_three_step(c->L, parity, id - lbm::num_two_step(), c->stream, c->side, c->ev_bulk,
                                      c->ev_edge, flags);
}
// Whether launch `id` runs a closure lattice's edge tiles on the second stream.
bool forks_closure(const lbm_ctx* c, int id) {
  return id >= lbm::num_two_step() && c->L.closure && c->L.net && c->side && c->ev_bulk && c->ev_edge;
}
// One launch of a run of consecutive launches: a closure launch leaves the
// stream's wait for its edge-tile kernel pending (the next launch issues it
// before its own kernel on the stream, settle_join otherwise).
hipError_t launch_multi_run(const lbm_ctx* c, int parity, int id, bool& pending) {
  if (!forks_closure(c, id)) {
    if (pending) {
      pending = false;
      const hipError_t e = hipStreamWaitEvent(c->stream, c->ev_edge, 0);
      if (e != hipSuccess) return e;
    }
    return launch_multi(c, parity, id);
  }
  const hipError_t e = launch_multi(c, parity, id, lbm::kJoinDefer | (pending ? lbm::kJoinPrev : 0));
  pending = true;  // (also after a failure: waiting for the last recorded edge-tile kernel is harmless)
  return e;
}
// The stream waits for the last edge-tile kernel of the run, if one is pending.
hipError_t settle_join(const lbm_ctx* c, bool& pending) {
  if (!pending) return hipSuccess;
  pending = false;
  return hipStreamWaitEvent(c->stream, c->ev_edge, 0);
}
void multi_name(int id, char* buf, size_t len) {
  if (id < lbm::num_two_step())
    lbm::two_step_name(id, buf, len);
  else
    lbm::three_step_name(id - lbm::num_two_step(), buf, len);
}

// Two or three steps in one launch of multi-step shape `id` (same results as
// that many step_once calls).
int step_multi(lbm_ctx* c, int id) {
  hipEvent_t t[4] = {nullptr, nullptr, nullptr, nullptr};
  if (c->timing) {
    if (c->ev_used + 4 > 4 * 4096) {
      int rc = flush_timing(c);
      if (rc) return rc;
    }
    for (int k = 0; k < 4; ++k) {
      int rc = next_event(c, &t[k]);
      if (rc) return rc;
    }
    c->ev_two.push_back(1);
  }
  if (t[0]) HIPCHK(settle_join(c, c->join_pending));
  if (t[0]) HIPCHK(hipEventRecord(t[0], c->stream));
  HIPCHK(launch_multi_run(c, c->parity, id, c->join_pending));
  // (timed launches take the edge-tile kernel into their interval)
  if (t[1]) HIPCHK(settle_join(c, c->join_pending));
  if (t[1]) HIPCHK(hipEventRecord(t[1], c->stream));
  // the last level is in the other buffer: the launch wrote buffer parity ^ 1
  c->parity ^= 1;
  c->t += multi_steps(id);
  return LBM_OK;
}

// Shape that runs a remainder of k steps (2 <= k <= 4): the autotuner's best
// supported shape with k steps per launch, else (k = 2) the two-step shape
// measured fastest at 4096^2 for the format (tiles 64x12/512 for FP64,
// 64x20/768 for FP32, the 64x8 march for the 16-bit formats); -1 if none.
int rem_shape(const lbm_ctx* c, int k) {
  if (k < 2 || k > 4) return -1;
  if (c->rem_best[k] >= 0 && multi_supported(c->L, c->rem_best[k])) return c->rem_best[k];
  if (k == 2) {
    const char* want = c->p.store == LBM_STORE_F64   ? "2step:64x12/512+xcdband+nts"
                       : c->p.store == LBM_STORE_F32 ? "2step:64x20/768+xcdband+nts"
                                                     : "2step:64x8/512+march7xh96+xcdband+nts";
    char buf[64];
    for (int id = 0; id < lbm::num_two_step(); ++id) {
      lbm::two_step_name(id, buf, sizeof(buf));
      if (std::strcmp(buf, want) == 0 && multi_supported(c->L, id)) return id;
    }
  }
  return -1;
}

bool use_two_step(const lbm_ctx* c) {
  return c->two_step >= 0 && !c->overlap && multi_supported(c->L, c->two_step);
}

}  // namespace

extern "C" {

int lbm_params_default(lbm_params* p) {
  if (!p) return fail(LBM_ERR_ARG, "params is NULL");
  std::memset(p, 0, sizeof(*p));
  p->nx = 3;
  p->ny = 3;
  p->tau = 0.6;
  p->rho0 = 1.0;
  for (int e = 0; e < 4; ++e) p->bc[e] = LBM_BC_NSBC;
  p->gamma = 0.6;
  p->store = LBM_STORE_F32;
  p->corr_mode = 0;
  p->grad_order = 1;
  p->corner_mode = 0;
  p->f16_exp = LBM_F16_EXP_AUTO;
  p->collision = LBM_COLL_BGK;
  p->omega_e = p->omega_eps = p->omega_q = 1.9;
  return LBM_OK;
}

int lbm_workspace_bytes(const lbm_params* p, size_t* bytes) {
  int rc = check_params(p);
  if (rc) return rc;
  if (!bytes) return fail(LBM_ERR_ARG, "bytes is NULL");
  *bytes = layout(p).total;
  return LBM_OK;
}

int lbm_init(lbm_ctx** out, const lbm_params* p, void* workspace, size_t bytes, const double* drho,
             const double* ux, const double* uy, void* hip_stream) {
  if (!out) return fail(LBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  int rc = check_params(p);
  if (rc) return rc;
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(LBM_ERR_ARG, "workspace NULL or not 256-byte aligned");
  if (!drho || !ux || !uy) return fail(LBM_ERR_ARG, "initial fields must not be NULL");
  Layout lay = layout(p);
  if (bytes < lay.total) return fail(LBM_ERR_ARG, "workspace of %zu bytes < %zu required", bytes, lay.total);

  lbm_ctx* c = new lbm_ctx();
  {
    hipError_t e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_bulk, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_edge, hipEventDisableTiming);
    if (e != hipSuccess) {
      lbm_destroy(c);
      return fail(LBM_ERR_HIP, "stream/event creation: %s", hipGetErrorString(e));
    }
  }
  {
    // set-up of the allocation-free entry point's scratch on this GPU
    void* sp = nullptr;
    int rc2 = hipGetDevice(&c->device) == hipSuccess ? scratch_of_current_device(&sp)
                                                     : fail(LBM_ERR_HIP, "hipGetDevice failed");
    if (rc2) {
      lbm_destroy(c);
      return rc2;
    }
  }
  c->p = *p;
  c->lay = lay;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->ws = static_cast<char*>(workspace);
  c->scratch = c->ws + 2 * lay.buf_bytes;
  lbm::LatDesc& L = c->L;
  lbm::host::fill_desc(L, p, lay, c->ws, c->ws + lay.buf_bytes);
  c->tile = default_tile(p);

  int k = 0;
  if (p->store == LBM_STORE_F16DEV) {
    if (p->f16_exp == LBM_F16_EXP_AUTO) {
      float* part = reinterpret_cast<float*>(c->scratch + kOffAbsmax);
      std::vector<float> host(lbm::absmax_blocks());
      hipError_t e = lbm::launch_absmax_init(L, drho, ux, uy, part, c->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(host.data(), part, host.size() * sizeof(float), hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) {
        lbm_destroy(c);
        return fail(LBM_ERR_HIP, "f16 exponent reduction: %s", hipGetErrorString(e));
      }
      float mx = 0.f;
      for (float v : host) mx = std::max(mx, v);
      if (!std::isfinite(mx)) {
        lbm_destroy(c);
        return fail(LBM_ERR_ARG, "initial fields are not finite");
      }
      k = lbm::host::f16_exp_from_max(mx);
    } else {
      k = p->f16_exp;
    }
  }
  c->f16_exp = k;
  lbm::host::set_scales(L, p->store, k);

  hipError_t e = lbm::launch_init(L, 0, drho, ux, uy, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    lbm_destroy(c);
    return fail(LBM_ERR_HIP, "init kernel: %s", hipGetErrorString(e));
  }
  *out = c;
  return LBM_OK;
}

int lbm_set_farfield(lbm_ctx* c, double beta, double rho_ref, double ux_ref, double uy_ref) {
  if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
  return lbm::host::set_farfield(c->L, beta, rho_ref, ux_ref, uy_ref);
}

int lbm_set_velocity_edge(lbm_ctx* c, double ux, double uy) {
  if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
  return lbm::host::set_velocity_edge(c->L, ux, uy);
}

int lbm_step(lbm_ctx* c, int32_t n) {
  const lbm::TraceRange trace_range("lbm_step");
  if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
  if (n < 0) return fail(LBM_ERR_ARG, "n = %d < 0", n);
  if (n == 0) return LBM_OK;
  if (c->overlap) {
    // fork: the side stream starts after everything already on the stream
    HIPCHK(hipEventRecord(c->ev_bulk, c->stream));
    HIPCHK(hipEventRecord(c->ev_edge, c->stream));
  }
  int32_t s = 0;
  if (use_two_step(c)) {
    const int k = multi_steps(c->two_step);
    int rc = LBM_OK;
    for (; s + k <= n && rc == LBM_OK; s += k) rc = step_multi(c, c->two_step);
    // a remainder of two or more steps: one launch of a shape with that
    // many steps instead of single steps (same results)
    if (rc == LBM_OK && n - s >= 2) {
      const int r = rem_shape(c, n - s);
      if (r >= 0) {
        rc = step_multi(c, r);
        s += multi_steps(r);
      }
    }
    // nothing else runs on the stream before the last edge-tile kernel is done
    const hipError_t e = settle_join(c, c->join_pending);
    if (rc) return rc;
    HIPCHK(e);
  }
  for (; s < n; ++s) {
    int rc = step_once(c);
    if (rc) return rc;
  }
  // join: later work on the stream sees the last edge kernel too
  if (c->overlap) HIPCHK(hipStreamWaitEvent(c->stream, c->ev_edge, 0));
  int rc = lbm::host::debug_sync(c->stream, "lbm_step");
  if (rc == LBM_OK && lbm::host::debug_level() >= 2) {
    int ok = 1;
    rc = lbm_check_finite(c, &ok);
  }
  return rc;
}

int lbm_set_overlap(lbm_ctx* c, int on) {
  if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
  c->overlap = on != 0;
  return LBM_OK;
}

int lbm_moments(lbm_ctx* c, void* r, void* u, void* v, int out_f64, int deviation) {
  if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
  HIPCHK(lbm::launch_moments(c->L, c->parity, r, u, v, out_f64 ? 1 : 0, deviation ? 1 : 0, c->stream));
  return lbm::host::debug_sync(c->stream, "lbm_moments");
}

int lbm_time(const lbm_ctx* c, int64_t* t) {
  if (!c || !t) return fail(LBM_ERR_ARG, "NULL argument");
  *t = c->t;
  return LBM_OK;
}

const char* lbm_last_error(void) { return lbm::host::last_error(); }

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  if (c->ev_bulk) (void)hipEventDestroy(c->ev_bulk);
  if (c->ev_edge) (void)hipEventDestroy(c->ev_edge);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  delete c;
}

int lbm_get_populations(lbm_ctx* c, double* g_out) {
  if (!c || !g_out) return fail(LBM_ERR_ARG, "NULL argument");
  HIPCHK(lbm::launch_get_pops(c->L, c->parity, g_out, c->stream));
  return lbm::host::debug_sync(c->stream, "lbm_get_populations");
}

int lbm_set_populations(lbm_ctx* c, const double* g) {
  if (!c || !g) return fail(LBM_ERR_ARG, "NULL argument");
  HIPCHK(lbm::launch_set_pops(c->L, c->parity, g, c->stream));
  return lbm::host::debug_sync(c->stream, "lbm_set_populations");
}

int lbm_check_finite(lbm_ctx* c, int* ok) {
  if (!c || !ok) return fail(LBM_ERR_ARG, "NULL argument");
  int* flag = reinterpret_cast<int*>(c->scratch + kOffFlag);
  int host = 0;
  HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), c->stream));
  HIPCHK(lbm::launch_finite(c->L, c->parity, flag, c->stream));
  HIPCHK(hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *ok = host ? 0 : 1;
  return host ? fail(LBM_ERR_NONFINITE, "populations hold a non-finite value at t = %lld", (long long)c->t) : LBM_OK;
}

int lbm_f16_exp(const lbm_ctx* c, int32_t* k) {
  if (!c || !k) return fail(LBM_ERR_ARG, "NULL argument");
  *k = c->p.store == LBM_STORE_F16DEV ? c->f16_exp : 0;
  return LBM_OK;
}

int lbm_energy(lbm_ctx* test, const lbm_ctx* ref, int32_t x_off, int32_t y_off, double ux_ref, double uy_ref,
               double* out_dev) {
  if (!test || !out_dev) return fail(LBM_ERR_ARG, "NULL argument");
  if (ref) {
    if (ref->p.rho0 != test->p.rho0) return fail(LBM_ERR_ARG, "test and reference rho0 differ");
    if (x_off < 0 || y_off < 0 || x_off + test->p.nx > ref->p.nx || y_off + test->p.ny > ref->p.ny)
      return fail(LBM_ERR_ARG, "window %dx%d at (%d, %d) does not fit in the %dx%d reference", test->p.nx,
                  test->p.ny, x_off, y_off, ref->p.nx, ref->p.ny);
  }
  double* part = reinterpret_cast<double*>(test->scratch + kOffEnergy);
  HIPCHK(lbm::launch_energy(test->L, test->parity, ref ? &ref->L : nullptr, ref ? ref->parity : 0, x_off, y_off,
                            ux_ref, uy_ref, part, out_dev, test->stream));
  return lbm::host::debug_sync(test->stream, "lbm_energy");
}

int lbm_energy_noalloc(lbm_ctx* test, const lbm_ctx* ref, int32_t x_off, int32_t y_off, double ux_ref,
                       double uy_ref, double* out_dev) {
  if (!test || !out_dev) return fail(LBM_ERR_ARG, "NULL argument");
  if (ref) {
    if (ref->p.rho0 != test->p.rho0) return fail(LBM_ERR_ARG, "test and reference rho0 differ");
    if (x_off < 0 || y_off < 0 || x_off + test->p.nx > ref->p.nx || y_off + test->p.ny > ref->p.ny)
      return fail(LBM_ERR_ARG, "window %dx%d at (%d, %d) does not fit in the %dx%d reference", test->p.nx,
                  test->p.ny, x_off, y_off, ref->p.nx, ref->p.ny);
  }
  const int parts = lbm::energy_partials();
  if (parts > kNoAllocPartials)
    return fail(LBM_ERR_UNSUPPORTED, "the reduction needs %d partials; the static scratch holds %d", parts,
                kNoAllocPartials);
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != test->device || (ref && ref->device != test->device))
    return fail(LBM_ERR_ARG, "call with the contexts' device (%d) current, not %d", test->device, dev);
  void* ptr = nullptr;
  int rc = scratch_of_current_device(&ptr);
  if (rc) return rc;
  // every block writes its partial before the final sum reads it: nothing to clear
  HIPCHK(lbm::launch_energy(test->L, test->parity, ref ? &ref->L : nullptr, ref ? ref->parity : 0, x_off, y_off,
                            ux_ref, uy_ref, static_cast<double*>(ptr), out_dev, test->stream));
  return lbm::host::debug_sync(test->stream, "lbm_energy_noalloc");
}

int lbm_tile_count(void) { return lbm::num_tiles(); }

int lbm_tile_describe(int32_t id, char* buf, size_t len) {
  if (!buf || len == 0) return fail(LBM_ERR_ARG, "NULL buffer");
  if (id < 0 || id >= lbm::num_tiles()) return fail(LBM_ERR_ARG, "tile id %d out of range", id);
  lbm::tile_name(id, buf, len);
  return LBM_OK;
}

int lbm_set_tile(lbm_ctx* c, int32_t id) {
  if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
  if (id < 0 || id >= lbm::num_tiles()) return fail(LBM_ERR_ARG, "tile id %d out of range", id);
  c->tile = id;
  return LBM_OK;
}

int lbm_get_tile(const lbm_ctx* c, int32_t* id) {
  if (!c || !id) return fail(LBM_ERR_ARG, "NULL argument");
  *id = c->tile;
  return LBM_OK;
}

namespace {

// The tuners time launches that advance the state, as stepping does.  A
// launch repeated on one unchanged input re-reads one buffer, which for a
// lattice whose buffer fits in the GPU's last-level cache (256 MB on MI355X)
// and whose two buffers do not is served partly from that cache, a speed no
// run of consecutive steps sees.  The current buffer is saved to a temporary
// device copy first and restored at the end, so tuning leaves the state (and
// t) as it was.
// Steps in one timed run of a tuner candidate (consecutive launches): short
// runs of a lattice whose state partly fits in the last-level cache rank
// shapes differently from long ones.
constexpr int kTuneRunSteps = 24;

struct StateSnapshot {
  lbm_ctx* c = nullptr;
  void* copy = nullptr;
  size_t bytes = 0;
  int save(lbm_ctx* ctx) {
    c = ctx;
    bytes = 9 * (size_t)c->L.plane * c->lay.esize;
    HIPCHK(hipMalloc(&copy, bytes));
    HIPCHK(hipMemcpyAsync(copy, lbm::buf_of(c->L, c->parity), bytes, hipMemcpyDeviceToDevice, c->stream));
    return LBM_OK;
  }
  int restore() {
    HIPCHK(hipMemcpyAsync(lbm::buf_of(c->L, c->parity), copy, bytes, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return LBM_OK;
  }
  ~StateSnapshot() {
    if (copy) (void)hipFree(copy);
  }
};

}  // namespace

int lbm_autotune(lbm_ctx* c, int32_t reps, int32_t* best, float* times_ms) {
  const lbm::TraceRange trace_range("lbm_autotune");
  if (!c || !best) return fail(LBM_ERR_ARG, "NULL argument");
  if (reps < 1 || reps > 1000) return fail(LBM_ERR_ARG, "reps = %d outside [1, 1000]", reps);
  // The launches timed are those of an lbm_step: the fused step (edge
  // segments + bulk tiles) or, without fusion (the closure, or fusion off),
  // the bulk kernel and then the edge kernel, over consecutive steps from a
  // saved state; the candidates differ in the bulk tile only, and their
  // times are those of whole steps, comparable with the multi-step shapes'.
  const bool fused = use_fused(c);
  StateSnapshot snap;
  if (int rc = snap.save(c)) return rc;
  int par = c->parity;
  auto launch = [&](int id) {
    hipError_t e = fused ? lbm::launch_step(c->L, par, id, c->stream) : lbm::launch_bulk(c->L, par, id, c->stream);
    if (!fused && e == hipSuccess) e = lbm::launch_edge(c->L, par, c->stream);
    par ^= 1;
    return e;
  };
  const int nt = lbm::num_tiles();
  std::vector<hipEvent_t> ev(2 * reps);
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  float best_t = 1e30f;
  int best_id = c->tile;
  int rc = LBM_OK;
  for (int id = 0; id < nt && rc == LBM_OK; ++id) {
    hipError_t e = launch(id);
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
      e = hipEventRecord(ev[2 * r], c->stream);
      for (int k = 0; k < kTuneRunSteps && e == hipSuccess; ++k) e = launch(id);
      if (e == hipSuccess) e = hipEventRecord(ev[2 * r + 1], c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    std::vector<float> ts(reps);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = hipEventElapsedTime(&ts[r], ev[2 * r], ev[2 * r + 1]);
    if (e != hipSuccess) {
      rc = fail(LBM_ERR_HIP, "autotune candidate %d: %s", id, hipGetErrorString(e));
      break;
    }
    std::sort(ts.begin(), ts.end());
    const float med = ts[reps / 2] / (float)kTuneRunSteps;
    if (times_ms) times_ms[id] = med;
    if (med < best_t) {
      best_t = med;
      best_id = id;
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (rc) return rc;
  if (int r = snap.restore()) return r;
  c->tile = best_id;
  *best = best_id;
  return LBM_OK;
}

int lbm_enable_timing(lbm_ctx* c, int on) {
  if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
  int rc = flush_timing(c);
  if (rc) return rc;
  c->timing = on != 0;
  c->bulk_ms = c->edge_ms = c->two_ms = 0;
  c->bulk_n = c->edge_n = c->two_n = 0;
  return LBM_OK;
}

int lbm_two_step_count(void) { return multi_count(); }

int lbm_two_step_describe(int32_t id, char* buf, size_t len) {
  if (!buf || len == 0) return fail(LBM_ERR_ARG, "NULL buffer");
  if (id < 0 || id >= multi_count()) return fail(LBM_ERR_ARG, "multi-step shape %d out of range", id);
  multi_name(id, buf, len);
  return LBM_OK;
}

int lbm_two_step_steps(int32_t id, int32_t* steps) {
  if (!steps) return fail(LBM_ERR_ARG, "NULL argument");
  if (id < 0 || id >= multi_count()) return fail(LBM_ERR_ARG, "multi-step shape %d out of range", id);
  *steps = multi_steps(id);
  return LBM_OK;
}

int lbm_set_two_step(lbm_ctx* c, int32_t id) {
  if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
  if (id < -1 || id >= multi_count()) return fail(LBM_ERR_ARG, "multi-step shape %d out of range", id);
  if (id >= 0 && !lbm::two_step_supported(c->L))
    return fail(LBM_ERR_ARG, "the multi-step sweeps need NSBC on all four edges");
  // the shape must suit the lattice; whether it carries the closure is
  // decided per lbm_step (single steps where it does not)
  lbm::LatDesc geom = c->L;
  geom.closure = 0;
  if (id >= 0 && !multi_supported(geom, id))
    return fail(LBM_ERR_ARG,
                "multi-step shape %d: three-step shapes need whole tiles (nx >= 64, ny >= its tile rows) and "
                "their LDS for this format",
                id);
  c->two_step = id;
  return LBM_OK;
}

int lbm_get_two_step(const lbm_ctx* c, int32_t* id) {
  if (!c || !id) return fail(LBM_ERR_ARG, "NULL argument");
  *id = c->two_step;
  return LBM_OK;
}

int lbm_autotune_two_step(lbm_ctx* c, int32_t reps, int32_t* best, float* times_ms) {
  const lbm::TraceRange trace_range("lbm_autotune_two_step");
  if (!c || !best) return fail(LBM_ERR_ARG, "NULL argument");
  if (reps < 1 || reps > 1000) return fail(LBM_ERR_ARG, "reps = %d outside [1, 1000]", reps);
  if (!lbm::two_step_supported(c->L))
    return fail(LBM_ERR_ARG, "the multi-step sweeps need NSBC on all four edges");
  // consecutive launches from a saved state (as lbm_autotune); shapes are
  // compared by time per step, and a shape the lattice cannot take reports a
  // negative time
  StateSnapshot snap;
  if (int r = snap.save(c)) return r;
  int par = c->parity;
  bool pending = false;  // as in lbm_step: a closure launch's wait for its edge-tile kernel
  auto launch = [&](int id) {
    const hipError_t e = launch_multi_run(c, par, id, pending);
    par ^= 1;  // a multi-step launch writes its last level to the other buffer
    return e;
  };
  const int nt = multi_count();
  std::vector<hipEvent_t> ev(2 * reps);
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  float best_t = 1e30f, best_k_t[5] = {1e30f, 1e30f, 1e30f, 1e30f, 1e30f};
  int best_id = 0, best_k[5] = {-1, -1, -1, -1, -1};
  int rc = LBM_OK;
  for (int id = 0; id < nt && rc == LBM_OK; ++id) {
    if (!multi_supported(c->L, id)) {
      if (times_ms) times_ms[id] = -1.f;
      continue;
    }
    hipError_t e = launch(id);
    const int runs = (kTuneRunSteps + multi_steps(id) - 1) / multi_steps(id);  // launches per timed run
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
      e = settle_join(c, pending);
      if (e == hipSuccess) e = hipEventRecord(ev[2 * r], c->stream);
      for (int k = 0; k < runs && e == hipSuccess; ++k) e = launch(id);
      if (e == hipSuccess) e = settle_join(c, pending);
      if (e == hipSuccess) e = hipEventRecord(ev[2 * r + 1], c->stream);
    }
    {
      const hipError_t e2 = settle_join(c, pending);
      if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    std::vector<float> ts(reps);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = hipEventElapsedTime(&ts[r], ev[2 * r], ev[2 * r + 1]);
    if (e != hipSuccess) {
      rc = fail(LBM_ERR_HIP, "two-step candidate %d: %s", id, hipGetErrorString(e));
      break;
    }
    std::sort(ts.begin(), ts.end());
    const float med = ts[reps / 2] / (float)(runs * multi_steps(id));
    if (times_ms) times_ms[id] = med;
    if (med < best_t) {
      best_t = med;
      best_id = id;
    }
    const int k = multi_steps(id);
    if (med < best_k_t[k]) {
      best_k_t[k] = med;
      best_k[k] = id;
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (rc) return rc;
  if (int r = snap.restore()) return r;
  c->two_step = best_id;
  for (int k = 2; k <= 4; ++k)
    if (best_k[k] >= 0) c->rem_best[k] = best_k[k];
  *best = best_id;
  return LBM_OK;
}

int lbm_two_step_times(lbm_ctx* c, double* ms, int64_t* launches) {
  if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
  int rc = flush_timing(c);
  if (rc) return rc;
  if (ms) *ms = c->two_ms;
  if (launches) *launches = c->two_n;
  c->two_ms = 0;
  c->two_n = 0;
  return LBM_OK;
}

int lbm_kernel_times(lbm_ctx* c, double* bulk_ms, int64_t* bulk_launches, double* edge_ms, int64_t* edge_launches) {
  if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
  int rc = flush_timing(c);
  if (rc) return rc;
  if (bulk_ms) *bulk_ms = c->bulk_ms;
  if (bulk_launches) *bulk_launches = c->bulk_n;
  if (edge_ms) *edge_ms = c->edge_ms;
  if (edge_launches) *edge_launches = c->edge_n;
  c->bulk_ms = c->edge_ms = 0;
  c->bulk_n = c->edge_n = 0;
  return LBM_OK;
}

int lbm_bulk_traffic(const lbm_ctx* c, int64_t* bytes_per_node, int64_t* nodes_per_launch) {
  if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
  if (bytes_per_node) *bytes_per_node = 18 * (int64_t)c->lay.esize;
  if (nodes_per_launch)
    *nodes_per_launch = use_fused(c) ? (int64_t)c->p.nx * c->p.ny : (int64_t)(c->p.nx - 2) * (c->p.ny - 2);
  return LBM_OK;
}

int lbm_set_fused(lbm_ctx* c, int on) {
  if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
  c->fused = on != 0;
  return LBM_OK;
}

int lbm_set_closure(lbm_ctx* c, const void* net, int mode) {
  if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
  if (mode != 0 && mode != 1) return fail(LBM_ERR_ARG, "closure mode %d", mode);
  if (mode == 1 && !net) return fail(LBM_ERR_ARG, "closure mode 1 needs a network");
  if (net && ((uintptr_t)net & 15)) return fail(LBM_ERR_ARG, "network blob not 16-byte aligned");
  c->L.net = mode ? net : nullptr;
  c->L.closure = mode;
  return LBM_OK;
}

int lbm_closure_features(lbm_ctx* c, const int32_t* sites, int32_t n, float* feat_out, float* mc_out) {
  if (!c || (n > 0 && (!sites || !feat_out || !mc_out))) return fail(LBM_ERR_ARG, "NULL argument");
  if (n < 0) return fail(LBM_ERR_ARG, "n < 0");
  HIPCHK(lbm::host::closure_features(&c->L, nullptr, 1, c->parity, sites, n, feat_out, mc_out, c->stream));
  return LBM_OK;
}

int lbm_closure_moments(lbm_ctx* c, const int32_t* sites, int32_t n, const float* sub, float* m_out) {
  if (!c || (n > 0 && (!sites || !m_out))) return fail(LBM_ERR_ARG, "NULL argument");
  if (n < 0) return fail(LBM_ERR_ARG, "n < 0");
  HIPCHK(lbm::host::closure_moments(&c->L, nullptr, 1, c->parity, sites, n, sub, m_out, c->stream));
  return LBM_OK;
}

int lbm_set_debug(int32_t level) {
  if (level < 0 || level > 2) return fail(LBM_ERR_ARG, "debug level %d outside [0, 2]", level);
  lbm::host::set_debug_level(level);
  return LBM_OK;
}

int lbm_debug_level(int32_t* level) {
  if (!level) return fail(LBM_ERR_ARG, "NULL argument");
  *level = lbm::host::debug_level();
  return LBM_OK;
}

}  // extern "C"

extern "C" int lbm_closure_net_bytes(size_t* bytes);  // include/lbm_closure.h

namespace {

// Checkpoint header (include/lbm.h, lbm_save): fixed 256 bytes, host byte
// order, followed by the populations of the 9 planes as stored, [9][ny][nx].
struct SaveHeader {
  char magic[8];
  uint32_t version, header_bytes;
  int32_t nx, ny, store, f16_exp;
  int32_t bc[4];
  int32_t corr_mode, grad_order, corner_mode, collision;
  int64_t t;
  double tau, rho0, ubase[2], gamma, omega_e, omega_eps, omega_q;
  double beta, m0[3], uw[2];
  int32_t closure, _pad;
  uint64_t net_bytes, net_hash;
  uint64_t payload_bytes, payload_hash;
};
static_assert(sizeof(SaveHeader) <= 256, "checkpoint header exceeds 256 bytes");
constexpr char kSaveMagic[8] = {'L', 'B', 'M', 'C', 'K', 'P', 'T', '1'};
constexpr size_t kHeaderBytes = 256;

size_t payload_bytes(const lbm_ctx* c) { return 9 * (size_t)c->p.nx * c->p.ny * c->lay.esize; }

// Hash of the closure network the context uses (0 bytes, hash 0 without one).
int net_identity(lbm_ctx* c, uint64_t* bytes, uint64_t* hash) {
  *bytes = 0;
  *hash = 0;
  if (!(c->L.closure && c->L.net)) return LBM_OK;
  size_t nb = 0;
  int rc = lbm_closure_net_bytes(&nb);
  if (rc) return rc;
  std::vector<unsigned char> host(nb);
  HIPCHK(hipMemcpyAsync(host.data(), c->L.net, nb, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *bytes = nb;
  *hash = lbm::host::fnv1a(host.data(), nb);
  return LBM_OK;
}

// Copy the current buffer's 9 planes to/from a compact host [9][ny][nx] array.
int copy_planes(lbm_ctx* c, void* host, bool to_host) {
  const size_t es = c->lay.esize, row = (size_t)c->p.nx * es;
  char* dev = static_cast<char*>(lbm::buf_of(c->L, c->parity));
  char* h = static_cast<char*>(host);
  for (int i = 0; i < 9; ++i) {
    char* d = dev + (size_t)i * c->lay.plane * es;
    char* hp = h + (size_t)i * row * c->p.ny;
    if (to_host)
      HIPCHK(hipMemcpy2DAsync(hp, row, d, (size_t)c->lay.pitch * es, row, c->p.ny, hipMemcpyDeviceToHost, c->stream));
    else
      HIPCHK(hipMemcpy2DAsync(d, (size_t)c->lay.pitch * es, hp, row, row, c->p.ny, hipMemcpyHostToDevice, c->stream));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_save_bytes(const lbm_ctx* c, size_t* bytes) {
  if (!c || !bytes) return fail(LBM_ERR_ARG, "NULL argument");
  *bytes = kHeaderBytes + payload_bytes(c);
  return LBM_OK;
}

int lbm_save(lbm_ctx* c, void* host_buf, size_t bytes) {
  if (!c || !host_buf) return fail(LBM_ERR_ARG, "NULL argument");
  const size_t need = kHeaderBytes + payload_bytes(c);
  if (bytes < need) return fail(LBM_ERR_ARG, "checkpoint buffer of %zu bytes < %zu required", bytes, need);
  SaveHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kSaveMagic, 8);
  h.version = 1;
  h.header_bytes = kHeaderBytes;
  h.nx = c->p.nx;
  h.ny = c->p.ny;
  h.store = c->p.store;
  h.f16_exp = c->p.store == LBM_STORE_F16DEV ? c->f16_exp : 0;
  for (int e = 0; e < 4; ++e) h.bc[e] = c->p.bc[e];
  h.corr_mode = c->p.corr_mode;
  h.grad_order = c->p.grad_order;
  h.corner_mode = c->p.corner_mode;
  h.collision = c->p.collision;
  h.t = c->t;
  h.tau = c->p.tau;
  h.rho0 = c->p.rho0;
  h.ubase[0] = c->p.ubase[0];
  h.ubase[1] = c->p.ubase[1];
  h.gamma = c->p.gamma;
  h.omega_e = c->p.omega_e;
  h.omega_eps = c->p.omega_eps;
  h.omega_q = c->p.omega_q;
  h.beta = c->L.beta;
  for (int k = 0; k < 3; ++k) h.m0[k] = c->L.m0[k];
  h.uw[0] = c->L.uw[0];
  h.uw[1] = c->L.uw[1];
  h.closure = (c->L.closure && c->L.net) ? 1 : 0;
  int rc = net_identity(c, &h.net_bytes, &h.net_hash);
  if (rc) return rc;
  char* out = static_cast<char*>(host_buf);
  rc = copy_planes(c, out + kHeaderBytes, true);
  if (rc) return rc;
  h.payload_bytes = payload_bytes(c);
  h.payload_hash = lbm::host::fnv1a(out + kHeaderBytes, h.payload_bytes);
  std::memset(out, 0, kHeaderBytes);
  std::memcpy(out, &h, sizeof(h));
  return LBM_OK;
}

int lbm_load(lbm_ctx* c, const void* host_buf, size_t bytes) {
  if (!c || !host_buf) return fail(LBM_ERR_ARG, "NULL argument");
  if (bytes < kHeaderBytes) return fail(LBM_ERR_ARG, "checkpoint of %zu bytes is shorter than its header", bytes);
  SaveHeader h;
  std::memcpy(&h, host_buf, sizeof(h));
  if (std::memcmp(h.magic, kSaveMagic, 8) != 0 || h.version != 1 || h.header_bytes != kHeaderBytes)
    return fail(LBM_ERR_ARG, "not a version-1 lbm checkpoint");
  if (h.payload_bytes != payload_bytes(c) || bytes < kHeaderBytes + h.payload_bytes)
    return fail(LBM_ERR_ARG, "checkpoint payload of %llu bytes does not fit this %dx%d lattice or the buffer",
                (unsigned long long)h.payload_bytes, c->p.nx, c->p.ny);
  const char* in = static_cast<const char*>(host_buf);
  if (lbm::host::fnv1a(in + kHeaderBytes, h.payload_bytes) != h.payload_hash)
    return fail(LBM_ERR_ARG, "checkpoint payload is corrupt (hash mismatch)");
  // the checkpoint continues the same problem: lattice, storage and physics must match
  const lbm_params& p = c->p;
  bool same = h.nx == p.nx && h.ny == p.ny && h.store == p.store &&
              h.corr_mode == p.corr_mode && h.grad_order == p.grad_order && h.corner_mode == p.corner_mode &&
              h.collision == p.collision && h.tau == p.tau && h.rho0 == p.rho0 && h.ubase[0] == p.ubase[0] &&
              h.ubase[1] == p.ubase[1] && h.gamma == p.gamma;
  for (int e = 0; e < 4; ++e) same = same && h.bc[e] == p.bc[e];
  if (p.collision == LBM_COLL_MRT)
    same = same && h.omega_e == p.omega_e && h.omega_eps == p.omega_eps && h.omega_q == p.omega_q;
  if (!same) return fail(LBM_ERR_STATE, "checkpoint was taken on a lattice with other parameters or storage");
  uint64_t nb = 0, nh = 0;
  int rc = net_identity(c, &nb, &nh);
  if (rc) return rc;
  const int closure = (c->L.closure && c->L.net) ? 1 : 0;
  if (closure != h.closure || nb != h.net_bytes || nh != h.net_hash)
    return fail(LBM_ERR_STATE, "checkpoint closure (mode %d) differs from the context's (mode %d or another network)",
                h.closure, closure);
  if (!(h.beta >= 0.0 && h.beta <= 1.0)) return fail(LBM_ERR_ARG, "checkpoint beta %g outside [0, 1]", h.beta);
  if (p.store == LBM_STORE_F16DEV && (h.f16_exp < -30 || h.f16_exp > 60))
    return fail(LBM_ERR_ARG, "checkpoint FP16 exponent %d outside [-30, 60]", h.f16_exp);
  lbm::LatDesc L = c->L;
  rc = lbm::host::set_velocity_edge(L, h.uw[0], h.uw[1]);
  if (rc) return rc;
  rc = copy_planes(c, const_cast<char*>(in) + kHeaderBytes, false);
  if (rc) return rc;
  L.beta = h.beta;
  for (int k = 0; k < 3; ++k) L.m0[k] = h.m0[k];
  if (p.store == LBM_STORE_F16DEV) {
    // the saved values are encoded with the saved exponent
    c->f16_exp = h.f16_exp;
    lbm::host::set_scales(L, p.store, h.f16_exp);
  }
  c->L = L;
  c->t = h.t;
  return LBM_OK;
}

int lbm_stream_copy(const void* src, void* dst, size_t bytes, void* hip_stream) {
  if (bytes == 0) return LBM_OK;
  if (!src || !dst) return fail(LBM_ERR_ARG, "NULL pointer");
  if (((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return fail(LBM_ERR_ARG, "src/dst not 16-byte aligned");
  const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
  if (a < b + bytes && b < a + bytes) return fail(LBM_ERR_ARG, "src and dst overlap");
  HIPCHK(lbm::launch_copy(src, dst, bytes, static_cast<hipStream_t>(hip_stream)));
  return LBM_OK;
}

}  // extern "C"
