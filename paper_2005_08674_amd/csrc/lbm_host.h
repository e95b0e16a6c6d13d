// lbm_host.h -- host-side helpers shared by the single-lattice and the
// ensemble C-ABI implementations: error reporting, parameter checks, the
// workspace layout and the lattice descriptor.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "lbm.h"
#include "lbm_device.h"

namespace lbm {
namespace host {

constexpr size_t kScratchBytes = 1 << 20;

// Record a formatted message for lbm_last_error() and return `code`.
int fail(int code, const char* fmt, ...);
const char* last_error();

size_t round_up(size_t v, size_t a);
size_t elem_bytes(int store);

// Population buffers of one lattice: pitch (elements per row, rows of 256
// bytes), plane (elements per population plane), one buffer = 9 planes.
struct Layout {
  size_t esize;
  int32_t pitch;
  int64_t plane;
  size_t buf_bytes;
  size_t total;  // two buffers + scratch
};

Layout layout(const lbm_params* p);
int check_params(const lbm_params* p);
void set_scales(LatDesc& L, int store, int k);
void fill_desc(LatDesc& L, const lbm_params* p, const Layout& lay, void* buf0, void* buf1);
int set_farfield(LatDesc& L, double beta, double rho_ref, double ux_ref, double uy_ref);
int set_velocity_edge(LatDesc& L, double ux, double uy);
int f16_exp_from_max(float mx);

// Debug level: 0 off; 1 every call that enqueues work synchronizes its
// stream and reports any HIP error as LBM_ERR_HIP; 2 also checks after every
// step call that the populations are finite (LBM_ERR_NONFINITE).  Starts
// from the environment variable LBM_DEBUG, read once; lbm_set_debug changes
// it for the process.
int debug_level();
void set_debug_level(int level);
// With debug on: synchronize `s` and turn a pending HIP error into
// LBM_ERR_HIP naming `call`.  LBM_OK when debug is off.
int debug_sync(hipStream_t s, const char* call);

// 64-bit FNV-1a hash of `n` bytes (checkpoint integrity and identity).
uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ull);

// Closure sampling launchers (lbm_closure.hip).  Exactly one of `single`
// (one lattice) or `descs` (device descriptors of an ensemble) is used.
hipError_t closure_features(const LatDesc* single, const LatDesc* descs, int count, int parity, const int32_t* sites,
                            int n, float* feat, float* mc, hipStream_t s);
hipError_t closure_moments(const LatDesc* single, const LatDesc* descs, int count, int parity, const int32_t* sites,
                           int n, const float* sub, float* out, hipStream_t s);

}  // namespace host
}  // namespace lbm
