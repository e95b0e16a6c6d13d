// lbm_march.hip -- the marched two- and three-step sweeps' instances
// (kernels and shapes in lbm_threestep.h): edge tiles and strips in one
// launch.
#include <hip/hip_runtime.h>

#include "lbm_device.h"
#include "lbm_launch.h"
#include "lbm_threestep.h"

namespace lbm {

// March shape `id` (among the march shapes) in format S.
template <int S>
static hipError_t launch_march_s(const LatDesc& L, int parity, int id, hipStream_t s, bool ring, int part) {
  int k = 0;
#define X(a, m, b, h, p, n)                                                     \
  if (id == k) return launch_march_t<S, a, m, b, n, p>(L, parity, s, h, ring, part); \
  ++k;
  LBM_THREE_MARCH(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_three_march(const LatDesc& L, int parity, int id, hipStream_t s, bool ring, int part) {
  if (part < 0 || part > 2) return hipErrorInvalidValue;
  switch (L.store) {
    case ST_F64: return launch_march_s<ST_F64>(L, parity, id, s, ring, part);
    case ST_F32: return launch_march_s<ST_F32>(L, parity, id, s, ring, part);
    case ST_F16: return launch_march_s<ST_F16>(L, parity, id, s, ring, part);
    case ST_BF16: return launch_march_s<ST_BF16>(L, parity, id, s, ring, part);
  }
  return hipErrorInvalidValue;
}

template <int S>
static hipError_t launch_two_march_s(const LatDesc& L, int parity, int id, hipStream_t s) {
  int k = 0;
#define X(a, m, b, h, n)                                                  \
  if (id == k) return launch_two_march_t<S, a, m, b, n>(L, parity, s, h); \
  ++k;
  LBM_TWO_MARCH(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_two_march(const LatDesc& L, int parity, int id, hipStream_t s) {
  switch (L.store) {
    case ST_F64: return launch_two_march_s<ST_F64>(L, parity, id, s);
    case ST_F32: return launch_two_march_s<ST_F32>(L, parity, id, s);
    case ST_F16: return launch_two_march_s<ST_F16>(L, parity, id, s);
    case ST_BF16: return launch_two_march_s<ST_BF16>(L, parity, id, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbm
