// lbm_twostep_cl.hip -- the three-step kernel for the edge tiles of a lattice
// on the learned closure (three_step_tile with CL), one instance per storage
// format, shape and collision model, in a translation unit of its own.
#include <hip/hip_runtime.h>

#include "lbm_threestep.h"

namespace lbm {

hipError_t launch_three_step_closure(const LatDesc& L, int parity, int id, hipStream_t s) {
  switch (L.store) {
    case ST_F64: return launch_three_s<ST_F64, true>(L, parity, id, s, 2);
    case ST_F32: return launch_three_s<ST_F32, true>(L, parity, id, s, 2);
    case ST_F16: return launch_three_s<ST_F16, true>(L, parity, id, s, 2);
    case ST_BF16: return launch_three_s<ST_BF16, true>(L, parity, id, s, 2);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbm
