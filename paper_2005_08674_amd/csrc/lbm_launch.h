// lbm_launch.h -- host-side launchers of the kernels in lbm_kernels.hip
// (internal to the library; the public interface is include/lbm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "lbm_device.h"

namespace lbm {

int num_tiles();
void tile_name(int id, char* buf, size_t len);
hipError_t launch_bulk(const LatDesc& L, int parity, int tile, hipStream_t s);
int edge_blocks(int nx, int ny);
hipError_t launch_edge(const LatDesc& L, int parity, hipStream_t s);
// edge segments and bulk tiles of one step in a single launch (not with the closure)
hipError_t launch_step(const LatDesc& L, int parity, int tile, hipStream_t s);
int num_two_step();
void two_step_name(int id, char* buf, size_t len);
bool two_step_supported(const LatDesc& L);
// whether two-step shape id is a column march (single lattices only)
bool two_step_is_march(int id);
hipError_t launch_two_step(const LatDesc& L, int parity, int id, hipStream_t s);
// output tile rows of two-step shape id (0 if invalid), and the smallest over all shapes
int two_step_tile_rows(int id);
int two_step_min_rows();
// three-step sweep (t -> t + 3), single lattices
int num_three_step();
void three_step_name(int id, char* buf, size_t len);
bool three_step_supported(const LatDesc& L, int id);
// whether three-step shape id is a column march (single lattices only)
bool three_step_is_march(int id);
// (with the learned closure: edge tiles on `side` beside the inner tiles on s when side, fork and join are given)
// Flags of a closure launch on two streams.  kJoinPrev: s waits for the
// previous launch's edge-tile kernel (the last record of join) before this
// launch's kernel on s.  kJoinDefer: s does not wait for this launch's
// edge-tile kernel on return; the caller issues that wait (the next launch
// with kJoinPrev, or hipStreamWaitEvent(s, join)) before s runs anything else
// that touches the lattice.
constexpr int kJoinPrev = 1, kJoinDefer = 2;
hipError_t launch_three_step(const LatDesc& L, int parity, int id, hipStream_t s, hipStream_t side = nullptr,
                             hipEvent_t fork = nullptr, hipEvent_t join = nullptr, int flags = 0);
int three_step_tile_rows(int id);
int three_step_min_rows();
// ensemble two-step: one block per list entry (member, 64-column tile x, tile y); lat < 0 = padding
struct TwoTile {
  int32_t lat, txi, tyi, pad;
};
hipError_t launch_ens_two_step(int store, int id, const LatDesc* d, const TwoTile* list, int n, int parity,
                               hipStream_t s);
// the same over the three-step shapes (id among the three-step shapes)
hipError_t launch_ens_three_step(int store, int id, const LatDesc* d, const TwoTile* list, int n, int parity,
                                 hipStream_t s);
hipError_t launch_init(const LatDesc& L, int parity, const double* drho, const double* ux, const double* uy,
                       hipStream_t s);
int absmax_blocks();
hipError_t launch_absmax_init(const LatDesc& L, const double* drho, const double* ux, const double* uy,
                              float* partial, hipStream_t s);
hipError_t launch_moments(const LatDesc& L, int parity, void* r, void* u, void* v, int f64, int deviation,
                          hipStream_t s);
hipError_t launch_get_pops(const LatDesc& L, int parity, double* out, hipStream_t s);
hipError_t launch_set_pops(const LatDesc& L, int parity, const double* in, hipStream_t s);
hipError_t launch_finite(const LatDesc& L, int parity, int* bad, hipStream_t s);
int energy_partials();
hipError_t launch_energy(const LatDesc& T_, int pt, const LatDesc* R_, int pr, int xo, int yo, double ux_ref,
                         double uy_ref, double* partial, double* out, hipStream_t s);

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);

}  // namespace lbm
